"""Pins of the oracle's fluid solvation force (Sec. 2, Eq. solvation_lambda):
each particle acts on the 8 vertices r of its lattice cell with
-lambda_zeta rho_zeta(r) sum_j c_j/|c_j|^2 over the links j pointing into
the particle's half space (d . c_j > 0, d = x_p - r; the paper's Theta with
cos = 1 included), and the particle receives minus the total.

Values below are worked out by hand from the definition, not from the code:
 * particle at a cell centre, d = (1/2)(sx, sy, sz): the three axis links
   +s_a (weight 1 each) and the three diagonals in the particle's octant
   (weight 1/2 each, two per axis) give S = 2 (sx, sy, sz) at every vertex;
 * particle at (3.5, 3, 3): at vertex (3,3,3), d = (1/2, 0, 0): +x (cos = 1,
   counted) and the four diagonals with a +x part (1/2 each) give (3, 0, 0);
   at vertex (3,4,3), d = (1/2, -1, 0): +x, -y, (+1,-1,0), (-1,-1,0),
   (+1,0,+-1), (0,-1,+-1) give (1,0,0) + (0,-1,0) + (1,-2,0) = (2, -3, 0).
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def site(shape, x, y, z):
    return (z * shape[1] + y) * shape[0] + x


def test_cell_centre_closed_form_and_no_net_force():
    shape = (8, 8, 8)
    N = 512
    lam = (0.7, -0.3)
    P = oracle.make_params(shape, lambda_fs=(lam,))
    rho = np.empty((2, N))
    rho[0], rho[1] = 1.3, 0.6
    fs, back = oracle.solvation_fluid_force(P, rho, [[3.5, 3.5, 3.5]])
    for ox in (0, 1):
        for oy in (0, 1):
            for oz in (0, 1):
                sgn = np.array([1.0 - 2 * ox, 1.0 - 2 * oy, 1.0 - 2 * oz])  # towards the particle
                s_ = site(shape, 3 + ox, 3 + oy, 3 + oz)
                for c in range(2):
                    assert np.allclose(fs[c, :, s_], -lam[c] * rho[c, 0] * 2.0 * sgn, atol=1e-15)
    # only the 8 vertices are touched
    assert np.count_nonzero(np.abs(fs).sum(axis=(0, 1))) == 8
    # uniform densities: the 8 contributions cancel, nothing to return
    assert np.abs(fs.sum(axis=2)).max() < 1e-14 and np.abs(back).max() < 1e-14


def test_particle_on_a_link_counts_the_aligned_link():
    shape = (8, 8, 8)
    P = oracle.make_params(shape, lambda_fs=((1.0, 0.0),))
    rho = np.ones((2, 512))
    fs, back = oracle.solvation_fluid_force(P, rho, [[3.5, 3.0, 3.0]])
    assert np.allclose(-fs[0, :, site(shape, 3, 3, 3)], [3.0, 0.0, 0.0], atol=1e-15)
    assert np.allclose(-fs[0, :, site(shape, 4, 3, 3)], [-3.0, 0.0, 0.0], atol=1e-15)
    assert np.allclose(-fs[0, :, site(shape, 3, 4, 3)], [2.0, -3.0, 0.0], atol=1e-15)
    assert np.abs(fs[1]).max() == 0.0  # lambda_B = 0


def test_proportional_to_local_density_and_returned_exactly():
    shape = (6, 5, 7)
    N = int(np.prod(shape))
    g = np.random.default_rng(4)
    rho = 0.5 + g.random((2, N))
    x = g.random((30, 3)) * np.array(shape)
    t = (np.arange(30) % 2).astype(np.int32)
    P = oracle.make_params(shape, lambda_fs=((0.4, -0.9), (-0.2, 0.3)), mass=(1.0, 1.0), kappa=((0, 0), (0, 0)))
    fs, back = oracle.solvation_fluid_force(P, rho, x, t)
    # momentum balance per particle, summed: what the fluid gets, the
    # particles lose
    assert np.abs(fs.sum(axis=(0, 2)) + back.sum(axis=0)).max() < 1e-12
    # doubling one component's density doubles its part only
    rho2 = rho.copy()
    rho2[1] *= 2.0
    fs2, _ = oracle.solvation_fluid_force(P, rho2, x, t)
    assert np.allclose(fs2[0], fs[0], atol=1e-15) and np.allclose(fs2[1], 2 * fs[1], atol=1e-14)
    # linear in lambda
    P3 = oracle.make_params(shape, lambda_fs=((0.8, -1.8), (-0.4, 0.6)), mass=(1.0, 1.0), kappa=((0, 0), (0, 0)))
    fs3, back3 = oracle.solvation_fluid_force(P3, rho, x, t)
    assert np.allclose(fs3, 2 * fs, atol=1e-14) and np.allclose(back3, 2 * back, atol=1e-14)


def test_momentum_invariant_with_fluid_solvation():
    """The invariant fluid raw momentum + sum (m v + F_c/2) stays constant
    with the fluid solvation force on (F_c = everything the fluid exerts on
    the particle: friction, kappa solvation, and the lambda return)."""
    from paper_1306_0788_amd import workloads
    shape = (6, 5, 4)
    rho = workloads.initial_densities(shape, 8, amp=0.05).reshape(2, -1)
    g = np.random.default_rng(8)
    x = workloads.free_particles(10, shape, 8, min_dist=1.5)
    v = 0.05 * (g.random((10, 3)) - 0.5)
    t = (np.arange(10) % 2).astype(np.int32)
    P = oracle.make_params(shape, G=((0.0, 1.2), (1.2, 0.0)), gamma=0.7, kappa=((0.3, -0.2), (-0.1, 0.4)),
                           mass=(400.0, 600.0), lambda_fs=((0.05, -0.03), (-0.02, 0.04)))
    s = oracle.Sim(P, rho, x, v, t)
    m = np.array([P.mass[k] for k in t])[:, None]

    def inv():
        return s.fluid_momentum() + (m * s.v).sum(axis=0) + 0.5 * s.Fc.sum(axis=0)

    I0 = inv()
    for _ in range(30):
        assert s.step(1) == oracle.OK
        assert np.abs(inv() - I0).max() < 1e-13
    # the lambda force did act: switching it off changes the state
    P0 = oracle.make_params(shape, G=((0.0, 1.2), (1.2, 0.0)), gamma=0.7, kappa=((0.3, -0.2), (-0.1, 0.4)),
                            mass=(400.0, 600.0))
    s0 = oracle.Sim(P0, rho, x, v, t)
    s0.step(30)
    assert np.abs(s0.f - s.f).max() > 1e-6


def test_positive_lambda_pushes_its_component_away():
    """As printed, F^fs at a vertex is -lambda rho times links pointing to the
    particle: with lambda_A > 0 the A fluid is pushed away and its density at
    the particle's cell drops below the far field."""
    shape = (12, 12, 12)
    N = 12 ** 3
    P = oracle.make_params(shape, G=((0.0, 0.0), (0.0, 0.0)), lambda_fs=((0.02, 0.0),), mass=(1e12,))
    s = oracle.Sim(P, np.ones((2, N)), x=np.array([[6.5, 6.5, 6.5]]))
    assert s.step(40) == oracle.OK
    r = s.rho()
    near = np.mean([r[0, site(shape, 6 + ox, 6 + oy, 6 + oz)] for ox in (0, 1) for oy in (0, 1) for oz in (0, 1)])
    far = r[0, site(shape, 0, 0, 0)]
    assert near < far - 1e-4
    assert abs(r[1, site(shape, 6, 6, 6)] - 1.0) < abs(near - 1.0)  # B only follows through the mixture
