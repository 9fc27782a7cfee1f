"""GPU parity: the HIP path through the C ABI against the oracle, element by
element on identical seeded inputs.

Tolerances: FP64 storage 1e-12 relative per population after one step
(rounding order only); FP32 storage 1e-5 after one step and 1e-4 on the
densities after 100 steps below or just above the spinodal; particles at
the same levels.  Several sizes are ragged on purpose (not multiples of the
64 x TY tiles or of the z chunk)."""
import numpy as np
import pytest

from paper_1306_0788_amd import lbmd
from parity_cases import Case, compare, rel_err

pytestmark = pytest.mark.gpu

FP64, FP32 = lbmd.FP64, lbmd.FP32
PAPER, SHIFT = lbmd.FORCE_PAPER, lbmd.FORCE_SHIFT
FUSED, TWOPASS, PUSH = lbmd.KERNEL_FUSED, lbmd.KERNEL_TWOPASS, lbmd.KERNEL_PUSH


def run_pair(case, steps):
    print("case shape=%s prec=%d forcing=%d kernel=%d steps=%d" % (case.shape, case.precision, case.forcing,
                                                                   case.kernel, steps), flush=True)
    g = case.gpu_sim()
    o = case.oracle_sim()
    g.step(steps)
    assert o.step(steps) == 0
    assert g.sync() == lbmd.OK, g.last_error()
    return g, o


@pytest.mark.parametrize("precision,tol", [(FP64, 1e-12), (FP32, 1e-5)])
@pytest.mark.parametrize("forcing", [PAPER, SHIFT])
@pytest.mark.parametrize("kernel", [FUSED, TWOPASS, PUSH])
def test_one_step_32cubed(precision, tol, forcing, kernel):
    """The 32^3 mixture with 64 particles (G_AB = 1.6, gamma = 0.5)."""
    c = Case((32, 32, 32), precision, forcing, kernel, G=1.6, gamma=0.5, vel_amp=0.02,
             kappa=((0.3, -0.2),), mass=(2.0,))
    g, o = run_pair(c, 1)
    compare(c, g, o, tol, tol, "1 step")


@pytest.mark.parametrize("kernel", [FUSED, TWOPASS, PUSH])
def test_hundred_steps_fp64_paper(kernel):
    """The 32^3 workload, 100 steps, paper forcing (G rho = 1.6 is above the
    spinodal: round-off grows by about 40x per 100 steps)."""
    c = Case((32, 32, 32), FP64, PAPER, kernel, G=1.6, gamma=0.5, mass=(1.0,))
    g, o = run_pair(c, 100)
    compare(c, g, o, 1e-10, 1e-10, "100 steps")


def test_velocity_shift_error_growth_fp64():
    """Velocity shift at G = 1.6 is deep in the spinodal (growth ~1e10 per 100
    steps), so round-off is compared at 20 steps with a looser bound."""
    c = Case((32, 32, 32), FP64, SHIFT, FUSED, G=1.6, gamma=0.5, mass=(1.0,))
    g, o = run_pair(c, 20)
    compare(c, g, o, 1e-9, 1e-9, "20 steps shift")


@pytest.mark.parametrize("kernel", [FUSED, TWOPASS, PUSH])
def test_hundred_steps_fp32_density(kernel):
    """FP32 storage, 100 steps: densities within 1e-4 of the FP64 oracle."""
    c = Case((32, 32, 32), FP32, PAPER, kernel, G=1.6, gamma=0.5, mass=(1.0,))
    g, o = run_pair(c, 100)
    e = rel_err(g.rho(), o.rho())
    assert e <= 1e-4, e


@pytest.mark.parametrize("shape", [(37, 29, 23), (3, 3, 3), (4, 5, 6), (70, 3, 5), (65, 9, 17), (1, 7, 9)])
@pytest.mark.parametrize("kernel", [FUSED, TWOPASS, PUSH])
def test_ragged_shapes(shape, kernel):
    n = 6 if np.prod(shape) < 200 else 40
    c = Case(shape, FP64, PAPER, kernel, G=1.3, gamma=0.7, npart=n, vel_amp=0.02, kappa=((0.2, 0.1),),
             mass=(3.0,), amp=0.03)
    g, o = run_pair(c, 5)
    compare(c, g, o, 1e-11, 1e-11, "ragged")


@pytest.mark.parametrize("tiling", [(2, 1, 1, 1), (4, 3, 0, 1), (8, 5, 1, 0), (8, 7, 0, 0), (16, 40, 1, 1),
                                    (16, 2, 0, 1)])
@pytest.mark.parametrize("kernel", [FUSED, TWOPASS, PUSH])
def test_tilings_agree(tiling, kernel):
    c = Case((37, 29, 23), FP64, PAPER, kernel, G=1.3, gamma=0.7, npart=40, vel_amp=0.02, tiling=tiling)
    g, o = run_pair(c, 3)
    compare(c, g, o, 1e-11, 1e-11, "tiling %s" % (tiling,))


@pytest.mark.parametrize("precision,tol", [(FP64, 1e-12), (FP32, 1e-5)])
@pytest.mark.parametrize("kernel", [FUSED, TWOPASS, PUSH])
def test_fluctuating_identical_draws(precision, tol, kernel):
    """kT > 0: both sides draw the same Philox4x32-10 normals for the fluid modes
    and the particle random force."""
    c = Case((20, 18, 16), precision, PAPER, kernel, G=1.2, gamma=1.0, kT=1e-4, seed=11, npart=30,
             kappa=((0.1, 0.0),), mass=(5.0,))
    g, o = run_pair(c, 3)
    compare(c, g, o, tol * 10, tol * 10, "noise")


@pytest.mark.parametrize("precision,tol", [(FP64, 1e-11), (FP32, 1e-5)])
@pytest.mark.parametrize("kernel", [FUSED, PUSH])
def test_chains_fene_wca_debye_hueckel(precision, tol, kernel):
    """Bead-spring chains (FENE + WCA + screened Debye-Hueckel, all beads
    charged), solvation on A, fluctuating fluid: the polyelectrolyte set-up at
    a small box."""
    c = Case((24, 24, 24), precision, PAPER, kernel, G=1.8, gamma=1.0, kT=1e-4, seed=3, chains=(6, 20),
             kappa=((0.1, 0.0),), mass=(2000.0,), charge=(1.0,), wca=(1.0, 1.0), fene=(30.0, 1.5),
             dh=(1.0, 3.0, 1.0))
    g, o = run_pair(c, 4)
    compare(c, g, o, tol, tol, "chains")


@pytest.mark.parametrize("shape,chains", [((30, 22, 26), (12, 20)), ((17, 40, 21), (10, 25))])
def test_pair_cells_dense_chains(shape, chains):
    """Dense bead chains with the Debye-Hueckel cut-off 3 in ragged boxes
    (cell rows whose x-runs wrap around the box); forces against the
    all-pairs oracle."""
    c = Case(shape, FP64, PAPER, TWOPASS, G=1.5, gamma=1.0, seed=5, chains=chains, kappa=((0.1, 0.0),),
             mass=(2000.0,), charge=(1.0,), wca=(1.0, 1.0), fene=(30.0, 1.5), dh=(1.3, 3.0, 0.8))
    g, o = run_pair(c, 3)
    compare(c, g, o, 1e-11, 1e-11, "pair cells, dense chains")


@pytest.mark.parametrize("kernel", [FUSED, TWOPASS, PUSH])
def test_particles_on_nodes_edges_and_shared_cells(kernel):
    L = 12
    pos = [[3.0, 4.0, 5.0], [0.0, 0.0, 0.0], [L - 1e-13, 2.5, 7.25], [6.5, 6.5, 6.5], [6.6, 6.4, 6.55],
           [6.45, 6.52, 6.51], [11.999999, 11.999999, 0.0]]
    c = Case((L, L, L), FP64, PAPER, kernel, G=1.2, gamma=0.9, positions=pos, vel_amp=0.05,
             kappa=((0.4, -0.3),), mass=(50.0,))
    g, o = run_pair(c, 6)
    compare(c, g, o, 1e-11, 1e-11, "edges")


@pytest.mark.parametrize("kernel", [FUSED, TWOPASS, PUSH])
def test_no_particles(kernel):
    c = Case((33, 17, 12), FP32, PAPER, kernel, G=1.5, npart=0)
    g, o = run_pair(c, 4)
    compare(c, g, o, 1e-5, 1e-5, "no particles")


@pytest.mark.parametrize("kernel", [FUSED, PUSH])
def test_invariants_on_gpu(kernel):
    """Per-component mass to round-off and the fluid + particle momentum
    invariant, read from the device reductions."""
    c = Case((24, 20, 16), FP64, PAPER, kernel, G=1.4, gamma=0.8, npart=50, vel_amp=0.05,
             kappa=((0.3, -0.1),), mass=(400.0,), wca=(1.0, 0.05), min_dist=1.3)
    g = c.gpu_sim()
    first = None
    for k in range(60):
        g.step(1)
        red, st = g.reductions()
        assert st == k
        if first is None:
            first = red.copy()
        assert abs(red[0] - first[0]) < 1e-12 * first[0]
        assert abs(red[1] - first[1]) < 1e-12 * first[1]
        inv, inv0 = red[2:5] + red[5:8], first[2:5] + first[5:8]
        assert np.abs(inv - inv0).max() < 1e-12, (k, inv - inv0)


def test_determinism_without_particles():
    c = Case((40, 24, 20), FP32, PAPER, FUSED, G=1.7, npart=0)
    a = c.gpu_sim()
    b = c.gpu_sim()
    a.step(10)
    b.step(10)
    assert np.array_equal(a.populations(), b.populations())


def test_unstable_state_is_latched():
    c = Case((16, 16, 16), FP64, PAPER, FUSED, G=1.2, npart=4)
    g = c.gpu_sim()
    pop = g.populations()
    pop[1, :, 100] = -0.01  # rho_B < 0 at one site
    g.set_populations(pop)
    g.step(3)
    assert g.sync() == lbmd.EUNSTABLE
    assert "step 0" in g.last_error()
    assert g.step_rc(1) == lbmd.ESTATE


def test_invalid_parameters_rejected():
    with pytest.raises(lbmd.LbmdError):
        lbmd.Sim((8, 8, 8), tau=(0.5, 0.5))
    with pytest.raises(lbmd.LbmdError):
        lbmd.Sim((8, 8, 8), tau=(1.0, 0.9))  # paper forcing needs equal tau
    with pytest.raises(lbmd.LbmdError):
        lbmd.Sim((8, 8, 8), forcing=SHIFT, kT=1e-3)
    s = lbmd.Sim((8, 8, 8))
    with pytest.raises(lbmd.LbmdError):
        s.set_pair_potential(lbmd.PAIR_DH, (1.0, 5.0, 1.0))  # cut-off above half the box
    with pytest.raises(lbmd.LbmdError):
        s.set_particles([[1.0, np.nan, 2.0]])


@pytest.mark.parametrize("kernel", [FUSED, TWOPASS, PUSH])
def test_stepping_on_after_a_failure_stays_in_bounds(kernel):
    """Regression: after a numerical failure the particle velocities diverge
    before they turn non-finite, and positions far outside the box once gave
    node indices outside the lattice.  A job far above the spinodal (G = 4)
    with particles and WCA pairs is stepped well past its failure without
    polling; the failure stays latched at its first step."""
    c = Case((24, 20, 16), FP32, PAPER, kernel, G=4.0, gamma=1.0, npart=200, vel_amp=0.05,
             kappa=((0.5, -0.5),), mass=(1.0,), wca=(1.0, 1.0), min_dist=1.2)
    print("stepping past a failure, kernel %d" % kernel, flush=True)
    g = c.gpu_sim()
    g.step(120)
    assert g.sync() == lbmd.EUNSTABLE
    first = int(g.last_error().split("step ")[1].split()[0])
    assert first < 100


@pytest.mark.parametrize("precision,tol", [(FP64, 1e-11), (FP32, 1e-5)])
@pytest.mark.parametrize("kernel", [FUSED, TWOPASS, PUSH])
def test_fluid_solvation_force(precision, tol, kernel):
    """The fluid solvation force (lambda per type and component) with its
    momentum return, next to friction and kappa solvation, two particle
    types: 5 steps against the oracle."""
    c = Case((28, 22, 18), precision, PAPER, kernel, G=1.3, gamma=0.6, npart=60, vel_amp=0.03,
             kappa=((0.2, -0.1), (-0.15, 0.25)), mass=(20.0, 30.0), lambda_fs=((0.08, -0.05), (-0.03, 0.06)))
    g, o = run_pair(c, 5)
    compare(c, g, o, tol * 5, tol * 5, "lambda")


@pytest.mark.parametrize("kernel", [FUSED, TWOPASS, PUSH])
def test_invariant_with_fluid_solvation_on_gpu(kernel):
    """Fluid raw momentum + sum (m v + F_c/2) stays constant on the GPU with
    friction, kappa and lambda solvation (FP64; both organisations: the fused
    records, and the density pass's sums with the coupling kernel's neighbour
    sums)."""
    c = Case((24, 20, 16), FP64, PAPER, kernel, G=1.4, gamma=0.8, npart=50, vel_amp=0.05,
             kappa=((0.3, -0.1),), mass=(400.0,), lambda_fs=((0.05, -0.04),))
    print("invariant kernel=%d" % kernel, flush=True)
    g = c.gpu_sim()
    first = None
    for k in range(40):
        g.step(1)
        red, st = g.reductions()
        if first is None:
            first = red.copy()
        inv, inv0 = red[2:5] + red[5:8], first[2:5] + first[5:8]
        assert np.abs(inv - inv0).max() < 1e-12, (k, inv - inv0)
    x, v, F, Fc = g.particles()
    assert np.abs(Fc).max() > 0


MRT = (-1.3, -0.8, -1.1, -1.6)  # bulk, shear, momentum, kinetic eigenvalues


@pytest.mark.parametrize("precision,tol", [(FP64, 1e-11), (FP32, 1e-5)])
@pytest.mark.parametrize("kernel", [lbmd.KERNEL_AUTO, TWOPASS])
def test_mrt_with_particles(precision, tol, kernel):
    """Distinct eigenvalues for the four mode groups, the general forcing
    source term, particles with kappa and lambda solvation: 5 steps."""
    c = Case((30, 20, 14), precision, PAPER, kernel, G=1.3, gamma=0.6, npart=40, vel_amp=0.03,
             kappa=((0.2, -0.1),), mass=(20.0,), lambda_fs=((0.05, -0.02),), mrt=MRT)
    g, o = run_pair(c, 5)
    assert g.organisation() == (PUSH if kernel == lbmd.KERNEL_AUTO else TWOPASS)
    compare(c, g, o, tol * 5, tol * 5, "mrt")


@pytest.mark.parametrize("precision,tol", [(FP64, 1e-11), (FP32, 1e-5)])
@pytest.mark.parametrize("kernel,tiling", [(lbmd.KERNEL_AUTO, None), (PUSH, None), (PUSH, (16, 4, 0, 0, 1))])
def test_mrt_fluctuating_identical_draws(precision, tol, kernel, tiling):
    """kT > 0 under MRT: each mode's noise amplitude follows its own
    eigenvalue; the same Philox draws on both sides.  Automatic choice
    (two-pass with noise) and the push kernel, also with 16 rows requested
    (the fluctuating push kernel has at most 8)."""
    c = Case((20, 18, 16), precision, PAPER, kernel, G=1.2, gamma=1.0, kT=1e-4, seed=11, npart=30,
             kappa=((0.1, 0.0),), mass=(5.0,), mrt=MRT, tiling=tiling)
    g, o = run_pair(c, 3)
    assert g.organisation() == (TWOPASS if kernel == lbmd.KERNEL_AUTO else PUSH)
    compare(c, g, o, tol * 10, tol * 10, "mrt noise")


@pytest.mark.parametrize("kernel", [TWOPASS, PUSH])
def test_mrt_reduces_to_bgk(kernel):
    """All four eigenvalues -1/tau give the BGK step (up to rounding)."""
    tau = 0.8
    c1 = Case((18, 14, 12), FP64, PAPER, kernel, G=1.3, tau=tau, gamma=0.5, npart=20, vel_amp=0.02,
              kappa=((0.2, -0.1),), mass=(5.0,), mrt=(-1 / tau,) * 4)
    c0 = Case((18, 14, 12), FP64, PAPER, kernel, G=1.3, tau=tau, gamma=0.5, npart=20, vel_amp=0.02,
              kappa=((0.2, -0.1),), mass=(5.0,))
    a, b = c1.gpu_sim(), c0.gpu_sim()
    a.step(6)
    b.step(6)
    pa, pb = a.populations(), b.populations()
    assert np.max(np.abs(pa - pb) / np.abs(pb)) < 1e-13


def test_mrt_rejects_bad_eigenvalues():
    s = lbmd.Sim((8, 8, 8))
    with pytest.raises(lbmd.LbmdError):
        s.set_mrt((-1.0, 0.1, -1.0, -1.0))
    with pytest.raises(lbmd.LbmdError):
        s.set_mrt((-2.0, -1.0, -1.0, -1.0))
    f = lbmd.Sim((8, 8, 8), kernel=FUSED)
    with pytest.raises(lbmd.LbmdError):
        f.set_mrt(MRT)


@pytest.mark.parametrize("shape,tiling", [((130, 37, 29), (4, 5, 1, 1)), ((128, 12, 10), (2, 3, 0, 1)),
                                          ((64, 17, 6), (8, 1, 0, 0)), ((65, 9, 40), (16, 7, 1, 1))])
@pytest.mark.parametrize("precision,tol", [(FP64, 1e-11), (FP32, 1e-5)])
def test_push_moments_across_box_faces_edges_and_corners(shape, tiling, precision, tol):
    """The push organisation forms each step's densities and momentum from
    the previous step's post-collision values, adding the contributions of
    neighbouring boxes at box faces, edges and corners; many boxes in every
    direction (full 64-lane tiles, a 1-lane tail, one-plane chunks), 8 steps
    with particles against the oracle."""
    c = Case(shape, precision, PAPER, PUSH, G=1.4, gamma=0.7, npart=60, vel_amp=0.02, kappa=((0.2, 0.1),),
             mass=(3.0,), amp=0.03, tiling=tiling)
    g, o = run_pair(c, 8)
    assert g.organisation() == PUSH
    compare(c, g, o, tol * 8, tol * 8, "push boxes %s %s" % (shape, tiling))
