"""Pins of the oracle's tables and single-site pieces.

Each check is fixed by the paper or by mathematics, not by the oracle itself:
D3Q19 isotropy (Appendix, Eqs. isotropy/isotropyb), the equilibrium moments
that the Chapman-Enskog section relies on, the two moment constraints from
which the paper derives its forcing source term (Appendix, Eqs. CON1/CON2),
the BGK special case of that term, the orthogonality of the mode basis, and
the published Philox4x32-10 known-answer vectors.
"""
import itertools
import os

import numpy as np
import pytest

import oracle

CS2 = 1.0 / 3.0
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_velocity_set_is_d3q19():
    c, w = oracle.lattice()
    # Eq. velo: rest, the 6 axis links, the 12 face diagonals, each once
    got = sorted(map(tuple, c))
    want = sorted([(0, 0, 0)] + [v for v in itertools.product((-1, 0, 1), repeat=3)
                                 if sum(map(abs, v)) in (1, 2)])
    assert got == want
    # Eq. weights
    for i in range(19):
        n = int(np.abs(c[i]).sum())
        assert w[i] == {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}[n]
    # opposite pairs adjacent (exact cancellation order used everywhere)
    for k in range(9):
        assert tuple(c[2 * k + 1]) == tuple(-c[2 * k + 2])


def test_isotropy():
    c, w = oracle.lattice()
    c = c.astype(float)
    d = np.eye(3)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(np.einsum("i,ia->a", w, c)).max() < 1e-16
    assert np.abs(np.einsum("i,ia,ib->ab", w, c, c) - CS2 * d).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib,ig->abg", w, c, c, c)).max() < 1e-16
    delta4 = (np.einsum("ab,gd->abgd", d, d) + np.einsum("ag,bd->abgd", d, d)
              + np.einsum("ad,bg->abgd", d, d))
    assert np.abs(np.einsum("i,ia,ib,ig,id->abgd", w, c, c, c, c) - CS2 ** 2 * delta4).max() < 1e-15


def test_mode_basis_orthogonal_and_hydrodynamic():
    c, w = oracle.lattice()
    e, b = oracle.mode_basis()
    gram = (e * w) @ e.T
    assert np.abs(gram - np.diag(b)).max() < 1e-15
    assert np.all(b > 0)
    # first modes: mass and momentum (Appendix: m_0 = rho, m_1..3 = momentum)
    assert np.all(e[0] == 1.0)
    assert np.array_equal(e[1:4], c.T.astype(float))
    # inverse transform f_i = w_i sum_k e_ki m_k / b_k reproduces any f
    f = np.random.default_rng(0).random(19)
    m = e @ f
    back = w * (e.T @ (m / b))
    assert np.abs(back - f).max() < 1e-15


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(seed):
    """sum f^eq = rho, sum f^eq c = rho u, sum f^eq c c = rho c_s^2 1 + rho u u.
    The last one fixes the c_s^2 in the second-order term of Eq. feq."""
    g = np.random.default_rng(seed)
    rho = 0.5 + g.random()
    u = 0.1 * (g.random(3) - 0.5)
    c, w = oracle.lattice()
    c = c.astype(float)
    feq = oracle.equilibrium(rho, u)
    assert abs(feq.sum() - rho) < 1e-15
    assert np.abs(feq @ c - rho * u).max() < 1e-16
    P = np.einsum("i,ia,ib->ab", feq, c, c)
    assert np.abs(P - rho * CS2 * np.eye(3) - rho * np.outer(u, u)).max() < 1e-15


@pytest.mark.parametrize("lams", [(-0.7, -1.3, -0.4), (-1.0, -1.0, -1.0), (-1.8, -0.6, -1.1)])
def test_forcing_term_moment_constraints(lams):
    """Constraints CON1 and CON2 of the Appendix, with distinct eigenvalues so
    that a swapped lambda is caught:
      sum_i Delta^g = 0
      sum_i c Delta^g = (2+lam_M)/2 g
      traceless part of sum_i c c Delta^g = (2+lam_s)/2 (u g + g u) traceless
      trace of sum_i c c Delta^g = (2+lam_b) u.g"""
    lam_m, lam_s, lam_b = lams
    g_ = np.random.default_rng(1)
    u = 0.05 * (g_.random(3) - 0.5)
    gf = 1e-3 * (g_.random(3) - 0.5)
    c, w = oracle.lattice()
    c = c.astype(float)
    dg = oracle.forcing_term(lam_m, lam_s, lam_b, u, gf)
    assert abs(dg.sum()) < 1e-18
    assert np.abs(dg @ c - 0.5 * (2 + lam_m) * gf).max() < 1e-18
    S = np.einsum("i,ia,ib->ab", dg, c, c)
    ug = u @ gf
    sym = np.outer(u, gf) + np.outer(gf, u)
    tl = lambda A: A - np.trace(A) / 3 * np.eye(3)
    assert np.abs(tl(S) - 0.5 * (2 + lam_s) * tl(sym)).max() < 1e-18
    assert abs(np.trace(S) - (2 + lam_b) * ug) < 1e-18


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_forcing_term_bgk_is_guo(tau):
    """All eigenvalues -1/tau: the term reduces to the textbook BGK forcing
    (1 - 1/(2 tau)) w_i [3 (c_i - u).g + 9 (u.c_i)(c_i.g)]."""
    lam = -1.0 / tau
    g_ = np.random.default_rng(2)
    u = 0.05 * (g_.random(3) - 0.5)
    gf = 1e-3 * (g_.random(3) - 0.5)
    c, w = oracle.lattice()
    c = c.astype(float)
    dg = oracle.forcing_term(lam, lam, lam, u, gf)
    guo = (1 - 0.5 / tau) * w * (3 * (c - u) @ gf + 9 * (c @ u) * (c @ gf))
    assert np.abs(dg - guo).max() < 1e-19


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat())
def test_philox_known_answers(ctr, key, want):
    assert list(oracle.philox(ctr, key)) == want


def test_normals_statistics_and_independence():
    import scipy.stats
    z = np.concatenate([oracle.site_normals(7, 3, i, 0, 9) for i in range(20000)])
    # 720k draws: 5-sigma bounds on mean, variance and excess kurtosis
    assert abs(z.mean()) < 0.006
    assert abs(z.var() - 1) < 0.009
    assert abs(scipy.stats.kurtosis(z)) < 0.03
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    # different tag / step / index give different streams
    a = oracle.site_normals(7, 3, 5, 0, 1)
    assert not np.allclose(a, oracle.site_normals(7, 3, 5, 1, 1))
    assert not np.allclose(a, oracle.site_normals(7, 4, 5, 0, 1))
    assert not np.allclose(a, oracle.site_normals(8, 3, 5, 0, 1))


def test_box_muller_special_values():
    # u2 = 1/2 - 2^-33 ... angle ~ pi: z0 ~ -r, z1 ~ 0; u1 with a = 2^31 gives r^2 ~ 2 ln 2
    z0, z1 = oracle.box_muller(1 << 31, (1 << 31) - 1)
    r = np.sqrt(-2 * np.log((2 ** 31 + 0.5) / 2 ** 32))
    assert abs(z0 + r) < 1e-9 and abs(z1) < 1e-8
    z0, z1 = oracle.box_muller(1 << 31, (1 << 30))  # angle ~ pi/2
    assert abs(z0) < 1e-8 and abs(z1 - r) < 1e-9


def test_interp_weights_reproduce_linear_fields():
    shape = (7, 5, 6)
    g = np.random.default_rng(3)
    for _ in range(200):
        x = g.random(3) * np.array(shape)
        node, W = oracle.interp_weights(x, shape)
        assert abs(W.sum() - 1) < 1e-15 and np.all(W >= 0)
        # position of each node, unwrapped next to floor(x)
        i0 = np.floor(x)
        pos = np.array([i0 + [k & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)])
        assert np.abs(W @ pos - x).max() < 1e-13
        # node indices are the wrapped corners
        wrapped = np.mod(pos.astype(int), shape)
        idx = (wrapped[:, 2] * shape[1] + wrapped[:, 1]) * shape[0] + wrapped[:, 0]
        assert np.array_equal(idx, node)


def test_interp_on_node_and_cell_centre():
    node, W = oracle.interp_weights(np.array([2.0, 3.0, 4.0]), (8, 8, 8))
    assert W[0] == 1.0 and np.all(W[1:] == 0.0)
    node, W = oracle.interp_weights(np.array([2.5, 3.5, 4.5]), (8, 8, 8))
    assert np.all(W == 0.125)


@pytest.mark.parametrize("kind,qq", [(0, 0.0), (1, 1.0), (1, -2.0), (2, 0.0)])
def test_pair_force_is_minus_energy_derivative(kind, qq):
    P = oracle.make_params((10, 10, 10), wca=(1.0, 1.0), fene=(30.0, 1.5), dh=(1.0, 3.0, 1.0))
    rs = {0: np.linspace(0.85, 1.12, 30), 1: np.linspace(0.5, 2.9, 30), 2: np.linspace(0.3, 1.45, 30)}[kind]
    for r in rs:
        h = 1e-6
        num = -(oracle.pair_energy(P, kind, r + h, qq) - oracle.pair_energy(P, kind, r - h, qq)) / (2 * h)
        ana = oracle.pair_force(P, kind, r, qq)
        assert abs(num - ana) <= 1e-6 * max(1.0, abs(ana))
    if kind == 0:  # WCA: zero energy and force at and beyond 2^(1/6) sigma
        rc = 2 ** (1 / 6)
        assert abs(oracle.pair_energy(P, 0, rc * (1 - 1e-12))) < 1e-9
        assert oracle.pair_force(P, 0, rc * 1.0001) == 0.0
    if kind == 2:  # FENE diverges at R0
        assert np.isnan(oracle.pair_force(P, 2, 1.5))


def test_conservative_forces_antisymmetric():
    P = oracle.make_params((12, 12, 12), wca=(1.0, 1.0), fene=(30.0, 1.5), dh=(1.0, 3.0, 1.0),
                           charge=(1.0, -1.0), mass=(1.0, 1.0), kappa=((0, 0), (0, 0)))
    g = np.random.default_rng(4)
    x = g.random((40, 3)) * 12
    t = g.integers(0, 2, 40).astype(np.int32)
    bonds = np.array([[i, i + 1] for i in range(0, 39, 2)], np.int32)
    x[1::2] = np.mod(x[0::2] + 0.9 * np.array([1, 0, 0]), 12)  # bonded partners at 0.9
    st, F = oracle.conservative_forces(P, x, t, bonds)
    assert st == oracle.OK
    assert np.abs(F.sum(axis=0)).max() < 1e-10 * np.abs(F).max()
    # one-particle version agrees with the all-particle one
    for p in (0, 7, 39):
        st1, Fp = oracle.conservative_force_one(P, x, p, t, bonds)
        assert np.array_equal(Fp, F[p])


@pytest.mark.parametrize("lB", [0.6, 1.0, 2.3])
def test_debye_hueckel_bjerrum_length_and_cutoff_energy(lB):
    """Screened electrostatics in the paper's reduced units.

    * Sec. 3 (remapping to physical units): the Bjerrum length l_B is the
      distance at which two unit charges interact with an energy of kT (= 1
      here), so the unscreened pair energy of q_i = q_j = 1 at r = l_B is 1.
    * Sec. 4 (polyelectrolytes): with screening length kappa_D^-1 = 4 l_B and
      cut-off r_c = 6 l_B the screened energy of an ion pair at the cut-off is
      about 0.04 kT -- for every l_B, since only r / l_B enters.
    Both fail if the l_B prefactor is dropped or misplaced."""
    P = oracle.make_params((40, 40, 40), dh=(0.0, 10.0, lB))
    assert abs(oracle.pair_energy(P, 1, lB, 1.0) - 1.0) < 1e-14
    assert abs(oracle.pair_energy(P, 1, lB, -1.0) + 1.0) < 1e-14
    P = oracle.make_params((40, 40, 40), dh=(1.0 / (4.0 * lB), 6.0 * lB, lB))
    u_cut = oracle.pair_energy(P, 1, 6.0 * lB * (1.0 - 1e-12), 1.0)
    assert round(u_cut, 2) == 0.04
    assert oracle.pair_energy(P, 1, 6.0 * lB, 1.0) == 0.0  # zero at and beyond r_c


@pytest.mark.parametrize("lB,qq", [(0.6, -2.5), (2.3, 4.0)])
def test_debye_hueckel_force_with_bjerrum_length_and_charges(lB, qq):
    """Radial DH force = -dU/dr (central differences of the pinned energy) at
    l_B != 1 and q_i q_j != 1, and linear in both l_B and q_i q_j."""
    P = oracle.make_params((40, 40, 40), dh=(0.8, 3.0, lB))
    P1 = oracle.make_params((40, 40, 40), dh=(0.8, 3.0, 1.0))
    for r in np.linspace(0.4, 2.95, 25):
        h = 1e-6
        num = -(oracle.pair_energy(P, 1, r + h, qq) - oracle.pair_energy(P, 1, r - h, qq)) / (2 * h)
        ana = oracle.pair_force(P, 1, r, qq)
        assert abs(num - ana) <= 1e-6 * max(1.0, abs(ana))
        assert abs(ana - lB * qq * oracle.pair_force(P1, 1, r, 1.0)) <= 1e-13 * abs(ana)
    # like charges repel: positive radial force
    assert oracle.pair_force(P, 1, 1.0, abs(qq)) > 0.0
