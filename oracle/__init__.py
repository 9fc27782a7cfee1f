"""Oracle for the two-component Shan-Chen LB fluid coupled to point particles.

TEST INFRASTRUCTURE ONLY.  A plain FP64 CPU statement of one time step of the
method of arXiv 1306.0788 (Sec. 2 and the Appendix), written in C (``orc.c``)
and wrapped here with ctypes.  Only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module; the GPU library never
does, and this module never imports the GPU library.

Every function here is checked by ``tests/test_oracle_*.py`` against
something other than itself: closed forms, invariants, values the paper
prints (the Debye-Hueckel energy at its cut-off, the definition of the
Bjerrum length), the relaxation factor of each mode group, equipartition,
published test vectors or brute force.  None is currently unpinned; a
function added without such a check must say "parity unpinned" in its
docstring.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FORCE_PAPER = 0
FORCE_SHIFT = 1
OK, EINVAL, EUNSTABLE = 0, -1, -4
Q = 19
MAXTYPES = 8


def build(force=True):
    """Compile orc.c into liboracle.so with gcc (strict IEEE, no fast-math, OpenMP)."""
    src = os.path.join(_HERE, "orc.c")
    if force or not os.path.exists(_LIBPATH) or os.path.getmtime(_LIBPATH) < os.path.getmtime(src):
        tmp = _LIBPATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIBPATH)
    return _LIBPATH


class Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("forcing", ctypes.c_int32), ("mrt", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("tau", ctypes.c_double * 2),
        ("lambda_bulk", ctypes.c_double), ("lambda_shear", ctypes.c_double),
        ("lambda_mom", ctypes.c_double), ("lambda_ghost", ctypes.c_double),
        ("G", (ctypes.c_double * 2) * 2),
        ("gamma", ctypes.c_double), ("kT", ctypes.c_double), ("seed", ctypes.c_uint64),
        ("ntypes", ctypes.c_int32), ("pad1", ctypes.c_int32),
        ("kappa", (ctypes.c_double * 2) * MAXTYPES),
        ("mass", ctypes.c_double * MAXTYPES), ("charge", ctypes.c_double * MAXTYPES),
        ("wca_on", ctypes.c_int32), ("fene_on", ctypes.c_int32), ("dh_on", ctypes.c_int32),
        ("pad2", ctypes.c_int32),
        ("wca_sigma", ctypes.c_double), ("wca_eps", ctypes.c_double),
        ("fene_k", ctypes.c_double), ("fene_R0", ctypes.c_double),
        ("dh_kappa", ctypes.c_double), ("dh_rc", ctypes.c_double), ("dh_lB", ctypes.c_double),
        ("lambda_fs", (ctypes.c_double * 2) * MAXTYPES),
    ]


def make_params(shape, tau=(1.0, 1.0), G=((0.0, 1.6), (1.6, 0.0)), forcing=FORCE_PAPER,
                gamma=0.0, kT=0.0, seed=0, kappa=((0.0, 0.0),), mass=(1.0,), charge=(0.0,),
                wca=None, fene=None, dh=None, mrt=None, lambda_fs=None):
    """Build the C parameter struct.  shape = (nx, ny, nz).
    wca = (sigma, eps); fene = (k, R0); dh = (kappa_D, r_c, l_B);
    mrt = (lambda_bulk, lambda_shear, lambda_mom, lambda_ghost) or None (BGK);
    lambda_fs = per-type (lambda_A, lambda_B) of the fluid solvation force."""
    p = Params()
    p.nx, p.ny, p.nz = (int(s) for s in shape)
    p.forcing = forcing
    p.tau[0], p.tau[1] = tau
    if mrt is not None:
        p.mrt = 1
        p.lambda_bulk, p.lambda_shear, p.lambda_mom, p.lambda_ghost = mrt
    for a in range(2):
        for b in range(2):
            p.G[a][b] = G[a][b]
    p.gamma, p.kT, p.seed = gamma, kT, seed
    p.ntypes = len(mass)
    for t in range(len(mass)):
        p.kappa[t][0], p.kappa[t][1] = kappa[t]
        p.mass[t] = mass[t]
        p.charge[t] = charge[t] if t < len(charge) else 0.0
    if wca is not None:
        p.wca_on, (p.wca_sigma, p.wca_eps) = 1, wca
    if fene is not None:
        p.fene_on, (p.fene_k, p.fene_R0) = 1, fene
    if dh is not None:
        p.dh_on, (p.dh_kappa, p.dh_rc, p.dh_lB) = 1, dh
    if lambda_fs is not None:
        for t in range(len(lambda_fs)):
            p.lambda_fs[t][0], p.lambda_fs[t][1] = lambda_fs[t]
    return p


_D = ctypes.POINTER(ctypes.c_double)
_I32 = ctypes.POINTER(ctypes.c_int32)
_I64 = ctypes.POINTER(ctypes.c_int64)
_U32 = ctypes.POINTER(ctypes.c_uint32)
_PP = ctypes.POINTER(Params)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            build()
        L = ctypes.CDLL(_LIBPATH)
        L.orc_lattice.argtypes = [_I32, _D]
        L.orc_set_threads.argtypes = [ctypes.c_int32]
        L.orc_get_threads.restype = ctypes.c_int32
        L.orc_mode_basis.argtypes = [_D, _D]
        L.orc_equilibrium.argtypes = [ctypes.c_double, _D, _D]
        L.orc_forcing_term.argtypes = [ctypes.c_double] * 3 + [_D, _D, _D]
        L.orc_philox4x32_10.argtypes = [_U32, _U32, _U32]
        L.orc_box_muller.argtypes = [ctypes.c_uint32, ctypes.c_uint32, _D, _D]
        L.orc_site_normals.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_int32, ctypes.c_int32, _D]
        L.orc_interp_weights.argtypes = [_D, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _I64, _D]
        L.orc_pair_energy.argtypes = [_PP, ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        L.orc_pair_energy.restype = ctypes.c_double
        L.orc_pair_force.argtypes = [_PP, ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        L.orc_pair_force.restype = ctypes.c_double
        L.orc_moments.argtypes = [_PP, _D, _D, _D, _D]
        L.orc_neighbour_sums.argtypes = [_PP, _D, _D]
        L.orc_init_populations.argtypes = [_PP, _D, _D]
        L.orc_step.argtypes = [_PP, ctypes.c_int64, _D, ctypes.c_int64, _D, _D, _D, _D, _I32,
                               ctypes.c_int64, _I32, _D]
        L.orc_step.restype = ctypes.c_int
        L.orc_conservative_forces.argtypes = [_PP, ctypes.c_int64, _D, _I32, ctypes.c_int64, _I32, _D]
        L.orc_conservative_forces.restype = ctypes.c_int
        L.orc_conservative_force_one.argtypes = [_PP, ctypes.c_int64, _D, _I32, ctypes.c_int64, _I32,
                                                 ctypes.c_int64, _D]
        L.orc_conservative_force_one.restype = ctypes.c_int
        L.orc_site_collide.argtypes = [_PP, ctypes.c_int64, _D, ctypes.c_int64, _D, _D]
        L.orc_site_collide.restype = ctypes.c_int
        L.orc_node_fields.argtypes = [_PP, _D, ctypes.c_int64, _D, _D]
        L.orc_coupling_force_one.argtypes = [_PP, ctypes.c_int64, _D, _D, _D, ctypes.c_int32, ctypes.c_int64, _D]
        L.orc_solvation_fluid_force.argtypes = [_PP, _D, ctypes.c_int64, _D, _I32, _D, _D]
        L.orc_particle_force_at.argtypes = [_PP, ctypes.c_int64, _D, ctypes.c_int64, _D, _D, _I32,
                                            ctypes.c_int64, _D]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _c64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def set_threads(n):
    """OpenMP threads of the oracle's site and particle loops (bit-identical
    results for any count)."""
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())


def lattice():
    c = np.zeros((Q, 3), np.int32)
    w = np.zeros(Q)
    lib().orc_lattice(c.ctypes.data_as(_I32), _dp(w))
    return c, w


def mode_basis():
    e = np.zeros((Q, Q))
    b = np.zeros(Q)
    lib().orc_mode_basis(_dp(e), _dp(b))
    return e, b


def equilibrium(rho, u):
    u = _c64(u)
    out = np.zeros(Q)
    lib().orc_equilibrium(float(rho), _dp(u), _dp(out))
    return out


def forcing_term(lam_mom, lam_shear, lam_bulk, u, g):
    u, g = _c64(u), _c64(g)
    out = np.zeros(Q)
    lib().orc_forcing_term(lam_mom, lam_shear, lam_bulk, _dp(u), _dp(g), _dp(out))
    return out


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data_as(_U32), k.ctypes.data_as(_U32), o.ctypes.data_as(_U32))
    return o


def box_muller(a, b):
    z0, z1 = ctypes.c_double(), ctypes.c_double()
    lib().orc_box_muller(a, b, ctypes.byref(z0), ctypes.byref(z1))
    return z0.value, z1.value


def site_normals(seed, step, index, tag, nblocks):
    z = np.zeros(4 * nblocks)
    lib().orc_site_normals(seed, step, index, tag, nblocks, _dp(z))
    return z


def interp_weights(x, shape):
    x = _c64(x)
    node = np.zeros(8, np.int64)
    W = np.zeros(8)
    lib().orc_interp_weights(_dp(x), shape[0], shape[1], shape[2], node.ctypes.data_as(_I64), _dp(W))
    return node, W


def pair_energy(P, kind, r, qq=0.0):
    return lib().orc_pair_energy(ctypes.byref(P), kind, r, qq)


def pair_force(P, kind, r, qq=0.0):
    return lib().orc_pair_force(ctypes.byref(P), kind, r, qq)


def nsites(P):
    return P.nx * P.ny * P.nz


def moments(P, f):
    N = nsites(P)
    f = _c64(f)
    rho = np.zeros((2, N))
    j = np.zeros((3, N))
    jc = np.zeros((2, 3, N))
    lib().orc_moments(ctypes.byref(P), _dp(f), _dp(rho), _dp(j), _dp(jc))
    return rho, j, jc


def neighbour_sums(P, rho):
    N = nsites(P)
    rho = _c64(rho)
    out = np.zeros((2, 3, N))
    lib().orc_neighbour_sums(ctypes.byref(P), _dp(rho), _dp(out))
    return out


def init_populations(P, rho):
    N = nsites(P)
    rho = _c64(rho).reshape(2, N)
    f = np.zeros((2, Q, N))
    lib().orc_init_populations(ctypes.byref(P), _dp(rho), _dp(f))
    return f


def conservative_forces(P, x, type_=None, bonds=None):
    x = _c64(x)
    n = x.shape[0]
    F = np.zeros((n, 3))
    t = None if type_ is None else np.ascontiguousarray(type_, np.int32)
    b = np.zeros((0, 2), np.int32) if bonds is None else np.ascontiguousarray(bonds, np.int32)
    st = lib().orc_conservative_forces(ctypes.byref(P), n, _dp(x),
                                       None if t is None else t.ctypes.data_as(_I32),
                                       b.shape[0], b.ctypes.data_as(_I32), _dp(F))
    return st, F


def conservative_force_one(P, x, p, type_=None, bonds=None):
    x = _c64(x)
    Fp = np.zeros(3)
    t = None if type_ is None else np.ascontiguousarray(type_, np.int32)
    b = np.zeros((0, 2), np.int32) if bonds is None else np.ascontiguousarray(bonds, np.int32)
    st = lib().orc_conservative_force_one(ctypes.byref(P), x.shape[0], _dp(x),
                                          None if t is None else t.ctypes.data_as(_I32),
                                          b.shape[0], b.ctypes.data_as(_I32), p, _dp(Fp))
    return st, Fp


def site_collide(P, step, f, site, gP=(0.0, 0.0, 0.0)):
    f = _c64(f)
    gP = _c64(gP)
    out = np.zeros((2, Q))
    st = lib().orc_site_collide(ctypes.byref(P), step, _dp(f), site, _dp(gP), _dp(out))
    if st != OK:
        raise ValueError("orc_site_collide: invalid parameters")
    return out


def node_fields(P, f, site):
    f = _c64(f)
    uc = np.zeros(3)
    grad = np.zeros((2, 3))
    lib().orc_node_fields(ctypes.byref(P), _dp(f), site, _dp(uc), _dp(grad))
    return uc, grad


def coupling_force_one(P, step, f, xp, vp, type_, p):
    Fc = np.zeros(3)
    lib().orc_coupling_force_one(ctypes.byref(P), step, _dp(_c64(f)), _dp(_c64(xp)), _dp(_c64(vp)), int(type_),
                                 int(p), _dp(Fc))
    return Fc


def particle_force_at(P, step, f, x, v, type_, site):
    """-sum_p W_p(site) F_coup,p (positions/velocities after the half kick and drift)."""
    gP = np.zeros(3)
    x, v = _c64(x), _c64(v)
    t = np.ascontiguousarray(type_, np.int32)
    lib().orc_particle_force_at(ctypes.byref(P), step, _dp(_c64(f)), x.shape[0], _dp(x), _dp(v),
                                t.ctypes.data_as(_I32), int(site), _dp(gP))
    return gP


class Sim:
    """Holds an oracle state and advances it with orc_step."""

    def __init__(self, P, rho_init, x=None, v=None, type_=None, bonds=None):
        self.P = P
        self.N = nsites(P)
        self.f = init_populations(P, rho_init)
        n = 0 if x is None else len(x)
        self.x = np.zeros((n, 3)) if x is None else _c64(x).copy()
        self.v = np.zeros((n, 3)) if v is None else _c64(v).copy()
        self.F = np.zeros((n, 3))
        self.Fc = np.zeros((n, 3))
        self.type = np.zeros(n, np.int32) if type_ is None else np.ascontiguousarray(type_, np.int32)
        self.bonds = np.zeros((0, 2), np.int32) if bonds is None else np.ascontiguousarray(bonds, np.int32)
        self.step_index = 0
        self.red = np.zeros(5)

    def step(self, n=1):
        st = OK
        for _ in range(n):
            st = lib().orc_step(ctypes.byref(self.P), self.step_index, _dp(self.f), self.x.shape[0],
                                _dp(self.x), _dp(self.v), _dp(self.F), _dp(self.Fc),
                                self.type.ctypes.data_as(_I32), self.bonds.shape[0],
                                self.bonds.ctypes.data_as(_I32), _dp(self.red))
            self.step_index += 1
            if st != OK:
                return st
        return st

    def rho(self):
        return moments(self.P, self.f)[0]

    def fluid_momentum(self):
        return moments(self.P, self.f)[1].sum(axis=1)


def solvation_fluid_force(P, rho, x, types=None):
    """Fluid solvation force of particles at x on the nodes, fs [2][3][N],
    and the momentum returned to each particle, back [n][3]."""
    N = P.nx * P.ny * P.nz
    rho = _c64(np.asarray(rho, dtype=np.float64).reshape(2, N))
    x = _c64(np.asarray(x, dtype=np.float64).reshape(-1, 3))
    n = len(x)
    t = None if types is None else np.ascontiguousarray(types, dtype=np.int32)
    fs = np.zeros((2, 3, N))
    back = np.zeros((max(n, 1), 3))
    lib().orc_solvation_fluid_force(ctypes.byref(P), rho.ctypes.data_as(_D), n, x.ctypes.data_as(_D),
                                     None if t is None else t.ctypes.data_as(_I32), fs.ctypes.data_as(_D),
                                     back.ctypes.data_as(_D))
    return fs, back[:n]
