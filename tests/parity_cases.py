"""Case builder for the GPU-vs-oracle parity tests: one seeded input set,
handed to the HIP library (through the C ABI) and to the oracle."""
import numpy as np

import oracle
from paper_1306_0788_amd import lbmd, workloads


def rel_err(a, b, floor=1e-300):
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor)))


def min_image_err(xg, xo, shape):
    L = np.asarray(shape, dtype=float)
    d = xg - xo
    d -= L * np.round(d / L)
    return float(np.max(np.abs(d))) if d.size else 0.0


class Case:
    def __init__(self, shape, precision=lbmd.FP64, forcing=lbmd.FORCE_PAPER, kernel=lbmd.KERNEL_FUSED,
                 G=1.6, tau=1.0, gamma=0.5, kappa=((0.0, 0.0),), mass=(1.0,), charge=(0.0,), kT=0.0, seed=1,
                 npart=64, min_dist=0.0, wca=None, fene=None, dh=None, chains=None, amp=0.01, vel_amp=0.0,
                 positions=None, tiling=None, lambda_fs=None, mrt=None):
        self.shape = tuple(shape)
        self.N = int(np.prod(shape))
        self.precision, self.forcing, self.kernel = precision, forcing, kernel
        self.G = ((0.0, G), (G, 0.0)) if np.isscalar(G) else G
        self.tau = (tau, tau) if np.isscalar(tau) else tau
        self.gamma, self.kappa, self.mass, self.charge, self.kT, self.seed = gamma, kappa, mass, charge, kT, seed
        self.wca, self.fene, self.dh = wca, fene, dh
        self.tiling = tiling
        self.lambda_fs = lambda_fs
        self.mrt = mrt
        self.rho = workloads.initial_densities(self.shape, seed, amp).reshape(2, -1)
        self.bonds = None
        if positions is not None:
            self.x = np.asarray(positions, dtype=float).reshape(-1, 3)
        elif chains is not None:
            self.x, self.bonds = workloads.chains(chains[0], chains[1], self.shape, seed, bond=0.97, min_dist=workloads.WCA_CUT)
        else:
            self.x = workloads.free_particles(npart, self.shape, seed, min_dist)
        n = len(self.x)
        g = np.random.default_rng(seed + 77)
        self.v = vel_amp * (g.random((n, 3)) - 0.5)
        self.type = (np.arange(n) % len(mass)).astype(np.int32)

    # ---- oracle side
    def oracle_params(self):
        return oracle.make_params(self.shape, tau=self.tau, G=self.G,
                                  forcing=oracle.FORCE_SHIFT if self.forcing == lbmd.FORCE_SHIFT else oracle.FORCE_PAPER,
                                  gamma=self.gamma, kT=self.kT, seed=self.seed, kappa=self.kappa, mass=self.mass,
                                  charge=self.charge, wca=self.wca, fene=self.fene, dh=self.dh,
                                  lambda_fs=self.lambda_fs, mrt=self.mrt)

    def oracle_sim(self):
        return oracle.Sim(self.oracle_params(), self.rho, self.x, self.v, self.type, self.bonds)

    # ---- GPU side
    def gpu_sim(self):
        s = lbmd.Sim(self.shape, precision=self.precision, forcing=self.forcing, kernel=self.kernel, tau=self.tau,
                     G=self.G, gamma=self.gamma, kappa=self.kappa[0], mass=self.mass[0], kT=self.kT, seed=self.seed,
                     rho_init=self.rho)
        s.set_particle_types(self.kappa, self.mass, self.charge)
        if self.wca is not None:
            s.set_pair_potential(lbmd.PAIR_WCA, self.wca)
        if self.dh is not None:
            s.set_pair_potential(lbmd.PAIR_DH, self.dh)
        if self.fene is not None:
            s.set_pair_potential(lbmd.BOND_FENE, self.fene)
        if len(self.x):
            s.set_particles(self.x, self.v, self.type)
        if self.bonds is not None:
            s.set_bonds(self.bonds)
        if self.tiling is not None:
            s.set_tiling(*self.tiling)
        if self.lambda_fs is not None:
            s.set_solvation_lambda(self.lambda_fs)
        if self.mrt is not None:
            s.set_mrt(self.mrt)
        return s


def compare(case, gs, os_, tol_pop, tol_part, what=""):
    """Populations element by element, then particles."""
    pg = gs.populations()
    po = os_.f.reshape(2, 19, -1)
    e = rel_err(pg, po)
    assert e <= tol_pop, "%s populations rel err %.3e > %.1e" % (what, e, tol_pop)
    if len(case.x):
        x, v, F, Fc = gs.particles()
        ex = min_image_err(x, os_.x, case.shape)
        sv = max(np.abs(os_.v).max(), 1e-3)
        sF = max(np.abs(os_.F).max(), 1e-6)
        ev = np.abs(v - os_.v).max() / sv
        eF = np.abs(F - os_.F).max() / sF
        eFc = np.abs(Fc - os_.Fc).max() / max(np.abs(os_.Fc).max(), 1e-6)
        assert ex <= tol_part * max(1.0, np.abs(os_.x).max()), "%s x err %.3e" % (what, ex)
        assert ev <= tol_part, "%s v err %.3e" % (what, ev)
        assert eF <= tol_part and eFc <= tol_part, "%s F err %.3e Fc err %.3e" % (what, eF, eFc)
    return e
