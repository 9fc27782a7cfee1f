"""GPU checks of the deviation storage forms: populations stored as
f_i - w_i rho0 in IEEE binary16 (FP16DEV) or bfloat16 (BF16DEV), all
arithmetic in FP32, compared with the FP64 oracle on the same seeded inputs.

Tolerances.  The initial state is rounded to nearest (error <= u |d_i|,
u = 2^-11 for binary16, 2^-8 for bfloat16, d_i = f_i - w_i rho0); every
step stores its output with stochastic rounding (error < 1 ulp = 2 u |d_i|,
unbiased).  Write D = max |d_i| / w_i over sites and velocities (the largest
deviation in density units).  With tau = 1 a step's output depends on its
inputs only through rho, j and the Shan-Chen force: input errors move rho by
at most u D, each momentum component by u D / 3 (sum_i w_i |c_ix| = 1/3)
and the neighbour sums by u D / 3, so population i moves by at most
w_i u D (1 + |c_i|_1 (1 + G/2)) (|c_i|_1 <= 2); adding the output rounding,
|f_gpu - f_oracle| / w_i < (3 + 2 (1 + G/2)) u D after one step: 6.6 u D at
G = 1.6, 6.3 u D at G = 1.3; the tests allow 7 u D.  Particle forces
inherit the node errors through the interpolation weights (sum 1): the
friction part by gamma times the velocity error (about 3 u D at rho ~ 1),
the solvation part by 3 sum|kappa| times the neighbour-sum error (about
u D); the tests allow 4 times (3 gamma + 3 sum|kappa|) u D.  Over many steps
the error grows with the Shan-Chen modes (x40 per 100 steps at G rho = 1.6,
as the FP64 round-off does); the 100-step bounds are 100 times the one-step
bound.
"""
import numpy as np
import pytest

from paper_1306_0788_amd import lbmd
from parity_cases import Case

pytestmark = pytest.mark.gpu

FP16DEV, BF16DEV = lbmd.FP16DEV, lbmd.BF16DEV
UNIT = {FP16DEV: 2.0 ** -11, BF16DEV: 2.0 ** -8}
W = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def weighted_dev(f, rho0=1.0):
    """max |f_i - w_i rho0| / w_i over a [2][19][N] population array."""
    return float(np.max(np.abs(f - W[None, :, None] * rho0) / W[None, :, None]))


def weighted_err(a, b):
    return float(np.max(np.abs(a - b) / W[None, :, None]))


def run(case, steps):
    print("deviation storage: shape=%s prec=%d kernel=%d steps=%d" % (case.shape, case.precision, case.kernel,
                                                                      steps), flush=True)
    g = case.gpu_sim()
    o = case.oracle_sim()
    f0 = o.f.reshape(2, 19, -1).copy()
    g.step(steps)
    assert o.step(steps) == 0
    assert g.sync() == lbmd.OK, g.last_error()
    return g, o, f0


@pytest.mark.parametrize("precision", [FP16DEV, BF16DEV])
@pytest.mark.parametrize("kernel", [lbmd.KERNEL_FUSED, lbmd.KERNEL_TWOPASS, lbmd.KERNEL_PUSH])
def test_one_step_against_oracle(precision, kernel):
    """The 32^3 mixture with 64 moving particles, one step."""
    G = 1.6
    c = Case((32, 32, 32), precision, lbmd.FORCE_PAPER, kernel, G=G, gamma=0.5, vel_amp=0.02,
             kappa=((0.3, -0.2),), mass=(2.0,))
    g, o, f0 = run(c, 1)
    f1 = o.f.reshape(2, 19, -1)
    u = UNIT[precision]
    D = max(weighted_dev(f0), weighted_dev(f1))
    err = weighted_err(g.populations(), f1)
    print("D = %.4g, weighted population error %.3e = %.2f u D" % (D, err, err / (u * D)), flush=True)
    assert err <= 7 * u * D
    x, v, F, Fc = g.particles()
    fscale = (3 * 0.5 + 3 * (0.3 + 0.2)) * u * D  # 3 gamma u D + 3 sum|kappa| u D
    eF = np.abs(Fc - o.Fc).max()
    print("particle coupling force error %.3e (scale %.3e)" % (eF, fscale), flush=True)
    assert eF <= 4 * fscale
    assert np.abs(F - o.F).max() <= 4 * fscale


@pytest.mark.parametrize("shape", [(37, 29, 23), (5, 3, 4)])
@pytest.mark.parametrize("precision", [FP16DEV, BF16DEV])
def test_ragged_shapes(shape, precision):
    c = Case(shape, precision, lbmd.FORCE_PAPER, lbmd.KERNEL_FUSED, G=1.3, gamma=0.7, npart=8, vel_amp=0.02,
             kappa=((0.2, 0.1),), mass=(3.0,), amp=0.03)
    g, o, f0 = run(c, 1)
    f1 = o.f.reshape(2, 19, -1)
    D = max(weighted_dev(f0), weighted_dev(f1))
    err = weighted_err(g.populations(), f1)
    print("ragged %s: %.2f u D" % (shape, err / (UNIT[precision] * D)), flush=True)
    assert err <= 7 * UNIT[precision] * D


@pytest.mark.parametrize("precision,growth", [(FP16DEV, 100.0), (BF16DEV, 100.0)])
@pytest.mark.parametrize("kernel", [lbmd.KERNEL_FUSED, lbmd.KERNEL_TWOPASS, lbmd.KERNEL_PUSH])
def test_hundred_steps_density(precision, growth, kernel):
    """Densities after 100 steps at G = 1.6 (above the spinodal): within the
    one-step bound times the growth of the unstable modes over 100 steps
    (x40 for FP64 round-off; x100 allowed), and the FP32 step beside it for
    reference."""
    c = Case((32, 32, 32), precision, lbmd.FORCE_PAPER, kernel, G=1.6, gamma=0.5, mass=(1.0,))
    g, o, f0 = run(c, 100)
    D = max(weighted_dev(f0), weighted_dev(o.f.reshape(2, 19, -1)))
    e = float(np.abs(g.rho() - o.rho()).max())
    c32 = Case((32, 32, 32), lbmd.FP32, lbmd.FORCE_PAPER, kernel, G=1.6, gamma=0.5, mass=(1.0,))
    g32 = c32.gpu_sim()
    g32.step(100)
    e32 = float(np.abs(g32.rho() - o.rho()).max())
    print("100 steps: max |rho - rho_oracle| %.3e (FP32 %.3e), D = %.3g, bound %.3e"
          % (e, e32, D, growth * 7 * UNIT[precision] * D), flush=True)
    assert e <= growth * 7 * UNIT[precision] * D


@pytest.mark.parametrize("precision", [FP16DEV, BF16DEV])
def test_mass_drift_is_rounding_sized(precision):
    """Rounding the stored deviations is not mass-conserving.  Stochastic
    rounding is unbiased per value, so the total mass of a component performs
    a random walk of step ~ 2 u D w sqrt(19 N) per step; after n steps its
    drift stays below n 2 u D sqrt(19 N) / 19 (n steps of that size in one
    direction, an upper bound for the walk), relative to the mass N rho."""
    shape = (24, 20, 16)
    c = Case(shape, precision, lbmd.FORCE_PAPER, lbmd.KERNEL_TWOPASS, G=1.4, gamma=0.8, npart=50, vel_amp=0.05,
             kappa=((0.3, -0.1),), mass=(400.0,), wca=(1.0, 0.05), min_dist=1.3)
    g = c.gpu_sim()
    g.step(1)
    r0, _ = g.reductions()
    n = 60
    g.step(n)
    r1, _ = g.reductions()
    N = c.N
    D = max(weighted_dev(g.populations()), 0.01)
    bound = n * 2 * UNIT[precision] * D * np.sqrt(19 * N) / 19 / N
    for comp in range(2):
        drift = abs(r1[comp] - r0[comp]) / r0[comp]
        print("component %d: relative mass drift over %d steps %.3e (bound %.3e)" % (comp, n, drift, bound),
              flush=True)
        assert drift <= bound


def test_rejects_bad_reference_density():
    with pytest.raises(lbmd.LbmdError):
        lbmd.Sim((8, 8, 8), precision=FP16DEV, rho0=0.0)
    with pytest.raises(lbmd.LbmdError):
        lbmd.Sim((8, 8, 8), precision=BF16DEV, rho0=float("nan"))


@pytest.mark.parametrize("precision", [FP16DEV, BF16DEV])
def test_stochastic_rounding_is_reproducible_across_tilings(precision):
    """The rounding draws depend only on the site, the velocity and the step,
    so two tilings of the same organisation give identical bits."""
    c = Case((37, 29, 23), precision, lbmd.FORCE_PAPER, lbmd.KERNEL_FUSED, G=1.4, npart=0)
    a = c.gpu_sim()
    b = c.gpu_sim()
    a.set_tiling(4, 16, 1, 0, 1)
    b.set_tiling(8, 5, 0, 1, 1)
    a.step(5)
    b.step(5)
    assert np.array_equal(a.populations(), b.populations())
