"""Checkpoint and resume through lbmd_get_state / lbmd_set_state.

100 steps straight must equal 50 steps, a state round trip, and 50 more:
bit for bit where the step is deterministic (no particles: no float atomics),
within the FP64 parity tolerance with particles (the spread's float atomics
may add in another order), and with kT > 0 on the same random draws (the
Philox counter holds the step index, which the state carries).  The resumed
run is also checked against the oracle."""
import numpy as np
import pytest

from paper_1306_0788_amd import lbmd
from parity_cases import Case, compare, rel_err

pytestmark = pytest.mark.gpu


def _run_split(c, first, second, fresh=True, graph=False):
    a = c.gpu_sim()
    a.step(first)
    assert a.sync() == lbmd.OK, a.last_error()
    blob = a.get_state()
    if fresh:
        b = c.gpu_sim()
        b.set_state(blob)
        a.close()
    else:
        a.step(7)  # move on, then come back
        a.set_state(blob)
        b = a
    if graph:
        b.set_graph(True)
    assert b.step_index == first
    b.step(second)
    assert b.sync() == lbmd.OK, b.last_error()
    return b


@pytest.mark.parametrize("kT", [0.0, 1e-4])
@pytest.mark.parametrize("kernel", [lbmd.KERNEL_FUSED, lbmd.KERNEL_TWOPASS])
@pytest.mark.parametrize("fresh", [True, False])
def test_resume_without_particles_is_bitwise(kT, kernel, fresh):
    c = Case((19, 13, 11), lbmd.FP64, lbmd.FORCE_PAPER, kernel, G=1.4, kT=kT, seed=4, npart=0)
    print("state resume, no particles: kT=%g kernel=%d fresh=%d" % (kT, kernel, fresh), flush=True)
    ref = c.gpu_sim()
    ref.step(100)
    assert ref.sync() == lbmd.OK
    b = _run_split(c, 50, 50, fresh=fresh)
    assert b.step_index == 100
    assert np.array_equal(b.populations(), ref.populations())
    ra, sa = ref.reductions()
    rb, sb = b.reductions()
    assert sa == sb and np.array_equal(ra, rb)


@pytest.mark.parametrize("precision,tol", [(lbmd.FP64, 1e-11), (lbmd.FP32, 2e-5), (lbmd.BF16DEV, None)])
def test_resume_with_particles_and_noise(precision, tol):
    """Chains with FENE + WCA + Debye-Hueckel, fluctuating fluid, solvation:
    the resumed run matches the straight one and the oracle."""
    c = Case((24, 20, 18), precision, lbmd.FORCE_PAPER, lbmd.KERNEL_AUTO, G=1.6, gamma=1.0, kT=1e-4, seed=3,
             chains=(4, 12), kappa=((0.1, 0.0),), mass=(2000.0,), charge=(1.0,), wca=(1.0, 1.0),
             fene=(30.0, 1.5), dh=(1.0, 3.0, 1.0))
    print("state resume with particles, precision %d" % precision, flush=True)
    ref = c.gpu_sim()
    ref.step(40)
    assert ref.sync() == lbmd.OK
    b = _run_split(c, 20, 20, graph=True)
    if tol is None:
        # 16-bit deviation storage: the stored words are restored exactly and
        # the stochastic rounding is keyed by the step, so the two runs differ
        # only through the order of float atomic additions (the spread, and
        # the moments added at box edges); a last-bit difference can move a
        # stochastically rounded word by one bfloat16 step, up to 1/128 of the
        # deviation it stores (~1e-3 of f here), and 20 steps above the
        # spinodal with noise spread such steps
        e = rel_err(b.populations(), ref.populations())
        assert e < 2e-2, e
    else:
        assert rel_err(b.populations(), ref.populations()) <= tol
        o = c.oracle_sim()
        assert o.step(40) == 0
        compare(c, b, o, tol * 10, tol * 10, "resumed")
    xa, va, Fa, Fca = ref.particles()
    xb, vb, Fb, Fcb = b.particles()
    # the same float-atomic ordering reaches the particles through the fluid
    xtol = 1e-9 if precision == lbmd.FP64 else 1e-6
    assert np.abs(xa - xb).max() < xtol and np.abs(Fa - Fb).max() < 1e-4 * max(1.0, np.abs(Fa).max())


def test_state_errors_and_particle_count_change():
    c = Case((12, 10, 8), lbmd.FP64, lbmd.FORCE_PAPER, lbmd.KERNEL_AUTO, G=1.2, gamma=0.5, npart=10)
    print("state errors", flush=True)
    a = c.gpu_sim()
    a.step(3)
    blob = a.get_state()
    # another lattice size or precision is refused and leaves the handle usable
    other = Case((12, 10, 9), lbmd.FP64).gpu_sim()
    with pytest.raises(lbmd.LbmdError) as e:
        other.set_state(blob)
    assert e.value.code == lbmd.EINVAL
    other32 = Case((12, 10, 8), lbmd.FP32).gpu_sim()
    with pytest.raises(lbmd.LbmdError):
        other32.set_state(blob)
    with pytest.raises(lbmd.LbmdError):
        a.set_state(blob[:100])
    bad = blob.copy()
    bad[0] ^= 0xff
    with pytest.raises(lbmd.LbmdError):
        a.set_state(bad)
    # a handle with no particles takes the blob's particles
    fresh = Case((12, 10, 8), lbmd.FP64, lbmd.FORCE_PAPER, lbmd.KERNEL_AUTO, G=1.2, gamma=0.5, npart=0).gpu_sim()
    fresh.set_state(blob)
    assert fresh.np == 10 and fresh.step_index == 3
    fresh.step(5)
    a.step(5)
    assert fresh.sync() == lbmd.OK and a.sync() == lbmd.OK
    assert rel_err(fresh.populations(), a.populations()) < 1e-12
    assert np.abs(fresh.particles()[0] - a.particles()[0]).max() < 1e-12


def test_resume_after_numerical_failure():
    """Restoring a state saved before a failure clears the latch and steps on."""
    c = Case((16, 16, 16), lbmd.FP64, lbmd.FORCE_PAPER, lbmd.KERNEL_AUTO, G=2.4, amp=0.05, npart=0, seed=8)
    print("state resume after failure", flush=True)
    a = c.gpu_sim()
    blob = a.get_state()
    a.step(400)
    assert a.sync() == lbmd.EUNSTABLE
    a.set_state(blob)
    assert a.sync() == lbmd.OK and a.step_index == 0
    a.step(3)
    assert a.sync() == lbmd.OK
