"""Captured step sequences (HIP graphs) and the tiling autotuner.

A graph replays the same launches as the eager path, reading the step index
from the device counter, so without particles (no float atomics) the two
agree bit for bit (the push organisation to rounding: it adds the next
step's moments at box edges with float atomics); every replay is checked,
with eager steps and host synchronisation between replays.  With particles the float atomics of the
spread make the order of additions vary, so the graph run is compared with
the oracle at the eager tolerances instead."""
import os
import tempfile

import numpy as np
import pytest

from paper_1306_0788_amd import lbmd
from parity_cases import Case, compare

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kT", [0.0, 1e-4])
@pytest.mark.parametrize("kernel", [lbmd.KERNEL_FUSED, lbmd.KERNEL_TWOPASS, lbmd.KERNEL_PUSH])
def test_graph_replays_match_eager_bitwise(kT, kernel):
    c = Case((37, 29, 23), lbmd.FP32, lbmd.FORCE_PAPER, kernel, G=1.4, kT=kT, seed=5, npart=0)
    print("graph vs eager: kT=%g kernel=%d" % (kT, kernel), flush=True)
    a = c.gpu_sim()
    b = c.gpu_sim()
    b.set_graph(True)
    for chunk in (4, 3, 6, 1, 2):
        a.step(chunk)
        b.step(chunk)
        assert a.sync() == lbmd.OK and b.sync() == lbmd.OK
        assert a.step_index == b.step_index
        pa, pb = a.populations(), b.populations()
        ra, sa = a.reductions()
        rb, sb = b.reductions()
        assert sa == sb
        if kernel == lbmd.KERNEL_PUSH:
            # the push pass adds to the next step's moments at box edges with
            # float atomics in varying order: equal to rounding, not bitwise
            e = np.max(np.abs(pa - pb) / np.abs(pb))
            assert e <= 1e-5 * a.step_index, "after %d steps: %.2e" % (a.step_index, e)
            # FP32 sums over c.N sites of values that differ by rounding:
            # masses to 1e-6 relative, the (nearly cancelling) momenta to a
            # random walk of 38 populations' rounding per site
            assert np.abs(ra[:2] - rb[:2]).max() <= 1e-6 * np.abs(rb[:2]).max()
            assert np.abs(ra[2:5] - rb[2:5]).max() <= np.sqrt(c.N) * 38 * 2.0 ** -24 * 0.1 * a.step_index
        else:
            assert np.array_equal(pa, pb), "after %d steps" % a.step_index
            assert np.array_equal(ra, rb)


@pytest.mark.parametrize("precision,tol", [(lbmd.FP64, 1e-11), (lbmd.FP32, 1e-5)])
def test_graph_with_particles_pairs_and_bonds_matches_oracle(precision, tol):
    """Chains with FENE + WCA + Debye-Hueckel (pair forces on the second
    stream), fluctuating fluid, solvation: 6 steps as 3 graph replays."""
    c = Case((24, 24, 24), precision, lbmd.FORCE_PAPER, lbmd.KERNEL_TWOPASS, G=1.8, gamma=1.0, kT=1e-4, seed=3,
             chains=(6, 20), kappa=((0.1, 0.0),), mass=(2000.0,), charge=(1.0,), wca=(1.0, 1.0),
             fene=(30.0, 1.5), dh=(1.0, 3.0, 1.0))
    print("graph with particles, precision %d" % precision, flush=True)
    g = c.gpu_sim()
    g.set_graph(True)
    o = c.oracle_sim()
    g.step(6)
    assert o.step(6) == 0
    assert g.sync() == lbmd.OK, g.last_error()
    compare(c, g, o, tol * 10, tol * 10, "graph chains")


def test_graph_recaptured_after_tiling_change_and_particles():
    c = Case((33, 17, 12), lbmd.FP64, lbmd.FORCE_PAPER, lbmd.KERNEL_FUSED, G=1.3, gamma=0.7, npart=20,
             vel_amp=0.02, kappa=((0.2, 0.1),), mass=(3.0,))
    print("graph recapture", flush=True)
    g = c.gpu_sim()
    g.set_graph(True)
    o = c.oracle_sim()
    g.step(4)
    g.set_tiling(4, 5, 0, 1, 1)
    g.step(5)
    assert o.step(9) == 0
    assert g.sync() == lbmd.OK
    compare(c, g, o, 1e-11, 1e-11, "graph recapture")


@pytest.mark.parametrize("kernel", [lbmd.KERNEL_FUSED, lbmd.KERNEL_TWOPASS, lbmd.KERNEL_PUSH])
def test_autotune_leaves_state_and_results_unchanged(kernel):
    c = Case((70, 33, 21), lbmd.FP32, lbmd.FORCE_PAPER, kernel, G=1.3, gamma=0.7, npart=30, vel_amp=0.02,
             kappa=((0.2, 0.1),), mass=(3.0,))
    print("autotune kernel=%d" % kernel, flush=True)
    a = c.gpu_sim()
    a.step(2)
    before = a.populations()
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tiles.txt")
        ty, tz, flags, ms = a.autotune(reps=2, cache_path=path)
        print("chosen tile_y %d tile_z %d flags %d: %.4f ms per pass pair" % (ty, tz, flags, ms), flush=True)
        assert ty in (2, 4, 8, 16) and 1 <= tz <= 21 and ms > 0
        assert np.array_equal(a.populations(), before)
        assert a.step_index == 2
        # the cache answers the same key without timing
        b = c.gpu_sim()
        assert b.autotune(reps=2, cache_path=path)[:3] == (ty, tz, flags)
        assert open(path).read().count("\n") == 1
    o = c.oracle_sim()
    a.step(3)
    assert o.step(5) == 0
    assert a.sync() == lbmd.OK
    # five FP32 steps: the one-step FP32 bound (1e-5) times the step count
    compare(c, a, o, 5e-5, 5e-5, "after autotune")


@pytest.mark.parametrize("precision", [lbmd.FP64, lbmd.FP32, lbmd.BF16DEV])
def test_stream_ceiling_leaves_state_unchanged(precision):
    """The pattern-ceiling pass writes only the scratch buffer: populations,
    step index and the next steps are those of a handle that never ran it."""
    # no particles: no float atomics, so two handles agree bit for bit
    c = Case((70, 33, 21), precision, lbmd.FORCE_PAPER, lbmd.KERNEL_TWOPASS, G=1.3, npart=0)
    print("stream ceiling precision=%d" % precision, flush=True)
    a, b = c.gpu_sim(), c.gpu_sim()
    a.step(2)
    b.step(2)
    before = a.populations()
    ms = a.stream_ceiling(3)
    assert ms > 0
    assert np.array_equal(a.populations(), before) and a.step_index == 2
    a.step(3)
    b.step(3)
    assert a.sync() == lbmd.OK and b.sync() == lbmd.OK
    assert np.array_equal(a.populations(), b.populations())
