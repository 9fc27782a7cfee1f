"""lbmd_get_fields_noalloc against lbmd_get_fields, through the C ABI.

Two calls in a row on one GPU, the second on a smaller lattice, each with
host and device outputs, must give the same float64 values as the
allocating entry point (same kernels on the same state: bit for bit); a
request beyond the static scratch is refused with LBMD_EINVAL."""
import numpy as np
import pytest
import torch

from paper_1306_0788_amd import lbmd
from parity_cases import Case

pytestmark = pytest.mark.gpu


def _check(sim, mask):
    want = sim.get_fields(mask)
    got = sim.get_fields_noalloc(mask)
    assert np.array_equal(got, want)
    dev = torch.empty(want.size, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    sim.get_fields_noalloc(mask, dev.data_ptr())
    assert sim.sync() == lbmd.OK
    assert np.array_equal(dev.cpu().numpy(), want)


def test_noalloc_fields_match_get_fields_twice_then_smaller():
    torch.cuda.set_device(0)
    big = Case((40, 36, 30), lbmd.FP32, lbmd.FORCE_PAPER, lbmd.KERNEL_AUTO, G=1.5, gamma=0.8, npart=60,
               kappa=((0.1, -0.1),), mass=(5.0,))
    print("noalloc: 40x36x30 FP32", flush=True)
    a = big.gpu_sim()
    a.step(4)
    assert a.sync() == lbmd.OK
    _check(a, lbmd.RHO | lbmd.U)
    _check(a, lbmd.RHO | lbmd.U | lbmd.POP)
    small = Case((17, 9, 11), lbmd.FP64, lbmd.FORCE_PAPER, lbmd.KERNEL_AUTO, G=1.2, gamma=0.5, npart=8)
    print("noalloc: 17x9x11 FP64", flush=True)
    b = small.gpu_sim()
    b.step(3)
    assert b.sync() == lbmd.OK
    _check(b, lbmd.RHO | lbmd.U | lbmd.POP)
    _check(b, lbmd.U)
    a.close()
    b.close()


def test_noalloc_refuses_requests_beyond_the_scratch():
    print("noalloc: 64^3 populations refused", flush=True)
    s = Case((64, 64, 64), lbmd.FP32, npart=0).gpu_sim()
    with pytest.raises(lbmd.LbmdError) as e:
        s.get_fields_noalloc(lbmd.POP)  # 38 * 8 B per site for the host staging: ~80 MB
    assert e.value.code == lbmd.EINVAL
    # the field export to a device pointer needs only the density field
    dev = torch.empty(2 * s.N, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    s.get_fields_noalloc(lbmd.RHO, dev.data_ptr())
    assert s.sync() == lbmd.OK
    assert np.array_equal(dev.cpu().numpy(), s.get_fields(lbmd.RHO))
    s.close()
