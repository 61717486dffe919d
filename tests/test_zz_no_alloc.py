"""The allocation-free norm (hfgpe_norm_noalloc, for callers that cannot
allocate) against hfgpe_norm, through the C ABI: two calls in a row, the
second with a smaller input, and the size limit of the static scratch."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_1007_3470_amd as p
    p.load()
    return p


def noalloc_norm(pkg, plan, buf):
    import torch
    out = torch.full((plan.n_inst,), float("nan"), dtype=torch.float64, device="cuda")
    rc = plan.lib.hfgpe_norm_noalloc(plan.handle, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    assert rc == 0, rc
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check(pkg, w, dtype):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt)
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, 5)
    torch.cuda.synchronize()
    ref = plan.norm(buf)
    got = noalloc_norm(pkg, plan, buf)
    print("noalloc %s %d instances: max |diff| %.3e" % (dtype, len(w.instances), np.abs(got - ref).max()), flush=True)
    # the same compensated sums in the same order: equal to FP64 rounding
    assert np.allclose(got, ref, rtol=1e-15, atol=0.0)
    return plan, buf


def test_noalloc_norm_two_calls_second_smaller(pkg):
    big = W.batch_1d(n_inst=300, sizes=(64, 256, 1024, 4096), nsteps=5, seed=41)
    check(pkg, big, "c128")
    small = W.batch_1d(n_inst=7, sizes=(32, 128), nsteps=5, seed=42)
    check(pkg, small, "c64")


def test_noalloc_norm_nd(pkg):
    check(pkg, W.gpe_2d(n=256, n_inst=3, nsteps=5), "c64")     # several partial blocks per instance
    check(pkg, W.gpe_3d(n=32, nsteps=5), "c128")


def test_noalloc_norm_rejects_beyond_the_scratch(pkg):
    import torch
    # HFGPE_NOALLOC_SCRATCH_BYTES = 1 MiB: 32769 one-block instances need
    # 32769 * 32 bytes of partial sums, one more than it holds
    n = (1 << 20) // 32 + 1
    insts = [W.Instance(1, (64, 1, 1), (-1.0, 0.0, 0.0), (1.0, 1.0, 1.0))] * n
    plan = pkg.Plan(insts, "leapfrog", "cf4", "c64", 1e-3)
    buf = torch.zeros(n * 64, dtype=torch.complex64, device="cuda")
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    rc = plan.lib.hfgpe_norm_noalloc(plan.handle, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    assert rc == -9
    # and a plan at the limit is accepted
    plan2 = pkg.Plan(insts[: n - 1], "leapfrog", "cf4", "c64", 1e-3)
    rc = plan2.lib.hfgpe_norm_noalloc(plan2.handle, ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    assert rc == 0
    torch.cuda.synchronize()
    assert np.all(out[: n - 1].cpu().numpy() == 0.0)
