"""The Python binding's checks on what it hands to the library as device
pointers (they must hold under python -O, so they are not asserts), and the
chaining of a failing stage callback's exception."""
import subprocess
import sys

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


def test_buffer_checks(pkg):
    import torch
    w = W.gpe_1d(n=256, nsteps=2)
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, "c128", w.dt)
    good = plan.pack(w.psi0)
    with pytest.raises(TypeError):
        plan.evolve(good.to(torch.complex64), 0.0, 1)        # wrong element type
    with pytest.raises(ValueError):
        plan.evolve(good[:100].clone(), 0.0, 1)                # too short
    with pytest.raises(ValueError):
        plan.evolve(torch.stack([good, good], 1)[:, 0], 0.0, 1)  # strided view
    with pytest.raises(TypeError):
        plan.evolve(good.cpu(), 0.0, 1)                        # host tensor
    with pytest.raises(ValueError):
        plan.pack([np.zeros(17, complex)])
    with pytest.raises(TypeError):
        plan.set_potential(torch.zeros(256, dtype=torch.float16, device="cuda"))
    with pytest.raises(ValueError):
        plan.set_potential(torch.zeros(255, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        plan.set_potential(torch.zeros(255, dtype=torch.float32, device="cuda"))
    plan.set_potential(None)
    plan.evolve(good, 0.0, 2)
    torch.cuda.synchronize()
    assert plan.device_status() == 0


def test_buffer_checks_hold_under_optimised_python(pkg):
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import torch, workloads as W, paper_1007_3470_amd as p\n"
            "w = W.gpe_1d(n=256, nsteps=1)\n"
            "plan = p.Plan(w.instances, w.scheme, w.ho_rule, 'c128', w.dt)\n"
            "b = plan.pack(w.psi0).to(torch.complex64)\n"
            "try:\n"
            "    plan.evolve(b, 0.0, 1)\n"
            "except TypeError:\n"
            "    print('rejected')\n" % (pkg.__file__.rsplit('/', 2)[0],))
    r = subprocess.run([sys.executable, "-O", "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert "rejected" in r.stdout


def test_callback_exception_is_chained(pkg):
    w = W.gpe_1d(n=128, nsteps=3)
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, "c128", w.dt)

    def bad(inst, axis, t0, tau, mu):
        raise ZeroDivisionError("no coefficients here")
    plan.set_stage_callback(bad)
    with pytest.raises(pkg.HfgpeError) as e:
        plan.evolve(plan.pack(w.psi0), 0.0, 3)
    assert isinstance(e.value.__cause__, ZeroDivisionError)


def test_misaligned_buffers_are_rejected(pkg):
    """A raw C caller that passes a pointer off its element alignment gets
    INVALID_ARG before any work is enqueued; the buffer is untouched."""
    import ctypes
    import torch
    w = W.gpe_1d(n=256, nsteps=2)
    for dtype, size in (("c128", 16), ("c64", 8)):
        plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt)
        big = torch.zeros(int(plan.offsets[-1]) + 1, dtype=plan.torch_dtype, device="cuda")
        big[:int(plan.offsets[-1])] = plan.pack(w.psi0)
        before = big.clone()
        off = ctypes.c_void_p(big.data_ptr() + size // 2)
        assert plan.lib.hfgpe_evolve(plan.handle, off, 0.0, 2) == -1
        out = (ctypes.c_double * 4)()
        assert plan.lib.hfgpe_norm(plan.handle, off, out) == -1
        assert plan.lib.hfgpe_energy(plan.handle, off, 0.0, out) == -1
        torch.cuda.synchronize()
        assert torch.equal(big, before)
        assert plan.device_status() == 0
    vi = torch.zeros(int(plan.offsets[-1]) + 1, dtype=torch.float64, device="cuda")
    assert plan.lib.hfgpe_set_potential(plan.handle, ctypes.c_void_p(vi.data_ptr() + 4)) == -1
