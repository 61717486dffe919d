"""GPU parity with a caller-supplied perturbation: eps V_I given as a device
array at every grid point, in FP64 (hfgpe_set_potential) or FP32
(hfgpe_set_potential_f32), against the oracle given the same values (for
FP32, the rounded values written out in FP64)."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-11, "c64": 5e-5}


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_1007_3470_amd as p
    p.load()
    return p


def potential(inst, k=0):
    """A non-separable potential on the instance's grid (not a product of
    per-axis factors)."""
    m = inst.mesh()
    if inst.ndim == 1:
        x = m[0]
        v = 0.05 * x * np.sin(x + 0.1 * k) + 0.01 * np.abs(x)
    elif inst.ndim == 2:
        x, y = m
        v = 0.2 * (x + y) + 0.02 * np.cos(x * y) + 0.01 * k
    else:
        x, y, z = m
        v = 0.1 * (x - y + 0.5 * z) + 0.02 * np.cos(x * y + z)
    return np.broadcast_to(v, inst.shape).copy()


def run(pkg, w, dtype, vis, nsteps=None, **kw):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, **kw)
    plan.set_potential(plan.pack_real(vis))
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, w.nsteps if nsteps is None else nsteps)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return plan, buf, plan.unpack(buf)


def check(w, got, vis, tol):
    for k, inst in enumerate(w.instances):
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps, vi=vis[k])
        err = W.rel_l2(got[k], ref)
        print("potential %dD k=%d N=%s rel_l2 %.3e" % (inst.ndim, k, inst.n[: inst.ndim], err), flush=True)
        assert err < tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_potential_1d_all_kernels(pkg, dtype):
    """Sizes that run the generic (N < 64), fixed-shape and N = 4096 kernels."""
    sizes = (32, 256, 1024, 4096)
    base = W.batch_1d(n_inst=8, sizes=sizes, nsteps=25, seed=6)
    insts = []
    for k, inst in enumerate(base.instances):
        n = sizes[k % 4]
        insts.append(replace(inst, n=(n, 1, 1), lo=(-n / 64.0, 0.0, 0.0), hi=(n / 64.0, 1.0, 1.0)))
    psis = [W._normalise(i, np.exp(-(i.axis(0) - 0.1) ** 2 / 2).astype(complex)) for i in insts]
    w = replace(base, instances=insts, psi0=psis)
    vis = [potential(i, k) for k, i in enumerate(insts)]
    _, _, got = run(pkg, w, dtype, vis)
    check(w, got, vis, TOL[dtype])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_potential_2d_3d(pkg, dtype):
    for w in (W.gpe_2d(n=64, n_inst=2, nsteps=12), W.gpe_3d(n=32, nsteps=3)):
        vis = [potential(i, k) for k, i in enumerate(w.instances)]
        _, _, got = run(pkg, w, dtype, vis)
        check(w, got, vis, TOL[dtype])


def test_potential_coupled_and_graph(pkg):
    w = W.coupled_2d(n=64, n_inst=2, nsteps=20)
    vis = [potential(i, k) for k, i in enumerate(w.instances)]
    _, _, direct = run(pkg, w, "c128", vis)
    check(w, direct, vis, 1e-11)
    _, _, graphed = run(pkg, w, "c128", vis, use_graph=True)
    for k in range(2):
        assert np.array_equal(graphed[k], direct[k])


def test_potential_energy_and_reset(pkg):
    import torch
    w = W.gpe_2d(n=64, n_inst=2, nsteps=5)
    vis = [potential(i, k) for k, i in enumerate(w.instances)]
    plan, buf, got = run(pkg, w, "c128", vis)
    t = w.t0 + w.nsteps * w.dt
    en = plan.energy(buf, t)
    for k, inst in enumerate(w.instances):
        assert np.allclose(en[k], oracle.energy(inst, got[k], t, vi=vis[k]), rtol=1e-11, atol=1e-11)
    # NULL restores the factor form: same bits as a plan that never had a potential
    plan.set_potential(None)
    b2 = plan.pack(w.psi0)
    plan.evolve(b2, w.t0, w.nsteps)
    ref_plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, "c128", w.dt)
    b3 = ref_plan.pack(w.psi0)
    ref_plan.evolve(b3, w.t0, w.nsteps)
    torch.cuda.synchronize()
    for a, b in zip(plan.unpack(b2), ref_plan.unpack(b3)):
        assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# the FP32 form: the oracle takes the same (rounded) values in FP64
# ---------------------------------------------------------------------------
def run_f32(pkg, w, dtype, vis, **kw):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, **kw)
    plan.set_potential(plan.pack_real(vis).to(torch.float32))
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, w.nsteps)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return plan, buf, plan.unpack(buf)


def rounded(vis):
    return [np.asarray(v, dtype=np.float32).astype(np.float64) for v in vis]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_potential_f32_1d_2d_3d(pkg, dtype):
    base = W.batch_1d(n_inst=6, sizes=(32, 256, 1024, 4096), nsteps=20, seed=16)
    for w, kw in ((base, {}), (W.gpe_2d(n=64, n_inst=2, nsteps=12), {"use_graph": True}),
                  (W.gpe_3d(n=32, nsteps=3), {})):
        vis = rounded([potential(i, k) for k, i in enumerate(w.instances)])
        _, _, got = run_f32(pkg, w, dtype, vis, **kw)
        check(w, got, vis, TOL[dtype])


def test_potential_f32_energy_and_switch(pkg):
    """Energy with the FP32 array; switching to the FP64 array of the same
    values gives the same bits (the same doubles enter the phase)."""
    import torch
    w = W.coupled_2d(n=64, n_inst=2, nsteps=8)
    vis = rounded([potential(i, k) for k, i in enumerate(w.instances)])
    plan, buf, got = run_f32(pkg, w, "c128", vis)
    check(w, got, vis, 1e-11)
    t = w.t0 + w.nsteps * w.dt
    en = plan.energy(buf, t)
    for k, inst in enumerate(w.instances):
        assert np.allclose(en[k], oracle.energy(inst, got[k], t, vi=vis[k]), rtol=1e-11, atol=1e-11)
    plan.set_potential(plan.pack_real(vis))
    b2 = plan.pack(w.psi0)
    plan.evolve(b2, w.t0, w.nsteps)
    torch.cuda.synchronize()
    for a, b in zip(plan.unpack(b2), got):
        assert np.array_equal(a, b)
