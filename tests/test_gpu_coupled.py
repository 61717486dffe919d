"""GPU parity of the coupled-trap path (off-diagonal W, non-separable drift)
against the CPU oracle, through the C ABI."""
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


def run_gpu(pkg, w, dtype, nsteps=None, **kw):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, **kw)
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, w.nsteps if nsteps is None else nsteps)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return plan, buf, plan.unpack(buf)


def say(*a):
    print(*a, flush=True)


def check(w, got, tol):
    for k, inst in enumerate(w.instances):
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        err = W.rel_l2(got[k], ref)
        say("coupled %dD %s %s k=%d rel_l2 %.3e" % (inst.ndim, w.scheme, w.ho_rule, k, err))
        assert err < tol


@pytest.mark.parametrize("rule", ["cf4", "fsplit"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_coupled_2d(pkg, rule, dtype):
    w = W.coupled_2d(n=64, n_inst=3, nsteps=20, rule=rule)
    _, _, got = run_gpu(pkg, w, dtype)
    check(w, got, TOL[dtype])


@pytest.mark.parametrize("scheme,rule", [("ni5_84", "cf4"), ("leapfrog", "fsplit"), ("srkn6_4", "cf4")])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_coupled_3d(pkg, scheme, rule, dtype):
    w = W.coupled_3d(n=32, nsteps=4, scheme=scheme, rule=rule)
    _, _, got = run_gpu(pkg, w, dtype)
    check(w, got, TOL[dtype])


def test_coupled_exact_rule_2d(pkg):
    """Constant W, exact rule: oracle parity and exactness on the rotated ground state."""
    w = W.coupled_2d(n=128, n_inst=2, nsteps=10, rule="exact_const", constant=True, dt=0.05)
    _, _, got = run_gpu(pkg, w, "c128")
    check(w, got, 1e-11)
    inst = replace(w.instances[0], sigma=(0.0, 0.0, 0.0, 0.0), eps=0.0, lo=(-9.0, -9.0, 0.0),
                   hi=(9.0, 9.0, 1.0))
    Wm = np.array([[inst.omega[0][0] ** 2, inst.wcross[0]], [inst.wcross[0], inst.omega[1][0] ** 2]])
    lam, Q = np.linalg.eigh(Wm)
    Om = Q @ np.diag(np.sqrt(lam)) @ Q.T
    X = np.stack([m * np.ones(inst.shape) for m in inst.mesh()], axis=-1)
    g0 = np.exp(-0.5 * inst.mu * np.einsum("...i,ij,...j->...", X, Om, X)).astype(complex)
    lin = replace(w, instances=[inst], psi0=[g0], dt=0.4, nsteps=6)
    _, _, out = run_gpu(pkg, lin, "c128")
    T = 0.4 * 6
    assert W.rel_l2(out[0], np.exp(-0.5j * T * np.sqrt(lam).sum()) * g0) < 1e-11


@pytest.mark.parametrize("shape", [(64, 16, 1), (8, 128, 1), (32, 1, 1), (1, 32, 1)])
def test_coupled_anisotropic_shapes(pkg, shape):
    base = W.coupled_2d(n=16, n_inst=2, nsteps=8)
    insts, psis = [], []
    for k, inst in enumerate(base.instances):
        i2 = replace(inst, n=shape, lo=(-6.0, -5.0, 0.0), hi=(7.0, 5.0, 1.0))
        x, y = i2.mesh()
        insts.append(i2)
        psis.append(W._normalise(i2, np.exp(-((x - 0.2 * k) ** 2 + 1.3 * y ** 2) / 2).astype(complex)))
    w = replace(base, instances=insts, psi0=psis)
    _, _, got = run_gpu(pkg, w, "c128")
    check(w, got, 1e-11)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_coupled_graph_replay(pkg, dtype):
    import torch
    w = W.coupled_2d(n=64, n_inst=2, nsteps=37)
    _, _, direct = run_gpu(pkg, w, dtype)
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, use_graph=True)
    for rep in range(2):
        buf = plan.pack(w.psi0)
        plan.evolve(buf, w.t0, w.nsteps)
        torch.cuda.synchronize()
        got = plan.unpack(buf)
        for k in range(2):
            assert np.array_equal(got[k], direct[k]), (rep, k)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_coupled_norm_energy(pkg, dtype):
    for w in (W.coupled_2d(n=64, n_inst=2, nsteps=6), W.coupled_3d(n=32, nsteps=2)):
        plan, buf, got = run_gpu(pkg, w, dtype)
        t = w.t0 + w.nsteps * w.dt
        nrm, en = plan.norm(buf), plan.energy(buf, t)
        for k, inst in enumerate(w.instances):
            assert abs(nrm[k] - oracle.norm(inst, got[k])) < 1e-12 * max(1, abs(nrm[k]))
            ref = oracle.energy(inst, got[k], t)
            assert np.allclose(en[k], ref, rtol=1e-11, atol=1e-11), (en[k], ref)


# ---------------------------------------------------------------------------
# full sizes, in the launch configuration of the solver (graph replay)
# ---------------------------------------------------------------------------
def test_coupled_2d_full_size(pkg):
    w = W.coupled_2d()   # 16 x 512^2, leapfrog + cf4 (two drifts per stage), 2000 steps
    _, _, short = run_gpu(pkg, w, "c128", nsteps=40, use_graph=True)
    ref = oracle.evolve(w.instances[3], w.psi0[3], w.scheme, w.ho_rule, w.dt, w.t0, 40)
    err = W.rel_l2(short[3], ref)
    say("coupled 2d full size, 40 steps, instance 3 vs oracle: %.3e" % err)
    assert err < 1e-11
    p128, b128, full128 = run_gpu(pkg, w, "c128", use_graph=True)
    p64, b64, full64 = run_gpu(pkg, w, "c64", use_graph=True)
    n0 = np.array([oracle.norm(i, p) for i, p in zip(w.instances, w.psi0)])
    drift = np.abs(p128.norm(b128) - n0).max()
    e64 = max(W.rel_l2(a, b) for a, b in zip(full64, full128))
    say("coupled 2d full 2000 steps: c128 norm drift %.3e, c64 vs c128 max %.3e" % (drift, e64))
    assert drift < 1e-11 and e64 < 5e-5


def test_coupled_3d_full_size(pkg):
    # oracle parity on the same recipe at 128^3 (one 256^3 oracle step takes ~45 s);
    # at 256^3: norm conservation and c64 against c128 over the full run
    half = W.coupled_3d(n=128)
    _, _, one = run_gpu(pkg, half, "c128", nsteps=1)
    ref = oracle.evolve(half.instances[0], half.psi0[0], half.scheme, half.ho_rule, half.dt, half.t0, 1)
    err = W.rel_l2(one[0], ref)
    say("coupled 3d 128^3, 1 step vs oracle: %.3e" % err)
    assert err < 1e-11
    w = W.coupled_3d()   # 256^3, NI5 + cf4, 500 steps
    p128, b128, full128 = run_gpu(pkg, w, "c128", use_graph=True)
    p64, b64, full64 = run_gpu(pkg, w, "c64", use_graph=True)
    drift = abs(p128.norm(b128)[0] - oracle.norm(w.instances[0], w.psi0[0]))
    e64 = W.rel_l2(full64[0], full128[0])
    say("coupled 3d full 500 steps: c128 norm drift %.3e, c64 vs c128 %.3e" % (drift, e64))
    assert drift < 1e-11 and e64 < 5e-5
