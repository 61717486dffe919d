"""GPU parity with a time-dependent quadratic part and perturbation (Sec. 1:
V = x^T M(t) x + eps V_I(x, t)): modulated off-diagonal trap entries W_ij(t)
and a time factor m(t) of eps V_I, against the CPU oracle through the C ABI,
and the forced centre-of-mass identity, which needs no oracle."""
import math
from dataclasses import replace

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-11, "c64": 5e-5}
WMOD = ((0.5, 2.3, 0.4, 0), (0.8, 2.0, 0.6, 2), (-0.4, 1.1, 0.0, 0))
# 3-D: amplitudes that keep the Gershgorin bound of the plan's validation
# (off-diagonal row sums below the smallest omega_j^2) for the recipe's cross terms
WMOD3 = ((0.25, 2.3, 0.4, 0), (0.3, 2.0, 0.6, 2), (-0.3, 1.1, 0.0, 0))
VMOD_SINE = (0.7, 2.5, 0.3, 0)
VMOD_PULSE = (0.9, 2.0, 0.8, 2)


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_1007_3470_amd as p
    p.load()
    return p


def run_gpu(pkg, w, dtype, nsteps=None, vis=None, **kw):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, **kw)
    if vis is not None:
        plan.set_potential(plan.pack_real(vis))
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, w.nsteps if nsteps is None else nsteps)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return plan, buf, plan.unpack(buf)


def say(*a):
    print(*a, flush=True)


def check(w, got, tol, vis=None, label=""):
    for k, inst in enumerate(w.instances):
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps,
                            vi=None if vis is None else vis[k])
        err = W.rel_l2(got[k], ref)
        say("%s %dD %s %s k=%d rel_l2 %.3e" % (label, inst.ndim, w.scheme, w.ho_rule, k, err))
        assert err < tol, (k, err)


@pytest.mark.parametrize("rule", ["cf4", "fsplit"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_modulated_coupled_2d(pkg, rule, dtype):
    w = W.coupled_2d(n=64, n_inst=3, nsteps=30, rule=rule)
    w = replace(w, instances=[replace(i, wmod=WMOD, vmod=VMOD_SINE) for i in w.instances])
    _, _, got = run_gpu(pkg, w, dtype, use_graph=True)
    check(w, got, TOL[dtype], label="modulated coupled")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_modulated_coupled_3d(pkg, dtype):
    w = W.coupled_3d(n=32, nsteps=4)
    w = replace(w, instances=[replace(i, wmod=WMOD3, vmod=VMOD_PULSE) for i in w.instances])
    _, _, got = run_gpu(pkg, w, dtype)
    check(w, got, TOL[dtype], label="modulated coupled")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_vi_time_factor_1d_batch(pkg, dtype):
    """Every 1-D kernel (sizes below 64, fixed shape, 4096) with the factor
    form and a pulse or sine time factor."""
    base = W.batch_1d(n_inst=8, sizes=(32, 256, 1024, 4096), nsteps=40, seed=12)
    insts = [replace(i, vmod=(VMOD_SINE if k % 2 else VMOD_PULSE), eps=0.5) for k, i in enumerate(base.instances)]
    w = replace(base, instances=insts)
    _, _, got = run_gpu(pkg, w, dtype)
    check(w, got, TOL[dtype], label="vi time factor")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_vi_time_factor_2d_array(pkg, dtype):
    """The caller's array takes the time factor too."""
    w = W.gpe_2d(n=64, n_inst=2, nsteps=20)
    w = replace(w, instances=[replace(i, vmod=VMOD_PULSE) for i in w.instances])
    vis = []
    for i in w.instances:
        x, y = i.mesh()
        vis.append(np.broadcast_to(0.2 * (x - 0.5 * y) + 0.05 * np.cos(x * y), i.shape).copy())
    _, _, got = run_gpu(pkg, w, dtype, vis=vis, use_graph=True)
    check(w, got, TOL[dtype], vis=vis, label="vi array time factor")


def test_modulated_energy(pkg):
    w = W.coupled_2d(n=64, n_inst=2, nsteps=10)
    w = replace(w, instances=[replace(i, wmod=WMOD, vmod=VMOD_SINE) for i in w.instances])
    plan, buf, got = run_gpu(pkg, w, "c128")
    for t in (0.0, 0.37, 1.9):
        en = plan.energy(buf, t)
        for k, inst in enumerate(w.instances):
            ref = oracle.energy(inst, got[k], t)
            assert np.allclose(en[k], ref, rtol=1e-11, atol=1e-12), (t, k, en[k], ref)


# ---------------------------------------------------------------------------
# forced centre of mass: eps V_I(x, t) = m(t) F x is a uniform force, so for
# any sigma <x>, <p> follow the classical split map (exact HO flow of Lemma 2,
# kicks -h b_i F m(tau_i) at the stage times); no oracle involved
# ---------------------------------------------------------------------------
def _m(vm, t):
    amp, fr, ph, form = vm
    if form == 2:
        return 1.0 + amp * t / math.cosh(fr * (t - ph)) ** 2
    return 1.0 + amp * math.sin(fr * t + ph)


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-10), ("c64", 2e-6)])
@pytest.mark.parametrize("vm", [VMOD_SINE, VMOD_PULSE])
def test_forced_centre_of_mass(pkg, dtype, tol, vm):
    mu, w, F, sigma = 1.3, 1.1, 0.3, 20.0
    inst = W.Instance(1, (512, 1, 1), (-16.0, 0.0, 0.0), (16.0, 1.0, 1.0), mu=mu,
                      omega=((w, 0.0, 0.0, 0.0), W.CONST_OMEGA, W.CONST_OMEGA),
                      sigma=(sigma, 0.0, 0.0, 0.0), eps=1.0, vmod=vm)
    x = inst.axis(0)
    x0, p0 = 1.2, -0.4
    u0 = W._normalise(inst, np.exp(-0.5 * mu * w * (x - x0) ** 2 + 1j * p0 * x).astype(complex))
    t0, h, n = 0.2, 0.02, 150
    wl = W.Workload("forced", [inst], [u0], "ni5_84", "exact_const", h, n, t0=t0)
    _, _, got = run_gpu(pkg, wl, dtype, vis=[F * x])
    u = got[0]
    rho = np.abs(u) ** 2
    X = float((x * rho).sum() / rho.sum())
    k = 2 * math.pi / 32.0 * np.fft.fftfreq(512, d=1.0 / 512)
    rh = np.abs(np.fft.fft(u)) ** 2
    P = float((k * rh).sum() / rh.sum())
    a, b = pkg.scheme_preset("ni5_84")
    z = np.array([x0, p0])
    for s in range(n):
        tau = t0 + s * h
        z[1] -= h * b[0] * F * _m(vm, tau)
        for i in range(len(a)):
            th = w * a[i] * h
            R = np.array([[math.cos(th), math.sin(th) / (mu * w)], [-mu * w * math.sin(th), math.cos(th)]])
            z = R @ z
            tau += a[i] * h
            z[1] -= h * b[i + 1] * F * _m(vm, tau)
    say("forced centre of mass %s: |dx| %.3e |dp| %.3e" % (dtype, abs(X - z[0]), abs(P - z[1])))
    assert abs(X - z[0]) < tol and abs(P - z[1]) < tol
