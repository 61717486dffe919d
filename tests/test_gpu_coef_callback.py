"""omega_j(t) and sigma(t) from a caller's host function (hfgpe_set_coef_callback):
the plan's HO rule samples the function on the host.  Checked against the
library's own time forms and the oracle, and, for a frequency with no
built-in form, against the Kohn identity (with V_I = 0 the centre of mass
follows the classical oscillator x'' = -omega(t)^2 x for any sigma(t)),
solved independently by DOP853."""
import math
from dataclasses import replace

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_1007_3470_amd as p
    p.load()
    return p


def say(*a):
    print(*a, flush=True)


def form_value(f, t):
    """The workload's time form (v0, amp, freq, phase[, kind]) written out in Python."""
    v0, a, fr, ph = f[:4]
    kind = f[4] if len(f) > 4 else 0
    if kind == 2:
        return v0 * (1.0 + a * t / math.cosh(fr * (t - ph)) ** 2)
    v = v0 * (1.0 + a * math.sin(fr * t + ph))
    return math.sqrt(v) if kind == 1 else v


def forms_callback(instances):
    def fn(inst, which, t):
        I = instances[inst]
        return form_value(I.sigma if which == 3 else I.omega[which], t)
    return fn


def run(pkg, w, dtype, fn=None, nsteps=None):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt)
    if fn is not None:
        plan.set_coef_callback(fn)
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, w.nsteps if nsteps is None else nsteps)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return plan, plan.unpack(buf)


@pytest.mark.parametrize("rule", ["cf4", "magnus6", "fundamental:8", "fsplit"])
def test_callback_reproduces_time_forms_1d(pkg, rule):
    w = W.gpe_1d(n=512, nsteps=300, rule=rule)
    _, got = run(pkg, w, "c128", forms_callback(w.instances))
    _, lib = run(pkg, w, "c128")
    ref = oracle.evolve(w.instances[0], w.psi0[0], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
    e_lib, e_orc = W.rel_l2(got[0], lib[0]), W.rel_l2(got[0], ref)
    say("%s: callback vs built-in forms %.2e, vs oracle %.2e" % (rule, e_lib, e_orc))
    assert e_lib < 1e-12 and e_orc < 1e-11


def test_callback_reproduces_pulse_and_squared_forms(pkg):
    base = W.timedep_1d(form="pulse", n=512, T=0.5, nsteps=50, scheme="srkn6_4", rule="magnus6")
    cos2 = W.timedep_1d(form="cos", n=512, T=0.5, nsteps=50, scheme="srkn6_4", rule="magnus6")
    w = replace(base, instances=base.instances + cos2.instances, psi0=base.psi0 + cos2.psi0)
    _, got = run(pkg, w, "c128", forms_callback(w.instances))
    for k, inst in enumerate(w.instances):
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        assert W.rel_l2(got[k], ref) < 1e-11


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_callback_2d_time_dependent(pkg, dtype):
    w = W.gpe_2d(n=64, n_inst=3, nsteps=20)
    _, got = run(pkg, w, dtype, forms_callback(w.instances))
    for k, inst in enumerate(w.instances):
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        assert W.rel_l2(got[k], ref) < (1e-11 if dtype == "c128" else 5e-5)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_callback_with_graph_replay(pkg, dtype):
    """d-D plan with hipGraph replay (16-step blocks and a remainder): the
    host-staged records feed the captured passes, giving the same bits as
    direct launches, and the oracle's result."""
    import torch
    w = W.gpe_2d(n=64, n_inst=3, nsteps=40)
    outs = []
    for graph in (False, True):
        plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, use_graph=graph)
        plan.set_coef_callback(forms_callback(w.instances))
        buf = plan.pack(w.psi0)
        plan.evolve(buf, w.t0, 20)
        plan.evolve(buf, w.t0 + 20 * w.dt, 20)
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        outs.append(plan.unpack(buf))
    for k, inst in enumerate(w.instances):
        assert np.array_equal(outs[0][k], outs[1][k])
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        assert W.rel_l2(outs[1][k], ref) < (1e-11 if dtype == "c128" else 5e-5)


def omega_free(t):
    """A frequency with no built-in form."""
    return 1.0 + 0.4 * t * math.exp(-t) + 0.1 * math.sin(3.0 * t) ** 2


def sigma_free(t):
    return 20.0 * (1.0 + 0.5 * math.cos(3.0 * t))


def moments_1d(inst, u):
    x = inst.axis(0)
    rho = np.abs(u) ** 2
    X = float((x * rho).sum() / rho.sum())
    uh = np.fft.fft(u)
    k = 2 * math.pi / (inst.hi[0] - inst.lo[0]) * np.fft.fftfreq(inst.n[0], d=1.0 / inst.n[0])
    P = float((k * np.abs(uh) ** 2).sum() / (np.abs(uh) ** 2).sum())
    return X, P


@pytest.mark.parametrize("rule,tol", [("cf4", 1e-8), ("magnus6", 1e-10), ("fundamental:8", 1e-10)])
def test_callback_kohn_mode_arbitrary_omega(pkg, rule, tol):
    inst = W.Instance(1, (1024, 1, 1), (-16.0, 0.0, 0.0), (16.0, 1.0, 1.0))
    x = inst.axis(0)
    x0, p0 = 1.1, -0.6
    u0 = W._normalise(inst, np.exp(-(x - x0) ** 2 / 2 + 1j * p0 * x))
    T, n = 3.0, 300
    w = W.Workload("kohn", [inst], [u0], "ni5_84", rule, T / n, n)

    def fn(i, which, t):
        return sigma_free(t) if which == 3 else omega_free(t)
    plan, got = run(pkg, w, "c128", fn)
    X, P = moments_1d(inst, got[0])
    sol = solve_ivp(lambda t, y: [y[1], -omega_free(t) ** 2 * y[0]], (0.0, T), [x0, p0], method="DOP853",
                    rtol=1e-13, atol=1e-14)
    err = max(abs(X - sol.y[0, -1]), abs(P - sol.y[1, -1]))
    say("%s: centre of mass vs classical orbit, omega(t) with no built-in form: %.2e" % (rule, err))
    assert err < tol
    buf = plan.pack([got[0]])
    assert abs(plan.norm(buf)[0] - 1.0) < 1e-12


def test_callback_errors_and_reset(pkg):
    import torch
    w = W.gpe_1d(n=256, nsteps=4)
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, "c128", w.dt)
    plan.set_coef_callback(lambda i, which, t: -1.0 if which == 0 else 5.0)
    with pytest.raises(pkg.HfgpeError) as e:
        plan.evolve(plan.pack(w.psi0), 0.0, 4)
    assert e.value.code == -4
    plan.set_coef_callback(lambda i, which, t: float("nan") if which == 3 else 1.0)
    with pytest.raises(pkg.HfgpeError) as e:
        plan.evolve(plan.pack(w.psi0), 0.0, 4)
    assert e.value.code == -7

    def bad(i, which, t):
        raise KeyError("no such instance")
    plan.set_coef_callback(bad)
    with pytest.raises(pkg.HfgpeError) as e:
        plan.evolve(plan.pack(w.psi0), 0.0, 4)
    assert isinstance(e.value.__cause__, KeyError)
    # None restores the parameters' forms: the same bits as a plan without callbacks
    plan.set_coef_callback(None)
    b = plan.pack(w.psi0)
    plan.evolve(b, 0.0, 4)
    _, ref = run(pkg, w, "c128")
    torch.cuda.synchronize()
    assert np.array_equal(plan.unpack(b)[0], ref[0])


def test_stage_and_coef_callbacks_are_exclusive(pkg):
    w = W.gpe_1d(n=256, nsteps=6)
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, "c128", w.dt)
    plan.set_stage_callback(lambda *a: (_ for _ in ()).throw(RuntimeError("stage callback must be off")))
    plan.set_coef_callback(forms_callback(w.instances))  # clears the stage callback
    buf = plan.pack(w.psi0)
    plan.evolve(buf, 0.0, 6)
    ref = oracle.evolve(w.instances[0], w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, 6)
    assert W.rel_l2(plan.unpack(buf)[0], ref) < 1e-11


def test_coef_callback_rejected_for_coupled_plan(pkg):
    w = W.coupled_2d(n=16, n_inst=1, nsteps=1)
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, "c128", w.dt)
    with pytest.raises(pkg.HfgpeError) as e:
        plan.set_coef_callback(lambda i, which, t: 1.0)
    assert e.value.code == -1
