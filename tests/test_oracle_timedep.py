"""Pins of the oracle's time-dependent trap forms and of the fundamental-matrix
rule (the exact harmonic-oscillator flow for any omega(t), Eq. HO(t)sol).

Every expected value comes from outside the oracle: the trap frequencies of
Sec. 4.2 written out from their printed formulas, scipy's DOP853 integration
of the classical 2x2 system and of the Gaussian-packet equations, and
reductions to closed forms."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
import workloads as W


def omega_sq(spec, t):
    """omega(t)^2 from the printed formulas (Sec. 4.2) and the sine form."""
    v0, amp, freq, phase = spec[:4]
    form = spec[4] if len(spec) > 4 else 0
    if form == 1:      # omega^2 = A (1 + eps sin(w t + phase)); phase pi/2 gives cos
        return v0 * (1.0 + amp * math.sin(freq * t + phase))
    if form == 2:      # omega = w0 (1 + A t / cosh^2(B (t - t_c)))
        return (v0 * (1.0 + amp * t / math.cosh(freq * (t - phase)) ** 2)) ** 2
    return (v0 * (1.0 + amp * math.sin(freq * t + phase))) ** 2


def classical_flow(spec, mu, t0, tau):
    """2x2 flow of x' = p/mu, p' = -mu omega(t)^2 x over [t0, t0+tau] (DOP853)."""
    def rhs(t, y):
        Y = y.reshape(2, 2)
        A = np.array([[0.0, 1.0 / mu], [-mu * omega_sq(spec, t), 0.0]])
        return (A @ Y).ravel()
    sol = solve_ivp(rhs, (t0, t0 + tau), np.eye(2).ravel(), method="DOP853",
                    rtol=1e-13, atol=1e-15)
    return sol.y[:, -1].reshape(2, 2)


def inst_with(spec, mu=1.0, n=256, lo=-10.0, hi=10.0, eps=0.0, vfac=W.NO_V):
    return W.Instance(1, (n, 1, 1), (lo, 0.0, 0.0), (hi, 1.0, 1.0), mu=mu,
                      omega=(tuple(spec), W.CONST_OMEGA, W.CONST_OMEGA), eps=eps,
                      vfac=(vfac, W.NO_V, W.NO_V))


COS = W.TIMEDEP_OMEGA["cos"]
PULSE = W.TIMEDEP_OMEGA["pulse"]
SINE = (1.4, 0.3, 3.0, 0.2, 0)


# ---------------------------------------------------------------------------
# the fundamental-matrix rule against an independent ODE solution
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("spec,mu,t0,tau", [(COS, 1.0, 0.3, 0.6), (COS, 1.0, 7.0, -0.5),
                                            (PULSE, 1.0, 1.7, 0.5), (PULSE, 2.0, 2.1, 0.3),
                                            (SINE, 1.7, 0.3, 0.9)])
def test_fundamental_matches_dop853(spec, mu, t0, tau):
    inst = inst_with(spec, mu=mu)
    S = oracle.stage_matrix(inst, "fundamental:64", 0, t0, tau)
    ref = classical_flow(spec, mu, t0, tau)
    assert np.abs(S - ref).max() < 1e-11 * max(1.0, np.abs(ref).max()), (S, ref)


@pytest.mark.parametrize("spec", [COS, PULSE])
def test_fundamental_substep_order(spec):
    """Sixth order in the sub-step length: halving it divides the error by ~64."""
    inst = inst_with(spec)
    t0, tau = 1.6, 0.7
    ref = classical_flow(spec, 1.0, t0, tau)
    errs = [np.abs(oracle.stage_matrix(inst, "fundamental:%d" % q, 0, t0, tau) - ref).max()
            for q in (4, 8, 16)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 5.4, (errs, rates)


def test_fundamental_one_substep_is_magnus6():
    inst = inst_with(PULSE)
    a = oracle.stage_matrix(inst, "fundamental:1", 0, 1.9, 0.2)
    b = oracle.stage_matrix(inst, "magnus6", 0, 1.9, 0.2)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("spec", [(1.3, 0.0, 0.0, 0.0, 0), (1.69, 0.0, 0.0, 0.0, 1)])
def test_fundamental_constant_frequency_is_exact(spec):
    """Constant omega: the flow is the rotation of Lemma 2's proof."""
    mu, tau = 1.4, 1.1
    inst = inst_with(spec, mu=mu)
    S = oracle.stage_matrix(inst, "fundamental:8", 0, 0.0, tau)
    w = 1.3
    ref = np.array([[math.cos(w * tau), math.sin(w * tau) / (mu * w)],
                    [-mu * w * math.sin(w * tau), math.cos(w * tau)]])
    assert np.abs(S - ref).max() < 1e-14


@pytest.mark.parametrize("rule", ["cf4", "magnus6", "fundamental:16"])
def test_time_forms_enter_every_rule(rule):
    """Each rule sees the trap forms of Sec. 4.2: local error against DOP853
    shrinks with the stage length at the rule's order."""
    order = {"cf4": 4, "magnus6": 6, "fundamental:16": 6}[rule]
    for spec in (COS, PULSE):
        inst = inst_with(spec)
        errs = []
        for tau in (0.2, 0.1, 0.05):
            S = oracle.stage_matrix(inst, rule, 0, 1.8, tau)
            errs.append(np.abs(S - classical_flow(spec, 1.0, 1.8, tau)).max())
        if rule.startswith("fundamental"):
            # 16 sub-steps: near round-off already; first halving still at order 6+
            assert errs[0] < 1e-10, errs
            assert errs[0] < 1e-13 or errs[0] / errs[1] > 2 ** 6, errs
        else:
            rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
            assert min(rates) > order + 0.6, (spec, errs, rates)


# ---------------------------------------------------------------------------
# linear HO with a time-dependent trap: the fundamental rule makes the HF
# step exact in time (B = 0), whatever the step
# ---------------------------------------------------------------------------
def gaussian_packet(spec, mu, x, a0, b0, c0, t0, T):
    """psi = exp(a x^2 + b x + c) solves i psi_t = -psi_xx/(2mu) + mu omega^2 x^2/2 psi
    when a' = 2i a^2/mu - i mu omega^2/2, b' = 2i a b/mu, c' = i (b^2/2 + a)/mu."""
    def rhs(t, y):
        a, b = y[0] + 1j * y[1], y[2] + 1j * y[3]
        da = 2j * a * a / mu - 0.5j * mu * omega_sq(spec, t)
        db = 2j * a * b / mu
        dc = 1j * (0.5 * b * b + a) / mu
        return [da.real, da.imag, db.real, db.imag, dc.real, dc.imag]
    y0 = [a0.real, a0.imag, b0.real, b0.imag, c0.real, c0.imag]
    sol = solve_ivp(rhs, (t0, T), y0, method="DOP853", rtol=1e-13, atol=1e-14)
    y = sol.y[:, -1]
    a, b, c = y[0] + 1j * y[1], y[2] + 1j * y[3], y[4] + 1j * y[5]
    return np.exp(a * x * x + b * x + c)


@pytest.mark.parametrize("form", ["cos", "pulse"])
def test_linear_timedep_fundamental_is_exact_in_time(form):
    spec = W.TIMEDEP_OMEGA[form]
    inst = inst_with(spec, n=512, lo=-10.0, hi=10.0)
    x = inst.axis(0)
    x0 = 0.6
    psi0 = (2.0 / math.pi) ** 0.25 * np.exp(-(x - x0) ** 2)
    T = 4.0
    ref = gaussian_packet(spec, 1.0, x, -1.0 + 0j, 2.0 * x0 + 0j,
                          -x0 * x0 + 0.25 * math.log(2.0 / math.pi) + 0j, 0.0, T)
    u = oracle.evolve(inst, psi0, "leapfrog", "fundamental:32", T / 16, 0.0, 16)
    err = W.rel_l2(u, ref)
    assert err < 1e-10
    # the fourth-order rule at the same step is not exact
    v = oracle.evolve(inst, psi0, "leapfrog", "cf4", T / 16, 0.0, 16)
    assert W.rel_l2(v, ref) > 100 * err


def test_magnus6_beats_cf4_on_pulse():
    """Sec. 4.2: for high accuracy the sixth-order Magnus rule improves on the
    two-exponential rule for the pulse trap (linear case, B = 0, so the global
    error is the HO rule's own: order 4 vs order 6 under step halving)."""
    inst = inst_with(PULSE, n=512, lo=-10.0, hi=10.0)
    x = inst.axis(0)
    psi0 = (2.0 / math.pi) ** 0.25 * np.exp(-(x - 0.6) ** 2)
    T = 4.0
    ref = gaussian_packet(PULSE, 1.0, x, -1.0 + 0j, 1.2 + 0j,
                          -0.36 + 0.25 * math.log(2.0 / math.pi) + 0j, 0.0, T)
    e4, e6 = [], []
    for n in (64, 128, 256):
        e4.append(W.rel_l2(oracle.evolve(inst, psi0, "leapfrog", "cf4", T / n, 0.0, n), ref))
        e6.append(W.rel_l2(oracle.evolve(inst, psi0, "leapfrog", "magnus6", T / n, 0.0, n), ref))
    r4 = [math.log2(e4[i] / e4[i + 1]) for i in range(2)]
    r6 = [math.log2(e6[i] / e6[i + 1]) for i in range(2)]
    assert min(r4) > 3.7 and min(r6) > 5.6, (e4, e6)
    assert e6[1] < 0.5 * e4[1] and e6[2] < 0.05 * e4[2], (e4, e6)


def test_energy_uses_time_form():
    """Potential energy of a Gaussian at the pulse peak: closed form
    h sum mu omega(t)^2 x^2/2 |u|^2 -> mu omega^2 <x^2>/2 with <x^2> = 1/4
    for |u|^2 = sqrt(2/pi) exp(-2 x^2)."""
    inst = inst_with(PULSE, n=512, lo=-10.0, hi=10.0)
    x = inst.axis(0)
    u = (2.0 / math.pi) ** 0.25 * np.exp(-x * x)
    t = 2.3
    e = oracle.energy(inst, u, t)
    assert abs(e[2] - omega_sq(PULSE, t) / 8.0) < 1e-12 * omega_sq(PULSE, t)
