"""Pins of the times at which the oracle freezes sigma(t) in the B flow.

Table "algorithm" freezes time in the B flow: the B step of weight b_i acts at
the stage time tau_i = t_n + h c_i, c_i = a_0 + ... + a_{i-1} (c_0 = 0,
c_m = 1).  A slip here (sigma taken at t_n for the whole step, or the B
weights paired with the wrong stage times) would leave every constant-sigma
test green, so these pins use a time-dependent sigma(t) in its sine and pulse
forms and check against values from outside the oracle:

  * a one-point grid (N = 1 on [0, 1): x = 0 and k = 0) reduces the equation
    to the ODE i u' = (eps V_I + sigma(t) |u|^2) u, whose solution keeps |u|
    and turns the phase by eps V_I t + |u|^2 * int sigma dt.  The split step
    then applies the quadrature h sum_i b_i sigma(tau_i) of that integral:
    checked against the sum written out from the printed coefficients of
    Table tab.1, and against the closed-form integral at the quadrature's
    order under step halving;
  * a nonlinear 1-D problem with time-dependent omega(t) and sigma(t):
    time reversibility of the symmetric compositions (Sec. 2, P10) and the
    observed order 2 / 4 under step halving on smooth data;
  * the slip itself, built inside the test from the oracle's public calls
    (one step at a time with sigma held at sigma(t_n)), fails both.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import oracle
import workloads as W


def _golden_scheme(name):
    """(a, b) of a composition from the printed values of Table tab.1
    (tests/golden/table1_coefficients.txt), completed by its printed relations."""
    from test_golden import read_sections, table1_scheme
    if name == "leapfrog":  # Eq. LeapFrogB
        return [1.0], [0.5, 0.5]
    return table1_scheme(name, read_sections("table1_coefficients.txt")[name])


# sigma(t) forms: (v0, amp, freq, phase, form)
SIG_SINE = (5.0, 0.5, 3.0, 0.2, 0)       # 5 (1 + 0.5 sin(3t + 0.2))
SIG_PULSE = (4.0, 0.8, 2.5, 0.9, 2)      # 4 (1 + 0.8 t sech^2(2.5 (t - 0.9)))
SIG_FAST = (5.0, 0.5, 20.0, 0.2, 0)      # a fast modulation for the high-order schemes


def sigma_of(spec, t):
    v0, amp, fr, ph, form = spec
    if form == 2:
        return v0 * (1.0 + amp * t / math.cosh(fr * (t - ph)) ** 2)
    return v0 * (1.0 + amp * math.sin(fr * t + ph))


def sigma_integral(spec, t0, t1):
    """int_{t0}^{t1} sigma dt in closed form (sine), or by adaptive Gauss-Kronrod
    quadrature to 1e-14 (pulse: t sech^2 has no elementary antiderivative in
    the form needed here; scipy's quad is independent of the oracle)."""
    v0, amp, fr, ph, form = spec
    if form == 0:
        F = lambda t: v0 * (t - amp / fr * math.cos(fr * t + ph))
        return F(t1) - F(t0)
    from scipy.integrate import quad
    val, _ = quad(lambda t: sigma_of(spec, t), t0, t1, epsabs=1e-14, epsrel=1e-13, limit=200)
    return val


def point_instance(sig, eps=0.3, v0=2.0):
    # one grid point at x = 0 (box [0, 1)); omega(t) time-dependent so that the
    # HO rule runs its full path; V_I = v0 there
    return W.Instance(1, (1, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0),
                      omega=((1.3, 0.2, 2.0, 0.1), W.CONST_OMEGA, W.CONST_OMEGA),
                      sigma=sig, eps=eps, vfac=((v0, 0.0, 0.0, 0.0, 0.0, 0.0), W.NO_V, W.NO_V))


U0 = np.array([0.9 + 1.2j])  # |u| = 1.5


def point_phase(u):
    return -np.angle(u[0] / U0[0])


def wrap(x):
    return (x + math.pi) % (2.0 * math.pi) - math.pi


@pytest.mark.parametrize("scheme", ["leapfrog", "srkn6_4", "ni4_82", "ni5_84"])
@pytest.mark.parametrize("sig", [SIG_SINE, SIG_PULSE])
def test_point_grid_is_the_stage_time_quadrature(scheme, sig):
    """On one grid point the split step turns the phase by exactly
    h sum_n sum_i b_i (eps V_I + sigma(t_n + h c_i) |u|^2): B weights at the
    stage times of Table "algorithm", with the printed coefficients."""
    inst = point_instance(sig)
    a, b = _golden_scheme(scheme)
    c = np.concatenate([[0.0], np.cumsum(a)])
    t0, h, n = 0.3, 0.05, 24
    u = oracle.evolve(inst, U0, scheme, "cf4", h, t0, n)
    assert abs(abs(u[0]) - abs(U0[0])) < 1e-14
    expect = 0.0
    for s in range(n):
        tn = t0 + s * h
        for i in range(len(b)):
            expect += h * b[i] * (0.3 * 2.0 + sigma_of(sig, tn + h * c[i]) * abs(U0[0]) ** 2)
    assert abs(wrap(point_phase(u) - expect)) < 1e-12, (point_phase(u), expect)


def _point_errors(inst, sig, scheme, steps, T=1.0, t0=0.3, frozen_at_tn=False):
    """Phase error against the closed-form integral for each step count."""
    exact = 0.3 * 2.0 * T + abs(U0[0]) ** 2 * sigma_integral(sig, t0, t0 + T)
    errs = []
    for n in steps:
        h = T / n
        if frozen_at_tn:
            # the slip: sigma held at sigma(t_n) over the whole step, built from
            # the oracle's public calls one step at a time
            u = U0.copy()
            for s in range(n):
                tn = t0 + s * h
                frozen = point_instance((sigma_of(sig, tn), 0.0, 0.0, 0.0, 0))
                u = oracle.evolve(frozen, u, scheme, "cf4", h, tn, 1)
        else:
            u = oracle.evolve(inst, U0, scheme, "cf4", h, t0, n)
        errs.append(abs(wrap(point_phase(u) - exact)))
    return errs


def _rates(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


@pytest.mark.parametrize("sig", [SIG_SINE, SIG_PULSE])
def test_point_grid_order_against_closed_form(sig):
    inst = point_instance(sig)
    # leapfrog: the trapezoidal rule, order 2
    r = _rates(_point_errors(inst, sig, "leapfrog", (10, 20, 40, 80)))
    assert min(r) > 1.9, r
    # SRKN6_4: its B weights integrate to order 4
    r = _rates(_point_errors(inst, sig, "srkn6_4", (10, 20, 40)))
    assert min(r) > 3.8, r
    # the slip (sigma frozen at t_n): a left Riemann sum, order 1
    r = _rates(_point_errors(inst, sig, "leapfrog", (10, 20, 40, 80), frozen_at_tn=True))
    assert max(r) < 1.2, r


def test_point_grid_high_order_schemes():
    """NI4(8,2) and NI5(8,4) carry Gauss-Lobatto-type weights: on a fast
    modulation their quadrature error falls at order >= 6 (measured: ~8.5)
    until round-off."""
    for scheme in ("ni4_82", "ni5_84"):
        errs = _point_errors(point_instance(SIG_FAST), SIG_FAST, scheme, (6, 12, 24), T=1.0)
        assert errs[0] > 1e-7, errs   # well above round-off at the coarsest step
        r = _rates(errs)
        assert min(r) > 6.0, (scheme, errs, r)


# ---------------------------------------------------------------------------
# a spatially resolved nonlinear problem with omega(t) and sigma(t)
# ---------------------------------------------------------------------------
def nonlinear_instance(sig):
    return W.Instance(1, (128, 1, 1), (-8.0, 0.0, 0.0), (8.0, 1.0, 1.0),
                      omega=((1.2, 0.3, 1.7, 0.4), W.CONST_OMEGA, W.CONST_OMEGA),
                      sigma=sig, eps=0.05, vfac=((1.0, 0.0, 0.0, 0.0, 1.5, 0.3), W.NO_V, W.NO_V))


def smooth_state(inst):
    x = inst.axis(0)
    return W._normalise(inst, (np.exp(-(x - 0.7) ** 2 / 2.0) * np.exp(0.4j * x)).astype(np.complex128))


def frozen_run(inst, sig, psi, scheme, h, t0, n):
    """The slip of freezing sigma at t_n, one oracle step at a time."""
    u = psi
    for s in range(n):
        tn = t0 + s * h
        u = oracle.evolve(replace(inst, sigma=(sigma_of(sig, tn), 0.0, 0.0, 0.0, 0)), u, scheme, "cf4", h, tn, 1)
    return u


@pytest.mark.parametrize("sig", [SIG_SINE, SIG_PULSE])
@pytest.mark.parametrize("scheme", ["leapfrog", "ni5_84"])
def test_time_reversibility_with_sigma_t(sig, scheme):
    """Symmetric compositions are time-reversible (Sec. 2): K steps with +h
    from t0, then K steps with -h from t0 + K h, return the initial state.
    This needs every B at its own stage time; holding sigma at t_n breaks it."""
    inst = nonlinear_instance(sig)
    psi = smooth_state(inst)
    t0, h, K = 0.4, 0.02, 40
    fwd = oracle.evolve(inst, psi, scheme, "cf4", h, t0, K)
    back = oracle.evolve(inst, fwd, scheme, "cf4", -h, t0 + K * h, K)
    assert W.rel_l2(back, psi) < 1e-12
    wrong = frozen_run(inst, sig, frozen_run(inst, sig, psi, scheme, h, t0, K), scheme, -h, t0 + K * h, K)
    assert W.rel_l2(wrong, psi) > 1e-5


@pytest.mark.parametrize("sig", [SIG_SINE, SIG_PULSE])
def test_observed_order_with_sigma_t(sig):
    """Leapfrog and NI5(8,4) with the CF4 rule converge at orders 2 and 4 under
    step halving on smooth data with time-dependent omega(t) and sigma(t); the
    frozen-at-t_n slip converges at order 1 and fails the same check."""
    inst = nonlinear_instance(sig)
    psi = smooth_state(inst)
    t0, T = 0.4, 1.0
    ref = oracle.evolve(inst, psi, "ni5_84", "cf4", T / 1280, t0, 1280)

    def errs(scheme, steps, frozen=False):
        out = []
        for n in steps:
            run = frozen_run(inst, sig, psi, scheme, T / n, t0, n) if frozen else \
                oracle.evolve(inst, psi, scheme, "cf4", T / n, t0, n)
            out.append(W.rel_l2(run, ref))
        return out

    r = _rates(errs("leapfrog", (20, 40, 80)))
    assert min(r) > 1.85, r
    r = _rates(errs("ni5_84", (10, 20, 40)))
    assert min(r) > 3.6, r
    r = _rates(errs("leapfrog", (20, 40, 80), frozen=True))
    assert max(r) < 1.3, r


# ---------------------------------------------------------------------------
# a time factor of eps V_I: on the one-point grid the phase gains
# eps V_I h sum_i b_i m(tau_i)
# ---------------------------------------------------------------------------
VMODS = [(0.7, 2.5, 0.3, 0), (0.9, 2.0, 0.8, 2)]


def vmod_of(vm, t):
    amp, fr, ph, form = vm
    if form == 2:
        return 1.0 + amp * t / math.cosh(fr * (t - ph)) ** 2
    return 1.0 + amp * math.sin(fr * t + ph)


@pytest.mark.parametrize("scheme", ["leapfrog", "ni5_84"])
@pytest.mark.parametrize("vm", VMODS)
def test_point_grid_vi_time_factor(scheme, vm):
    inst = replace(point_instance(SIG_SINE), vmod=vm)
    a, b = _golden_scheme(scheme)
    c = np.concatenate([[0.0], np.cumsum(a)])
    t0, h, n = 0.3, 0.05, 24
    u = oracle.evolve(inst, U0, scheme, "cf4", h, t0, n)
    expect = sum(h * b[i] * (0.3 * 2.0 * vmod_of(vm, t0 + s * h + h * c[i])
                             + sigma_of(SIG_SINE, t0 + s * h + h * c[i]) * abs(U0[0]) ** 2)
                 for s in range(n) for i in range(len(b)))
    assert abs(wrap(point_phase(u) - expect)) < 1e-12


def test_point_grid_vi_time_factor_order():
    """Against the closed-form integral of the sine factor: order 2 for
    leapfrog, order 1 for the factor held at t_n."""
    vm = VMODS[0]
    amp, fr, ph, _ = vm
    t0, T = 0.3, 1.0
    inst = replace(point_instance((0.0, 0.0, 0.0, 0.0, 0)), vmod=vm)     # sigma = 0
    exact = 0.3 * 2.0 * (T - amp / fr * (math.cos(fr * (t0 + T) + ph) - math.cos(fr * t0 + ph)))
    errs, wrong = [], []
    for n in (10, 20, 40, 80):
        h = T / n
        errs.append(abs(wrap(point_phase(oracle.evolve(inst, U0, "leapfrog", "cf4", h, t0, n)) - exact)))
        u = U0.copy()
        for s in range(n):
            tn = t0 + s * h
            held = replace(point_instance((0.0, 0.0, 0.0, 0.0, 0), eps=0.3 * vmod_of(vm, tn)), vmod=(0.0, 0.0, 0.0, 0))
            u = oracle.evolve(held, u, "leapfrog", "cf4", h, tn, 1)
        wrong.append(abs(wrap(point_phase(u) - exact)))
    assert min(_rates(errs)) > 1.9, errs
    assert max(_rates(wrong)) < 1.2, wrong
