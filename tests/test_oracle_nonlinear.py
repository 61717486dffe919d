"""Pins of the oracle's nonlinear evolution (sigma != 0) against exact
identities of the Gross-Pitaevskii equation (Sec. 1) that hold for any
nonlinearity, so the nonlinear trajectory is checked against something other
than the oracle itself.  Every observable here is computed with NumPy from the
oracle's output, not with the oracle's own FFT or energy routine.

* Kohn mode (Ehrenfest): in a harmonic trap with V_I = 0 the mean-field term
  exerts no net force (the integral of rho grad rho vanishes), so <x> and <p>
  follow the classical oscillator x' = p/mu, p' = -mu W(t) x for every sigma.
  In the HO split the A flow moves (<x>, <p>) exactly as the classical matrix of
  the stage and the B flow (Lemma 1) leaves both unchanged, so with the exact
  rule of Lemma 2 the centre of mass is exact to round-off, independently of
  the step size, as long as the grid resolves the state: the discrete identity
  needs the product of the state with the B phase free of aliasing (with
  sigma = 30, steps of 0.05 let high wavenumbers grow and it fails at 1e-2).
  With the commutator-free rule it carries exactly that rule's classical error
  (global order 4).
* Forced Kohn mode: with a uniform, time-dependent force (eps V_I(x, t) =
  m(t) F x) the centre of mass is the classical split map with the B kicks
  at the stage times, for any sigma.
* 2-D breathing mode: in a 2-D isotropic trap the virial identity gives
  <r^2>'' = 4 E / mu - 4 omega^2 <r^2> exactly for the cubic nonlinearity, E the
  conserved energy including (sigma/2) int rho^2; a wrong weight or sign of the
  nonlinear phase changes the conserved E the evolution follows and breaks it.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

import oracle
import workloads as W

CONST = W.CONST_OMEGA


def gaussian(inst, centre, widths, momentum):
    m = inst.mesh()
    arg = sum(-0.5 * w * (x - c) ** 2 + 1j * p * x for x, c, w, p in zip(m, centre, widths, momentum))
    return W._normalise(inst, np.exp(arg) * np.ones(inst.shape))


def moments(inst, u):
    """<x_j> on the grid and <p_j> from a NumPy FFT (k_q = 2 pi/L (q < n/2 ? q : q - n))."""
    rho = np.abs(u) ** 2
    nrm = rho.sum()
    xs = [float((x * rho).sum() / nrm) for x in inst.mesh()]
    uh = np.fft.fftn(u)
    rh = np.abs(uh) ** 2
    ps = []
    for j in range(inst.ndim):
        L = inst.hi[j] - inst.lo[j]
        k = 2 * math.pi / L * np.fft.fftfreq(inst.n[j], d=1.0 / inst.n[j])
        s = [1] * inst.ndim
        s[inst.ndim - 1 - j] = inst.n[j]
        ps.append(float((k.reshape(s) * rh).sum() / rh.sum()))
    return np.array(xs), np.array(ps)


def test_kohn_mode_exact_rule_1d():
    """sigma = 30, mu = 1.3: the centre of mass is exactly the classical orbit
    over T = 10, for two compositions."""
    mu, w = 1.3, 1.1
    inst = W.Instance(1, (512, 1, 1), (-16.0, 0.0, 0.0), (16.0, 1.0, 1.0), mu=mu,
                      omega=((w, 0.0, 0.0, 0.0), CONST, CONST), sigma=(30.0, 0.0, 0.0, 0.0))
    x0, p0 = 1.5, 0.7
    u0 = gaussian(inst, (x0,), (mu * w,), (p0,))
    X0, P0 = moments(inst, u0)
    assert abs(X0[0] - x0) < 1e-13 and abs(P0[0] - p0) < 1e-13
    for scheme, dt, n in (("leapfrog", 0.01, 1000), ("ni5_84", 0.02, 500)):
        T = dt * n
        u = oracle.evolve(inst, u0, scheme, "exact_const", dt, 0.0, n)
        X, P = moments(inst, u)
        xc = x0 * math.cos(w * T) + p0 / (mu * w) * math.sin(w * T)
        pc = p0 * math.cos(w * T) - mu * w * x0 * math.sin(w * T)
        assert abs(X[0] - xc) < 1e-10, (scheme, X[0], xc)
        assert abs(P[0] - pc) < 1e-10, (scheme, P[0], pc)
        # the nonlinearity did act: the density is far from the moved initial packet
        moved = gaussian(inst, (xc,), (mu * w,), (pc,))
        assert W.rel_l2(np.abs(u), np.abs(moved)) > 1e-2


def test_kohn_mode_coupled_trap_2d():
    """Coupled trap (off-diagonal W) with sigma = 20: <x>, <p> against the
    classical flow exp(T [[0, I/mu], [-mu W, 0]])."""
    wx, wy, wxy = 1.0, 1.3, 0.4
    # the repulsive cloud spreads: a box of [-14, 14)^2 keeps it off the periodic
    # boundary (on [-10, 10)^2 its tail, 5e-6 at the edge, wraps and moves <x> by 2e-9)
    inst = W.Instance(2, (128, 128, 1), (-14.0, -14.0, 0.0), (14.0, 14.0, 1.0),
                      omega=((wx, 0.0, 0.0, 0.0), (wy, 0.0, 0.0, 0.0), CONST),
                      sigma=(20.0, 0.0, 0.0, 0.0), wcross=(wxy, 0.0, 0.0))
    x0, p0 = np.array([0.8, -0.5]), np.array([0.3, 0.6])
    u0 = gaussian(inst, x0, (1.0, 1.2), p0)
    dt, n = 0.02, 200
    u = oracle.evolve(inst, u0, "leapfrog", "exact_const", dt, 0.0, n)
    X, P = moments(inst, u)
    Wm = np.array([[wx * wx, wxy], [wxy, wy * wy]])
    A = np.block([[np.zeros((2, 2)), np.eye(2)], [-Wm, np.zeros((2, 2))]])
    z = expm(A * dt * n) @ np.concatenate([x0, p0])
    assert np.abs(X - z[:2]).max() < 1e-10, (X, z[:2])
    assert np.abs(P - z[2:]).max() < 1e-10, (P, z[2:])


def test_kohn_mode_time_dependent_cf4_order():
    """omega(t) = 1 + 0.3 sin 2t, sigma = 20, NI5(8,4) + CF4: the centre of mass
    carries only the commutator-free rule's classical error, global order 4."""
    inst = W.Instance(1, (512, 1, 1), (-16.0, 0.0, 0.0), (16.0, 1.0, 1.0),
                      omega=((1.0, 0.3, 2.0, 0.0), CONST, CONST), sigma=(20.0, 0.0, 0.0, 0.0))
    x0, p0 = 1.2, -0.4
    u0 = gaussian(inst, (x0,), (1.0,), (p0,))
    T = 4.0

    def rhs(t, y):
        om = 1.0 + 0.3 * math.sin(2.0 * t)
        return [y[1], -om * om * y[0]]

    ref = solve_ivp(rhs, (0.0, T), [x0, p0], method="DOP853", rtol=1e-13, atol=1e-14).y[:, -1]
    errs = []
    for n in (40, 80):
        u = oracle.evolve(inst, u0, "ni5_84", "cf4", T / n, 0.0, n)
        X, P = moments(inst, u)
        errs.append(max(abs(X[0] - ref[0]), abs(P[0] - ref[1])))
    rate = math.log2(errs[0] / errs[1])
    assert errs[1] < 1e-6 and 3.5 < rate < 4.6, (errs, rate)


def energy_numpy(inst, u, w, sigma):
    """E = T + V + U for mu = 1, isotropic trap, from a NumPy FFT."""
    h = inst.cell
    uh = np.fft.fftn(u)
    k2 = 0.0
    for j in range(inst.ndim):
        L = inst.hi[j] - inst.lo[j]
        k = 2 * math.pi / L * np.fft.fftfreq(inst.n[j], d=1.0 / inst.n[j])
        s = [1] * inst.ndim
        s[inst.ndim - 1 - j] = inst.n[j]
        k2 = k2 + k.reshape(s) ** 2
    kin = 0.5 * float((k2 * np.abs(uh) ** 2).sum()) * h / u.size
    rho = np.abs(u) ** 2
    r2 = sum(x ** 2 for x in inst.mesh())
    pot = 0.5 * w * w * float((r2 * rho).sum()) * h
    inter = 0.5 * sigma * float((rho ** 2).sum()) * h
    return kin + pot + inter


@pytest.mark.parametrize("sigma", [15.0, -2.0])
def test_breathing_mode_2d(sigma):
    """<r^2>(t) = E/w^2 + (<r^2>_0 - E/w^2) cos 2wt for a real initial state, any
    sigma; checked at T = 1.5 with NI5(8,4) + exact rule, with the step error
    decreasing at order 4."""
    w = 1.3
    inst = W.Instance(2, (128, 128, 1), (-10.0, -10.0, 0.0), (10.0, 10.0, 1.0),
                      omega=((w, 0.0, 0.0, 0.0), (w, 0.0, 0.0, 0.0), CONST),
                      sigma=(sigma, 0.0, 0.0, 0.0))
    u0 = gaussian(inst, (0.3, -0.2), (1.4, 0.8), (0.0, 0.0))
    h = inst.cell
    r2 = sum(x ** 2 for x in inst.mesh())
    I0 = float((r2 * np.abs(u0) ** 2).sum()) * h
    E = energy_numpy(inst, u0, w, sigma)
    T = 1.5
    exact = E / w ** 2 + (I0 - E / w ** 2) * math.cos(2 * w * T)
    assert abs(exact - I0) > 0.05  # the cloud does breathe
    errs = []
    for n in (30, 60):
        u = oracle.evolve(inst, u0, "ni5_84", "exact_const", T / n, 0.0, n)
        errs.append(abs(float((r2 * np.abs(u) ** 2).sum()) * h - exact))
    rate = math.log2(errs[0] / errs[1])
    assert errs[1] < 1e-6 and rate > 3.5, (errs, rate)
    # the same run with the nonlinear coefficient halved inside the evolution
    # follows another energy: the identity with this E is then off by far more
    wrong = W.Instance(**{**inst.__dict__, "sigma": (0.5 * sigma, 0.0, 0.0, 0.0)})
    u = oracle.evolve(wrong, u0, "ni5_84", "exact_const", T / 60, 0.0, 60)
    assert abs(float((r2 * np.abs(u) ** 2).sum()) * h - exact) > 1e3 * errs[1]


# ---------------------------------------------------------------------------
# time-dependent perturbation eps V_I(x, t) = m(t) F x (Sec. 1): a uniform,
# time-dependent force.  For any sigma the centre of mass obeys
# x' = p/mu, p' = -mu omega^2 x - F m(t); the HO split moves (<x>, <p>) by the
# stage's classical matrix in A (exact rule: Lemma 2) and kicks <p> by
# -h b_i F m(tau_i) in each B flow, the mean field giving no net force.  So the
# oracle's centre of mass must equal that classical split map applied to
# (x0, p0) with the B kicks at the stage times of Table "algorithm", and
# converge to the forced orbit (DOP853) at the scheme's order.
# ---------------------------------------------------------------------------
def _forced_setup(vmod, sigma=20.0):
    mu, w, F = 1.3, 1.1, 0.3
    inst = W.Instance(1, (512, 1, 1), (-16.0, 0.0, 0.0), (16.0, 1.0, 1.0), mu=mu,
                      omega=((w, 0.0, 0.0, 0.0), CONST, CONST), sigma=(sigma, 0.0, 0.0, 0.0), eps=1.0,
                      vmod=vmod)
    x = inst.axis(0)
    return inst, mu, w, F, F * x


def _m(vmod, t):
    amp, fr, ph, form = vmod
    if form == 2:
        return 1.0 + amp * t / math.cosh(fr * (t - ph)) ** 2
    return 1.0 + amp * math.sin(fr * t + ph)


def _classical_split(scheme, mu, w, F, vmod, x0, p0, t0, h, n):
    a, b = oracle.scheme_coefficients(scheme)
    z = np.array([x0, p0])
    for s in range(n):
        tau = t0 + s * h
        z[1] -= h * b[0] * F * _m(vmod, tau)
        for i in range(len(a)):
            th = w * a[i] * h
            R = np.array([[math.cos(th), math.sin(th) / (mu * w)], [-mu * w * math.sin(th), math.cos(th)]])
            z = R @ z
            tau = tau + a[i] * h
            z[1] -= h * b[i + 1] * F * _m(vmod, tau)
    return z


@pytest.mark.parametrize("vmod", [(0.6, 2.0, 0.3, 0), (0.9, 1.5, 1.0, 2)])
@pytest.mark.parametrize("scheme", ["leapfrog", "ni5_84"])
def test_forced_kohn_mode_is_the_classical_split(vmod, scheme):
    inst, mu, w, F, vi = _forced_setup(vmod)
    x0, p0 = 1.2, -0.4
    u0 = gaussian(inst, (x0,), (mu * w,), (p0,))
    t0, h, n = 0.2, 0.02, 150
    u = oracle.evolve(inst, u0, scheme, "exact_const", h, t0, n, vi=vi)
    X, P = moments(inst, u)
    z = _classical_split(scheme, mu, w, F, vmod, x0, p0, t0, h, n)
    assert abs(X[0] - z[0]) < 1e-10 and abs(P[0] - z[1]) < 1e-10, (X, P, z)
    # the slip of holding m at t_n over the whole step misses by far more
    wrong = np.array([x0, p0])
    for s in range(n):
        tn = t0 + s * h
        frozen = (0.0, 0.0, 0.0, 0)
        wrong = _classical_split(scheme, mu, w, F * _m(vmod, tn), frozen, wrong[0], wrong[1], tn, h, 1)
    assert abs(wrong[0] - z[0]) + abs(wrong[1] - z[1]) > 1e-5


def test_forced_kohn_mode_order():
    """The centre of mass converges to the forced orbit (DOP853) at order 2
    (leapfrog) and 4 (NI5), with sigma = 20 acting on the density."""
    vmod = (0.6, 2.0, 0.3, 0)
    inst, mu, w, F, vi = _forced_setup(vmod)
    x0, p0, t0, T = 1.2, -0.4, 0.2, 2.0
    u0 = gaussian(inst, (x0,), (mu * w,), (p0,))
    sol = solve_ivp(lambda t, y: [y[1] / mu, -mu * w * w * y[0] - F * _m(vmod, t)], (t0, t0 + T), [x0, p0],
                    method="DOP853", rtol=1e-13, atol=1e-14)
    ref = sol.y[:, -1]
    for scheme, steps, order in (("leapfrog", (40, 80, 160), 2), ("ni5_84", (20, 40, 80), 4)):
        errs = []
        for n in steps:
            X, P = moments(inst, oracle.evolve(inst, u0, scheme, "exact_const", T / n, t0, n, vi=vi))
            errs.append(abs(X[0] - ref[0]) + abs(P[0] - ref[1]))
        rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert min(rates) > order - 0.3, (scheme, errs, rates)
