"""Pins of the oracle's coupled trap: V_HO = (mu/2) x^T W(t) x with
off-diagonal entries, constant or modulated in time (the general quadratic
potential x^T M(t) x of Sec. 1).

Expected values come from outside the oracle: scipy's matrix exponential and
DOP853 integrations of the 2d x 2d classical system, the d-dimensional
Gaussian-packet equations (a matrix Riccati equation), the normal-mode closed
form of the ground state, and Gaussian moments."""
import math

import numpy as np
import pytest
import scipy.linalg as sl
from scipy.integrate import solve_ivp

import oracle
import workloads as W


def modulation(m, t):
    """m(t) of a (amp, freq, phase, form) modulation, from its definition."""
    amp, fr, ph, form = m
    if form == 2:
        return 1.0 + amp * t / math.cosh(fr * (t - ph)) ** 2
    return 1.0 + amp * math.sin(fr * t + ph)


def wmat(inst, t):
    """W(t) written from its definition: W_jj = omega_j(t)^2, W_ij = wcross
    times its modulation."""
    d = inst.ndim
    M = np.zeros((d, d))
    for j in range(d):
        v0, a, f, ph = inst.omega[j][:4]
        M[j, j] = (v0 * (1.0 + a * math.sin(f * t + ph))) ** 2
    pairs = {(0, 1): 0, (0, 2): 1, (1, 2): 2}
    for (i, j), k in pairs.items():
        if i < d and j < d:
            M[i, j] = M[j, i] = inst.wcross[k] * modulation(inst.wmod[k], t)
    return M


def hamiltonian_matrix(inst, t):
    d, mu = inst.ndim, inst.mu
    return np.block([[np.zeros((d, d)), np.eye(d) / mu], [-mu * wmat(inst, t), np.zeros((d, d))]])


def flow_dop853(inst, t0, tau):
    n = 2 * inst.ndim
    sol = solve_ivp(lambda t, y: (hamiltonian_matrix(inst, t) @ y.reshape(n, n)).ravel(),
                    (t0, t0 + tau), np.eye(n).ravel(), method="DOP853", rtol=1e-13, atol=1e-15)
    return sol.y[:, -1].reshape(n, n)


NO_MOD = ((0.0, 0.0, 0.0, 0),) * 3
# modulated cross terms: a sine on W_xy, a pulse on W_xz, a sine on W_yz
WMOD = ((0.5, 2.3, 0.4, 0), (0.8, 2.0, 0.6, 2), (-0.4, 1.1, 0.0, 0))


def coupled(d=2, n=32, mu=1.0, omega=None, wcross=(0.3, 0.2, -0.25), L=6.0, wmod=NO_MOD):
    if omega is None:
        omega = ((1.2, 0.2, 1.5, 0.3), (0.9, 0.0, 0.0, 0.0), (1.4, 0.1, 0.7, 0.0))
    nn = tuple([n] * d + [1] * (3 - d))
    lo = tuple([-L] * d + [0.0] * (3 - d))
    hi = tuple([L] * d + [1.0] * (3 - d))
    return W.Instance(d, nn, lo, hi, mu=mu, omega=tuple(omega[:3]), wcross=tuple(wcross), wmod=tuple(wmod))


CONST = ((1.2, 0.0, 0.0, 0.0), (0.9, 0.0, 0.0, 0.0), (1.4, 0.0, 0.0, 0.0))


# ---------------------------------------------------------------------------
# stage matrices
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("mu,tau", [(1.0, 0.7), (1.6, -0.4), (0.5, 1.3)])
def test_exact_flow_is_matrix_exponential(d, mu, tau):
    inst = coupled(d=d, mu=mu, omega=CONST)
    S = oracle.stage_matrix_full(inst, "exact_const", 0.0, tau)
    ref = sl.expm(tau * hamiltonian_matrix(inst, 0.0))
    assert np.abs(S - ref).max() < 1e-14 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("d", [2, 3])
def test_cf4_local_order(d):
    inst = coupled(d=d, mu=1.3)
    errs = []
    for tau in (0.2, 0.1, 0.05):
        S = oracle.stage_matrix_full(inst, "cf4", 0.4, tau)
        errs.append(np.abs(S - flow_dop853(inst, 0.4, tau)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 4.6, (errs, rates)


@pytest.mark.parametrize("d", [2, 3])
def test_symplectic_and_factorisation(d):
    """A constant-W flow is symplectic and equals K(F) D(G) K(E) with symmetric
    F = E and G (per normal mode this is Lemma 2)."""
    inst = coupled(d=d, mu=0.8, omega=CONST)
    tau = 0.3
    S = oracle.stage_matrix_full(inst, "exact_const", 0.2, tau)
    J = np.block([[np.zeros((d, d)), np.eye(d)], [-np.eye(d), np.zeros((d, d))]])
    assert np.abs(S.T @ J @ S - J).max() < 1e-14
    trip = oracle.stage_coeffs_full(inst, "leapfrog", "exact_const", tau, 0.2)
    assert trip.shape == (1, 3, d, d)
    F, G, E = trip[0]
    for M in (F, G, E):
        assert np.abs(M - M.T).max() < 1e-13
    assert np.abs(F - E).max() < 1e-13
    I = np.eye(d)
    K = lambda C: np.block([[I, np.zeros((d, d))], [-C, I]])
    D = np.block([[I, G], [np.zeros((d, d)), I]])
    assert np.abs(K(F) @ D @ K(E) - S).max() < 1e-13


@pytest.mark.parametrize("d", [2, 3])
def test_cf4_product_leaves_the_kdk_family(d):
    """The two-exponential product has a non-symmetric S12 in general, so it is
    applied as two factor triples whose product reproduces it."""
    inst = coupled(d=d, mu=1.1)
    tau = 0.4
    S = oracle.stage_matrix_full(inst, "cf4", 0.3, tau)
    assert np.abs(S[:d, d:] - S[:d, d:].T).max() > 1e-6
    trip = oracle.stage_coeffs_full(inst, "leapfrog", "cf4", tau, 0.3)
    assert trip.shape == (2, 3, d, d)
    I = np.eye(d)
    K = lambda C: np.block([[I, np.zeros((d, d))], [-C, I]])
    D = lambda G: np.block([[I, G], [np.zeros((d, d)), I]])
    prod = np.eye(2 * d)
    for F, G, E in trip:       # later triples act last
        prod = K(F) @ D(G) @ K(E) @ prod
    assert np.abs(prod - S).max() < 1e-13


def test_unsupported_rules_rejected():
    inst = coupled(d=2)
    for rule in ("magnus6", "fundamental"):
        with pytest.raises(RuntimeError):
            oracle.stage_matrix_full(inst, rule, 0.0, 0.1)


# ---------------------------------------------------------------------------
# evolution: d-D Gaussian packets (matrix Riccati reference)
# ---------------------------------------------------------------------------
def gaussian_packet(inst, A0, b0, c0, t0, T):
    """psi = exp(x^T A x + b^T x + c) with A complex symmetric solves
    i psi_t = -Lap psi/(2 mu) + (mu/2) x^T W(t) x psi when
      A' = (2i/mu) A^2 - (i mu/2) W,  b' = (2i/mu) A b,  c' = (i/mu)(tr A + b^T b / 2)."""
    d, mu = inst.ndim, inst.mu

    def pack(A, b, c):
        z = np.concatenate([A.ravel(), b, [c]])
        return np.concatenate([z.real, z.imag])

    def unpack(y):
        n = d * d + d + 1
        z = y[:n] + 1j * y[n:]
        return z[: d * d].reshape(d, d), z[d * d: d * d + d], z[-1]

    def rhs(t, y):
        A, b, c = unpack(y)
        dA = 2j / mu * A @ A - 0.5j * mu * wmat(inst, t)
        db = 2j / mu * A @ b
        dc = 1j / mu * (np.trace(A) + 0.5 * b @ b)
        return pack(dA, db, dc)

    sol = solve_ivp(rhs, (t0, T), pack(A0, b0, c0), method="DOP853", rtol=1e-13, atol=1e-14)
    A, b, c = unpack(sol.y[:, -1])
    X = np.stack([m * np.ones(inst.shape) for m in inst.mesh()], axis=-1)
    q = np.einsum("...i,ij,...j->...", X, A, X)
    return np.exp(q + X @ b + c)


def initial_packet(inst, centre):
    d = inst.ndim
    A0 = -0.5 * np.diag(np.linspace(1.0, 1.3, d)).astype(complex)
    b0 = (-2.0 * A0 @ np.array(centre[:d])).astype(complex)
    X = np.stack([m * np.ones(inst.shape) for m in inst.mesh()], axis=-1)
    psi = np.exp(np.einsum("...i,ij,...j->...", X, A0, X) + X @ b0)
    return A0, b0, psi


def test_rotated_ground_state_is_stationary():
    """Constant coupled W: the ground state exp(-(mu/2) x^T Q diag(w) Q^T x) only
    rotates its phase, by T sum(w)/2 (normal modes, Lemma 2 per mode)."""
    inst = coupled(d=2, n=128, mu=1.2, omega=CONST, wcross=(0.35, 0.0, 0.0), L=9.0)
    Wm = wmat(inst, 0.0)
    lam, Q = np.linalg.eigh(Wm)
    Om = Q @ np.diag(np.sqrt(lam)) @ Q.T
    X = np.stack([m * np.ones(inst.shape) for m in inst.mesh()], axis=-1)
    g0 = np.exp(-0.5 * inst.mu * np.einsum("...i,ij,...j->...", X, Om, X))
    T = 2.5
    u = oracle.evolve(inst, g0, "leapfrog", "exact_const", T / 5, 0.0, 5)
    assert W.rel_l2(u, np.exp(-0.5j * T * np.sqrt(lam).sum()) * g0) < 1e-12


@pytest.mark.parametrize("d", [2, 3])
def test_constant_coupled_trap_exact_in_time(d):
    """Linear, constant W, exact rule: the HF step is exact whatever the step."""
    # the squeezed packet breathes out to exp(-0.25 x^2): boxes wide enough for round-off
    n = 128 if d == 2 else 64
    inst = coupled(d=d, n=n, mu=0.9, omega=CONST, L=12.0 if d == 2 else 10.0)
    A0, b0, psi0 = initial_packet(inst, (0.5, -0.3, 0.2))
    T = 1.5
    ref = gaussian_packet(inst, A0, b0, 0j, 0.0, T)
    u = oracle.evolve(inst, psi0, "leapfrog", "exact_const", T / 3, 0.0, 3)
    assert W.rel_l2(u, ref) < (1e-11 if d == 2 else 1e-9)


@pytest.mark.parametrize("scheme,rule,order", [("leapfrog", "cf4", 4), ("ni5_84", "cf4", 4),
                                               ("leapfrog", "fsplit", 2), ("ni5_84", "fsplit", 4)])
def test_time_dependent_coupled_order(scheme, rule, order):
    inst = coupled(d=2, n=128, mu=1.0, L=12.0)
    A0, b0, psi0 = initial_packet(inst, (0.5, -0.3, 0.0))
    T = 1.0
    ref = gaussian_packet(inst, A0, b0, 0j, 0.0, T)
    errs = []
    for nst in (8, 16, 32):
        errs.append(W.rel_l2(oracle.evolve(inst, psi0, scheme, rule, T / nst, 0.0, nst), ref))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > order - 0.4, (errs, rates)


def test_coupled_potential_energy():
    """(mu/2) <x^T W x> = (mu/2) tr(W Sigma) for |u|^2 a Gaussian of covariance Sigma."""
    inst = coupled(d=2, n=128, mu=1.4, wcross=(0.4, 0.0, 0.0), L=9.0)
    P = np.array([[1.0, 0.3], [0.3, 0.8]])
    X = np.stack([m * np.ones(inst.shape) for m in inst.mesh()], axis=-1)
    u = np.exp(-0.5 * np.einsum("...i,ij,...j->...", X, P, X)).astype(complex)
    u /= math.sqrt(inst.cell * np.sum(np.abs(u) ** 2))
    Sigma = np.linalg.inv(2.0 * P)      # |u|^2 ~ exp(-x^T P x)
    t = 0.7
    e = oracle.energy(inst, u, t)
    assert abs(e[2] - 0.5 * inst.mu * np.trace(wmat(inst, t) @ Sigma)) < 1e-12


# ---------------------------------------------------------------------------
# modulated cross terms W_ij(t) (Sec. 1's M(t))
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d", [2, 3])
def test_cf4_local_order_modulated_cross_terms(d):
    """The commutator-free rule averages the whole W(t), cross terms included,
    at its Gauss nodes: local order 4 against DOP853 of the classical system."""
    inst = coupled(d=d, mu=1.3, wmod=WMOD)
    errs = []
    for tau in (0.2, 0.1, 0.05):
        S = oracle.stage_matrix_full(inst, "cf4", 0.4, tau)
        errs.append(np.abs(S - flow_dop853(inst, 0.4, tau)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 4.6, (errs, rates)
    # a rule that froze the cross terms at the stage start would lose the order:
    # the same instance with W_ij held at their t = 0.4 values differs at O(tau^2)
    frozen = coupled(d=d, mu=1.3, wmod=NO_MOD,
                     wcross=tuple(c * modulation(m, 0.4) for c, m in zip((0.3, 0.2, -0.25), WMOD)))
    e_frozen = np.abs(oracle.stage_matrix_full(frozen, "cf4", 0.4, 0.05) - flow_dop853(inst, 0.4, 0.05)).max()
    assert e_frozen > 100 * errs[-1]


@pytest.mark.parametrize("scheme,rule,order", [("leapfrog", "cf4", 4), ("ni5_84", "cf4", 4),
                                               ("leapfrog", "fsplit", 2), ("ni5_84", "fsplit", 4)])
def test_modulated_coupled_order(scheme, rule, order):
    """Linear evolution with W_xy(t) modulated: global order against the
    Gaussian packet of the matrix Riccati equation."""
    inst = coupled(d=2, n=128, mu=1.0, L=12.0, wcross=(0.35, 0.0, 0.0), wmod=WMOD)
    A0, b0, psi0 = initial_packet(inst, (0.5, -0.3, 0.0))
    T = 1.0
    ref = gaussian_packet(inst, A0, b0, 0j, 0.0, T)
    errs = []
    for nst in (8, 16, 32):
        errs.append(W.rel_l2(oracle.evolve(inst, psi0, scheme, rule, T / nst, 0.0, nst), ref))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > order - 0.4, (errs, rates)


def test_modulated_coupled_3d_order():
    inst = coupled(d=3, n=64, mu=1.1, L=10.0, wmod=WMOD)
    A0, b0, psi0 = initial_packet(inst, (0.4, -0.3, 0.2))
    T = 0.8
    ref = gaussian_packet(inst, A0, b0, 0j, 0.0, T)
    errs = [W.rel_l2(oracle.evolve(inst, psi0, "leapfrog", "cf4", T / n, 0.0, n, threads=4), ref)
            for n in (8, 16, 32)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 3.6, (errs, rates)


def test_modulated_coupled_potential_energy():
    inst = coupled(d=2, n=128, mu=1.4, wcross=(0.4, 0.0, 0.0), L=9.0, wmod=WMOD)
    P = np.array([[1.0, 0.3], [0.3, 0.8]])
    X = np.stack([m * np.ones(inst.shape) for m in inst.mesh()], axis=-1)
    u = np.exp(-0.5 * np.einsum("...i,ij,...j->...", X, P, X)).astype(complex)
    u /= math.sqrt(inst.cell * np.sum(np.abs(u) ** 2))
    Sigma = np.linalg.inv(2.0 * P)
    for t in (0.0, 0.7, 2.1):
        e = oracle.energy(inst, u, t)
        assert abs(e[2] - 0.5 * inst.mu * np.trace(wmat(inst, t) @ Sigma)) < 1e-12
