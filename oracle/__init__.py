"""FP64 CPU oracle for the Hermite-Fourier split-step integrator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
never imports, links or calls it, and the two share no code: the oracle has its
own FFT, its own coefficient route (build the 2x2 classical matrix of each
harmonic-oscillator stage, then factor it as K(f) D(g) K(e)), its own copy of
the splitting-coefficient tables, and it applies every flow of a step one after
the other without merging adjacent x-phases.

Paper: P. Bader and S. Blanes, "Fourier methods for the perturbed harmonic
oscillator in linear and nonlinear Schroedinger equations", arXiv:1007.3470.

Parity status per function (the pins live in ``tests/test_oracle_*.py``):
  fftn            pinned: brute-force DFT, round trip, Parseval
  stage_matrix    pinned: Lemma 2 / Theorem 1 / Theorem 2 closed forms,
                  local order against an RK4-integrated fundamental matrix;
                  the fundamental-matrix rule against scipy's DOP853 solution
                  of the same 2x2 system, its sub-step order, and its
                  reductions (one sub-step = Magnus6; constant omega = exact)
  stage_coeffs    pinned: K(f) D(g) K(e) product reproduces the stage matrix
  coupled trap    pinned: stage matrix vs scipy expm / DOP853; symplectic, F and E
                  symmetric, K(F) D(G) K(E) reproduces S; rotated-trap coherent
                  state and ground state closed forms; d-D Gaussian-packet
                  (matrix Riccati) reference for the time-dependent order
  evolve          pinned: coherent-state closed form (linear, constant omega),
                  ground-state single step (Fig. 1 experiment), norm
                  conservation, time reversibility, observed order under
                  step halving, linear time-dependent exact reference; the
                  nonlinear evolution against exact identities of the GPE:
                  the Kohn mode (centre of mass = classical orbit for any
                  sigma, also coupled and time-dependent) and the 2-D
                  breathing mode (which fixes the nonlinear coefficient)
  evolve(vi=...)  pinned: equals the factor form; a linear potential's
                  shifted ground state (closed form)
  sigma(t) in B   pinned: on a one-point grid the step is the ODE
                  i u' = (eps V_I + sigma(t)|u|^2) u, and its phase equals the
                  stage-time quadrature of Table "algorithm" written out from
                  the printed Table tab.1 values, converging to the closed-form
                  integral at orders 2 (leapfrog), 4 (SRKN6_4), >= 6 (NI4, NI5);
                  time reversibility and orders 2 / 4 with time-dependent
                  sigma(t) (sine and pulse); sigma frozen at t_n, built in the
                  test, fails both
  V_I factors     pinned: potential energy and the B flow of the factor form
                  (c0 + c2 x^2 + c4 x^4) exp(-x^2/gs) cos(k x + phi) against
                  NumPy evaluations of the formula, with gs, c4 and the other
                  coefficients varied
  norm, energy    pinned: closed-form Gaussian values
  scheme_coefficients
                  pinned: sums, palindromes and quadrature moments of the
                  B weights; the values printed in Table tab.1 (stored with
                  their citation under tests/golden/)
The absolute trajectory of nonlinear, time-dependent runs has no independent
exact value; it is trusted through the pins above.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hfgpe_oracle.c")
_SO = os.path.join(_HERE, "libhfgpe_oracle.so")
_LIB = None

NPAR = 59
HO_RULES = {"exact_const": 0, "cf4": 1, "magnus6": 2, "fsplit": 3, "fundamental": 4}
FUNDAMENTAL_DEFAULT_SUBSTEPS = 16
_ERRORS = {-1: "invalid argument", -2: "singular stage (g = 0)",
           -3: "non-positive squared frequency", -4: "out of memory"}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99 with OpenMP loops, no FMA
    contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fopenmp", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _LIB
    if _LIB is None:
        build()
        lib = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.orc_fftn.argtypes = [ctypes.c_int, ip, dp, ctypes.c_int]
        lib.orc_stage_matrix.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_int,
                                         ctypes.c_double, ctypes.c_double, dp]
        lib.orc_stage_coeffs.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]
        lib.orc_evolve.argtypes = [ctypes.c_int, ip, dp, dp, dp, ctypes.c_int, dp, dp,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_long, dp, dp, ctypes.c_int]
        lib.orc_drift.argtypes = [ctypes.c_int, ip, dp, dp, dp, dp]
        lib.orc_stage_matrix_full.argtypes = [ctypes.c_int, dp, ctypes.c_int, ctypes.c_double,
                                              ctypes.c_double, dp]
        lib.orc_stage_coeffs_full.argtypes = [ctypes.c_int, dp, ctypes.c_int, dp, ctypes.c_int,
                                              ctypes.c_double, ctypes.c_double, dp, ip]
        lib.orc_norm.argtypes = [ctypes.c_int, ip, dp, dp, dp, dp]
        lib.orc_energy.argtypes = [ctypes.c_int, ip, dp, dp, dp, ctypes.c_double, dp, dp, dp,
                                   ctypes.c_int]
        assert lib.orc_npar() == NPAR
        _LIB = lib
    return _LIB


def rule_id(name: str):
    """Rule name -> (rule number, sub-steps).  "fundamental:q" integrates each
    stage with q sixth-order Magnus sub-steps ("fundamental": 16)."""
    base, _, q = name.partition(":")
    if base == "fundamental":
        return HO_RULES[base], int(q) if q else FUNDAMENTAL_DEFAULT_SUBSTEPS
    return HO_RULES[base], 0


def _check(rc: int) -> None:
    if rc != 0:
        raise RuntimeError("oracle error %d: %s" % (rc, _ERRORS.get(rc, "?")))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


# ---------------------------------------------------------------------------
# Splitting coefficients: the oracle's own copy of Table "tab.1".
# Each scheme is (a[0..m-1], b[0..m]) for the BAB composition of Eq. prod-gen.
# NI4(8,2): b2 is printed as 49/18; read as 49/180, the 5-point Gauss-Lobatto
# weight (with 49/18 the weights do not even sum to a consistent quadrature).
# ---------------------------------------------------------------------------
def scheme_coefficients(name: str):
    if name == "leapfrog":  # Eq. LeapFrogB: B(h/2) A(h) B(h/2)
        return [1.0], [0.5, 0.5]
    if name == "lie":  # first-order B(h) A(h)
        return [1.0], [1.0, 0.0]
    if name == "srkn6_4":
        b1, b2, b3 = 0.0829844064174052, 0.396309801498368, -0.0390563049223486
        b4 = 1.0 - 2.0 * (b1 + b2 + b3)
        a1, a2 = 0.245298957184271, 0.604872665711080
        a3 = 0.5 - (a1 + a2)
        return [a1, a2, a3, a3, a2, a1], [b1, b2, b3, b4, b3, b2, b1]
    if name == "ni4_82":
        b1, b2 = 1.0 / 20.0, 49.0 / 180.0
        b3 = 1.0 - 2.0 * (b1 + b2)
        a1 = 0.5 - math.sqrt(3.0 / 28.0)
        a2 = 0.5 - a1
        return [a1, a2, a2, a1], [b1, b2, b3, b2, b1]
    if name == "ni5_84":
        b1, b2 = 0.811862738544516, -0.677480399532169
        b3 = 0.5 - (b1 + b2)
        a1, a2 = -0.00758691311877447, 0.317218277973169
        a3 = 1.0 - 2.0 * (a1 + a2)
        return [a1, a2, a3, a2, a1], [b1, b2, b3, b3, b2, b1]
    raise ValueError("unknown scheme %r" % name)


def params_block(inst) -> np.ndarray:
    """Flatten an instance description into the oracle's parameter block.
    omega[j] and sigma are (v0, amp, freq, phase[, form])."""
    p = np.zeros(NPAR)
    p[0] = inst.mu
    for j in range(3):
        p[1 + 4 * j: 5 + 4 * j] = inst.omega[j][:4]
        p[36 + j] = inst.omega[j][4] if len(inst.omega[j]) > 4 else 0
        p[18 + 6 * j: 24 + 6 * j] = inst.vfac[j]
    p[13:17] = inst.sigma[:4]
    p[39] = inst.sigma[4] if len(inst.sigma) > 4 else 0
    p[17] = inst.eps
    p[40:43] = getattr(inst, "wcross", (0.0, 0.0, 0.0))
    p[43:47] = getattr(inst, "vmod", (0.0, 0.0, 0.0, 0))
    for k, m in enumerate(getattr(inst, "wmod", ((0.0, 0.0, 0.0, 0),) * 3)):
        p[47 + 4 * k: 51 + 4 * k] = m
    return p


def _grid_arrays(inst):
    n = np.array(list(inst.n) + [1] * (3 - len(inst.n)), dtype=np.int32)[:3]
    lo = np.array(list(inst.lo) + [0.0] * (3 - len(inst.lo)), dtype=np.float64)[:3]
    hi = np.array(list(inst.hi) + [1.0] * (3 - len(inst.hi)), dtype=np.float64)[:3]
    return n, lo, hi


def _as_c128(psi: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(psi, dtype=np.complex128).copy()


def fftn(z: np.ndarray, sign: int = -1) -> np.ndarray:
    """The oracle's own d-D FFT.  ``z`` has shape (n,), (ny, nx) or (nz, ny, nx)
    with x fastest; sign -1 forward unnormalised, +1 inverse scaled by 1/N."""
    out = _as_c128(z)
    shape = out.shape
    n = np.array(list(reversed(shape)), dtype=np.int32)
    _check(_lib().orc_fftn(len(shape), _ip(n), _dp(out.view(np.float64)), int(sign)))
    return out


def stage_matrix(inst, rule: str, axis: int, t0: float, tau: float) -> np.ndarray:
    S = np.zeros(4)
    _check(_lib().orc_stage_matrix(*rule_id(rule), _dp(params_block(inst)), axis, t0, tau,
                                   _dp(S)))
    return S.reshape(2, 2)


def stage_matrix_full(inst, rule: str, t0: float, tau: float) -> np.ndarray:
    """2d x 2d stage matrix S of a coupled trap (non-diagonal W), acting on (x, p)."""
    d = inst.ndim
    S = np.zeros(4 * d * d)
    _check(_lib().orc_stage_matrix_full(HO_RULES[rule], _dp(params_block(inst)), d, t0, tau,
                                        _dp(S)))
    return S.reshape(2 * d, 2 * d)


def stage_coeffs_full(inst, scheme: str, rule: str, dt: float, tn: float) -> np.ndarray:
    """F, G, E (d x d each) of every factor triple of a coupled-trap step, in
    the order they act (one per stage for exact_const, two for cf4):
    shape (triples, 3, d, d)."""
    a, _ = scheme_coefficients(scheme)
    a = np.array(a)
    d = inst.ndim
    out = np.zeros(2 * len(a) * 3 * d * d)
    nout = np.zeros(1, dtype=np.int32)
    _check(_lib().orc_stage_coeffs_full(d, _dp(params_block(inst)), len(a), _dp(a),
                                        HO_RULES[rule], dt, tn, _dp(out), _ip(nout)))
    k = int(nout[0])
    return out[: k * 3 * d * d].reshape(k, 3, d, d)


def stage_coeffs(inst, scheme: str, rule: str, dt: float, tn: float) -> np.ndarray:
    """(f, g, e) per stage and axis of the step starting at tn: shape (m, ndim, 3)."""
    a, _ = scheme_coefficients(scheme)
    a = np.array(a)
    out = np.zeros(len(a) * inst.ndim * 3)
    _check(_lib().orc_stage_coeffs(inst.ndim, _dp(params_block(inst)), len(a), _dp(a),
                                   *rule_id(rule), dt, tn, _dp(out)))
    return out.reshape(len(a), inst.ndim, 3)


def _vi_ptr(inst, vi):
    if vi is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(vi, dtype=np.float64).reshape(inst.shape))
    return arr, _dp(arr)


def evolve(inst, psi: np.ndarray, scheme: str, rule: str, dt: float, t0: float,
           nsteps: int, vi=None, threads: int = 1) -> np.ndarray:
    """Advance one instance ``nsteps`` steps of size ``dt`` from ``t0``.  ``vi``
    (optional, shape of the grid) gives eps V_I at every point and replaces
    the instance's factor form.  ``threads`` splits the pencil and point loops
    of the C code; the result is bitwise the same for any thread count."""
    a, b = scheme_coefficients(scheme)
    a, b = np.array(a), np.array(b)
    n, lo, hi = _grid_arrays(inst)
    out = _as_c128(psi)
    keep, vp = _vi_ptr(inst, vi)
    _check(_lib().orc_evolve(inst.ndim, _ip(n), _dp(lo), _dp(hi), _dp(params_block(inst)),
                             len(a), _dp(a), _dp(b), *rule_id(rule), float(dt), float(t0),
                             int(nsteps), vp, _dp(out.view(np.float64)), int(threads)))
    return out


def drift(inst, psi: np.ndarray, g) -> np.ndarray:
    """Apply the drift D(g) = F^-1 exp(-i sum_j g_j k_j^2/2) F alone."""
    n, lo, hi = _grid_arrays(inst)
    out = _as_c128(psi)
    gg = np.zeros(3)
    gg[: len(g)] = g
    _check(_lib().orc_drift(inst.ndim, _ip(n), _dp(lo), _dp(hi), _dp(gg),
                            _dp(out.view(np.float64))))
    return out


def norm(inst, psi: np.ndarray) -> float:
    """h^d sum |u|^2 with compensated summation."""
    n, lo, hi = _grid_arrays(inst)
    z = _as_c128(psi)
    out = np.zeros(1)
    _check(_lib().orc_norm(inst.ndim, _ip(n), _dp(lo), _dp(hi), _dp(z.view(np.float64)),
                           _dp(out)))
    return float(out[0])


def energy(inst, psi: np.ndarray, t: float, vi=None, threads: int = 1) -> np.ndarray:
    """[total, kinetic, potential, interaction] energy at time t (``vi`` and
    ``threads`` as in ``evolve``; the sums themselves are sequential)."""
    n, lo, hi = _grid_arrays(inst)
    z = _as_c128(psi)
    out = np.zeros(4)
    keep, vp = _vi_ptr(inst, vi)
    _check(_lib().orc_energy(inst.ndim, _ip(n), _dp(lo), _dp(hi), _dp(params_block(inst)),
                             float(t), vp, _dp(z.view(np.float64)), _dp(out), int(threads)))
    return out
