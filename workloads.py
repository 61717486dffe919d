"""Seeded synthetic inputs for the Hermite-Fourier GPE time step.

This module only describes problems and draws initial data; it contains none
of the method's arithmetic (no FFT, no coefficients, no phases).  Both the GPU
library's tests/benchmark and the CPU oracle start from the bytes it produces.

Physics (Sec. 1 of the paper, Eq. GP1 generalised to d dimensions):
    i psi_t = ( p^2/(2 mu) + sum_j mu omega_j(t)^2 x_j^2 / 2
                + eps V_I(x) + sigma(t) |psi|^2 ) psi
with omega_j(t) and sigma(t) given as (v0, amp, freq, phase[, form]):
    form 0 (default)  v(t)   = v0 (1 + amp sin(freq t + phase))
    form 1            v(t)^2 = v0 (1 + amp sin(freq t + phase))   (omega only)
    form 2            v(t)   = v0 (1 + amp t / cosh^2(freq (t - phase)))
    V_I(x)     = prod_j (c0 + c2 x_j^2 + c4 x_j^4) exp(-x_j^2/gs) cos(k x_j + phi)
                 (the Gaussian factor is dropped when gs == 0).
Grid: x_{j,i} = lo_j + i (hi_j - lo_j)/n_j, periodic, arrays stored with x
fastest (numpy shape (nz, ny, nx) / (ny, nx) / (nx,)).

Workloads follow the five benchmark configurations of the project: a 1-D
coherent state, a 1-D GPE with a time-dependent trap, a heterogeneous batch of
4096 1-D GPEs, 16 anisotropic 2-D GPEs and one 3-D GPE.  Two more recipes
follow the paper's own numerical examples: the weakly to strongly nonlinear
problem of Sec. 4.1 (Figs. 2-6) and the time-dependent traps with a quartic
perturbation of Sec. 4.2 (Figs. 7-8).  Every generator takes size overrides so
tests can run the same recipe at small sizes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

NO_V = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)      # v_j(x) = 1
CONST_OMEGA = (1.0, 0.0, 0.0, 0.0)


@dataclass(frozen=True)
class Instance:
    ndim: int
    n: Tuple[int, int, int]
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    mu: float = 1.0
    omega: Tuple[Tuple[float, float, float, float], ...] = (CONST_OMEGA,) * 3
    sigma: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)
    eps: float = 0.0
    vfac: Tuple[Tuple[float, ...], ...] = (NO_V,) * 3
    # off-diagonal W_xy, W_xz, W_yz of the squared-frequency matrix of a coupled
    # trap V_HO = (mu/2) x^T W(t) x, W_jj = omega_j(t)^2, each times its
    # modulation in wmod
    wcross: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    # time modulations (amp, freq, phase, form) of eps V_I and of W_xy, W_xz,
    # W_yz: form 0: m(t) = 1 + amp sin(freq t + phase); form 2: m(t) = 1 + amp t
    # / cosh^2(freq (t - phase)); all zero: static
    vmod: Tuple[float, float, float, int] = (0.0, 0.0, 0.0, 0)
    wmod: Tuple[Tuple[float, float, float, int], ...] = ((0.0, 0.0, 0.0, 0),) * 3

    @property
    def points(self) -> int:
        return int(np.prod(self.n[: self.ndim]))

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(reversed(self.n[: self.ndim]))

    def axis(self, j: int) -> np.ndarray:
        """Grid coordinates along axis j (x_i = lo + i*(hi-lo)/n)."""
        return self.lo[j] + np.arange(self.n[j]) * ((self.hi[j] - self.lo[j]) / self.n[j])

    def mesh(self) -> List[np.ndarray]:
        """Broadcastable coordinate arrays [x, y, z] matching ``shape``."""
        out = []
        for j in range(self.ndim):
            s = [1] * self.ndim
            s[self.ndim - 1 - j] = self.n[j]
            out.append(self.axis(j).reshape(s))
        return out

    @property
    def cell(self) -> float:
        return float(np.prod([(self.hi[j] - self.lo[j]) / self.n[j] for j in range(self.ndim)]))


@dataclass
class Workload:
    name: str
    instances: List[Instance]
    psi0: List[np.ndarray]
    scheme: str
    ho_rule: str
    dt: float
    nsteps: int
    t0: float = 0.0
    notes: str = ""

    @property
    def points(self) -> int:
        return sum(i.points for i in self.instances)


def _normalise(inst: Instance, u: np.ndarray) -> np.ndarray:
    return u / math.sqrt(inst.cell * float(np.sum(np.abs(u) ** 2)))


def _grid1(n: int, lo: float, hi: float) -> Tuple[Tuple[int, int, int], Tuple, Tuple]:
    return (n, 1, 1), (lo, 0.0, 0.0), (hi, 1.0, 1.0)


# ---------------------------------------------------------------------------
# C1: 1-D linear harmonic oscillator, coherent state (FP64)
# ---------------------------------------------------------------------------
def coherent_1d(n: int = 256, lo: float = -10.0, hi: float = 10.0, x0: float = 1.0,
                dt: float = 0.01, nsteps: int = 1000, omega: float = 1.0,
                mu: float = 1.0) -> Workload:
    g = _grid1(n, lo, hi)
    inst = Instance(1, *g, mu=mu, omega=((omega, 0.0, 0.0, 0.0),) + (CONST_OMEGA,) * 2)
    x = inst.axis(0)
    # ground state of p^2/(2mu) + mu w^2 x^2/2 displaced to x0
    s = mu * omega
    psi = (s / math.pi) ** 0.25 * np.exp(-s * (x - x0) ** 2 / 2.0)
    return Workload("coherent_1d", [inst], [psi.astype(np.complex128)], "leapfrog",
                    "exact_const", dt, nsteps,
                    notes="mu=%g omega=%g, N=%d on [%g,%g), x0=%g" % (mu, omega, n, lo, hi, x0))


# ---------------------------------------------------------------------------
# C2: 1-D GPE with omega(t) = 1 + 0.5 sin 2t, quartic-Gaussian V_I, sigma = 10
# ---------------------------------------------------------------------------
def gpe_1d(n: int = 1024, lo: float = -16.0, hi: float = 16.0, dt: float = 1e-3,
           nsteps: int = 10000, seed: int = 10072, scheme: str = "leapfrog",
           rule: str = "cf4", sigma: float = 10.0, noise: float = 1e-3) -> Workload:
    g = _grid1(n, lo, hi)
    inst = Instance(1, *g, omega=((1.0, 0.5, 2.0, 0.0),) + (CONST_OMEGA,) * 2,
                    sigma=(sigma, 0.0, 0.0, 0.0), eps=0.01,
                    vfac=((0.0, 0.0, 1.0, 16.0, 0.0, 0.0), NO_V, NO_V))
    rng = np.random.default_rng(seed)
    x = inst.axis(0)
    psi = np.exp(-x ** 2 / 2.0) + noise * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    return Workload("gpe_1d", [inst], [_normalise(inst, psi)], scheme, rule, dt, nsteps,
                    notes="N=%d on [%g,%g), sigma=%g, seed %d" % (n, lo, hi, sigma, seed))


# ---------------------------------------------------------------------------
# C3: batch of independent 1-D GPEs with their own N, omega(t), sigma
# ---------------------------------------------------------------------------
def batch_1d(n_inst: int = 4096, sizes=(256, 512, 1024, 2048), dt: float = 1e-3,
             nsteps: int = 5000, seed: int = 34701, scheme: str = "leapfrog",
             rule: str = "cf4") -> Workload:
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.array(sizes), size=n_inst)
    w0 = rng.uniform(0.5, 2.0, n_inst)
    amp = rng.uniform(0.0, 0.5, n_inst)
    nu = rng.uniform(0.5, 3.0, n_inst)
    sig = rng.uniform(-1.0, 50.0, n_inst)
    x0 = rng.uniform(-1.0, 1.0, n_inst)
    insts, psis = [], []
    for i in range(n_inst):
        n = int(ns[i])
        L = n / 64.0
        inst = Instance(1, *_grid1(n, -L, L),
                        omega=((float(w0[i]), float(amp[i]), float(nu[i]), 0.0),)
                        + (CONST_OMEGA,) * 2,
                        sigma=(float(sig[i]), 0.0, 0.0, 0.0), eps=0.01,
                        vfac=((1.0, 0.0, 0.0, 0.0, 3.0, 0.0), NO_V, NO_V))
        x = inst.axis(0)
        insts.append(inst)
        psis.append(_normalise(inst, np.exp(-(x - x0[i]) ** 2 / 2.0).astype(np.complex128)))
    return Workload("batch_1d", insts, psis, scheme, rule, dt, nsteps,
                    notes="%d instances, N in %s, seed %d" % (n_inst, list(sizes), seed))


# ---------------------------------------------------------------------------
# C4: 16 anisotropic 2-D GPEs, omega_y(t) = 1.5 + 0.3 sin t, sigma = 100
# ---------------------------------------------------------------------------
def gpe_2d(n: int = 512, n_inst: int = 16, lo: float = -12.0, hi: float = 12.0,
           dt: float = 5e-4, nsteps: int = 2000, seed: int = 34702,
           scheme: str = "leapfrog", rule: str = "cf4") -> Workload:
    rng = np.random.default_rng(seed)
    insts, psis = [], []
    for _ in range(n_inst):
        jit = 1.0 + rng.uniform(-0.1, 0.1, 4)   # wx, 1.5, 0.3, sigma
        c = rng.uniform(-0.5, 0.5, 2)
        wx, wy0, wy1, sig = 1.0 * jit[0], 1.5 * jit[1], 0.3 * jit[2], 100.0 * jit[3]
        sinx = (1.0, 0.0, 0.0, 0.0, 1.0, -math.pi / 2.0)   # cos(x - pi/2) = sin x
        inst = Instance(2, (n, n, 1), (lo, lo, 0.0), (hi, hi, 1.0),
                        omega=((wx, 0.0, 0.0, 0.0), (wy0, wy1 / wy0, 1.0, 0.0), CONST_OMEGA),
                        sigma=(sig, 0.0, 0.0, 0.0), eps=0.01, vfac=(sinx, sinx, NO_V))
        x, y = inst.mesh()
        psi = np.exp(-wx * (x - c[0]) ** 2 / 2.0 - wy0 * (y - c[1]) ** 2 / 2.0)
        insts.append(inst)
        psis.append(_normalise(inst, psi.astype(np.complex128)))
    return Workload("gpe_2d", insts, psis, scheme, rule, dt, nsteps,
                    notes="%d x %d^2 on [%g,%g)^2, seed %d" % (n_inst, n, lo, hi, seed))


# ---------------------------------------------------------------------------
# C5: one 3-D GPE, fourth-order composition
# ---------------------------------------------------------------------------
def gpe_3d(n: int = 256, lo: float = -8.0, hi: float = 8.0, dt: float = 1e-3,
           nsteps: int = 500, seed: int = 34703, scheme: str = "ni5_84",
           rule: str = "cf4", sigma: float = 500.0) -> Workload:
    rng = np.random.default_rng(seed)
    w0 = (1.0, 1.2, 1.5)
    c = rng.uniform(-0.5, 0.5, 3)
    cos2 = (1.0, 0.0, 0.0, 0.0, 2.0, 0.0)
    inst = Instance(3, (n, n, n), (lo,) * 3, (hi,) * 3,
                    omega=tuple((w, 0.2, 1.3, 0.0) for w in w0),
                    sigma=(sigma, 0.0, 0.0, 0.0), eps=0.01, vfac=(cos2, cos2, cos2))
    x, y, z = inst.mesh()
    psi = np.exp(-(w0[0] * (x - c[0]) ** 2 + w0[1] * (y - c[1]) ** 2
                   + w0[2] * (z - c[2]) ** 2) / 2.0)
    return Workload("gpe_3d", [inst], [_normalise(inst, psi.astype(np.complex128))], scheme,
                    rule, dt, nsteps, notes="%d^3 on [%g,%g)^3, seed %d" % (n, lo, hi, seed))


# ---------------------------------------------------------------------------
# Sec. 4.1 (Figs. 2-6): mu = omega = 1, V_I = 0, sigma in {0.01, 1, 100},
# psi(x, 0) = rho exp(-(x-1)^2/2); [-20, 20] for sigma = 0.01, [-30, 30] else.
# The figures (absent) hold N and T; N = 1024 and T = 10 are this recipe's.
# ---------------------------------------------------------------------------
def perturbed_1d(sigma: float = 1.0, n: int = 1024, T: float = 10.0, nsteps: int = 1000,
                 scheme: str = "leapfrog", rule: str = "exact_const") -> Workload:
    L = 20.0 if sigma < 0.1 else 30.0
    inst = Instance(1, *_grid1(n, -L, L), sigma=(float(sigma), 0.0, 0.0, 0.0))
    x = inst.axis(0)
    psi = _normalise(inst, np.exp(-(x - 1.0) ** 2 / 2.0).astype(np.complex128))
    return Workload("perturbed_1d", [inst], [psi], scheme, rule, T / nsteps, nsteps,
                    notes="sigma=%g, N=%d on [%g,%g), T=%g" % (sigma, n, -L, L, T))


# ---------------------------------------------------------------------------
# Sec. 4.2 (Figs. 7-8): linear HO with a time-dependent frequency plus the
# static quartic eps_Q x^4/4, eps_Q = 0.01, on [-20, 20]:
#   "cos":   omega^2(t) = 4 (1 + 0.1 cos(t/2))        (form 1, phase pi/2)
#   "pulse": omega(t) = 4 (1 + 0.25 t / cosh^2(2 (t - 2)))   (form 2)
# The paper states neither the initial state nor T nor N; this recipe takes
# the Sec. 4.1 state exp(-(x-1)^2/2), T = 5 and N = 1024.
# ---------------------------------------------------------------------------
TIMEDEP_OMEGA = {
    "cos": (4.0, 0.1, 0.5, math.pi / 2.0, 1),
    "pulse": (4.0, 0.25, 2.0, 2.0, 2),
}


def timedep_1d(form: str = "cos", n: int = 1024, T: float = 5.0, nsteps: int = 500,
               scheme: str = "srkn6_4", rule: str = "magnus6", eps_q: float = 0.01) -> Workload:
    inst = Instance(1, *_grid1(n, -20.0, 20.0),
                    omega=(TIMEDEP_OMEGA[form], CONST_OMEGA, CONST_OMEGA),
                    eps=eps_q, vfac=((0.0, 0.0, 0.25, 0.0, 0.0, 0.0), NO_V, NO_V))
    x = inst.axis(0)
    psi = _normalise(inst, np.exp(-(x - 1.0) ** 2 / 2.0).astype(np.complex128))
    return Workload("timedep_1d", [inst], [psi], scheme, rule, T / nsteps, nsteps,
                    notes="%s trap, N=%d on [-20,20), T=%g" % (form, n, T))


# ---------------------------------------------------------------------------
# Coupled traps (off-diagonal W, Sec. 1's general x^T M x): the 2-D and 3-D
# GPE recipes above with constant cross terms, W(t) positive definite
# (Gershgorin) over the whole modulation.
# ---------------------------------------------------------------------------
def coupled_2d(n: int = 512, n_inst: int = 16, lo: float = -12.0, hi: float = 12.0,
               dt: float = 5e-4, nsteps: int = 2000, seed: int = 34704, scheme: str = "leapfrog",
               rule: str = "cf4", wxy: float = 0.4, constant: bool = False) -> Workload:
    w = gpe_2d(n=n, n_inst=n_inst, lo=lo, hi=hi, dt=dt, nsteps=nsteps, seed=seed, scheme=scheme,
               rule=rule)
    insts = []
    for inst in w.instances:
        om = inst.omega
        if constant:
            om = ((om[0][0], 0.0, 0.0, 0.0), (om[1][0], 0.0, 0.0, 0.0), CONST_OMEGA)
        insts.append(replace(inst, omega=om, wcross=(wxy, 0.0, 0.0)))
    return replace(w, name="coupled_2d", instances=insts,
                   notes=w.notes + ", W_xy=%g%s" % (wxy, ", constant omega" if constant else ""))


def coupled_3d(n: int = 256, lo: float = -8.0, hi: float = 8.0, dt: float = 1e-3,
               nsteps: int = 500, seed: int = 34705, scheme: str = "ni5_84", rule: str = "cf4",
               wcross=(0.3, 0.2, -0.25)) -> Workload:
    w = gpe_3d(n=n, lo=lo, hi=hi, dt=dt, nsteps=nsteps, seed=seed, scheme=scheme, rule=rule)
    inst = replace(w.instances[0], wcross=tuple(wcross))
    return replace(w, name="coupled_3d", instances=[inst],
                   notes=w.notes + ", W_offdiag=%s" % (tuple(wcross),))


CONFIGS = {
    "coherent_1d": coherent_1d,
    "gpe_1d": gpe_1d,
    "batch_1d": batch_1d,
    "gpe_2d": gpe_2d,
    "gpe_3d": gpe_3d,
    "perturbed_1d": perturbed_1d,
    "timedep_1d": timedep_1d,
    "coupled_2d": coupled_2d,
    "coupled_3d": coupled_3d,
}


def subset(w: Workload, idx) -> Workload:
    """The same workload restricted to the given instance indices."""
    return replace(w, instances=[w.instances[i] for i in idx], psi0=[w.psi0[i] for i in idx])


def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """Relative L2 difference ||a - b|| / ||b|| (a metric, not method arithmetic)."""
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))
