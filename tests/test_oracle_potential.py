"""Pins of the oracle's perturbation eps V_I (Sec. 1).

The explicit input (eps V_I given at every grid point): a linear potential
F (x + y) is not a product of per-axis factors; with it the trap is a shifted
oscillator whose ground state is known in closed form, so the split evolution
must converge to a pure phase rotation of it.

The separable factor form: its potential energy and its B flow against NumPy
evaluations of the formula, with the Gaussian width and the polynomial
coefficients varied."""
import math
from dataclasses import replace

import numpy as np
import pytest

import oracle
import workloads as W


def test_array_equal_to_factor_form():
    w = W.gpe_2d(n=32, n_inst=1, nsteps=6)
    inst = w.instances[0]
    x, y = inst.mesh()
    # the recipe's factor form, written out: 0.01 sin x sin y
    vi = 0.01 * np.sin(x) * np.sin(y) * np.ones(inst.shape)
    a = oracle.evolve(inst, w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, w.nsteps)
    b = oracle.evolve(inst, w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, w.nsteps, vi=vi)
    assert W.rel_l2(b, a) < 1e-13
    ea = oracle.energy(inst, a, 0.1)
    eb = oracle.energy(inst, a, 0.1, vi=vi)
    assert np.allclose(ea, eb, rtol=1e-13, atol=1e-15)


def shifted_ground_state(inst, F):
    wx, wy = inst.omega[0][0], inst.omega[1][0]
    x, y = inst.mesh()
    g = np.exp(-wx * (x + F / wx ** 2) ** 2 / 2 - wy * (y + F / wy ** 2) ** 2 / 2)
    E = 0.5 * (wx + wy) - F ** 2 / (2 * wx ** 2) - F ** 2 / (2 * wy ** 2)
    return W._normalise(inst, g.astype(complex)), E


def test_linear_potential_ground_state_order_two():
    inst = W.Instance(2, (64, 64, 1), (-8.0, -8.0, 0.0), (8.0, 8.0, 1.0),
                      omega=((1.0, 0.0, 0.0, 0.0), (1.4, 0.0, 0.0, 0.0), W.CONST_OMEGA), eps=1.0)
    F = 0.3
    x, y = inst.mesh()
    vi = F * (x + y) * np.ones(inst.shape)
    g, E = shifted_ground_state(inst, F)
    T = 2.0
    exact = np.exp(-1j * E * T) * g
    errs = []
    for n in (10, 20, 40):
        u = oracle.evolve(inst, g, "leapfrog", "exact_const", T / n, 0.0, n, vi=vi)
        errs.append(W.rel_l2(u, exact))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, (errs, rates)
    # and the potential energy of the shifted state: <V_HO + F(x+y)>
    e = oracle.energy(inst, g, 0.0, vi=vi)
    ref = 0.25 * (1.0 + 1.4) + 0.5 * (F ** 2 / 1.0 ** 2 + F ** 2 / 1.4 ** 2) \
        - F ** 2 / 1.0 ** 2 - F ** 2 / 1.4 ** 2
    assert abs(e[2] - ref) < 1e-12


# ---------------------------------------------------------------------------
# The separable factor form of V_I, pinned against NumPy evaluations of the
# formula (c0 + c2 x^2 + c4 x^4) exp(-x^2/gs) cos(k x + phi) written out here:
# the 1-D GPE recipe's 0.01 x^4 exp(-x^2/16) (Sec. 1's eps V_I) and variants
# with the Gaussian width, the quartic and the other coefficients changed.
# ---------------------------------------------------------------------------
VFACTOR_CASES = [
    # (c0, c2, c4, gs, k, phi), eps
    ((0.0, 0.0, 1.0, 16.0, 0.0, 0.0), 0.01),   # the 1-D GPE recipe
    ((0.0, 0.0, 1.0, 4.0, 0.0, 0.0), 0.01),    # narrower Gaussian
    ((0.0, 0.0, 2.5, 16.0, 0.0, 0.0), 0.03),   # larger quartic
    ((0.7, -0.3, 0.05, 9.0, 1.3, 0.4), 0.2),   # every term
    ((0.0, 0.0, 0.25, 0.0, 0.0, 0.0), 0.01),   # gs = 0: no Gaussian (Sec. 4.2's x^4/4)
]


def numpy_vfactor(v, x):
    c0, c2, c4, gs, k, phi = v
    gauss = np.exp(-x ** 2 / gs) if gs > 0 else 1.0
    return (c0 + c2 * x ** 2 + c4 * x ** 4) * gauss * np.cos(k * x + phi)


@pytest.mark.parametrize("vf,eps", VFACTOR_CASES)
def test_vfactor_potential_energy(vf, eps):
    """The potential energy h sum (mu omega^2 x^2/2 + eps V_I) |u|^2 with V_I
    from the factor form equals its NumPy evaluation."""
    inst = W.Instance(1, (256, 1, 1), (-16.0, 0.0, 0.0), (16.0, 1.0, 1.0), mu=1.3,
                      omega=((0.8, 0.0, 0.0, 0.0), W.CONST_OMEGA, W.CONST_OMEGA), eps=eps,
                      vfac=(vf, W.NO_V, W.NO_V))
    x = inst.axis(0)
    psi = W._normalise(inst, (np.exp(-(x - 1.5) ** 2 / 8.0) * (1 + 0.3j * x)).astype(complex))
    e = oracle.energy(inst, psi, 0.0)
    rho = np.abs(psi) ** 2
    ref = inst.cell * np.sum((0.5 * 1.3 * 0.8 ** 2 * x ** 2 + eps * numpy_vfactor(vf, x)) * rho)
    assert abs(e[2] - ref) < 1e-13 * max(1.0, abs(ref)), (e[2], ref)


def test_vfactor_potential_energy_2d_product():
    """d-D: V_I is the product of the per-axis factors."""
    va, vb = VFACTOR_CASES[3][0], VFACTOR_CASES[1][0]
    inst = W.Instance(2, (64, 32, 1), (-6.0, -5.0, 0.0), (6.0, 5.0, 1.0),
                      omega=((1.1, 0.0, 0.0, 0.0), (0.9, 0.0, 0.0, 0.0), W.CONST_OMEGA),
                      eps=0.4, vfac=(va, vb, W.NO_V))
    x, y = inst.mesh()
    psi = W._normalise(inst, np.exp(-(x ** 2 + 2 * (y - 0.5) ** 2) / 3.0).astype(complex))
    e = oracle.energy(inst, psi, 0.0)
    V = 0.5 * (1.1 ** 2 * x ** 2 + 0.9 ** 2 * y ** 2) + 0.4 * numpy_vfactor(va, x) * numpy_vfactor(vb, y)
    ref = inst.cell * np.sum(V * np.abs(psi) ** 2)
    assert abs(e[2] - ref) < 1e-13 * abs(ref)


@pytest.mark.parametrize("vf,eps", VFACTOR_CASES)
def test_vfactor_evolution_matches_numpy_array(vf, eps):
    """The B flow with the factor form equals the B flow with eps V_I given
    as an array evaluated by NumPy (the array path is pinned above by the
    linear potential's closed form), over the 1-D GPE recipe at N = 256.  The
    reading exp(-gs x^2) of the Gaussian would differ by orders of magnitude
    more than the tolerance (checked for the cases that have one)."""
    w = W.gpe_1d(n=256, nsteps=50)
    inst = replace(w.instances[0], eps=eps, vfac=(vf, W.NO_V, W.NO_V))
    x = inst.axis(0)
    vi = eps * numpy_vfactor(vf, x)
    a = oracle.evolve(inst, w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, w.nsteps)
    b = oracle.evolve(inst, w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, w.nsteps, vi=vi)
    assert W.rel_l2(a, b) < 1e-13
    if vf[3] > 0:
        c0, c2, c4, gs, k, phi = vf
        wrong = eps * (c0 + c2 * x ** 2 + c4 * x ** 4) * np.exp(-gs * x ** 2) * np.cos(k * x + phi)
        c = oracle.evolve(inst, w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, w.nsteps, vi=wrong)
        assert W.rel_l2(a, c) > 1e3 * 1e-13
