"""Pins of the oracle's explicit perturbation input: eps V_I given at every
grid point instead of the separable factor form.

A linear potential F (x + y) is not a product of per-axis factors; with it
the trap is a shifted oscillator whose ground state is known in closed form,
so the split evolution must converge to a pure phase rotation of it."""
import math

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
