"""d-D parity over long horizons (the 2-D recipe's full 2000 steps at 64^2,
1000 steps of the coupled trap, 200 NI5 steps in 3-D) and time reversal of
the symmetric d-D compositions, through the C ABI."""
from dataclasses import replace

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-11, "c64": 5e-5}


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_1007_3470_amd as p
    p.load()
    return p


def run(pkg, w, dtype, dt=None, t0=None, psi=None, **kw):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt if dt is None else dt, **kw)
    buf = plan.pack(w.psi0 if psi is None else psi)
    plan.evolve(buf, w.t0 if t0 is None else t0, w.nsteps)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return plan.unpack(buf)


def check(w, got, tol, label):
    for k, inst in enumerate(w.instances):
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        err = W.rel_l2(got[k], ref)
        print("%s k=%d: %d steps, rel_l2 %.3e" % (label, k, w.nsteps, err), flush=True)
        assert err < tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_2d_full_length_small_grid(pkg, dtype):
    w = W.gpe_2d(n=64, n_inst=2)   # the recipe's 2000 steps of leapfrog + CF4
    check(w, run(pkg, w, dtype, use_graph=True), TOL[dtype], "gpe_2d 64^2 %s" % dtype)


def test_coupled_2d_long(pkg):
    w = W.coupled_2d(n=64, n_inst=2, nsteps=1000)
    check(w, run(pkg, w, "c128", use_graph=True), 1e-11, "coupled_2d 64^2 c128")


def test_3d_ni5_long(pkg):
    w = W.gpe_3d(n=32, nsteps=200)
    check(w, run(pkg, w, "c128", use_graph=True), 1e-11, "gpe_3d 32^3 c128")


@pytest.mark.parametrize("make", [lambda: W.gpe_2d(n=64, n_inst=2, nsteps=400),
                                  lambda: W.coupled_2d(n=64, n_inst=2, nsteps=300),
                                  lambda: W.gpe_3d(n=32, nsteps=40)])
def test_nd_time_reversal(pkg, make):
    """Symmetric compositions with the symmetric HO rules: n steps of dt from
    t0, then n steps of -dt from t0 + n dt, return the initial state."""
    w = make()
    fwd = run(pkg, w, "c128", use_graph=True)
    back = run(pkg, w, "c128", dt=-w.dt, t0=w.t0 + w.nsteps * w.dt, psi=fwd, use_graph=True)
    for k in range(len(w.instances)):
        err = W.rel_l2(back[k], w.psi0[k])
        moved = W.rel_l2(fwd[k], w.psi0[k])
        print("%s k=%d: forward moved %.2e, back to start %.2e" % (w.name, k, moved, err), flush=True)
        assert moved > 1e-3 and err < 1e-11
