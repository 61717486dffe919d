"""Fixed-shape axis passes (axes of 128 .. 1024 points): the same bits as the
runtime-shaped passes (nd_generic), and oracle parity, on shapes that reach
every fixed-shape instance: separable passes (padded-row and interleaved
layouts, 256- and 512-thread groups, drift-only and closing x-phase) and the
coupled-trap kinds (forward, forward + whole drift + inverse, inverse with and
without the closing x-phase)."""
from dataclasses import replace

import numpy as np
import pytest

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


def reshaped(shape, n_inst, nsteps, seed=0):
    """gpe_2d / gpe_3d recipe on another grid shape (box scaled with N)."""
    d = 3 if shape[2] > 1 else 2
    base = W.gpe_3d(n=8, nsteps=nsteps) if d == 3 else W.gpe_2d(n=8, n_inst=n_inst, nsteps=nsteps, seed=34702 + seed)
    insts = base.instances * (n_inst if d == 3 else 1)
    out, psis = [], []
    for k, inst in enumerate(insts[:n_inst]):
        half = tuple(max(4.0, n / 24.0) for n in shape)
        lo = tuple(-h if j < d else 0.0 for j, h in enumerate(half))
        hi = tuple(h + 0.3 * j if j < d else 1.0 for j, h in enumerate(half))
        i2 = replace(inst, n=shape, lo=lo, hi=hi)
        m = i2.mesh()
        r2 = sum((1.0 + 0.2 * j) * (x - 0.1 * (k + 1)) ** 2 for j, x in enumerate(m))
        out.append(i2)
        psis.append(W._normalise(i2, (np.exp(-r2 / 2) * (1 + 0.1j * m[0])).astype(complex)))
    return replace(base, instances=out, psi0=psis)


def coupled(shape, n_inst, nsteps, rule="cf4"):
    """The coupled-trap recipes (off-diagonal W) on another grid shape."""
    w = reshaped(shape, n_inst, nsteps)
    wc = (0.3, 0.2, -0.25) if shape[2] > 1 else (0.4, 0.0, 0.0)
    return replace(w, instances=[replace(i, wcross=wc) for i in w.instances], ho_rule=rule)


def run(pkg, w, dtype, **kw):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, **kw)
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, w.nsteps)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return plan.unpack(buf)


SHAPES = [
    ((128, 128, 1), 2),     # LOGN 7 both layouts
    ((256, 512, 1), 1),     # LOGN 8 rows, LOGN 9 interleaved (c64: 512-thread groups)
    ((1024, 128, 1), 1),    # LOGN 10 rows, LOGN 7 interleaved
    ((128, 1024, 1), 1),    # LOGN 10 interleaved (c64: 512-thread groups)
    ((128, 256, 128), 1),   # 3-D: interleaved drift-only pass (axis 1)
    ((256, 128, 256), 1),
    ((16, 16, 1024), 1),    # 3-D: longest axis outermost (stride 256 elements)
]


@pytest.mark.parametrize("shape,n_inst", SHAPES)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fixed_equals_generic_bitwise(pkg, shape, n_inst, dtype):
    w = reshaped(shape, n_inst, nsteps=3)
    say("fixed vs generic %s x%d %s" % (shape, n_inst, dtype))
    fixed = run(pkg, w, dtype)
    generic = run(pkg, w, dtype, nd_generic=True)
    for a, b in zip(fixed, generic):
        assert np.array_equal(a, b)


def test_fixed_graph_replay(pkg):
    w = reshaped((256, 256, 1), 2, nsteps=21)
    direct = run(pkg, w, "c64")
    graphed = run(pkg, w, "c64", use_graph=True)
    for a, b in zip(direct, graphed):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape,n_inst", [((128, 128, 1), 2), ((256, 128, 1), 1), ((128, 256, 16), 1),
                                           ((16, 16, 1024), 1), ((1024, 8, 16), 1)])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fixed_oracle_parity(pkg, shape, n_inst, dtype):
    w = reshaped(shape, n_inst, nsteps=4)
    got = run(pkg, w, dtype)
    for k, inst in enumerate(w.instances):
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        err = W.rel_l2(got[k], ref)
        say("fixed-shape %s k=%d %s rel_l2 %.3e" % (shape, k, dtype, err))
        assert err < (1e-11 if dtype == "c128" else 5e-5)


COUPLED_SHAPES = [
    ((128, 128, 1), 2),
    ((1024, 256, 1), 1),
    ((256, 128, 512), 1),
    ((128, 512, 128), 1),
    ((16, 16, 1024), 1),
]


@pytest.mark.parametrize("shape,n_inst", COUPLED_SHAPES)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_coupled_fixed_equals_generic_bitwise(pkg, shape, n_inst, dtype):
    w = coupled(shape, n_inst, nsteps=2)
    say("coupled fixed vs generic %s x%d %s" % (shape, n_inst, dtype))
    fixed = run(pkg, w, dtype)
    generic = run(pkg, w, dtype, nd_generic=True)
    for a, b in zip(fixed, generic):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("shape,rule", [((128, 128, 1), "cf4"), ((128, 256, 1), "fsplit"),
                                        ((128, 128, 16), "cf4")])
def test_coupled_fixed_oracle_parity(pkg, shape, rule):
    w = coupled(shape, 1, nsteps=3, rule=rule)
    for dtype in ("c128", "c64"):
        got = run(pkg, w, dtype)
        ref = oracle.evolve(w.instances[0], w.psi0[0], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        err = W.rel_l2(got[0], ref)
        say("coupled fixed-shape %s %s %s rel_l2 %.3e" % (shape, rule, dtype, err))
        assert err < (1e-11 if dtype == "c128" else 5e-5)
