"""GPU parity of the 2-D / 3-D axis-pass HIP path against the CPU oracle."""
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


def run_gpu(pkg, w, dtype, nsteps=None, **kw):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, **kw)
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, w.nsteps if nsteps is None else nsteps)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return plan, buf, plan.unpack(buf)


def say(*a):
    print(*a, flush=True)


def reshape_workload(w, n, lo, hi):
    """Same physics on another grid shape; fresh Gaussian initial data."""
    insts, psis = [], []
    for k, inst in enumerate(w.instances):
        i2 = replace(inst, n=n, lo=lo, hi=hi)
        mesh = i2.mesh()
        r2 = sum((1.0 + 0.2 * j) * (m - 0.1 * k) ** 2 for j, m in enumerate(mesh))
        insts.append(i2)
        psis.append(W._normalise(i2, np.exp(-r2 / 2).astype(complex)))
    return replace(w, instances=insts, psi0=psis)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_2d_small_batch(pkg, dtype):
    w = W.gpe_2d(n=64, n_inst=3, nsteps=30)
    _, _, got = run_gpu(pkg, w, dtype)
    for k, inst in enumerate(w.instances):
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        err = W.rel_l2(got[k], ref)
        say("2d %s k=%d rel_l2 %.3e" % (dtype, k, err))
        assert err < TOL[dtype]


@pytest.mark.parametrize("shape", [(128, 32, 1), (8, 256, 1), (2, 8, 1), (64, 2, 1), (64, 1, 1), (1, 64, 1)])
def test_2d_anisotropic_shapes(pkg, shape):
    w = reshape_workload(W.gpe_2d(n=8, n_inst=2, nsteps=12), shape, (-6.0, -5.0, 0.0), (7.0, 5.0, 1.0))
    _, _, got = run_gpu(pkg, w, "c128")
    for k, inst in enumerate(w.instances):
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        err = W.rel_l2(got[k], ref)
        say("2d shape %s k=%d rel_l2 %.3e" % (shape, k, err))
        assert err < 1e-11


@pytest.mark.parametrize("scheme,rule", [("ni5_84", "cf4"), ("srkn6_4", "magnus6"), ("leapfrog", "cf4")])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_3d_small(pkg, scheme, rule, dtype):
    w = W.gpe_3d(n=32, nsteps=6, scheme=scheme, rule=rule)
    _, _, got = run_gpu(pkg, w, dtype)
    ref = oracle.evolve(w.instances[0], w.psi0[0], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
    err = W.rel_l2(got[0], ref)
    say("3d %s %s %s rel_l2 %.3e" % (scheme, rule, dtype, err))
    assert err < TOL[dtype]


@pytest.mark.parametrize("shape", [(16, 64, 8), (4, 2, 32), (64, 16, 128), (16, 1, 8), (1, 1, 32)])
def test_3d_anisotropic_shapes(pkg, shape):
    base = W.gpe_3d(n=8, nsteps=5)
    w = reshape_workload(replace(base, instances=base.instances * 2, psi0=base.psi0 * 2), shape,
                         (-5.0, -6.0, -4.0), (5.0, 6.0, 4.5))
    _, _, got = run_gpu(pkg, w, "c128")
    for k, inst in enumerate(w.instances):
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        err = W.rel_l2(got[k], ref)
        say("3d shape %s k=%d rel_l2 %.3e" % (shape, k, err))
        assert err < 1e-11


def test_nd_batch_vs_alone_bitwise(pkg):
    w = W.gpe_2d(n=64, n_inst=4, nsteps=10)
    _, _, a = run_gpu(pkg, w, "c128")
    _, _, b = run_gpu(pkg, W.subset(w, [2]), "c128")
    assert np.array_equal(a[2], b[0])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_nd_norm_energy(pkg, dtype):
    for w in (W.gpe_2d(n=64, n_inst=2, nsteps=8), W.gpe_3d(n=32, nsteps=3)):
        plan, buf, got = run_gpu(pkg, w, dtype)
        t = w.t0 + w.nsteps * w.dt
        nrm, en = plan.norm(buf), plan.energy(buf, t)
        for k, inst in enumerate(w.instances):
            assert abs(nrm[k] - oracle.norm(inst, got[k])) < 1e-12 * max(1, abs(nrm[k]))
            ref = oracle.energy(inst, got[k], t)
            assert np.allclose(en[k], ref, rtol=1e-11, atol=1e-11), (en[k], ref)


# ---------------------------------------------------------------------------
# full sizes, in the launch configuration of the solver
# ---------------------------------------------------------------------------
def test_2d_full_size(pkg):
    w = W.gpe_2d()   # 16 x 512^2, 2000 steps
    # sampled parity: the full batch for 60 steps, instance 5 against the oracle
    _, _, short = run_gpu(pkg, w, "c128", nsteps=60)
    ref = oracle.evolve(w.instances[5], w.psi0[5], w.scheme, w.ho_rule, w.dt, w.t0, 60)
    err = W.rel_l2(short[5], ref)
    say("2d full size, 60 steps, instance 5 vs oracle: %.3e" % err)
    assert err < 1e-11
    # the full run: norm conservation and c64 against c128
    p128, b128, full128 = run_gpu(pkg, w, "c128")
    p64, b64, full64 = run_gpu(pkg, w, "c64")
    n0 = np.array([oracle.norm(i, p) for i, p in zip(w.instances, w.psi0)])
    drift = np.abs(p128.norm(b128) - n0).max()
    e64 = max(W.rel_l2(a, b) for a, b in zip(full64, full128))
    say("2d full size 2000 steps: c128 norm drift %.3e, c64 vs c128 max %.3e" % (drift, e64))
    assert drift < 1e-11 and e64 < 5e-5


def test_3d_full_size(pkg):
    w = W.gpe_3d()   # 256^3, NI5 + CF4, 500 steps
    _, _, one = run_gpu(pkg, w, "c128", nsteps=1)
    ref = oracle.evolve(w.instances[0], w.psi0[0], w.scheme, w.ho_rule, w.dt, w.t0, 1)
    err = W.rel_l2(one[0], ref)
    say("3d full size, 1 step vs oracle: %.3e" % err)
    assert err < 1e-11
    p128, b128, full128 = run_gpu(pkg, w, "c128")
    p64, b64, full64 = run_gpu(pkg, w, "c64")
    drift = abs(p128.norm(b128)[0] - oracle.norm(w.instances[0], w.psi0[0]))
    e64 = W.rel_l2(full64[0], full128[0])
    say("3d full size 500 steps: c128 norm drift %.3e, c64 vs c128 %.3e" % (drift, e64))
    assert drift < 1e-11 and e64 < 5e-5


# ---------------------------------------------------------------------------
# graph replay and autotuning give the same results as direct launches
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_graph_replay_matches_direct(pkg, dtype):
    import torch
    w = W.gpe_2d(n=64, n_inst=3, nsteps=53)
    _, _, direct = run_gpu(pkg, w, dtype)
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, use_graph=True)
    buf = plan.pack(w.psi0)
    for rep in range(3):   # replays of the cached graph, eager work in between
        buf.copy_(plan.pack(w.psi0))
        plan.evolve(buf, w.t0, w.nsteps)
        torch.cuda.synchronize()
        assert plan.norm(buf).shape == (3,)
        got = plan.unpack(buf)
        for k in range(3):
            assert np.array_equal(got[k], direct[k]), (rep, k)
    # a split call crosses graph blocks differently and stores the state in the
    # storage precision between the calls: results agree to that rounding
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, 20)
    plan.evolve(buf, w.t0 + 20 * w.dt, 33)
    torch.cuda.synchronize()
    split = plan.unpack(buf)
    for k in range(3):
        assert W.rel_l2(split[k], direct[k]) < (1e-12 if dtype == "c128" else 1e-6)


def test_graph_3d_ni5_matches_oracle(pkg):
    w = W.gpe_3d(n=32, nsteps=20)
    _, _, got = run_gpu(pkg, w, "c128", use_graph=True)
    ref = oracle.evolve(w.instances[0], w.psi0[0], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
    assert W.rel_l2(got[0], ref) < 1e-11


@pytest.mark.parametrize("make", [lambda: W.gpe_2d(n=512, n_inst=2, nsteps=12),
                                  lambda: W.gpe_3d(n=128, nsteps=3),
                                  lambda: W.coupled_2d(n=256, n_inst=2, nsteps=4)],
                         ids=["2d_512", "3d_128", "coupled_2d_256"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_autotune_keeps_results(pkg, make, dtype):
    """The per-pass tuner (workgroups per CU, 256/512-thread groups) changes
    how pencils are shared out, not their arithmetic: bitwise the default
    results, direct and replayed from a graph captured after tuning."""
    import torch
    w = make()
    _, _, ref = run_gpu(pkg, w, dtype)
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, use_graph=True)
    n = plan.autotune(w.psi0, trial_steps=3)
    tuned = plan.tune_settings()
    say("autotune %s: %d pass positions -> %s" % (dtype, n, tuned))
    assert n == len(tuned) > 0 and all(0 <= pc <= 4 and tpb in (0, 256, 512) for pc, tpb in tuned)
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, w.nsteps)
    torch.cuda.synchronize()
    got = plan.unpack(buf)
    for k in range(len(w.instances)):
        assert np.array_equal(got[k], ref[k])
    # a new plan of the same shape starts from the process-wide cache
    again = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt)
    assert again.tune_settings() == tuned


@pytest.mark.parametrize("make", [lambda: W.gpe_3d(n=128, nsteps=3),
                                  lambda: W.gpe_2d(n=512, n_inst=2, nsteps=3),
                                  lambda: W.coupled_2d(n=256, n_inst=2, nsteps=2)],
                         ids=["3d_128", "2d_512", "coupled_2d_256"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_persistent_grid_does_not_change_results(pkg, make, dtype):
    """The default grid (sized per pass from the kernel's occupancy), 512 and
    15 workgroups give the same bits.  On the 512-point axes (and c64 on
    256-point ones) the strided rows are shorter than a 128-byte line, so grids
    that are multiples of 16 pair workgroups on one XCD and 15 does not (each
    of its workgroups also takes many groups); the 128-point axes never pair."""
    import torch
    w = make()
    outs = []
    for wg in (0, 512, 15):
        plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, nd_workgroups=wg)
        buf = plan.pack(w.psi0)
        plan.evolve(buf, w.t0, w.nsteps)
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        outs.append(plan.unpack(buf))
    for k in range(len(w.instances)):
        assert np.array_equal(outs[0][k], outs[1][k]) and np.array_equal(outs[0][k], outs[2][k])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fourier_split_nd(pkg, dtype):
    for w in (W.gpe_2d(n=64, n_inst=2, nsteps=15, rule="fsplit"),
              W.gpe_3d(n=32, nsteps=4, rule="fsplit")):
        _, _, got = run_gpu(pkg, w, dtype)
        for k, inst in enumerate(w.instances):
            ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
            err = W.rel_l2(got[k], ref)
            say("fsplit %dD %s k=%d rel_l2 %.3e" % (inst.ndim, dtype, k, err))
            assert err < TOL[dtype]


@pytest.mark.parametrize("rule", ["fundamental", "magnus6"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_nd_time_forms(pkg, rule, dtype):
    """2-D and 3-D grids with the Sec. 4.2 trap forms on different axes."""
    w2 = W.gpe_2d(n=64, n_inst=2, nsteps=12, rule=rule, dt=2e-3)
    insts = [replace(i, omega=(W.TIMEDEP_OMEGA["pulse"], W.TIMEDEP_OMEGA["cos"], W.CONST_OMEGA),
                     sigma=(5.0, 0.5, 3.0, 0.0, 2)) for i in w2.instances]
    w2 = replace(w2, instances=insts, t0=1.95)
    w3 = W.gpe_3d(n=32, nsteps=3, rule=rule)
    i3 = replace(w3.instances[0], omega=(W.TIMEDEP_OMEGA["cos"], (1.2, 0.2, 1.3, 0.0),
                                         W.TIMEDEP_OMEGA["pulse"]))
    w3 = replace(w3, instances=[i3], t0=1.99)
    for w in (w2, w3):
        _, _, got = run_gpu(pkg, w, dtype)
        for k, inst in enumerate(w.instances):
            ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
            err = W.rel_l2(got[k], ref)
            say("nd forms %dD %s %s k=%d rel_l2 %.3e" % (inst.ndim, rule, dtype, k, err))
            assert err < TOL[dtype]


def test_plain_schedule_launches_every_pass(pkg):
    """plain = 1 is the reference schedule: with use_graph also set, a d-D plan
    still launches every pass itself (each one bracketed by profiling events,
    which captured graphs do not carry) and gives the graph schedule's bits."""
    import torch
    w = W.gpe_2d(n=64, n_inst=2, nsteps=40)
    outs, launches = [], []
    for plain in (False, True):
        plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, "c128", w.dt, use_graph=True,
                        plain=plain, profile=True)
        buf = plan.pack(w.psi0)
        plan.evolve(buf, w.t0, w.nsteps)
        torch.cuda.synchronize()
        launches.append(plan.profile()[2])
        outs.append(plan.unpack(buf))
    passes = 2 * w.nsteps  # leapfrog, two axes
    assert launches[1] == passes
    assert launches[0] < passes  # the graph blocks are not bracketed
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("make,mu,rules", [
    (lambda: W.gpe_2d(n=64, n_inst=2, nsteps=10), 1.7, ("cf4", "magnus6", "fsplit")),
    (lambda: W.gpe_3d(n=32, nsteps=4), 0.6, ("cf4", "magnus6", "fsplit")),
    (lambda: W.coupled_2d(n=64, n_inst=2, nsteps=10), 1.4, ("cf4", "fsplit")),
], ids=["2d", "3d", "coupled_2d"])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_general_mass_nd(pkg, make, mu, rules, dtype):
    """mu != 1 in 2-D, 3-D and coupled grids (the canonical scaling of the HO
    factors and the drift 1/mu), every rule against the oracle, and the energy."""
    import torch
    base = make()
    insts = [replace(i, mu=mu) for i in base.instances]
    for rule in rules:
        w = replace(base, instances=insts, ho_rule=rule)
        plan, buf, got = run_gpu(pkg, w, dtype)
        for k, inst in enumerate(insts):
            ref = oracle.evolve(inst, w.psi0[k], w.scheme, rule, w.dt, w.t0, w.nsteps)
            err = W.rel_l2(got[k], ref)
            say("mu=%g %s %s k=%d rel_l2 %.2e" % (mu, rule, dtype, k, err))
            assert err < TOL[dtype]
    if dtype == "c128":
        T = w.t0 + w.dt * w.nsteps
        e = plan.energy(buf, T)
        for k, inst in enumerate(insts):
            eo = oracle.energy(inst, got[k], T)
            assert np.allclose(e[k], eo, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_instances_with_different_boxes(pkg, dtype):
    """Instances of one d-D plan share the grid shape, not the box: per
    instance coordinates, wavenumber scales and drift factors (recomputed
    whenever a workgroup's range crosses into another instance)."""
    base = W.gpe_2d(n=128, n_inst=3, nsteps=12)
    boxes = (((-12.0, -12.0), (12.0, 12.0)), ((-8.0, -6.0), (10.0, 9.0)), ((-15.0, -3.0), (5.0, 13.0)))
    insts, psis = [], []
    for k, (inst, (lo, hi)) in enumerate(zip(base.instances, boxes)):
        i2 = replace(inst, lo=(lo[0], lo[1], 0.0), hi=(hi[0], hi[1], 1.0))
        x, y = i2.mesh()
        cx, cy = 0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1])
        psis.append(W._normalise(i2, np.exp(-((x - 0.3 * cx) ** 2 + 1.5 * (y - 0.3 * cy) ** 2) / 2).astype(complex)))
        insts.append(i2)
    w = replace(base, instances=insts, psi0=psis)
    _, _, got = run_gpu(pkg, w, dtype, use_graph=True)
    for k, inst in enumerate(insts):
        ref = oracle.evolve(inst, psis[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        err = W.rel_l2(got[k], ref)
        say("box %s %s rel_l2 %.2e" % (boxes[k], dtype, err))
        assert err < TOL[dtype]
