"""Oracle parity at the benchmark recipes' full sizes and run lengths, in the
launch configuration bench.py times (resident 1-D batch; d-D passes replayed
from hipGraph blocks), plus d-D runs that cross coefficient chunks.

The oracle is the threaded C oracle (bitwise the single-thread result, see
test_oracle_threads.py) on this host's cores.  Tolerances (relative L2 per
instance, after the whole run): 1e-11 for the FP64 (c128) path, 5e-5 for c64.
"""
import concurrent.futures
import os
import time

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-11, "c64": 5e-5}


def host_threads(cap=16):
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_1007_3470_amd as p
    p.load()
    return p


def gpu_run(pkg, w, dtype, nsteps=None, **kw):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, **kw)
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, w.nsteps if nsteps is None else nsteps)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    out = plan.unpack(buf)
    del buf, plan
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# the 4096-instance 1-D batch, 5000 steps
# ---------------------------------------------------------------------------
def test_batch_1d_full_run_sampled(pkg):
    w = W.batch_1d()
    say("batch_1d: %d instances, %d steps" % (len(w.instances), w.nsteps))
    got = {d: gpu_run(pkg, w, d) for d in ("c128", "c64")}
    c64_err = np.array([W.rel_l2(a, b) for a, b in zip(got["c64"], got["c128"])])
    sig = np.array([inst.sigma[0] for inst in w.instances])
    pick = []
    for n in (256, 512, 1024, 2048):
        pick += [k for k, inst in enumerate(w.instances) if inst.n[0] == n][:16]
    pick += list(np.argsort(-sig)[:8])          # strongest nonlinearity
    pick += list(np.argsort(-c64_err)[:8])      # furthest c64 from c128
    pick = sorted(set(int(k) for k in pick), key=lambda k: -w.instances[k].n[0])
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=host_threads()) as ex:
        futs = {k: ex.submit(oracle.evolve, w.instances[k], w.psi0[k], w.scheme, w.ho_rule, w.dt, 0.0,
                             w.nsteps) for k in pick}
        refs = {k: f.result() for k, f in futs.items()}
    say("batch_1d: oracle on %d instances in %.1f s" % (len(pick), time.perf_counter() - t0))
    worst = {}
    for dtype in ("c128", "c64"):
        errs = {k: W.rel_l2(got[dtype][k], refs[k]) for k in pick}
        k = max(errs, key=errs.get)
        worst[dtype] = (errs[k], k)
        say("batch_1d %s vs oracle: max %.3e (instance %d, N=%d, sigma=%.1f), median %.3e"
            % (dtype, errs[k], k, w.instances[k].n[0], w.instances[k].sigma[0], np.median(list(errs.values()))))
        assert errs[k] < TOL[dtype], (dtype, k, errs[k])


# ---------------------------------------------------------------------------
# 16 x 512^2, 2000 steps: oracle on two instances
# ---------------------------------------------------------------------------
def test_gpe_2d_full_run_two_instances(pkg):
    w = W.gpe_2d()
    say("gpe_2d: %d x 512^2, %d steps" % (len(w.instances), w.nsteps))
    got = {d: gpu_run(pkg, w, d, use_graph=True) for d in ("c128", "c64")}
    # the instance with the strongest and the one with the weakest coupling
    sig = [inst.sigma[0] for inst in w.instances]
    pick = [int(np.argmax(sig)), int(np.argmin(sig))]
    th = max(1, host_threads() // 2)
    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=2) as ex:
        futs = {k: ex.submit(oracle.evolve, w.instances[k], w.psi0[k], w.scheme, w.ho_rule, w.dt, 0.0,
                             w.nsteps, None, th) for k in pick}
        refs = {k: f.result() for k, f in futs.items()}
    say("gpe_2d: oracle on 2 instances x %d threads in %.1f s" % (th, time.perf_counter() - t0))
    for dtype in ("c128", "c64"):
        for k in pick:
            err = W.rel_l2(got[dtype][k], refs[k])
            say("gpe_2d %s instance %d (sigma %.1f) vs oracle: %.3e" % (dtype, k, sig[k], err))
            assert err < TOL[dtype], (dtype, k, err)


# ---------------------------------------------------------------------------
# 256^3, NI5(8,4) + CF4: 20 steps (15 axis passes each)
# ---------------------------------------------------------------------------
def test_gpe_3d_full_size_20_steps(pkg):
    w = W.gpe_3d(nsteps=20)
    got = {d: gpu_run(pkg, w, d, use_graph=True)[0] for d in ("c128", "c64")}
    t0 = time.perf_counter()
    ref = oracle.evolve(w.instances[0], w.psi0[0], w.scheme, w.ho_rule, w.dt, 0.0, w.nsteps,
                        threads=host_threads())
    say("gpe_3d: oracle 20 steps on %d threads in %.1f s" % (host_threads(), time.perf_counter() - t0))
    for dtype in ("c128", "c64"):
        err = W.rel_l2(got[dtype], ref)
        say("gpe_3d %s vs oracle after 20 steps: %.3e" % (dtype, err))
        assert err < TOL[dtype], (dtype, err)


# ---------------------------------------------------------------------------
# d-D runs that cross coefficient chunks (chunk_steps caps a chunk): the
# merged phase carries over the boundary, later chunks skip the opening
# phase, the graph is recaptured for a chunk of another length and a tail
# shorter than a graph block runs as direct launches.  Bitwise equal to the
# single-chunk run in FP64 and within tolerance of the oracle.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,make,nsteps,chunk", [
    ("gpe_2d", lambda: W.gpe_2d(n=128, n_inst=3, nsteps=0), 90, 40),     # 40, 40, 10
    ("gpe_2d", lambda: W.gpe_2d(n=128, n_inst=3, nsteps=0), 100, 40),    # 40, 40, 20
    ("coupled_2d", lambda: W.coupled_2d(n=128, n_inst=2, nsteps=0), 70, 32),   # 32, 32, 6
    ("gpe_3d", lambda: W.gpe_3d(n=32, nsteps=0), 37, 17),                # 17, 17, 3
])
def test_nd_chunked_run(pkg, name, make, nsteps, chunk):
    w = make()
    one = gpu_run(pkg, w, "c128", nsteps=nsteps, use_graph=True)
    many = gpu_run(pkg, w, "c128", nsteps=nsteps, use_graph=True, chunk_steps=chunk)
    for a, b in zip(one, many):
        assert np.array_equal(a.view(np.float64), b.view(np.float64))
    many64 = gpu_run(pkg, w, "c64", nsteps=nsteps, use_graph=True, chunk_steps=chunk)
    for k, inst in enumerate(w.instances):
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, 0.0, nsteps, threads=host_threads())
        e128, e64 = W.rel_l2(many[k], ref), W.rel_l2(many64[k], ref)
        say("%s chunked (%d / %d) instance %d: c128 %.3e, c64 %.3e" % (name, nsteps, chunk, k, e128, e64))
        assert e128 < TOL["c128"] and e64 < TOL["c64"], (k, e128, e64)
