"""The two sources of the 1-D stage records agree: records evaluated inside
the resident step kernel (in_kernel_records=True, for plans whose grid sizes
all lie in 64..2048) and the record table written by the coefficient kernel
(the default).  Both run the same per-step arithmetic (the merged
records of Table "algorithm" / Eq. prod-genHarmOsc), so FP64 results must be
bitwise equal, over every HO rule, schemes with 1 to 6 stages, block sizes
from two steps per block (32 instances of N = 64 with a 6-stage scheme) to
512, launches split by steps_per_launch, a start time t0 != 0, modulated
sigma and eps V_I, and both storage types.  The oracle parity of the table
path is covered by the other 1-D tests."""
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


def mixed_batch(rule, scheme, seed=5):
    """40 instances of N = 64 (two workgroups, one full with 32 instances),
    then 128 .. 2048, with time-dependent omega (sine or pulse), sigma
    modulated and a time factor on eps V_I."""
    rng = np.random.default_rng(seed)
    sizes = [64] * 40 + [128] * 9 + [256] * 5 + [512] * 3 + [1024] * 2 + [2048] * 2
    insts, psis = [], []
    for k, n in enumerate(sizes):
        L = max(4.0, n / 64.0)
        if rule == "exact_const":
            om = (float(rng.uniform(0.6, 1.8)), 0.0, 0.0, 0.0)
        elif k % 2:
            om = (float(rng.uniform(0.6, 1.8)), float(rng.uniform(0.0, 0.4)), float(rng.uniform(0.5, 2.5)),
                  float(rng.uniform(0, 1)))
        else:
            om = (float(rng.uniform(0.8, 1.5)), 0.3, 1.5, 0.4, 2)
        inst = W.Instance(1, (n, 1, 1), (-L, 0.0, 0.0), (L, 1.0, 1.0),
                          omega=(om, W.CONST_OMEGA, W.CONST_OMEGA),
                          sigma=(float(rng.uniform(0.0, 20.0)), 0.3, 1.1, 0.2), eps=0.05,
                          vfac=((1.0, 0.0, 0.0, 0.0, 2.0, 0.0), W.NO_V, W.NO_V),
                          vmod=(0.4, 1.7, 0.2, 0) if k % 3 else (0.5, 2.0, 0.3, 2))
        x = inst.axis(0)
        x0 = float(rng.uniform(-0.5, 0.5))
        psis.append(W._normalise(inst, np.exp(-(x - x0) ** 2 / 2.0 + 0.3j * x).astype(complex)))
        insts.append(inst)
    return W.Workload("mixed", insts, psis, scheme, rule, 2e-3, 37, t0=0.41)


def run(pkg, w, dtype, in_kernel, **kw):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, in_kernel_records=in_kernel, **kw)
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, w.nsteps)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return plan.unpack(buf)


@pytest.mark.parametrize("rule", ["exact_const", "cf4", "magnus6", "fsplit", "fundamental:4"])
@pytest.mark.parametrize("scheme", ["leapfrog", "ni5_84", "srkn6_4"])
def test_in_kernel_records_match_record_table_fp64(pkg, rule, scheme):
    w = mixed_batch(rule, scheme)
    a = run(pkg, w, "c128", True)
    b = run(pkg, w, "c128", False)
    worst = max(float(np.max(np.abs(x - y))) for x, y in zip(a, b))
    say("%s %s: max |in-kernel - table| %.3e" % (scheme, rule, worst))
    assert worst == 0.0


@pytest.mark.parametrize("spl", [0, 1, 10])
def test_in_kernel_records_split_launches(pkg, spl):
    """Launches of 1 and 10 steps (the records of a later launch start at its
    own global step) give the bits of one launch and of the table."""
    w = mixed_batch("cf4", "ni5_84", seed=9)
    a = run(pkg, w, "c128", True, steps_per_launch=spl)
    b = run(pkg, w, "c128", False)
    worst = max(float(np.max(np.abs(x - y))) for x, y in zip(a, b))
    say("steps_per_launch %d: max |in-kernel - table| %.3e" % (spl, worst))
    assert worst == 0.0


def test_in_kernel_records_c64(pkg):
    """c64 storage: the same records, so the same bits as the table path."""
    w = mixed_batch("cf4", "leapfrog", seed=11)
    a = run(pkg, w, "c64", True)
    b = run(pkg, w, "c64", False)
    worst = max(float(np.max(np.abs(x - y))) for x, y in zip(a, b))
    say("c64: max |in-kernel - table| %.3e" % worst)
    assert worst == 0.0


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-11), ("c64", 5e-5)])
def test_in_kernel_records_against_oracle(pkg, dtype, tol):
    w = mixed_batch("magnus6", "srkn6_4", seed=13)
    got = run(pkg, w, dtype, True)
    for k in (0, 31, 39, 40, 48, 49, 54, 57, 59, 60):
        inst = w.instances[k]
        ref = oracle.evolve(inst, w.psi0[k], w.scheme, w.ho_rule, w.dt, w.t0, w.nsteps)
        err = W.rel_l2(got[k], ref)
        say("oracle %s N=%d k=%d rel_l2 %.3e" % (dtype, inst.n[0], k, err))
        assert err < tol


def test_plan_with_a_generic_size_uses_the_table(pkg):
    """A plan that holds a size outside 64..2048 takes the record table for
    every group; its results do not depend on in_kernel_records."""
    w = mixed_batch("cf4", "leapfrog", seed=17)
    extra = W.batch_1d(n_inst=2, sizes=(32, 4096), nsteps=w.nsteps, seed=3)
    w = replace(w, instances=w.instances + extra.instances, psi0=w.psi0 + extra.psi0)
    a = run(pkg, w, "c128", True)
    b = run(pkg, w, "c128", False)
    assert all(np.array_equal(x, y) for x, y in zip(a, b))


def test_in_kernel_records_across_launches_of_16384_steps(pkg):
    """Evolve calls longer than 16384 steps run as several resident launches
    (the records of each start at its global step, the opening phase only in
    the first); the bits match the record-table path."""
    w = mixed_batch("cf4", "leapfrog", seed=23)
    w = replace(w, instances=w.instances[36:44], psi0=w.psi0[36:44], nsteps=16384 + 37, dt=2e-5)
    a = run(pkg, w, "c128", True)
    b = run(pkg, w, "c128", False)
    worst = max(float(np.max(np.abs(x - y))) for x, y in zip(a, b))
    say("16421 steps: max |in-kernel - table| %.3e" % worst)
    assert worst == 0.0
