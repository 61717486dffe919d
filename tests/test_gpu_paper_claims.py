"""The paper's Sec. 4.1 findings (Figs. 3-6) through the GPU path: at the same
cost (leapfrog, 200 FFT pairs over T = 10) the Hermite-Fourier split (Lemma 2
for the HO part) beats the Fourier split by orders of magnitude when the
nonlinearity is a small perturbation (sigma = 0.01), keeps a smaller gain at
sigma = 1, and the two coincide at sigma = 100.  The reference is NI5(8,4)
with the exact HO rule at 8192 steps.  Problem parameters as printed in
Sec. 4.1 (tests/golden/sec4_problems.txt)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import torch
    assert torch.cuda.is_available()
    import paper_1007_3470_amd as p
    p.load()
    return p


def final_state(pkg, w):
    import torch
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, "c128", w.dt)
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, w.nsteps)
    torch.cuda.synchronize()
    assert plan.device_status() == 0
    return plan.unpack(buf)[0]


@pytest.mark.parametrize("sigma,scheme,nsteps,lo,hi", [(0.01, "leapfrog", 200, 30.0, None),
                                                       (1.0, "leapfrog", 200, 1.5, 20.0),
                                                       (1.0, "srkn6_4", 100, 0.5, 3.0),
                                                       (100.0, "ni5_84", 2000, 0.5, 2.0)])
def test_hermite_vs_fourier_split(pkg, sigma, scheme, nsteps, lo, hi):
    """At sigma = 1 the gain shrinks to about 2x in cost for the second-order
    method (4x in error) and disappears for the fourth-order one.  At
    sigma = 100 a second-order method is nowhere near the solution at 200
    steps (both errors are O(1)), so the comparison there is made with
    NI5(8,4) at a cost where both splits are accurate."""
    ref = final_state(pkg, W.perturbed_1d(sigma=sigma, nsteps=8192, scheme="ni5_84", rule="exact_const"))
    err_h = W.rel_l2(final_state(pkg, W.perturbed_1d(sigma=sigma, nsteps=nsteps, scheme=scheme,
                                                     rule="exact_const")), ref)
    err_f = W.rel_l2(final_state(pkg, W.perturbed_1d(sigma=sigma, nsteps=nsteps, scheme=scheme,
                                                     rule="fsplit")), ref)
    ratio = err_f / err_h
    print("sigma=%g, %s x %d: HF split %.2e, F split %.2e, ratio %.1f"
          % (sigma, scheme, nsteps, err_h, err_f, ratio), flush=True)
    assert err_h < 1e-2 and err_f < 1e-1  # both resolve the solution at this cost
    assert ratio > lo and (hi is None or ratio < hi)


@pytest.mark.parametrize("form", ["cos", "pulse"])
def test_time_dependent_traps(pkg, form):
    """Sec. 4.2 (Figs. 7-8), NI5(8,4) with 50 steps over T = 5 (250 FFT
    pairs): the HO split with any HO rule beats the Fourier split by orders of
    magnitude on both traps.  On the faster pulse the HO rule's own error
    shows: the sixth-order Magnus rule beats CF4, and the exact
    fundamental-matrix rule beats both.  Reference: RKN6_4 with the
    fundamental rule at 2^14 steps."""
    ref = final_state(pkg, W.timedep_1d(form=form, nsteps=1 << 14, scheme="srkn6_4", rule="fundamental"))
    err = {rule: W.rel_l2(final_state(pkg, W.timedep_1d(form=form, nsteps=50, scheme="ni5_84", rule=rule)), ref)
           for rule in ("fsplit", "cf4", "magnus6", "fundamental")}
    print("%s trap: %s" % (form, ", ".join("%s %.2e" % kv for kv in err.items())), flush=True)
    assert err["fsplit"] > 100 * max(err["cf4"], err["magnus6"], err["fundamental"])
    if form == "pulse":
        assert err["cf4"] > 1.5 * err["magnus6"] and err["magnus6"] > err["fundamental"]


def test_second_vs_fourth_order_crossover(pkg):
    """Sec. 4.1 at sigma = 0.01 (Fig. 4-5): with the HO split the (8,2) method
    NI4 is the cheaper one at low accuracy and the (8,4) method NI5 at high
    accuracy: at 40 FFT pairs NI4 (10 steps) has the smaller error than NI5
    (8 steps), at 400 pairs (100 and 80 steps) the larger."""
    ref = final_state(pkg, W.perturbed_1d(sigma=0.01, nsteps=8192, scheme="ni5_84", rule="exact_const"))

    def err(scheme, nsteps):
        return W.rel_l2(final_state(pkg, W.perturbed_1d(sigma=0.01, nsteps=nsteps, scheme=scheme,
                                                      rule="exact_const")), ref)
    low = (err("ni4_82", 10), err("ni5_84", 8))
    high = (err("ni4_82", 100), err("ni5_84", 80))
    print("40 pairs: NI4 %.2e, NI5 %.2e; 400 pairs: NI4 %.2e, NI5 %.2e" % (low + high), flush=True)
    assert 3 * low[0] < low[1]     # measured 8.8e-6 vs 1.6e-4
    assert 10 * high[1] < high[0]  # measured 6.6e-11 vs 1.3e-8
