"""Benchmark: batched 1-D Hermite-Fourier GPE time stepping on one MI355X.

Workload: 4096 independent 1-D GPE instances, grid sizes drawn from
{256, 512, 1024, 2048} on [-N/64, N/64) (dx = 1/32), omega(t) = w0 (1 + a sin(nu t)),
sigma ~ U[-1, 50], eps V_I = 0.01 cos 3x, BAB leapfrog with the fourth-order
commutator-free HO rule, dt = 1e-3; inputs seeded (workloads.batch_1d).

One benchmark "step" advances every instance of the batch by one time step
(one FFT pair per instance).  The headline value is the complex64-storage
batched solver (state resident on chip for a chunk of steps, one launch per
chunk) in grid-point-steps per second; the plain FP64 solver (complex128, one
launch per step per grid size) and the complex128 batched solver are timed
beside it, and the relative L2 error of every result is stated.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "grid-point-steps/s + %HBM peak, c64 batched vs FP64 plain, at stated L2 error"
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_hf1d_batch1d.json")


# Sources of a measured kernel's translation unit (the .hip file and every
# header it includes): a change to any of them makes stored counters stale;
# host-only changes (the API runtime) do not.
KERNEL_TU_1D = ("kern_1d.hip", "hf1d_fixed.hpp", "coeff_step.hpp", "coeff.hpp", "devmath.hpp",
                "fft_lds.hpp", "kernels.hpp", "layout.hpp")
KERNEL_TU_ND = ("nd_pass.hpp", "kern_nd.hip", "kern_nd_fix.hip", "kern_nd_fix_coupled.hip",
                "devmath.hpp", "fft_lds.hpp", "kernels.hpp", "layout.hpp")


def kernel_source_hash(names=KERNEL_TU_1D) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1007_3470_amd", "csrc")
    for name in sorted(names):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def flops_per_gp_step(n: int, m: int) -> float:
    """Algorithmic flops of one grid point advanced one step: per stage the
    radix-2 count of an FFT pair (2 x 5 log2 N per point), two complex phase
    multiplies (12) and the phase arguments (x-phase 5, drift 2)."""
    return m * (10.0 * np.log2(n) + 19.0)


def progress(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def timed_evolve(pkg, torch, w, dtype, K, warmup, **kw):
    plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, profile=True, **kw)
    # both buffers are packed first, so the timed call follows the warm-up
    # steps without the host-to-device copy in between
    buf = plan.pack(w.psi0)
    if warmup > 0:
        scratch = plan.pack(w.psi0)
        torch.cuda.synchronize()
        plan.evolve(scratch, 0.0, warmup)
    torch.cuda.synchronize()
    plan.profile()  # reset counters
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    plan.evolve(buf, 0.0, K)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    step_ms, coeff_ms, launches = plan.profile()
    status = plan.device_status()
    if status != 0:
        raise RuntimeError("device status %d" % status)
    progress("%s %s%s: %d steps in %.3f s" % (w.name, dtype, " plain" if kw.get("plain") else "", K, wall))
    return plan, buf, wall, gpu_ms, step_ms, coeff_ms, launches


def nd_passes_per_step(pkg, w) -> int:
    """Axis passes of one d-D step: d per stage for a separable trap; for a
    coupled trap 2d - 1 per exponential (two per stage under CF4, one
    otherwise), the Fourier split staying separable."""
    d = w.instances[0].ndim
    m = len(pkg.scheme_preset(w.scheme)[0])
    coupled = any(any(v != 0.0 for v in getattr(i, "wcross", (0.0, 0.0, 0.0))) for i in w.instances)
    if not coupled or w.ho_rule == "fsplit":
        return m * d
    return (2 * m if w.ho_rule == "cf4" else m) * (2 * d - 1)


def nd_workload(pkg, torch, W, w, reps=5, tune=True):
    """Secondary measurement: a d-D workload at full size and length, c64 and
    c128, steps replayed from hipGraph blocks.  The run is timed with HIP
    events on the plan's stream, median of `reps` runs from the same input;
    the per-pass time is that step time over the passes per step (the one
    opening pass and the coefficient kernel of the run included)."""
    out = {}
    res = {}
    npass = nd_passes_per_step(pkg, w)
    for dtype, sc in (("c64", 8), ("c128", 16)):
        plan = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, use_graph=True)
        # per-pass tuning on a scratch copy of the input (bitwise the same results)
        if tune:
            plan.autotune(w.psi0, trial_steps=8)
        scratch = plan.pack(w.psi0)
        plan.evolve(scratch, 0.0, 2)
        del scratch
        stream = torch.cuda.current_stream()
        runs = []
        for _ in range(reps):
            buf = plan.pack(w.psi0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            plan.evolve(buf, 0.0, w.nsteps)
            e1.record(stream)
            torch.cuda.synchronize()
            runs.append(e0.elapsed_time(e1) / 1e3)
        res[dtype] = plan.unpack(buf)
        run_s = float(np.median(runs))
        pass_s = run_s / (w.nsteps * npass)
        bw = 2.0 * sc * w.points / pass_s / 1e9
        out[dtype] = {"value": w.points * w.nsteps / run_s, "ms_per_step": run_s * 1e3 / w.nsteps,
                      "runs_s": [round(r, 6) for r in runs], "passes_per_step": npass,
                      "tuned_passes": [list(t) for t in plan.tune_settings()],
                      "pass_us": pass_s * 1e6, "pass_GBs": bw, "pass_frac_of_hbm_peak": bw / HBM_PEAK_GBS}
        del plan, buf
    out["c64_pass_time_over_c128"] = out["c64"]["pass_us"] / out["c128"]["pass_us"]
    out["l2_c64_vs_c128_max"] = max(W.rel_l2(a, b) for a, b in zip(res["c64"], res["c128"]))
    progress("%s done" % w.name)
    out["workload"] = w.notes + ", %s + %s, dt=%g, %d steps" % (w.scheme, w.ho_rule, w.dt, w.nsteps)
    return out


def load_traffic(src_hash):
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != src_hash:
        return None  # kernel changed since the counters were taken
    return t.get("bytes_per_launch")


def host_threads(cap: int = 16) -> int:
    """CPUs this process may run on, at most `cap` (a one-GPU share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def cpu_baseline(w, K, per_size, gpu_out, target_s=15.0):
    """The oracle on a bounded sample: the first `per_size` instances of each
    grid size, one instance per task on a pool of host threads (the oracle's C
    evolve runs outside the GIL), largest first.  Each task advances its
    instance the benchmark's K steps (those states give the parity figures),
    then continues from there until the whole sample has run about
    `target_s` seconds; the rate is over every step the sample ran."""
    import concurrent.futures
    import oracle
    import workloads as W
    picks = {}
    for k, inst in enumerate(w.instances):
        lst = picks.setdefault(inst.n[0], [])
        if len(lst) < per_size:
            lst.append(k)
    sample = sorted((k for lst in picks.values() for k in lst), key=lambda k: -w.instances[k].n[0])
    threads = min(host_threads(), len(sample))
    pts = sum(w.instances[k].n[0] for k in sample)
    oracle._lib()  # load (and if needed build) once, before the threads start

    def run(steps_of, t0_of, start):
        with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
            futs = {k: ex.submit(oracle.evolve, w.instances[k], start[k], w.scheme, w.ho_rule, w.dt, t0_of,
                                 steps_of) for k in sample}
            return {k: f.result() for k, f in futs.items()}

    t0 = time.perf_counter()
    refs = run(K, 0.0, {k: w.psi0[k] for k in sample})
    dt1 = time.perf_counter() - t0
    steps, state, last = K, refs, (K, dt1)
    # continue the same instances until the sample has run about target_s;
    # each round is sized from the rate of the round before it
    while dt1 < 0.9 * target_s:
        per_step = last[1] / last[0]
        n = max(K, min(int((target_s - dt1) / max(per_step, 1e-9)), 64 * last[0]))
        t1 = time.perf_counter()
        state = run(n, steps * w.dt, state)
        last = (n, time.perf_counter() - t1)
        dt1 += last[1]
        steps += n
    progress("cpu baseline: %d instances x %d steps on %d threads in %.1f s" % (len(sample), steps, threads, dt1))
    errs = {name: max(W.rel_l2(out[k], refs[k]) for k in sample) for name, out in gpu_out.items()}
    return {"value": pts * steps / dt1, "unit": "grid-point-steps/s", "cores": threads, "kind": "oracle",
            "sample": "%d instances (%d per grid size) x %d steps (the benchmark's %d, then continued), C oracle, "
                      "one instance per task on %d threads, %.1f s wall" % (len(sample), per_size, steps, K,
                                                                            threads, dt1),
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}, errs


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# The paper's accuracy comparisons, run through the library (complex128):
#   sec41: Figs. 3-6 -- F-split vs HO-split (Hermite-Fourier) for LF, NI4(8,2),
#          RKN6_4 and NI5(8,4) at sigma = 0.01, 1, 100 (mu = omega = 1, V_I = 0);
#   sec42: Figs. 7-8 -- time-dependent traps with a quartic perturbation: F-split
#          vs HO-split with the CF4, Magnus6 and fundamental-matrix HO rules for
#          the two fourth-order methods RKN6_4 and NI5(8,4).
# Error: relative L2 at the final time against a reference run of the same
# problem with RKN6_4 at 2^14 steps (HO-split; exact_const or fundamental:16).
# Cost: exponentials per run = FFT pairs = m x steps (the paper's cost axis).
# ---------------------------------------------------------------------------
STUDY_SCHEMES = {"sec41": ("leapfrog", "ni4_82", "srkn6_4", "ni5_84"),
                 "sec42": ("srkn6_4", "ni5_84")}


def _study_run(pkg, torch, w, scheme, rule, nsteps):
    T = w.dt * w.nsteps
    plan = pkg.Plan(w.instances, scheme, rule, "c128", T / nsteps)
    buf = plan.pack(w.psi0)
    plan.evolve(buf, w.t0, nsteps)
    torch.cuda.synchronize()
    if plan.device_status() != 0:
        raise RuntimeError("device status")
    return plan.unpack(buf)[0]


def _cost_at(series, target):
    """FFT pairs needed for rel. error `target` (log-log interpolation), or None."""
    for (c0, e0), (c1, e1) in zip(series, series[1:]):
        if e0 >= target > e1 > 0:
            f = (np.log(target) - np.log(e0)) / (np.log(e1) - np.log(e0))
            return float(np.exp(np.log(c0) + f * (np.log(c1) - np.log(c0))))
    return series[0][0] if series and series[0][1] < target else None


def study(which):
    import torch
    import paper_1007_3470_amd as pkg
    import workloads as W
    pkg.load()
    problems = []
    if which in ("sec41", "all"):
        for sig in (0.01, 1.0, 100.0):
            problems.append(("sec41", "sigma=%g" % sig, W.perturbed_1d(sigma=sig), "exact_const",
                             ("fsplit", "exact_const")))
    if which in ("sec42", "all"):
        for form in ("cos", "pulse"):
            problems.append(("sec42", form, W.timedep_1d(form=form), "fundamental:16",
                             ("fsplit", "cf4", "magnus6", "fundamental:8")))
    steps = [10 * 2 ** k for k in range(11)]
    for sec, label, w, ref_rule, rules in problems:
        ref = _study_run(pkg, torch, w, "srkn6_4", ref_rule, 2 ** 14)
        check = _study_run(pkg, torch, w, "ni5_84", ref_rule, 2 ** 14)
        out = {"study": sec, "problem": label, "notes": w.notes,
               "reference": "srkn6_4 + %s, 2^14 steps (ni5_84 at 2^14 differs by %.1e)"
                            % (ref_rule, W.rel_l2(check, ref)), "curves": {}}
        for scheme in STUDY_SCHEMES[sec]:
            m = len(pkg.scheme_preset(scheme)[0])
            for rule in rules:
                series = []
                for n in steps:
                    try:
                        u = _study_run(pkg, torch, w, scheme, rule, n)
                    except pkg.HfgpeError:
                        continue   # step beyond the rule's validity bound
                    series.append((m * n, W.rel_l2(u, ref)))
                out["curves"]["%s/%s" % (scheme, rule)] = {
                    "fft_pairs_err": [[c, float("%.3e" % e)] for c, e in series],
                    "cost_1e-4": _cost_at(series, 1e-4), "cost_1e-8": _cost_at(series, 1e-8)}
        print(json.dumps(out), flush=True)
    return 0


def precision_study():
    """c64 storage against c128 over 10^2 .. 10^4 steps on the 1-D, batch, 2-D
    and 3-D workloads: relative L2 distance (max and median over instances) and
    the norm drift of both storages, at checkpoints of one continuing run (an
    evolve call split into pieces gives the same bits as one call).  A
    distance that grows linearly with the step count would flag a systematic
    error; rounding the stored state grows like its square root."""
    import torch
    import paper_1007_3470_amd as pkg
    import workloads as W
    pkg.load()
    marks = (100, 1000, 10000)
    sets = (("gpe_1d", W.gpe_1d()), ("batch_1d", W.batch_1d()), ("gpe_2d", W.gpe_2d()),
            ("gpe_3d", W.gpe_3d()), ("coupled_2d", W.coupled_2d()), ("coupled_3d", W.coupled_3d()))
    for name, w in sets:
        plans, bufs = {}, {}
        for dtype in ("c64", "c128"):
            plans[dtype] = pkg.Plan(w.instances, w.scheme, w.ho_rule, dtype, w.dt, use_graph=w.instances[0].ndim > 1)
            bufs[dtype] = plans[dtype].pack(w.psi0)
        n0 = plans["c128"].norm(bufs["c128"])
        out = {"study": "precision", "workload": name, "notes": w.notes, "scheme": w.scheme, "rule": w.ho_rule,
               "dt": w.dt, "checkpoints": []}
        done = 0
        for mark in marks:
            for dtype in ("c64", "c128"):
                plans[dtype].evolve(bufs[dtype], w.t0 + done * w.dt, mark - done)
            torch.cuda.synchronize()
            done = mark
            a, b = plans["c64"].unpack(bufs["c64"]), plans["c128"].unpack(bufs["c128"])
            errs = np.array([W.rel_l2(x, y) for x, y in zip(a, b)])
            out["checkpoints"].append({
                "steps": mark, "c64_vs_c128_max": float("%.3e" % errs.max()),
                "c64_vs_c128_median": float("%.3e" % np.median(errs)),
                "norm_drift_c64": float("%.3e" % np.abs(plans["c64"].norm(bufs["c64"]) - n0).max()),
                "norm_drift_c128": float("%.3e" % np.abs(plans["c128"].norm(bufs["c128"]) - n0).max())})
            progress("precision %s: %d steps" % (name, mark))
        print(json.dumps(out), flush=True)
        del plans, bufs
    return 0


def mall_study(steps: int = 1000):
    """The 1-D batch scaled past the 256 MB MALL (AMD's last-level cache):
    4096, 16384 and 40960 instances of the batch recipe, c64 and c128, the
    rate over `steps` steps.  The resident kernel touches HBM once per launch,
    so the rate should not depend on whether the state fits in the cache."""
    import torch
    import paper_1007_3470_amd as pkg
    import workloads as W
    pkg.load()
    for n_inst in (4096, 16384, 40960):
        w = W.batch_1d(n_inst=n_inst, nsteps=steps)
        out = {"study": "mall", "instances": n_inst, "grid_points": w.points, "steps": steps}
        for dtype, sc in (("c64", 8), ("c128", 16)):
            plan, buf, wall, *_ = timed_evolve(pkg, torch, w, dtype, steps, 20)
            out[dtype] = {"state_MB": w.points * sc / 1e6, "value": w.points * steps / wall}
            del plan, buf
        print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-per-size", type=int, default=16,
                    help="oracle sample: instances per grid size (0 disables)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--no-nd", action="store_true", help="skip the 2-D and 3-D workloads")
    ap.add_argument("--nd-steps", type=int, default=0,
                    help="steps of the 2-D and 3-D workloads (0 = their full runs)")
    ap.add_argument("--nd-only", action="store_true",
                    help="only the 2-D and 3-D workloads (for profiling their kernels)")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the d-D workloads with the default pass settings (no autotuning)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (HBM counter calibration)")
    ap.add_argument("--study", choices=("sec41", "sec42", "all", "precision", "mall"),
                    help="run the paper's accuracy-vs-cost comparisons instead of the "
                         "benchmark (one JSON line per problem)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(independent instances would be sharded across GPUs with no exchange); use --gpus 1",
              file=sys.stderr)
        return 2

    if args.study == "precision":
        return precision_study()
    if args.study == "mall":
        return mall_study()
    if args.study:
        return study(args.study)

    import torch
    import paper_1007_3470_amd as pkg
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    pkg.load()
    K, WU = args.steps, args.warmup
    nd_kw = {"nsteps": args.nd_steps} if args.nd_steps > 0 else {}
    nd_sets = (("gpe_2d", W.gpe_2d), ("gpe_3d", W.gpe_3d), ("coupled_2d", W.coupled_2d),
               ("coupled_3d", W.coupled_3d))
    if args.nd_only:
        print(json.dumps({"other_workloads": {name: nd_workload(pkg, torch, W, gen(**nd_kw), tune=not args.no_tune)
                                              for name, gen in nd_sets}}), flush=True)
        return 0
    w = W.batch_1d(nsteps=K)
    npts = w.points
    m = len(pkg.scheme_preset(w.scheme)[0])
    sizes = np.array([i.n[0] for i in w.instances])
    flops_per_step = float(sum(n * flops_per_gp_step(n, m) for n in sizes))

    # headline: complex64 storage, batched resident solver
    plan64, buf64, wall64, ms64, kms64, cms64, nl64 = timed_evolve(pkg, torch, w, "c64", K, WU)
    out64 = plan64.unpack(buf64)
    # complex128 batched and the plain FP64 solver
    plan128, buf128, wall128, ms128, kms128, cms128, nl128 = timed_evolve(pkg, torch, w, "c128", K, WU)
    out128 = plan128.unpack(buf128)
    plain = None
    if not args.no_plain:
        pl, bufp, wallp, msp, kmsp, cmsp, nlp = timed_evolve(pkg, torch, w, "c128", K,
                                                             min(WU, 20), plain=True)
        outp = pl.unpack(bufp)
        plain = {"value": npts * K / wallp, "ms_per_step": wallp * 1e3 / K, "launches": nlp,
                 "max_rel_l2_vs_c128_batched": max(W.rel_l2(a, b) for a, b in zip(outp, out128))}
    errs64 = np.array([W.rel_l2(a, b) for a, b in zip(out64, out128)])

    value = npts * K / wall64
    # roofline of the dominant kernel: the resident step kernel, FP64 ALU bound
    avg_launch_s = kms64 / 1e3 / max(1, nl64)
    flops_per_launch = flops_per_step * K / max(1, nl64)
    achieved = flops_per_launch / avg_launch_s / 1e12
    traffic = load_traffic(kernel_source_hash())
    roof = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS, "traffic": traffic,
            "kernel": "hf1d_fixed_kernel<float2> (resident 1-D step, 64 <= N <= 2048)",
            "avg_launch_ms": avg_launch_s * 1e3, "launches": nl64,
            "flops_per_gp_step": "10 log2 N + 19 per stage"}

    line = {
        "metric": METRIC, "value": value, "unit": "grid-point-steps/s", "n_gpus": 1,
        "steps": K, "warmup": WU, "ms_per_step": wall64 * 1e3 / K, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch_1d: 4096 x 1-D GPE, N in {256,512,1024,2048}, L=N/64, "
                               "leapfrog + CF4, dt=1e-3, %d steps" % K,
                   "instances": len(w.instances), "grid_points": npts, "storage": "c64",
                   "arithmetic": "f64", "parallelism": "single GPU, batched resident kernel"},
        # bytes a design with one HBM read + write of the state per stage would
        # move at this rate (16 B per grid-point-step for c64), against 8 TB/s
        "hbm_equivalent": {"GBs": 16.0 * m * value / 1e9,
                           "frac_of_peak": 16.0 * m * value / 1e9 / HBM_PEAK_GBS},
        "gpu_event_ms": {"c64": ms64, "c128": ms128},
        "c128_batched": {"value": npts * K / wall128, "ms_per_step": wall128 * 1e3 / K},
        "fp64_plain": plain,
        "speedup_vs_fp64_plain": (value / plain["value"]) if plain else None,
        "l2": {"c64_vs_c128_max": float(errs64.max()), "c64_vs_c128_median": float(np.median(errs64))},
        "roofline": roof,
        "wall_s": {"c64": wall64, "c128": wall128},
    }
    if not args.no_nd:
        line["other_workloads"] = {name: nd_workload(pkg, torch, W, gen(**nd_kw), tune=not args.no_tune) for name, gen in nd_sets}
    if args.copy_calibration:
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = {"read": 512 << 20, "write": 512 << 20}
    if args.cpu_per_size > 0:
        cpu, errs = cpu_baseline(w, K, args.cpu_per_size, {"c64": out64, "c128": out128})
        line["cpu_baseline"] = cpu
        line["l2"]["c64_vs_oracle_sample_max"] = errs["c64"]
        line["l2"]["c128_vs_oracle_sample_max"] = errs["c128"]
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
