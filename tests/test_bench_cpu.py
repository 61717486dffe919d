"""Host logic of bench.py (no GPU): the kernel-source hashes that decide
whether stored HBM counters still describe the measured kernels, the stored
counters' lookup, the algorithmic flop count, the single-GPU guard and the bounded
oracle sample."""
import json
import math
import os
import re

import bench

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1007_3470_amd", "csrc")


def include_closure(name):
    """Local headers a source pulls in, transitively (#include "...")."""
    seen, todo = set(), [name]
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        with open(os.path.join(CSRC, f)) as fh:
            for inc in re.findall(r'^\s*#include\s+"([^"]+)"', fh.read(), re.M):
                if os.path.exists(os.path.join(CSRC, inc)):
                    todo.append(inc)
    return seen


def test_hash_lists_cover_every_header_of_the_measured_kernels():
    for tu in ("kern_1d.hip", "kern_1d_fused.hip"):
        assert include_closure(tu) <= set(bench.KERNEL_TU_1D) | {"kern_1d_fused.hip"}, tu
    for tu in ("kern_nd.hip", "kern_nd_fix.hip", "kern_nd_fix_coupled.hip"):
        assert include_closure(tu) <= set(bench.KERNEL_TU_ND), tu


def test_hash_changes_with_the_sources_only(tmp_path, monkeypatch):
    h1 = bench.kernel_source_hash()
    assert h1 == bench.kernel_source_hash() and len(h1) == 16
    assert bench.kernel_source_hash(bench.KERNEL_TU_ND) != h1
    # the same files under another root with one byte changed hash differently
    fake = tmp_path / "paper_1007_3470_amd" / "csrc"
    fake.mkdir(parents=True)
    for n in bench.KERNEL_TU_1D:
        data = open(os.path.join(CSRC, n), "rb").read()
        (fake / n).write_bytes(data + (b" " if n == "kern_1d.hip" else b""))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_hash() != h1


def test_stored_traffic_is_used_only_for_matching_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"source_hash": "abc", "bytes_per_launch": 123.0}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic("abc") == 123.0
    assert bench.load_traffic("abd") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.json"))
    assert bench.load_traffic("abc") is None


def test_flops_per_grid_point_step():
    # per stage: a radix-2 FFT pair (10 log2 N), two complex phase products
    # (12) and the phase arguments (7)
    for n in (64, 256, 2048):
        for m in (1, 5):
            assert bench.flops_per_gp_step(n, m) == m * (10 * math.log2(n) + 19)


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU only" in capsys.readouterr().err


def test_nd_passes_per_step():
    """Passes per d-D step, from which the bench derives per-pass times:
    m d for separable traps, (2d - 1) per exponential for coupled ones (CF4
    applies two exponentials per stage)."""
    import bench
    import paper_1007_3470_amd as pkg
    import workloads as W
    assert bench.nd_passes_per_step(pkg, W.gpe_2d(n=16, n_inst=1, nsteps=1)) == 2
    assert bench.nd_passes_per_step(pkg, W.gpe_3d(n=16, nsteps=1)) == 15
    assert bench.nd_passes_per_step(pkg, W.coupled_2d(n=16, n_inst=1, nsteps=1)) == 6
    assert bench.nd_passes_per_step(pkg, W.coupled_3d(n=16, nsteps=1)) == 50
    assert bench.nd_passes_per_step(pkg, W.coupled_2d(n=16, n_inst=1, nsteps=1, rule="fsplit")) == 2
    assert bench.nd_passes_per_step(pkg, W.coupled_2d(n=16, n_inst=1, nsteps=1, rule="exact_const",
                                                      constant=True)) == 3


def test_cpu_baseline_runs_a_bounded_sample():
    """The oracle leg runs the benchmark's K steps on every sampled instance,
    then continues the same instances until about target_s seconds have run,
    and reports the rate over every step it ran."""
    import workloads as W
    w = W.batch_1d(n_inst=12, sizes=(256, 512), nsteps=3, seed=5)
    t0 = bench.time.perf_counter()
    cpu, errs = bench.cpu_baseline(w, 3, 2, {}, target_s=0.4)
    wall = bench.time.perf_counter() - t0
    assert errs == {}
    assert cpu["kind"] == "oracle" and cpu["unit"] == "grid-point-steps/s"
    assert 1 <= cpu["cores"] <= 16 and cpu["value"] > 0
    steps = int(re.search(r"x (\d+) steps", cpu["sample"]).group(1))
    assert steps >= 3
    # the sample is 2 instances per size, about 0.4 s of work: not far beyond
    assert re.match(r"4 instances \(2 per grid size\)", cpu["sample"])
    assert wall < 10.0
