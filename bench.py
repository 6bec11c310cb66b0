"""Benchmark of the gfx950 stable merge sort.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one whole sort (tile sort + every merge pass) of one fresh copy of
the workload, already resident in HBM.  K + W distinct copies are generated
on the GPU before timing, so no restore copy sits inside the timed region.
The K timed steps are bracketed by torch.cuda.synchronize(); while they run
the library's event profiler brackets every kernel launch with HIP events
on the launch stream, which gives the dominant kernel's average duration.

Prints one JSON line.  `roofline` prices the dominant kernel (the merge pass)
at its algorithmic bytes per launch (read + write of every key and value)
against MI355X's 8 TB/s HBM peak; `cpu_baseline` times the CPU oracle
(single-threaded C merge sort) on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (description, n, key bytes, value bytes, C-ABI key type)
    "zipf_pairs_u32_2p27": ("stable key/value sort of 2^27 pairs: uint32 keys Zipf(s=1.1) over 2^20 "
                            "distinct values, uint32 value = original index", 1 << 27, 4, 4, 0),
    "uniform_u32_2p27": ("merge sort of 2^27 uint32 keys uniform in [0, 2^32), keys only", 1 << 27, 4, 0, 0),
    "uniform_u32_2p20": ("merge sort of 2^20 uint32 keys uniform in [0, 2^32), seed 0, keys only",
                         1 << 20, 4, 0, 0),
    "normal_i64_2p28": ("merge sort of 2^28 int64 keys round(N(0, 1) * 2^40), keys only", 1 << 28, 8, 0, 3),
    "nearly_sorted_i64_2p28": ("merge sort of the sorted 2^28 int64 normal array with 1% disjoint adjacent "
                               "swaps, keys only", 1 << 28, 8, 0, 3),
    "lognormal_u32_2p29": ("2^29 uint32 keys from an equal-weight mixture of 8 lognormals (mu ~ U(0,4), "
                           "sigma ~ U(0.1,1), scaled and clipped to uint32): learned-bucket sort vs plain merge "
                           "path", 1 << 29, 4, 0, 0),
    "segments_u32_10000": ("batched segmented sort: 10,000 independent uint32 arrays, lengths log-uniform in "
                           "[16, 2^18], uniform keys, one graph launch, autotuned shape per size class",
                           None, 4, 0, 0),
}


MERGE_KERNEL_SOURCES = ("ms_common.hpp", "ms_merge.hpp", "ms_plain_cfg.hpp")


def merge_kernel_source_hash() -> str:
    """sha256 over the sources that define the merge kernel and its shape."""
    import hashlib
    h = hashlib.sha256()
    for f in MERGE_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2211_16479_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(workload: str, kernel: str = "merge_kernel"):
    """Calibrated HBM bytes per launch of `kernel` from the committed counter
    summary, or None when there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", " ", "#")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != merge_kernel_source_hash():
        return None
    try:
        return int(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def make_inputs(name, copies, dev):
    import torch
    import workloads
    if name == "zipf_pairs_u32_2p27":
        k, v = workloads.zipf_pairs_u32(1 << 27, seed=0, device=dev)
        return [(k.clone(), v.clone()) for _ in range(copies)], (k, v)
    if name == "uniform_u32_2p27":
        k = workloads.uniform_u32(1 << 27, seed=0, device=dev)
        return [(k.clone(), None) for _ in range(copies)], (k, None)
    if name == "uniform_u32_2p20":
        k = workloads.uniform_u32(1 << 20, seed=0, device=dev)
        return [(k.clone(), None) for _ in range(copies)], (k, None)
    if name == "segments_u32_10000":
        k, off = workloads.segments_u32(10000, seed=0, device=dev)
        return [(k.clone(), off)], (k, off)
    if name in ("normal_i64_2p28", "nearly_sorted_i64_2p28"):
        k = workloads.normal_i64(1 << 28, seed=0, device=dev)
        if name == "nearly_sorted_i64_2p28":
            k = workloads.nearly_sorted(torch.sort(k).values, 0.01, seed=0)
        return [(k.clone(), None) for _ in range(copies)], (k, None)
    raise SystemExit(f"unknown workload {name}")


def _host(t):
    """Host numpy copy of a tensor (uint32 through an int32 view)."""
    import numpy as np
    import torch
    if t.dtype == torch.uint32:
        return t.cpu().view(torch.int32).numpy().view(np.uint32)
    return t.cpu().numpy()


def cpu_baseline(name, pristine, budget_s=20.0):
    """Time the CPU oracle on a bounded prefix of the workload: the largest
    power-of-two prefix whose estimated single-threaded sort time fits the
    budget (estimated from a small calibration sort)."""
    import numpy as np
    import oracle
    k, v = pristine
    kn = _host(k)
    vn = None if v is None else _host(v)
    # calibration on 2^18 keys
    m = min(kn.size, 1 << 18)
    t0 = time.perf_counter()
    if vn is None:
        oracle.sort(kn[:m])
    else:
        oracle.sort_pairs(kn[:m], vn[:m])
    t_cal = time.perf_counter() - t0
    per_key_level = t_cal / (m * max(1, np.log2(m)))
    s = m
    while s * 2 <= kn.size and per_key_level * (2 * s) * np.log2(2 * s) < budget_s:
        s *= 2
    t0 = time.perf_counter()
    if vn is None:
        oracle.sort(kn[:s])
    else:
        oracle.sort_pairs(kn[:s], vn[:s])
    dt = time.perf_counter() - t0
    what = "pairs" if vn is not None else "keys"
    return {"value": s / dt / 1e9, "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
            "sample": f"first 2^{int(np.log2(s))} {what} of the workload, one single-threaded oracle "
                      f"merge sort, {dt:.2f} s"}


def time_restored(fn, work, pristine, steps, warmup):
    """Mean event-timed duration (ms) of fn() over `steps` runs; before each
    run the pristine input is copied into `work`, outside the event window."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        work.copy_(pristine)
        fn()
    torch.cuda.synchronize()
    total = 0.0
    for _ in range(steps):
        work.copy_(pristine)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        total += a.elapsed_time(b)
    return total / steps


def learned_vs_plain(steps=5, warmup=2):
    """Both forms on the 2^29 lognormal-mixture workload, the same way:
    Gkeys/s of each, the speedup, whether the two outputs are byte-identical,
    and the learned run's device-side statistics."""
    import torch
    import paper_2211_16479_amd as msort
    import workloads
    dev = torch.device("cuda:0")
    n = 1 << 29
    pristine = workloads.lognormal_mix_u32(n, seed=0, device=dev)
    work = torch.empty_like(pristine)
    t_plain = time_restored(lambda: msort.ms_sort(work), work, pristine, steps, warmup)
    out_plain = work.clone()
    t_learned = time_restored(lambda: msort.ms_sort_ex(work, algo=msort.MS_ALGO_LEARNED_BUCKET, stats=False),
                              work, pristine, steps, warmup)
    work.copy_(pristine)
    _, st = msort.ms_sort_ex(work, algo=msort.MS_ALGO_LEARNED_BUCKET)
    torch.cuda.synchronize()
    same = bool((work.view(torch.int32) == out_plain.view(torch.int32)).all())
    del out_plain, work, pristine
    torch.cuda.empty_cache()
    return {"workload": WORKLOADS["lognormal_u32_2p29"][0], "n": n,
            "plain_ms": round(t_plain, 4), "plain_Gkeys_s": round(n / (t_plain * 1e-3) / 1e9, 3),
            "learned_ms": round(t_learned, 4), "learned_Gkeys_s": round(n / (t_learned * 1e-3) / 1e9, 3),
            "speedup": round(t_plain / t_learned, 3), "outputs_identical": same,
            "learned_stats": {k: (round(v, 8) if isinstance(v, float) else v) for k, v in st.items()}}


def bench_segmented(args, desc):
    """One step = one ms_segmented_sort (one graph launch) of all 10,000
    arrays.  The same buffers are reused so the cached graph is replayed; the
    pristine keys are restored before each step, outside the event window,
    and the K event-timed steps are summed."""
    import torch
    import paper_2211_16479_amd as msort
    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    [(work, off)], (pristine, _) = make_inputs(args.workload, 1, dev)
    n = work.numel()
    stream = torch.cuda.current_stream()
    for _ in range(W):
        work.copy_(pristine)
        msort.ms_segmented_sort(work, off, max_segment_len=1 << 18)
    torch.cuda.synchronize()
    total_ms = 0.0
    for _ in range(K):
        work.copy_(pristine)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        msort.ms_segmented_sort(work, off, max_segment_len=1 << 18)
        b.record(stream)
        torch.cuda.synchronize()
        total_ms += a.elapsed_time(b)
    ms_per_step = total_ms / K
    shapes = {f"class{c}(<={bd})": "x".join(map(str, msort.ms_tuning_get(0, 0, c)))
              for c, (bd, _) in enumerate(msort.ms_seg_classes(0, 0))}
    out = {
        "metric": "Gkeys/s and HBM GB/s vs peak, plain merge-path vs learned-bucket, bit-exact",
        "value": round(n / (ms_per_step * 1e-3) / 1e9, 4),
        "unit": "Gkeys/s", "n_gpus": 1, "steps": K, "warmup": W, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": desc, "n": n, "segments": off.numel() - 1, "class_shapes": shapes},
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="zipf_pairs_u32_2p27", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain comparison on the lognormal-mixture workload")
    ap.add_argument("--no-kernel-events", action="store_true",
                    help="time without the per-launch events (no roofline)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run torch's plain device copy of the workload's byte size 3 times "
                         "(reference dispatches for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the sharded design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2211_16479_amd as msort

    dev = torch.device("cuda:0")
    desc, n, kb, vb, kt = WORKLOADS[args.workload]
    if args.copy_calibration:
        nbytes = n * (kb + vb)
        a = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes, "dispatches": 3}))
        return
    K, W = args.steps, args.warmup
    if args.workload == "segments_u32_10000":
        return bench_segmented(args, desc)
    if args.workload == "lognormal_u32_2p29":
        r = learned_vs_plain(K, W)
        print(json.dumps({
            "metric": "Gkeys/s and HBM GB/s vs peak, plain merge-path vs learned-bucket, bit-exact",
            "value": r["learned_Gkeys_s"], "unit": "Gkeys/s", "n_gpus": 1, "steps": K, "warmup": W,
            "ms_per_step": r["learned_ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u32", "data": "synthetic", "config": {"workload": desc, "n": n},
            "learned_vs_plain": r, "roofline": None, "cpu_baseline": None}))
        return
    bufs, pristine = make_inputs(args.workload, K + W, dev)
    torch.cuda.synchronize()

    def step(i):
        k, v = bufs[i]
        if v is None:
            msort.ms_sort(k)
        else:
            msort.ms_sort_pairs(k, v)

    for i in range(W):
        step(i)
    torch.cuda.synchronize()
    msort.ms_profile_reset()
    msort.ms_profile_enable(not args.no_kernel_events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(W, W + K):
        step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    msort.ms_profile_enable(False)
    ms_per_step = (t1 - t0) * 1e3 / K
    value = n / (ms_per_step * 1e-3) / 1e9

    kernels = {}
    for name in ("tile_sort", "partition", "merge", "partition4", "merge4"):
        cnt, tot = msort.ms_profile_read(name)
        if cnt:
            kernels[name] = {"launches": cnt, "avg_ms": tot / cnt, "ms_per_step": tot / K}
    # the dominant merge kernel: the fused four-run merge when passes are
    # fused, else the two-run merge
    dom = max((k for k in ("merge", "merge4") if k in kernels), key=lambda k: kernels[k]["ms_per_step"],
              default=None)
    roofline = None
    if dom:
        bytes_per_launch = n * (kb + vb) * 2          # read + write of every key and value
        achieved = bytes_per_launch / (kernels[dom]["avg_ms"] * 1e-3) / 1e9
        kname = "merge4_kernel" if dom == "merge4" else "merge_kernel"
        levels = 2 if dom == "merge4" else 1       # merge-tree levels one launch completes
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(args.workload, kname),
                    "kernel": kname, "bytes_per_launch": bytes_per_launch, "tree_levels_per_launch": levels,
                    "per_level_equivalent_GBs": round(achieved * levels, 1)}
    # whole-sort algorithmic bytes (tile sort pass + HBM merge passes)
    plan = msort.ms_plan_query(n, kt, vb)
    total_bytes = n * (kb + vb) * 2 * (1 + plan["hbm_passes"])

    del bufs
    torch.cuda.empty_cache()
    lvp = None
    if not args.no_learned and args.workload == "zipf_pairs_u32_2p27":
        lvp = learned_vs_plain()
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload, pristine)

    out = {
        "metric": "Gkeys/s and HBM GB/s vs peak, plain merge-path vs learned-bucket, bit-exact",
        "value": round(value, 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32" if kb == 4 else "int64",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "key_bytes": kb, "value_bytes": vb,
                   "tile": plan["tile"], "merge_tile": plan["merge_tile"], "merge4_tile": plan["merge4_tile"],
                   "merge_levels": plan["passes"], "hbm_merge_passes": plan["hbm_passes"]},
        "whole_sort_hbm_GBs": round(total_bytes / (ms_per_step * 1e-3) / 1e9, 1),
        "kernels": kernels,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "learned_vs_plain": lvp,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
