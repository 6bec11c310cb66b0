"""Benchmark of the gfx950 stable merge sort.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Default workload: 2^29 uint32 keys from the 8-lognormal mixture, sorted by
the learned-bucket form (the headline: its Gkeys/s is `value`) and by the
plain merge-path form beside it, with a byte-for-byte comparison of the two
outputs.  A step is one whole sort of one fresh copy of the workload,
already resident in HBM: K + W copies are made before timing, so nothing but
the sorts runs in the timed region.  The K timed steps are bracketed by
torch.cuda.synchronize() on both sides; while they run the library's event
profiler brackets every kernel launch with HIP events on the launch stream,
which gives each kernel class's average duration.

`roofline` prices the headline form's dominant kernel at its algorithmic
bytes per launch against MI355X's 8 TB/s HBM peak; the plain form and the
extra workloads (2^27 Zipf pairs, 2^27 uint32 keys) carry their own.
`cpu_baseline` times the CPU oracle (the plain C merge sort) on a bounded
sample of the same workload with every host core (threaded top levels), and
on one core beside it.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# The paper's own measurements (CPU wall-clock of its Python sorts of 10^7
# integers), as context only: another workload, machine and language.
PAPER_CONTEXT = {
    "workload": "10^7 integers (Python lists; the MPI runs' NumPy int64 uniform in [0, n))",
    "hardware": "Lenovo NeXtScale nx360 M5, 2 x 12-core Intel Xeon E5-2680 v3, 256 GB",
    "best_multiprocessing": {"seconds": 2.487, "Mkeys_s": 4.021, "workers": 12,
                             "where": "section Analysis of Single Processor Sorting, multiprocessing table"},
    "sequential_python": {"seconds": 85.611, "Mkeys_s": 0.117, "where": "same section, sequential table"},
    "python_sorted": {"seconds": 3.860, "Mkeys_s": 2.591, "where": "same section"},
}
METRIC = "Gkeys/s and HBM GB/s vs peak, plain merge-path vs learned-bucket, bit-exact"

WORKLOADS = {
    # name: (description, n, key bytes, value bytes, C-ABI key type)
    "lognormal_u32_2p29": ("2^29 uint32 keys from an equal-weight mixture of 8 lognormals (mu ~ U(0,4), "
                           "sigma ~ U(0.1,1), scaled and clipped to uint32): learned-bucket sort vs plain merge "
                           "path", 1 << 29, 4, 0, 0),
    "zipf_pairs_u32_2p27": ("stable key/value sort of 2^27 pairs: uint32 keys Zipf(s=1.1) over 2^20 "
                            "distinct values, uint32 value = original index", 1 << 27, 4, 4, 0),
    "uniform_u32_2p27": ("merge sort of 2^27 uint32 keys uniform in [0, 2^32), keys only", 1 << 27, 4, 0, 0),
    "uniform_u32_2p20": ("merge sort of 2^20 uint32 keys uniform in [0, 2^32), seed 0, keys only",
                         1 << 20, 4, 0, 0),
    "normal_i64_2p28": ("merge sort of 2^28 int64 keys round(N(0, 1) * 2^40), keys only", 1 << 28, 8, 0, 3),
    "nearly_sorted_i64_2p28": ("merge sort of the sorted 2^28 int64 normal array with 1% disjoint adjacent "
                               "swaps, keys only", 1 << 28, 8, 0, 3),
    "segments_u32_10000": ("batched segmented sort: 10,000 independent uint32 arrays, lengths log-uniform in "
                           "[16, 2^18], uniform keys, one graph launch, autotuned shape per size class",
                           None, 4, 0, 0),
}

KERNEL_SOURCES = ("ms_common.hpp", "ms_merge.hpp", "ms_plain_cfg.hpp", "ms_learned.hpp", "ms_segmented.hpp",
                  "ms_block_sort.hpp")


def kernel_source_hash() -> str:
    """sha256 over the sources that define the kernels and their shapes."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2211_16479_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(workload: str, kernel: str):
    """Calibrated HBM bytes (FETCH_SIZE + WRITE_SIZE) per launch of `kernel`
    (or per sort, for a stage of several kernels) from the committed counter
    summary profiles/traffic_<workload>.md, or None when there is none or the
    kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", " ", "#")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != kernel_source_hash():
        return None
    try:
        return int(fields[f"traffic.{kernel}"])
    except (KeyError, ValueError):
        return None


def host_info() -> dict:
    """Host cores and CPU model (the oracle's machine)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"nproc": os.cpu_count(), "affinity_cpus": affinity, "cpu_model": model}


def _host(t):
    """Host numpy copy of a tensor (uint32 through an int32 view)."""
    import numpy as np
    import torch
    if t.dtype == torch.uint32:
        return t.cpu().view(torch.int32).numpy().view(np.uint32)
    return t.cpu().numpy()


def sha256_of(*tensors) -> str:
    h = hashlib.sha256()
    for t in tensors:
        h.update(memoryview(_host(t)).cast("B"))
    return h.hexdigest()


def make_pristine(name, dev):
    """The workload's input on the device: (keys, values or None)."""
    import torch
    import workloads
    n = WORKLOADS[name][1]
    if name == "lognormal_u32_2p29":
        return workloads.lognormal_mix_u32(n, seed=0, device=dev), None
    if name == "zipf_pairs_u32_2p27":
        return workloads.zipf_pairs_u32(n, seed=0, device=dev)
    if name in ("uniform_u32_2p27", "uniform_u32_2p20"):
        return workloads.uniform_u32(n, seed=0, device=dev), None
    if name in ("normal_i64_2p28", "nearly_sorted_i64_2p28"):
        k = workloads.normal_i64(n, seed=0, device=dev)
        if name == "nearly_sorted_i64_2p28":
            k = workloads.nearly_sorted(torch.sort(k).values, 0.01, seed=0)
        return k, None
    raise SystemExit(f"unknown workload {name}")


def read_kernels(K: int) -> dict:
    import paper_2211_16479_amd as msort
    out = {}
    for name in msort.PROFILE_KERNELS:
        cnt, tot = msort.ms_profile_read(name)
        if cnt:
            out[name] = {"launches": cnt, "avg_us": round(tot / cnt * 1e3, 2), "ms_per_step": round(tot / K, 4)}
    return out


def timed_steps(step, K: int, W: int, events: bool, classes=None):
    """W untimed steps, then exactly K steps between two synchronisations;
    returns (ms per step, per-kernel-class event times of the K steps).
    classes: the kernel classes bracketed by events (None: all)."""
    import torch
    import paper_2211_16479_amd as msort
    for i in range(W):
        step(i)
    torch.cuda.synchronize()
    msort.ms_profile_reset()
    msort.ms_profile_select(classes)
    msort.ms_profile_enable(events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(W, W + K):
        step(i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    msort.ms_profile_enable(False)
    return (t1 - t0) * 1e3 / K, (read_kernels(K) if events else {})


def hbm_entry(kernel: str, bytes_per_launch: int, avg_us: float, workload: str = None, trace_name: str = None):
    achieved = bytes_per_launch / (avg_us * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": profiled_traffic(workload, trace_name) if workload and trace_name else None,
            "kernel": kernel, "bytes_per_launch": int(bytes_per_launch), "avg_us": round(avg_us, 2)}


MERGE4_TRACE = "merge4_kernel"


def plain_roofline(name, n, kb, vb, kernels):
    """The plain form's dominant kernel (the fused four-run merge, else the
    two-run merge) and the whole fused pass (its sampling partition, four-way
    partition and merge)."""
    per = n * (kb + vb) * 2      # read + write of every key and value per pass
    dom = max((k for k in ("merge", "merge4") if k in kernels), key=lambda k: kernels[k]["ms_per_step"],
              default=None)
    if dom is None:
        return None, None
    kname = "merge4_kernel" if dom == "merge4" else "merge_kernel"
    roof = hbm_entry(kname, per, kernels[dom]["avg_us"], name, kname)
    if roof["achieved"] > HBM_PEAK_GBS:
        # run detection skipped the passes (their kernels returned at once):
        # the bytes never moved, so there is no roofline to report
        return {"kernel": kname, "avg_us": roof["avg_us"], "skipped": True,
                "note": "merge passes skipped by run detection; no roofline"}, None
    fused = None
    if "merge4" in kernels and "partition4" in kernels and "partition_samples" in kernels:
        m4 = kernels["merge4"]
        if kernels["partition4"]["launches"] == m4["launches"] == kernels["partition_samples"]["launches"]:
            us = sum(kernels[k]["avg_us"] for k in ("partition_samples", "partition4", "merge4"))
            fused = hbm_entry("partition_kernel (samples) + partition4_kernel + merge4_kernel", per, us, name,
                              "fused_pass")
            fused["share_of_pass"] = {k: round(kernels[k]["avg_us"] / us, 3)
                                      for k in ("partition_samples", "partition4", "merge4")}
    return roof, fused


PLAIN_TIMED = ["tile_sort", "partition", "merge", "partition_samples", "partition4", "merge4"]


def plain_form(name, K, W, dev, events=True):
    """K timed plain sorts of fresh copies of workload `name`."""
    import torch
    import paper_2211_16479_amd as msort
    desc, n, kb, vb, kt = WORKLOADS[name]
    pk, pv = make_pristine(name, dev)
    sha = sha256_of(pk) if pv is None else sha256_of(pk, pv)
    bufs = [(pk.clone(), None if pv is None else pv.clone()) for _ in range(K + W)]
    torch.cuda.synchronize()

    def step(i):
        k, v = bufs[i]
        if v is None:
            msort.ms_sort(k)
        else:
            msort.ms_sort_pairs(k, v)

    ms, kernels = timed_steps(step, K, W, events, classes=PLAIN_TIMED)
    plan = msort.ms_plan_query(n, kt, vb)
    roof, fused = plain_roofline(name, n, kb, vb, kernels)
    out = {"workload": desc, "n": n, "key_bytes": kb, "value_bytes": vb, "ms_per_step": round(ms, 4),
           "Gkeys_s": round(n / (ms * 1e-3) / 1e9, 3),
           "whole_sort_hbm_GBs": round(n * (kb + vb) * 2 * (1 + plan["hbm_passes"]) / (ms * 1e-3) / 1e9, 1),
           "plan": plan, "input_sha256": sha, "kernels": kernels, "roofline": roof, "fused_pass": fused}
    result = bufs[W][0]           # sorted output of the first timed step
    del bufs
    return out, pk, pv, result


LEARNED_STAGES = {
    # profiler class: (kernels, trace name, algorithmic key transfers per key processed)
    # level 1: size estimate from a random sample (from 2^23 keys), else the
    # exact histogram
    "learned_estimate": ("ls_est1_kernel", "ls_est1_kernel", 1),      # read every sampled key
    "learned_hist": ("ls_hist1_kernel", "ls_hist1_kernel", 1),       # read every key
    "learned_scatter": ("ls_scatter1_kernel", "ls_scatter1_kernel", 2),  # read and write every key
    "learned_hist2": ("ls_hist2_kernel", "ls_hist2_kernel", 1),
    "learned_scatter2": ("ls_scatter2_kernel", "ls_scatter2_kernel", 2),
    # kept keys, read + write
    "bucket_sort": ("seg_init/classify/owner + seg_small_kernel per class", "bucket_sort", 2),
}


def est_sample_size(n):
    """Keys the learned form's level-1 size estimate reads: min(2^20, n / 128)
    as a power of two, at least 2^16."""
    s = 1 << 16
    while s < (1 << 20) and 2 * s * 128 <= n:
        s *= 2
    return s


def learned_form(K, W, dev, pristine, use_graph, workload="lognormal_u32_2p29"):
    """K timed learned-bucket sorts of fresh copies of `pristine` (the
    workload's keys; any of the four key types)."""
    import torch
    import paper_2211_16479_amd as msort
    n = pristine.numel()
    kb = pristine.element_size()
    kt = WORKLOADS[workload][4]
    bufs = [pristine.clone() for _ in range(K + W)]
    torch.cuda.synchronize()

    def step(i):
        msort.ms_sort_ex(bufs[i], key_type=kt, algo=msort.MS_ALGO_LEARNED_BUCKET, stats=False,
                         use_graph=1 if use_graph else 0)

    # only the stages priced below are bracketed by events (the training
    # steps and the small kernels would add an event pair per launch)
    ms, kernels = timed_steps(step, K, W, events=not use_graph, classes=list(LEARNED_STAGES))
    # device-side statistics of one more sort of the same input (untimed)
    extra = pristine.clone()
    _, st = msort.ms_sort_ex(extra, key_type=kt, algo=msort.MS_ALGO_LEARNED_BUCKET, use_graph=1 if use_graph else 0)
    torch.cuda.synchronize()
    kept = n - int(st["spilled"]) if not st["fallback_taken"] else 0
    stages = {}
    for cls, (kname, tname, transfers) in LEARNED_STAGES.items():
        if cls in kernels:
            keys = kept if cls == "bucket_sort" else est_sample_size(n) if cls == "learned_estimate" else n
            stages[cls] = hbm_entry(kname, transfers * kb * keys, kernels[cls]["avg_us"], workload, tname)
            stages[cls]["ms_per_step"] = kernels[cls]["ms_per_step"]
    dom = max(stages, key=lambda c: stages[c]["ms_per_step"], default=None)
    roof = None
    if dom:
        roof = dict(stages[dom])
        roof.pop("ms_per_step")
    out = {"ms_per_step": round(ms, 4), "Gkeys_s": round(n / (ms * 1e-3) / 1e9, 3), "graph_replay": bool(use_graph),
           "learned_stats": {k: (round(v, 8) if isinstance(v, float) else v) for k, v in st.items()},
           "kernels": kernels, "stages": stages, "dominant": dom}
    result = bufs[W]
    del bufs
    return out, roof, result, extra


def cpu_baselines(name, keys, vals, budget_s=25.0):
    """The CPU oracle on a bounded power-of-two prefix of the workload:
    with every host core (the oracle's threaded top levels; the paper's
    multiprocessing form) and with one core (its sequential form).  The
    prefix is the largest whose single-core sort is estimated to fit the
    budget (from a small calibration sort)."""
    import numpy as np
    import oracle
    kn = _host(keys)
    vn = None if vals is None else _host(vals)
    m = min(kn.size, 1 << 18)

    def run(s, threads):
        t0 = time.perf_counter()
        if vn is None:
            oracle.sort(kn[:s], threads=threads)
        else:
            oracle.sort_pairs(kn[:s], vn[:s], threads=threads)
        return time.perf_counter() - t0

    t_cal = run(m, 1)
    per_key_level = t_cal / (m * max(1, np.log2(m)))
    s = m
    while s * 2 <= kn.size and per_key_level * (2 * s) * np.log2(2 * s) < budget_s:
        s *= 2
    what = "pairs" if vn is not None else "keys"
    threads = oracle.host_threads()
    t_all = run(s, threads)
    t_one = run(s, 1)
    sample = f"first 2^{int(np.log2(s))} {what} of the workload"
    return {"value": round(s / t_all / 1e9, 5), "unit": "Gkeys/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample}, oracle merge sort with its top levels on {threads} threads, {t_all:.2f} s",
            "single_core": {"value": round(s / t_one / 1e9, 5), "unit": "Gkeys/s", "cores": 1,
                            "sample": f"{sample}, single-threaded oracle merge sort, {t_one:.2f} s"},
            "host": host_info()}


def copy_ceiling(dev, nbytes=1 << 31, reps=5):
    """torch's device-to-device copy of nbytes, event-timed: read + write
    bytes per second (a practical HBM ceiling next to the 8 TB/s peak)."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_copy": nbytes, "avg_us": round(ms * 1e3, 2),
            "GBs_read_plus_write": round(2 * nbytes / (ms * 1e-3) / 1e9, 1),
            "frac_of_peak": round(2 * nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def bench_segmented(args, dev):
    """One step = one ms_segmented_sort (one graph launch) of all 10,000
    arrays; a fresh copy of the keys per step."""
    import torch
    import paper_2211_16479_amd as msort
    import workloads
    desc = WORKLOADS["segments_u32_10000"][0]
    K, W = args.steps, args.warmup
    keys, off = workloads.segments_u32(10000, seed=0, device=dev)
    n = keys.numel()
    bufs = [keys.clone() for _ in range(K + W)]
    torch.cuda.synchronize()
    ms, _ = timed_steps(lambda i: msort.ms_segmented_sort(bufs[i], off, max_segment_len=1 << 18), K, W, False)
    shapes = {f"class{c}(<={bd})": "x".join(map(str, msort.ms_tuning_get(0, 0, c)))
              for c, (bd, _) in enumerate(msort.ms_seg_classes(0, 0))}
    print(json.dumps({
        "metric": METRIC, "value": round(n / (ms * 1e-3) / 1e9, 4), "unit": "Gkeys/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": desc, "n": n, "segments": off.numel() - 1, "class_shapes": shapes,
                   "input_sha256": sha256_of(keys, off)},
        "roofline": None, "cpu_baseline": None}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lognormal_u32_2p29", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra plain workloads (2^27 Zipf pairs, 2^27 uint32 keys)")
    ap.add_argument("--learned-graph", action="store_true",
                    help="time the learned form by graph replay (no per-kernel events, no roofline)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run torch's plain device copy of the workload's byte size 3 times "
                         "(reference dispatches for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the sharded design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

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
        return bench_segmented(args, dev)

    if args.workload != "lognormal_u32_2p29":
        # a plain workload on its own (the normal int64 keys also by the
        # learned-bucket form beside it, with a byte comparison)
        res, pk, pv, plain_out = plain_form(args.workload, K, W, dev)
        lrn = None
        if args.workload == "normal_i64_2p28":
            plain_out = plain_out.clone()
            lres, _, lout, lextra = learned_form(K, W, dev, pk, args.learned_graph, args.workload)
            lrn = dict(lres, speedup_vs_plain=round(res["ms_per_step"] / lres["ms_per_step"], 3),
                       outputs_identical=bool(torch.equal(lout, plain_out) and torch.equal(lextra, plain_out)))
            del lout, lextra
        del plain_out
        torch.cuda.empty_cache()
        cpu = None if args.no_cpu_baseline else cpu_baselines(args.workload, pk, pv)
        print(json.dumps({
            "metric": METRIC, "value": res["Gkeys_s"], "unit": "Gkeys/s", "n_gpus": 1, "steps": K, "warmup": W,
            "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "u32" if kb == 4 else "int64", "data": "synthetic",
            "config": {"workload": desc, "n": n, "key_bytes": kb, "value_bytes": vb,
                       "input_sha256": res["input_sha256"], "plan": res["plan"]},
            "roofline": res["roofline"], "cpu_baseline": cpu, "fused_pass": res["fused_pass"],
            "kernels": res["kernels"], "whole_sort_hbm_GBs": res["whole_sort_hbm_GBs"], "learned": lrn}))
        return

    # headline: the learned-bucket form on the lognormal mixture, plain beside it
    plain, pristine, _, plain_out = plain_form(args.workload, K, W, dev)
    plain_out = plain_out.clone()
    learned, roof, learned_out, extra_out = learned_form(K, W, dev, pristine, args.learned_graph, args.workload)
    identical = bool(torch.equal(learned_out.view(torch.int32), plain_out.view(torch.int32))) and \
        bool(torch.equal(extra_out.view(torch.int32), plain_out.view(torch.int32)))
    del learned_out, extra_out, plain_out
    torch.cuda.empty_cache()
    extras = {}
    if not args.no_extras:
        for name in ("uniform_u32_2p27", "zipf_pairs_u32_2p27"):
            r, _, _, _ = plain_form(name, max(3, K // 2), 2, dev)
            extras[name] = r
            torch.cuda.empty_cache()
    ceiling = copy_ceiling(dev)
    cpu = None if args.no_cpu_baseline else cpu_baselines(args.workload, pristine, None)
    print(json.dumps({
        "metric": METRIC,
        "value": learned["Gkeys_s"],
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": learned["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "form": "learned-bucket (headline) vs plain merge path",
                   "input_sha256": plain["input_sha256"]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "learned": learned,
        "plain": plain,
        "learned_vs_plain": {"speedup": round(plain["ms_per_step"] / learned["ms_per_step"], 3),
                             "outputs_identical": identical},
        "extra_workloads": extras,
        "copy_ceiling": ceiling,
        "paper_context": PAPER_CONTEXT,
    }))


if __name__ == "__main__":
    main()
