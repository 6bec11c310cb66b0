"""The GPU counterpart of the paper's single-processor scaling study (section
"Analysis of Single Processor Sorting": time against worker count, speedup
and efficiency; and the leaf cutoff of the hybrid sort in "Sequential Merge
Sort").

    python -m paper_2211_16479_amd.scaling --sizes      # time against n
    python -m paper_2211_16479_amd.scaling --workers    # time against CUs
    python -m paper_2211_16479_amd.scaling --build-tile-variants   # CPU, once
    python -m paper_2211_16479_amd.scaling --tiles      # time against tile size

* sizes: n = 10^2 .. 10^7 and 2^24 .. 2^29 uniform uint32 keys: the plain
  merge path, the learned-bucket form (n >= 2^22), and the CPU oracle with
  one thread and with every host thread (n <= 10^7), as the paper's
  sequential and multiprocessing rows.
* workers: the paper's workers are processes; here they are workgroups.
  The plain sort of 2^24 keys runs with every launch capped at 1, 2, 4, ...
  65536 workgroups (ms_options.max_workgroups: each workgroup loops over
  tiles, as each worker process loops over its chunks); speedup =
  T(1) / T(p), efficiency = speedup / p.
* tiles: the paper's hybrid sort hands arrays below a cutoff to insertion
  sort; here arrays up to one tile are sorted inside one workgroup.  Library
  builds with 1024-thread tiles of 4, 8, 16 and 32 keys per thread
  (4096 .. 32768 keys) sort 2^24 and 2^27 keys; tile-sort and merge times.

Every timing is the mean of `--reps` event-timed sorts of fresh copies of
the input after one warm-up sort.  Prints one JSON object.
"""
import argparse
import json
import os
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TILE_VARIANTS = {4: "MS_BS_IPT_K=4", 8: "MS_BS_IPT_K=8", 16: "MS_BS_IPT_K=16", 32: "MS_BS_IPT_K=32"}
VARIANT_DIR = os.path.join(PKG, "_tile_variants")


def _timed(fn, make, reps, stream=None):
    """Mean ms of fn(x) over `reps` fresh inputs x = make(), event-timed on
    `stream` (default: the current stream)."""
    import torch
    s = stream or torch.cuda.current_stream()
    x = make()
    fn(x)
    torch.cuda.synchronize()
    xs = [make() for _ in range(reps)]
    torch.cuda.synchronize()
    total = 0.0
    for x in xs:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn(x)
        b.record(s)
        torch.cuda.synchronize()
        total += a.elapsed_time(b)
    return total / reps


def study_sizes(reps):
    import numpy as np
    import torch
    import oracle
    import paper_2211_16479_amd as msort
    import workloads
    dev = torch.device("cuda:0")
    rows = []
    sizes = [10 ** e for e in range(2, 8)] + [1 << e for e in range(24, 30)]
    for n in sizes:
        base = workloads.uniform_u32(n, seed=0, device=dev)
        row = {"n": n}
        row["plain_ms"] = round(_timed(msort.ms_sort, base.clone, reps), 4)
        if n >= 1 << 22:
            row["learned_ms"] = round(_timed(lambda t: msort.ms_sort_ex(t, algo=msort.MS_ALGO_LEARNED_BUCKET,
                                                                        stats=False), base.clone, reps), 4)
        if n <= 10 ** 7:
            h = base.cpu().view(torch.int32).numpy().view(np.uint32)
            for name, threads in (("oracle_1_thread_ms", 1), ("oracle_all_threads_ms", oracle.host_threads())):
                t0 = time.perf_counter()
                oracle.sort(h, threads=threads)
                row[name] = round((time.perf_counter() - t0) * 1e3, 3)
        row["plain_Gkeys_s"] = round(n / (row["plain_ms"] * 1e-3) / 1e9, 4)
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
        del base
        torch.cuda.empty_cache()
    return {"sizes": rows, "oracle_threads": oracle.host_threads()}


def study_workers(reps, n=1 << 24):
    import torch
    import paper_2211_16479_amd as msort
    import workloads
    dev = torch.device("cuda:0")
    base = workloads.uniform_u32(n, seed=0, device=dev)
    rows = []
    for w in [1 << e for e in range(0, 17, 1)]:
        ms = _timed(lambda t: msort.ms_sort_ex(t, algo=msort.MS_ALGO_MERGE_PATH, stats=False, max_workgroups=w),
                    base.clone, reps)
        rows.append({"workgroups": w, "ms": round(ms, 4)})
        print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    t1 = rows[0]["ms"]
    for r in rows:
        r["speedup"] = round(t1 / r["ms"], 3)
        r["efficiency"] = round(t1 / r["ms"] / r["workgroups"], 5)
    full = _timed(msort.ms_sort, base.clone, reps)
    return {"workers": rows, "n": n, "uncapped_ms": round(full, 4),
            "device_cus": torch.cuda.get_device_properties(dev).multi_processor_count}


def build_tile_variants():
    """Compile one library per tile size (CPU; hipcc cross-compiles)."""
    from paper_2211_16479_amd import build as b
    os.makedirs(VARIANT_DIR, exist_ok=True)
    for ipt, define in TILE_VARIANTS.items():
        lib = os.path.join(VARIANT_DIR, f"libmsort_ipt{ipt}.so")
        b.build(lib=lib, build_dir=os.path.join(VARIANT_DIR, f"obj_ipt{ipt}"), defines=(define,))
        print(lib)


def study_tiles(reps):
    """Time against tile size: each variant library in a child process (a
    library is loaded once per process)."""
    import subprocess
    rows = []
    for ipt in TILE_VARIANTS:
        lib = os.path.join(VARIANT_DIR, f"libmsort_ipt{ipt}.so")
        if not os.path.exists(lib):
            raise SystemExit(f"{lib} is missing: run --build-tile-variants first")
        r = subprocess.run([sys.executable, "-m", "paper_2211_16479_amd.scaling", "--tile-child", lib,
                            "--reps", str(reps)], capture_output=True, text=True, cwd=ROOT)
        if r.returncode != 0:
            raise SystemExit(r.stderr)
        row = json.loads(r.stdout.strip().splitlines()[-1])
        row["keys_per_thread"] = ipt
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    return {"tiles": rows}


def tile_child(lib, reps):
    import torch
    import paper_2211_16479_amd as msort
    import workloads
    msort.LIB_PATH = lib
    dev = torch.device("cuda:0")
    out = {}
    for n in (1 << 24, 1 << 27):
        base = workloads.uniform_u32(n, seed=0, device=dev)
        plan = msort.ms_plan_query(n, msort.MS_KEY_U32)
        ms = _timed(msort.ms_sort, base.clone, reps)
        msort.ms_profile_reset()
        msort.ms_profile_enable(True)
        x = base.clone()
        msort.ms_sort(x)
        torch.cuda.synchronize()
        msort.ms_profile_enable(False)
        tile_ms = msort.ms_profile_read("tile_sort")[1]
        out[str(n)] = {"tile": plan["tile"], "hbm_passes": plan["hbm_passes"], "ms": round(ms, 4),
                       "tile_sort_ms": round(tile_ms, 4), "merge_ms": round(ms - tile_ms, 4)}
        del base, x
        torch.cuda.empty_cache()
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", action="store_true")
    ap.add_argument("--workers", action="store_true")
    ap.add_argument("--tiles", action="store_true")
    ap.add_argument("--build-tile-variants", action="store_true")
    ap.add_argument("--tile-child", default=None)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    if a.build_tile_variants:
        return build_tile_variants()
    if a.tile_child:
        return tile_child(a.tile_child, a.reps)
    out = {}
    if a.sizes:
        out.update(study_sizes(a.reps))
    if a.workers:
        out.update(study_workers(a.reps))
    if a.tiles:
        out.update(study_tiles(a.reps))
    print(json.dumps(out))


if __name__ == "__main__":
    main()
