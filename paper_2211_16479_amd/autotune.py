"""Autotuner of the segmented sort's per-class shapes (run on the GPU).

For every (key type, value width) family and every small size class it
times ms_segmented_sort on synthetic segments whose lengths are log-uniform
inside that class, once per compiled (workgroup size, items per thread)
candidate, and keeps the fastest.  The table is written as text lines
"arch key_type value_bytes class wg ipt" that ms_tuning_load() applies.

    python -m paper_2211_16479_amd.autotune [--out PATH] [--keys-per-class N]

Timing: HIP events around each call on the current stream (the graph for a
candidate is captured on its first call, which is not timed); median of the
timed repetitions.  Keys are uniform unsigned (the signed family of the same
width takes the same shapes); families swept: 32-bit keys alone, with 4-byte
and with 8-byte values, and 64-bit keys alone (64-bit keys with values have a
single compiled shape per class).
"""
import argparse
import math
import os
import statistics
import sys

import torch

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import paper_2211_16479_amd as msort  # noqa: E402

FAMILIES = [("u32", msort.MS_KEY_U32, 0), ("u32", msort.MS_KEY_U32, 4), ("u32", msort.MS_KEY_U32, 8),
            ("u64", msort.MS_KEY_U64, 0)]
SIGNED = {msort.MS_KEY_U32: "i32", msort.MS_KEY_U64: "i64"}
KT_NAME = {msort.MS_KEY_U32: "u32", msort.MS_KEY_I32: "i32", msort.MS_KEY_U64: "u64", msort.MS_KEY_I64: "i64"}


def class_segments(lo: int, hi: int, total: int, gen: torch.Generator, dev):
    """Lengths log-uniform in [lo, hi] until about `total` keys; int64 offsets."""
    lens = []
    acc = 0
    while acc < total:
        u = torch.rand(4096, generator=gen, dtype=torch.float64)
        L = torch.floor(torch.exp(math.log(lo) + (math.log(hi + 1) - math.log(lo)) * u)).clamp_(lo, hi)
        L = L.to(torch.int64)
        lens.append(L)
        acc += int(L.sum())
    lens = torch.cat(lens)
    lens = lens[: int(torch.searchsorted(torch.cumsum(lens, 0), torch.tensor(total)).item()) + 1]
    off = torch.zeros(lens.numel() + 1, dtype=torch.int64)
    off[1:] = torch.cumsum(lens, 0)
    return off.to(dev), int(lens.max())


def time_call(fn, reps: int) -> float:
    s = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return statistics.median(times)


def tune(keys_per_class: int = 1 << 24, reps: int = 7, arch: str = None, verbose: bool = True):
    dev = torch.device("cuda:0")
    if arch is None:
        arch = torch.cuda.get_device_properties(dev).gcnArchName.split(":")[0]
    gen = torch.Generator().manual_seed(1234)
    lines = []
    for name, kt, vb in FAMILIES:
        classes = msort.ms_seg_classes(kt, vb)
        for c, (bound, shapes) in enumerate(classes):
            lo = 2 if c == 0 else classes[c - 1][0] + 1
            off, max_len = class_segments(lo, bound, keys_per_class, gen, dev)
            n = int(off[-1])
            if kt == msort.MS_KEY_U64:
                pristine = torch.randint(-2 ** 63, 2 ** 63 - 1, (n,), dtype=torch.int64, generator=gen).to(dev)
            else:
                base = torch.randint(0, 2 ** 32, (n,), dtype=torch.int64, generator=gen).to(dev)
                pristine = (base & 0xFFFFFFFF).to(torch.int32).view(torch.uint32)
            keys = torch.empty_like(pristine)
            vals = None
            if vb == 4:
                vals = torch.arange(n, dtype=torch.int32, device=dev).view(torch.uint32)
            elif vb == 8:
                vals = torch.arange(n, dtype=torch.int64, device=dev)
            best = None
            for wg, ipt in shapes:
                msort.ms_tuning_set(kt, vb, c, wg, ipt)

                def call():
                    keys.copy_(pristine)
                    msort.ms_segmented_sort(keys, off, vals, max_segment_len=max_len, key_type=kt)

                call()  # capture
                torch.cuda.synchronize()
                t_copy = time_call(lambda: keys.copy_(pristine), reps)
                t = time_call(call, reps) - t_copy
                if verbose:
                    print(f"{arch} {name} vb={vb} class {c} (<= {bound}) {wg}x{ipt}: {t:.3f} ms "
                          f"({n / t / 1e6:.2f} Gkeys/s, {off.numel() - 1} segments)", flush=True)
                if best is None or t < best[0]:
                    best = (t, wg, ipt)
            msort.ms_tuning_set(kt, vb, c, best[1], best[2])
            lines.append(f"{arch} {KT_NAME[kt]} {vb} {c} {best[1]} {best[2]}")
            # the same choice for the signed family of the same width
            lines.append(f"{arch} {SIGNED[kt]} {vb} {c} {best[1]} {best[2]}")
    return lines


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(msort.TUNING_DIR, "tuning.txt"))
    ap.add_argument("--keys-per-class", type=int, default=1 << 24)
    ap.add_argument("--reps", type=int, default=7)
    args = ap.parse_args()
    lines = tune(args.keys_per_class, args.reps)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    header = ["# segmented-sort shapes chosen by paper_2211_16479_amd.autotune",
              "# arch key_type value_bytes class wg ipt"]
    with open(args.out, "w") as f:
        f.write("\n".join(header + lines) + "\n")
    print(f"wrote {args.out}")


if __name__ == "__main__":
    main()
