"""Run-adaptive merging (merge passes that would change nothing are
skipped, the result copied back when it ends in the scratch buffer) against
the CPU oracle, element by element, on inputs whose tree levels are all,
some or none already in order: sorted, the nearly sorted layout of
configuration 3 (disjoint adjacent swaps, which never cross a tile), swaps
that cross tile boundaries, a sorted array with its minimum moved to the
end, reversed, blocks that are each unordered but in order with each other
(only the low levels merge, so an odd number of passes can run), and
ascending blocks in descending order.  Keys only (u32, int64) and stable
pairs with ties."""
import numpy as np
import pytest
import torch

import oracle
import paper_2211_16479_amd as msort
from gpu_helpers import assert_equal_arrays, to_dev

pytestmark = pytest.mark.gpu


def layout(name: str, n: int, dtype, tile: int, rng) -> np.ndarray:
    info = np.iinfo(dtype)
    base = np.sort(rng.integers(info.min, info.max, size=n, dtype=dtype, endpoint=True))
    a = base.copy()
    if name == "sorted":
        return a
    if name == "adjacent_swaps_even":        # configuration 3's rule: pairs (2j, 2j+1)
        j = np.unique(rng.integers(0, n // 2, size=max(1, n // 100)))
        a[2 * j], a[2 * j + 1] = base[2 * j + 1], base[2 * j]
        return a
    if name == "adjacent_swaps_cross_tiles":  # pairs (t*tile - 1, t*tile): every tile boundary
        t = np.arange(1, (n - 1) // tile + 1) * tile
        a[t - 1], a[t] = base[t], base[t - 1]
        return a
    if name == "min_at_end":
        return np.concatenate([base[1:], base[:1]])
    if name == "reversed":
        return base[::-1].copy()
    if name.startswith("blocks_shuffled_"):    # blocks of w tiles, shuffled inside, in order overall
        w = int(name.rsplit("_", 1)[1]) * tile
        for b0 in range(0, n, w):
            seg = a[b0:b0 + w]
            a[b0:b0 + w] = seg[rng.permutation(seg.size)]
        return a
    if name == "descending_blocks":           # sorted tiles, tiles in descending order
        chunks = [a[i:i + tile] for i in range(0, n, tile)]
        return np.concatenate(chunks[::-1])
    raise ValueError(name)


LAYOUTS = ["sorted", "adjacent_swaps_even", "adjacent_swaps_cross_tiles", "min_at_end", "reversed",
           "blocks_shuffled_1", "blocks_shuffled_2", "blocks_shuffled_4", "descending_blocks"]


@pytest.mark.parametrize("form", ["u32", "i64", "u32_pairs", "i64_pairs8"])
def test_adaptive_layouts_vs_oracle(gpu, form):
    kdt, vdt, kt, vb = {"u32": (np.uint32, None, msort.MS_KEY_U32, 0),
                        "i64": (np.int64, None, msort.MS_KEY_I64, 0),
                        "u32_pairs": (np.uint32, np.uint32, msort.MS_KEY_U32, 4),
                        "i64_pairs8": (np.int64, np.uint64, msort.MS_KEY_I64, 8)}[form]
    rng = np.random.default_rng(31)
    tile = msort.ms_plan_query(1 << 20, kt, vb)["tile"]
    parities = set()
    for n in (64 * tile + 17, 32 * tile + 5):   # 65 runs (7 levels) and 33 runs (6 levels)
        p = msort.ms_plan_query(n, kt, vb)
        parities.add(p["passes"] % 2)
        for name in LAYOUTS:
            k = layout(name, n, kdt, tile, rng)
            print(f"{form} n={n} layout={name} passes={p['hbm_passes']}", flush=True)
            if vdt is None:
                t = to_dev(k, gpu)
                msort.ms_sort(t)
                torch.cuda.synchronize()
                assert_equal_arrays(t.cpu().numpy(), oracle.sort(k), f"{form} {name} n={n}")
            else:
                # ties across run boundaries: keys coarsened so equal keys straddle tiles
                k = (k // 7) if kdt == np.uint32 else (k >> 20)
                v = np.arange(n, dtype=vdt)
                tk, tv = to_dev(k, gpu), to_dev(v, gpu)
                msort.ms_sort_pairs(tk, tv)
                torch.cuda.synchronize()
                ek, ev = oracle.sort_pairs(k, v)
                assert_equal_arrays(tk.cpu().numpy(), ek, f"{form} {name} n={n} keys")
                assert_equal_arrays(tv.cpu().numpy(), ev, f"{form} {name} n={n} values")
    assert parities == {0, 1}


def test_adaptive_equal_keys_everywhere(gpu):
    """All keys equal: every level is in order (ties), every pass is skipped,
    values stay where they are."""
    n = 3 * (1 << 20) + 11
    k = np.full(n, 42, dtype=np.uint32)
    v = np.arange(n, dtype=np.uint32)[::-1].copy()
    tk, tv = to_dev(k, gpu), to_dev(v, gpu)
    msort.ms_sort_pairs(tk, tv)
    torch.cuda.synchronize()
    assert_equal_arrays(tv.cpu().numpy(), v, "values of equal keys")


@pytest.mark.parametrize("level", [7, 8, 9])
def test_adaptive_single_unordered_level(gpu, level):
    """int64 keys over more than 256 tiles (the run check pairs tiles inside
    groups of 256, then groups): a sorted array whose first two runs of
    2^level tiles are exchanged, so exactly one merge level is out of order
    and only the pass holding it runs (an odd number of passes: the result
    is copied back from the scratch buffer)."""
    rng = np.random.default_rng(40 + level)
    kt = msort.MS_KEY_I64
    tile = msort.ms_plan_query(1 << 20, kt, 0)["tile"]
    n = 1100 * tile + 7
    base = np.sort(rng.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64))
    w = (1 << level) * tile
    k = np.concatenate([base[w:2 * w], base[:w], base[2 * w:]])
    print(f"level={level} n={n} plan={msort.ms_plan_query(n, kt, 0)}", flush=True)
    t = to_dev(k, gpu)
    msort.ms_sort(t)
    torch.cuda.synchronize()
    assert_equal_arrays(t.cpu().numpy(), base, f"level {level} exchanged")
