"""GPU parity of the plain merge sort (ms_sort, ms_sort_pairs) against the CPU
oracle, element by element; full-size configurations via properties that
determine the unique result plus oracle-sampled positions."""
import numpy as np
import pytest
import torch

import oracle
import paper_2211_16479_amd as msort
import workloads
from gpu_helpers import assert_equal_arrays, check_sorted_permutation_pairs, keys_fill, to_dev

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 2, 3, 63, 64, 65, 1000, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193,
         12289, 65537, 131071, 300_007, 1_000_003]
DTYPES = [np.uint32, np.int32, np.uint64, np.int64]


def gpu_sort(a: np.ndarray, dev) -> np.ndarray:
    t = to_dev(a, dev)
    msort.ms_sort(t)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gpu_sort_pairs(k: np.ndarray, v: np.ndarray, dev):
    tk, tv = to_dev(k, dev), to_dev(v, dev)
    msort.ms_sort_pairs(tk, tv)
    torch.cuda.synchronize()
    return tk.cpu().numpy(), tv.cpu().numpy()


@pytest.mark.parametrize("dtype", DTYPES, ids=lambda d: np.dtype(d).name)
def test_sort_sizes_uniform(gpu, dtype):
    rng = np.random.default_rng(11)
    for n in SIZES:
        a = keys_fill(n, dtype, "uniform", rng)
        assert_equal_arrays(gpu_sort(a, gpu), oracle.sort(a), f"{np.dtype(dtype).name} n={n}")


@pytest.mark.parametrize("dist", ["few", "equal", "sorted", "reverse", "extremes"])
@pytest.mark.parametrize("dtype", DTYPES, ids=lambda d: np.dtype(d).name)
def test_sort_distributions(gpu, dtype, dist):
    rng = np.random.default_rng(12)
    for n in (4097, 70_001):
        a = keys_fill(n, dtype, dist, rng)
        assert_equal_arrays(gpu_sort(a, gpu), oracle.sort(a), f"{dist} n={n}")


@pytest.mark.parametrize("kdt,vdt", [(np.uint32, np.uint32), (np.int32, np.uint32), (np.uint32, np.uint64),
                                     (np.int64, np.uint32), (np.uint64, np.uint64), (np.int64, np.uint64)],
                         ids=lambda d: np.dtype(d).name)
def test_pairs_stable_with_ties(gpu, kdt, vdt):
    rng = np.random.default_rng(13)
    for n in (0, 1, 5, 4096, 4097, 9000, 100_003):
        for dist in ("few", "uniform", "equal"):
            k = keys_fill(n, kdt, dist, rng)
            v = np.arange(n, dtype=vdt) * 3 + 1
            gk, gv = gpu_sort_pairs(k, v, gpu)
            ek, ev = oracle.sort_pairs(k, v)
            assert_equal_arrays(gk, ek, f"pairs keys {dist} n={n}")
            assert_equal_arrays(gv, ev, f"pairs vals {dist} n={n}")


def test_config_uniform_u32_2p20_seed0(gpu):
    keys = workloads.uniform_u32(1 << 20, seed=0).numpy()
    assert_equal_arrays(gpu_sort(keys, gpu), oracle.sort(keys), "2^20 uniform u32")


def test_zipf_pairs_reduced(gpu):
    k, v = workloads.zipf_pairs_u32(1 << 22, seed=0)
    gk, gv = gpu_sort_pairs(k.numpy(), v.numpy(), gpu)
    ek, ev = oracle.sort_pairs(k.numpy(), v.numpy())
    assert_equal_arrays(gk, ek, "zipf keys")
    assert_equal_arrays(gv, ev, "zipf vals")


def test_normal_i64_and_nearly_sorted_reduced(gpu):
    a = workloads.normal_i64(1 << 22, seed=0)
    b = workloads.nearly_sorted(torch.sort(a).values, 0.01, seed=0)
    ga, gb = gpu_sort(a.numpy(), gpu), gpu_sort(b.numpy(), gpu)
    ea = oracle.sort(a.numpy())
    assert_equal_arrays(ga, ea, "normal i64")
    assert_equal_arrays(gb, ea, "nearly sorted i64 (same multiset)")


def test_repeat_runs_identical(gpu):
    k, v = workloads.zipf_pairs_u32(1 << 21, seed=3, distinct=5000)
    outs = []
    for _ in range(3):
        tk, tv = k.to(gpu), v.to(gpu)
        msort.ms_sort_pairs(tk, tv)
        torch.cuda.synchronize()
        outs.append((tk.cpu().numpy(), tv.cpu().numpy()))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def _np(t: torch.Tensor) -> np.ndarray:
    """Host copy of a device tensor (uint32 through an int32 view)."""
    if t.dtype == torch.uint32:
        return t.cpu().view(torch.int32).numpy().view(np.uint32)
    return t.cpu().numpy()


def test_full_zipf_pairs_2p27(gpu):
    """Configuration 2 at full size in the benchmark's launch configuration:
    2^27 Zipf(1.1) pairs, value = original index; keys and values equal the
    oracle's stable sort element by element (threaded oracle, same output as
    the single-thread one)."""
    k, v = workloads.zipf_pairs_u32(1 << 27, seed=0, device=gpu)
    ok, ov = k.clone(), v.clone()
    msort.ms_sort_pairs(ok, ov)
    torch.cuda.synchronize()
    check_sorted_permutation_pairs(k, ok, ov)
    ek, ev = oracle.sort_pairs(_np(k), _np(v), threads=oracle.host_threads())
    assert_equal_arrays(_np(ok), ek, "2^27 zipf keys")
    assert_equal_arrays(_np(ov), ev, "2^27 zipf values")


def test_full_normal_i64_2p28_both_arrays(gpu):
    """Configuration 3 at full size: both 2^28 int64 arrays (random, and the
    sorted array with 1% adjacent swaps) equal the oracle's sort of the
    random array element by element (the two are the same multiset)."""
    a = workloads.normal_i64(1 << 28, seed=0, device=gpu)
    oa = a.clone()
    msort.ms_sort(oa)
    torch.cuda.synchronize()
    exp = oracle.sort(_np(a), threads=oracle.host_threads())
    assert_equal_arrays(_np(oa), exp, "2^28 normal int64")
    b = workloads.nearly_sorted(oa, 0.01, seed=0)   # sorted order, then the swaps
    del a, oa
    ob = b.clone()
    msort.ms_sort(ob)
    torch.cuda.synchronize()
    assert_equal_arrays(_np(ob), exp, "2^28 nearly sorted int64")


def test_full_uniform_u32_2p27_keys(gpu):
    """2^27 uint32 keys only (the merge-pass bandwidth workload) against the
    oracle element by element."""
    a = workloads.uniform_u32(1 << 27, seed=0, device=gpu)
    o = a.clone()
    msort.ms_sort(o)
    torch.cuda.synchronize()
    assert_equal_arrays(_np(o), oracle.sort(_np(a), threads=oracle.host_threads()), "2^27 uniform u32")


# Lanes per partition search (the library's rule, restated): the largest G of
# 64, 16, 4, 1 with searches * G <= 2^16.
def search_group(searches: int) -> int:
    for g in (64, 16, 4):
        if searches * g <= 1 << 16:
            return g
    return 1


def partition_groups(n: int, kt: int, vb: int) -> dict:
    """{"two_run": G or None, "fused": G or None}: the lane-group size of the
    two-run pass's partition (only when the level count is odd) and of the
    fused passes' partition and four-way partition."""
    p = msort.ms_plan_query(n, kt, vb)
    ceil = lambda a, b: -(-a // b)
    two = search_group(ceil(n, p["merge_tile"])) if p["passes"] % 2 else None
    fused = search_group(ceil(n, p["merge4_tile"])) if p["passes"] >= 2 else None
    return {"two_run": two, "fused": fused}


GROUP_SIZES = [3 * (1 << 20) + 7, (1 << 22) + 3, (1 << 23) + 5, (1 << 24) + 1, (1 << 25) + 3, (1 << 26) + 777]


@pytest.mark.parametrize("form", ["u32", "u32_pairs", "i64"])
def test_partition_group_sizes_vs_oracle(gpu, form):
    """Sizes 3*2^20 .. 2^26 + 777, chosen so that both partition kernels run
    with every lane-group size G = 16, 4 and 1 (and the two-run pass with
    G = 16, 4, 1), each compared with the oracle element by element.  Keys:
    uniform u32; Zipf pairs with value = index (ties, stability); int64 keys
    alternating the normal workload and the paper's uniform [0, n) integers
    (many ties)."""
    kt, vb = {"u32": (msort.MS_KEY_U32, 0), "u32_pairs": (msort.MS_KEY_U32, 4), "i64": (msort.MS_KEY_I64, 0)}[form]
    seen = {"two_run": set(), "fused": set()}
    for i, n in enumerate(GROUP_SIZES):
        g = partition_groups(n, kt, vb)
        for w in seen:
            if g[w] is not None:
                seen[w].add(g[w])
        print(f"{form} n={n} groups={g}", flush=True)
        if form == "u32":
            k = workloads.uniform_u32(n, seed=40 + i, device=gpu)
            o = k.clone()
            msort.ms_sort(o)
            torch.cuda.synchronize()
            assert_equal_arrays(_np(o), oracle.sort(_np(k), threads=oracle.host_threads()), f"u32 n={n}")
        elif form == "u32_pairs":
            k, v = workloads.zipf_pairs_u32(n, seed=40 + i, distinct=1 << 16, device=gpu)
            ok, ov = k.clone(), v.clone()
            msort.ms_sort_pairs(ok, ov)
            torch.cuda.synchronize()
            ek, ev = oracle.sort_pairs(_np(k), _np(v), threads=oracle.host_threads())
            assert_equal_arrays(_np(ok), ek, f"pair keys n={n}")
            assert_equal_arrays(_np(ov), ev, f"pair values n={n}")
        else:
            k = (workloads.normal_i64(n, seed=40 + i, device=gpu) if i % 2 else
                 workloads.randint_i64(n, seed=40 + i, device=gpu))
            o = k.clone()
            msort.ms_sort(o)
            torch.cuda.synchronize()
            assert_equal_arrays(_np(o), oracle.sort(_np(k), threads=oracle.host_threads()), f"i64 n={n}")
    assert {16, 4, 1} <= seen["fused"], seen
    assert {16, 4, 1} <= seen["two_run"], seen


def test_randint_i64_paper_workload(gpu):
    """The paper's MPI workload (int64 uniform in [0, n)), keys only and as
    pairs with value = index, against the oracle."""
    n = 3_000_017
    k = workloads.randint_i64(n, seed=9)
    assert_equal_arrays(gpu_sort(k.numpy(), gpu), oracle.sort(k.numpy()), "randint keys")
    v = np.arange(n, dtype=np.uint32)
    gk, gv = gpu_sort_pairs(k.numpy(), v, gpu)
    ek, ev = oracle.sort_pairs(k.numpy(), v)
    assert_equal_arrays(gk, ek, "randint pair keys")
    assert_equal_arrays(gv, ev, "randint pair values")


@pytest.mark.parametrize("kdt,vdt", [(np.uint32, None), (np.uint32, np.uint32), (np.int64, None)],
                         ids=["u32", "u32_pairs", "i64"])
def test_fused_pass_run_counts(gpu, kdt, vdt):
    """Run counts m after the tile sort that exercise every shape of the
    fused four-run passes: full quads, a last quad of 1, 2 or 3 runs, a short
    last run, an odd level count (one two-run pass first) and an even one."""
    kt = {np.dtype(np.uint32): msort.MS_KEY_U32, np.dtype(np.int64): msort.MS_KEY_I64}[np.dtype(kdt)]
    T = msort.ms_plan_query(1 << 20, kt, 0 if vdt is None else 4)["tile"]
    rng = np.random.default_rng(31)
    for m in (2, 3, 4, 5, 6, 7, 8, 9, 16, 17):
        for delta in (0, 1, T // 2):
            n = T * (m - 1) + (delta if delta else T)
            k = keys_fill(n, kdt, "few" if m % 2 else "uniform", rng)
            if vdt is None:
                assert_equal_arrays(gpu_sort(k, gpu), oracle.sort(k), f"m={m} n={n}")
            else:
                v = np.arange(n, dtype=vdt)
                gk, gv = gpu_sort_pairs(k, v, gpu)
                ek, ev = oracle.sort_pairs(k, v)
                assert_equal_arrays(gk, ek, f"keys m={m} n={n}")
                assert_equal_arrays(gv, ev, f"values m={m} n={n}")



def test_workgroup_cap_same_result(gpu):
    """The scaling study's worker count: every launch capped at 1, 3, 64
    workgroups (each looping over tiles) gives the oracle's sort, for u32
    and int64 keys with a ragged last tile."""
    rng = np.random.default_rng(51)
    for dtype in (np.uint32, np.int64):
        k = keys_fill(300_007, dtype, "uniform", rng)
        exp = oracle.sort(k)
        for cap in (1, 3, 64):
            t = to_dev(k, gpu)
            msort.ms_sort_ex(t, algo=msort.MS_ALGO_MERGE_PATH, stats=False, max_workgroups=cap)
            torch.cuda.synchronize()
            assert_equal_arrays(t.cpu().numpy(), exp, f"{np.dtype(dtype).name} cap {cap}")


def test_small_repeated_sorts_replay_a_graph(gpu):
    """Keys-only sorts of at most 2^22 keys replay a cached graph from the
    second call with the same size on a stream (the caller's buffer bound
    per launch): fresh buffers every call, one capture per size, every
    output equal to the oracle's."""
    import workloads
    for n in (1 << 20, (1 << 20) + 777):
        before = msort.ms_graph_captures()
        for rep in range(4):
            k = workloads.uniform_u32(n, seed=300 + rep, device=gpu)
            exp = oracle.sort(k.cpu().view(torch.int32).numpy().view(np.uint32))
            msort.ms_sort(k)
            torch.cuda.synchronize()
            assert_equal_arrays(k.cpu().view(torch.int32).numpy().view(np.uint32), exp, f"n={n} call {rep}")
        assert msort.ms_graph_captures() - before == 1, n
