"""GPU parity of the learned-bucket form on int32, uint64 and int64 keys: the
whole sort bit-exact against the CPU merge-sort oracle (keys only: the
sorted sequence is unique), on the normal int64 workload, heavy ties,
keys at the ends of the type's range, keys far from zero (the 64-bit
feature works on offsets from the sample's smallest key), nearly sorted
input, forced spill / repair and forced fallback, and one captured graph
replayed on fresh buffers."""
import numpy as np
import pytest
import torch

import oracle
import paper_2211_16479_amd as msort
import workloads
from gpu_helpers import assert_equal_arrays

pytestmark = pytest.mark.gpu

KT = {np.int32: msort.MS_KEY_I32, np.uint64: msort.MS_KEY_U64, np.int64: msort.MS_KEY_I64}


def to_dev(a: np.ndarray, dev) -> torch.Tensor:
    """Device tensor with the bytes of a (uint64 travels as int64)."""
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64).copy()).to(dev)
    return torch.from_numpy(a.copy()).to(dev)


def from_dev(t: torch.Tensor, dtype) -> np.ndarray:
    return t.cpu().numpy().view(dtype)


def learned(keys: np.ndarray, dev, **opt):
    t = to_dev(keys, dev)
    t, st = msort.ms_sort_ex(t, key_type=KT[keys.dtype.type], algo=msort.MS_ALGO_LEARNED_BUCKET, **opt)
    return from_dev(t, keys.dtype), st


def i64(t: torch.Tensor) -> np.ndarray:
    return t.numpy().astype(np.int64)


def check(keys: np.ndarray, dev, what: str, expect_learned: bool = True, **opt):
    got, st = learned(keys, dev, **opt)
    assert_equal_arrays(got, oracle.sort(keys), what)
    if expect_learned:
        assert st["algo_used"] == msort.MS_ALGO_LEARNED_BUCKET and st["fallback_taken"] == 0, (what, st)
        assert st["misordered"] == 0
    return st


@pytest.mark.parametrize("use_graph", [1, 0])
def test_normal_int64_exact(gpu, use_graph):
    """The normal int64 workload (sigma 2^40): nothing spills."""
    keys = i64(workloads.normal_i64((1 << 22) + 777, seed=1))
    st = check(keys, gpu, "normal int64", use_graph=use_graph)
    assert st["spilled"] == 0
    assert st["loss_final"] < st["loss_initial"]


@pytest.mark.parametrize("dist", ["randint_ties", "few", "equal", "extremes", "far_from_zero", "nearly_sorted",
                                  "uniform_u64", "sorted_desc"])
def test_int64_inputs_exact(gpu, dist):
    n = 1 << 20
    rng = np.random.default_rng(3)
    info = np.iinfo(np.int64)
    dtype = np.int64
    if dist == "randint_ties":
        keys = i64(workloads.randint_i64(n, seed=2)) // 64  # each value about 64 times
    elif dist == "few":
        keys = rng.integers(-3, 4, size=n).astype(np.int64)
    elif dist == "equal":
        keys = np.full(n, -5, np.int64)
    elif dist == "extremes":
        keys = i64(workloads.normal_i64(n, seed=4))
        pos = rng.integers(0, n, size=4096)
        keys[pos[:2048]] = info.min
        keys[pos[2048:]] = info.max
    elif dist == "far_from_zero":
        keys = (np.uint64(1) << np.uint64(63)) + np.abs(i64(workloads.normal_i64(n, seed=5))).astype(np.uint64)
        dtype = np.uint64
    elif dist == "nearly_sorted":
        keys = i64(workloads.nearly_sorted(torch.sort(workloads.normal_i64(n, seed=6)).values, 0.01, seed=6))
    elif dist == "uniform_u64":
        keys = workloads.raw64(n, 3, 7, 2).numpy().view(np.uint64)
        dtype = np.uint64
    else:
        keys = np.sort(i64(workloads.normal_i64(n, seed=8)))[::-1].copy()
    keys = keys.astype(dtype)
    check(keys, gpu, f"learned {dist}", expect_learned=False, spill_threshold=0.5)


@pytest.mark.parametrize("kt", ["u32", "i64"])
def test_ragged_sizes_take_the_learned_path(gpu, kt):
    """Sizes that end in a partial histogram chunk (any remainder modulo the
    8192-key chunk of 32-bit keys, 4096 of 64-bit keys) must still count
    every key once: the learned path is taken and the output is exact."""
    for r in (1, 777, 4095, 4097, 8191):
        n = (1 << 20) + r
        if kt == "u32":
            keys = workloads.lognormal_mix_u32(n, seed=r).view(torch.int32).numpy().view(np.uint32)
            t = torch.from_numpy(keys.view(np.int32).copy()).to(gpu).view(torch.uint32)
            t, st = msort.ms_sort_ex(t, algo=msort.MS_ALGO_LEARNED_BUCKET)
            got = t.cpu().view(torch.int32).numpy().view(np.uint32)
        else:
            keys = i64(workloads.normal_i64(n, seed=r))
            got, st = learned(keys, gpu)
        assert_equal_arrays(got, oracle.sort(keys), f"{kt} n = 2^20 + {r}")
        assert st["fallback_taken"] == 0 and st["algo_used"] == msort.MS_ALGO_LEARNED_BUCKET, (kt, r, st)


def test_int32_exact(gpu):
    """int32 keys (the unsigned image flips the sign bit): normal keys of
    both signs take the learned path; the mixture's uint32 keys reinterpreted
    as int32 (a spike of small positive keys inside a range spanning all
    int32) overflow the buckets of the offset feature and fall back, still
    exact; and heavy ties."""
    keys = (i64(workloads.normal_i64(1 << 21, sigma=2.0 ** 28, seed=9))).astype(np.int32)
    check(keys, gpu, "int32 normal")
    mix = workloads.lognormal_mix_u32(1 << 21, seed=9).view(torch.int32).numpy().copy()
    check(mix, gpu, "int32 mixture", expect_learned=False)
    few = np.random.default_rng(10).integers(-9, 9, size=1 << 20).astype(np.int32)
    check(few, gpu, "int32 few", expect_learned=False, spill_threshold=0.5)


def test_int64_spill_repair_and_fallback(gpu):
    keys = i64(workloads.normal_i64(1 << 21, seed=11))
    st = check(keys, gpu, "int64 spill", bucket_capacity=4096, bucket_fill=2048, spill_threshold=0.5,
               train_steps=0)
    assert st["repaired"] == 1 and st["spilled"] > 0
    got, st = learned(keys, gpu, force_fallback=1)
    assert_equal_arrays(got, oracle.sort(keys), "int64 forced fallback")
    assert st["fallback_taken"] == 1 and st["algo_used"] == msort.MS_ALGO_MERGE_PATH


def test_int64_fresh_buffers_replay_one_graph(gpu):
    before = msort.ms_graph_captures()
    for rep in range(8):
        keys = i64(workloads.normal_i64(1 << 20, seed=200 + rep))
        got, st = learned(keys, gpu)
        assert_equal_arrays(got, oracle.sort(keys), f"int64 call {rep}")
        assert st["fallback_taken"] == 0
    assert msort.ms_graph_captures() - before == 1


def test_full_normal_int64_2p28_learned_equals_oracle(gpu):
    """The normal int64 workload at 2^28 keys: the learned output equals the
    oracle's sort element by element (threaded oracle)."""
    k = workloads.normal_i64(1 << 28, seed=0, device=gpu)
    a = k.clone()
    _, st = msort.ms_sort_ex(a, algo=msort.MS_ALGO_LEARNED_BUCKET)
    torch.cuda.synchronize()
    assert st["fallback_taken"] == 0 and st["spilled"] == 0
    exp = oracle.sort(k.cpu().numpy(), threads=oracle.host_threads())
    assert_equal_arrays(a.cpu().numpy(), exp, "2^28 int64 learned")


def test_automatic_choice_by_key_width(gpu):
    """MS_ALGO_AUTO: 64-bit keys take the learned form from 2^26 keys, 32-bit
    keys from 2^27 (below, the plain sort); either way the output is the
    oracle's."""
    for n, expect in ((1 << 25, msort.MS_ALGO_MERGE_PATH), (1 << 26, msort.MS_ALGO_LEARNED_BUCKET)):
        k = workloads.normal_i64(n, seed=40, device=gpu)
        exp = oracle.sort(k.cpu().numpy(), threads=oracle.host_threads())
        _, st = msort.ms_sort_ex(k)
        torch.cuda.synchronize()
        assert st["algo_used"] == expect, (n, st)
        assert_equal_arrays(k.cpu().numpy(), exp, f"auto int64 n={n}")
        del k
    k = workloads.normal_i64(1 << 26, sigma=2.0 ** 28, seed=41, device=gpu).to(torch.int32)
    _, st = msort.ms_sort_ex(k)
    torch.cuda.synchronize()
    assert st["algo_used"] == msort.MS_ALGO_MERGE_PATH
