"""GPU parity of the learned-bucket form on (key, value) pairs
(ms_sort_pairs_ex): 32-bit keys packed with their input positions into
64-bit keys, sorted by the learned form, unpacked, values gathered.  Every
output is compared element by element with the CPU oracle's stable pair
sort (keys and values), including heavy ties, signed keys, 8-byte values,
the Zipf workload (which falls back), forced spill / repair and graph
replays on fresh buffers."""
import numpy as np
import pytest
import torch

import oracle
import paper_2211_16479_amd as msort
import workloads
from gpu_helpers import assert_equal_arrays

pytestmark = pytest.mark.gpu


def u32_dev(a: np.ndarray, dev) -> torch.Tensor:
    return torch.from_numpy(a.view(np.int32).copy()).to(dev).view(torch.uint32)


def host(t: torch.Tensor, dtype) -> np.ndarray:
    if t.dtype == torch.uint32:
        return t.cpu().view(torch.int32).numpy().view(dtype)
    return t.cpu().numpy().view(dtype)


def run(keys: np.ndarray, vals: np.ndarray, dev, **opt):
    k = u32_dev(keys, dev) if keys.dtype == np.uint32 else torch.from_numpy(keys.copy()).to(dev)
    v = torch.from_numpy(vals.view(np.int64 if vals.dtype.itemsize == 8 else np.int32).copy()).to(dev)
    k, v, st = msort.ms_sort_pairs_ex(k, v, algo=msort.MS_ALGO_LEARNED_BUCKET, **opt)
    return host(k, keys.dtype), host(v, vals.dtype), st


def check(keys, vals, dev, what, expect_learned=True, **opt):
    gk, gv, st = run(keys, vals, dev, **opt)
    ek, ev = oracle.sort_pairs(keys, vals)
    assert_equal_arrays(gk, ek, what + " keys")
    assert_equal_arrays(gv, ev, what + " values")
    if expect_learned:
        assert st["algo_used"] == msort.MS_ALGO_LEARNED_BUCKET and st["fallback_taken"] == 0, (what, st)
    return st


def mix_keys(n, seed):
    return workloads.lognormal_mix_u32(n, seed=seed).view(torch.int32).numpy().view(np.uint32).copy()


@pytest.mark.parametrize("use_graph", [1, 0])
def test_mixture_pairs_index_values(gpu, use_graph):
    n = (1 << 21) + 777
    keys = mix_keys(n, 1)
    vals = np.arange(n, dtype=np.uint32)
    st = check(keys, vals, gpu, "mixture pairs", use_graph=use_graph)
    assert st["spilled"] == 0


def test_ties_keep_input_order(gpu):
    """Each key about 64 times, values random: the values of equal keys must
    come out in input order."""
    n = 1 << 21
    keys = (workloads.randint_i64(n, seed=2).numpy() // 64).astype(np.uint32)
    vals = np.random.default_rng(3).integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    check(keys, vals, gpu, "ties")


def test_signed_keys_and_wide_values(gpu):
    n = 1 << 21
    keys = workloads.normal_i64(n, sigma=2.0 ** 28, seed=4).numpy().astype(np.int32)
    keys[::97] = keys[5]  # a run of equal keys spread over the input
    vals = np.random.default_rng(5).integers(0, 2 ** 63, size=n, dtype=np.int64).view(np.uint64)
    check(keys, vals, gpu, "int32 keys, 8-byte values")


def test_zipf_pairs_fall_back_exactly(gpu):
    """The Zipf workload: its most frequent key holds ~9% of the pairs, over
    any bucket's capacity and the spill threshold, so the plain sort runs."""
    k, v = workloads.zipf_pairs_u32(1 << 21, seed=6)
    keys = k.view(torch.int32).numpy().view(np.uint32).copy()
    vals = v.view(torch.int32).numpy().view(np.uint32).copy()
    st = check(keys, vals, gpu, "zipf pairs", expect_learned=False)
    # the five most frequent keys hold about 20% of the pairs, each over
    # twice a bucket's capacity: the sorted sample already decides
    assert st["fallback_taken"] == 1 and st["sample_fallback"] == 1, st


def test_spill_repair_keeps_stability(gpu):
    n = 1 << 21
    keys = (mix_keys(n, 7) // 16) * 16  # ties
    vals = np.arange(n, dtype=np.uint32)[::-1].copy()
    st = check(keys, vals, gpu, "spill", bucket_capacity=4096, bucket_fill=2048, spill_threshold=0.5,
               train_steps=0)
    assert st["repaired"] == 1 and st["spilled"] > 0


def test_fresh_buffers_one_graph(gpu):
    before = msort.ms_graph_captures()
    for rep in range(6):
        n = 1 << 20
        keys = mix_keys(n, 100 + rep)
        vals = np.random.default_rng(rep).integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
        check(keys, vals, gpu, f"call {rep}")
    assert msort.ms_graph_captures() - before == 1


def test_unsupported_and_plain_routes(gpu):
    k = torch.zeros(1 << 20, dtype=torch.int64, device=gpu)
    v = torch.zeros(1 << 20, dtype=torch.int32, device=gpu)
    with pytest.raises(msort.MSortError):
        msort.ms_sort_pairs_ex(k, v, algo=msort.MS_ALGO_LEARNED_BUCKET)
    # the plain route of the same entry point
    n = 100000
    keys = mix_keys(n, 8)
    vals = np.arange(n, dtype=np.uint32)
    kk, vv, st = msort.ms_sort_pairs_ex(u32_dev(keys, gpu), u32_dev(vals, gpu))
    ek, ev = oracle.sort_pairs(keys, vals)
    assert_equal_arrays(host(kk, np.uint32), ek, "plain route keys")
    assert_equal_arrays(host(vv, np.uint32), ev, "plain route values")
    assert st["algo_used"] == msort.MS_ALGO_MERGE_PATH


def test_full_mixture_pairs_2p27(gpu):
    """2^27 mixture pairs (value = index) at full size against the threaded
    oracle."""
    n = 1 << 27
    k = workloads.lognormal_mix_u32(n, seed=0, device=gpu)
    v = torch.arange(n, dtype=torch.int32, device=gpu).view(torch.uint32)
    kh, vh = host(k, np.uint32), host(v, np.uint32)
    k, v, st = msort.ms_sort_pairs_ex(k, v, algo=msort.MS_ALGO_LEARNED_BUCKET)
    assert st["fallback_taken"] == 0
    ek, ev = oracle.sort_pairs(kh, vh, threads=oracle.host_threads())
    assert_equal_arrays(host(k, np.uint32), ek, "2^27 keys")
    assert_equal_arrays(host(v, np.uint32), ev, "2^27 values")
