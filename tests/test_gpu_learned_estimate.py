"""GPU parity of the learned form's estimated first level: each coarse
bucket's region in the first-level buffer is sized from a random sample of
the input, the scatter checks every reservation against its region, and the
exact count-then-scatter pass runs when a region proves too small
(stats.coarse_recounted).  Every output is compared element by element with
the CPU oracle: the three modes (exact only, estimate, estimate then forced
recount) on 32- and 64-bit keys and on pairs; inputs built so that the
estimate misses (every position the estimate samples holds the same key);
and one cached graph replayed on such an input, then on an ordinary one,
then on the first again (the flag that opens the exact pass starts clear on
every launch)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2211_16479_amd as msort
import workloads
from gpu_helpers import assert_equal_arrays

pytestmark = pytest.mark.gpu

KT = {np.uint32: msort.MS_KEY_U32, np.int32: msort.MS_KEY_I32, np.uint64: msort.MS_KEY_U64,
      np.int64: msort.MS_KEY_I64}
EST_FROM = 1 << 23  # the estimate is used from this many keys


def est_sample_size(n: int) -> int:
    """Keys the estimate samples: min(2^20, n / 128) as a power of two, at least 2^16."""
    s = 1 << 16
    while s < (1 << 20) and 2 * s * 128 <= n:
        s *= 2
    return s


def est_positions(n_log2: int, seed: int = 0) -> np.ndarray:
    """Input positions the estimate reads for n = 2^n_log2: draws 2^32 + i of
    the library's sampling generator (the splitmix64 finaliser of the Weyl
    point seed * g + (draw + 1) * h, top n_log2 bits).  Used only to build
    inputs on which the estimate misses; the test checks that it did."""
    i = np.arange(est_sample_size(1 << n_log2), dtype=np.uint64) + np.uint64(1 << 32)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) * np.uint64(0x9E3779B97F4A7C15) + (i + np.uint64(1)) * np.uint64(0xD1B54A32D192ED03)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return (z >> np.uint64(64 - n_log2)).astype(np.int64)


def to_dev(a: np.ndarray, dev) -> torch.Tensor:
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32).copy()).to(dev).view(torch.uint32)
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64).copy()).to(dev)
    return torch.from_numpy(a.copy()).to(dev)


def from_dev(t: torch.Tensor, dtype) -> np.ndarray:
    if t.dtype == torch.uint32:
        return t.cpu().view(torch.int32).numpy().view(dtype)
    return t.cpu().numpy().view(dtype)


def learned(keys: np.ndarray, dev, **opt):
    t = to_dev(keys, dev)
    t, st = msort.ms_sort_ex(t, key_type=KT[keys.dtype.type], algo=msort.MS_ALGO_LEARNED_BUCKET, **opt)
    return from_dev(t, keys.dtype), st


def inputs(name: str) -> np.ndarray:
    if name == "lognormal_u32":
        return workloads.lognormal_mix_u32((1 << 24) + 777, seed=11).view(torch.int32).numpy().view(np.uint32)
    if name == "normal_i64":
        return workloads.normal_i64(EST_FROM + 5, seed=12).numpy().astype(np.int64)
    if name == "uniform_u64":
        return np.random.default_rng(13).integers(0, 2 ** 64 - 1, size=EST_FROM, dtype=np.uint64, endpoint=True)
    if name == "randint_i32":
        return np.random.default_rng(14).integers(-2 ** 31, 2 ** 31 - 1, size=(1 << 24) + 3, dtype=np.int32)
    raise ValueError(name)


@pytest.mark.parametrize("name", ["lognormal_u32", "normal_i64", "uniform_u64", "randint_i32"])
def test_three_modes_equal_the_oracle(gpu, name):
    keys = inputs(name)
    exp = oracle.sort(keys, threads=oracle.host_threads())
    for mode, recount in ((0, 0), (1, 0), (2, 1)):
        got, st = learned(keys, gpu, coarse_estimate=mode)
        assert_equal_arrays(got, exp, f"{name} coarse_estimate={mode}")
        assert st["algo_used"] == msort.MS_ALGO_LEARNED_BUCKET and st["fallback_taken"] == 0, (name, mode, st)
        assert st["coarse_recounted"] == recount, (name, mode, st)


def missed_u32(n_log2: int, seed: int) -> np.ndarray:
    """Uniform uint32 keys, except that every position the estimate samples holds 7."""
    keys = np.random.default_rng(seed).integers(0, 2 ** 32, size=1 << n_log2, dtype=np.uint64).astype(np.uint32)
    keys[est_positions(n_log2)] = 7
    return keys


def test_estimate_miss_takes_the_exact_pass(gpu):
    keys = missed_u32(24, seed=21)
    got, st = learned(keys, gpu)
    assert st["coarse_recounted"] == 1, st
    assert st["algo_used"] == msort.MS_ALGO_LEARNED_BUCKET and st["fallback_taken"] == 0, st
    assert_equal_arrays(got, oracle.sort(keys, threads=oracle.host_threads()), "estimate miss, uint32")


def test_estimate_miss_int64(gpu):
    n_log2 = 23
    keys = np.random.default_rng(22).integers(-2 ** 63, 2 ** 63 - 1, size=1 << n_log2, dtype=np.int64)
    keys[est_positions(n_log2)] = -(2 ** 62)
    got, st = learned(keys, gpu)
    assert st["coarse_recounted"] == 1, st
    assert_equal_arrays(got, oracle.sort(keys, threads=oracle.host_threads()), "estimate miss, int64")


def test_graph_replays_miss_clean_miss(gpu):
    """One cached graph (same n and options): the flag set by a miss does
    not leak into the next launch."""
    miss = missed_u32(24, seed=23)
    clean = np.random.default_rng(24).integers(0, 2 ** 32, size=1 << 24, dtype=np.uint64).astype(np.uint32)
    for keys, recount, what in ((miss, 1, "miss"), (clean, 0, "clean"), (miss, 1, "miss again")):
        got, st = learned(keys, gpu, use_graph=1)
        assert st["coarse_recounted"] == recount, (what, st)
        assert_equal_arrays(got, oracle.sort(keys, threads=oracle.host_threads()), "graph replay, " + what)


def test_below_the_threshold_counts_exactly(gpu):
    """Under 2^23 keys only the exact pass runs, whatever the option."""
    keys = workloads.lognormal_mix_u32(EST_FROM - 1, seed=25).view(torch.int32).numpy().view(np.uint32)
    got, st = learned(keys, gpu, coarse_estimate=2)
    assert st["coarse_recounted"] == 0, st
    assert_equal_arrays(got, oracle.sort(keys, threads=oracle.host_threads()), "below the threshold")


@pytest.mark.parametrize("mode", [1, 2])
def test_pairs_with_the_estimate(gpu, mode):
    keys = workloads.lognormal_mix_u32(EST_FROM + 99, seed=26).view(torch.int32).numpy().view(np.uint32)
    vals = np.arange(keys.size, dtype=np.uint32)
    k, v, st = msort.ms_sort_pairs_ex(to_dev(keys, gpu), to_dev(vals, gpu), algo=msort.MS_ALGO_LEARNED_BUCKET,
                                      coarse_estimate=mode)
    ek, ev = oracle.sort_pairs(keys, vals, threads=oracle.host_threads())
    assert_equal_arrays(from_dev(k, np.uint32), ek, f"pairs keys, coarse_estimate={mode}")
    assert_equal_arrays(from_dev(v, np.uint32), ev, f"pairs values, coarse_estimate={mode}")
    assert st["coarse_recounted"] == (1 if mode == 2 else 0), st



@pytest.mark.parametrize("dist", ["equal", "two_values", "sorted", "reverse"])
def test_degenerate_inputs_with_the_estimate(gpu, dist):
    """All keys in one coarse bin, two bins, and inputs already in (reverse)
    order: every region bound still holds its bin's keys or the exact pass
    takes over; the output is the oracle's either way."""
    n = EST_FROM + 17
    rng = np.random.default_rng(31)
    if dist == "equal":
        keys = np.full(n, 123456789, np.uint32)
    elif dist == "two_values":
        keys = np.where(rng.random(n) < 0.3, 5, 4_000_000_000).astype(np.uint32)
    elif dist == "sorted":
        keys = np.sort(rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32))
    else:
        keys = np.sort(rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32))[::-1].copy()
    got, st = learned(keys, gpu)
    assert_equal_arrays(got, oracle.sort(keys, threads=oracle.host_threads()), "estimate, " + dist)
    assert st["misordered"] == 0, st


@pytest.mark.parametrize("n", [(1 << 22) + 5, EST_FROM + 5])
def test_keys_at_the_limits(gpu, n):
    """A tenth of the keys at the largest uint32 and a twentieth at 0 among
    the mixture: ties with the key the bucket sort pads its LDS runs with."""
    keys = workloads.lognormal_mix_u32(n, seed=41).view(torch.int32).numpy().view(np.uint32).copy()
    rng = np.random.default_rng(42)
    keys[rng.random(n) < 0.1] = np.uint32(0xFFFFFFFF)
    keys[rng.random(n) < 0.05] = np.uint32(0)
    got, st = learned(keys, gpu)
    assert_equal_arrays(got, oracle.sort(keys, threads=oracle.host_threads()), f"keys at the limits, n={n}")
    assert st["misordered"] == 0, st
