"""Shared helpers of the GPU parity tests (test infrastructure)."""
import numpy as np
import torch

import oracle

TORCH_OF = {np.dtype(np.uint32): torch.uint32, np.dtype(np.int32): torch.int32,
            np.dtype(np.uint64): torch.uint64, np.dtype(np.int64): torch.int64}


def to_dev(a: np.ndarray, dev) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def as_i64(t: torch.Tensor) -> torch.Tensor:
    """Order-preserving int64 view of a 32-bit key tensor (for torch ops)."""
    if t.dtype == torch.uint32:
        return t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    return t.to(torch.int64)


def first_mismatch(a: np.ndarray, b: np.ndarray):
    bad = np.flatnonzero(a != b)
    return None if bad.size == 0 else int(bad[0])


def assert_equal_arrays(got: np.ndarray, exp: np.ndarray, what: str):
    assert got.shape == exp.shape, f"{what}: shape {got.shape} vs {exp.shape}"
    i = first_mismatch(got, exp)
    assert i is None, f"{what}: first mismatch at {i}: got {got[i]} expected {exp[i]}"


def keys_fill(n: int, dtype, dist: str, rng: np.random.Generator) -> np.ndarray:
    info = np.iinfo(dtype)
    if dist == "uniform":
        return rng.integers(info.min, info.max, size=n, dtype=dtype, endpoint=True)
    if dist == "few":
        return rng.integers(0, 5, size=n).astype(dtype)
    if dist == "equal":
        return np.full(n, 7, dtype)
    if dist == "sorted":
        return np.sort(rng.integers(info.min, info.max, size=n, dtype=dtype, endpoint=True))
    if dist == "reverse":
        return np.sort(rng.integers(info.min, info.max, size=n, dtype=dtype, endpoint=True))[::-1].copy()
    if dist == "extremes":
        pool = np.array([info.min, info.max, 0, 1, info.max - 1, info.min + 1], dtype=dtype)
        return pool[rng.integers(0, pool.size, size=n)]
    raise ValueError(dist)


def check_sorted_permutation_pairs(in_k: torch.Tensor, out_k: torch.Tensor, out_v: torch.Tensor):
    """For values = original index: output is the unique stable sort iff keys
    are non-decreasing, values are a permutation of [0, n), every output key
    is the input key at its value's index, and values rise within equal keys."""
    n = in_k.numel()
    ok = as_i64(out_k)
    ov = as_i64(out_v)
    assert bool((ok[1:] >= ok[:-1]).all()), "keys not sorted"
    seen = torch.zeros(n, dtype=torch.bool, device=ov.device)
    assert int(ov.min()) >= 0 and int(ov.max()) < n
    seen[ov] = True
    assert bool(seen.all()), "values are not a permutation"
    assert bool((as_i64(in_k)[ov] == ok).all()), "a key did not travel with its value"
    same = ok[1:] == ok[:-1]
    assert bool((ov[1:][same] > ov[:-1][same]).all()), "equal keys lost their input order"


def check_sampled_ranks(in_np: np.ndarray, out_np: np.ndarray, samples: int, seed: int):
    """Oracle check of sampled positions: out[r] is correct at r exactly when
    #(keys < out[r]) <= r < #(keys <= out[r])."""
    rng = np.random.default_rng(seed)
    n = out_np.size
    r = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, size=samples)]))
    lt, le = oracle.rank_bounds(in_np, out_np[r])
    ok = (lt <= r) & (r < le)
    assert ok.all(), f"sampled rank check failed at positions {r[~ok][:5]}"
