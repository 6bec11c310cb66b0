"""Seeded synthetic inputs for the sort, shared by the tests, the smoke check
and the benchmark.  This module holds no sorting arithmetic: it only draws
keys.  It imports neither the CPU oracle nor the GPU library.

Every random number comes from a counter-based generator (splitmix64 applied
to ``stream_base + i``), written with torch int64 ops so the same code runs on
the CPU (tests) and on the GPU (full-size runs); integer draws are identical
on both, float transforms may differ in the last ulp between the two, which
is harmless because both sides of a parity check consume the same bytes.

Workloads (all seed 0 unless a caller says otherwise):
  uniform_u32      n uint32 keys uniform in [0, 2^32)
  zipf_pairs_u32   n uint32 keys, truncated Zipf(s) over `distinct` ranks,
                   each rank mapped to a distinct uint32 by a seeded 32-bit
                   bijection; values = original index (uint32)
  normal_i64       n int64 keys round(sigma * N(0, 1)), sigma = 2^40
  nearly_sorted    the sorted normal_i64 array with 1% disjoint adjacent swaps
  segments_u32     `num` segment lengths floor(2^(4 + 14u)) clamped to
                   [16, 2^18], CSR int64 offsets, uniform uint32 keys
  lognormal_mix_u32  n uint32 keys from an equal-weight mixture of 8
                   lognormals, mu ~ U(0, 4), sigma ~ U(0.1, 1), scaled so the
                   largest component's mu + 4 sigma point maps to 2^32 - 1
  randint_i64      n int64 keys uniform in [0, n) (the paper's MPI workload)
"""
import math

import torch

_M64 = (1 << 64) - 1


def _s64(v: int) -> int:
    """Python int -> the int64 with the same low 64 bits."""
    v &= _M64
    return v - (1 << 64) if v >= (1 << 63) else v


_GOLD = _s64(0x9E3779B97F4A7C15)
_C1 = _s64(0xBF58476D1CE4E5B9)
_C2 = _s64(0x94D049BB133111EB)


def _lsr(x: torch.Tensor, s: int) -> torch.Tensor:
    return (x >> s) & ((1 << (64 - s)) - 1)


def splitmix64(x: torch.Tensor) -> torch.Tensor:
    """splitmix64 finaliser (Steele, Lea, Flood 2014) on int64 bit patterns."""
    z = x + _GOLD
    z = (z ^ _lsr(z, 30)) * _C1
    z = (z ^ _lsr(z, 27)) * _C2
    return z ^ _lsr(z, 31)


def _splitmix_int(v: int) -> int:
    z = (v + 0x9E3779B97F4A7C15) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def stream_base(workload: int, seed: int, stream: int) -> int:
    return _s64(_splitmix_int((workload << 40) ^ (seed << 8) ^ stream))


def raw64(n: int, workload: int, seed: int, stream: int, device="cpu") -> torch.Tensor:
    i = torch.arange(n, dtype=torch.int64, device=device)
    return splitmix64(i + stream_base(workload, seed, stream))


def uniform_f64(n, workload, seed, stream, device="cpu") -> torch.Tensor:
    """Doubles uniform in [0, 1) from the top 53 bits."""
    return _lsr(raw64(n, workload, seed, stream, device), 11).to(torch.float64) * (2.0 ** -53)


def to_u32(x64: torch.Tensor) -> torch.Tensor:
    """Low 32 bits of an int64 tensor as a torch.uint32 tensor (same bits)."""
    lo = x64 & 0xFFFFFFFF
    return torch.where(lo >= (1 << 31), lo - (1 << 32), lo).to(torch.int32).view(torch.uint32)


def u32_as_i64(x: torch.Tensor) -> torch.Tensor:
    return x.view(torch.int32).to(torch.int64) & 0xFFFFFFFF


def _mix32(x: torch.Tensor) -> torch.Tensor:
    """A bijection of 32-bit values (xorshift-multiply finaliser), on int64."""
    m = 0xFFFFFFFF
    x = x & m
    x = x ^ (x >> 16)
    x = (x * 0x7FEB352D) & m
    x = x ^ (x >> 15)
    x = (x * 0x846CA68B) & m
    return x ^ (x >> 16)


def _normal(n, workload, seed, s1, s2, device):
    """Box-Muller standard normals from two independent uniform streams."""
    u1 = uniform_f64(n, workload, seed, s1, device)
    u2 = uniform_f64(n, workload, seed, s2, device)
    return torch.sqrt(-2.0 * torch.log1p(-u1)) * torch.cos((2.0 * math.pi) * u2)


# ---------------------------------------------------------------- workloads

def uniform_u32(n: int, seed: int = 0, device="cpu") -> torch.Tensor:
    return to_u32(_lsr(raw64(n, 1, seed, 0, device), 32))


def zipf_pairs_u32(n: int, s: float = 1.1, distinct: int = 1 << 20, seed: int = 0, device="cpu"):
    """(keys uint32, values uint32 = original index)."""
    r = torch.arange(1, distinct + 1, dtype=torch.float64, device=device)
    cdf = torch.cumsum(r ** (-s), 0)
    cdf = cdf / cdf[-1]
    u = uniform_f64(n, 2, seed, 0, device)
    rank = torch.searchsorted(cdf, u, right=True).clamp_(max=distinct - 1)
    salt = _splitmix_int((2 << 40) ^ (seed << 8) ^ 99) & 0xFFFFFFFF
    keys = to_u32(_mix32(rank ^ salt))
    vals = to_u32(torch.arange(n, dtype=torch.int64, device=device))
    return keys, vals


def normal_i64(n: int, sigma: float = 2.0 ** 40, seed: int = 0, device="cpu") -> torch.Tensor:
    z = _normal(n, 3, seed, 0, 1, device)
    return torch.round(sigma * z).to(torch.int64)  # round half to even


def nearly_sorted(keys_sorted: torch.Tensor, frac: float = 0.01, seed: int = 0) -> torch.Tensor:
    """Apply floor(frac * n) draws of adjacent swaps (2j, 2j+1) to a sorted
    array.  Swap positions are even, so the swaps are disjoint and commute;
    repeated draws of the same j are applied once."""
    n = keys_sorted.numel()
    out = keys_sorted.clone()
    if n < 2:
        return out
    m = int(math.floor(frac * n))
    half = n // 2
    j = (uniform_f64(m, 3, seed, 7, keys_sorted.device) * half).to(torch.int64).clamp_(max=half - 1)
    j = torch.unique(j) * 2
    a = out[j].clone()
    out[j] = out[j + 1]
    out[j + 1] = a
    return out


def segment_lengths(num: int, lo_log2: int = 4, hi_log2: int = 18, seed: int = 0, device="cpu"):
    u = uniform_f64(num, 4, seed, 0, device)
    L = torch.floor(torch.exp2(lo_log2 + (hi_log2 - lo_log2) * u)).to(torch.int64)
    return L.clamp_(1 << lo_log2, 1 << hi_log2)


def segments_u32(num: int = 10000, lo_log2: int = 4, hi_log2: int = 18, seed: int = 0, device="cpu"):
    """(keys uint32, offsets int64 of length num + 1)."""
    L = segment_lengths(num, lo_log2, hi_log2, seed, device)
    off = torch.zeros(num + 1, dtype=torch.int64, device=device)
    off[1:] = torch.cumsum(L, 0)
    total = int(off[-1].item())
    keys = to_u32(_lsr(raw64(total, 4, seed, 1, device), 32))
    return keys, off


def lognormal_mix_params(seed: int = 0, k: int = 8):
    u = uniform_f64(2 * k, 5, seed, 0, "cpu").tolist()
    mus = [4.0 * u[i] for i in range(k)]
    sigmas = [0.1 + 0.9 * u[k + i] for i in range(k)]
    return mus, sigmas


def lognormal_mix_u32(n: int, seed: int = 0, k: int = 8, device="cpu") -> torch.Tensor:
    mus, sigmas = lognormal_mix_params(seed, k)
    mu_t = torch.tensor(mus, dtype=torch.float64, device=device)
    sg_t = torch.tensor(sigmas, dtype=torch.float64, device=device)
    comp = (uniform_f64(n, 5, seed, 1, device) * k).to(torch.int64).clamp_(max=k - 1)
    z = torch.exp(mu_t[comp] + sg_t[comp] * _normal(n, 5, seed, 2, 3, device))
    scale = (2.0 ** 32 - 1.0) / max(math.exp(m + 4.0 * s) for m, s in zip(mus, sigmas))
    key = torch.floor(z * scale).clamp_(max=2.0 ** 32 - 1.0).to(torch.int64)
    return to_u32(key)


def randint_i64(n: int, seed: int = 0, device="cpu") -> torch.Tensor:
    u = uniform_f64(n, 6, seed, 0, device)
    return (u * n).to(torch.int64).clamp_(max=max(n - 1, 0))
