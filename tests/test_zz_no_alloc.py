"""ms_sort_noalloc (the entry point that allocates nothing, for callers that
cannot allocate) against ms_sort, through the C ABI: two calls in a row on
one stream, the second with a smaller input, bit-exact against ms_sort's
output and the oracle; sizes beyond the fixed scratch array are refused
before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2211_16479_amd as msort
import workloads
from gpu_helpers import assert_equal_arrays

pytestmark = pytest.mark.gpu


def _np(t: torch.Tensor) -> np.ndarray:
    if t.dtype == torch.uint32:
        return t.cpu().view(torch.int32).numpy().view(np.uint32)
    return t.cpu().numpy()


def _call(fn, t: torch.Tensor, kt: int):
    L = msort.lib()
    st = getattr(L, fn)(ctypes.c_void_p(t.data_ptr()), t.numel(), kt,
                        ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream))
    assert st == 0, f"{fn}: status {st}: {L.ms_last_error().decode()}"


def _max_n(kt: int) -> int:
    """Largest n whose plain-sort scratch fits the fixed array (host query)."""
    lo, hi = 1, 1 << 30
    while lo < hi:
        m = (lo + hi + 1) // 2
        if msort.ms_temp_bytes(m, kt, 0) <= msort.NOALLOC_SCRATCH_BYTES:
            lo = m
        else:
            hi = m - 1
    return lo


@pytest.mark.parametrize("kt", [msort.MS_KEY_U32, msort.MS_KEY_I64])
def test_noalloc_matches_ms_sort_two_calls(gpu, kt):
    nmax = _max_n(kt)
    for n, seed in ((nmax, 11), (300_007, 12)):     # the second call is smaller
        print(f"kt={kt} n={n} seed={seed}", flush=True)
        if kt == msort.MS_KEY_U32:
            k = workloads.uniform_u32(n, seed=seed, device=gpu)
        else:
            k = workloads.normal_i64(n, seed=seed, device=gpu)
        a, b = k.clone(), k.clone()
        _call("ms_sort_noalloc", a, kt)
        _call("ms_sort", b, kt)
        torch.cuda.synchronize()
        got, ref = _np(a), _np(b)
        assert_equal_arrays(got, ref, f"noalloc vs ms_sort n={n}")
        assert_equal_arrays(got, oracle.sort(_np(k), threads=oracle.host_threads()), f"noalloc vs oracle n={n}")


def test_noalloc_refuses_oversize(gpu):
    kt = msort.MS_KEY_U32
    n = _max_n(kt) + 1
    k = torch.zeros(n, dtype=torch.int32, device=gpu)
    L = msort.lib()
    st = L.ms_sort_noalloc(ctypes.c_void_p(k.data_ptr()), n, kt,
                           ctypes.c_void_p(torch.cuda.current_stream(gpu).cuda_stream))
    assert st == 1 and b"scratch" in L.ms_last_error()
    torch.cuda.synchronize()
    assert int(k.abs().sum()) == 0
