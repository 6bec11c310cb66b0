"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU product path never imports it,
and it imports nothing from the product package: the two share no code.

Contents
--------
* :func:`sort`, :func:`sort_pairs`, :func:`segmented_sort` -- the plain
  top-down stable merge sort of the paper's section "Sequential Merge Sort"
  (its step list and the mergesort figure, with the right half read as
  ``array[mid:]`` and ``merge`` taking the right head only when strictly
  smaller), in plain C (``msort_oracle.c``), single threaded.
* :func:`sort` / :func:`sort_pairs` with ``threads > 1`` -- the same
  recursion with its top ceil(log2(threads)) levels on threads (the paper's
  section "Multiprocessing Merge Sort": independent chunk sorts, then a tree
  of merges of adjacent runs); identical output, used to time the CPU
  baseline on all host cores and to check full-size GPU outputs quickly.
* :func:`rank_bounds` -- by-definition rank counts used to verify sampled
  positions of outputs too large to sort on the CPU within a test.
* :mod:`oracle.mlp` -- the fp64 two-layer MLP CDF model (forward, analytic
  backward, Adam) that the learned-bucket form trains on the GPU in FP32.
"""
import ctypes
import os

import numpy as np

from .build import LIB, SRC, compile_oracle

KEY_TYPES = {np.dtype(np.uint32): 0, np.dtype(np.int32): 1,
             np.dtype(np.uint64): 2, np.dtype(np.int64): 3}

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            compile_oracle(force=True)
        lib = ctypes.CDLL(LIB)
        lib.oracle_sort.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_int, ctypes.c_size_t]
        lib.oracle_sort.restype = ctypes.c_int
        lib.oracle_sort_parallel.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                             ctypes.c_int, ctypes.c_size_t, ctypes.c_int]
        lib.oracle_sort_parallel.restype = ctypes.c_int
        lib.oracle_segmented_sort.argtypes = [ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_size_t,
                                              ctypes.c_int, ctypes.c_size_t]
        lib.oracle_segmented_sort.restype = ctypes.c_int
        lib.oracle_rank_bounds.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                           ctypes.c_void_p, ctypes.c_size_t,
                                           ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_rank_bounds.restype = ctypes.c_int
        _lib = lib
    return _lib


def _kt(a: np.ndarray) -> int:
    try:
        return KEY_TYPES[a.dtype]
    except KeyError:
        raise TypeError(f"unsupported key dtype {a.dtype}") from None


def host_threads() -> int:
    """Threads the parallel oracle uses by default: this host's cores, at
    most 16."""
    return max(1, min(16, os.cpu_count() or 1))


def _run(k: np.ndarray, v, threads: int) -> None:
    L = _load()
    vp = None if v is None else v.ctypes.data
    vb = 0 if v is None else v.dtype.itemsize
    if threads == 1:
        rc = L.oracle_sort(k.ctypes.data, vp, k.size, _kt(k), vb)
    else:
        rc = L.oracle_sort_parallel(k.ctypes.data, vp, k.size, _kt(k), vb, int(threads))
    if rc:
        raise RuntimeError(f"oracle sort failed ({rc})")


def sort(keys: np.ndarray, threads: int = 1) -> np.ndarray:
    """Return the ascending (stable) merge sort of ``keys`` (a new array).
    threads > 1 runs the top recursion levels on threads (same output)."""
    out = np.ascontiguousarray(keys).copy()
    _run(out, None, threads)
    return out


def sort_pairs(keys: np.ndarray, vals: np.ndarray, threads: int = 1):
    """Stable sort of (key, value) pairs: equal keys keep their input order."""
    k = np.ascontiguousarray(keys).copy()
    v = np.ascontiguousarray(vals).copy()
    if k.shape != v.shape or v.dtype.itemsize not in (4, 8):
        raise ValueError("keys/values shape or value width mismatch")
    _run(k, v, threads)
    return k, v


def segmented_sort(keys: np.ndarray, offsets: np.ndarray, vals: np.ndarray = None):
    """Sort every segment [offsets[s], offsets[s+1]) independently and stably."""
    k = np.ascontiguousarray(keys).copy()
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    if off[0] != 0 or off[-1] != k.size:
        raise ValueError("offsets must start at 0 and end at len(keys)")
    v = None if vals is None else np.ascontiguousarray(vals).copy()
    rc = _load().oracle_segmented_sort(k.ctypes.data, None if v is None else v.ctypes.data,
                                       off.ctypes.data, off.size - 1, _kt(k),
                                       0 if v is None else v.dtype.itemsize)
    if rc:
        raise RuntimeError(f"oracle_segmented_sort failed ({rc})")
    return k if v is None else (k, v)


def rank_bounds(keys: np.ndarray, probes: np.ndarray):
    """(lt, le): how many keys are < and <= each probe, counted by definition."""
    k = np.ascontiguousarray(keys)
    p = np.ascontiguousarray(probes, dtype=k.dtype)
    lt = np.zeros(p.size, np.uint64)
    le = np.zeros(p.size, np.uint64)
    rc = _load().oracle_rank_bounds(k.ctypes.data, k.size, _kt(k), p.ctypes.data, p.size,
                                    lt.ctypes.data, le.ctypes.data)
    if rc:
        raise RuntimeError("oracle_rank_bounds failed")
    return lt, le
