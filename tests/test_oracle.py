"""Pins of the CPU oracle against things other than itself: brute force over
all small inputs, the by-definition selection procedure, library routines,
closed forms and invariants.  CPU only."""
import itertools
import math

import numpy as np
import pytest

import oracle

U32MAX = np.iinfo(np.uint32).max
I64MIN, I64MAX = np.iinfo(np.int64).min, np.iinfo(np.int64).max


def select_by_definition(keys, vals):
    """Stable sort by its definition: repeatedly take the minimum (key, index)."""
    rest = list(range(len(keys)))
    ko, vo = [], []
    while rest:
        best = min(rest, key=lambda i: (keys[i], i))
        ko.append(keys[best])
        vo.append(vals[best])
        rest.remove(best)
    return ko, vo


@pytest.mark.parametrize("dtype", [np.uint32, np.int64])
def test_all_permutations_sort_to_identity(dtype):
    # n <= 7 one call each; n = 8 (40320 permutations) as one segmented call.
    for n in range(0, 8):
        for p in itertools.permutations(range(n)):
            out = oracle.sort(np.array(p, dtype=dtype))
            assert out.tolist() == list(range(n))
    perms = np.array(list(itertools.permutations(range(8))), dtype=dtype)
    off = np.arange(0, perms.size + 1, 8, dtype=np.int64)
    out = oracle.segmented_sort(perms.ravel(), off).reshape(-1, 8)
    assert (out == np.arange(8, dtype=dtype)).all()


def test_ternary_sequences_match_definition():
    for n in range(0, 9):
        seqs = list(itertools.product((0, 1, 2), repeat=n))
        for s in seqs:
            keys = np.array(s, dtype=np.uint32)
            vals = np.arange(n, dtype=np.uint32)
            ko, vo = oracle.sort_pairs(keys, vals)
            ek, ev = select_by_definition(list(s), list(range(n)))
            assert ko.tolist() == ek and vo.tolist() == ev, s


def test_signed_and_unsigned_orders():
    u = np.array([U32MAX, 0, 1 << 31, (1 << 31) - 1, 5, U32MAX, 0], np.uint32)
    assert oracle.sort(u).tolist() == sorted(u.tolist())
    i = np.array([I64MAX, -1, 0, I64MIN, 1, -(1 << 40), I64MIN, I64MAX], np.int64)
    assert oracle.sort(i).tolist() == sorted(i.tolist())
    i32 = np.array([-1, 2 ** 31 - 1, -2 ** 31, 0, 7], np.int32)
    assert oracle.sort(i32).tolist() == sorted(i32.tolist())
    u64 = np.array([2 ** 64 - 1, 0, 2 ** 63, 2 ** 63 - 1], np.uint64)
    assert oracle.sort(u64).tolist() == sorted(u64.tolist())


@pytest.mark.parametrize("dtype,vdtype", [(np.uint32, np.uint32), (np.int64, np.uint32),
                                          (np.int32, np.uint64), (np.uint64, np.uint64)])
def test_random_against_numpy_stable(dtype, vdtype):
    rng = np.random.default_rng(1)
    for n in (1, 2, 3, 17, 1000, 4097, 100_003):
        info = np.iinfo(dtype)
        # few distinct values -> many ties; also full range
        for hi in (7, None):
            if hi is None:
                k = rng.integers(info.min, info.max, size=n, dtype=dtype, endpoint=True)
            else:
                k = rng.integers(0, hi, size=n).astype(dtype)
            v = np.arange(n, dtype=vdtype)
            ko, vo = oracle.sort_pairs(k, v)
            order = np.argsort(k, kind="stable")
            assert (ko == k[order]).all() and (vo == v[order]).all()
            assert (oracle.sort(k) == np.sort(k, kind="stable")).all()


def test_stability_invariant_with_duplicates():
    rng = np.random.default_rng(2)
    n = 50_000
    k = rng.integers(0, 50, size=n).astype(np.uint32)
    v = np.arange(n, dtype=np.uint32)
    ko, vo = oracle.sort_pairs(k, v)
    assert (np.diff(ko.astype(np.int64)) >= 0).all()
    same = ko[1:] == ko[:-1]
    assert (vo[1:][same] > vo[:-1][same]).all()
    assert (np.sort(vo) == v).all()                  # a permutation
    assert (k[vo] == ko).all()                       # values travel with keys


def test_sorted_and_idempotent_and_reverse():
    rng = np.random.default_rng(3)
    k = rng.integers(0, 2 ** 32, size=10_000, dtype=np.uint64).astype(np.uint32)
    s = oracle.sort(k)
    assert (oracle.sort(s) == s).all()
    assert (oracle.sort(s[::-1].copy()) == s).all()
    assert (oracle.sort(np.full(1000, 9, np.uint32)) == 9).all()


def _merge_left_wins(a, b):
    out, i, j = [], 0, 0
    while i < len(a) and j < len(b):
        if b[j][0] < a[i][0]:
            out.append(b[j]); j += 1
        else:
            out.append(a[i]); i += 1
    return out + a[i:] + b[j:]


def test_paper_mpi_tree_pairing_and_stability_reading():
    """The paper's rank tree (golden file) pairs r with r + split.  With ties,
    that strided order keeps the same keys as the plain sort but not the
    stable order of values; pairing adjacent runs (2j, 2j+1) does."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "mpi_tree_pairs_8.txt")
    golden = [tuple(map(int, l.split())) for l in open(path) if l.strip() and l[0] != "#"]
    size = 8
    got, split, level = [], size // 2, 0
    while split >= 1:
        for r in range(size):
            if split <= r < 2 * split:
                got.append((level, split, r - split, r))
        split //= 2
        level += 1
    assert sorted(got) == sorted(golden)

    rng = np.random.default_rng(4)
    n = 8 * 64
    k = rng.integers(0, 5, size=n).astype(np.uint32)
    v = np.arange(n, dtype=np.uint32)
    chunks = [sorted(zip(k[c * 64:(c + 1) * 64].tolist(), v[c * 64:(c + 1) * 64].tolist()),
                     key=lambda t: t[0]) for c in range(size)]
    # strided (paper) tree
    local = list(chunks)
    split = size // 2
    while split >= 1:
        for r in range(split):
            local[r] = _merge_left_wins(local[r], local[r + split])
        split //= 2
    strided = local[0]
    # adjacent tree
    runs = list(chunks)
    while len(runs) > 1:
        runs = [_merge_left_wins(runs[2 * i], runs[2 * i + 1]) for i in range(len(runs) // 2)]
    adjacent = runs[0]
    ko, vo = oracle.sort_pairs(k, v)
    assert [t[0] for t in strided] == ko.tolist()
    assert [t[0] for t in adjacent] == ko.tolist()
    assert [t[1] for t in adjacent] == vo.tolist()
    assert [t[1] for t in strided] != vo.tolist()


@pytest.mark.parametrize("p", [1, 3, 4, 7, 12])
def test_paper_chunking_rule_then_tree_merge(p):
    """Multiprocessing form: chunks arr[size*i : size*(i+1)] with
    size = ceil(n/p) (trailing chunks may be short or empty), each sorted,
    then merged pairwise with adjacent pairing: same result as one sort."""
    rng = np.random.default_rng(p)
    n = 1000
    k = rng.integers(0, 30, size=n).astype(np.int64)
    v = np.arange(n, dtype=np.uint32)
    size = int(math.ceil(n / p))
    chunks = []
    for i in range(p):
        kc, vc = oracle.sort_pairs(k[size * i:size * (i + 1)], v[size * i:size * (i + 1)])
        chunks.append(list(zip(kc.tolist(), vc.tolist())))
    while len(chunks) > 1:
        nxt = [_merge_left_wins(chunks[2 * i], chunks[2 * i + 1]) for i in range(len(chunks) // 2)]
        if len(chunks) % 2:
            nxt.append(chunks[-1])
        chunks = nxt
    ko, vo = oracle.sort_pairs(k, v)
    assert [t[0] for t in chunks[0]] == ko.tolist() and [t[1] for t in chunks[0]] == vo.tolist()


def test_segmented_matches_per_segment_and_keeps_boundaries():
    rng = np.random.default_rng(5)
    lens = [0, 1, 5, 0, 100, 3, 0, 2048, 1]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    k = rng.integers(0, 10, size=off[-1]).astype(np.uint32)
    v = np.arange(off[-1], dtype=np.uint32)
    ko, vo = oracle.segmented_sort(k, off, v)
    for s in range(len(lens)):
        a, b = off[s], off[s + 1]
        order = np.argsort(k[a:b], kind="stable")
        assert (ko[a:b] == k[a:b][order]).all()
        assert (vo[a:b] == v[a:b][order]).all()
    with pytest.raises(ValueError):
        oracle.segmented_sort(k, off[:-1])


def test_rank_bounds_brute_force():
    rng = np.random.default_rng(6)
    k = rng.integers(-5, 5, size=300).astype(np.int64)
    probes = np.arange(-7, 8, dtype=np.int64)
    lt, le = oracle.rank_bounds(k, probes)
    for q, p in enumerate(probes):
        assert lt[q] == (k < p).sum() and le[q] == (k <= p).sum()
    s = oracle.sort(k)
    lt, le = oracle.rank_bounds(k, s)
    r = np.arange(k.size)
    assert ((lt <= r) & (r < le)).all()


@pytest.mark.parametrize("dtype,vdtype", [(np.uint32, None), (np.uint32, np.uint32), (np.int32, np.uint64),
                                          (np.int64, None), (np.uint64, np.uint32), (np.int64, np.uint64)])
def test_threaded_top_levels_equal_single_thread(dtype, vdtype):
    """The threaded variant (top recursion levels on threads, sequential
    merges of adjacent halves) gives the single-thread oracle's output, which
    numpy's stable sort confirms: sizes below, at and above the thread count,
    odd sizes, and tie-heavy keys with value = index (stability)."""
    rng = np.random.default_rng(5)
    info = np.iinfo(dtype)
    for threads in (2, 3, 4, 7, 8, 16):
        for n in (0, 1, 2, 3, 5, 15, 16, 17, 1000, 65_537, 300_001):
            for hi in (3, None):
                if hi is None:
                    k = rng.integers(info.min, info.max, size=n, dtype=dtype, endpoint=True)
                else:
                    k = rng.integers(0, hi, size=n).astype(dtype)
                if vdtype is None:
                    got = oracle.sort(k, threads=threads)
                    assert np.array_equal(got, oracle.sort(k)), (threads, n)
                    assert np.array_equal(got, np.sort(k, kind="stable")), (threads, n)
                else:
                    v = np.arange(n, dtype=vdtype)
                    gk, gv = oracle.sort_pairs(k, v, threads=threads)
                    ek, ev = oracle.sort_pairs(k, v)
                    assert np.array_equal(gk, ek) and np.array_equal(gv, ev), (threads, n)
                    order = np.argsort(k, kind="stable")
                    assert np.array_equal(gv, v[order]), (threads, n)
