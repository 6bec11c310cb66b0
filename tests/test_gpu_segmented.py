"""GPU parity of ms_segmented_sort against the CPU oracle: class boundaries,
every compiled per-class shape, all key/value types, the batched workload
reduced and at full size, and graph replay with new data."""
import numpy as np
import pytest
import torch

import oracle
import paper_2211_16479_amd as msort
import workloads
from gpu_helpers import assert_equal_arrays, keys_fill, to_dev

pytestmark = pytest.mark.gpu

BOUNDARY_LENS = [0, 1, 2, 3, 0, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097,
                 8191, 8192, 8193, 16383, 16384, 16385, 40000, 65536, 100_003, 1, 0]


def run_seg(keys_np, off_np, vals_np, dev, max_len=0):
    k = to_dev(keys_np, dev)
    o = to_dev(off_np.astype(np.int64), dev)
    v = None if vals_np is None else to_dev(vals_np, dev)
    msort.ms_segmented_sort(k, o, v, max_segment_len=max_len)
    torch.cuda.synchronize()
    return k.cpu().numpy(), None if v is None else v.cpu().numpy()


def offsets_of(lens):
    return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


@pytest.mark.parametrize("kdt,vdt", [(np.uint32, None), (np.uint32, np.uint32), (np.int32, np.uint64),
                                     (np.uint64, None), (np.int64, np.uint32), (np.int64, np.uint64)],
                         ids=lambda d: "none" if d is None else np.dtype(d).name)
def test_class_boundaries(gpu, kdt, vdt):
    rng = np.random.default_rng(21)
    off = offsets_of(BOUNDARY_LENS)
    # extremes: heavy ties at the type's largest key, which the keys-only
    # merges also use to pad their runs in LDS
    for dist in ("uniform", "few", "extremes"):
        k = keys_fill(int(off[-1]), kdt, dist, rng)
        v = None if vdt is None else np.arange(off[-1], dtype=vdt)
        gk, gv = run_seg(k, off, v, gpu)
        if v is None:
            assert_equal_arrays(gk, oracle.segmented_sort(k, off), f"{dist} keys")
        else:
            ek, ev = oracle.segmented_sort(k, off, v)
            assert_equal_arrays(gk, ek, f"{dist} keys")
            assert_equal_arrays(gv, ev, f"{dist} values")


FAMILIES = [(np.uint32, None, msort.MS_KEY_U32), (np.uint32, np.uint32, msort.MS_KEY_U32),
            (np.int32, np.uint64, msort.MS_KEY_I32), (np.uint64, None, msort.MS_KEY_U64),
            (np.int64, None, msort.MS_KEY_I64)]


@pytest.mark.parametrize("kdt,vdt,kt", FAMILIES,
                         ids=lambda d: "none" if d is None else (np.dtype(d).name if not isinstance(d, int) else str(d)))
def test_every_class_candidate(gpu, kdt, vdt, kt):
    """Each compiled per-class shape of every tuned family sorts correctly
    (tuning table entries), against the oracle, heavy ties (few values, and
    values at the type's limits)."""
    rng = np.random.default_rng(22)
    vb = 0 if vdt is None else np.dtype(vdt).itemsize
    classes = msort.ms_seg_classes(kt, vb)
    saved = [msort.ms_tuning_get(kt, vb, c) for c in range(len(classes))]
    try:
        for c, (bound, shapes) in enumerate(classes):
            lo = 2 if c == 0 else classes[c - 1][0] + 1
            lens = np.concatenate([[lo, bound, (lo + bound) // 2], rng.integers(lo, bound + 1, size=40)])
            off = offsets_of(lens)
            for dist in ("few", "extremes"):
                k = keys_fill(int(off[-1]), kdt, dist, rng)
                v = None if vdt is None else np.arange(off[-1], dtype=vdt)
                exp = oracle.segmented_sort(k, off, v)
                for wg, ipt in shapes:
                    msort.ms_tuning_set(kt, vb, c, wg, ipt)
                    gk, gv = run_seg(k, off, v, gpu)
                    if v is None:
                        assert_equal_arrays(gk, exp, f"class {c} shape {wg}x{ipt} {dist}")
                    else:
                        assert_equal_arrays(gk, exp[0], f"class {c} shape {wg}x{ipt} {dist} keys")
                        assert_equal_arrays(gv, exp[1], f"class {c} shape {wg}x{ipt} {dist} values")
    finally:
        for c, (wg, ipt) in enumerate(saved):
            msort.ms_tuning_set(kt, vb, c, wg, ipt)


def test_batched_reduced(gpu):
    keys, off = workloads.segments_u32(1000, seed=1)
    k = keys.numpy() if keys.dtype != torch.uint32 else keys.view(torch.int32).numpy().view(np.uint32)
    gk, _ = run_seg(k, off.numpy(), None, gpu, max_len=1 << 18)
    assert_equal_arrays(gk, oracle.segmented_sort(k, off.numpy()), "1000 log-uniform segments")


def test_graph_replay_with_new_data(gpu):
    """Same buffers twice: the second call replays the cached graph on new keys."""
    rng = np.random.default_rng(23)
    lens = rng.integers(0, 30000, size=300)
    off = offsets_of(lens)
    kt = to_dev(np.zeros(int(off[-1]), np.uint32), gpu)
    ot = to_dev(off, gpu)
    for rep in range(3):
        k = keys_fill(int(off[-1]), np.uint32, "uniform", rng)
        kt.copy_(to_dev(k, gpu))
        msort.ms_segmented_sort(kt, ot, max_segment_len=30000)
        torch.cuda.synchronize()
        assert_equal_arrays(kt.cpu().numpy(), oracle.segmented_sort(k, off), f"replay {rep}")


def oracle_segmented_threaded(k: np.ndarray, off: np.ndarray, parts: int) -> np.ndarray:
    """The oracle's segmented sort over `parts` contiguous groups of segments
    at once (the C oracle releases the GIL); segments are independent, so the
    result is oracle.segmented_sort(k, off)."""
    import concurrent.futures as cf
    nseg = off.size - 1
    cuts = np.linspace(0, nseg, parts + 1).astype(np.int64)
    out = np.empty_like(k)

    def one(i):
        s0, s1 = cuts[i], cuts[i + 1]
        a, b = off[s0], off[s1]
        out[a:b] = oracle.segmented_sort(k[a:b], off[s0:s1 + 1] - a)

    with cf.ThreadPoolExecutor(parts) as ex:
        list(ex.map(one, range(parts)))
    return out


def test_full_batched_10000(gpu):
    """Configuration 4 at full size: 10,000 uint32 arrays, lengths
    log-uniform in [16, 2^18], one call; every segment equals the oracle's
    sort of it, element by element."""
    keys, off = workloads.segments_u32(10000, seed=0, device=gpu)
    out = keys.clone()
    msort.ms_segmented_sort(out, off, max_segment_len=1 << 18)
    torch.cuda.synchronize()
    on = off.cpu().numpy()
    kin = keys.view(torch.int32).cpu().numpy().view(np.uint32)
    kout = out.view(torch.int32).cpu().numpy().view(np.uint32)
    exp = oracle_segmented_threaded(kin, on, oracle.host_threads())
    assert_equal_arrays(kout, exp, "10,000 segments")


def test_fresh_buffers_replay_one_graph(gpu):
    """20 calls, each on freshly allocated key, value and offset tensors of
    the same sizes: one graph capture in all, every output equal to the
    oracle's (the graph reads the buffers bound at each launch)."""
    rng = np.random.default_rng(24)
    lens = rng.integers(0, 40000, size=257)
    off = offsets_of(lens)
    n = int(off[-1])
    before = msort.ms_graph_captures()
    for rep in range(20):
        k = keys_fill(n, np.uint32, "few" if rep % 2 else "uniform", rng)
        v = np.arange(n, dtype=np.uint32)
        kt, vt, ot = to_dev(k, gpu), to_dev(v, gpu), to_dev(off, gpu)
        msort.ms_segmented_sort(kt, ot, vt, max_segment_len=40000)
        torch.cuda.synchronize()
        ek, ev = oracle.segmented_sort(k, off, v)
        assert_equal_arrays(kt.cpu().numpy(), ek, f"call {rep} keys")
        assert_equal_arrays(vt.cpu().numpy(), ev, f"call {rep} values")
        del kt, vt, ot
    assert msort.ms_graph_captures() - before == 1


@pytest.mark.parametrize("hint", [1000, 20000, 70000])
def test_too_small_length_hint_still_sorts(gpu, hint):
    """A max_segment_len below the longest segment (at or below the small
    classes, or a few merge levels short) still sorts every segment: the
    merge steps beyond the hint run on the device when it finds a longer
    segment."""
    rng = np.random.default_rng(25)
    lens = np.concatenate([[300_000, 5, 70_001, 16_385, 200_000], rng.integers(0, 3000, size=100)])
    off = offsets_of(lens)
    for kdt, vdt in ((np.uint32, None), (np.int64, np.uint32)):
        k = keys_fill(int(off[-1]), kdt, "uniform", rng)
        v = None if vdt is None else np.arange(off[-1], dtype=vdt)
        gk, gv = run_seg(k, off, v, gpu, max_len=hint)
        if v is None:
            assert_equal_arrays(gk, oracle.segmented_sort(k, off), f"hint {hint} keys")
        else:
            ek, ev = oracle.segmented_sort(k, off, v)
            assert_equal_arrays(gk, ek, f"hint {hint} pair keys")
            assert_equal_arrays(gv, ev, f"hint {hint} pair values")


def test_no_internal_errors_raised(gpu):
    """No kernel of the runs before this one (the whole GPU session when the
    files run in order) found inconsistent merge offsets."""
    assert msort.ms_device_errors() == 0
    assert msort.ms_device_errors() == 0
