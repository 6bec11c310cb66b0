"""C-ABI checks that need no GPU: the library loads, exports every function
include/*.h declares, rejects bad arguments before touching the device, and
plans passes as ceil(log2(ceil(n / tile)))."""
import ctypes
import glob
import math
import os
import re

import pytest

import paper_2211_16479_amd as msort

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(ms_[a-z0-9_]+)\s*\(",
                             text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(msort.LIB_PATH)
    names = declared_functions()
    assert "ms_sort" in names and "ms_sort_pairs" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_version():
    L = msort.lib()
    assert L.ms_version() >= 100
    for s in range(6):
        assert L.ms_status_string(s)
    assert L.ms_status_string(99) == b"unknown status"


def test_argument_checks_enqueue_nothing():
    L = msort.lib()
    # n == 0 is a no-op, even with NULL pointers
    assert L.ms_sort(None, 0, 0, None) == 0
    assert L.ms_sort_pairs(None, None, 0, 0, 4, None) == 0
    # NULL with n > 0
    assert L.ms_sort(None, 10, 0, None) == 1
    assert b"NULL" in L.ms_last_error()
    # unknown key type, bad value widths
    assert L.ms_sort(ctypes.c_void_p(16), 10, 7, None) == 2
    assert L.ms_sort_pairs(ctypes.c_void_p(16), ctypes.c_void_p(64), 10, 0, 3, None) == 2
    assert L.ms_sort_pairs(ctypes.c_void_p(16), None, 10, 0, 4, None) == 1
    assert L.ms_sort_pairs(ctypes.c_void_p(16), ctypes.c_void_p(16), 10, 0, 4, None) == 1
    assert L.ms_profile_read(99, None, None) == 1


@pytest.mark.parametrize("kt,vb", [(0, 0), (1, 4), (3, 0), (2, 8), (3, 4), (0, 8)])
def test_plan_arithmetic(kt, vb):
    for n in [0, 1, 2, 1000, 4095, 4096, 4097, 8192, 8193, 1 << 20, (1 << 20) + 1, 1 << 27,
              (1 << 28) + 12345, 1 << 29]:
        p = msort.ms_plan_query(n, kt, vb)
        T = p["tile"]
        assert T & (T - 1) == 0 and (2 * T) % p["merge_tile"] == 0
        runs = max(1, math.ceil(n / T))
        assert p["passes"] == math.ceil(math.log2(runs))
        if p["merge4_tile"]:
            # pairs of levels fused into one four-run pass
            assert (4 * T) % p["merge4_tile"] == 0 and (2 * T) % p["merge4_tile"] == 0
            assert p["hbm_passes"] == p["passes"] // 2 + p["passes"] % 2
        else:
            assert p["hbm_passes"] == p["passes"]
        assert p["tile_sort_in_place"] == (p["hbm_passes"] % 2 == 0)
        tb = msort.ms_temp_bytes(n, kt, vb)
        if p["passes"] == 0:
            assert tb == 0
        else:
            kb = 4 if kt in (0, 1) else 8
            assert tb >= n * (kb + vb)
    assert msort.ms_temp_bytes(100, 9, 0) == 0


def test_segmented_argument_checks():
    L = msort.lib()
    # nothing to do
    assert L.ms_segmented_sort(None, None, None, 0, 0, 0, 0, 0, None) == 0
    assert L.ms_segmented_sort(ctypes.c_void_p(64), None, None, 0, 10, 0, 0, 0, None) == 0
    # missing offsets / values, bad widths, bad key type
    assert L.ms_segmented_sort(ctypes.c_void_p(64), None, None, 3, 10, 0, 0, 0, None) == 1
    assert L.ms_segmented_sort(ctypes.c_void_p(64), None, ctypes.c_void_p(128), 3, 10, 0, 0, 4, None) == 1
    assert L.ms_segmented_sort(ctypes.c_void_p(64), None, ctypes.c_void_p(128), 3, 10, 0, 0, 3, None) == 2
    assert L.ms_segmented_sort(ctypes.c_void_p(64), None, ctypes.c_void_p(128), 3, 10, 0, 9, 0, None) == 2
    assert L.ms_segmented_sort(None, None, ctypes.c_void_p(128), 3, 10, 0, 0, 0, None) == 1


@pytest.mark.parametrize("kt,vb", [(0, 0), (0, 4), (1, 8), (2, 0), (3, 4), (3, 8)])
def test_size_classes_and_candidates(kt, vb):
    classes = msort.ms_seg_classes(kt, vb)
    assert 2 <= len(classes) <= 8
    bounds = [b for b, _ in classes]
    # powers of two from 256: a segment pads its tile sort by less than 2x
    assert bounds == [256 << c for c in range(len(bounds))]
    tile = msort.ms_plan_query(1 << 20, kt, vb)["tile"]
    assert bounds[-1] == min(tile, 16384)  # the last small class: one tile of at most 16384 keys
    for b, shapes in classes:
        assert shapes, b
        for wg, ipt in shapes:
            assert wg * ipt == b and wg % 64 == 0 and ipt >= 2


def test_tuning_set_get_load(tmp_path):
    classes = msort.ms_seg_classes(0, 0)
    for c, (b, shapes) in enumerate(classes):
        for wg, ipt in shapes:
            msort.ms_tuning_set(0, 0, c, wg, ipt)
            assert msort.ms_tuning_get(0, 0, c) == (wg, ipt)
        msort.ms_tuning_set(0, 0, c, *shapes[0])
    with pytest.raises(msort.MSortError):
        msort.ms_tuning_set(0, 0, 0, 64, 8)          # 512 != class bound
    with pytest.raises(msort.MSortError):
        msort.ms_tuning_set(0, 0, 99, 64, 4)
    b, shapes = classes[1]
    alt = shapes[-1]
    f = tmp_path / "t.txt"
    f.write_text(f"# comment\ngfx950 u32 0 1 {alt[0]} {alt[1]}\ngfx942 u32 0 1 {shapes[0][0]} {shapes[0][1]}\n")
    assert msort.ms_tuning_load(str(f), "gfx950") == 1
    assert msort.ms_tuning_get(0, 0, 1) == alt
    msort.ms_tuning_set(0, 0, 1, *shapes[0])
    bad = tmp_path / "bad.txt"
    bad.write_text("gfx950 u32 zero\n")
    with pytest.raises(msort.MSortError):
        msort.ms_tuning_load(str(bad), "gfx950")


def test_temp_bytes_of_every_form():
    """Scratch sizes are host arithmetic: positive, growing with the input,
    0 for unsupported types or invalid options."""
    seg = [msort.ms_temp_bytes_segmented(m, n, 0, 0) for m, n in ((10, 1 << 16), (10, 1 << 20), (1000, 1 << 20))]
    assert 0 < seg[0] < seg[1] < seg[2]
    assert msort.ms_temp_bytes_segmented(10, 1 << 20, 3, 8) > seg[1]
    assert msort.ms_temp_bytes_segmented(10, 1 << 20, 7, 0) == 0
    lrn = [msort.ms_temp_bytes_learned(n) for n in (1 << 20, 1 << 24, 1 << 29)]
    assert 0 < lrn[0] < lrn[1] < lrn[2]
    # the learned scratch holds two n-key arrays (bucketed copy and spill) at least
    assert lrn[2] >= 8 * (1 << 29)
    assert msort.ms_temp_bytes_learned(1 << 20, bucket_capacity=1000) == 0
    # 64-bit keys: twice the key bytes; an unknown key type gets 0
    b64 = msort.ms_temp_bytes_learned(1 << 24, msort.MS_KEY_I64)
    assert b64 > msort.ms_temp_bytes_learned(1 << 24, msort.MS_KEY_U32) > 0
    assert b64 >= 16 * (1 << 24)
    assert msort.ms_temp_bytes_learned(1 << 24, 7) == 0
    # from 2^23 keys the first-level buffer takes the estimated regions'
    # slack (a quarter of n plus a margin per coarse bucket); the exact
    # pass alone needs n keys
    est = msort.ms_temp_bytes_learned(1 << 23)
    exact = msort.ms_temp_bytes_learned(1 << 23, coarse_estimate=0)
    assert est > exact + 4 * (1 << 23) // 4
    assert msort.ms_temp_bytes_learned((1 << 23) - 1) <= exact
    assert msort.ms_temp_bytes_learned(1 << 23, coarse_estimate=3) == 0
