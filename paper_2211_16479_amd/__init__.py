"""Python binding of libmsort.so, the gfx950 stable merge sort library.

Argument marshalling only: every step of every sort runs in the library's HIP
kernels.  Tensors supply device pointers and torch supplies the current HIP
stream; nothing here computes.  If the library has not been built, importing
works but every call raises ``RuntimeError`` -- there is no fallback.

Names follow the C ABI in ``include/msort.h``: ``ms_sort``, ``ms_sort_pairs``
and so on, each taking torch tensors instead of raw pointers.
"""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmsort.so")

MS_KEY_U32, MS_KEY_I32, MS_KEY_U64, MS_KEY_I64 = 0, 1, 2, 3
STATUS = {0: "MS_OK", 1: "MS_ERR_INVALID_ARG", 2: "MS_ERR_UNSUPPORTED",
          3: "MS_ERR_OUT_OF_MEMORY", 4: "MS_ERR_HIP", 5: "MS_ERR_INTERNAL"}

KEY_TYPES = {torch.uint32: MS_KEY_U32, torch.int32: MS_KEY_I32,
             torch.uint64: MS_KEY_U64, torch.int64: MS_KEY_I64}

PROFILE_KERNELS = {"tile_sort": 0, "partition": 1, "merge": 2, "seg_classify": 3,
                   "seg_small": 4, "seg_large": 5, "mlp_train": 6, "learned_hist": 7,
                   "learned_scatter": 8, "bucket_sort": 9, "learned_other": 10,
                   "partition4": 11, "merge4": 12, "learned_hist2": 13, "learned_scatter2": 14,
                   "partition_samples": 15, "learned_estimate": 16}

MS_ALGO_AUTO, MS_ALGO_MERGE_PATH, MS_ALGO_LEARNED_BUCKET = 0, 1, 2
MS_FEATURE_LOG, MS_FEATURE_LINEAR, MS_FEATURE_AUTO = 0, 1, 2
MLP_HIDDEN = 16
MLP_PARAMS = 3 * MLP_HIDDEN + 1


class MsOptions(ctypes.Structure):
    """ms_options of include/msort.h."""
    _fields_ = [("algo", ctypes.c_int), ("spill_threshold", ctypes.c_float),
                ("bucket_capacity", ctypes.c_uint32), ("bucket_fill", ctypes.c_uint32),
                ("train_steps", ctypes.c_uint32), ("learning_rate", ctypes.c_float),
                ("sample_log2", ctypes.c_uint32), ("seed", ctypes.c_uint64), ("feature", ctypes.c_int),
                ("use_network", ctypes.c_int), ("force_fallback", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("max_workgroups", ctypes.c_uint32), ("coarse_estimate", ctypes.c_int)]


class MsStats(ctypes.Structure):
    """ms_stats of include/msort.h."""
    _fields_ = [("algo_used", ctypes.c_int32), ("fallback_taken", ctypes.c_int32),
                ("misordered", ctypes.c_int32), ("repaired", ctypes.c_int32), ("spilled", ctypes.c_uint64),
                ("max_bucket", ctypes.c_uint64), ("buckets", ctypes.c_uint64), ("loss_initial", ctypes.c_float),
                ("loss_final", ctypes.c_float), ("coarse_recounted", ctypes.c_int32),
                ("sample_fallback", ctypes.c_int32)]


_lib = None


class MSortError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")


def _declare(lib):
    c = ctypes
    sz, vp, i32 = c.c_size_t, c.c_void_p, c.c_int
    sig = {
        "ms_version": (i32, []),
        "ms_status_string": (c.c_char_p, [i32]),
        "ms_last_error": (c.c_char_p, []),
        "ms_sort": (i32, [vp, sz, i32, vp]),
        "ms_sort_pairs": (i32, [vp, vp, sz, i32, sz, vp]),
        "ms_sort_noalloc": (i32, [vp, sz, i32, vp]),
        "ms_temp_bytes": (sz, [sz, i32, sz]),
        "ms_temp_bytes_segmented": (sz, [sz, sz, i32, sz]),
        "ms_temp_bytes_learned": (sz, [sz, c.c_int, c.POINTER(MsOptions)]),
        "ms_sort_pairs_ex": (c.c_int, [vp, vp, sz, c.c_int, sz, c.POINTER(MsOptions), vp, vp]),
        "ms_temp_bytes_learned_pairs": (sz, [sz, c.c_int, sz, c.POINTER(MsOptions)]),
        "ms_graph_captures": (c.c_uint64, []),
        "ms_device_errors": (i32, [c.POINTER(c.c_uint32)]),
        "ms_plan_query": (i32, [sz, i32, sz, c.POINTER(i32), c.POINTER(i32), c.POINTER(i32),
                                c.POINTER(i32), c.POINTER(i32), c.POINTER(i32)]),
        "ms_release_workspace": (i32, []),
        "ms_segmented_sort": (i32, [vp, vp, vp, sz, sz, sz, i32, sz, vp]),
        "ms_seg_num_classes": (i32, [i32, sz, c.POINTER(i32)]),
        "ms_seg_class_info": (i32, [i32, sz, i32, c.POINTER(c.c_uint32), c.POINTER(i32)]),
        "ms_seg_candidate": (i32, [i32, sz, i32, i32, c.POINTER(i32), c.POINTER(i32)]),
        "ms_tuning_set": (i32, [i32, sz, i32, i32, i32]),
        "ms_tuning_get": (i32, [i32, sz, i32, c.POINTER(i32), c.POINTER(i32)]),
        "ms_tuning_load": (i32, [c.c_char_p, c.c_char_p, c.POINTER(i32)]),
        "ms_options_default": (None, [c.POINTER(MsOptions)]),
        "ms_sort_ex": (i32, [vp, sz, i32, c.POINTER(MsOptions), vp, vp]),
        "ms_learned_grad": (i32, [vp, c.c_uint32, i32, vp, vp, vp]),
        "ms_learned_train": (i32, [vp, c.c_uint32, i32, c.c_uint32, c.c_float, vp, vp, vp, vp]),
        "ms_learned_table": (i32, [vp, vp, c.c_uint32, i32, vp, vp, vp, vp]),
        "ms_learned_bucket_ids": (i32, [vp, sz, vp, vp, c.c_uint32, i32, i32, c.c_uint32, vp, vp]),
        "ms_profile_enable": (i32, [i32]),
        "ms_profile_select": (i32, [c.c_uint32]),
        "ms_profile_reset": (i32, []),
        "ms_profile_read": (i32, [i32, c.POINTER(c.c_uint64), c.POINTER(c.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != 0:
        raise MSortError(status, where, lib().ms_last_error().decode())


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _key_type(t: torch.Tensor, key_type=None) -> int:
    if key_type is not None:
        return int(key_type)
    try:
        return KEY_TYPES[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported key dtype {t.dtype}; pass key_type explicitly") from None


def _dev(t: torch.Tensor, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def ms_sort(keys: torch.Tensor, key_type=None) -> torch.Tensor:
    """Sort ``keys`` in place (ascending) on the current stream; returns it."""
    _dev(keys, "keys")
    _check(lib().ms_sort(ctypes.c_void_p(keys.data_ptr()), keys.numel(), _key_type(keys, key_type),
                         _stream(keys)), "ms_sort")
    return keys


def ms_sort_noalloc(keys: torch.Tensor, key_type=None) -> torch.Tensor:
    """ms_sort with the library's fixed per-GPU scratch array (no device
    allocation); n is limited by MS_NOALLOC_SCRATCH_BYTES.  Returns keys."""
    _dev(keys, "keys")
    _check(lib().ms_sort_noalloc(ctypes.c_void_p(keys.data_ptr()), keys.numel(), _key_type(keys, key_type),
                                 _stream(keys)), "ms_sort_noalloc")
    return keys


NOALLOC_SCRATCH_BYTES = 64 << 20


def ms_sort_pairs(keys: torch.Tensor, vals: torch.Tensor, key_type=None):
    """Stable in-place sort of (keys, vals) by key; returns (keys, vals)."""
    _dev(keys, "keys")
    _dev(vals, "vals")
    if vals.numel() != keys.numel():
        raise ValueError("keys and vals differ in length")
    _check(lib().ms_sort_pairs(ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
                               keys.numel(), _key_type(keys, key_type), vals.element_size(),
                               _stream(keys)), "ms_sort_pairs")
    return keys, vals


def ms_segmented_sort(keys: torch.Tensor, offsets: torch.Tensor, vals: torch.Tensor = None,
                      max_segment_len: int = 0, key_type=None):
    """Sort every segment keys[offsets[s]:offsets[s+1]] in place (stable).

    ``offsets`` is an int64 GPU tensor of num_segments + 1 entries starting at
    0 and ending at len(keys).  One cached hipGraph launch on the current
    stream does all segments.  Returns (keys, vals)."""
    _dev(keys, "keys")
    _dev(offsets, "offsets")
    _ensure_tuning()
    if offsets.dtype != torch.int64:
        raise TypeError("offsets must be int64")
    vb = 0
    vp = None
    if vals is not None:
        _dev(vals, "vals")
        if vals.numel() != keys.numel():
            raise ValueError("keys and vals differ in length")
        vb = vals.element_size()
        vp = ctypes.c_void_p(vals.data_ptr())
    _check(lib().ms_segmented_sort(ctypes.c_void_p(keys.data_ptr()), vp, ctypes.c_void_p(offsets.data_ptr()),
                                   max(0, offsets.numel() - 1), keys.numel(), int(max_segment_len),
                                   _key_type(keys, key_type), vb, _stream(keys)), "ms_segmented_sort")
    return keys, vals


def ms_seg_classes(key_type: int, val_bytes: int = 0) -> list:
    """[(max_len, [(wg, ipt), ...]), ...] for every small class of a family."""
    L = lib()
    nc = ctypes.c_int()
    _check(L.ms_seg_num_classes(key_type, val_bytes, ctypes.byref(nc)), "ms_seg_num_classes")
    out = []
    for c in range(nc.value):
        ml, ncand = ctypes.c_uint32(), ctypes.c_int()
        _check(L.ms_seg_class_info(key_type, val_bytes, c, ctypes.byref(ml), ctypes.byref(ncand)),
               "ms_seg_class_info")
        shapes = []
        for i in range(ncand.value):
            wg, ipt = ctypes.c_int(), ctypes.c_int()
            _check(L.ms_seg_candidate(key_type, val_bytes, c, i, ctypes.byref(wg), ctypes.byref(ipt)),
                   "ms_seg_candidate")
            shapes.append((wg.value, ipt.value))
        out.append((ml.value, shapes))
    return out


def ms_tuning_set(key_type: int, val_bytes: int, cls: int, wg: int, ipt: int):
    _check(lib().ms_tuning_set(key_type, val_bytes, cls, wg, ipt), "ms_tuning_set")


def ms_tuning_get(key_type: int, val_bytes: int, cls: int) -> tuple:
    wg, ipt = ctypes.c_int(), ctypes.c_int()
    _check(lib().ms_tuning_get(key_type, val_bytes, cls, ctypes.byref(wg), ctypes.byref(ipt)), "ms_tuning_get")
    return wg.value, ipt.value


def ms_tuning_load(path: str, arch: str = None) -> int:
    n = ctypes.c_int()
    _check(lib().ms_tuning_load(path.encode(), None if arch is None else arch.encode(), ctypes.byref(n)),
           "ms_tuning_load")
    return n.value


TUNING_DIR = os.path.join(_PKG, "tuning")
_tuning_loaded = False


def _ensure_tuning():
    """Apply the committed per-class shape table once per process (GPU runs)."""
    global _tuning_loaded
    if not _tuning_loaded:
        _tuning_loaded = True
        load_default_tuning()


def load_default_tuning(arch: str = None) -> int:
    """Apply the committed tuning table for this GPU architecture, if present."""
    path = os.path.join(TUNING_DIR, "tuning.txt")
    if not os.path.exists(path):
        return 0
    return ms_tuning_load(path, arch)


def ms_options_default() -> MsOptions:
    o = MsOptions()
    lib().ms_options_default(ctypes.byref(o))
    return o


def ms_sort_ex(keys: torch.Tensor, key_type=None, stats: bool = True, **options):
    """ms_sort with an algorithm choice; keyword arguments set ms_options
    fields (algo, spill_threshold, bucket_capacity, ...).  Returns
    (keys, stats dict or None); stats are read after a stream sync."""
    _dev(keys, "keys")
    _ensure_tuning()  # the learned form sorts its buckets with the per-class shapes
    o = ms_options_default()
    for k, v in options.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    st = torch.zeros(ctypes.sizeof(MsStats), dtype=torch.uint8, device=keys.device) if stats else None
    _check(lib().ms_sort_ex(ctypes.c_void_p(keys.data_ptr()), keys.numel(), _key_type(keys, key_type),
                            ctypes.byref(o), None if st is None else ctypes.c_void_p(st.data_ptr()),
                            _stream(keys)), "ms_sort_ex")
    if st is None:
        return keys, None
    torch.cuda.current_stream(keys.device).synchronize()
    raw = MsStats.from_buffer_copy(bytes(st.cpu().numpy()))
    return keys, {f: getattr(raw, f) for f, _ in MsStats._fields_}


def ms_sort_pairs_ex(keys: torch.Tensor, vals: torch.Tensor, key_type=None, stats: bool = True, **options):
    """ms_sort_pairs with an algorithm choice (stable); keyword arguments set
    ms_options fields.  Returns (keys, vals, stats dict or None)."""
    _dev(keys, "keys")
    _dev(vals, "vals")
    if vals.numel() != keys.numel():
        raise ValueError("keys and vals differ in length")
    _ensure_tuning()
    o = ms_options_default()
    for k, v in options.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    st = torch.zeros(ctypes.sizeof(MsStats), dtype=torch.uint8, device=keys.device) if stats else None
    _check(lib().ms_sort_pairs_ex(ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(vals.data_ptr()),
                                  keys.numel(), _key_type(keys, key_type), vals.element_size(), ctypes.byref(o),
                                  None if st is None else ctypes.c_void_p(st.data_ptr()), _stream(keys)),
           "ms_sort_pairs_ex")
    if st is None:
        return keys, vals, None
    torch.cuda.current_stream(keys.device).synchronize()
    raw = MsStats.from_buffer_copy(bytes(st.cpu().numpy()))
    return keys, vals, {f: getattr(raw, f) for f, _ in MsStats._fields_}


def ms_temp_bytes_learned_pairs(n: int, key_type: int = MS_KEY_U32, val_bytes: int = 4, **options) -> int:
    o = ms_options_default()
    for k, v in options.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return int(lib().ms_temp_bytes_learned_pairs(n, key_type, val_bytes, ctypes.byref(o)))


def _f32(t: torch.Tensor, n: int, name: str):
    _dev(t, name)
    if t.dtype != torch.float32 or t.numel() < n:
        raise ValueError(f"{name} must be float32 with at least {n} elements")


def ms_learned_grad(sample_sorted: torch.Tensor, theta: torch.Tensor, feature: int = MS_FEATURE_LOG):
    """Gradient (49) and squared-error sum (1) of the MLP at theta on a sorted
    uint32 sample; returns a float32 tensor of 50."""
    _dev(sample_sorted, "sample")
    _f32(theta, MLP_PARAMS, "theta")
    out = torch.empty(MLP_PARAMS + 1, dtype=torch.float32, device=theta.device)
    _check(lib().ms_learned_grad(ctypes.c_void_p(sample_sorted.data_ptr()), sample_sorted.numel(), feature,
                                 ctypes.c_void_p(theta.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 _stream(theta)), "ms_learned_grad")
    return out


def ms_learned_train(sample_sorted: torch.Tensor, steps: int, learning_rate: float, theta0: torch.Tensor = None,
                     feature: int = MS_FEATURE_LOG):
    """(theta after `steps` Adam steps, loss before each step)."""
    _dev(sample_sorted, "sample")
    dev = sample_sorted.device
    th = torch.empty(MLP_PARAMS, dtype=torch.float32, device=dev)
    hist = torch.empty(max(1, steps), dtype=torch.float32, device=dev)
    if theta0 is not None:
        _f32(theta0, MLP_PARAMS, "theta0")
    _check(lib().ms_learned_train(ctypes.c_void_p(sample_sorted.data_ptr()), sample_sorted.numel(), feature, steps,
                                  learning_rate, None if theta0 is None else ctypes.c_void_p(theta0.data_ptr()),
                                  ctypes.c_void_p(th.data_ptr()), ctypes.c_void_p(hist.data_ptr()),
                                  _stream(sample_sorted)), "ms_learned_train")
    return th, hist[:steps]


def ms_learned_table(theta: torch.Tensor, sample_sorted: torch.Tensor, feature: int = MS_FEATURE_LOG):
    """(points, values, count) of theta's inference table on the sorted sample's range."""
    _f32(theta, MLP_PARAMS, "theta")
    _dev(sample_sorted, "sample")
    t = torch.empty(32, dtype=torch.float32, device=theta.device)
    v = torch.empty(32, dtype=torch.float32, device=theta.device)
    c = torch.empty(1, dtype=torch.int32, device=theta.device)
    _check(lib().ms_learned_table(ctypes.c_void_p(theta.data_ptr()), ctypes.c_void_p(sample_sorted.data_ptr()),
                                  sample_sorted.numel(), feature, ctypes.c_void_p(t.data_ptr()),
                                  ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(c.data_ptr()), _stream(theta)),
           "ms_learned_table")
    n = int(c.item())
    return t[:n], v[:n], n


def ms_learned_bucket_ids(keys: torch.Tensor, theta: torch.Tensor, sample_sorted: torch.Tensor, log2_buckets: int,
                          feature: int = MS_FEATURE_LOG, use_network: bool = True):
    _dev(keys, "keys")
    _dev(sample_sorted, "sample")
    _f32(theta, MLP_PARAMS, "theta")
    out = torch.empty(keys.numel(), dtype=torch.int32, device=keys.device)
    _check(lib().ms_learned_bucket_ids(ctypes.c_void_p(keys.data_ptr()), keys.numel(),
                                       ctypes.c_void_p(theta.data_ptr()), ctypes.c_void_p(sample_sorted.data_ptr()),
                                       sample_sorted.numel(), feature, 1 if use_network else 0, log2_buckets,
                                       ctypes.c_void_p(out.data_ptr()), _stream(keys)),
           "ms_learned_bucket_ids")
    return out


def ms_temp_bytes(n: int, key_type: int, val_bytes: int = 0) -> int:
    return int(lib().ms_temp_bytes(n, key_type, val_bytes))


def ms_temp_bytes_segmented(num_segments: int, n_total: int, key_type: int, val_bytes: int = 0) -> int:
    return int(lib().ms_temp_bytes_segmented(num_segments, n_total, key_type, val_bytes))


def ms_temp_bytes_learned(n: int, key_type: int = MS_KEY_U32, **options) -> int:
    o = ms_options_default()
    for k, v in options.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return int(lib().ms_temp_bytes_learned(n, key_type, ctypes.byref(o)))


def ms_device_errors() -> int:
    """Error bits raised by the kernels since the last call (0: none);
    synchronises the device."""
    v = ctypes.c_uint32()
    _check(lib().ms_device_errors(ctypes.byref(v)), "ms_device_errors")
    return int(v.value)


def ms_graph_captures() -> int:
    """hipGraphs captured so far by this process."""
    return int(lib().ms_graph_captures())


def ms_plan_query(n: int, key_type: int, val_bytes: int = 0) -> dict:
    t, mt, p, ip, h, mt4 = (ctypes.c_int() for _ in range(6))
    _check(lib().ms_plan_query(n, key_type, val_bytes, ctypes.byref(t), ctypes.byref(mt),
                               ctypes.byref(p), ctypes.byref(ip), ctypes.byref(h), ctypes.byref(mt4)),
           "ms_plan_query")
    return {"tile": t.value, "merge_tile": mt.value, "passes": p.value,
            "tile_sort_in_place": bool(ip.value), "hbm_passes": h.value, "merge4_tile": mt4.value}


def ms_release_workspace():
    _check(lib().ms_release_workspace(), "ms_release_workspace")


def ms_profile_enable(on: bool = True):
    _check(lib().ms_profile_enable(1 if on else 0), "ms_profile_enable")


def ms_profile_select(classes=None):
    """Time only the named kernel classes (None: all)."""
    mask = 0xFFFFFFFF if classes is None else sum(1 << (PROFILE_KERNELS[c] if isinstance(c, str) else int(c))
                                                  for c in classes)
    _check(lib().ms_profile_select(mask), "ms_profile_select")


def ms_profile_reset():
    _check(lib().ms_profile_reset(), "ms_profile_reset")


def ms_profile_read(kernel) -> tuple:
    """(launches, total_ms) for a kernel class name or id since the last reset."""
    k = PROFILE_KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    n = ctypes.c_uint64()
    ms = ctypes.c_double()
    _check(lib().ms_profile_read(k, ctypes.byref(n), ctypes.byref(ms)), "ms_profile_read")
    return int(n.value), float(ms.value)


def version() -> int:
    return int(lib().ms_version())
