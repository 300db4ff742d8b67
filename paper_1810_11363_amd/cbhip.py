"""ctypes binding of libcbhip (include/cbhip.h), same names as the C calls.

Argument marshalling only: every step runs in the HIP library. Device buffers
are passed as integers (``tensor.data_ptr()``) or torch tensors; streams as
integers (``torch.cuda.current_stream().cuda_stream``) or None.

Importing this module raises if the library has not been built: there is no
CPU fallback for any call.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbhip.so")

CBH_OK, CBH_EINVAL, CBH_ENOMEM, CBH_EDEVICE, CBH_EOVERFLOW, CBH_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
CBH_EBUSY = -6
CBH_LOSS_RMSE, CBH_LOSS_LOGLOSS, CBH_LOSS_MULTICLASS = 0, 1, 2
CBH_PREC_FP32, CBH_PREC_TWOFLOAT, CBH_PREC_INT16, CBH_PREC_F64 = 0, 1, 2, 3
PREC_NAMES = {CBH_PREC_FP32: "fp32", CBH_PREC_TWOFLOAT: "twofloat", CBH_PREC_INT16: "int16",
              CBH_PREC_F64: "f64"}
STATUS_NAMES = {0: "CBH_OK", -1: "CBH_EINVAL", -2: "CBH_ENOMEM", -3: "CBH_EDEVICE",
                -4: "CBH_EOVERFLOW", -5: "CBH_EUNSUPPORTED", -6: "CBH_EBUSY"}

# Every symbol include/cbhip.h declares.
EXPORTS = [
    "cbh_create", "cbh_destroy", "cbh_last_error", "cbh_set_workspace_limit",
    "cbh_workspace_size", "cbh_reserve_workspace", "cbh_sync", "cbh_probe_lds_rates",
    "cbh_device_timestamp", "cbh_device_clock_khz",
    "cbh_select_borders", "cbh_uniform_borders",
    "cbh_quantize", "cbh_tile_bins",
    "cbh_compute_ordered_ts", "cbh_quantize_gradients", "cbh_build_histograms",
    "cbh_build_histograms_sub", "cbh_apply_build_histograms_sub",
    "cbh_score_splits", "cbh_score_splits_noalloc", "cbh_apply_split", "cbh_update_approx", "cbh_batch_create",
    "cbh_batch_destroy", "cbh_batch_level", "cbh_batch_update", "cbh_batch_set_fused",
    "cbh_graph_capture_iteration", "cbh_graph_launch", "cbh_graph_destroy",
    "cbh_fit_tree", "cbh_graph_capture_tree",
    "cbh_autotune", "cbh_autotune_load", "cbh_set_hist_knobs",
    "cbh_part_create", "cbh_part_destroy", "cbh_part_split", "cbh_part_build_histograms",
    "cbh_part_build_histograms_sub",
    "cbh_apply_model", "cbh_combine_categories", "cbh_category_counts", "cbh_pack_bins",
    "cbh_ordered_models", "cbh_ordered_offset", "cbh_ordered_support_size",
    "cbh_ordered_gradients", "cbh_ordered_update", "cbh_fit_tree_ordered",
    "cbh_split_values", "cbh_ts_bins", "cbh_binarize", "cbh_apply_model_binarized",
    "cbh_graph_begin", "cbh_graph_end", "cbh_category_order", "cbh_ordered_ts_crossings",
    "cbh_counter_bins",
]


class cbh_problem(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("n_features", C.c_int32), ("max_bins", C.c_int32),
        ("bins", C.c_void_p), ("n_bins", C.c_void_p), ("K", C.c_int32),
        ("loss", C.c_int32), ("depth", C.c_int32), ("bin_bits", C.c_int32),
        ("label", C.c_void_p), ("g", C.c_void_p), ("h", C.c_void_p),
        ("gq", C.c_void_p), ("grad_scale", C.c_void_p), ("leaf", C.c_void_p),
        ("approx", C.c_void_p), ("seg_stride", C.c_void_p), ("weight", C.c_void_p),
    ]


class cbh_ordered(C.Structure):
    _fields_ = [("n", C.c_int64), ("perm", C.c_void_p), ("support", C.c_void_p)]


class cbh_split(C.Structure):
    _fields_ = [("feature", C.c_int32), ("border", C.c_int32), ("score", C.c_float),
                ("margin", C.c_float)]


CBH_SOURCE_BINS, CBH_SOURCE_VALUES, CBH_SOURCE_PAIR = 0, 1, 2


class cbh_split_source(C.Structure):
    _fields_ = [("ptr", C.c_void_p), ("ptr_b", C.c_void_p), ("seg_stride", C.c_int64),
                ("kind", C.c_int32), ("reserved", C.c_int32)]


class CbhError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1810_11363_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    i32, i64, dbl, vp = C.c_int32, C.c_int64, C.c_double, C.c_void_p
    sig = {
        "cbh_create": ([C.c_int, C.POINTER(vp)], C.c_int),
        "cbh_destroy": ([vp], None),
        "cbh_last_error": ([], C.c_char_p),
        "cbh_set_workspace_limit": ([vp, i64], C.c_int),
        "cbh_workspace_size": ([vp], i64),
        "cbh_reserve_workspace": ([vp, i64], C.c_int),
        "cbh_sync": ([vp, vp], C.c_int),
        "cbh_device_timestamp": ([vp, vp, vp], C.c_int),
        "cbh_device_clock_khz": ([vp, C.POINTER(i64)], C.c_int),
        "cbh_probe_lds_rates": ([vp, C.POINTER(dbl)], C.c_int),
        "cbh_select_borders": ([vp, i64, i32, vp, C.POINTER(i32)], C.c_int),
        "cbh_uniform_borders": ([dbl, dbl, i32, vp], C.c_int),
        "cbh_quantize": ([vp, vp, i64, vp, i32, vp, vp], C.c_int),
        "cbh_tile_bins": ([vp, vp, i32, i64, vp, vp], C.c_int),
        "cbh_compute_ordered_ts": ([vp, vp, vp, i64, vp, i32, i32, i64, dbl, vp, vp, i32,
                                    vp, vp, vp, vp, vp], C.c_int),
        "cbh_quantize_gradients": ([vp, C.POINTER(cbh_problem), vp], C.c_int),
        "cbh_build_histograms": ([vp, C.POINTER(cbh_problem), i32, i32, vp, vp], C.c_int),
        "cbh_build_histograms_sub": ([vp, C.POINTER(cbh_problem), i32, i32, vp, vp, vp, vp],
                                     C.c_int),
        "cbh_apply_build_histograms_sub": ([vp, C.POINTER(cbh_problem), i32, i32, vp, vp, vp,
                                            vp], C.c_int),
        "cbh_score_splits": ([vp, C.POINTER(cbh_problem), i32, vp, i32, dbl, vp, vp, vp],
                             C.c_int),
        "cbh_score_splits_noalloc": ([vp, C.POINTER(cbh_problem), i32, vp, i32, dbl, vp, vp,
                                      vp], C.c_int),
        "cbh_apply_split": ([vp, C.POINTER(cbh_problem), i32, vp, vp], C.c_int),
        "cbh_update_approx": ([vp, C.POINTER(cbh_problem), vp, i32, vp, dbl, dbl, vp, vp, vp],
                              C.c_int),
        "cbh_apply_model": ([vp, vp, vp, i64, i32, i32, i32, i32, vp, vp, vp, dbl, vp, vp],
                            C.c_int),
        "cbh_combine_categories": ([vp, vp, vp, i64, vp, vp, vp], C.c_int),
        "cbh_category_counts": ([vp, vp, i64, vp, vp], C.c_int),
        "cbh_split_values": ([vp, vp, vp, i32, i64, vp, vp, vp], C.c_int),
        "cbh_category_order": ([vp, vp, vp, i64, vp, vp, vp, vp], C.c_int),
        "cbh_ordered_ts_crossings": ([vp, vp, i32, i32, vp, vp, i64, vp, i32, i32, i64, dbl, i32,
                                      vp, vp, i32, i32, vp, i64, vp], C.c_int),
        "cbh_counter_bins": ([vp, vp, i64, i32, vp, vp], C.c_int),
        "cbh_binarize": ([vp, vp, vp, i64, i32, i32, vp, vp, vp, vp], C.c_int),
        "cbh_apply_model_binarized": ([vp, vp, i64, i32, i32, i32, i32, vp, vp, dbl, vp, vp],
                                      C.c_int),
        "cbh_ts_bins": ([vp, vp, vp, i64, i32, dbl, dbl, vp, i32, vp, vp, vp], C.c_int),
        "cbh_batch_create": ([vp, C.POINTER(cbh_problem), i32, i32, i32, vp, vp, C.POINTER(vp)],
                             C.c_int),
        "cbh_batch_destroy": ([vp], None),
        "cbh_batch_level": ([vp, vp, i32, dbl, vp], C.c_int),
        "cbh_batch_set_fused": ([vp, i32], C.c_int),
        "cbh_batch_update": ([vp, vp, dbl, dbl, vp, i32, vp], C.c_int),
        "cbh_graph_capture_iteration": ([vp, vp, dbl, dbl, vp, vp, C.POINTER(vp)], C.c_int),
        "cbh_graph_launch": ([vp, vp], C.c_int),
        "cbh_graph_begin": ([vp, vp], C.c_int),
        "cbh_graph_end": ([vp, vp, C.POINTER(vp)], C.c_int),
        "cbh_fit_tree": ([vp, C.POINTER(cbh_problem), vp, i32, i32, vp, vp, dbl, dbl, vp, vp,
                          vp, vp], C.c_int),
        "cbh_graph_capture_tree": ([vp, C.POINTER(cbh_problem), vp, i32, i32, vp, vp, dbl, dbl,
                                    vp, vp, vp, vp, C.POINTER(vp)], C.c_int),
        "cbh_graph_destroy": ([vp], None),
        "cbh_pack_bins": ([vp, vp, vp, i32, i64, i32, vp, vp], C.c_int),
        "cbh_ordered_models": ([i64], i32),
        "cbh_ordered_offset": ([i64, i32], i64),
        "cbh_ordered_support_size": ([i64], i64),
        "cbh_ordered_gradients": ([vp, C.POINTER(cbh_ordered), C.POINTER(cbh_problem), vp],
                                  C.c_int),
        "cbh_ordered_update": ([vp, C.POINTER(cbh_ordered), C.POINTER(cbh_problem), dbl, dbl,
                                vp, vp, vp], C.c_int),
        "cbh_fit_tree_ordered": ([vp, C.POINTER(cbh_problem), C.POINTER(cbh_ordered), vp, i32,
                                  i32, vp, vp, dbl, dbl, vp, vp, vp], C.c_int),
        "cbh_autotune": ([vp, C.POINTER(cbh_problem), i32, i32, C.c_char_p, vp], C.c_int),
        "cbh_autotune_load": ([vp, C.c_char_p], C.c_int),
        "cbh_set_hist_knobs": ([vp, i32, i32, i64, i32, i32, i32, i32, i32], C.c_int),
        "cbh_part_create": ([vp, C.POINTER(cbh_problem), C.POINTER(vp)], C.c_int),
        "cbh_part_destroy": ([vp], None),
        "cbh_part_split": ([vp, vp, C.POINTER(cbh_problem), i32, i32, vp, vp], C.c_int),
        "cbh_part_build_histograms": ([vp, vp, C.POINTER(cbh_problem), i32, i32, vp, vp],
                                      C.c_int),
        "cbh_part_build_histograms_sub": ([vp, vp, C.POINTER(cbh_problem), i32, i32, vp, vp,
                                           vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(f"cannot take a pointer of {type(x)}")


def _stream(s):
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _check(rc):
    if rc != CBH_OK:
        raise CbhError(rc, _lib.cbh_last_error().decode())
    return rc


# ---------------------------------------------------------------- context
def cbh_create(device: int = 0):
    h = C.c_void_p()
    _check(_lib.cbh_create(device, C.byref(h)))
    return h.value


def cbh_destroy(ctx):
    _lib.cbh_destroy(ctx)


def cbh_last_error() -> str:
    return _lib.cbh_last_error().decode()


def cbh_set_workspace_limit(ctx, nbytes: int):
    return _check(_lib.cbh_set_workspace_limit(ctx, nbytes))


def cbh_workspace_size(ctx) -> int:
    return _lib.cbh_workspace_size(ctx)


def cbh_reserve_workspace(ctx, nbytes: int):
    return _check(_lib.cbh_reserve_workspace(ctx, nbytes))


def cbh_sync(ctx, stream=None):
    return _check(_lib.cbh_sync(ctx, _stream(stream)))


# ---------------------------------------------------------- preprocessing
def cbh_select_borders(x_host, max_bins: int):
    """x_host: contiguous float32 numpy array. Returns a float32 numpy array."""
    import numpy as np
    x = np.ascontiguousarray(x_host, dtype=np.float32)
    out = np.zeros(max(1, max_bins - 1), np.float32)
    nb = C.c_int32(0)
    _check(_lib.cbh_select_borders(x.ctypes.data, x.size, max_bins, out.ctypes.data,
                                   C.byref(nb)))
    return out[: nb.value].copy()


def cbh_uniform_borders(lo: float, hi: float, n_bins: int):
    """Returns a float64 numpy array of n_bins-1 uniform borders."""
    import numpy as np
    out = np.zeros(max(1, n_bins - 1), np.float64)
    _check(_lib.cbh_uniform_borders(float(lo), float(hi), n_bins, out.ctypes.data))
    return out[: n_bins - 1].copy()


def cbh_quantize(ctx, x, n: int, borders, n_borders: int, bins_out, stream=None):
    return _check(_lib.cbh_quantize(ctx, _ptr(x), n, _ptr(borders), n_borders, _ptr(bins_out),
                                    _stream(stream)))


def cbh_device_timestamp(ctx, slot, stream=None):
    return _check(_lib.cbh_device_timestamp(ctx, _ptr(slot), _stream(stream)))


def cbh_device_clock_khz(ctx) -> int:
    v = C.c_int64()
    _check(_lib.cbh_device_clock_khz(ctx, C.byref(v)))
    return v.value


LDS_RATE_NAMES = ("ds_add_u32", "ds_add_f32", "ds_add_f64", "ds_add_u64", "cas32_f32",
                  "cas64_pair")


def cbh_probe_lds_rates(ctx) -> dict:
    """Measured LDS update rates (lane updates per clock per CU), by name."""
    r = (C.c_double * 6)()
    _check(_lib.cbh_probe_lds_rates(ctx, r))
    return dict(zip(LDS_RATE_NAMES, (float(v) for v in r)))


def cbh_tile_bins(ctx, cols, n_cols: int, n: int, out, stream=None):
    """cols: device int64 tensor (or address) of n_cols column pointers."""
    return _check(_lib.cbh_tile_bins(ctx, _ptr(cols), n_cols, n, _ptr(out), _stream(stream)))


def cbh_compute_ordered_ts(ctx, cat, perm, n: int, y_num, n_targets: int, y_shift: int,
                           y_abs_max: int, a: float, priors, ts_borders, n_ts_borders: int,
                           num_out=None, den_out=None, ts_bin_out=None, ts_out=None,
                           stream=None):
    pri = (C.c_double * n_targets)(*[float(p) for p in priors])
    return _check(_lib.cbh_compute_ordered_ts(
        ctx, _ptr(cat), _ptr(perm), n, _ptr(y_num), n_targets, y_shift, y_abs_max, float(a),
        C.cast(pri, C.c_void_p), _ptr(ts_borders), n_ts_borders, _ptr(num_out), _ptr(den_out),
        _ptr(ts_bin_out), _ptr(ts_out), _stream(stream)))


# ------------------------------------------------------------- split search
def cbh_quantize_gradients(ctx, prob: cbh_problem, stream=None):
    return _check(_lib.cbh_quantize_gradients(ctx, C.byref(prob), _stream(stream)))


def cbh_build_histograms(ctx, prob: cbh_problem, level: int, precision: int, hist_out,
                         stream=None):
    return _check(_lib.cbh_build_histograms(ctx, C.byref(prob), level, precision,
                                            _ptr(hist_out), _stream(stream)))


def cbh_part_create(ctx, prob: cbh_problem):
    out = C.c_void_p()
    _check(_lib.cbh_part_create(ctx, C.byref(prob), C.byref(out)))
    return out.value


def cbh_part_destroy(part):
    _lib.cbh_part_destroy(part)


def cbh_part_split(ctx, part, prob: cbh_problem, level: int, precision: int, split,
                   stream=None):
    return _check(_lib.cbh_part_split(ctx, part, C.byref(prob), level, precision, _ptr(split),
                                      _stream(stream)))


def cbh_part_build_histograms(ctx, part, prob: cbh_problem, level: int, precision: int,
                              hist_out, stream=None):
    return _check(_lib.cbh_part_build_histograms(ctx, part, C.byref(prob), level, precision,
                                                 _ptr(hist_out), _stream(stream)))


def cbh_part_build_histograms_sub(ctx, part, prob: cbh_problem, level: int, precision: int,
                                  parent_hist, hist_out, stream=None):
    return _check(_lib.cbh_part_build_histograms_sub(ctx, part, C.byref(prob), level, precision,
                                                     _ptr(parent_hist), _ptr(hist_out),
                                                     _stream(stream)))


def cbh_build_histograms_sub(ctx, prob: cbh_problem, level: int, precision: int, parent_hist,
                             parent_split, hist_out, stream=None):
    return _check(_lib.cbh_build_histograms_sub(ctx, C.byref(prob), level, precision,
                                                _ptr(parent_hist), _ptr(parent_split),
                                                _ptr(hist_out), _stream(stream)))


def cbh_apply_build_histograms_sub(ctx, prob: cbh_problem, level: int, precision: int,
                                   parent_hist, parent_split, hist_out, stream=None):
    return _check(_lib.cbh_apply_build_histograms_sub(ctx, C.byref(prob), level, precision,
                                                      _ptr(parent_hist), _ptr(parent_split),
                                                      _ptr(hist_out), _stream(stream)))


def cbh_score_splits(ctx, prob: cbh_problem, level: int, hist, precision: int, l2: float,
                     best_out, scores_out=None, stream=None):
    return _check(_lib.cbh_score_splits(ctx, C.byref(prob), level, _ptr(hist), precision,
                                        float(l2), _ptr(best_out), _ptr(scores_out),
                                        _stream(stream)))


def cbh_score_splits_noalloc(ctx, prob: cbh_problem, level: int, hist, precision: int, l2: float,
                             best_out, scores_out=None, stream=None):
    return _check(_lib.cbh_score_splits_noalloc(ctx, C.byref(prob), level, _ptr(hist),
                                                precision, float(l2), _ptr(best_out),
                                                _ptr(scores_out), _stream(stream)))


def cbh_apply_split(ctx, prob: cbh_problem, level: int, best, stream=None):
    return _check(_lib.cbh_apply_split(ctx, C.byref(prob), level, _ptr(best), _stream(stream)))


def cbh_update_approx(ctx, prob: cbh_problem, hist_last, precision: int, last, lr: float,
                      l2: float, leaf_values_out=None, leaf_counts_out=None, stream=None):
    return _check(_lib.cbh_update_approx(ctx, C.byref(prob), _ptr(hist_last), precision,
                                         _ptr(last), float(lr), float(l2),
                                         _ptr(leaf_values_out), _ptr(leaf_counts_out),
                                         _stream(stream)))


def cbh_apply_model(ctx, bins, seg_stride, n: int, n_features: int, K: int, n_trees: int,
                    depth: int, split_feature, split_border, leaf_values, lr: float, approx,
                    stream=None):
    return _check(_lib.cbh_apply_model(ctx, _ptr(bins), _ptr(seg_stride), int(n),
                                       int(n_features), int(K), int(n_trees), int(depth),
                                       _ptr(split_feature), _ptr(split_border),
                                       _ptr(leaf_values), float(lr), _ptr(approx),
                                       _stream(stream)))


# ------------------------------------------------------------------ batched
def cbh_batch_create(ctx, probs, precision: int, hist_ptrs, best, subtract=None):
    """subtract: None builds levels >= 1 by subtraction for the two-float and
    int16 forms (not for plain float32), as the single-problem trees do."""
    P = len(probs)
    if subtract is None:
        subtract = precision != CBH_PREC_FP32
    arr = (cbh_problem * P)(*probs)
    hp = (C.c_void_p * P)(*[_ptr(h) for h in hist_ptrs])
    out = C.c_void_p()
    _check(_lib.cbh_batch_create(ctx, arr, P, precision, int(bool(subtract)),
                                 C.cast(hp, C.c_void_p), _ptr(best), C.byref(out)))
    return out.value


def cbh_batch_destroy(batch):
    _lib.cbh_batch_destroy(batch)


def cbh_batch_level(ctx, batch, level: int, l2: float, stream=None):
    return _check(_lib.cbh_batch_level(ctx, batch, level, float(l2), _stream(stream)))


def cbh_batch_update(ctx, batch, lr: float, l2: float, leaf_values, init: bool, stream=None):
    P = len(leaf_values)
    lv = (C.c_void_p * P)(*[_ptr(v) for v in leaf_values])
    return _check(_lib.cbh_batch_update(ctx, batch, float(lr), float(l2),
                                        C.cast(lv, C.c_void_p), int(bool(init)),
                                        _stream(stream)))


def cbh_batch_set_fused(batch, fused: bool):
    return _check(_lib.cbh_batch_set_fused(batch, int(bool(fused))))


def cbh_graph_capture_iteration(ctx, batch, lr: float, l2: float, leaf_values, stream=None):
    P = len(leaf_values)
    lv = (C.c_void_p * P)(*[_ptr(v) for v in leaf_values])
    out = C.c_void_p()
    _check(_lib.cbh_graph_capture_iteration(ctx, batch, float(lr), float(l2),
                                            C.cast(lv, C.c_void_p), _stream(stream),
                                            C.byref(out)))
    return out.value


def _two(hist):
    arr = (C.c_void_p * 2)(_ptr(hist[0]), _ptr(hist[1]))
    return arr


def cbh_fit_tree(ctx, prob: cbh_problem, part, precision: int, subtract: bool, hist, best,
                 lr: float, l2: float, leaf_values, leaf_counts=None, stamps=None, stream=None):
    arr = _two(hist)
    return _check(_lib.cbh_fit_tree(ctx, C.byref(prob), part, precision, int(bool(subtract)),
                                    C.cast(arr, C.c_void_p), _ptr(best), float(lr), float(l2),
                                    _ptr(leaf_values), _ptr(leaf_counts), _ptr(stamps),
                                    _stream(stream)))


def cbh_graph_capture_tree(ctx, prob: cbh_problem, part, precision: int, subtract: bool, hist,
                           best, lr: float, l2: float, leaf_values, leaf_counts=None,
                           stamps=None, stream=None):
    arr = _two(hist)
    out = C.c_void_p()
    _check(_lib.cbh_graph_capture_tree(ctx, C.byref(prob), part, precision, int(bool(subtract)),
                                       C.cast(arr, C.c_void_p), _ptr(best), float(lr), float(l2),
                                       _ptr(leaf_values), _ptr(leaf_counts), _ptr(stamps),
                                       _stream(stream), C.byref(out)))
    return out.value


def cbh_pack_bins(ctx, bins_table, seg_stride, n_features: int, n: int, bits: int,
                  packed_table, stream=None):
    return _check(_lib.cbh_pack_bins(ctx, _ptr(bins_table), _ptr(seg_stride), int(n_features),
                                     int(n), int(bits), _ptr(packed_table), _stream(stream)))


def cbh_ordered_models(n: int) -> int:
    return int(_lib.cbh_ordered_models(int(n)))


def cbh_ordered_offset(n: int, m: int) -> int:
    return int(_lib.cbh_ordered_offset(int(n), int(m)))


def cbh_ordered_support_size(n: int) -> int:
    return int(_lib.cbh_ordered_support_size(int(n)))


def make_ordered(n: int, perm, support) -> cbh_ordered:
    return cbh_ordered(n=int(n), perm=_ptr(perm), support=_ptr(support))


def cbh_ordered_gradients(ctx, ord_: cbh_ordered, prob: cbh_problem, stream=None):
    return _check(_lib.cbh_ordered_gradients(ctx, C.byref(ord_), C.byref(prob),
                                             _stream(stream)))


def cbh_ordered_update(ctx, ord_: cbh_ordered, prob: cbh_problem, lr: float, l2: float,
                       leaf_values, support_values=None, stream=None):
    return _check(_lib.cbh_ordered_update(ctx, C.byref(ord_), C.byref(prob), float(lr),
                                          float(l2), _ptr(leaf_values), _ptr(support_values),
                                          _stream(stream)))


def cbh_fit_tree_ordered(ctx, prob: cbh_problem, ord_: cbh_ordered, part, precision: int,
                         subtract: bool, hist, best, lr: float, l2: float, leaf_values,
                         support_values=None, stream=None):
    arr = _two(hist)
    return _check(_lib.cbh_fit_tree_ordered(ctx, C.byref(prob), C.byref(ord_), part, precision,
                                            int(bool(subtract)), C.cast(arr, C.c_void_p),
                                            _ptr(best), float(lr), float(l2),
                                            _ptr(leaf_values), _ptr(support_values),
                                            _stream(stream)))


def cbh_graph_launch(graph, stream=None):
    return _check(_lib.cbh_graph_launch(graph, _stream(stream)))


def cbh_graph_destroy(graph):
    _lib.cbh_graph_destroy(graph)


def cbh_autotune(ctx, prob: cbh_problem, precision: int, subtract: bool = False,
                 cache_path=None, stream=None):
    return _check(_lib.cbh_autotune(ctx, C.byref(prob), precision, int(bool(subtract)),
                                    cache_path.encode() if cache_path else None,
                                    _stream(stream)))


def cbh_set_hist_knobs(ctx, lds_budget=0, target_blocks=512, min_rows=32768, partial_pct=25,
                       max_rep=32, rep_target=32, kernel=1, lpf_w=0):
    return _check(_lib.cbh_set_hist_knobs(ctx, lds_budget, target_blocks, min_rows,
                                          partial_pct, max_rep, rep_target, kernel, lpf_w))


def cbh_autotune_load(ctx, cache_path: str):
    return _check(_lib.cbh_autotune_load(ctx, cache_path.encode()))


def cbh_combine_categories(ctx, cat_a, cat_b, n: int, ids_out, n_distinct_out, stream=None):
    return _check(_lib.cbh_combine_categories(ctx, _ptr(cat_a), _ptr(cat_b), int(n),
                                              _ptr(ids_out), _ptr(n_distinct_out),
                                              _stream(stream)))


def cbh_category_counts(ctx, ids, n: int, counts_out, stream=None):
    return _check(_lib.cbh_category_counts(ctx, _ptr(ids), int(n), _ptr(counts_out),
                                           _stream(stream)))


def cbh_split_values(ctx, split, sources, n_sources: int, n: int, a_out, b_out, stream=None):
    return _check(_lib.cbh_split_values(ctx, _ptr(split), _ptr(sources), int(n_sources), int(n),
                                        _ptr(a_out), _ptr(b_out), _stream(stream)))


def cbh_category_order(ctx, cat, perm, n: int, order_out=None, ids_out=None,
                       n_distinct_out=None, stream=None):
    return _check(_lib.cbh_category_order(ctx, _ptr(cat), _ptr(perm), int(n), _ptr(order_out),
                                          _ptr(ids_out), _ptr(n_distinct_out), _stream(stream)))


def cbh_ordered_ts_crossings(ctx, e_ids, e_bits: int, n_cross: int, c_order, c_ids, n: int,
                             y_num, n_targets: int, y_shift: int, y_abs_max: int, a: float,
                             n_priors: int, priors, ts_borders, n_ts_borders: int, ts_bin_out,
                             ld: int, counter_bins: int = 0, stream=None):
    pri = (C.c_double * (n_targets * n_priors))(*[float(p) for p in priors])
    return _check(_lib.cbh_ordered_ts_crossings(
        ctx, _ptr(e_ids), int(e_bits), int(n_cross), _ptr(c_order), _ptr(c_ids), int(n),
        _ptr(y_num), int(n_targets), int(y_shift), int(y_abs_max), float(a), int(n_priors),
        C.cast(pri, C.c_void_p), _ptr(ts_borders), int(n_ts_borders), int(counter_bins),
        _ptr(ts_bin_out), int(ld), _stream(stream)))


def cbh_counter_bins(ctx, counts, n: int, n_bins: int, bins_out, stream=None):
    return _check(_lib.cbh_counter_bins(ctx, _ptr(counts), int(n), int(n_bins), _ptr(bins_out),
                                        _stream(stream)))


def cbh_ts_bins(ctx, num, den, n: int, y_shift: int, a: float, prior: float, ts_borders,
                n_ts_borders: int, ts_bin_out=None, ts_out=None, stream=None):
    return _check(_lib.cbh_ts_bins(ctx, _ptr(num), _ptr(den), int(n), int(y_shift), float(a),
                                   float(prior), _ptr(ts_borders), int(n_ts_borders),
                                   _ptr(ts_bin_out), _ptr(ts_out), _stream(stream)))


def cbh_binarize(ctx, bins, seg_stride, n: int, n_features: int, n_binary: int, bin_feature,
                 bin_border, bits_out, stream=None):
    return _check(_lib.cbh_binarize(ctx, _ptr(bins), _ptr(seg_stride), int(n), int(n_features),
                                    int(n_binary), _ptr(bin_feature), _ptr(bin_border),
                                    _ptr(bits_out), _stream(stream)))


def cbh_apply_model_binarized(ctx, bits, n: int, n_binary: int, K: int, n_trees: int,
                              depth: int, split_binary, leaf_values, lr: float, approx,
                              stream=None):
    return _check(_lib.cbh_apply_model_binarized(
        ctx, _ptr(bits), int(n), int(n_binary), int(K), int(n_trees), int(depth),
        _ptr(split_binary), _ptr(leaf_values), float(lr), _ptr(approx), _stream(stream)))


def cbh_graph_begin(ctx, stream):
    return _check(_lib.cbh_graph_begin(ctx, _stream(stream)))


def cbh_graph_end(ctx, stream):
    g = C.c_void_p()
    _check(_lib.cbh_graph_end(ctx, _stream(stream), C.byref(g)))
    return g.value
