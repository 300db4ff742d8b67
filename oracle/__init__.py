"""CPU FP64 oracle for the oblivious-tree split search and ordered target
statistics of arXiv:1810.11363 (CatBoost).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``. The GPU library never imports,
links or calls anything here, and nothing here imports the GPU library.

The arithmetic lives in ``oracle.c`` (plain loops, double precision); this
module is argument marshalling through ctypes plus ``boost.py``'s loop that
chains the steps into trees.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        _lib = C.CDLL(path)
        _declare(_lib)
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _declare(L):
    i64, i32, dbl, vp = C.c_int64, C.c_int32, C.c_double, C.c_void_p
    L.orc_select_borders.argtypes = [vp, i64, i32, vp, vp]
    L.orc_select_borders.restype = C.c_int
    L.orc_quantize.argtypes = [vp, i64, vp, i32, vp]
    L.orc_ts_borders.argtypes = [dbl, dbl, i32, vp]
    L.orc_ordered_ts.argtypes = [vp, vp, vp, i64, i32, dbl, dbl, vp, i32, vp, vp, vp, vp]
    L.orc_ordered_ts.restype = C.c_int
    L.orc_gradients.argtypes = [i32, i32, i64, vp, vp, vp, vp]
    L.orc_histogram.argtypes = [i64, i32, vp, i32, i32, vp, vp, vp, i32, vp]
    L.orc_score.argtypes = [i32, i32, i32, i32, vp, vp, dbl, vp]
    L.orc_best_split.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp]
    L.orc_apply_split.argtypes = [i64, vp, i32, i32, vp]
    L.orc_leaf_values.argtypes = [i64, i32, i32, vp, vp, vp, dbl, vp, vp, vp, vp]
    L.orc_update_approx.argtypes = [i64, i32, vp, vp, dbl, vp]
    L.orc_grad_codes.argtypes = [i64, i32, vp, vp, i32, vp, vp, vp]
    L.orc_histogram_int.argtypes = [i64, i32, vp, i32, i32, vp, vp, vp, i32, vp]
    L.orc_apply_model.argtypes = [i64, i32, vp, i32, i32, i32, vp, vp, vp, dbl, vp]
    L.orc_ordered_models.argtypes = [i64]
    L.orc_ordered_models.restype = i32
    L.orc_ordered_offset.argtypes = [i64, i32]
    L.orc_ordered_offset.restype = i64
    L.orc_ordered_gradients.argtypes = [i32, i32, i64, vp, vp, vp, vp, vp]
    L.orc_ordered_update.argtypes = [i32, i32, i64, vp, vp, vp, i32, dbl, dbl, vp, vp]
    L.orc_pack_bins.argtypes = [vp, i64, i32, vp]
    L.orc_num_threads.restype = C.c_int
    L.orc_set_threads.argtypes = [i32]


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(t: int) -> None:
    """Threads of the oracle's parallel loops (its results do not depend on it)."""
    lib().orc_set_threads(int(t))


def select_borders(x, max_bins: int) -> np.ndarray:
    """Value-at-rank quantile borders of one numeric column (Sec. 5)."""
    x = _c(x, np.float32)
    out = np.zeros(max(1, max_bins), np.float32)
    nb = C.c_int32(0)
    rc = lib().orc_select_borders(_p(x), x.size, max_bins, _p(out), C.byref(nb))
    if rc != 0:
        raise ValueError(f"orc_select_borders failed ({rc})")
    return out[: nb.value].copy()


def quantize(x, borders) -> np.ndarray:
    x = _c(x, np.float32)
    borders = _c(borders, np.float32)
    out = np.empty(x.size, np.uint8)
    lib().orc_quantize(_p(x), x.size, _p(borders), borders.size, _p(out))
    return out


def ts_borders(lo: float, hi: float, n_bins: int) -> np.ndarray:
    out = np.zeros(max(1, n_bins - 1), np.float64)
    lib().orc_ts_borders(float(lo), float(hi), n_bins, _p(out))
    return out[: n_bins - 1].copy()


def ordered_ts(cat, perm, y_num, y_shift: int, a: float, prior: float, borders=None):
    """Eq. (1): returns (num int64, den int32, ts float64, ts_bin uint8|None)."""
    cat = _c(cat, np.int32)
    perm = _c(perm, np.int32)
    y_num = _c(y_num, np.int64)
    n = cat.size
    num = np.empty(n, np.int64)
    den = np.empty(n, np.int32)
    ts = np.empty(n, np.float64)
    tb = np.empty(n, np.uint8) if borders is not None else None
    b = _c(borders, np.float64) if borders is not None else np.zeros(1)
    nb = b.size if borders is not None else 0
    rc = lib().orc_ordered_ts(_p(cat), _p(perm), _p(y_num), n, y_shift, float(a),
                              float(prior), _p(b), nb, _p(num), _p(den), _p(ts), _p(tb))
    if rc != 0:
        raise ValueError(f"orc_ordered_ts failed ({rc})")
    return num, den, ts, tb


def gradients(loss: int, K: int, approx, label):
    """Loss derivatives at approx [K][n] -> (g, h) float64 [K][n]."""
    approx = _c(approx, np.float64).reshape(K, -1)
    label = _c(label, np.float32)
    n = label.size
    g = np.empty((K, n), np.float64)
    h = np.empty((K, n), np.float64)
    lib().orc_gradients(loss, K, n, _p(approx), _p(label), _p(g), _p(h))
    return g, h


def histogram(bins, g, h, leaf, n_leaves: int, B: int):
    """hist[L][F][B][2K] float64 of (sum g_c, sum h_c) per leaf, feature, bin."""
    bins = _c(bins, np.uint8)
    F, n = bins.shape
    g = _c(g, np.float64).reshape(-1, n)
    h = _c(h, np.float64).reshape(-1, n)
    K = g.shape[0]
    leaf = _c(leaf, np.uint16)
    out = np.empty((n_leaves, F, B, 2 * K), np.float64)
    lib().orc_histogram(n, F, _p(bins), B, K, _p(g), _p(h), _p(leaf), n_leaves, _p(out))
    return out


def score(hist, n_bins, l2: float):
    """scores [F][B-1] float64 of every candidate split; -inf where invalid."""
    hist = _c(hist, np.float64)
    L, F, B, S = hist.shape
    n_bins = _c(n_bins, np.int32)
    out = np.empty((F, max(1, B - 1)), np.float64)
    lib().orc_score(L, F, B, S // 2, _p(hist), _p(n_bins), float(l2), _p(out))
    return out[:, : B - 1]


def best_split(scores, n_bins):
    """(feature, border, best score, second-best score); (-1, -1, ...) if none."""
    scores = _c(scores, np.float64)
    F, Bm1 = scores.shape
    n_bins = _c(n_bins, np.int32)
    bf, bk = C.c_int32(), C.c_int32()
    s1, s2 = C.c_double(), C.c_double()
    lib().orc_best_split(F, Bm1 + 1, _p(scores), _p(n_bins), C.byref(bf), C.byref(bk),
                         C.byref(s1), C.byref(s2))
    return bf.value, bk.value, s1.value, s2.value


def apply_split(bin_col, k: int, level: int, leaf):
    """In place: leaf |= [bin > k] << level."""
    bin_col = _c(bin_col, np.uint8)
    assert leaf.dtype == np.uint16 and leaf.flags.c_contiguous
    lib().orc_apply_split(bin_col.size, _p(bin_col), int(k), int(level), _p(leaf))
    return leaf


def leaf_values(leaf, g, h, n_leaves: int, l2: float):
    """Direct per-leaf sums and Newton leaf values -G/(H+l2).
    Returns (values [L][K], G [L][K], H [L][K], counts [L])."""
    leaf = _c(leaf, np.uint16)
    n = leaf.size
    g = _c(g, np.float64).reshape(-1, n)
    h = _c(h, np.float64).reshape(-1, n)
    K = g.shape[0]
    G = np.empty((n_leaves, K)); H = np.empty((n_leaves, K))
    cnt = np.empty(n_leaves, np.int64); val = np.empty((n_leaves, K))
    lib().orc_leaf_values(n, K, n_leaves, _p(leaf), _p(g), _p(h), float(l2),
                          _p(G), _p(H), _p(cnt), _p(val))
    return val, G, H, cnt


def update_approx(approx, leaf, values, lr: float):
    """In place: approx[c][i] += lr * values[leaf[i]][c]."""
    assert approx.dtype == np.float64 and approx.flags.c_contiguous
    K = approx.shape[0] if approx.ndim == 2 else 1
    leaf = _c(leaf, np.uint16)
    values = _c(values, np.float64)
    lib().orc_update_approx(leaf.size, K, _p(leaf), _p(values), float(lr), _p(approx))
    return approx


def apply_model(bins, feat, border, values, lr: float, approx):
    """In place: approx[c][i] += lr * values[t][leaf_t(i)][c] for every tree t in
    order, leaf_t(i) = sum_l 2^l [bins[feat[t][l]][i] > border[t][l]] (Sec. 4).
    bins [F][n] uint8, feat / border [T][d] int32, values [T][2^d][K] float64,
    approx [K][n] float64."""
    bins = _c(bins, np.uint8)
    F, n = bins.shape
    feat = _c(feat, np.int32)
    border = _c(border, np.int32)
    T, d = feat.shape
    assert border.shape == (T, d) and (T == 0 or (feat.min() >= 0 and feat.max() < F))
    values = _c(values, np.float64).reshape(T, 1 << d, -1)
    K = values.shape[2]
    assert approx.dtype == np.float64 and approx.flags.c_contiguous and approx.size == K * n
    lib().orc_apply_model(n, F, _p(bins), T, d, K, _p(feat), _p(border), _p(values),
                          float(lr), _p(approx))
    return approx


def binarize(bins, bin_feature, bin_border) -> np.ndarray:
    """The scorer's binary features (Sec. 4: every (feature, border) pair a
    model uses becomes one binary feature of every row): uint32
    [n_binary][ceil(n/32)], bit r of word w = [bins[f_j][32 w + r] > k_j],
    rows past n zero."""
    bins = np.asarray(bins, np.uint8)
    n = bins.shape[1]
    nw = (n + 31) // 32
    out = np.zeros((len(bin_feature), nw), np.uint32)
    weight = np.uint32(1) << np.arange(32, dtype=np.uint32)
    for j, (f, k) in enumerate(zip(bin_feature, bin_border)):
        b = np.zeros(nw * 32, np.uint32)
        b[:n] = bins[int(f)].astype(np.int64) > int(k)
        out[j] = (b.reshape(nw, 32) * weight).sum(axis=1, dtype=np.uint64).astype(np.uint32)
    return out


def combine_categories(cat_a, cat_b):
    """Dense ids of category pairs (the perfect hash of feature combinations,
    Sec. 2): equal pairs share an id, ids 0..m-1 in increasing order of
    ((uint32) a, (uint32) b). Returns (ids int32 [n], m)."""
    a = np.ascontiguousarray(cat_a, np.int32).view(np.uint32).astype(np.uint64)
    b = np.ascontiguousarray(cat_b, np.int32).view(np.uint32).astype(np.uint64)
    key = (a << np.uint64(32)) | b
    uniq, inv = np.unique(key, return_inverse=True)
    return inv.astype(np.int32).reshape(-1), int(uniq.size)


def category_counts(ids):
    """The counter statistic (Sec. 2): each row's number of rows with its id."""
    ids = np.ascontiguousarray(ids, np.int64).reshape(-1)
    return np.bincount(ids, minlength=1)[ids].astype(np.int32)


def grad_codes(g32, h32, with_h: bool):
    """int16 gradient codes with per-class scales (float32 decisions)."""
    g32 = _c(g32, np.float32)
    n = g32.shape[-1]
    g32 = g32.reshape(-1, n)
    K = g32.shape[0]
    h32 = _c(h32, np.float32).reshape(K, n) if h32 is not None else np.ones((K, n), np.float32)
    gq = np.empty((K, n), np.int16); hq = np.empty((K, n), np.int16)
    sc = np.empty((K, 2), np.float32)
    lib().orc_grad_codes(n, K, _p(g32), _p(h32), int(bool(with_h)), _p(gq), _p(hq), _p(sc))
    return gq, hq, sc


def histogram_int(bins, gq, hq, leaf, n_leaves: int, B: int):
    bins = _c(bins, np.uint8)
    F, n = bins.shape
    gq = _c(gq, np.int16).reshape(-1, n)
    hq = _c(hq, np.int16).reshape(-1, n)
    K = gq.shape[0]
    leaf = _c(leaf, np.uint16)
    out = np.empty((n_leaves, F, B, 2 * K), np.int64)
    lib().orc_histogram_int(n, F, _p(bins), B, K, _p(gq), _p(hq), _p(leaf), n_leaves, _p(out))
    return out


def ordered_models(n: int) -> int:
    """Number M of supporting approximations ordered boosting keeps for n
    positions (Sec. 3): model m learns from the first 2^(m-1) positions
    (none for m = 0) and is kept for the first min(n, 2^m)."""
    return int(lib().orc_ordered_models(int(n)))


def ordered_offsets(n: int) -> np.ndarray:
    """off[m] for m = 0..M: where model m's values start in a support row of
    S = off[M] doubles (position order)."""
    M = ordered_models(n)
    return np.array([lib().orc_ordered_offset(int(n), m) for m in range(M + 1)], np.int64)


def ordered_gradients(loss: int, K: int, perm, label, support):
    """(g, h) float64 [K][n] in row order: row perm[p] at the model that
    position p reads."""
    perm = _c(perm, np.int32)
    label = _c(label, np.float32)
    n = perm.size
    support = _c(support, np.float64).reshape(K, -1)
    g = np.empty((K, n), np.float64)
    h = np.empty((K, n), np.float64)
    lib().orc_ordered_gradients(loss, K, n, _p(perm), _p(label), _p(support), _p(g), _p(h))
    return g, h


def ordered_update(loss: int, K: int, perm, label, leaf, n_leaves: int, lr: float,
                   l2: float, support):
    """In place on support [K][S] (float64, C order): every supporting model
    takes its own leaf values for the tree whose row leaves are given and adds
    them to its kept positions. Returns the values [M][n_leaves][K]."""
    perm = _c(perm, np.int32)
    label = _c(label, np.float32)
    leaf = _c(leaf, np.uint16)
    n = perm.size
    assert support.dtype == np.float64 and support.flags.c_contiguous
    M = ordered_models(n)
    vals = np.empty((M, n_leaves, K), np.float64)
    lib().orc_ordered_update(loss, K, n, _p(perm), _p(label), _p(leaf), int(n_leaves),
                             float(lr), float(l2), _p(support), _p(vals))
    return vals


def pack_bins(bins, bits: int) -> np.ndarray:
    """The packed column (ceil(n/16) * 2 * bits bytes) of one feature's byte
    bins."""
    bins = _c(bins, np.uint8)
    n = bins.size
    out = np.empty(((n + 15) // 16) * 2 * bits, np.uint8)
    lib().orc_pack_bins(_p(bins), n, int(bits), _p(out))
    return out
