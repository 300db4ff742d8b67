"""Helpers for GPU tests: device buffers, problem descriptors and error metrics.

Tolerances follow one error model: a float32 sum is judged by its error
relative to the sum of the magnitudes of its terms (the summation condition
number), because cancelling gradient sums make a plain relative error
unbounded for any float32 accumulation.
"""
from __future__ import annotations

import numpy as np
import torch

FP32_TOL = 1e-5        # normalized error bound for float32 histogram sums and leaf values
TWOFLOAT_TOL = 1e-9    # compensated and float64-accumulated sums: exact to about 2^-46
MARGIN_TOL = 1e-5      # splits must agree where the oracle's top-two gap exceeds this

# histogram forms (CBH_PREC_*): float32, compensated float32, int16 codes,
# float64 LDS accumulation (written in the compensated form's (hi, lo) layout)
FP32, TWOFLOAT, INT16, F64 = 0, 1, 2, 3
PRECS = [FP32, TWOFLOAT, INT16, F64]


def pair_layout(precision):
    """True for the forms whose histograms hold (hi, lo) float pairs."""
    return precision in (TWOFLOAT, F64)


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def column_table(bins_dev):
    """int64 device table of column pointers of a [F][ld] uint8 device tensor."""
    return torch.tensor([bins_dev[f].data_ptr() for f in range(bins_dev.shape[0])],
                        dtype=torch.int64, device=dev())


def make_problem(cb, *, n, F, B, K, loss, depth, cols, nbins, label, g, h, leaf, approx,
                 gq=None, scale=None):
    p = cb.cbh_problem()
    p.n, p.n_features, p.max_bins = n, F, B
    p.bins, p.n_bins = cols.data_ptr(), nbins.data_ptr()
    p.K, p.loss, p.depth = K, loss, depth
    p.label, p.g, p.h = label.data_ptr(), g.data_ptr(), h.data_ptr()
    p.gq = gq.data_ptr() if gq is not None else None
    p.grad_scale = scale.data_ptr() if scale is not None else None
    p.leaf, p.approx = leaf.data_ptr(), approx.data_ptr()
    return p


def hist_to_f64(hist_dev, L, F, B, K, precision, rmse):
    """Device histogram -> float64 [L][F][B][2K] (counts as integers)."""
    if precision == 0:
        raw = hist_dev[: L * F * B * 2 * K * 4].view(torch.float32).cpu().numpy()
        out = raw.astype(np.float64).reshape(L, F, B, 2 * K)
        if rmse:
            u = hist_dev[: L * F * B * 2 * K * 4].view(torch.int32).cpu().numpy()
            out[..., 1::2] = u.reshape(L, F, B, 2 * K)[..., 1::2].astype(np.uint32)
        return out
    if pair_layout(precision):
        raw = hist_dev[: L * F * B * 2 * K * 8].view(torch.float32).cpu().numpy()
        pair = raw.reshape(L, F, B, 2 * K, 2).astype(np.float64)
        out = pair[..., 0] + pair[..., 1]
        if rmse:
            u = hist_dev[: L * F * B * 2 * K * 8].view(torch.int32).cpu().numpy()
            cnt = u.reshape(L, F, B, 2 * K, 2)[..., 0].astype(np.uint32)
            out[..., 1::2] = cnt[..., 1::2]
        return out
    raw = hist_dev[: L * F * B * 2 * K * 8].view(torch.int64).cpu().numpy()
    return raw.reshape(L, F, B, 2 * K)


# Allowance, relative to the bin's mass over all rows, for histograms built
# by subtraction (a sibling is its parent minus the accumulated child, so it
# carries the parent's rounding): compensated and float64 forms, plain float32.
SUB_SLACK_PAIR = 1e-12
SUB_SLACK_FP32 = 1e-5


def normalized_err(x, ref, mag, slack=None):
    """max |x - ref| / mag over cells; cells with mag == 0 must match exactly.
    With `slack` (an array broadcastable to x), that much absolute error is
    allowed in every cell first (a subtraction's share)."""
    x, ref, mag = np.asarray(x, np.float64), np.asarray(ref, np.float64), np.asarray(mag, np.float64)
    d = np.abs(x - ref)
    if slack is not None:
        d = np.maximum(d - np.asarray(slack, np.float64), 0.0)
    zero = mag == 0
    assert np.all(d[zero] == 0), "empty cells differ"
    if (~zero).sum() == 0:
        return 0.0
    return float(np.max(d[~zero] / mag[~zero]))


def cell_bound(precision, counts):
    """Normalised error bound of a histogram cell of m rows in a form:
    float32 sums in any order are within (m - 1) u of the sum of magnitudes
    (u = 2^-24, first order), so large cells may exceed FP32_TOL; the
    compensated form carries every addition's error exactly in a float32
    low word whose own roundings add up to about (m u)^2; the float64 form
    stays below TWOFLOAT_TOL for any m here."""
    m = np.asarray(counts, np.float64)
    u = 2.0 ** -24
    if precision == FP32:
        return np.maximum(FP32_TOL, (m - 1.0) * u)
    if precision == TWOFLOAT:
        return np.maximum(TWOFLOAT_TOL, (m * u) ** 2)
    return np.full_like(m, TWOFLOAT_TOL)


def bound_ratio(x, ref, mag, counts, precision):
    """Largest ratio of a cell's normalised error to its bound (cell_bound);
    counts broadcast to x. <= 1 passes."""
    x, ref, mag = np.asarray(x, np.float64), np.asarray(ref, np.float64), np.asarray(mag, np.float64)
    d = np.abs(x - ref)
    zero = mag == 0
    assert np.all(d[zero] == 0), "empty cells differ"
    if (~zero).sum() == 0:
        return 0.0
    bound = np.broadcast_to(cell_bound(precision, counts), x.shape)
    return float(np.max(d[~zero] / mag[~zero] / bound[~zero]))


def sub_slack(precision, root_mag):
    """Slack of a level built by subtraction: root_mag is the histogram of the
    absolute statistics over all rows ([1][F][B][2K], one leaf)."""
    return (SUB_SLACK_FP32 if precision == FP32 else SUB_SLACK_PAIR) * root_mag


def split_of(best_dev, level=0):
    b = best_dev.cpu().numpy().reshape(-1, 4)[level]
    return int(b[0]), int(b[1]), float(b[2:3].view(np.float32)[0]), float(b[3:4].view(np.float32)[0])


def check_split(gpu_fk, oracle_scores, nbins, tol=MARGIN_TOL):
    """The GPU split equals the oracle's argmax wherever the oracle's
    top-two margin is clear; otherwise it must be one of the near-tied best."""
    import oracle
    f, k, s1, s2 = oracle.best_split(oracle_scores, nbins)
    if f < 0:
        assert gpu_fk[0] < 0
        return True
    if s1 - s2 > tol * max(abs(s1), 1e-300):
        assert tuple(gpu_fk) == (f, k), (gpu_fk, (f, k), s1, s2)
        return True
    gs = oracle_scores[gpu_fk[0], gpu_fk[1]]
    assert s1 - gs <= tol * max(abs(s1), 1e-300) * 4, (gpu_fk, (f, k), s1, gs)
    return False
