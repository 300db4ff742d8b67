"""Brute-force references for tiny inputs (n <= 64), independent of the oracle.

No histograms and no closed-form leaf score: for every candidate split the
rows of each child are collected directly and the per-leaf objective
    sum_i (g_i v + h_i v^2 / 2) + l2 v^2 / 2
is minimised over v by golden-section search. The best split minimises the
total objective over all leaves and both sides.
"""
from __future__ import annotations

import math

import numpy as np

PHI = (math.sqrt(5.0) - 1.0) / 2.0


def leaf_objective(g, h, l2):
    """min over v of sum(g v + h v^2/2) + l2 v^2/2, found numerically."""
    G = float(np.sum(g))
    Hs = float(np.sum(h)) + l2

    def f(v):
        return float(np.sum(g * v + 0.5 * h * v * v)) + 0.5 * l2 * v * v

    if len(g) == 0:
        return 0.0, 0.0
    if Hs <= 0:
        return 0.0, 0.0
    # the minimiser lies within |G|/Hs of 0; bracket generously
    r = 4.0 * (abs(G) / Hs + 1.0)
    a, b = -r, r
    c, d = b - PHI * (b - a), a + PHI * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(200):
        if fc < fd:
            b, d, fd = d, c, fc
            c = b - PHI * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + PHI * (b - a)
            fd = f(d)
    v = 0.5 * (a + b)
    return f(v), v


def split_objectives(bins, n_bins, g, h, leaf, n_leaves, l2):
    """objective[f][k] of splitting every current leaf by bin_f > k.
    g, h are [K][n]; the objective sums over classes independently."""
    F, n = bins.shape
    K = g.shape[0]
    out = {}
    for f in range(F):
        for k in range(int(n_bins[f]) - 1):
            total = 0.0
            for L in range(n_leaves):
                for side in (0, 1):
                    m = (leaf == L) & ((bins[f] > k) == bool(side))
                    for c in range(K):
                        total += leaf_objective(g[c][m], h[c][m], l2)[0]
            out[(f, k)] = total
    return out


def best_by_objective(objs):
    """Smallest objective; ties (within 1e-9 relative) to smallest (f, k)."""
    items = sorted(objs.items())
    best = min(v for _, v in items)
    tol = 1e-9 * max(1.0, abs(best))
    for key, v in items:
        if v <= best + tol:
            return key, best
    raise AssertionError


def _loss_derivs(loss, K, a, y):
    """First and second loss derivatives at a [K][m] for labels y [m]:
    RMSE 1/2 (a-y)^2, Logloss with p = sigmoid(a), MultiClass with softmax
    p (diagonal second derivative)."""
    if loss == 0:
        return a - y[None, :], np.ones_like(a)
    if loss == 1:
        p = 1.0 / (1.0 + np.exp(-a))
        return p - y[None, :], p * (1.0 - p)
    e = np.exp(a - a.max(axis=0, keepdims=True))
    p = e / e.sum(axis=0, keepdims=True)
    t = np.zeros_like(a)
    t[y.astype(np.int64), np.arange(a.shape[1])] = 1.0
    return p - t, p * (1.0 - p)


def algorithm1_models(loss, K, y_pos, leaves_pos, n_leaves, lr, l2):
    """Algorithm 1 of Sec. 3 with every model sharing the given tree
    structures: model i (i = 0..n) learns from positions 0..i-1 only, and
    after every tree each model adds its own Newton leaf values (from its
    learning positions' gradients at its own approximation) to its value at
    every position. y_pos [n] and the trees' leaves leaves_pos [T][n] are in
    permutation (position) order. Returns the approximations [n+1][K][n].
    O(n^2) per tree: for tiny n only."""
    n = y_pos.size
    models = np.zeros((n + 1, K, n))
    for leaf in leaves_pos:
        for i in range(n + 1):
            G = np.zeros((n_leaves, K))
            H = np.zeros((n_leaves, K))
            if i > 0:
                g, h = _loss_derivs(loss, K, models[i][:, :i], y_pos[:i])
                for j in range(i):
                    G[leaf[j]] += g[:, j]
                    H[leaf[j]] += h[:, j]
            d = H + l2
            v = np.where(d == 0.0, 0.0, -G / np.where(d == 0.0, 1.0, d))
            models[i] += lr * v[leaf].T
    return models
