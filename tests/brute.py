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
