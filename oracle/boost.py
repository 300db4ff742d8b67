"""Classic (non-ordered) boosting of oblivious trees on the CPU oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows the paper's plain scheme: binarize numeric features (Sec. 5), replace
every categorical feature by its ordered target statistic for a permutation
(Sec. 2, Eq. 1), start from the zero model (Algorithm 1 initialises M to 0),
and per tree choose one split per level for the whole level (oblivious trees,
Sec. 4), then set leaf values and add the tree to the model (Sec. 3, two-phase
tree building; the second phase is the ordinary GBDT step).

Readings the paper leaves open (border rule, score, regulariser, which
permutation a tree sees) are the ones documented in ``oracle.c``; tree t uses
the statistic columns of permutation t mod s.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import (apply_split, best_split, category_counts, combine_categories, gradients,
               histogram, leaf_values, ordered_ts, quantize, score, select_borders, ts_borders,
               update_approx)


@dataclass
class Prepared:
    num_bins: np.ndarray                 # uint8 [F_num][n]
    num_borders: list                    # per numeric feature, float32 borders
    ts_bins: np.ndarray                  # uint8 [s][F_cat*T*Q][n]
    ts_num: np.ndarray                   # int64 [s][F_cat*T][n]
    ts_den: np.ndarray                   # int32 [s][F_cat][n]
    ts_borders: np.ndarray               # float64 [ts_bins-1]
    nb_num: np.ndarray                   # int32 bins per numeric feature
    nb_ts: int
    timings: dict = field(default_factory=dict)
    n_priors: int = 1                    # Q statistic columns per (feature, target)
    counters: bool = False               # one counter column after each feature's statistics

    _n_cat: int = 0

    def tree_features(self, t: int):
        """Histogram features of tree t: numeric bins then TS bins of perm t mod s."""
        s = self.ts_bins.shape[0]
        if s == 0 or self.ts_bins.shape[1] == 0:
            return self.num_bins, self.nb_num
        r = t % s
        bins = np.concatenate([self.num_bins, self.ts_bins[r]], axis=0)
        nb = np.concatenate([self.nb_num,
                             np.full(self.ts_bins.shape[1], self.nb_ts, np.int32)])
        return bins, nb


def prior_lists(p) -> list:
    """Priors of every statistic target: the problem's own prior of target t
    first, then the extra priors shared by all targets (Sec. 2: several priors,
    one feature each)."""
    extra = [float(v) for v in getattr(p, "extra_priors", [])]
    return [[float(p.priors[t])] + extra for t in range(p.n_targets)]


def prepare(p) -> Prepared:
    t0 = time.perf_counter()
    borders = [select_borders(p.x_num[f], p.num_bins) for f in range(p.n_num)]
    t1 = time.perf_counter()
    num_bins = np.stack([quantize(p.x_num[f], borders[f]) for f in range(p.n_num)]) \
        if p.n_num else np.zeros((0, p.n), np.uint8)
    t2 = time.perf_counter()
    tb = ts_borders(p.ts_lo, p.ts_hi, p.ts_bins)
    s = p.perms.shape[0] if p.n_cat else 0
    T = p.n_targets
    pl = prior_lists(p)
    Q = len(pl[0]) if T else 1
    cnt = bool(getattr(p, "counters", False))
    per = T * Q + (1 if cnt else 0)
    ts_bins = np.zeros((s, p.n_cat * per, p.n), np.uint8)
    ts_num = np.zeros((s, p.n_cat * T, p.n), np.int64)
    ts_den = np.zeros((s, p.n_cat, p.n), np.int32)
    for r in range(s):
        for c in range(p.n_cat):
            for j in range(T):
                for q in range(Q):
                    num, den, _, tbin = ordered_ts(p.cat[c], p.perms[r], p.y_num[j], p.y_shift,
                                                   p.a, pl[j][q], tb)
                    ts_bins[r, c * per + j * Q + q] = tbin
                ts_num[r, c * T + j] = num
                ts_den[r, c] = den
            if cnt:
                ts_bins[r, c * per + T * Q] = counter_bins(p.cat[c], p.ts_bins)
    t3 = time.perf_counter()
    nb_num = np.array([len(b) + 1 for b in borders], np.int32)
    prep = Prepared(num_bins, borders, ts_bins, ts_num, ts_den, tb, nb_num, p.ts_bins,
                    {"borders_s": t1 - t0, "quantize_s": t2 - t1, "ordered_ts_s": t3 - t2}, Q,
                    cnt)
    prep._n_cat = p.n_cat
    return prep


def counter_bins(values, n_bins: int) -> np.ndarray:
    """The counter statistic (Sec. 2: a category, or a combination, replaced
    by its number of appearances in the dataset) binarized on a log2 scale:
    bin = floor(log2(count)), at most n_bins - 1 (the paper gives no
    binarization; Zipf-like counts spread over these bins)."""
    ids, _ = combine_categories(np.asarray(values, np.int32), np.zeros(len(values), np.int32))
    cnt = category_counts(ids).astype(np.int64)
    b = np.floor(np.log2(np.maximum(cnt, 1))).astype(np.int64)
    return np.minimum(b, n_bins - 1).astype(np.uint8)


@dataclass
class Tree:
    splits: list            # [(feature, border, best score, second score)] per level
    values: np.ndarray      # float64 [2^d][K]
    counts: np.ndarray      # int64 [2^d]


def fit_tree(bins, nb, approx, label, loss: int, K: int, depth: int, lr: float,
             l2: float, B: int) -> Tree:
    """One oblivious tree on FP64 gradients of the current approx (updated in place)."""
    n = label.size
    g, h = gradients(loss, K, approx, label)
    leaf = np.zeros(n, np.uint16)
    splits = []
    for lvl in range(depth):
        hist = histogram(bins, g, h, leaf, 1 << lvl, B)
        sc = score(hist, nb, l2)
        f, k, s1, s2 = best_split(sc, nb)
        splits.append((f, k, s1, s2))
        if f >= 0:
            apply_split(bins[f], k, lvl, leaf)
    vals, G, H, cnt = leaf_values(leaf, g, h, 1 << depth, l2)
    update_approx(approx, leaf, vals, lr)
    return Tree(splits, vals, cnt)


class CombinationTree:
    """Candidate features of one tree with greedy combinations of categorical
    features (Sec. 2, "Feature combinations"). The first split considers no
    combination. After each split, the split's own categorical value per row
    (the categorical feature or combination behind a statistic column, or the
    two-valued [bin > border] of a numeric split; a level without a split
    gives one value for every row) is combined with every categorical feature
    of the dataset; each such combination's values are numbered (the perfect
    hash) and its ordered statistics, for every target and prior on the
    tree's permutation, become candidates of every later level.

    Candidate order at a level: the tree's own columns (numeric, then per
    categorical feature its statistic columns by target and prior, then its
    counter column when counters are on), then for every earlier level j in
    order and every categorical feature c in order, the columns of
    combination (j, c) in the same order.
    Combinations equal to a column already present (a feature combined with
    itself) stay candidates; equal scores go to the lower index."""

    def __init__(self, prep: Prepared, p, t: int):
        self.p, self.prep = p, prep
        self.r = t % p.perms.shape[0] if p.n_cat else 0
        self.base_bins, self.base_nb = prep.tree_features(t)
        self.F_num = p.n_num
        self.T, self.Q = p.n_targets, prep.n_priors
        self.counters = prep.counters
        # columns per categorical feature or crossing: statistics, then counter
        self.TQ = self.T * self.Q + (1 if self.counters else 0)
        self.F_base = self.base_bins.shape[0]
        self.pl = prior_lists(p)
        self.combo_ids = []      # [level j][categorical feature c] int32 [n]
        self.combo_bins = []     # uint8 [n] columns in candidate order

    def features(self):
        """(bins uint8 [F][n], n_bins int32 [F]) of the current candidates."""
        if not self.combo_bins:
            return self.base_bins, self.base_nb
        bins = np.concatenate([self.base_bins, np.stack(self.combo_bins)], axis=0)
        nb = np.concatenate([self.base_nb,
                             np.full(len(self.combo_bins), self.prep.nb_ts, np.int32)])
        return bins, nb

    def split_values(self, f: int, k: int, bins) -> np.ndarray:
        """The categorical value of every row under split (f, k)."""
        if f < 0:
            return np.zeros(self.p.n, np.int32)
        if f < self.F_num:
            return (bins[f] > k).astype(np.int32)
        if f < self.F_base:
            return np.ascontiguousarray(self.p.cat[(f - self.F_num) // self.TQ], np.int32)
        j, c = divmod((f - self.F_base) // self.TQ, self.p.n_cat)
        return self.combo_ids[j][c]

    def add_split(self, f: int, k: int):
        """Record the split just made; its combinations with every categorical
        feature become candidates of the levels below."""
        p = self.p
        bins, _ = self.features()
        v = self.split_values(f, k, bins)
        perm = p.perms[self.r]
        level_ids = []
        for c in range(p.n_cat):
            ids, _ = combine_categories(v, p.cat[c])
            level_ids.append(ids)
            for t in range(self.T):
                for q in range(self.Q):
                    _, _, _, tb = ordered_ts(ids, perm, p.y_num[t], p.y_shift, p.a,
                                             self.pl[t][q], self.prep.ts_borders)
                    self.combo_bins.append(tb)
            if self.counters:
                self.combo_bins.append(counter_bins(ids, self.prep.nb_ts))
        self.combo_ids.append(level_ids)


def fit_tree_combinations(prep: Prepared, p, t: int, approx, B: int):
    """One oblivious tree with greedy feature combinations (Sec. 2) on FP64
    gradients of approx (updated in place). Returns (Tree, CombinationTree)."""
    n = p.n
    g, h = gradients(p.loss, p.K, approx, p.label)
    ct = CombinationTree(prep, p, t)
    leaf = np.zeros(n, np.uint16)
    splits = []
    for lvl in range(p.depth):
        bins, nb = ct.features()
        hist = histogram(bins, g, h, leaf, 1 << lvl, B)
        sc = score(hist, nb, p.l2)
        f, k, s1, s2 = best_split(sc, nb)
        splits.append((f, k, s1, s2))
        if f >= 0:
            apply_split(bins[f], k, lvl, leaf)
        if lvl + 1 < p.depth and p.n_cat:
            ct.add_split(f, k)
    vals, G, H, cnt = leaf_values(leaf, g, h, 1 << p.depth, p.l2)
    update_approx(approx, leaf, vals, p.lr)
    return Tree(splits, vals, cnt), ct


def fit(p, iterations: int | None = None, prep: Prepared | None = None,
        combinations: bool = False):
    """Full classic boosting; returns (trees, approx [K][n], prepared).
    combinations: trees consider greedy feature combinations (Sec. 2)."""
    prep = prep or prepare(p)
    iters = p.iterations if iterations is None else iterations
    approx = np.zeros((p.K, p.n), np.float64)
    B = max(int(prep.nb_num.max()) if prep.nb_num.size else 1,
            prep.nb_ts if prep.ts_bins.shape[1] else 1)
    trees = []
    for t in range(iters):
        if combinations:
            trees.append(fit_tree_combinations(prep, p, t, approx, B)[0])
            continue
        bins, nb = prep.tree_features(t)
        trees.append(fit_tree(bins, nb, approx, p.label, p.loss, p.K, p.depth, p.lr, p.l2, B))
    return trees, approx, prep
