"""Seeded synthetic inputs for the split-search path and its CPU oracle.

This module only draws random numbers and arranges them into arrays. It holds
none of the boosting arithmetic (no borders, bins, statistics, gradients or
scores), so both the HIP path and the oracle may consume what it produces.

The paper benchmarks on Epsilon, Criteo and eight public classification sets
(Sec. 6, Tables 1-3), none of which are available here. The five workloads
below are synthetic stand-ins with the shapes, value distributions and
category-frequency skew of those workloads: dense numeric columns (Epsilon-like)
and Zipf-distributed high-cardinality categorical columns (Criteo-like).

Every stream is ``numpy.random.default_rng(SeedSequence([181011363, cfg, k]))``
with k = 0 for numeric features, 1 for categorical values, 2 for labels,
3 + r for permutation r and 100 + p for problem p of a batch.

Arrays are feature-major: ``x_num`` is float32 ``[F_num][n]``, ``cat`` is raw
int32 category values ``[F_cat][n]`` (arbitrary, non-dense values, so the
consumer has to build its own dense ids), ``perms`` is int32 ``[s][n]`` with
``perm[p]`` = row placed at position p, ``label`` is float32 ``[n]`` (0/1 for
Logloss, class index for MultiClass, real value for RMSE).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 181011363

RMSE, LOGLOSS, MULTICLASS = 0, 1, 2
LOSS_NAMES = {RMSE: "RMSE", LOGLOSS: "Logloss", MULTICLASS: "MultiClass"}

# Fixed-point exponent for regression labels fed to the ordered statistic:
# y_num = llrint(y * 2**Y_SHIFT) so that per-category sums are exact integers.
Y_SHIFT = 32


def rng_for(cfg: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([BASE_SEED, cfg, stream]))


@dataclass
class Problem:
    """One boosting problem: raw inputs plus the training parameters."""
    name: str
    x_num: np.ndarray            # float32 [F_num][n]
    cat: np.ndarray              # int32 [F_cat][n] raw category values
    label: np.ndarray            # float32 [n]
    perms: np.ndarray            # int32 [s][n]
    loss: int
    K: int                       # approx width (1, or number of classes)
    depth: int
    iterations: int
    lr: float
    l2: float
    num_bins: int                # bins per numeric feature (borders = bins - 1)
    ts_bins: int                 # bins per ordered-statistic column
    a: float                     # prior weight
    priors: list = field(default_factory=list)   # one prior per target column
    y_num: np.ndarray | None = None   # int64 [T][n] targets for the statistic
    y_shift: int = 0
    ts_lo: float = 0.0
    ts_hi: float = 1.0
    extra_priors: list = field(default_factory=list)  # priors beside priors[t], every target

    @property
    def n(self) -> int:
        return int(self.label.shape[0])

    @property
    def n_num(self) -> int:
        return int(self.x_num.shape[0])

    @property
    def n_cat(self) -> int:
        return int(self.cat.shape[0])

    @property
    def n_targets(self) -> int:
        return int(self.y_num.shape[0]) if self.y_num is not None else 0

    @property
    def n_features(self) -> int:
        """Histogram features a tree sees: numeric + one permutation's TS columns."""
        return self.n_num + self.n_cat * self.n_targets


def zipf_ids(g: np.random.Generator, n: int, C: int, s: float) -> np.ndarray:
    """Dense ids in [0, C) with P(rank r) proportional to (r+1)^-s; ids are a
    seeded shuffle of the ranks so that frequency is unrelated to the id."""
    w = (np.arange(1, C + 1, dtype=np.float64)) ** (-s)
    w /= w.sum()
    ranks = g.choice(C, size=n, p=w)
    shuffle = g.permutation(C)
    return shuffle[ranks].astype(np.int64)


def raw_values(g: np.random.Generator, C: int) -> np.ndarray:
    """C distinct, non-dense, non-negative int32 values standing for category names."""
    vals = g.choice(2**31 - 1, size=C, replace=False)
    return vals.astype(np.int32)


def _finish_targets(p: Problem) -> Problem:
    """Encode the statistic targets as int64 numerators, one row per target."""
    y = p.label.astype(np.float64)
    if p.loss == RMSE:
        p.y_shift = Y_SHIFT
        p.y_num = np.rint(y * float(2**Y_SHIFT)).astype(np.int64)[None, :]
        p.priors = [float(np.mean(y))]
        p.ts_lo, p.ts_hi = float(y.min()), float(y.max())
    elif p.loss == LOGLOSS:
        p.y_shift = 0
        p.y_num = (y > 0.5).astype(np.int64)[None, :]
        if not p.priors:
            p.priors = [float(np.mean(y > 0.5))]
        p.ts_lo, p.ts_hi = 0.0, 1.0
    else:
        p.y_shift = 0
        rows = [(p.label == c).astype(np.int64) for c in range(p.K - 1)]
        p.y_num = np.stack(rows) if rows else np.zeros((0, p.n), np.int64)
        p.priors = [float(np.mean(p.label == c)) for c in range(p.K - 1)]
        p.ts_lo, p.ts_hi = 0.0, 1.0
    return p


def _perms(cfg: int, n: int, s: int, base_stream: int = 3) -> np.ndarray:
    return np.stack([rng_for(cfg, base_stream + r).permutation(n).astype(np.int32)
                     for r in range(s)]) if s else np.zeros((0, n), np.int32)


def _sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def make_c1(n: int = 10_000) -> Problem:
    """Small Logloss problem: 20 N(0,1) numeric features with 32 quantile
    borders, 2 categorical features of cardinality 50 with Zipf(1.2)
    frequencies, one permutation, depth 4, 10 iterations."""
    cfg = 1
    gx, gc, gy = rng_for(cfg, 0), rng_for(cfg, 1), rng_for(cfg, 2)
    x = gx.standard_normal((20, n), dtype=np.float32)
    ids, cats = [], []
    for _ in range(2):
        d = zipf_ids(gc, n, 50, 1.2)
        vals = raw_values(gc, 50)
        ids.append(d)
        cats.append(vals[d])
    w = gy.standard_normal(20)
    offs = [gy.normal(0.0, 0.5, 50) for _ in range(2)]
    logit = x.astype(np.float64).T @ w + offs[0][ids[0]] + offs[1][ids[1]]
    y = (gy.random(n) < _sigmoid(logit)).astype(np.float32)
    p = Problem("c1_small_logloss", x, np.stack(cats), y, _perms(cfg, n, 1),
                LOGLOSS, 1, depth=4, iterations=10, lr=0.1, l2=3.0,
                num_bins=33, ts_bins=33, a=1.0, priors=[0.5])
    return _finish_targets(p)


def _step_function(g, x, n_feat_total, n_numeric):
    """A random oblivious depth-3 step function of 3 distinct numeric features."""
    feats = g.choice(n_numeric, 3, replace=False)
    out_idx = np.zeros(x.shape[1], np.int64)
    for lvl, f in enumerate(feats):
        q = g.uniform(0.1, 0.9)
        thr = np.quantile(x[f], q)
        out_idx |= (x[f] > thr).astype(np.int64) << lvl
    vals = g.standard_normal(8)
    return vals[out_idx]


def make_c2(n: int = 1_000_000, s: int = 4) -> Problem:
    """RMSE at scale: 50 N(0,1) + 50 lognormal(0,1) numeric features at 128
    bins, 10 Zipf(1.1) categorical features of cardinality 10..1e5, label =
    sum of 5 random depth-3 step functions + category effects + N(0, 0.1^2),
    4 permutations, depth 6, 500 iterations."""
    cfg = 2
    gx, gc, gy = rng_for(cfg, 0), rng_for(cfg, 1), rng_for(cfg, 2)
    x = np.empty((100, n), np.float32)
    x[:50] = gx.standard_normal((50, n), dtype=np.float32)
    x[50:] = np.exp(gx.standard_normal((50, n), dtype=np.float32))
    cards = [10, 10, 100, 100, 1000, 1000, 10_000, 10_000, 100_000, 100_000]
    ids, cats = [], []
    for C in cards:
        C = min(C, max(2, n))
        d = zipf_ids(gc, n, C, 1.1)
        vals = raw_values(gc, C)
        ids.append(d)
        cats.append(vals[d])
    y = np.zeros(n, np.float64)
    for _ in range(5):
        y += _step_function(gy, x, 100, 100)
    for d in ids:
        eff = gy.normal(0.0, 0.5, int(d.max()) + 1)
        y += eff[d]
    y += gy.normal(0.0, 0.1, n)
    p = Problem("c2_scale_rmse", x, np.stack(cats), y.astype(np.float32),
                _perms(cfg, n, s), RMSE, 1, depth=6, iterations=500, lr=0.1,
                l2=3.0, num_bins=128, ts_bins=128, a=1.0)
    return _finish_targets(p)


def make_c3(n: int = 10_000_000, F: int = 200) -> Problem:
    """Precision workload: F uniform(0,1) numeric features at 255 bins, with
    5% of each column overwritten by exact duplicates of other rows; Logloss
    with a 1% positive rate; depth 8, 200 iterations; no categorical data."""
    cfg = 3
    gx, gy = rng_for(cfg, 0), rng_for(cfg, 2)
    x = gx.random((F, n), dtype=np.float32)
    k = max(1, n // 20)
    for f in range(F):
        dst = gx.choice(n, k, replace=False)
        src = gx.integers(0, n, k)
        x[f, dst] = x[f, src]
    w = gy.standard_normal(F)
    z = (x.astype(np.float64).T - 0.5) @ w / math.sqrt(F)
    lo, hi = -20.0, 20.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        if np.mean(_sigmoid(z + mid)) > 0.01:
            hi = mid
        else:
            lo = mid
    b = 0.5 * (lo + hi)
    y = (gy.random(n) < _sigmoid(z + b)).astype(np.float32)
    p = Problem("c3_precision_logloss", x, np.zeros((0, n), np.int32), y,
                np.zeros((0, n), np.int32), LOGLOSS, 1, depth=8,
                iterations=200, lr=0.1, l2=3.0, num_bins=255, ts_bins=255,
                a=1.0)
    return _finish_targets(p)


def _c4_problem(cfg: int, stream: int, n: int, name: str) -> Problem:
    g = rng_for(cfg, stream)
    x = g.standard_normal((50, n), dtype=np.float32)
    ids, cats = [], []
    for _ in range(4):
        d = zipf_ids(g, n, 1000, 1.1)
        vals = raw_values(g, 1000)
        ids.append(d)
        cats.append(vals[d])
    w = g.standard_normal(50)
    y = x.astype(np.float64).T @ w
    for _ in range(10):
        a_, b_ = g.choice(50, 2, replace=False)
        y += g.standard_normal() * x[a_].astype(np.float64) * x[b_]
    for d in ids:
        y += g.normal(0.0, 0.5, 1000)[d]
    y += g.normal(0.0, 0.1, n)
    perm = g.permutation(n).astype(np.int32)[None, :]
    p = Problem(name, x, np.stack(cats), y.astype(np.float32), perm, RMSE, 1,
                depth=6, iterations=100, lr=0.1, l2=3.0, num_bins=64,
                ts_bins=64, a=1.0)
    return _finish_targets(p)


def cv_folds(p: Problem, k: int = 5, cfg: int = 4, stream: int = 200) -> list[Problem]:
    """k cross-validation training problems of p: a seeded shuffle of the rows
    cut into k near-equal parts; problem j trains on the rows outside part j
    (kept in their original order) with one seeded permutation of its own."""
    order = rng_for(cfg, stream).permutation(p.n)
    parts = np.array_split(order, k)
    out = []
    for j in range(k):
        keep = np.ones(p.n, bool)
        keep[parts[j]] = False
        rows = np.flatnonzero(keep)
        m = rows.size
        perm = rng_for(cfg, stream + 1 + j).permutation(m).astype(np.int32)[None, :]
        q = Problem(f"{p.name}_fold{j}", np.ascontiguousarray(p.x_num[:, rows]),
                    np.ascontiguousarray(p.cat[:, rows]), np.ascontiguousarray(p.label[rows]),
                    perm, p.loss, p.K, depth=p.depth, iterations=p.iterations, lr=p.lr,
                    l2=p.l2, num_bins=p.num_bins, ts_bins=p.ts_bins, a=p.a)
        out.append(_finish_targets(q))
    return out


def cv_fold_weights(p: Problem, k: int = 5, cfg: int = 4, stream: int = 200):
    """The same k folds as cv_folds, as row weights over p's rows: returns
    (q, w) with w float32 [k][n] (0 on fold j's held-out rows, else 1) and q a
    copy of p whose k permutations are the folds' own: fold j's training rows
    in the order of cv_folds' permutation of them, then its held-out rows, so
    that the training rows' ordered statistics count training rows only."""
    order = rng_for(cfg, stream).permutation(p.n)
    parts = np.array_split(order, k)
    perms = np.empty((k, p.n), np.int32)
    w = np.ones((k, p.n), np.float32)
    for j in range(k):
        keep = np.ones(p.n, bool)
        keep[parts[j]] = False
        rows = np.flatnonzero(keep)
        sub = rng_for(cfg, stream + 1 + j).permutation(rows.size)
        perms[j] = np.concatenate([rows[sub], np.sort(parts[j])]).astype(np.int32)
        w[j, parts[j]] = 0.0
    import copy
    q = copy.copy(p)
    q.name = f"{p.name}_cv{k}"
    q.perms = perms
    return q, w


def c4_sizes(P: int = 64, lo: int = 5_000, hi: int = 2_000_000, scale: float = 1.0):
    g = rng_for(4, 0)
    n = np.rint(np.exp(g.uniform(math.log(lo), math.log(hi), P))).astype(np.int64)
    return [max(16, int(v * scale)) for v in n]


def make_c4(P: int = 64, scale: float = 1.0) -> list[Problem]:
    """Batch of P independent RMSE problems with log-uniform row counts in
    [5e3, 2e6] (optionally scaled down), 50 numeric features at 64 bins and 4
    categorical features of cardinality 1000, depth 6, 100 iterations."""
    return [_c4_problem(4, 100 + i, n, f"c4_problem_{i}")
            for i, n in enumerate(c4_sizes(P, scale=scale))]


def make_c5(n: int = 50_000_000, n_cat: int = 20, K: int = 10, chunk: int = 1 << 21,
            workers: int = 16, progress=None) -> Problem:
    """Large MultiClass problem: 50 N(0,1) numeric features at 255 bins, 20
    Zipf(1.05) categorical features with cardinalities 10..1e6, K-class
    softmax labels from a seeded linear model plus per-category class effects,
    depth 10, 100 iterations.

    The per-feature tables (category ranks' shuffle, raw values, class
    effects) and the linear model are drawn once; the rows are drawn in chunks
    of `chunk` rows, chunk c from its own stream 1000 + c, filled by `workers`
    threads (numpy's generators release the interpreter lock while filling).
    `progress(done, total)` is called after each chunk if given."""
    from concurrent.futures import ThreadPoolExecutor
    cfg = 5
    gc, gy = rng_for(cfg, 1), rng_for(cfg, 2)
    cards = [min(int(round(10 ** (1 + 5 * j / max(1, n_cat - 1)))), max(2, n))
             for j in range(n_cat)]
    cdfs, shuffles, values = [], [], []
    for C in cards:
        w = np.arange(1, C + 1, dtype=np.float64) ** -1.05
        cdf = np.cumsum(w)
        cdfs.append(cdf / cdf[-1])
        shuffles.append(gc.permutation(C))
        values.append(raw_values(gc, C))
    W = gy.standard_normal((50, K)) / math.sqrt(50)
    E = [gy.normal(0.0, 0.5, (C, K)) for C in cards]
    x = np.empty((50, n), np.float32)
    cats = np.empty((n_cat, n), np.int32)
    y = np.empty(n, np.float32)
    n_chunks = (n + chunk - 1) // chunk
    done = [0]

    def fill(c):
        r0, r1 = c * chunk, min(n, (c + 1) * chunk)
        g = rng_for(cfg, 1000 + c)
        xs = g.standard_normal((50, r1 - r0), dtype=np.float32)
        x[:, r0:r1] = xs
        logits = xs.astype(np.float64).T @ W
        for j in range(n_cat):
            rank = np.minimum(np.searchsorted(cdfs[j], g.random(r1 - r0), side="right"),
                              cards[j] - 1)
            ids = shuffles[j][rank]
            cats[j, r0:r1] = values[j][ids]
            logits += E[j][ids]
        logits -= logits.max(axis=1, keepdims=True)
        pr = np.exp(logits)
        pr /= pr.sum(axis=1, keepdims=True)
        u = g.random(r1 - r0)[:, None]
        y[r0:r1] = (np.cumsum(pr, axis=1) < u).sum(axis=1).clip(0, K - 1)
        done[0] += 1
        if progress is not None:
            progress(done[0], n_chunks)

    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        list(ex.map(fill, range(n_chunks)))
    p = Problem("c5_large_multiclass", x, cats, y, _perms(cfg, n, 1),
                MULTICLASS, K, depth=10, iterations=100, lr=0.1, l2=3.0,
                num_bins=255, ts_bins=255, a=1.0)
    return _finish_targets(p)


def random_small(seed: int, n: int, F_num: int = 3, F_cat: int = 1, C: int = 5,
                 loss: int = RMSE, K: int = 1, depth: int = 3, num_bins: int = 8,
                 s: int = 1, dup: bool = True) -> Problem:
    """Tiny random problems for brute-force pins and ragged-size parity."""
    g = np.random.default_rng(np.random.SeedSequence([BASE_SEED, 999, seed]))
    if dup:
        x = g.integers(0, max(2, num_bins + 3), (F_num, n)).astype(np.float32) * 0.5
    else:
        x = g.standard_normal((F_num, n), dtype=np.float32)
    cats = [raw_values(g, C)[g.integers(0, C, n)] for _ in range(F_cat)]
    cat = np.stack(cats) if cats else np.zeros((0, n), np.int32)
    if loss == RMSE:
        y = g.standard_normal(n).astype(np.float32)
    elif loss == LOGLOSS:
        y = (g.random(n) < 0.4).astype(np.float32)
    else:
        y = g.integers(0, K, n).astype(np.float32)
    perms = np.stack([g.permutation(n).astype(np.int32) for _ in range(s)])
    p = Problem(f"small_{seed}", x, cat, y, perms, loss, K, depth=depth,
                iterations=3, lr=0.1, l2=1.0, num_bins=num_bins,
                ts_bins=num_bins, a=1.0)
    return _finish_targets(p)


def make_interactions(n: int = 20_000, loss: int = LOGLOSS, K: int = 1, seed: int = 0,
                      depth: int = 4, C: tuple = (6, 8, 5), s: int = 1,
                      extra_priors: tuple = (0.0, 1.0)) -> Problem:
    """A workload whose target depends on pairs of categories (the case
    feature combinations exist for, Sec. 2): 3 numeric N(0,1) features at 16
    bins, categorical features of small cardinalities C (Zipf(1.1)), and a
    target driven by a seeded effect table of the (c0, c1) pair, another of
    (c1, c2) crossed with the sign of x0, plus a small numeric term. Statistic
    columns use the problem's prior and the extra priors. Logloss (0/1),
    RMSE (real) or MultiClass (K classes)."""
    cfg = 6
    g = np.random.default_rng(np.random.SeedSequence([BASE_SEED, cfg, 1000 + seed]))
    x = g.standard_normal((3, n), dtype=np.float32)
    ids = [zipf_ids(g, n, c, 1.1) for c in C]
    cats = [raw_values(g, c)[d] for c, d in zip(C, ids)]
    t01 = g.normal(0.0, 1.5, (C[0], C[1], max(K, 1)))
    t12 = g.normal(0.0, 1.0, (C[1], C[2], max(K, 1)))
    sgn = np.where(x[0] > 0, 1.0, -1.0)[:, None]
    z = t01[ids[0], ids[1]] + sgn * t12[ids[1], ids[2]] + 0.3 * x[1].astype(np.float64)[:, None]
    if loss == RMSE:
        y = (z[:, 0] + g.normal(0.0, 0.1, n)).astype(np.float32)
    elif loss == LOGLOSS:
        y = (g.random(n) < _sigmoid(z[:, 0])).astype(np.float32)
    else:
        e = np.exp(z - z.max(axis=1, keepdims=True))
        pr = e / e.sum(axis=1, keepdims=True)
        y = (pr.cumsum(axis=1) < g.random(n)[:, None]).sum(axis=1).clip(0, K - 1)
        y = y.astype(np.float32)
    p = Problem(f"interactions_{seed}", x, np.stack(cats), y, _perms(cfg, n, s, 3 + 10 * seed),
                loss, K if loss == MULTICLASS else 1, depth=depth, iterations=5, lr=0.1,
                l2=3.0, num_bins=16, ts_bins=16, a=1.0)
    p = _finish_targets(p)
    if loss != RMSE:
        p.extra_priors = list(extra_priors)
    else:
        # extra priors in target units: the ends of the target range
        p.extra_priors = [p.ts_lo, p.ts_hi][: len(extra_priors)]
    return p


CONFIGS = {
    "c1": make_c1,
    "c2": make_c2,
    "c3": make_c3,
    "c4": make_c4,
    "c5": make_c5,
}
