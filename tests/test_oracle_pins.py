"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle through a route other than its own code: hand-
worked values (tests/golden/, derived from the equations they cite), closed
forms, invariants, library routines for special cases, finite differences and
brute force on tiny inputs. A dropped term, a flipped sign, a wrong index or a
transposed operand in the oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import datagen
import oracle
from tests import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


# ---------------------------------------------------------------- ordered TS
def test_ordered_ts_hand_examples(oracle_lib):
    """Sec. 2, Eq. (1) on the hand-worked examples."""
    o = oracle_lib
    for case in _gold("ordered_ts_hand.json")["cases"]:
        num, den, ts, _ = o.ordered_ts(case["cat"], case["perm"], np.array(case["y"]), 0,
                                       case["a"], case["prior"])
        assert num.tolist() == case["num"], case["name"]
        assert den.tolist() == case["den"], case["name"]
        np.testing.assert_allclose(ts, case["ts"], rtol=0, atol=1e-15)


def _rand_ts_inputs(seed, n=300, C=7):
    g = np.random.default_rng(seed)
    vals = g.choice(10**6, C, replace=False).astype(np.int32)
    cat = vals[g.integers(0, C, n)]
    perm = g.permutation(n).astype(np.int32)
    y = g.integers(0, 2, n).astype(np.int64)
    return cat, perm, y


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ordered_ts_invariants(oracle_lib, seed):
    o = oracle_lib
    cat, perm, y = _rand_ts_inputs(seed)
    n = cat.size
    num, den, ts, _ = o.ordered_ts(cat, perm, y, 0, 1.0, 0.3)
    pos = np.empty(n, np.int64)
    pos[perm] = np.arange(n)
    for c in np.unique(cat):
        rows = np.nonzero(cat == c)[0]
        rows = rows[np.argsort(pos[rows])]       # rows of c in permutation order
        # den enumerates 0..n_c-1 along the permutation
        assert den[rows].tolist() == list(range(rows.size))
        # num is the exclusive running total of y along the permutation
        assert num[rows].tolist() == np.concatenate([[0], np.cumsum(y[rows])[:-1]]).tolist()
        # closed form for the total: each y_j is counted by every later row
        nc = rows.size
        assert int(num[rows].sum()) == int(sum(y[r] * (nc - 1 - i) for i, r in enumerate(rows)))


def test_ordered_ts_excludes_own_and_later_rows(oracle_lib):
    """The statistic of the row at position p uses only positions < p: changing
    the label of that row or of any later row leaves its value unchanged."""
    o = oracle_lib
    cat, perm, y = _rand_ts_inputs(5, n=200, C=4)
    _, _, ts, _ = o.ordered_ts(cat, perm, y, 0, 1.0, 0.5)
    for p in (0, 17, 100, 199):
        y2 = y.copy()
        later = perm[p:]
        y2[later] = 1 - y2[later]
        _, _, ts2, _ = o.ordered_ts(cat, perm, y2, 0, 1.0, 0.5)
        assert np.array_equal(ts[perm[: p + 1]], ts2[perm[: p + 1]])


def test_ordered_ts_limits(oracle_lib):
    o = oracle_lib
    cat, perm, y = _rand_ts_inputs(7)
    # a -> infinity: the prior dominates
    _, _, ts, _ = o.ordered_ts(cat, perm, y, 0, 1e12, 0.37)
    np.testing.assert_allclose(ts, 0.37, atol=1e-9)
    # all categories distinct: no earlier row shares a category, TS == P exactly
    n = 50
    distinct = np.arange(n, dtype=np.int32) * 7919
    _, den, ts, _ = o.ordered_ts(distinct, np.random.default_rng(1).permutation(n), np.ones(n), 0,
                                 2.0, 0.25)
    assert np.all(den == 0) and np.all(ts == 0.25)


def test_ordered_ts_fixed_point_targets(oracle_lib):
    """Regression targets as int64 numerators with value y_num * 2^-e."""
    o = oracle_lib
    cat = np.array([1, 1, 1, 2], np.int32)
    perm = np.array([0, 1, 2, 3], np.int32)
    y = np.array([0.75, -1.5, 2.0, 9.0])
    y_num = np.rint(y * 2.0**32).astype(np.int64)
    num, den, ts, _ = o.ordered_ts(cat, perm, y_num, 32, 1.0, 0.5)
    assert num.tolist() == [0, int(0.75 * 2**32), int(-0.75 * 2**32), 0]
    np.testing.assert_allclose(ts, [0.5, (0.75 + 0.5) / 2, (-0.75 + 0.5) / 3, 0.5], rtol=0, atol=1e-15)


def test_ts_bins_from_uniform_borders(oracle_lib):
    o = oracle_lib
    b = o.ts_borders(0.0, 1.0, 4)
    assert b.tolist() == [0.25, 0.5, 0.75]
    cat, perm, y = _rand_ts_inputs(9)
    _, _, ts, tb = o.ordered_ts(cat, perm, y, 0, 1.0, 0.5, b)
    assert np.array_equal(tb, np.searchsorted(b, ts, side="left"))


# ----------------------------------------------------------- borders / bins
@pytest.mark.parametrize("max_bins", [2, 5, 33, 128, 255, 256])
def test_borders_properties(oracle_lib, max_bins):
    o = oracle_lib
    g = np.random.default_rng(max_bins)
    for x in (g.standard_normal(3000).astype(np.float32),
              np.exp(g.standard_normal(3000)).astype(np.float32),
              (g.integers(0, 40, 3000) * 0.5).astype(np.float32)):
        b = o.select_borders(x, max_bins)
        assert b.size <= max_bins - 1
        assert np.all(np.diff(b) > 0)
        assert np.all(np.isin(b, x))                   # borders are data values
        bins = o.quantize(x, b)
        assert np.array_equal(bins, np.searchsorted(b, x, side="left"))
        counts = np.bincount(bins, minlength=b.size + 1)
        assert counts.size == b.size + 1 and np.all(counts > 0)   # no empty bin
        assert np.array_equal(o.quantize(b, b), np.arange(b.size))  # bin(c_k) = k
        uniq = np.unique(x)
        if uniq.size <= max_bins:                      # one bin per distinct value
            assert np.array_equal(b, uniq[:-1])


def test_borders_value_at_rank(oracle_lib):
    o = oracle_lib
    x = np.arange(1, 101, dtype=np.float32)            # 100 distinct values, 4 bins
    assert o.select_borders(x, 4).tolist() == [25.0, 50.0, 75.0]
    assert o.select_borders(np.full(10, 3.0, np.float32), 8).size == 0
    with pytest.raises(ValueError):
        o.select_borders(np.array([1.0, np.nan], np.float32), 4)


# --------------------------------------------------------------- gradients
@pytest.mark.parametrize("loss", [datagen.RMSE, datagen.LOGLOSS])
def test_gradients_finite_difference(oracle_lib, loss):
    o = oracle_lib
    g0 = np.random.default_rng(3)
    a = g0.normal(0, 2, 50)
    y = (g0.random(50) < 0.5).astype(np.float32) if loss else g0.normal(0, 1, 50).astype(np.float32)
    yd = y.astype(np.float64)

    def L(v):
        if loss == datagen.RMSE:
            return 0.5 * (yd - v) ** 2
        p = 1 / (1 + np.exp(-v))
        return -(yd * np.log(p) + (1 - yd) * np.log(1 - p))

    g, h = o.gradients(loss, 1, a[None, :], y)
    e = 1e-4
    np.testing.assert_allclose(g[0], (L(a + e) - L(a - e)) / (2 * e), rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(h[0], (L(a + e) - 2 * L(a) + L(a - e)) / e**2, rtol=1e-4, atol=1e-6)


def test_gradients_multiclass_finite_difference(oracle_lib):
    o = oracle_lib
    K, n = 4, 30
    g0 = np.random.default_rng(4)
    a = g0.normal(0, 2, (K, n))
    y = g0.integers(0, K, n).astype(np.float32)

    def L(A):
        z = A - A.max(axis=0)
        return -(z[y.astype(int), np.arange(n)] - np.log(np.exp(z).sum(axis=0)))

    g, h = o.gradients(datagen.MULTICLASS, K, a, y)
    e = 1e-4
    for k in range(K):
        ap, am = a.copy(), a.copy()
        ap[k] += e
        am[k] -= e
        np.testing.assert_allclose(g[k], (L(ap) - L(am)) / (2 * e), rtol=1e-6, atol=1e-8)
        np.testing.assert_allclose(h[k], (L(ap) - 2 * L(a) + L(am)) / e**2, rtol=1e-4, atol=1e-6)


# -------------------------------------------------------------- histograms
def test_histogram_equals_one_hot_product(oracle_lib):
    """hist[L][f][b] = sum over rows with leaf L and bin b (Sec. 5), computed
    here as a one-hot matrix product, plus per-leaf totals and counts."""
    o = oracle_lib
    g0 = np.random.default_rng(11)
    n, F, B, K, Lv = 500, 3, 9, 2, 4
    bins = g0.integers(0, B, (F, n)).astype(np.uint8)
    g = g0.normal(size=(K, n))
    h = g0.random((K, n))
    leaf = g0.integers(0, Lv, n).astype(np.uint16)
    hist = o.histogram(bins, g, h, leaf, Lv, B)
    for f in range(F):
        onehot = np.zeros((n, Lv * B))
        onehot[np.arange(n), leaf.astype(int) * B + bins[f]] = 1.0
        for c in range(K):
            np.testing.assert_allclose(hist[:, f, :, 2 * c].ravel(), onehot.T @ g[c], atol=1e-12)
            np.testing.assert_allclose(hist[:, f, :, 2 * c + 1].ravel(), onehot.T @ h[c], atol=1e-12)
    # every feature's histogram sums to the leaf's gradient total
    for L in range(Lv):
        for c in range(K):
            tot = g[c][leaf == L].sum()
            np.testing.assert_allclose(hist[L, :, :, 2 * c].sum(axis=1), tot, atol=1e-10)
    # with h = 1 the second statistic is the row count; counts sum to n
    hc = o.histogram(bins, g[:1], np.ones((1, n)), leaf, Lv, B)
    assert hc[..., 1].sum(axis=(0, 2)).tolist() == [n] * F


def test_histogram_int_exact(oracle_lib):
    o = oracle_lib
    g0 = np.random.default_rng(12)
    n, F, B, Lv = 400, 2, 7, 2
    bins = g0.integers(0, B, (F, n)).astype(np.uint8)
    gq = g0.integers(-32767, 32768, (1, n)).astype(np.int16)
    hq = g0.integers(0, 32768, (1, n)).astype(np.int16)
    leaf = g0.integers(0, Lv, n).astype(np.uint16)
    hist = o.histogram_int(bins, gq, hq, leaf, Lv, B)
    for f in range(F):
        for L in range(Lv):
            for b in range(B):
                m = (leaf == L) & (bins[f] == b)
                assert hist[L, f, b, 0] == int(gq[0][m].astype(np.int64).sum())
                assert hist[L, f, b, 1] == int(hq[0][m].astype(np.int64).sum())


def test_grad_codes_bounds(oracle_lib):
    o = oracle_lib
    g0 = np.random.default_rng(13)
    g = g0.normal(size=(2, 1000)).astype(np.float32)
    h = g0.random((2, 1000)).astype(np.float32)
    gq, hq, sc = o.grad_codes(g, h, True)
    for c in range(2):
        s = np.float32(np.abs(g[c]).max()) / np.float32(32767)
        assert sc[c, 0] == s
        assert np.abs(gq[c]).max() == 32767
        # code = rint(fl(g / s)): the float32 quotient is within 2^-24 |g / s|
        # <= 2^-9 of g / s, so a code is within 1/2 + 2^-9 steps of g
        assert np.all(np.abs(g[c].astype(np.float64) - gq[c] * np.float64(s)) <=
                      (0.5 + 2.0**-9) * np.float64(s))
        assert np.all(hq[c] >= 0)
    _, hq1, _ = o.grad_codes(g[:1], None, False)
    assert np.all(hq1 == 1)


# -------------------------------------------------------- score and argmax
def test_depth2_hand_tree(oracle_lib):
    """Hand-worked depth-2 oblivious tree: scores, argmax, leaf bits, values."""
    o = oracle_lib
    d = _gold("tree_hand.json")["depth2"]
    bins = np.array(d["bins"], np.uint8)
    nb = np.array(d["n_bins"], np.int32)
    g = np.array(d["g"], np.float64)[None, :]
    h = np.ones_like(g)
    leaf = np.zeros(8, np.uint16)
    for lvl in range(2):
        hist = o.histogram(bins, g, h, leaf, 1 << lvl, 4)
        sc = o.score(hist, nb, d["l2"])
        want = np.array([[np.nan if v is None else v for v in row] for row in d["level_scores"][lvl]])
        m = ~np.isnan(want)
        np.testing.assert_allclose(sc[m], want[m], rtol=1e-12)
        assert np.all(np.isneginf(sc[~m]))
        f, k, s1, s2 = o.best_split(sc, nb)
        assert [f, k] == d["best"][lvl]
        if lvl == 0:
            np.testing.assert_allclose(s1 - s2, d["margin0"], rtol=1e-12)
        o.apply_split(bins[f], k, lvl, leaf)
        assert leaf.tolist() == d["leaf_after"][lvl]
    vals, G, H, cnt = o.leaf_values(leaf, g, h, 4, d["l2"])
    assert G[:, 0].tolist() == d["G"] and H[:, 0].tolist() == d["H"] and cnt.tolist() == d["counts"]
    np.testing.assert_allclose(vals[:, 0], d["values"], rtol=1e-15)
    approx = np.zeros((1, 8))
    o.update_approx(approx, leaf, vals, d["lr"])
    np.testing.assert_allclose(approx[0], np.array(d["approx_delta"])[leaf], rtol=1e-15)


def test_tie_break_and_clear_case(oracle_lib):
    o = oracle_lib
    d = _gold("tree_hand.json")["tie"]
    bins = np.array(d["bins"], np.uint8)
    nb = np.array(d["n_bins"], np.int32)
    leaf = np.zeros(4, np.uint16)
    for gk, sk in (("g_tie", "scores_tie"), ("g_clear", "scores_clear")):
        g = np.array(d[gk], np.float64)[None, :]
        hist = o.histogram(bins, g, np.ones_like(g), leaf, 1, 3)
        sc = o.score(hist, nb, d["l2"])
        np.testing.assert_allclose(sc[0], d[sk], rtol=1e-15)
        f, k, s1, s2 = o.best_split(sc, nb)
        assert (f, k) == (0, 0)
    assert s1 - s2 > 0
    lf = leaf.copy()
    o.apply_split(bins[0], 0, 0, lf)
    vals, *_ = o.leaf_values(lf, g, np.ones_like(g), 2, d["l2"])
    np.testing.assert_allclose(vals[:, 0], d["values_clear"], rtol=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_best_split_matches_brute_force(oracle_lib, seed):
    """Brute force (rows collected per child, objective minimised numerically)
    agrees with histogram + score + argmax on tiny random problems."""
    o = oracle_lib
    g0 = np.random.default_rng(100 + seed)
    n, F, K = 40, 3, 1 + seed % 2
    nb = g0.integers(2, 6, F).astype(np.int32)
    bins = np.stack([g0.integers(0, nb[f], n) for f in range(F)]).astype(np.uint8)
    g = g0.normal(size=(K, n))
    h = g0.random((K, n)) + 0.1
    n_leaves = 1 << (seed % 3)
    leaf = g0.integers(0, n_leaves, n).astype(np.uint16)
    l2 = [0.5, 1.0, 3.0][seed % 3]
    hist = o.histogram(bins, g, h, leaf, n_leaves, int(nb.max()))
    sc = o.score(hist, nb, l2)
    f, k, s1, s2 = o.best_split(sc, nb)
    objs = brute.split_objectives(bins, nb, g, h, leaf, n_leaves, l2)
    (bf, bk), bobj = brute.best_by_objective(objs)
    assert (f, k) == (bf, bk)
    # the score is -2 x the minimised objective of the split
    for (ff, kk), v in objs.items():
        np.testing.assert_allclose(sc[ff, kk], -2.0 * v, rtol=1e-7, atol=1e-9)


def test_rmse_stump_is_least_squares(oracle_lib):
    """Depth 1, RMSE from approx 0, l2 -> 0: the chosen split minimises the
    sum of squared errors around the child means, and with lr 1 the model
    becomes those means."""
    o = oracle_lib
    from oracle import boost
    g0 = np.random.default_rng(21)
    n = 60
    x = g0.integers(0, 6, (2, n)).astype(np.uint8)
    y = (g0.normal(size=n) + 2.0 * (x[1] > 2)).astype(np.float32)
    nb = np.array([6, 6], np.int32)
    sse = {}
    for f in range(2):
        for k in range(5):
            m = x[f] > k
            sse[(f, k)] = sum(float(((y[s] - y[s].mean()) ** 2).sum()) for s in (m, ~m) if s.any())
    best = min(sse, key=lambda t: (sse[t], t))
    approx = np.zeros((1, n))
    tree = boost.fit_tree(x, nb, approx, y, datagen.RMSE, 1, 1, 1.0, 1e-300, 6)
    assert tree.splits[0][:2] == best
    m = x[best[0]] > best[1]
    yd = y.astype(np.float64)
    np.testing.assert_allclose(approx[0][m], yd[m].mean(), rtol=1e-9)
    np.testing.assert_allclose(approx[0][~m], yd[~m].mean(), rtol=1e-9)


def test_leaf_value_minimises_objective(oracle_lib):
    o = oracle_lib
    g0 = np.random.default_rng(22)
    g = g0.normal(size=(1, 30))
    h = g0.random((1, 30))
    leaf = np.zeros(30, np.uint16)
    vals, *_ = o.leaf_values(leaf, g, h, 1, 2.0)
    _, v = brute.leaf_objective(g[0], h[0], 2.0)
    np.testing.assert_allclose(vals[0, 0], v, rtol=1e-7)


def test_leaf_bits_follow_levels(oracle_lib):
    """Sec. 4: bit i of the leaf index is the binary feature of depth i."""
    o = oracle_lib
    g0 = np.random.default_rng(23)
    n = 200
    bins = g0.integers(0, 10, (4, n)).astype(np.uint8)
    leaf = np.zeros(n, np.uint16)
    chosen = [(2, 3), (0, 7), (3, 1), (2, 5)]
    for lvl, (f, k) in enumerate(chosen):
        o.apply_split(bins[f], k, lvl, leaf)
    want = sum(((bins[f] > k).astype(np.int64) << i) for i, (f, k) in enumerate(chosen))
    assert np.array_equal(leaf, want)


def test_update_approx_gathers_leaf_values(oracle_lib):
    o = oracle_lib
    g0 = np.random.default_rng(24)
    K, n = 3, 50
    leaf = g0.integers(0, 8, n).astype(np.uint16)
    vals = g0.normal(size=(8, K))
    a = g0.normal(size=(K, n))
    b = a.copy()
    o.update_approx(b, leaf, vals, 0.25)
    np.testing.assert_allclose(b, a + 0.25 * vals[leaf].T, rtol=0, atol=1e-15)


def test_boosting_reduces_training_loss(oracle_lib):
    from oracle import boost
    p = datagen.make_c1(n=3000)
    p.iterations = 5
    trees, approx, _ = boost.fit(p)
    y = p.label.astype(np.float64)
    pr = 1 / (1 + np.exp(-approx[0]))
    ll = -np.mean(y * np.log(pr) + (1 - y) * np.log(1 - pr))
    assert ll < np.log(2) - 0.01
    assert all(t.counts.sum() == p.n for t in trees)


# ---------------------------------------------------------------- model apply
def _model_of(trees, depth):
    """(feat, border, values) of oracle trees; a level without a split (feature
    -1) never sets its bit, which border 255 reproduces."""
    T = len(trees)
    feat = np.zeros((T, depth), np.int32)
    border = np.full((T, depth), 255, np.int32)
    for t, tr in enumerate(trees):
        for l, (f, k, _, _) in enumerate(tr.splits):
            if f >= 0:
                feat[t, l], border[t, l] = f, k
    values = np.stack([tr.values for tr in trees])
    return feat, border, values


def test_apply_model_reproduces_training_approx(oracle_lib):
    """Sec. 4 scorer against the training loop: applying the trained trees to
    the training rows adds, row by row and tree by tree, exactly the leaf
    values the model updates of Algorithm 1 added (leaves found there by the
    level-by-level split rule)."""
    from oracle import boost
    o = oracle_lib
    p = datagen.make_c1(n=2000)
    p.iterations = 6
    trees, approx, prep = boost.fit(p)
    bins, _ = prep.tree_features(0)          # one permutation: every tree's features
    feat, border, values = _model_of(trees, p.depth)
    a = np.zeros_like(approx)
    o.apply_model(bins, feat, border, values, p.lr, a)
    assert np.array_equal(a, approx)


def test_apply_model_reproduces_multiclass_training(oracle_lib):
    """The same for K = 3 classes: the value table is [T][2^d][K]."""
    from oracle import boost
    o = oracle_lib
    g0 = np.random.default_rng(31)
    n, F, B, K, d = 1500, 5, 16, 3, 3
    bins = g0.integers(0, B, (F, n)).astype(np.uint8)
    label = ((bins[0] > 7).astype(np.int64) + (bins[1] > 11)).astype(np.float32)
    nb = np.full(F, B, np.int32)
    approx = np.zeros((K, n))
    trees = [boost.fit_tree(bins, nb, approx, label, 2, K, d, 0.3, 1.0, B) for _ in range(4)]
    feat, border, values = _model_of(trees, d)
    a = np.zeros((K, n))
    o.apply_model(bins, feat, border, values, 0.3, a)
    assert np.array_equal(a, approx)


def test_apply_model_constant_leaves(oracle_lib):
    """Border -1 sets every bit (leaf 2^d - 1), border 255 none (leaf 0): the
    model is then a constant per class."""
    o = oracle_lib
    g0 = np.random.default_rng(32)
    n, F, T, d, K = 40, 3, 5, 4, 2
    bins = g0.integers(0, 256, (F, n)).astype(np.uint8)
    feat = g0.integers(0, F, (T, d)).astype(np.int32)
    values = g0.normal(size=(T, 1 << d, K))
    for bval, leaf in ((-1, (1 << d) - 1), (255, 0)):
        a0 = g0.normal(size=(K, n))
        a = a0.copy()
        o.apply_model(bins, feat, np.full((T, d), bval, np.int32), values, 0.5, a)
        want = a0.copy()
        for t in range(T):
            want += 0.5 * values[t, leaf][:, None]
        assert np.array_equal(a, want)


def test_apply_model_splits_over_trees_and_classes(oracle_lib):
    """Applying trees 0..T-1 equals applying 0..j-1 and then j..T-1; a class's
    output depends only on that class's leaf values."""
    o = oracle_lib
    g0 = np.random.default_rng(33)
    n, F, T, d, K = 300, 6, 7, 3, 3
    bins = g0.integers(0, 32, (F, n)).astype(np.uint8)
    feat = g0.integers(0, F, (T, d)).astype(np.int32)
    border = g0.integers(-1, 32, (T, d)).astype(np.int32)
    values = g0.normal(size=(T, 1 << d, K))
    a = np.zeros((K, n))
    o.apply_model(bins, feat, border, values, 0.1, a)
    b = np.zeros((K, n))
    o.apply_model(bins, feat[:3], border[:3], values[:3], 0.1, b)
    o.apply_model(bins, feat[3:], border[3:], values[3:], 0.1, b)
    assert np.array_equal(a, b)
    v2 = values.copy()
    v2[..., 1] = 0.0
    c = np.zeros((K, n))
    o.apply_model(bins, feat, border, v2, 0.1, c)
    assert np.array_equal(c[[0, 2]], a[[0, 2]]) and not c[1].any()


# ------------------------------------------------------ category combinations
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_combine_categories_brute_force(oracle_lib, seed):
    """Sec. 2 "Feature combinations": a pair of categorical values is a new
    category. Brute force: the sorted set of distinct pairs (as unsigned 32-bit
    values) numbers them; every row gets its pair's rank."""
    o = oracle_lib
    g0 = np.random.default_rng(40 + seed)
    n = int(g0.integers(1, 60))
    a = g0.choice(np.array([-3, 0, 2, 7, 2 ** 31 - 1, -(2 ** 31)], np.int32), n)
    b = g0.integers(-2, 3, n).astype(np.int32)
    ids, m = o.combine_categories(a, b)
    u32 = lambda v: int(v) & 0xffffffff
    pairs = sorted({(u32(x), u32(y)) for x, y in zip(a, b)})
    rank = {p: i for i, p in enumerate(pairs)}
    assert m == len(pairs)
    assert [rank[(u32(x), u32(y))] for x, y in zip(a, b)] == ids.tolist()


def test_combine_categories_ts_groups(oracle_lib):
    """The ordered statistics of the combination (Eq. 1 over its ids) count
    exactly the earlier rows that share both values."""
    o = oracle_lib
    g0 = np.random.default_rng(44)
    n = 200
    a = g0.integers(0, 4, n).astype(np.int32)
    b = g0.integers(0, 3, n).astype(np.int32)
    y = g0.integers(0, 2, n).astype(np.int64)
    perm = g0.permutation(n).astype(np.int32)
    ids, _ = o.combine_categories(a, b)
    num, den, _, _ = o.ordered_ts(ids, perm, y, 0, 1.0, 0.5)
    for p in range(n):
        r = perm[p]
        prev = perm[:p]
        same = prev[(a[prev] == a[r]) & (b[prev] == b[r])]
        assert den[r] == same.size and num[r] == y[same].sum()


def test_category_counts_brute_force(oracle_lib):
    """The counter statistic (Sec. 2): a row's value is the number of rows
    that share its category, counted here pair by pair."""
    o = oracle_lib
    g0 = np.random.default_rng(45)
    ids = g0.integers(0, 7, 60).astype(np.int32)
    got = o.category_counts(ids)
    assert [sum(1 for y in ids if y == x) for x in ids] == got.tolist()
    assert got.sum() == sum(c * c for c in np.unique(ids, return_counts=True)[1])


# ---------------------------------------------------------------------------
# Ordered boosting's supporting approximations (Sec. 3)

def _read_model_of_each_position(n):
    """Fill every (model, position) value of the support with a distinct code
    and read back, through the RMSE gradient at label 0, which value each
    position's gradient takes."""
    off = oracle.ordered_offsets(n)
    S = int(off[-1])
    support = np.arange(S, dtype=np.float64)[None, :]
    perm = np.random.default_rng(n).permutation(n).astype(np.int32)
    g, _ = oracle.ordered_gradients(0, 1, perm, np.zeros(n, np.float32), support)
    code = g[0, perm]                      # value read by position p (row perm[p])
    m = np.searchsorted(off, code, side="right") - 1
    return off, m, code - off[m]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 9, 64, 65, 1000, 4097])
def test_ordered_support_layout(oracle_lib, n):
    """Sizes of the relaxation: model m is kept for min(n, 2^m) positions,
    the total stays below 4n, and position p reads its own entry of model
    floor(log2 p) + 1 (model 0 for p = 0), which learns only from positions
    below 2^floor(log2 p) <= p."""
    off, m, j = _read_model_of_each_position(n)
    M = oracle.ordered_models(n)
    assert len(off) == M + 1
    assert np.array_equal(np.diff(off), np.minimum(n, 2 ** np.arange(M)))
    assert off[-1] < 4 * n
    p = np.arange(n)
    assert np.array_equal(j, p)
    want = np.array([0 if q == 0 else int(q).bit_length() for q in range(n)])
    assert np.array_equal(m, want)
    learn = np.where(m == 0, 0, 2.0 ** (m - 1))
    assert np.all(learn <= p)
    assert m.max() == M - 1


def _ordered_run(loss, K, n, trees, depth, seed, lr=0.3, l2=1.0):
    g = np.random.default_rng(seed)
    perm = g.permutation(n).astype(np.int32)
    if loss == 0:
        y = g.normal(size=n).astype(np.float32)
    elif loss == 1:
        y = (g.random(n) < 0.4).astype(np.float32)
    else:
        y = g.integers(0, K, n).astype(np.float32)
    leaves = g.integers(0, 1 << depth, (trees, n)).astype(np.uint16)   # row order
    S = int(oracle.ordered_offsets(n)[-1])
    support = np.zeros((K, S))
    grads = []
    for t in range(trees):
        grads.append(oracle.ordered_gradients(loss, K, perm, y, support))
        oracle.ordered_update(loss, K, perm, y, leaves[t], 1 << depth, lr, l2, support)
    return perm, y, leaves, support, grads


@pytest.mark.parametrize("loss,K,n", [(0, 1, 37), (1, 1, 64), (2, 3, 29), (1, 1, 1), (0, 1, 2)])
def test_ordered_matches_algorithm1_brute_force(oracle_lib, loss, K, n):
    """Every supporting model equals the model of Algorithm 1 (brute force,
    one model per position, shared tree structures) that learns from the same
    first 2^(m-1) positions, at every position it is kept for; and the
    gradient a position gets before each tree is the one of that model."""
    depth, trees, lr, l2 = 2, 3, 0.3, 1.0
    perm, y, leaves, support, grads = _ordered_run(loss, K, n, trees, depth, 11 + n)
    models = brute.algorithm1_models(loss, K, y[perm], leaves[:, perm], 1 << depth, lr, l2)
    off = oracle.ordered_offsets(n)
    for m in range(len(off) - 1):
        learn = 0 if m == 0 else 2 ** (m - 1)
        keep = int(off[m + 1] - off[m])
        np.testing.assert_allclose(support[:, off[m]:off[m] + keep], models[learn][:, :keep],
                                   rtol=1e-12, atol=1e-14)
    # the gradients before the last tree, from the brute-force models
    before = brute.algorithm1_models(loss, K, y[perm], leaves[:-1, perm], 1 << depth, lr, l2)
    p = np.arange(n)
    read = np.array([0 if q == 0 else 2 ** (int(q).bit_length() - 1) for q in p])
    a = before[read, :, p].T                     # [K][n] in position order
    gb, hb = brute._loss_derivs(loss, K, a, y[perm])
    np.testing.assert_allclose(grads[-1][0][:, perm], gb, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(grads[-1][1][:, perm], hb, rtol=1e-12, atol=1e-14)


def test_ordered_gradient_never_sees_its_own_or_later_labels(oracle_lib):
    """Unbiasedness (Sec. 3): the approximation behind position p's gradient
    is unchanged, bit for bit, when the labels of positions p..n-1 change."""
    n, K, loss = 200, 1, 1
    perm, y, leaves, support, _ = _ordered_run(loss, K, n, 4, 3, 5)
    for p0 in (1, 7, 64, 130):
        y2 = y.copy()
        y2[perm[p0:]] = 1.0 - y2[perm[p0:]]
        S = support.shape[1]
        s2 = np.zeros((K, S))
        for t in range(4):
            oracle.ordered_update(loss, K, perm, y2, leaves[t], 8, 0.3, 1.0, s2)
        _, mm, _ = _read_model_of_each_position(n)
        off = oracle.ordered_offsets(n)
        e = off[mm] + np.arange(n)
        assert np.array_equal(support[0, e[:p0 + 1]], s2[0, e[:p0 + 1]]), p0
        # later positions whose model learned from a changed label can move
        learn = np.where(mm == 0, 0, 2 ** np.maximum(mm - 1, 0))
        moved = learn > p0
        if moved.any():
            assert not np.array_equal(support[0, e[moved]], s2[0, e[moved]]), p0


def test_ordered_single_leaf_rmse_is_prefix_mean(oracle_lib):
    """One tree with one leaf, RMSE, l2 = 0, lr = 1: model m's value is the
    mean label of its learning positions (0 for model 0), at every position
    it is kept for."""
    n = 300
    g = np.random.default_rng(3)
    perm = g.permutation(n).astype(np.int32)
    y = g.normal(size=n).astype(np.float32)
    off = oracle.ordered_offsets(n)
    support = np.zeros((1, int(off[-1])))
    vals = oracle.ordered_update(0, 1, perm, y, np.zeros(n, np.uint16), 1, 1.0, 0.0, support)
    yp = y[perm].astype(np.float64)
    for m in range(len(off) - 1):
        learn = 0 if m == 0 else 2 ** (m - 1)
        want = yp[:learn].mean() if learn else 0.0
        assert vals[m, 0, 0] == pytest.approx(want, rel=1e-13, abs=1e-15)
        np.testing.assert_allclose(support[0, off[m]:off[m + 1]], want, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------
# Packed bins (Sec. 5 widths; the library's byte layout)

def test_pack_bins_hand_examples(oracle_lib):
    """Bytes written out by hand from the documented layout."""
    for case in _gold("packed_bins_hand.json")["cases"]:
        got = oracle_lib.pack_bins(np.array(case["bins"], np.uint8), case["bits"])
        want = np.array([int(b, 16) for b in case["bytes_hex"]], np.uint8)
        assert np.array_equal(got, want), case


@pytest.mark.parametrize("bits", [4, 1])
def test_pack_bins_keeps_every_bin(oracle_lib, bits):
    """Every row's bin can be read back from its nibble or bit (sizes 1..70),
    and changing one row's bin changes exactly its own bits."""
    g = np.random.default_rng(bits)
    for n in list(range(1, 40)) + [63, 64, 65, 70]:
        b = g.integers(0, 1 << bits, n).astype(np.uint8)
        packed = oracle_lib.pack_bins(b, bits)
        assert packed.size == ((n + 15) // 16) * 2 * bits
        bitsarr = np.unpackbits(packed, bitorder="little")
        # per row, the set of bit positions its value occupies
        for i in range(n):
            b2 = b.copy()
            b2[i] = b[i] ^ ((1 << bits) - 1)
            diff = np.flatnonzero(bitsarr != np.unpackbits(oracle_lib.pack_bins(b2, bits),
                                                           bitorder="little"))
            assert diff.size == bits, (n, i)
            seg, r = divmod(i, 16)
            assert np.all(diff // (16 * bits) == seg)
        # total set bits = sum of popcounts of the values
        assert int(bitsarr.sum()) == int(sum(bin(int(v)).count("1") for v in b))


# ---------------------------------------------------------------------------
# Greedy feature combinations and several priors (Sec. 2)

def _brute_ts_bins(keys, perm, y_num, y_shift, a, prior, borders):
    """Eq. (1) row by row over hashable per-row keys (any grouping values):
    a row's statistic counts the strictly earlier positions with its key."""
    sums, cnts = {}, {}
    out = np.zeros(len(keys), np.uint8)
    for r in perm:
        k = keys[r]
        num, den = sums.get(k, 0), cnts.get(k, 0)
        ts = (float(num) * 2.0 ** -y_shift + a * prior) / (float(den) + a)
        out[r] = sum(1 for b in borders if ts > b)
        sums[k] = num + int(y_num[r])
        cnts[k] = den + 1
    return out


def _brute_counter_bins(keys, n_bins):
    """Every row's number of rows with its key, on the log2 scale (the bit
    length of the count, minus one), capped at n_bins - 1."""
    out = np.zeros(len(keys), np.uint8)
    for i, k in enumerate(keys):
        c = sum(1 for x in keys if x == k)
        out[i] = min(c.bit_length() - 1, n_bins - 1)
    return out


def _brute_candidates(p, prep, t, splits):
    """The candidate columns of a tree after the given splits, built without
    the oracle's combination code: a combination's value per row is the
    nested tuple of its parts' values, statistics are counted row by row."""
    from oracle import boost
    base_bins, _ = prep.tree_features(t)
    F_num, T, Q = p.n_num, p.n_targets, prep.n_priors
    cnt = bool(getattr(p, "counters", False))
    per = T * Q + (1 if cnt else 0)
    F_base = base_bins.shape[0]
    pl = boost.prior_lists(p)
    perm = p.perms[t % p.perms.shape[0]]
    combo_keys, cols = [], [base_bins[f] for f in range(F_base)]
    for f, k in splits:
        if f < 0:
            v = [0] * p.n
        elif f < F_num:
            v = [int(b > k) for b in cols[f]]
        elif f < F_base:
            v = [int(x) for x in p.cat[(f - F_num) // per]]
        else:
            j, c = divmod((f - F_base) // per, p.n_cat)
            v = combo_keys[j][c]
        level = []
        for c in range(p.n_cat):
            keys = [(v[i], int(p.cat[c][i])) for i in range(p.n)]
            level.append(keys)
            for tt in range(T):
                for q in range(Q):
                    cols.append(_brute_ts_bins(keys, perm, p.y_num[tt], p.y_shift, p.a,
                                               pl[tt][q], prep.ts_borders))
            if cnt:
                cols.append(_brute_counter_bins(keys, prep.nb_ts))
        combo_keys.append(level)
    return np.stack(cols)


@pytest.mark.parametrize("counters", [False, True])
@pytest.mark.parametrize("loss,K,seed", [(1, 1, 0), (0, 1, 1), (2, 3, 2)])
def test_combination_candidates_brute_force(oracle_lib, loss, K, seed, counters):
    """Sec. 2 "Feature combinations": after each split, the split's value
    (a categorical feature, a combination, or a numeric split's two values)
    crossed with every categorical feature gives new candidate columns whose
    ordered statistics (every target, every prior) count the earlier rows of
    the same combined value. Forced split sequences reach every kind of
    element: numeric, statistic column, combination column, no split."""
    from oracle import boost
    p = datagen.make_interactions(n=48, loss=loss, K=K, seed=seed, C=(3, 4, 2), depth=5)
    p.counters = counters
    prep = boost.prepare(p)
    if counters:
        # the tree's own counter columns: rows per category, brute force
        per = p.n_targets * prep.n_priors + 1
        for c in range(p.n_cat):
            want = _brute_counter_bins([int(x) for x in p.cat[c]], prep.nb_ts)
            assert np.array_equal(prep.ts_bins[0, c * per + per - 1], want)
    ct0 = boost.CombinationTree(prep, p, 0)
    F_base = ct0.F_base
    TQ = ct0.TQ
    seqs = [
        [(0, 7), (p.n_num, 5), (F_base + TQ, 3), (F_base + 4 * TQ + 1, 9)],
        [(p.n_num + TQ + 1, 2), (-1, -1), (F_base + 2 * TQ, 1), (1, 3)],
    ]
    for seq in seqs:
        ct = boost.CombinationTree(prep, p, 0)
        for lvl, (f, k) in enumerate(seq):
            ct.add_split(f, k)
            bins, nb = ct.features()
            want = _brute_candidates(p, prep, 0, seq[: lvl + 1])
            assert bins.shape == want.shape == (F_base + (lvl + 1) * p.n_cat * TQ, p.n)
            assert np.array_equal(bins, want), f"level {lvl}"
            assert np.all(nb[F_base:] == prep.nb_ts)


def test_combination_tree_splits_are_brute_force_best(oracle_lib):
    """Every level of a combination tree takes the best split over that
    level's candidates, scored by brute force with children built from rows;
    the first level considers the tree's own columns only."""
    from oracle import boost
    p = datagen.make_interactions(n=40, loss=0, seed=3, C=(3, 3, 2), depth=3)
    p.extra_priors = []
    prep = boost.prepare(p)
    approx = np.zeros((1, p.n))
    B = max(int(prep.nb_num.max()), prep.nb_ts)
    tree, ct = boost.fit_tree_combinations(prep, p, 0, approx, B)
    g, h = oracle_lib.gradients(p.loss, p.K, np.zeros((1, p.n)), p.label)
    leaf = np.zeros(p.n, np.uint16)
    seq = []
    for lvl, (f, k, _, _) in enumerate(tree.splits):
        bins = _brute_candidates(p, prep, 0, seq)
        nb = np.concatenate([prep.tree_features(0)[1],
                             np.full(bins.shape[0] - ct.F_base, prep.nb_ts, np.int32)])
        objs = brute.split_objectives(bins, nb, g, h, leaf, 1 << lvl, p.l2)
        (bf, bk), _ = brute.best_by_objective(objs)
        assert (f, k) == (bf, bk), f"level {lvl}"
        if lvl == 0:
            assert bins.shape[0] == ct.F_base
        oracle_lib.apply_split(bins[f], k, lvl, leaf)
        seq.append((f, k))


def test_combination_with_itself_is_the_feature(oracle_lib):
    """A categorical feature crossed with itself has the feature's own groups,
    so its statistic columns equal the feature's; without categorical
    features a combination tree is the classic tree."""
    from oracle import boost
    p = datagen.make_interactions(n=3000, loss=1, seed=4)
    prep = boost.prepare(p)
    ct = boost.CombinationTree(prep, p, 0)
    for c in range(p.n_cat):
        ct2 = boost.CombinationTree(prep, p, 0)
        ct2.add_split(p.n_num + c * ct.TQ, 0)
        bins, _ = ct2.features()
        got = bins[ct.F_base + c * ct.TQ: ct.F_base + (c + 1) * ct.TQ]
        want = bins[p.n_num + c * ct.TQ: p.n_num + (c + 1) * ct.TQ]
        assert np.array_equal(got, want)
    q = datagen.random_small(7, 300, F_num=4, F_cat=0, depth=4)
    prep_q = boost.prepare(q)
    tr_c, ap_c, _ = boost.fit(q, iterations=2, prep=prep_q, combinations=True)
    tr_p, ap_p, _ = boost.fit(q, iterations=2, prep=prep_q)
    assert [t.splits for t in tr_c] == [t.splits for t in tr_p]
    assert np.array_equal(ap_c, ap_p)


def test_several_priors_closed_form(oracle_lib):
    """Sec. 2: one statistic column per prior. For one grouping, two priors
    differ by a (P1 - P2) / (den + a) in every row (Eq. 1 is affine in P);
    a category seen once has no earlier rows, so its statistic is the prior."""
    o = oracle_lib
    g0 = np.random.default_rng(46)
    n = 500
    cat = g0.integers(0, 9, n).astype(np.int32)
    cat[:20] = 100 + np.arange(20)                  # singletons
    y = g0.integers(0, 2, n).astype(np.int64)
    perm = g0.permutation(n).astype(np.int32)
    a = 2.0
    res = {P: o.ordered_ts(cat, perm, y, 0, a, P) for P in (0.0, 0.25, 1.0)}
    for P1, P2 in ((0.0, 1.0), (0.25, 0.0)):
        _, den, t1, _ = res[P1]
        _, _, t2, _ = res[P2]
        np.testing.assert_allclose(t1 - t2, a * (P1 - P2) / (den + a), rtol=0, atol=1e-15)
    for P, (_, den, ts, _) in res.items():
        assert np.all(den[:20] == 0) and np.all(ts[:20] == P)
    from oracle import boost
    p = datagen.make_interactions(n=400, loss=1, seed=5)
    prep = boost.prepare(p)
    assert prep.n_priors == 3
    for c in range(p.n_cat):
        for q, P in enumerate(boost.prior_lists(p)[0]):
            _, _, _, tb = o.ordered_ts(p.cat[c], p.perms[0], p.y_num[0], p.y_shift, p.a, P,
                                       prep.ts_borders)
            assert np.array_equal(prep.ts_bins[0, c * 3 + q], tb)


# ---------------------------------------------------------------------------
# The scorer's binary features (Sec. 4)

def test_binarize_hand_example(oracle_lib):
    """Two features of 35 rows: bit r of word w is [bin of row 32 w + r >
    border]; rows past n are 0."""
    bins = np.zeros((2, 35), np.uint8)
    bins[0, [0, 3, 31, 32, 34]] = 5
    bins[1] = np.arange(35) % 4
    bits = oracle_lib.binarize(bins, [0, 1, 1, 0], [4, 2, -1, 5])
    assert bits.shape == (4, 2)
    assert bits[0].tolist() == [(1 << 0) | (1 << 3) | (1 << 31), (1 << 0) | (1 << 2)]
    threes = sum(1 << r for r in range(32) if r % 4 == 3)
    assert bits[1].tolist() == [threes, 0]          # rows 32..34 have bins 0, 1, 2
    assert bits[2].tolist() == [0xFFFFFFFF, 0b111]
    assert bits[3].tolist() == [0, 0]


@pytest.mark.parametrize("n", [1, 31, 32, 33, 1000])
def test_binarize_unpacks_to_the_comparisons(oracle_lib, n):
    """Reading the words back bit by bit (little-endian bytes unpacked with
    numpy) gives the comparisons of every row, and a model's leaf indices
    built from those bits equal the ones built from the bins."""
    g0 = np.random.default_rng(n)
    F = 5
    bins = g0.integers(0, 20, (F, n)).astype(np.uint8)
    bf = g0.integers(0, F, 12).astype(np.int32)
    bk = g0.integers(-1, 21, 12).astype(np.int32)
    bits = oracle_lib.binarize(bins, bf, bk)
    unpacked = np.unpackbits(bits.astype("<u4").view(np.uint8), axis=1,
                             bitorder="little")[:, :n]
    assert np.array_equal(unpacked, (bins[bf].astype(np.int64) > bk[:, None]).astype(np.uint8))
    assert not np.unpackbits(bits.astype("<u4").view(np.uint8), axis=1,
                             bitorder="little")[:, n:].any()
    T, d, K = 7, 3, 2
    sb = g0.integers(0, 12, (T, d)).astype(np.int32)
    vals = g0.standard_normal((T, 1 << d, K))
    a1 = np.zeros((K, n))
    oracle_lib.apply_model(bins, bf[sb], bk[sb], vals, 0.1, a1)
    a2 = np.zeros((K, n))
    for t in range(T):
        leaf = sum(unpacked[sb[t, l]].astype(np.int64) << l for l in range(d))
        for c in range(K):
            a2[c] = a2[c] + 0.1 * vals[t, leaf, c]
    assert np.array_equal(a1, a2)
