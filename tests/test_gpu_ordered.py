"""Ordered boosting's supporting approximations (Sec. 3) on the GPU against
the oracle: cbh_ordered_gradients and cbh_ordered_update on seeded leaves
(no split decision involved, so each side keeps its own state across trees),
and whole ordered trees in lock-step with the oracle.

Tolerance: the per-leaf sums are float64 in an order that varies between
runs (LDS adds), so leaf values agree to about n * 2^-53 of the summed
magnitude; supports and approximations inherit that (bound 1e-9 relative
to the magnitude of the values). Given equal supports the float32
gradients agree to one float32 rounding.
"""
import numpy as np
import pytest

import datagen
import oracle
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

REL = 1e-9


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_11363_amd import cbhip
    return cbhip


class _Ordered:
    """Device buffers of one problem with s permutations' supports."""

    def __init__(self, cb, ctx, *, n, K, loss, depth, label, perms):
        d = gu.dev()
        self.n, self.K, self.loss, self.depth = n, K, loss, depth
        self.cols_d = torch.zeros((1, n), dtype=torch.uint8, device=d)
        self.cols = gu.column_table(self.cols_d)
        self.nbins = torch.tensor([2], dtype=torch.uint16, device=d)
        self.label = gu.to_dev(label.astype(np.float32))
        self.g = torch.zeros((K, n), dtype=torch.float32, device=d)
        self.h = torch.zeros((K, n), dtype=torch.float32, device=d)
        self.leaf = torch.zeros(n, dtype=torch.uint16, device=d)
        self.approx = torch.zeros((K, n), dtype=torch.float64, device=d)
        self.prob = gu.make_problem(cb, n=n, F=1, B=2, K=K, loss=loss, depth=depth,
                                    cols=self.cols, nbins=self.nbins, label=self.label, g=self.g,
                                    h=self.h, leaf=self.leaf, approx=self.approx)
        S = cb.cbh_ordered_support_size(n)
        self.M = cb.cbh_ordered_models(n)
        self.perms = [gu.to_dev(p.astype(np.int32)) for p in perms]
        self.sup = [torch.zeros((K, S), dtype=torch.float64, device=d) for _ in perms]
        self.ords = [cb.make_ordered(n, p, s) for p, s in zip(self.perms, self.sup)]
        self.leaf_values = torch.zeros((1 << depth, K), dtype=torch.float64, device=d)
        self.sv = torch.zeros((self.M, 1 << depth, K), dtype=torch.float64, device=d)


def _labels(loss, K, n, g):
    if loss == 0:
        return g.normal(size=n).astype(np.float32)
    if loss == 1:
        return (g.random(n) < 0.35).astype(np.float32)
    return g.integers(0, K, n).astype(np.float32)


def _close(got, want, what):
    scale = max(1.0, float(np.abs(want).max()) if want.size else 1.0)
    err = float(np.abs(got - want).max()) if want.size else 0.0
    assert err <= REL * scale, (what, err, scale)
    return err


def _grads_close(o, perm, label, sup_host, what):
    rg, rh = oracle.ordered_gradients(o.loss, o.K, perm, label, sup_host)
    gg = o.g.cpu().numpy()
    assert np.max(np.abs(gg - rg.astype(np.float32))) <= 2e-7 * max(1.0, np.abs(rg).max()), what
    if o.loss != 0:
        hh = o.h.cpu().numpy()
        assert np.max(np.abs(hh - rh.astype(np.float32))) <= 2e-7, what


@pytest.mark.parametrize("loss,K,n,depth", [
    (0, 1, 1, 2), (1, 1, 2, 1), (0, 1, 1000, 3), (1, 1, 70001, 6), (0, 1, 70001, 10),
    (2, 3, 20011, 4), (2, 10, 4099, 3), (1, 1, 1 << 16, 5), (0, 1, 12, 12),
    (0, 1, 1000000, 6),
])
def test_ordered_update_matches_oracle(cb, loss, K, n, depth):
    """Seeded leaves for 4 trees: the kept model's leaf values and approx,
    every supporting model's leaf values and support, and the gradients for
    the next tree, against the oracle after every tree."""
    g = np.random.default_rng(1000 + n + depth)
    label = _labels(loss, K, n, g)
    perm = g.permutation(n).astype(np.int32)
    ctx = cb.cbh_create(0)
    try:
        o = _Ordered(cb, ctx, n=n, K=K, loss=loss, depth=depth, label=label, perms=[perm])
        S = o.sup[0].shape[1]
        sup_h = np.zeros((K, S))
        approx_h = np.zeros((K, n))
        cb.cbh_ordered_gradients(ctx, o.ords[0], o.prob)
        cb.cbh_sync(ctx)
        _grads_close(o, perm, label, sup_h, "init")
        lr, l2 = 0.3, 2.0
        for t in range(4):
            leaf = g.integers(0, 1 << depth, n).astype(np.uint16)
            o.leaf.copy_(gu.to_dev(leaf.astype(np.int32)).to(torch.uint16))
            cb.cbh_ordered_update(ctx, o.ords[0], o.prob, lr, l2, o.leaf_values, o.sv)
            cb.cbh_sync(ctx)
            # the kept model: its own gradients over all rows
            rg, rh = oracle.gradients(loss, K, approx_h, label)
            rv = oracle.leaf_values(leaf, rg, rh, 1 << depth, l2)[0]
            _close(o.leaf_values.cpu().numpy(), rv, ("kept values", t))
            oracle.update_approx(approx_h, leaf, rv, lr)
            _close(o.approx.cpu().numpy(), approx_h, ("approx", t))
            # the supporting models
            vals = oracle.ordered_update(loss, K, perm, label, leaf, 1 << depth, lr, l2, sup_h)
            _close(o.sv.cpu().numpy(), vals, ("support values", t))
            _close(o.sup[0].cpu().numpy(), sup_h, ("support", t))
            _grads_close(o, perm, label, sup_h, ("grads", t))
    finally:
        cb.cbh_destroy(ctx)


def test_ordered_update_without_kept_model_and_several_permutations(cb):
    """Two permutations: the tree goes into both supports; the call without
    leaf_values leaves the kept model alone, and the last call's permutation
    gives the gradients."""
    n, K, loss, depth = 30011, 1, 1, 4
    g = np.random.default_rng(7)
    label = _labels(loss, K, n, g)
    perms = [g.permutation(n).astype(np.int32) for _ in range(2)]
    ctx = cb.cbh_create(0)
    try:
        o = _Ordered(cb, ctx, n=n, K=K, loss=loss, depth=depth, label=label, perms=perms)
        S = o.sup[0].shape[1]
        sups = [np.zeros((K, S)) for _ in perms]
        for t in range(3):
            leaf = g.integers(0, 1 << depth, n).astype(np.uint16)
            o.leaf.copy_(gu.to_dev(leaf.astype(np.int32)).to(torch.uint16))
            before = o.approx.clone()
            first, second = (0, 1) if t % 2 == 0 else (1, 0)
            cb.cbh_ordered_update(ctx, o.ords[second], o.prob, 0.2, 1.0, None)
            cb.cbh_sync(ctx)
            assert torch.equal(o.approx, before)
            cb.cbh_ordered_update(ctx, o.ords[first], o.prob, 0.2, 1.0, o.leaf_values)
            cb.cbh_sync(ctx)
            for r in (second, first):
                oracle.ordered_update(loss, K, perms[r], label, leaf, 1 << depth, 0.2, 1.0,
                                      sups[r])
            for r in range(2):
                _close(o.sup[r].cpu().numpy(), sups[r], ("support", t, r))
            _grads_close(o, perms[first], label, sups[first], ("grads", t))
    finally:
        cb.cbh_destroy(ctx)


def test_ordered_bad_permutation_is_reported(cb):
    """A permutation entry outside [0, n) is skipped and reported by cbh_sync
    (every access stays in bounds)."""
    n = 5000
    g = np.random.default_rng(3)
    perm = g.permutation(n).astype(np.int32)
    perm[17] = n + 5
    ctx = cb.cbh_create(0)
    try:
        o = _Ordered(cb, ctx, n=n, K=1, loss=0, depth=3,
                     label=g.normal(size=n).astype(np.float32), perms=[perm])
        cb.cbh_ordered_gradients(ctx, o.ords[0], o.prob)
        with pytest.raises(cb.CbhError) as err:
            cb.cbh_sync(ctx)
        assert "permutation" in str(err.value)
        cb.cbh_ordered_update(ctx, o.ords[0], o.prob, 0.1, 1.0, o.leaf_values)
        with pytest.raises(cb.CbhError):
            cb.cbh_sync(ctx)
        cb.cbh_sync(ctx)   # the flag was cleared
    finally:
        cb.cbh_destroy(ctx)


def test_ordered_argument_errors(cb):
    n = 100
    ctx = cb.cbh_create(0)
    try:
        g = np.random.default_rng(4)
        o = _Ordered(cb, ctx, n=n, K=1, loss=0, depth=3,
                     label=g.normal(size=n).astype(np.float32), perms=[np.arange(n)])
        bad = cb.make_ordered(n + 1, o.perms[0], o.sup[0])
        with pytest.raises(cb.CbhError) as err:
            cb.cbh_ordered_gradients(ctx, bad, o.prob)
        assert err.value.code == cb.CBH_EINVAL
        o.prob.depth = 13           # 2^13 leaves x 1 class > 4096
        with pytest.raises(cb.CbhError) as err:
            cb.cbh_ordered_update(ctx, o.ords[0], o.prob, 0.1, 1.0, o.leaf_values)
        assert err.value.code == cb.CBH_EUNSUPPORTED
    finally:
        cb.cbh_destroy(ctx)


def _booster(cb, p, prec):
    from paper_1810_11363_amd.booster import GpuBooster
    return GpuBooster.from_problem(p, precision=prec, ordered=True).prepare()


@pytest.mark.parametrize("name,prec", [("c1", 3), ("c2_shape", 3), ("c2_shape", 2),
                                       ("c1", 0)])
def test_ordered_trees_lockstep(cb, name, prec):
    """Whole ordered trees (cbh_fit_tree_ordered, then the other permutation's
    support) against the oracle: before every tree the GPU's gradients are the
    oracle's ordered gradients of the oracle's own support; every level's
    split is checked against the oracle's score of the histogram of the
    gradients the tree used (margin rule); after the tree the leaves follow
    the splits, and every permutation's support and the kept model's leaf
    values and approx match the oracle's."""
    if name == "c1":
        p = datagen.make_c1()
    else:
        p = datagen.make_c2(n=30011, s=2)
    p.iterations = 4
    bst = _booster(cb, p, prec)
    n, K, L2, lr, s = bst.n, bst.K, bst.l2, bst.lr, bst.s
    perms = [bst.perm_d[r].cpu().numpy() for r in range(s)]
    S = cb.cbh_ordered_support_size(n)
    sup_h = [np.zeros((K, S)) for _ in range(s)]
    approx_h = np.zeros((K, n))
    ties = 0
    try:
        bst.init_gradients()
        for t in range(p.iterations):
            r = t % s
            torch.cuda.synchronize()
            rg, rh = oracle.ordered_gradients(bst.loss, K, perms[r], bst.label_h, sup_h[r])
            g32 = bst.g.cpu().numpy()
            assert np.max(np.abs(g32 - rg.astype(np.float32))) <= 2e-7 * max(1, np.abs(rg).max())
            h32 = bst.h.cpu().numpy() if bst.loss != 0 else np.ones((K, n), np.float32)
            bst.fit_tree(t)
            torch.cuda.synchronize()
            cb.cbh_sync(bst.ctx)
            leaf = bst.leaf.cpu().numpy()
            if prec == 2:
                gq = bst.gq.cpu().numpy()
                sc = bst.grad_scale.cpu().numpy().astype(np.float64)
                gd = gq[..., 0].astype(np.float64) * sc[:, 0:1]
                hd = (gq[..., 1].astype(np.float64) * sc[:, 1:2] if bst.loss != 0
                      else h32.astype(np.float64))
            else:
                gd, hd = g32.astype(np.float64), h32.astype(np.float64)
            bins = bst.bins_host(r)
            nb = bst.nbins_table[r].cpu().numpy()
            lv = np.zeros(n, np.uint16)
            for lvl in range(bst.depth):
                ref = oracle.score(oracle.histogram(bins, gd, hd, lv, 1 << lvl, bst.B), nb, L2)
                f, k, _, _ = gu.split_of(bst.best, lvl)
                ties += not gu.check_split((f, k), ref, nb)
                if f >= 0:
                    oracle.apply_split(bins[f], k, lvl, lv)
            assert np.array_equal(leaf, lv)
            kg, kh = oracle.gradients(bst.loss, K, approx_h, bst.label_h)
            kv = oracle.leaf_values(leaf, kg, kh, 1 << bst.depth, L2)[0]
            _close(bst.leaf_values.cpu().numpy(), kv, ("kept values", t))
            oracle.update_approx(approx_h, leaf, kv, lr)
            _close(bst.approx.cpu().numpy(), approx_h, ("approx", t))
            for r2 in range(s):
                oracle.ordered_update(bst.loss, K, perms[r2], bst.label_h, leaf, 1 << bst.depth,
                                      lr, L2, sup_h[r2])
                _close(bst.support[r2].cpu().numpy(), sup_h[r2], ("support", t, r2))
        print(name, prec, "near-ties", ties)
        assert ties <= p.iterations * bst.depth // 4
    finally:
        bst.close()
