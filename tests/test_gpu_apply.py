"""Model apply (the oblivious-tree scorer of Sec. 4) through the C-ABI,
against the CPU oracle: bit-exact, since both add lr * v in double, tree
after tree in model order, from leaves that are integer decisions."""
import numpy as np
import pytest

import datagen
import oracle
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_11363_amd import cbhip
    return cbhip


@pytest.fixture(scope="module")
def ctx(cb):
    c = cb.cbh_create(0)
    yield c
    torch.cuda.synchronize()
    cb.cbh_destroy(c)


def _device_bins(bins, tiled):
    """Device bins of [F][n] host bins: plain columns, or the 16-row tiled
    layout [ceil(n/16)][F][16] with per-feature segment strides 16 F.
    Returns (pointer table, seg strides or None, keep-alive tensors)."""
    F, n = bins.shape
    dev = gu.dev()
    if not tiled:
        cols = [torch.from_numpy(np.ascontiguousarray(bins[f])).to(dev) for f in range(F)]
        table = torch.tensor([c.data_ptr() for c in cols], dtype=torch.int64, device=dev)
        return table, None, cols
    ns = (n + 15) // 16
    t = np.zeros((ns, F, 16), np.uint8)
    pad = np.zeros((F, ns * 16), np.uint8)
    pad[:, :n] = bins
    t[:] = pad.reshape(F, ns, 16).transpose(1, 0, 2)
    buf = torch.from_numpy(t.reshape(-1)).to(dev)
    table = torch.tensor([buf.data_ptr() + 16 * f for f in range(F)], dtype=torch.int64,
                         device=dev)
    seg = torch.full((F,), 16 * F, dtype=torch.int64, device=dev)
    return table, seg, [buf]


def _apply(cb, ctx, bins, feat, border, values, lr, a0, tiled):
    F, n = bins.shape
    T, d = feat.shape
    K = values.shape[-1]
    table, seg, keep = _device_bins(bins, tiled)
    dev = gu.dev()
    df = torch.from_numpy(np.ascontiguousarray(feat, np.int32)).to(dev)
    db = torch.from_numpy(np.ascontiguousarray(border, np.int32)).to(dev)
    dv = torch.from_numpy(np.ascontiguousarray(values, np.float64)).to(dev)
    da = torch.from_numpy(np.ascontiguousarray(a0, np.float64)).to(dev)
    cb.cbh_apply_model(ctx, table, seg, n, F, K, T, d, df, db, dv, lr, da)
    cb.cbh_sync(ctx)
    out = da.cpu().numpy()
    del keep
    return out


def _random_model(g0, F, T, d, K, B):
    feat = g0.integers(0, F, (T, d)).astype(np.int32)
    border = g0.integers(-1, B, (T, d)).astype(np.int32)
    border[g0.random((T, d)) < 0.05] = 255
    values = g0.normal(size=(T, 1 << d, K))
    return feat, border, values


APPLY_CASES = [
    # n, F, T, d, K, B
    (1, 3, 4, 2, 1, 8),
    (3, 2, 7, 1, 1, 2),
    (17, 5, 9, 3, 1, 33),
    (1000, 12, 25, 6, 1, 128),
    (4099, 7, 40, 8, 1, 255),
    (65539, 20, 60, 6, 1, 256),
    (1003, 9, 12, 5, 3, 64),
    (5001, 30, 8, 10, 10, 255),
    (259, 4, 5, 16, 2, 16),
]


@pytest.mark.parametrize("tiled", [False, True])
@pytest.mark.parametrize("case", APPLY_CASES)
def test_apply_model_bit_exact(cb, ctx, case, tiled):
    n, F, T, d, K, B = case
    g0 = np.random.default_rng(hash(case) % 10007)
    bins = g0.integers(0, B, (F, n)).astype(np.uint8)
    feat, border, values = _random_model(g0, F, T, d, K, B)
    a0 = g0.normal(size=(K, n))
    want = oracle.apply_model(bins, feat, border, values, 0.3, a0.copy())
    got = _apply(cb, ctx, bins, feat, border, values, 0.3, a0, tiled)
    assert np.array_equal(got, want)


def test_apply_model_reproduces_oracle_training(cb, ctx):
    """A model grown by the oracle, applied on the GPU to its training rows,
    gives the oracle's training approx bit for bit."""
    from oracle import boost
    p = datagen.make_c1(n=3000)
    p.iterations = 8
    trees, approx, prep = boost.fit(p)
    bins, _ = prep.tree_features(0)
    T, d = len(trees), p.depth
    feat = np.zeros((T, d), np.int32)
    border = np.full((T, d), 255, np.int32)
    for t, tr in enumerate(trees):
        for l, (f, k, _, _) in enumerate(tr.splits):
            if f >= 0:
                feat[t, l], border[t, l] = f, k
    values = np.stack([tr.values for tr in trees])
    got = _apply(cb, ctx, bins, feat, border, values, p.lr, np.zeros_like(approx), False)
    assert np.array_equal(got, approx)


def test_apply_model_bad_feature_reported(cb, ctx):
    """A split feature outside [0, F) reads nothing, counts as bit 0 and is
    reported by cbh_sync."""
    g0 = np.random.default_rng(77)
    n, F, T, d, K = 500, 4, 3, 3, 1
    bins = g0.integers(0, 16, (F, n)).astype(np.uint8)
    feat, border, values = _random_model(g0, F, T, d, K, 16)
    bad = feat.copy()
    bad[1, 2] = F
    table, seg, keep = _device_bins(bins, False)
    dev = gu.dev()
    df = torch.from_numpy(bad).to(dev)
    db = torch.from_numpy(border).to(dev)
    dv = torch.from_numpy(values).to(dev)
    da = torch.zeros((K, n), dtype=torch.float64, device=dev)
    cb.cbh_apply_model(ctx, table, seg, n, F, K, T, d, df, db, dv, 1.0, da)
    with pytest.raises(cb.CbhError):
        cb.cbh_sync(ctx)
    cb.cbh_sync(ctx)                       # the flag is cleared
    b2 = border.copy()
    b2[1, 2] = 255                         # the same model with that bit never set
    want = oracle.apply_model(bins, feat, b2, values, 1.0, np.zeros((K, n)))
    assert np.array_equal(da.cpu().numpy(), want)
    del keep


def test_apply_model_arguments(cb, ctx):
    dev = gu.dev()
    a = torch.zeros((1, 8), dtype=torch.float64, device=dev)
    # nothing to do: no trees, or no rows
    cb.cbh_apply_model(ctx, None, None, 8, 3, 1, 0, 4, None, None, None, 1.0, a)
    cb.cbh_apply_model(ctx, None, None, 0, 3, 1, 5, 4, None, None, None, 1.0, a)
    with pytest.raises(cb.CbhError):
        cb.cbh_apply_model(ctx, None, None, 8, 3, 17, 5, 4, None, None, None, 1.0, a)
    with pytest.raises(cb.CbhError):
        cb.cbh_apply_model(ctx, None, None, 8, 3, 1, 5, 17, None, None, None, 1.0, a)
    with pytest.raises(cb.CbhError):
        cb.cbh_apply_model(ctx, None, None, 8, 3, 1, 5, 4, None, None, None, 1.0, a)
    with pytest.raises(cb.CbhError):
        cb.cbh_apply_model(ctx, None, None, 8, 3, 1, 5, 4, a, a, a, float("inf"), a)
    cb.cbh_sync(ctx)


def _binary_table(feat, border):
    """The model's distinct (feature, border) pairs in (feature, border)
    order, and every split's index among them."""
    pairs = np.stack([feat.reshape(-1), border.reshape(-1)], 1).astype(np.int64)
    uniq, inv = np.unique(pairs, axis=0, return_inverse=True)
    return (uniq[:, 0].astype(np.int32), uniq[:, 1].astype(np.int32),
            inv.reshape(feat.shape).astype(np.int32))


@pytest.mark.parametrize("tiled", [False, True])
@pytest.mark.parametrize("case", APPLY_CASES)
def test_binarized_apply_bit_exact(cb, ctx, case, tiled):
    """Sec. 4's two steps: cbh_binarize's bits equal the oracle's binary
    features, and the model applied from them equals the oracle's model
    apply (and so cbh_apply_model) bit for bit."""
    n, F, T, d, K, B = case
    g0 = np.random.default_rng(hash(case) % 10009)
    bins = g0.integers(0, B, (F, n)).astype(np.uint8)
    feat, border, values = _random_model(g0, F, T, d, K, B)
    a0 = g0.normal(size=(K, n))
    bf, bk, sb = _binary_table(feat, border)
    nb = bf.size
    nw = (n + 31) // 32
    table, seg, keep = _device_bins(bins, tiled)
    dev = gu.dev()
    bits = torch.full((nb, nw), 0x5A5A5A5A, dtype=torch.int32, device=dev)
    cb.cbh_binarize(ctx, table, seg, n, F, nb, gu.to_dev(bf), gu.to_dev(bk), bits)
    cb.cbh_sync(ctx)
    want_bits = oracle.binarize(bins, bf, bk)
    assert np.array_equal(bits.cpu().numpy().view(np.uint32), want_bits)
    da = gu.to_dev(a0)
    cb.cbh_apply_model_binarized(ctx, bits, n, nb, K, T, d, gu.to_dev(sb),
                                 gu.to_dev(values), 0.1, da)
    cb.cbh_sync(ctx)
    want = a0.copy()
    oracle.apply_model(bins, feat, border, values, 0.1, want)
    assert np.array_equal(da.cpu().numpy(), want)
    del keep


def test_binarized_apply_reports_bad_indices(cb, ctx):
    """A binary feature outside the features gives zero bits, a split index
    outside the binary features reads bit 0; both are reported by cbh_sync."""
    n, F = 100, 3
    g0 = np.random.default_rng(5)
    bins = g0.integers(0, 8, (F, n)).astype(np.uint8)
    table, seg, keep = _device_bins(bins, False)
    bits = torch.zeros((2, 4), dtype=torch.int32, device=gu.dev())
    cb.cbh_binarize(ctx, table, seg, n, F, 2, gu.to_dev(np.array([0, 7], np.int32)),
                    gu.to_dev(np.array([3, 3], np.int32)), bits)
    with pytest.raises(cb.CbhError):
        cb.cbh_sync(ctx)
    got = bits.cpu().numpy().view(np.uint32)
    assert np.array_equal(got[0], oracle.binarize(bins, [0], [3])[0]) and not got[1].any()
    vals = np.arange(4, dtype=np.float64).reshape(1, 4, 1)
    da = torch.zeros((1, n), dtype=torch.float64, device=gu.dev())
    cb.cbh_apply_model_binarized(ctx, bits, n, 2, 1, 1, 2,
                                 gu.to_dev(np.array([[0, 5]], np.int32)), gu.to_dev(vals), 1.0, da)
    with pytest.raises(cb.CbhError):
        cb.cbh_sync(ctx)
    want = (bins[0] > 3).astype(np.float64)           # leaf = bit 0 only
    assert np.array_equal(da.cpu().numpy()[0], want)
    del keep
