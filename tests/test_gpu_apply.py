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
