"""cbh_score_splits_noalloc (the split scoring for callers that cannot
allocate) against cbh_score_splits: the same best split and per-border scores
bit for bit, on two calls in a row, the second on a smaller problem (fewer
features and rows), from a context whose workspace stays empty."""
import numpy as np
import pytest
import torch

import datagen
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_11363_amd import cbhip
    return cbhip


def _grow_to(cb, bst, level):
    """Histograms of `level` of the booster's first tree, the levels before it
    split by the booster's own calls."""
    pr = bst.probs[0]
    bst.init_gradients()
    if bst.precision == gu.INT16:
        cb.cbh_quantize_gradients(bst.ctx, pr, bst.stream)
    for lvl in range(level + 1):
        bst.build_level_histograms(pr, lvl)
        cb.cbh_score_splits(bst.ctx, pr, lvl, bst.hist_ptr(lvl), bst.precision, bst.l2,
                            bst.split_ptr(lvl), None, bst.stream)
        if lvl < level:
            bst.advance(pr, lvl)
    torch.cuda.synchronize()
    return pr


@pytest.mark.parametrize("prec", [gu.F64, gu.INT16, gu.FP32])
def test_noalloc_matches_score_splits(cb, prec):
    from paper_1810_11363_amd.booster import GpuBooster
    ctx = cb.cbh_create(0)
    try:
        assert cb.cbh_workspace_size(ctx) == 0
        cases = [(datagen.make_c2(n=40000, s=1), 3), (datagen.make_c1(n=3000), 1)]
        for call, (p, level) in enumerate(cases):
            bst = GpuBooster.from_problem(p, precision=prec, partition=False).prepare()
            try:
                pr = _grow_to(cb, bst, level)
                hist = bst.hist_ptr(level)
                F, B = bst.F, bst.B
                ref_best = torch.zeros(4, dtype=torch.int32, device=gu.dev())
                got_best = torch.full((4,), -7, dtype=torch.int32, device=gu.dev())
                ref_sc = torch.zeros(F * (B - 1), dtype=torch.float32, device=gu.dev())
                got_sc = torch.full((F * (B - 1),), 7.0, dtype=torch.float32, device=gu.dev())
                cb.cbh_score_splits(bst.ctx, pr, level, hist, prec, bst.l2, ref_best, ref_sc)
                cb.cbh_score_splits_noalloc(ctx, pr, level, hist, prec, bst.l2, got_best, got_sc)
                cb.cbh_sync(ctx)
                assert torch.equal(ref_best, got_best), (call, ref_best, got_best)
                a, b = ref_sc.cpu().numpy(), got_sc.cpu().numpy()
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), call
                assert int(got_best[0].item()) >= 0, call
                # the call took nothing from the context's workspace
                assert cb.cbh_workspace_size(ctx) == 0, call
            finally:
                bst.close()
        # more features than the static scratch holds: refused, nothing enqueued
        p = datagen.make_c1(n=3000)
        bst = GpuBooster.from_problem(p, precision=prec).prepare()
        try:
            pr = bst.probs[0]
            pr.n_features = 65537
            with pytest.raises(cb.CbhError) as err:
                cb.cbh_score_splits_noalloc(ctx, pr, 0, bst.hist_ptr(0), prec, bst.l2,
                                            bst.split_ptr(0))
            assert err.value.code == cb.CBH_EINVAL
            assert "65536" in str(err.value)
        finally:
            bst.close()
    finally:
        cb.cbh_destroy(ctx)
