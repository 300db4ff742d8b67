"""The context workspace under graph capture (include/cbhip.h,
cbh_reserve_workspace): a call whose stream is being captured never
allocates (it returns CBH_EBUSY and enqueues nothing if the workspace would
have to grow), and a graph captured over earlier calls stays valid after the
workspace has grown, because the earlier buffer is kept until cbh_destroy."""
import numpy as np
import pytest
import torch

import oracle
from tests import gpu_util as gu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cb():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1810_11363_amd import cbhip
    return cbhip


def _ids(n, C, seed):
    g = np.random.default_rng(seed)
    return g.integers(0, C, n).astype(np.int32)


def test_growth_during_capture_is_refused(cb):
    ctx = cb.cbh_create(0)
    try:
        small = _ids(5000, 50, 1)
        d_small = gu.to_dev(small)
        out_small = torch.empty(small.size, dtype=torch.int32, device=gu.dev())
        cb.cbh_category_counts(ctx, d_small, small.size, out_small)   # workspace sized here
        cb.cbh_sync(ctx)
        size0 = cb.cbh_workspace_size(ctx)
        n_big = 32 << 20                       # needs 128 MB of workspace
        assert 4 * n_big > size0
        d_big = torch.zeros(n_big, dtype=torch.int32, device=gu.dev())
        out_big = torch.empty(n_big, dtype=torch.int32, device=gu.dev())
        stream = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=stream):
            with pytest.raises(cb.CbhError) as err:
                cb.cbh_category_counts(ctx, d_big, n_big, out_big, stream.cuda_stream)
            # a call that fits still captures normally
            cb.cbh_category_counts(ctx, d_small, small.size, out_small, stream.cuda_stream)
        assert err.value.code == cb.CBH_EBUSY
        assert "captured" in str(err.value)
        assert cb.cbh_workspace_size(ctx) == size0
        out_small.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out_small.cpu().numpy(), oracle.category_counts(small))
        # outside the capture the same call grows the workspace and succeeds
        cb.cbh_category_counts(ctx, d_big, n_big, out_big)
        cb.cbh_sync(ctx)
        assert cb.cbh_workspace_size(ctx) >= 4 * n_big
        assert int(out_big[:16].min().item()) == n_big
    finally:
        cb.cbh_destroy(ctx)


def test_graph_survives_workspace_growth(cb):
    ctx = cb.cbh_create(0)
    try:
        a = _ids(70001, 300, 2)
        d_a = gu.to_dev(a)
        out_a = torch.empty(a.size, dtype=torch.int32, device=gu.dev())
        cb.cbh_category_counts(ctx, d_a, a.size, out_a)
        cb.cbh_sync(ctx)
        stream = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(graph, stream=stream):
            cb.cbh_category_counts(ctx, d_a, a.size, out_a, stream.cuda_stream)
        size0 = cb.cbh_workspace_size(ctx)
        # grow the workspace twice (a reservation, then a call), and let the
        # new buffer be written by eager work on other data between replays
        cb.cbh_reserve_workspace(ctx, 8 * size0)
        assert cb.cbh_workspace_size(ctx) >= 8 * size0
        b = _ids(3 << 20, 7, 3)
        d_b = gu.to_dev(b)
        out_b = torch.empty(b.size, dtype=torch.int32, device=gu.dev())
        want_a = oracle.category_counts(a)
        for rep in range(3):
            cb.cbh_category_counts(ctx, d_b, b.size, out_b)
            out_a.fill_(-1)
            graph.replay()
            torch.cuda.synchronize()
            assert np.array_equal(out_a.cpu().numpy(), want_a), rep
        cb.cbh_sync(ctx)
        assert np.array_equal(out_b.cpu().numpy(), oracle.category_counts(b))
        with pytest.raises(cb.CbhError) as err:
            cb.cbh_reserve_workspace(ctx, -1)
        assert err.value.code == cb.CBH_EINVAL
    finally:
        cb.cbh_destroy(ctx)
