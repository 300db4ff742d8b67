"""CPU-side checks of the C-ABI library: it loads, exports every symbol the
header declares, validates arguments on the host, and its host-only
computations (quantile borders, statistic borders) equal the oracle's
bit for bit. No device compute is launched here."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cbhip.h")


def _header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(cbh_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def cb():
    from paper_1810_11363_amd import cbhip
    return cbhip


def test_library_exports_every_header_symbol(cb):
    declared = _header_functions()
    assert len(declared) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", cb.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (cbh_[a-z_0-9]+)", out))
    missing = [n for n in declared if n not in exported]
    assert not missing, missing
    assert sorted(cb.EXPORTS) == declared
    for name in declared:
        assert getattr(cb.lib(), name) is not None


def test_library_is_gfx950_only(cb):
    """The embedded device code objects target gfx950 and nothing else."""
    blob = open(cb.LIB_PATH, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa-+(gfx[0-9a-z]+)", blob))
    assert targets == {b"gfx950"}, targets


def test_null_arguments_rejected_without_launch(cb):
    L = cb.lib()
    assert L.cbh_quantize(None, None, 10, None, 3, None, None) == cb.CBH_EINVAL
    assert "ctx" in cb.cbh_last_error()
    assert L.cbh_build_histograms(None, None, 0, 0, None, None) == cb.CBH_EINVAL
    assert L.cbh_score_splits(None, None, 0, None, 0, 1.0, None, None, None) == cb.CBH_EINVAL
    assert L.cbh_apply_split(None, None, 0, None, None) == cb.CBH_EINVAL
    assert L.cbh_update_approx(None, None, None, 0, None, 0.1, 1.0, None, None, None) == cb.CBH_EINVAL
    assert L.cbh_graph_launch(None, None) == cb.CBH_EINVAL
    assert L.cbh_set_workspace_limit(None, 10) == cb.CBH_EINVAL
    L.cbh_destroy(None)


def test_create_without_device_reports_error(cb):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    rc = cb.lib().cbh_create(0, C.byref(h))
    assert rc in (cb.CBH_EDEVICE, cb.CBH_EINVAL)
    assert h.value is None
    assert cb.cbh_last_error()


@pytest.mark.parametrize("max_bins", [2, 3, 33, 64, 128, 255, 256])
def test_select_borders_equals_oracle(cb, oracle_lib, max_bins):
    g = np.random.default_rng(max_bins)
    cols = [g.standard_normal(5000).astype(np.float32),
            np.exp(g.standard_normal(4999)).astype(np.float32),
            (g.integers(0, 60, 3001) * 0.25).astype(np.float32),
            np.full(17, 2.5, np.float32),
            np.array([1.0], np.float32),
            g.random(10007).astype(np.float32)]
    for x in cols:
        mine = cb.cbh_select_borders(x, max_bins)
        ref = oracle_lib.select_borders(x, max_bins)
        assert mine.dtype == np.float32
        assert np.array_equal(mine, ref)


def test_select_borders_errors(cb):
    with pytest.raises(cb.CbhError) as e:
        cb.cbh_select_borders(np.array([1.0, np.nan], np.float32), 4)
    assert e.value.code == cb.CBH_EINVAL
    with pytest.raises(cb.CbhError) as e:
        cb.cbh_select_borders(np.ones(4, np.float32), 257)
    assert e.value.code == cb.CBH_EUNSUPPORTED
    with pytest.raises(cb.CbhError) as e:
        cb.cbh_select_borders(np.ones(4, np.float32), 1)
    assert e.value.code == cb.CBH_EUNSUPPORTED
    assert cb.cbh_select_borders(np.zeros(0, np.float32), 8).size == 0


@pytest.mark.parametrize("lo,hi,nb", [(0.0, 1.0, 33), (-3.25, 7.5, 128), (0.0, 1.0, 255),
                                      (-1e-3, 2e3, 2), (1.0, 1.0, 64)])
def test_uniform_borders_equal_oracle(cb, oracle_lib, lo, hi, nb):
    assert np.array_equal(cb.cbh_uniform_borders(lo, hi, nb), oracle_lib.ts_borders(lo, hi, nb))


def test_uniform_borders_errors(cb):
    for args, code in [((1.0, 0.0, 8), cb.CBH_EINVAL), ((0.0, float("inf"), 8), cb.CBH_EINVAL),
                       ((0.0, 1.0, 1), cb.CBH_EUNSUPPORTED), ((0.0, 1.0, 300), cb.CBH_EUNSUPPORTED)]:
        with pytest.raises(cb.CbhError) as e:
            cb.cbh_uniform_borders(*args)
        assert e.value.code == code


def test_missing_library_fails_loudly(tmp_path):
    """Without libcbhip.so the binding refuses to import: there is no CPU path."""
    import shutil
    import sys
    pkg = os.path.join(ROOT, "paper_1810_11363_amd")
    dst = tmp_path / "paper_1810_11363_amd"
    dst.mkdir()
    for f in ("__init__.py", "cbhip.py"):
        shutil.copy(os.path.join(pkg, f), dst / f)
    code = ("import sys; sys.path.insert(0, %r)\n"
            "try:\n import paper_1810_11363_amd.cbhip\n print('LOADED')\n"
            "except ImportError as e:\n print('IMPORTERROR', e)\n") % str(tmp_path)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert "IMPORTERROR" in out.stdout and "LOADED" not in out.stdout


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 8, 9, 1000, 1 << 20, (1 << 20) + 1, 10 ** 6])
def test_ordered_layout_equals_oracle(cb, oracle_lib, n):
    """The supporting approximations' count and offsets (host-only calls)
    are those of the oracle's reading of Sec. 3."""
    M = cb.cbh_ordered_models(n)
    assert M == oracle_lib.ordered_models(n)
    if n <= 4097:
        off = oracle_lib.ordered_offsets(n)
        assert [cb.cbh_ordered_offset(n, m) for m in range(M + 1)] == off.tolist()
    assert cb.cbh_ordered_support_size(n) == cb.cbh_ordered_offset(n, M) < 4 * n
    assert cb.cbh_ordered_offset(n, M + 1) == -1
    assert cb.cbh_ordered_offset(n, -1) == -1
    assert cb.cbh_ordered_models(0) == 0 and cb.cbh_ordered_support_size(0) == 0


def test_ordered_calls_reject_null_without_launch(cb):
    p = cb.cbh_problem()
    o = cb.cbh_ordered()
    for call in (lambda: cb.cbh_ordered_gradients(None, o, p),
                 lambda: cb.cbh_ordered_update(None, o, p, 0.1, 3.0, None)):
        with pytest.raises(cb.CbhError) as err:
            call()
        assert err.value.code == cb.CBH_EINVAL


def test_combination_calls_reject_null_without_launch(cb):
    L = cb.lib()
    assert L.cbh_split_values(None, None, None, 0, 10, None, None, None) == cb.CBH_EINVAL
    assert "ctx" in cb.cbh_last_error()
    assert L.cbh_ts_bins(None, None, None, 10, 0, 1.0, 0.5, None, 0, None, None,
                         None) == cb.CBH_EINVAL
    assert C.sizeof(cb.cbh_split_source) == 32
    assert L.cbh_category_order(None, None, None, 10, None, None, None, None) == cb.CBH_EINVAL
    assert L.cbh_ordered_ts_crossings(None, None, 20, 2, None, None, 10, None, 1, 0, 1, 1.0, 1,
                                      None, None, 0, 0, None, 10, None) == cb.CBH_EINVAL
    assert L.cbh_counter_bins(None, None, 10, 16, None, None) == cb.CBH_EINVAL
