"""Input recipes: the cross-validation split of a problem (CPU only)."""
import numpy as np

import datagen


def test_cv_folds_partition_rows():
    p = datagen.random_small(seed=11, n=1003, F_num=3, F_cat=2, C=7, s=1)
    folds = datagen.cv_folds(p, 5)
    assert len(folds) == 5
    held = np.zeros(p.n, np.int64)
    for q in folds:
        assert q.n in (p.n - p.n // 5 - 1, p.n - p.n // 5)
        assert q.perms.shape == (1, q.n)
        assert np.array_equal(np.sort(q.perms[0]), np.arange(q.n))
        assert q.x_num.shape == (p.n_num, q.n) and q.cat.shape == (p.n_cat, q.n)
        assert q.depth == p.depth and q.loss == p.loss and q.num_bins == p.num_bins
    # every row is left out by exactly one fold: rebuild the split from the
    # recipe's own shuffle and compare the training columns
    order = datagen.rng_for(4, 200).permutation(p.n)
    parts = np.array_split(order, 5)
    for j, q in enumerate(folds):
        keep = np.ones(p.n, bool)
        keep[parts[j]] = False
        held[parts[j]] += 1
        assert np.array_equal(q.x_num, p.x_num[:, keep])
        assert np.array_equal(q.cat, p.cat[:, keep])
        assert np.array_equal(q.label, p.label[keep])
    assert np.all(held == 1)


def test_cv_folds_deterministic():
    p = datagen.random_small(seed=3, n=200, s=1)
    a, b = datagen.cv_folds(p, 4), datagen.cv_folds(p, 4)
    for x, y in zip(a, b):
        assert np.array_equal(x.perms, y.perms) and np.array_equal(x.label, y.label)
