"""Boosting driver on the GPU: device buffers from PyTorch, every step in libcbhip.

The loop follows the paper's classic scheme (Sec. 3, two-phase tree
building; Sec. 4, oblivious trees; the paper benchmarks this mode on GPU):
binarize numeric features, replace each categorical feature by its ordered
target statistic for each of s permutations (Sec. 2, Eq. 1), start from the
zero model, and for tree t use the statistic columns of permutation t mod s.

PyTorch only allocates device memory and supplies the stream; all arithmetic
of the method runs in the HIP library behind the C-ABI.

Device layout (HBM):
  numeric bins   uint8 [F_num][ld]            ld = n rounded up to 16
  statistic bins uint8 [s][F_cat * T][ld]     T targets per categorical feature
  tiled bins     uint8 [s][ceil(n/16)][F][16] layout "tiled" (default): for
                                              permutation r, the 16-row
                                              segments of all F features a tree
                                              reads, side by side
  column table   int64 [s][F]                 device pointers of the F features
                                              a tree of permutation r reads
  segment table  int64 [s][F]                 bytes between their 16-row
                                              segments (16 F tiled; 16 columns)
  n_bins         int32 [s][F]
  label float32 [n], g/h float32 [K][n], gq int16 [K][n][2], leaf uint16 [n],
  approx float64 [K][n]
  hist           the deepest level's histogram, reused by every level
"""
from __future__ import annotations

import ctypes as C
import os
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np
import torch

from . import cbhip as cb


def _ld(n: int) -> int:
    return (n + 15) // 16 * 16


@dataclass
class TreeRecord:
    splits: np.ndarray        # int32 [depth][2] (feature, border)
    scores: np.ndarray        # float32 [depth][2] (score, margin)
    values: np.ndarray        # float64 [2^depth][K]


class GpuBooster:
    """One boosting problem resident on one GPU."""

    def __init__(self, *, x_num, cat, label, perms, y_num, y_shift, priors, loss, K, depth,
                 lr, l2, num_bins, ts_bins, a, ts_lo, ts_hi, precision=cb.CBH_PREC_FP32,
                 subtract=None, device="cuda:0", ctx=None, stream=None, layout="tiled",
                 borders=None, partition=None, ordered=False, extra_priors=(),
                 combinations=False, counters=False):
        self.device = torch.device(device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.graphs = []
        self.own_ctx = ctx is None
        self.ctx = ctx if ctx is not None else cb.cbh_create(self.device.index or 0)
        self.loss, self.K, self.depth = int(loss), int(K), int(depth)
        self.lr, self.l2 = float(lr), float(l2)
        self.num_bins, self.ts_bins, self.a = int(num_bins), int(ts_bins), float(a)
        self.precision = int(precision)
        if layout not in ("tiled", "columns"):
            raise ValueError(f"layout must be 'tiled' or 'columns', not {layout!r}")
        self.layout = layout
        # histogram subtraction at levels >= 1: exact for int16, two-float
        # difference for the compensated form; off for plain float32 by default
        self.subtract = (self.precision != cb.CBH_PREC_FP32) if subtract is None else bool(subtract)
        # rows kept in leaf order during a tree (levels >= 1 read each row once
        # whatever the number of leaves, at the cost of moving the rows after
        # every split). None: for several classes, and for deep trees (depth
        # >= 8) in the float forms; the int16 form of one class keeps
        # subtraction in the original order, which is cheaper there
        self.partition = partition if partition is None else bool(partition)
        self.part = None
        self.use_part = False
        self.x_num = np.ascontiguousarray(x_num, dtype=np.float32)
        self.cat = np.ascontiguousarray(cat, dtype=np.int32)
        self.label_h = np.ascontiguousarray(label, dtype=np.float32)
        self.perms = np.ascontiguousarray(perms, dtype=np.int32)
        self.y_num = np.ascontiguousarray(y_num, dtype=np.int64)
        self.y_shift, self.priors = int(y_shift), [float(p) for p in priors]
        self.ts_lo, self.ts_hi = float(ts_lo), float(ts_hi)
        self.n = int(self.label_h.shape[0])
        self.F_num, self.F_cat = self.x_num.shape[0], self.cat.shape[0]
        self.T = self.y_num.shape[0] if self.F_cat else 0
        self.s = self.perms.shape[0] if self.F_cat else 1
        # several priors (Sec. 2): target t's statistic columns use priors[t]
        # and then every extra prior, one column each
        self.extra_priors = [float(v) for v in extra_priors]
        self.Q = 1 + len(self.extra_priors)
        # the counter statistic (Sec. 2): one more column per categorical
        # feature (and per crossing), after its statistic columns
        self.counters = bool(counters) and self.F_cat > 0
        self.CPC = self.T * self.Q + (1 if self.counters else 0)
        self.F = self.F_num + self.F_cat * self.CPC
        # greedy feature combinations (Sec. 2): candidate columns added level
        # by level from the tree's own splits (direct builds in the original
        # row order)
        self.combinations = bool(combinations) and self.F_cat > 0
        if self.combinations and ordered:
            raise ValueError("combination trees are built in the plain scheme only")
        self.F_hist = self.F
        # numeric borders chosen elsewhere (e.g. on the whole dataset before a
        # split into folds), one float32 array per numeric feature; None: chosen
        # here from x_num
        self.given_borders = None if borders is None else [
            np.ascontiguousarray(v, dtype=np.float32) for v in borders]
        if self.given_borders is not None and len(self.given_borders) != self.x_num.shape[0]:
            raise ValueError("borders needs one array per numeric feature")
        self.timings = {}
        # ordered boosting (Sec. 3): tree structures chosen on the gradients of
        # the supporting approximations of permutation t mod s
        self.ordered = bool(ordered)
        # bins read by the trees: 8 (bytes) or packed 4 / 1 bits (set_bin_bits)
        self.bin_bits = 8
        self._packed = {}
        self._alloc()

    @classmethod
    def from_problem(cls, p, **kw):
        """Build from a datagen-style problem object (attribute names as below)."""
        return cls(x_num=p.x_num, cat=p.cat, label=p.label, perms=p.perms, y_num=p.y_num,
                   y_shift=p.y_shift, priors=p.priors, loss=p.loss, K=p.K, depth=p.depth,
                   lr=p.lr, l2=p.l2, num_bins=p.num_bins, ts_bins=p.ts_bins, a=p.a,
                   ts_lo=p.ts_lo, ts_hi=p.ts_hi,
                   extra_priors=getattr(p, "extra_priors", []),
                   counters=getattr(p, "counters", False), **kw)

    # ---------------------------------------------------------------- buffers
    def _alloc(self):
        d, n, K = self.device, self.n, self.K
        ld = _ld(n)
        self.ld = ld
        self.num_bins_d = torch.empty((max(self.F_num, 1), ld), dtype=torch.uint8, device=d)
        self.ts_bins_d = torch.empty((self.s, max(self.F_cat * self.CPC, 1), ld),
                                     dtype=torch.uint8, device=d)
        self.label = torch.from_numpy(self.label_h).to(d)
        self.g = torch.empty((K, n), dtype=torch.float32, device=d)
        self.h = torch.empty((K, n), dtype=torch.float32, device=d)
        self.gq = torch.empty((K, n, 2), dtype=torch.int16, device=d)
        self.grad_scale = torch.zeros((K, 2), dtype=torch.float32, device=d)
        self.leaf = torch.zeros(n, dtype=torch.uint16, device=d)
        self.approx = torch.zeros((K, n), dtype=torch.float64, device=d)
        self.best = torch.zeros((self.depth, 4), dtype=torch.int32, device=d)   # cbh_split[depth]
        self.leaf_values = torch.zeros((1 << self.depth, K), dtype=torch.float64, device=d)
        self.leaf_counts = torch.zeros(1 << self.depth, dtype=torch.int64, device=d)
        self.n_borders = np.zeros(self.F_num, np.int32)
        if self.ordered:
            self._alloc_ordered()

    def _alloc_ordered(self):
        d, n, K = self.device, self.n, self.K
        if getattr(self, "ords", None) is None:
            S = cb.cbh_ordered_support_size(n)
            self.support = [torch.zeros((K, S), dtype=torch.float64, device=d)
                            for _ in range(self.s)]
            # the permutations of the ordered statistics (Sec. 3 uses the same
            # ones); the identity where the problem brings none
            self.perm_d = [torch.from_numpy(np.ascontiguousarray(
                self.perms[r] if r < self.perms.shape[0] else np.arange(n), dtype=np.int32)).to(d)
                for r in range(self.s)]
            self.ords = [cb.make_ordered(n, self.perm_d[r], self.support[r])
                         for r in range(self.s)]

    def _hist_bytes(self, level: int) -> int:
        esz = 4 if self.precision == cb.CBH_PREC_FP32 else 8
        return (1 << level) * self.F_hist * self.B * 2 * self.K * esz

    def prior_lists(self):
        """Priors of every statistic target: its own, then the extra ones."""
        return [[self.priors[t]] + self.extra_priors for t in range(self.T)]

    # ----------------------------------------------------------- preprocessing
    def prepare(self):
        """Borders (host), bins and ordered statistics (device); once per dataset."""
        d, n = self.device, self.n
        st = self.stream
        torch.cuda.synchronize(d)
        t0 = time.perf_counter()
        # host border selection, one feature per task (the library call runs
        # without the interpreter lock)
        if self.given_borders is not None:
            borders = self.given_borders
        else:
            with ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1))) as ex:
                borders = list(ex.map(
                    lambda f: cb.cbh_select_borders(self.x_num[f], self.num_bins),
                    range(self.F_num)))
        t1 = time.perf_counter()
        self.num_borders = borders
        x_d = torch.from_numpy(self.x_num).to(d)
        bord_d = torch.zeros((max(self.F_num, 1), 256), dtype=torch.float32, device=d)
        for f, b in enumerate(borders):
            self.n_borders[f] = b.size
            if b.size:
                bord_d[f, : b.size] = torch.from_numpy(b).to(d)
        torch.cuda.synchronize(d)
        t2 = time.perf_counter()
        for f in range(self.F_num):
            cb.cbh_quantize(self.ctx, x_d[f], n, bord_d[f], int(self.n_borders[f]),
                            self.num_bins_d[f], st)
        torch.cuda.synchronize(d)
        t3 = time.perf_counter()
        self.ts_borders_h = cb.cbh_uniform_borders(self.ts_lo, self.ts_hi, self.ts_bins)
        ts_b = torch.from_numpy(self.ts_borders_h).to(d)
        t4 = t5 = t3
        if self.F_cat:
            cat_d = torch.from_numpy(self.cat).to(d)
            perm_d = torch.from_numpy(self.perms).to(d)
            y_d = torch.from_numpy(self.y_num).to(d)
            yabs = int(np.abs(self.y_num).max()) if self.y_num.size else 0
            tmp = torch.empty((self.T, n), dtype=torch.uint8, device=d) if self.ld != n else None
            torch.cuda.synchronize(d)
            t4 = time.perf_counter()
            if self.Q > 1:
                num_t = torch.empty((self.T, n), dtype=torch.int64, device=d)
                den_t = torch.empty(n, dtype=torch.int32, device=d)
                pl = self.prior_lists()
            for r in range(self.s):
                for c in range(self.F_cat):
                    if self.Q > 1:
                        # the grouping once, then one column per (target, prior)
                        cb.cbh_compute_ordered_ts(self.ctx, cat_d[c], perm_d[r], n, y_d, self.T,
                                                  self.y_shift, yabs, self.a, self.priors,
                                                  None, 0, num_out=num_t, den_out=den_t,
                                                  stream=st)
                        for t in range(self.T):
                            for q in range(self.Q):
                                cb.cbh_ts_bins(self.ctx, num_t[t], den_t, n, self.y_shift,
                                               self.a, pl[t][q], ts_b, self.ts_bins - 1,
                                               ts_bin_out=self.ts_bins_d[r, c * self.CPC
                                                                         + t * self.Q + q],
                                               stream=st)
                        continue
                    dst = self.ts_bins_d[r, c * self.CPC:c * self.CPC + self.T]
                    out = tmp if tmp is not None else dst
                    cb.cbh_compute_ordered_ts(self.ctx, cat_d[c], perm_d[r], n, y_d, self.T,
                                              self.y_shift, yabs, self.a, self.priors, ts_b,
                                              self.ts_bins - 1, ts_bin_out=out, stream=st)
                    if tmp is not None:
                        dst[:, :n].copy_(tmp)
            if self.counters:
                ids = torch.empty(n, dtype=torch.int32, device=d)
                cnt = torch.empty(n, dtype=torch.int32, device=d)
                for c in range(self.F_cat):
                    cb.cbh_category_order(self.ctx, cat_d[c], None, n, None, ids, None, st)
                    cb.cbh_category_counts(self.ctx, ids, n, cnt, st)
                    for r in range(self.s):
                        cb.cbh_counter_bins(self.ctx, cnt, n, self.ts_bins,
                                            self.ts_bins_d[r, c * self.CPC + self.T * self.Q], st)
            torch.cuda.synchronize(d)
            t5 = time.perf_counter()
        cb.cbh_sync(self.ctx, st)
        self.timings.update(borders_s=t1 - t0, quantize_s=t3 - t2, ordered_ts_s=t5 - t4)
        # per-permutation column tables and bin counts
        nb_num = (self.n_borders + 1).astype(np.int32)
        self.B = int(max(nb_num.max() if self.F_num else 2, self.ts_bins if self.F_cat else 2))
        cols, nbs = [], []
        for r in range(self.s):
            ptrs = [self.num_bins_d[f].data_ptr() for f in range(self.F_num)]
            ptrs += [self.ts_bins_d[r, j].data_ptr() for j in range(self.F_cat * self.CPC)]
            cols.append(ptrs)
            nbs.append(np.concatenate([nb_num, np.full(self.F_cat * self.CPC,
                                                       self.ts_bins, np.int32)]))
        self.col_table = torch.tensor(cols, dtype=torch.int64, device=d)
        self.seg_table = None
        if self.layout == "tiled":
            # one tiled matrix per permutation: the numeric segments are
            # repeated in each, so every lane group of features reads one
            # contiguous run of 16-byte segments
            T = (n + 15) // 16
            self.tiled = torch.empty((self.s, T, self.F, 16), dtype=torch.uint8, device=d)
            torch.cuda.synchronize(d)
            t6 = time.perf_counter()
            for r in range(self.s):
                cb.cbh_tile_bins(self.ctx, self.col_table[r], self.F, n, self.tiled[r], st)
            cb.cbh_sync(self.ctx, st)
            self.timings["tile_s"] = time.perf_counter() - t6
            base = [self.tiled[r].data_ptr() for r in range(self.s)]
            self.col_table = torch.tensor([[b + 16 * f for f in range(self.F)] for b in base],
                                          dtype=torch.int64, device=d)
            self.seg_table = torch.full((self.s, self.F), 16 * self.F, dtype=torch.int64,
                                        device=d)
        self.nbins_table = torch.from_numpy(np.stack(nbs).astype(np.int32)).to(d)
        if self.combinations:
            self._alloc_combos(ts_b)
        self._alloc_hists()
        self.probs = [self.problem(r) for r in range(self.s)]
        if self.combinations:
            self._choose_order()
            return self
        if self.partition or (self.partition is None and (self.K > 1 or self.depth >= 8)):
            self.part = cb.cbh_part_create(self.ctx, self.probs[0])
        self._choose_order()
        return self

    def _choose_order(self):
        if self.part is None or self.combinations:
            self.use_part = False
        elif self.partition is not None:
            self.use_part = bool(self.partition)
        else:
            self.use_part = self.K > 1 or self.precision != cb.CBH_PREC_INT16

    def _alloc_combos(self, ts_b):
        """Device state of combination trees: every categorical feature's
        dense ids and, per permutation, its rows in (category, position)
        order; per level the dense ids of the split's value and the
        statistic bins of its crossings (rewritten by every tree); per
        permutation the extended column tables (the tree's columns, then
        every combination column a tree can reach) and the split source of
        every column."""
        d, n, ld = self.device, self.n, self.ld
        D, Cn, TQ = max(self.depth - 1, 1), self.F_cat, self.CPC
        self.F_combo = (self.depth - 1) * Cn * TQ
        self.F_hist = self.F + self.F_combo
        self.ts_borders_d = ts_b
        self.cat_d = torch.from_numpy(self.cat).to(d)
        self.perm_dc = torch.from_numpy(self.perms).to(d)
        self.y_dc = torch.from_numpy(self.y_num).to(d)
        self.y_abs = int(np.abs(self.y_num).max()) if self.y_num.size else 0
        self.c_dense = torch.empty((Cn, n), dtype=torch.int32, device=d)
        self.c_order = torch.empty((self.s, Cn, n), dtype=torch.int32, device=d)
        for r in range(self.s):
            for c in range(Cn):
                cb.cbh_category_order(self.ctx, self.cat_d[c], self.perm_dc[r], n,
                                      self.c_order[r, c], self.c_dense[c] if r == 0 else None,
                                      None, self.stream)
        self.e_dense = torch.zeros((D, n), dtype=torch.int32, device=d)
        self.e_bits = max(1, int(n - 1).bit_length())
        self.elem_a = torch.empty(n, dtype=torch.int32, device=d)
        self.elem_b = torch.empty(n, dtype=torch.int32, device=d)
        self.ndist = torch.empty(1, dtype=torch.int64, device=d)
        self.combo_bins = torch.zeros((D, Cn, TQ, ld), dtype=torch.uint8, device=d)
        self.c_order_tab = [torch.tensor([self.c_order[r, c].data_ptr() for c in range(Cn)],
                                         dtype=torch.int64, device=d) for r in range(self.s)]
        self.c_ids_tab = torch.tensor([self.c_dense[c].data_ptr() for c in range(Cn)],
                                      dtype=torch.int64, device=d)
        self.bins_tab = [torch.tensor([self.combo_bins[j, c].data_ptr() for c in range(Cn)],
                                      dtype=torch.int64, device=d) for j in range(D)]
        self.priors_flat = [p for pl in self.prior_lists() for p in pl]
        combo_ptrs = [self.combo_bins[j, c, q].data_ptr() for j in range(self.depth - 1)
                      for c in range(Cn) for q in range(TQ)]
        base = self.col_table.cpu().numpy()
        seg = (self.seg_table.cpu().numpy() if self.seg_table is not None
               else np.full((self.s, self.F), 16, np.int64))
        nbb = self.nbins_table.cpu().numpy()
        self.col_x = torch.tensor(np.concatenate(
            [base, np.tile(np.array(combo_ptrs, np.int64), (self.s, 1))], axis=1),
            dtype=torch.int64, device=d)
        self.seg_x = torch.tensor(np.concatenate(
            [seg, np.full((self.s, self.F_combo), 16, np.int64)], axis=1), dtype=torch.int64,
            device=d)
        self.nb_x = torch.tensor(np.concatenate(
            [nbb, np.full((self.s, self.F_combo), self.ts_bins, np.int32)], axis=1),
            dtype=torch.int32, device=d)
        srcs = []
        for r in range(self.s):
            a = np.zeros(self.F_hist, dtype=[("ptr", np.uint64), ("ptr_b", np.uint64),
                                              ("seg", np.int64), ("kind", np.int32),
                                              ("res", np.int32)])
            for f in range(self.F_hist):
                if f < self.F_num:
                    a[f] = (base[r, f], 0, seg[r, f], cb.CBH_SOURCE_BINS, 0)
                elif f < self.F:
                    c = (f - self.F_num) // TQ
                    a[f] = (self.c_dense[c].data_ptr(), 0, 0, cb.CBH_SOURCE_VALUES, 0)
                else:
                    j, c = divmod((f - self.F) // TQ, Cn)
                    a[f] = (self.e_dense[j].data_ptr(), self.c_dense[c].data_ptr(), 0,
                            cb.CBH_SOURCE_PAIR, 0)
            srcs.append(torch.from_numpy(a.view(np.uint8).copy()).to(d))
        self.src_x = srcs

    def combo_problem(self, r: int, level: int) -> cb.cbh_problem:
        """The problem a combination tree of permutation r sees at `level`:
        the tree's columns and the combination columns of the levels above."""
        p = self.problem(r)
        p.bins = self.col_x[r].data_ptr()
        p.seg_stride = self.seg_x[r].data_ptr()
        p.n_bins = self.nb_x[r].data_ptr()
        p.n_features = self.F + level * self.F_cat * self.CPC
        return p

    def combo_level(self, t: int, level: int):
        """Histograms (direct, every candidate) and the split of `level`."""
        pr = self.combo_problem(t % self.s, level)
        if level == 0 and self.precision == cb.CBH_PREC_INT16:
            cb.cbh_quantize_gradients(self.ctx, pr, self.stream)
        cb.cbh_build_histograms(self.ctx, pr, level, self.precision, self.hist_ptr(level),
                                self.stream)
        cb.cbh_score_splits(self.ctx, pr, level, self.hist_ptr(level), self.precision, self.l2,
                            self.split_ptr(level), None, self.stream)

    def combo_advance(self, t: int, level: int):
        """Set the level's leaf bit; then the split's value per row (on the
        device, from the split itself) is numbered densely and crossed with
        every categorical feature at once (one sort for all crossings), and
        each crossing's statistic bins (every target and prior, the tree's
        permutation) become candidates below."""
        r = t % self.s
        pr = self.combo_problem(r, level)
        ctx, st, n = self.ctx, self.stream, self.n
        cb.cbh_apply_split(ctx, pr, level, self.split_ptr(level), st)
        if level + 1 >= self.depth:
            return
        cb.cbh_split_values(ctx, self.split_ptr(level), self.src_x[r], pr.n_features, n,
                            self.elem_a, self.elem_b, st)
        cb.cbh_combine_categories(ctx, self.elem_a, self.elem_b, n, self.e_dense[level],
                                  self.ndist, st)
        cb.cbh_ordered_ts_crossings(ctx, self.e_dense[level], self.e_bits, self.F_cat,
                                    self.c_order_tab[r], self.c_ids_tab, n, self.y_dc, self.T,
                                    self.y_shift, self.y_abs, self.a, self.Q, self.priors_flat,
                                    self.ts_borders_d, self.ts_bins - 1, self.bins_tab[level],
                                    self.ld, self.ts_bins if self.counters else 0, st)

    def _combo_tree(self, t: int, counts: bool = False):
        for lvl in range(self.depth):
            self.combo_level(t, lvl)
            self.combo_advance(t, lvl)
        pr = self.combo_problem(t % self.s, self.depth - 1)
        cb.cbh_update_approx(self.ctx, pr, self.hist_ptr(self.depth - 1), self.precision,
                             self.split_ptr(self.depth - 1), self.lr, self.l2, self.leaf_values,
                             self.leaf_counts if counts else None, self.stream)

    def combo_bins_host(self, level: int) -> np.ndarray:
        """uint8 [level * F_cat * T * Q][n]: the combination columns that are
        candidates at `level` (for checks)."""
        m = level * self.F_cat * self.CPC
        if m == 0:
            return np.zeros((0, self.n), np.uint8)
        cols = self.combo_bins[:level].reshape(-1, self.ld)[:, : self.n]
        return cols.cpu().numpy()

    def _alloc_hists(self):
        hb = max(256, self._hist_bytes(self.depth - 1))
        self.hists = [torch.empty(hb, dtype=torch.uint8, device=self.device) for _ in range(2)]
        self.hist = self.hists[(self.depth - 1) % 2]     # the last level's histogram

    def set_precision(self, precision: int, subtract=None):
        """Switch the histogram form; keeps the prepared bins and statistics."""
        self.precision = int(precision)
        self.subtract = (self.precision != cb.CBH_PREC_FP32) if subtract is None else bool(subtract)
        torch.cuda.synchronize(self.device)
        self.drop_graphs()    # captured trees point at the old buffers
        self._alloc_hists()
        self._choose_order()

    def set_bin_bits(self, bits: int):
        """Trees read packed bins (Sec. 5: 4 bits for features of at most 15
        bins, 1 bit for binary ones) or bytes (8). Packed columns are made
        once per width from the byte layout, which stays for the checks."""
        bits = int(bits)
        if bits not in (8, 4, 1):
            raise ValueError("bits must be 8, 4 or 1")
        if bits != 8:
            if self.B > (1 << bits):
                raise ValueError(f"{self.B} bins do not fit in {bits} bits")
            if self.part is not None:
                raise ValueError("packed bins take no leaf-ordered rows (partition=False)")
            if self.combinations:
                raise ValueError("combination trees read byte bins")
        torch.cuda.synchronize(self.device)
        self.drop_graphs()
        if bits != 8 and bits not in self._packed:
            n, F = self.n, self.F
            nseg = (n + 15) // 16
            pk = torch.empty((self.s, F, nseg * 2 * bits), dtype=torch.uint8, device=self.device)
            tables = torch.tensor([[pk[r, f].data_ptr() for f in range(F)] for r in range(self.s)],
                                  dtype=torch.int64, device=self.device)
            for r in range(self.s):
                seg = self.seg_table[r] if self.seg_table is not None else None
                cb.cbh_pack_bins(self.ctx, self.col_table[r], seg, F, n, bits, tables[r],
                                 self.stream)
            cb.cbh_sync(self.ctx, self.stream)
            self._packed[bits] = (pk, tables)
        self.bin_bits = bits
        self.probs = [self.problem(r) for r in range(self.s)]

    def problem(self, r: int) -> cb.cbh_problem:
        p = cb.cbh_problem()
        p.n = self.n
        p.n_features = self.F
        p.max_bins = self.B
        p.bins = self.col_table[r].data_ptr()
        p.n_bins = self.nbins_table[r].data_ptr()
        p.K = self.K
        p.loss = self.loss
        p.depth = self.depth
        p.label = self.label.data_ptr()
        p.g = self.g.data_ptr()
        p.h = self.h.data_ptr()
        p.gq = self.gq.data_ptr()
        p.grad_scale = self.grad_scale.data_ptr()
        p.leaf = self.leaf.data_ptr()
        p.approx = self.approx.data_ptr()
        p.seg_stride = self.seg_table[r].data_ptr() if self.seg_table is not None else None
        if self.bin_bits != 8:
            p.bins = self._packed[self.bin_bits][1][r].data_ptr()
            p.seg_stride = None
            p.bin_bits = self.bin_bits
        return p

    def bins_host(self, r: int) -> np.ndarray:
        """uint8 [F][n] bins a tree of permutation r reads (copied to host, for
        checks): from the tiled matrix when the problem uses it."""
        if self.seg_table is not None:
            t = self.tiled[r].cpu().numpy()                      # [T][F][16]
            return np.ascontiguousarray(t.transpose(1, 0, 2).reshape(self.F, -1)[:, : self.n])
        parts = [self.num_bins_d[: self.F_num, : self.n]]
        if self.F_cat:
            parts.append(self.ts_bins_d[r, :, : self.n])
        return torch.cat(parts, 0).cpu().numpy()

    # ------------------------------------------------------------------ trees
    def split_ptr(self, level: int) -> int:
        return self.best.data_ptr() + 16 * level

    def set_ordered(self, ordered: bool):
        """Switch between ordered boosting (Sec. 3) and plain boosting; call
        init_gradients before the next tree."""
        self.ordered = bool(ordered)
        if self.ordered:
            self._alloc_ordered()

    def init_gradients(self):
        self.approx.zero_()
        if self.ordered:
            for sup in self.support:
                sup.zero_()
            cb.cbh_ordered_gradients(self.ctx, self.ords[0], self.probs[0], self.stream)
            return
        cb.cbh_update_approx(self.ctx, self.probs[0], None, self.precision, None, 0.0, 0.0,
                             stream=self.stream)

    def _ordered_tree(self, t: int):
        """Ordered tree t: levels on permutation t mod s's gradients, the kept
        model and that permutation's support in the same call, then the other
        permutations' supports, the next tree's permutation last (its
        gradients are the ones left in g, h)."""
        r, nxt = t % self.s, (t + 1) % self.s
        pr = self.probs[r]
        cb.cbh_fit_tree_ordered(self.ctx, pr, self.ords[r], self.part if self.use_part else None,
                                self.precision, self.subtract, self.hists, self.best, self.lr,
                                self.l2, self.leaf_values, None, self.stream)
        rest = [q for q in range(self.s) if q not in (r, nxt)]
        if nxt != r:
            rest.append(nxt)
        for q in rest:
            cb.cbh_ordered_update(self.ctx, self.ords[q], pr, self.lr, self.l2, None, None,
                                  self.stream)

    def subtract_levels(self) -> bool:
        """True when levels >= 1 accumulate only the smaller child of every
        parent (the other child is the parent minus it)."""
        return bool(self.subtract)

    def hist_ptr(self, level: int) -> int:
        """Level `level` writes buffer level % 2 (its parent is the other one)."""
        return self.hists[level % 2].data_ptr()

    def build_level_histograms(self, pr, level: int):
        ctx, st, prec = self.ctx, self.stream, self.precision
        if level > 0 and self.use_part and self.subtract:
            cb.cbh_part_build_histograms_sub(ctx, self.part, pr, level, prec,
                                             self.hist_ptr(level - 1), self.hist_ptr(level), st)
        elif level > 0 and self.use_part:
            cb.cbh_part_build_histograms(ctx, self.part, pr, level, prec, self.hist_ptr(level), st)
        elif level > 0 and self.subtract:
            cb.cbh_build_histograms_sub(ctx, pr, level, prec, self.hist_ptr(level - 1),
                                        self.split_ptr(level - 1), self.hist_ptr(level), st)
        else:
            cb.cbh_build_histograms(ctx, pr, level, prec, self.hist_ptr(level), st)

    def advance(self, pr, level: int):
        """Route the rows by the split of `level`: the leaf bit, or the move
        into leaf order (which writes the leaf indices at the last level)."""
        if self.use_part:
            cb.cbh_part_split(self.ctx, self.part, pr, level, self.precision,
                              self.split_ptr(level), self.stream)
        else:
            cb.cbh_apply_split(self.ctx, pr, level, self.split_ptr(level), self.stream)

    def fit_tree(self, t: int, counts: bool = False, events=None):
        """One tree (all levels, leaf solve, approx and gradient update) in one
        library call (cbh_fit_tree). `events`: optional list of (start, end)
        objects with a record(stream) method, recorded around each level's
        histogram build; then the levels are issued one call at a time."""
        pr = self.probs[t % self.s]
        if self.combinations:
            if events is not None:
                raise ValueError("combination trees take no events")
            self._combo_tree(t, counts)
            return
        if self.ordered:
            if events is not None or counts:
                raise ValueError("ordered trees take no events or counts")
            self._ordered_tree(t)
            return
        if events is None:
            cb.cbh_fit_tree(self.ctx, pr, self.part if self.use_part else None, self.precision,
                            self.subtract, self.hists, self.best, self.lr, self.l2,
                            self.leaf_values, self.leaf_counts if counts else None, None,
                            self.stream)
            return
        ctx, st, prec = self.ctx, self.stream, self.precision
        if prec == cb.CBH_PREC_INT16:
            cb.cbh_quantize_gradients(ctx, pr, st)
        # with subtraction in the original row order, each level's leaf bit is
        # set by the next level's build, in its row-code pass
        fuse = not self.use_part and self.subtract
        for lvl in range(self.depth):
            events[lvl][0].record(st)
            if fuse and lvl > 0:
                cb.cbh_apply_build_histograms_sub(ctx, pr, lvl, prec, self.hist_ptr(lvl - 1),
                                                  self.split_ptr(lvl - 1), self.hist_ptr(lvl), st)
            else:
                self.build_level_histograms(pr, lvl)
            events[lvl][1].record(st)
            cb.cbh_score_splits(ctx, pr, lvl, self.hist_ptr(lvl), prec, self.l2,
                                self.split_ptr(lvl), None, st)
            if not fuse or lvl == self.depth - 1:
                self.advance(pr, lvl)
        cb.cbh_update_approx(ctx, pr, self.hist_ptr(self.depth - 1), prec,
                             self.split_ptr(self.depth - 1), self.lr, self.l2, self.leaf_values,
                             self.leaf_counts if counts else None, st)

    def _capture(self, t: int, stamps=None):
        """A library-owned graph of tree t (cbh_graph_capture_tree), captured
        on a side stream of default priority."""
        if self.combinations:
            if stamps is not None:
                raise ValueError("combination trees take no stamps")
            # the level loop is driven from here: its library calls are
            # recorded between cbh_graph_begin and cbh_graph_end
            cap = torch.cuda.Stream(self.device)
            torch.cuda.synchronize(self.device)
            own = self.stream
            self.stream = cap
            try:
                cb.cbh_graph_begin(self.ctx, cap)
                try:
                    self._combo_tree(t)
                finally:
                    g = cb.cbh_graph_end(self.ctx, cap)
            finally:
                self.stream = own
            torch.cuda.synchronize(self.device)
            return g
        cap = torch.cuda.Stream(self.device)
        torch.cuda.synchronize(self.device)
        g = cb.cbh_graph_capture_tree(self.ctx, self.probs[t % self.s],
                                      self.part if self.use_part else None, self.precision,
                                      self.subtract, self.hists, self.best, self.lr, self.l2,
                                      self.leaf_values, None, stamps, cap)
        torch.cuda.synchronize(self.device)
        return g

    def capture_trees(self):
        """Capture one tree per permutation into library-owned HIP graphs; tree
        t replays graph t mod s on the booster's stream. Grow at least one tree
        of every permutation first: the library's workspace must have reached
        its size, since a call under capture never allocates (it fails with
        CBH_EBUSY instead); a later growth of the workspace keeps the buffer
        the graphs point at. A change of form drops the graphs."""
        self.drop_graphs()
        self.graphs = [self._capture(r) for r in range(self.s)]
        return self.graphs

    def capture_tree(self, t: int, stamps=None):
        """One graph of tree t (permutation t mod s); `stamps`: device uint64
        [2 depth] receiving the device clock before and after every build.
        The caller launches it (cb.cbh_graph_launch) and destroys it."""
        return self._capture(t, stamps)

    def drop_graphs(self):
        for g in self.graphs:
            cb.cbh_graph_destroy(g)
        self.graphs = []

    def replay_tree(self, t: int):
        cb.cbh_graph_launch(self.graphs[t % self.s], self.stream)

    def tree_record(self) -> TreeRecord:
        b = self.best.cpu().numpy()
        return TreeRecord(b[:, :2].copy(), b[:, 2:].view(np.float32).copy(),
                          self.leaf_values.cpu().numpy())

    def fit(self, iterations: int, record: bool = True):
        self.init_gradients()
        trees = []
        for t in range(iterations):
            self.fit_tree(t)
            if record:
                trees.append(self.tree_record())
        return trees

    def predict(self, trees, approx=None) -> torch.Tensor:
        """Apply recorded trees (`tree_record`, in fit order) to this booster's
        rows with cbh_apply_model: approx [K][n] float64 on the device (zeros
        when not given) gains lr * the tree's leaf value, tree after tree,
        each tree reading the feature table of its own permutation. Applied
        to the trees of `fit`, this gives the training approx bit for bit."""
        d = self.device
        if self.combinations:
            raise ValueError("predict takes trees without combination columns")
        if approx is None:
            approx = torch.zeros((self.K, self.n), dtype=torch.float64, device=d)
        for t, tr in enumerate(trees):
            r = t % self.s
            feat = tr.splits[:, 0].astype(np.int32).copy()
            border = tr.splits[:, 1].astype(np.int32).copy()
            none = (feat < 0) | (feat >= self.F)       # a level without a split sets no bit
            feat[none], border[none] = 0, 255
            df = torch.from_numpy(feat).to(d)
            db = torch.from_numpy(border).to(d)
            dv = torch.from_numpy(np.ascontiguousarray(tr.values, np.float64)).to(d)
            seg = self.seg_table[r] if self.seg_table is not None else None
            cb.cbh_apply_model(self.ctx, self.col_table[r], seg, self.n, self.F, self.K, 1,
                               self.depth, df, db, dv, self.lr, approx, self.stream)
        return approx

    def model_state(self, r: int, weight=None) -> "ModelState":
        """A further model over permutation r's bins (see ModelState);
        `weight`: optional float32 [n] row weights (a cross-validation fold:
        0 on its held-out rows)."""
        return ModelState(self, r, weight)

    def close(self):
        if self.graphs:
            torch.cuda.synchronize(self.device)
            self.drop_graphs()
        if self.part is not None:
            torch.cuda.synchronize(self.device)
            cb.cbh_part_destroy(self.part)
            self.part = None
        if self.own_ctx and self.ctx:
            torch.cuda.synchronize(self.device)
            cb.cbh_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ModelState:
    """The per-model device state (gradients, int16 codes, leaf indices,
    approx, last-level histogram, leaf values) of one more model over the bins
    of a prepared booster's permutation r; bins, bin counts and labels stay
    shared with the booster. Ordered boosting keeps one model per permutation
    (Sec. 3); several such models run side by side through the batched calls
    (cbh_batch_create with `prob`, `hist` and `leaf_values` of each)."""

    def __init__(self, base: GpuBooster, r: int, weight=None):
        if not hasattr(base, "probs"):
            raise RuntimeError("prepare() the booster first")
        d, n, K = base.device, base.n, base.K
        self.base, self.r = base, int(r)
        self.weight = None
        if weight is not None:
            self.weight = torch.as_tensor(np.ascontiguousarray(weight, np.float32)).to(d)
            assert self.weight.numel() == n
        self.g = torch.empty((K, n), dtype=torch.float32, device=d)
        self.h = torch.empty((K, n), dtype=torch.float32, device=d)
        self.gq = torch.empty((K, n, 2), dtype=torch.int16, device=d)
        self.grad_scale = torch.zeros((K, 2), dtype=torch.float32, device=d)
        self.leaf = torch.zeros(n, dtype=torch.uint16, device=d)
        self.approx = torch.zeros((K, n), dtype=torch.float64, device=d)
        self.leaf_values = torch.zeros((1 << base.depth, K), dtype=torch.float64, device=d)
        self.hist = torch.empty(max(256, base._hist_bytes(base.depth - 1)), dtype=torch.uint8,
                                device=d)
        p = base.problem(self.r)
        p.g = self.g.data_ptr()
        p.h = self.h.data_ptr()
        p.gq = self.gq.data_ptr()
        p.grad_scale = self.grad_scale.data_ptr()
        p.leaf = self.leaf.data_ptr()
        p.approx = self.approx.data_ptr()
        p.weight = self.weight.data_ptr() if self.weight is not None else None
        self.prob = p
