/*
 * CPU reference ("oracle") for the per-level split search of oblivious
 * gradient-boosted trees and for ordered target statistics, following
 * "CatBoost: gradient boosting with categorical features support"
 * (Dorogush, Ershov, Gulin, arXiv:1810.11363).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it. It shares no code, header, table or helper with the
 * GPU library.
 *
 * Every routine is the plain definition written out as loops, in double
 * precision unless a step is an integer decision taken in the GPU kernel's
 * own precision (int16 gradient codes, stated where it happens). Results do
 * not depend on the number of OpenMP threads: parallel loops split work over
 * features, and each feature is summed sequentially in row order.
 *
 * Parity of the assembled tree is pinned only through the pieces below; the
 * paper prints no tree, score or statistic for any input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_RMSE 0
#define ORC_LOGLOSS 1
#define ORC_MULTICLASS 2

/* ------------------------------------------------------------------------ */
/* Borders and bins (Sec. 5, "Dense numerical features": discretization into
 * a fixed number of bins, at most 255 per feature). The paper does not give
 * the border rule. Reading used here: value-at-rank quantiles. Sort the
 * column; if it has m <= max_bins distinct values the borders are the m-1
 * smallest distinct values; otherwise border j (j = 1..max_bins-1) is the
 * sorted value at rank floor(j*n/max_bins)-1, skipping a candidate equal to
 * the previously kept border or to the column maximum. Borders are data
 * values, so there is no rounding anywhere in the rule.                     */

static int cmp_float(const void* a, const void* b) {
    float x = *(const float*)a, y = *(const float*)b;
    return (x > y) - (x < y);
}

int orc_select_borders(const float* x, int64_t n, int32_t max_bins,
                       float* borders, int32_t* n_borders) {
    *n_borders = 0;
    if (max_bins < 2 || max_bins > 256) return -1;
    if (n <= 0) return 0;
    float* s = (float*)malloc(sizeof(float) * (size_t)n);
    if (!s) return -2;
    for (int64_t i = 0; i < n; ++i) {
        if (isnan(x[i])) { free(s); return -1; }
        s[i] = x[i];
    }
    qsort(s, (size_t)n, sizeof(float), cmp_float);
    int64_t m = 1;
    for (int64_t i = 1; i < n; ++i) if (s[i] != s[i - 1]) ++m;
    int32_t nb = 0;
    if (m <= max_bins) {
        /* one bin per distinct value: every distinct value but the largest */
        for (int64_t i = 0; i < n; ++i) {
            if (s[i] == s[n - 1]) break;
            if (i == 0 || s[i] != s[i - 1]) borders[nb++] = s[i];
        }
    } else {
        for (int64_t j = 1; j < max_bins; ++j) {
            int64_t rank = (j * n) / max_bins - 1;
            float c = s[rank];
            if (c == s[n - 1]) continue;
            if (nb > 0 && c == borders[nb - 1]) continue;
            borders[nb++] = c;
        }
    }
    *n_borders = nb;
    free(s);
    return 0;
}

/* bin(x) = number of borders strictly below x; with increasing borders this
 * is the position of the first border that is not below x.                  */
void orc_quantize(const float* x, int64_t n, const float* borders, int32_t nb,
                  uint8_t* bins) {
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = 0;
        while (c < nb && x[i] > borders[c]) ++c;
        bins[i] = (uint8_t)c;
    }
}

/* ------------------------------------------------------------------------ */
/* Ordered target statistic, Sec. 2, Eq. (1). For the row sigma_p placed at
 * position p of the permutation, over the rows placed strictly earlier that
 * share its category:
 *     num = sum of their targets,  den = their count,
 *     TS  = (num + a*P) / (den + a).
 * Targets are int64 numerators y_num with value y_num * 2^-y_shift (0/1 for
 * classification, a fixed-point label for regression) so that num is exact.
 * The TS value is evaluated as (ldexp(num, -y_shift) + a*P) / (den + a) in
 * that operation order. Category values are arbitrary int32; a dense id is
 * found by binary search in the sorted distinct values (a perfect hash,
 * Sec. 5 "Categorical features").                                           */

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

static int64_t dense_id(const int32_t* uniq, int64_t m, int32_t v) {
    int64_t lo = 0, hi = m - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (uniq[mid] == v) return mid;
        if (uniq[mid] < v) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Uniform statistic borders t_j = lo + (hi-lo)*j/B, j = 1..B-1. The paper
 * states that statistics are binarized like float features (Sec. 4) but not
 * how; this uniform rule is the reading used throughout.                    */
void orc_ts_borders(double lo, double hi, int32_t n_bins, double* out) {
    for (int32_t j = 1; j < n_bins; ++j)
        out[j - 1] = lo + ((hi - lo) * (double)j) / (double)n_bins;
}

int orc_ordered_ts(const int32_t* cat, const int32_t* perm, const int64_t* y_num,
                   int64_t n, int32_t y_shift, double a, double prior,
                   const double* ts_borders, int32_t n_ts_borders,
                   int64_t* num, int32_t* den, double* ts, uint8_t* ts_bin) {
    if (n <= 0) return 0;
    int32_t* uniq = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!uniq) return -2;
    memcpy(uniq, cat, sizeof(int32_t) * (size_t)n);
    qsort(uniq, (size_t)n, sizeof(int32_t), cmp_i32);
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (i == 0 || uniq[i] != uniq[m - 1]) uniq[m++] = uniq[i];
    int64_t* sum = (int64_t*)calloc((size_t)m, sizeof(int64_t));
    int64_t* cnt = (int64_t*)calloc((size_t)m, sizeof(int64_t));
    if (!sum || !cnt) { free(uniq); free(sum); free(cnt); return -2; }
    for (int64_t p = 0; p < n; ++p) {
        int64_t r = perm[p];
        int64_t c = dense_id(uniq, m, cat[r]);
        num[r] = sum[c];
        den[r] = (int32_t)cnt[c];
        sum[c] += y_num[r];
        cnt[c] += 1;
    }
    for (int64_t r = 0; r < n; ++r) {
        double v = (ldexp((double)num[r], -y_shift) + a * prior) / ((double)den[r] + a);
        if (ts) ts[r] = v;
        if (ts_bin) {
            int32_t b = 0;
            while (b < n_ts_borders && v > ts_borders[b]) ++b;
            ts_bin[r] = (uint8_t)b;
        }
    }
    free(uniq); free(sum); free(cnt);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Loss derivatives. Algorithm 1 (Sec. 3) uses g = d Loss(y, a) / d a at the
 * current model value a; the paper does not write the losses out. Readings:
 *   RMSE       Loss = (y - a)^2 / 2        g = a - y,        h = 1
 *   Logloss    Loss = -y log p - (1-y) log(1-p), p = 1/(1+e^-a)
 *                                          g = p - y,        h = p (1 - p)
 *   MultiClass Loss = -log p_y, p = softmax(a) (max subtracted first)
 *                                          g_k = p_k - [y=k], h_k = p_k (1-p_k)
 * h is the second derivative (diagonal for MultiClass), used for Newton
 * steps (Sec. 3 mentions gradient or Newton leaf estimates).
 * approx, g, h are [K][n].                                                  */
void orc_gradients(int32_t loss, int32_t K, int64_t n, const double* approx,
                   const float* label, double* g, double* h) {
    for (int64_t i = 0; i < n; ++i) {
        double y = (double)label[i];
        if (loss == ORC_RMSE) {
            g[i] = approx[i] - y;
            h[i] = 1.0;
        } else if (loss == ORC_LOGLOSS) {
            double p = 1.0 / (1.0 + exp(-approx[i]));
            g[i] = p - y;
            h[i] = p * (1.0 - p);
        } else {
            double mx = approx[i];
            for (int32_t k = 1; k < K; ++k)
                if (approx[(int64_t)k * n + i] > mx) mx = approx[(int64_t)k * n + i];
            double z = 0.0;
            for (int32_t k = 0; k < K; ++k) z += exp(approx[(int64_t)k * n + i] - mx);
            for (int32_t k = 0; k < K; ++k) {
                double p = exp(approx[(int64_t)k * n + i] - mx) / z;
                double t = ((int32_t)y == k) ? 1.0 : 0.0;
                g[(int64_t)k * n + i] = p - t;
                h[(int64_t)k * n + i] = p * (1.0 - p);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Histograms (Sec. 5): hist[j][b] = sum of g[i] over rows whose feature j
 * falls in bin b, here additionally per current leaf and with a second
 * statistic (h, which is 1 per row for RMSE and hence the row count).
 * bins is [F][n]; g, h are [K][n]; hist is [L][F][B][2K] with stat
 * 2c = sum g_c and 2c+1 = sum h_c.                                          */
void orc_histogram(int64_t n, int32_t F, const uint8_t* bins, int32_t B,
                   int32_t K, const double* g, const double* h,
                   const uint16_t* leaf, int32_t L, double* hist) {
    int64_t S = 2 * (int64_t)K;
    memset(hist, 0, sizeof(double) * (size_t)((int64_t)L * F * B * S));
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t f = 0; f < F; ++f) {
        const uint8_t* col = bins + (int64_t)f * n;
        for (int64_t i = 0; i < n; ++i) {
            int64_t base = (((int64_t)leaf[i] * F + f) * B + col[i]) * S;
            for (int32_t c = 0; c < K; ++c) {
                hist[base + 2 * c] += g[(int64_t)c * n + i];
                hist[base + 2 * c + 1] += h[(int64_t)c * n + i];
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Split score. The paper says phase one scores candidate trees and keeps the
 * best split (Sec. 3) without giving the formula. Reading: the L2-regularised
 * second-order objective. For one leaf with sums G, H and regulariser l2 the
 * minimum of sum_i (g_i v + h_i v^2 / 2) + l2 v^2 / 2 is -G^2 / (2 (H + l2))
 * at v = -G / (H + l2). Splitting every current leaf by (f, k) (oblivious
 * tree, Sec. 4) and dropping the constant factor and the parent term gives
 *     S(f, k) = sum_L sum_c [ G_left^2/(H_left+l2) + G_right^2/(H_right+l2) ]
 * with left = bins <= k, right = bins > k; a side whose H + l2 is 0
 * contributes 0. Candidates are k = 0 .. n_bins[f]-2; other entries of
 * scores [F][B-1] are -INFINITY.                                            */
static double side_term(double G, double H, double l2) {
    double d = H + l2;
    return d == 0.0 ? 0.0 : (G * G) / d;
}

void orc_score(int32_t L, int32_t F, int32_t B, int32_t K, const double* hist,
               const int32_t* n_bins, double l2, double* scores) {
    int64_t S = 2 * (int64_t)K;
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t f = 0; f < F; ++f) {
        double* pre = (double*)malloc(sizeof(double) * (size_t)(2 * (B + 1)));
        double* suf = (double*)malloc(sizeof(double) * (size_t)(2 * (B + 1)));
        double* sc = scores + (int64_t)f * (B - 1);
        for (int32_t k = 0; k < B - 1; ++k) sc[k] = -INFINITY;
        for (int32_t k = 0; k + 1 < n_bins[f]; ++k) sc[k] = 0.0;
        for (int32_t l = 0; l < L; ++l) {
            for (int32_t c = 0; c < K; ++c) {
                const double* hb = hist + (((int64_t)l * F + f) * B) * S + 2 * c;
                /* pre[b] = sums over bins < b; suf[b] = sums over bins >= b */
                pre[0] = 0.0; pre[1] = 0.0;
                for (int32_t b = 0; b < B; ++b) {
                    pre[2 * (b + 1)] = pre[2 * b] + hb[b * S];
                    pre[2 * (b + 1) + 1] = pre[2 * b + 1] + hb[b * S + 1];
                }
                suf[2 * B] = 0.0; suf[2 * B + 1] = 0.0;
                for (int32_t b = B - 1; b >= 0; --b) {
                    suf[2 * b] = suf[2 * (b + 1)] + hb[b * S];
                    suf[2 * b + 1] = suf[2 * (b + 1) + 1] + hb[b * S + 1];
                }
                for (int32_t k = 0; k + 1 < n_bins[f]; ++k) {
                    sc[k] += side_term(pre[2 * (k + 1)], pre[2 * (k + 1) + 1], l2)
                           + side_term(suf[2 * (k + 1)], suf[2 * (k + 1) + 1], l2);
                }
            }
        }
        free(pre); free(suf);
    }
}

/* Best split: the largest score; among exactly equal scores the smallest
 * feature, then the smallest border. Also returns the second-best score over
 * the other candidates. If no candidate exists, feature = border = -1.      */
void orc_best_split(int32_t F, int32_t B, const double* scores,
                    const int32_t* n_bins, int32_t* best_f, int32_t* best_k,
                    double* best_s, double* second_s) {
    int32_t bf = -1, bk = -1;
    double s1 = -INFINITY, s2 = -INFINITY;
    for (int32_t f = 0; f < F; ++f) {
        for (int32_t k = 0; k + 1 < n_bins[f]; ++k) {
            double v = scores[(int64_t)f * (B - 1) + k];
            if (bf < 0 || v > s1) {
                if (bf >= 0) s2 = s1 > s2 ? s1 : s2;
                s1 = v; bf = f; bk = k;
            } else if (v > s2) {
                s2 = v;
            }
        }
    }
    *best_f = bf; *best_k = bk; *best_s = s1; *second_s = s2;
}

/* Leaf index of an oblivious tree (Sec. 4): the split chosen at depth i sets
 * bit i, so after level `level` the leaf is sum_i 2^i * [bin_{f_i} > k_i].  */
void orc_apply_split(int64_t n, const uint8_t* bin_col, int32_t k, int32_t level,
                     uint16_t* leaf) {
    for (int64_t i = 0; i < n; ++i)
        if ((int32_t)bin_col[i] > k) leaf[i] = (uint16_t)(leaf[i] | (1u << level));
}

/* Leaf values (phase two, Sec. 3): per leaf and class, sums taken directly
 * over the leaf's rows, then the Newton step v = -G / (H + l2).
 * G, H, values are [n_leaves][K]; counts is [n_leaves].                    */
void orc_leaf_values(int64_t n, int32_t K, int32_t n_leaves, const uint16_t* leaf,
                     const double* g, const double* h, double l2, double* G,
                     double* H, int64_t* counts, double* values) {
    memset(G, 0, sizeof(double) * (size_t)n_leaves * K);
    memset(H, 0, sizeof(double) * (size_t)n_leaves * K);
    memset(counts, 0, sizeof(int64_t) * (size_t)n_leaves);
    for (int64_t i = 0; i < n; ++i) {
        counts[leaf[i]] += 1;
        for (int32_t c = 0; c < K; ++c) {
            G[(int64_t)leaf[i] * K + c] += g[(int64_t)c * n + i];
            H[(int64_t)leaf[i] * K + c] += h[(int64_t)c * n + i];
        }
    }
    for (int64_t j = 0; j < (int64_t)n_leaves * K; ++j) {
        double d = H[j] + l2;
        values[j] = d == 0.0 ? 0.0 : -G[j] / d;
    }
}

/* Model update M <- M + lr * tree (Algorithm 1 adds each new tree to the
 * model): approx[c][i] += lr * values[leaf[i]][c].                          */
void orc_update_approx(int64_t n, int32_t K, const uint16_t* leaf,
                       const double* values, double lr, double* approx) {
    for (int64_t i = 0; i < n; ++i)
        for (int32_t c = 0; c < K; ++c)
            approx[(int64_t)c * n + i] += lr * values[(int64_t)leaf[i] * K + c];
}

/* ------------------------------------------------------------------------ */
/* Packed bins (Sec. 5 keeps features of at most 15 bins in 4 bits and
 * binary features in 1 bit). The paper fixes the widths, not a byte layout;
 * the layout here is the GPU library's documented one, written out byte by
 * byte: rows are taken in segments of 16, a segment is 2 * bits bytes;
 * 4 bits: row r of a segment (k = r / 8, q = r % 8) is nibble q / 4 (0 low,
 * 1 high) of byte 4k + q % 4; 1 bit: row r is bit r % 8 of byte r / 8.
 * Rows past n are 0; values are masked to the width. out has
 * ceil(n/16) * 2 * bits bytes.                                              */
void orc_pack_bins(const uint8_t* bins, int64_t n, int32_t bits, uint8_t* out) {
    int64_t nseg = (n + 15) / 16;
    memset(out, 0, (size_t)(nseg * 2 * bits));
    for (int64_t i = 0; i < n; ++i) {
        int64_t seg = i / 16;
        int r = (int)(i % 16);
        unsigned v = bins[i] & ((1u << bits) - 1u);
        if (bits == 4) {
            int k = r / 8, q = r % 8;
            out[seg * 8 + 4 * k + q % 4] |= (uint8_t)(v << (4 * (q / 4)));
        } else {
            out[seg * 2 + r / 8] |= (uint8_t)(v << (r % 8));
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Ordered boosting's supporting approximations (Sec. 3). Algorithm 1 keeps,
 * for one permutation, a model per position that never learns from that
 * position; the O(s n) relaxation keeps about log2(n) of them instead: model
 * i learns from the first 2^i positions, is maintained for the first
 * 2^(i+1), and a position's gradient for choosing the next tree structure is
 * taken at the model indexed by the floor of log2 of the position. All
 * models share the tree structures (the leaf of every row comes from the
 * tree built on those gradients); each model takes its own leaf values.
 * Reading, with 0-based positions p = 0..n-1 (perm[p] = row at position p):
 *   model m = 0..M-1 learns from the positions below T_m (T_0 = 0,
 *   T_m = 2^(m-1)) and is kept for the positions below min(n, 2^m);
 *   position p reads model m(p) = 0 for p = 0 and floor(log2 p) + 1
 *   otherwise, so T_m(p) <= p: the model a position reads never saw it;
 *   M = 1 for n = 1, else floor(log2(n-1)) + 2 (the model position n-1 reads
 *   is the last one).
 * Model m's leaf values are the Newton steps -G/(H+l2) of its own gradients
 * summed over its learning positions per leaf; every kept position then
 * gains lr * value of its leaf. support is [K][S] with model m at offset
 * off_m = sum over m' < m of min(n, 2^m'), in position order; S = off_M,
 * which is below 4n.                                                        */
int32_t orc_ordered_models(int64_t n) {
    if (n <= 1) return 1;
    int32_t fl = 0;
    while (((int64_t)1 << (fl + 1)) <= n - 1) ++fl;   /* floor(log2(n-1)) */
    return fl + 2;
}

static int64_t ord_keep(int64_t n, int32_t m) {
    int64_t c = (int64_t)1 << m;
    return c < n ? c : n;
}

static int64_t ord_learn(int32_t m) { return m == 0 ? 0 : (int64_t)1 << (m - 1); }

int64_t orc_ordered_offset(int64_t n, int32_t m) {
    int64_t off = 0;
    for (int32_t j = 0; j < m; ++j) off += ord_keep(n, j);
    return off;
}

static int32_t ord_model_of(int64_t p) {
    if (p == 0) return 0;
    int32_t fl = 0;
    while (((int64_t)1 << (fl + 1)) <= p) ++fl;          /* floor(log2 p) */
    return fl + 1;
}

/* Gradients for choosing the next tree: row perm[p] gets the loss
 * derivatives at model m(p)'s value for position p. g, h are [K][n] in
 * dataset (row) order.                                                      */
void orc_ordered_gradients(int32_t loss, int32_t K, int64_t n, const int32_t* perm,
                           const float* label, const double* support, double* g,
                           double* h) {
    int64_t S = orc_ordered_offset(n, orc_ordered_models(n));
    double* a = (double*)malloc(sizeof(double) * (size_t)K * n);
    for (int64_t p = 0; p < n; ++p) {
        int64_t e = orc_ordered_offset(n, ord_model_of(p)) + p;
        for (int32_t c = 0; c < K; ++c)
            a[(int64_t)c * n + perm[p]] = support[(int64_t)c * S + e];
    }
    orc_gradients(loss, K, n, a, label, g, h);
    free(a);
}

/* After a tree's structure is fixed (leaf in row order): every model takes
 * its leaf values from its learning positions and adds them to its kept
 * positions. values_out (nullable) is [M][n_leaves][K].                     */
void orc_ordered_update(int32_t loss, int32_t K, int64_t n, const int32_t* perm,
                        const float* label, const uint16_t* leaf, int32_t n_leaves,
                        double lr, double l2, double* support, double* values_out) {
    int32_t M = orc_ordered_models(n);
    int64_t S = orc_ordered_offset(n, M);
    double* a = (double*)malloc(sizeof(double) * (size_t)K * n);
    float* y = (float*)malloc(sizeof(float) * (size_t)n);
    uint16_t* lf = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)n);
    double* g = (double*)malloc(sizeof(double) * (size_t)K * n);
    double* h = (double*)malloc(sizeof(double) * (size_t)K * n);
    double* G = (double*)malloc(sizeof(double) * (size_t)n_leaves * K);
    double* H = (double*)malloc(sizeof(double) * (size_t)n_leaves * K);
    double* v = (double*)malloc(sizeof(double) * (size_t)n_leaves * K);
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_leaves);
    for (int32_t m = 0; m < M; ++m) {
        int64_t off = orc_ordered_offset(n, m), t = ord_learn(m), keep = ord_keep(n, m);
        /* the model's learning positions as a small dataset of their own */
        for (int64_t j = 0; j < t; ++j) {
            y[j] = label[perm[j]];
            lf[j] = leaf[perm[j]];
            for (int32_t c = 0; c < K; ++c)
                a[(int64_t)c * t + j] = support[(int64_t)c * S + off + j];
        }
        if (t > 0) {
            orc_gradients(loss, K, t, a, y, g, h);
            orc_leaf_values(t, K, n_leaves, lf, g, h, l2, G, H, cnt, v);
        } else {
            for (int64_t j = 0; j < (int64_t)n_leaves * K; ++j) v[j] = 0.0;
        }
        for (int64_t j = 0; j < keep; ++j)
            for (int32_t c = 0; c < K; ++c)
                support[(int64_t)c * S + off + j] += lr * v[(int64_t)leaf[perm[j]] * K + c];
        if (values_out)
            memcpy(values_out + (int64_t)m * n_leaves * K, v,
                   sizeof(double) * (size_t)n_leaves * K);
    }
    free(a); free(y); free(lf); free(g); free(h); free(G); free(H); free(v); free(cnt);
}

/* Model apply, the scorer of Sec. 4: for tree t of depth d the leaf of a row
 * is the binary vector sum_i 2^i * B(x, f(t, i)), where the binary feature
 * of level i is [bin_{feat[t][i]} > border[t][i]]; the row's approx gains
 * lr * values[t][leaf][c] for every class c, tree after tree in model
 * order, exactly as a sequence of model updates would add them.
 * bins is column-major [F][n]; values is [T][2^d][K]; approx is [K][n].     */
void orc_apply_model(int64_t n, int32_t F, const uint8_t* bins, int32_t T, int32_t d,
                     int32_t K, const int32_t* feat, const int32_t* border,
                     const double* values, double lr, double* approx) {
    (void)F;
    const int64_t n_leaves = (int64_t)1 << d;
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t t = 0; t < T; ++t) {
            int64_t leaf = 0;
            for (int32_t l = 0; l < d; ++l) {
                const int32_t f = feat[(int64_t)t * d + l];
                const int32_t b = bins[(int64_t)f * n + i];
                if (b > border[(int64_t)t * d + l]) leaf |= (int64_t)1 << l;
            }
            for (int32_t c = 0; c < K; ++c)
                approx[(int64_t)c * n + i] +=
                    lr * values[((int64_t)t * n_leaves + leaf) * K + c];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* int16 gradient codes. Not in the paper: a per-tree scale s = max|g| / 32767
 * (and s_h = max h / 32767), code = round-half-even(g / s). This turns a
 * real value into an integer, so the decision is taken in the GPU kernel's
 * precision: float32 division and float32 rounding. Codes of a zero scale
 * are 0. g and h are the float32 gradients; codes are [K][n].               */
void orc_grad_codes(int64_t n, int32_t K, const float* g, const float* h,
                    int32_t with_h, int16_t* gq, int16_t* hq, float* scales) {
    for (int32_t c = 0; c < K; ++c) {
        const float* gc = g + (int64_t)c * n;
        const float* hc = h + (int64_t)c * n;
        float mg = 0.0f, mh = 0.0f;
        for (int64_t i = 0; i < n; ++i) {
            float a = fabsf(gc[i]);
            if (a > mg) mg = a;
            if (with_h && hc[i] > mh) mh = hc[i];
        }
        volatile float sg = mg / 32767.0f;
        volatile float sh = with_h ? mh / 32767.0f : 1.0f;
        scales[2 * c] = sg;
        scales[2 * c + 1] = sh;
        for (int64_t i = 0; i < n; ++i) {
            float q = (sg > 0.0f) ? rintf(gc[i] / sg) : 0.0f;
            gq[(int64_t)c * n + i] = (int16_t)q;
            float r = with_h ? ((sh > 0.0f) ? rintf(hc[i] / sh) : 0.0f) : 1.0f;
            hq[(int64_t)c * n + i] = (int16_t)r;
        }
    }
}

/* Exact integer histogram of the int16 codes: [L][F][B][2K] int64.          */
void orc_histogram_int(int64_t n, int32_t F, const uint8_t* bins, int32_t B,
                       int32_t K, const int16_t* gq, const int16_t* hq,
                       const uint16_t* leaf, int32_t L, int64_t* hist) {
    int64_t S = 2 * (int64_t)K;
    memset(hist, 0, sizeof(int64_t) * (size_t)((int64_t)L * F * B * S));
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t f = 0; f < F; ++f) {
        const uint8_t* col = bins + (int64_t)f * n;
        for (int64_t i = 0; i < n; ++i) {
            int64_t base = (((int64_t)leaf[i] * F + f) * B + col[i]) * S;
            for (int32_t c = 0; c < K; ++c) {
                hist[base + 2 * c] += gq[(int64_t)c * n + i];
                hist[base + 2 * c + 1] += hq[(int64_t)c * n + i];
            }
        }
    }
}

int orc_num_threads(void) {
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the parallel loops from now on (timing the oracle at a chosen
 * core count; results do not depend on it). */
void orc_set_threads(int32_t t) {
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(t > 0 ? t : 1);
#else
    (void)t;
#endif
}
