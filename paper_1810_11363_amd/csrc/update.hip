// Leaf bits, leaf values and the model/gradient update.
//
// apply_split: the split of depth `level` sets bit `level` of the leaf index
// (Sec. 4: leaf = sum_i 2^i B(x, f(t, i))); at level 0 the leaf is
// overwritten, so a tree never needs a separate reset of the leaf array.
// leaf_solve: final-leaf sums taken from the last level's histogram row of the
// chosen feature (left of the border -> bit clear, right -> bit set), summed in
// double, and the Newton value -G / (H + l2) (Sec. 3: second phase is the
// ordinary boosting step; Newton or gradient leaf estimates).
// update: approx += lr * v[leaf] in double (Algorithm 1 adds each tree to the
// model), then g = dLoss/da and h = d2Loss/da2 at the new approx in double,
// stored as float.
// apply_model: the scorer of Sec. 4 over a whole model, from the bins.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "kernels_dev.h"
#include "update_dev.h"

namespace cbh {

template <int BITS>
__global__ __launch_bounds__(256) void apply_split_kernel(const uint8_t* const* __restrict__ bins,
                                                          const int64_t* __restrict__ seg,
                                                          int32_t F, const cbh_split* __restrict__ best,
                                                          uint16_t* __restrict__ leaf, int64_t n,
                                                          int32_t level) {
    int f = best->feature;
    int k = best->border;
    if (f < 0 || f >= F) {
        // no split: every row stays on the clear side of this level's bit
        if (level != 0) return;
        f = 0;
        k = 255;
    }
    const uint8_t* __restrict__ col = bins[f];
    // bytes between 16-row segments (packed bins: plain columns)
    const int64_t sstride = seg ? seg[f] : seg_bytes<BITS>();
    const uint32_t bit = 1u << level;
    const int64_t n8 = n / 8;
    const bool vec = ((reinterpret_cast<uintptr_t>(col) & (BITS == 8 ? 7 : 3)) == 0);
    const int64_t tid = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t stride = int64_t(gridDim.x) * 256;
    if (vec) {
        for (int64_t q = tid; q < n8; q += stride) {
            // rows 8q .. 8q+7 lie in one 16-row segment: half of it
            const uint8_t* half = col + (q >> 1) * sstride;
            uint32_t bv[8];
            if constexpr (BITS == 8) {
                const uint2 b = *reinterpret_cast<const uint2*>(half + 8 * (q & 1));
#pragma unroll
                for (int r = 0; r < 8; ++r) bv[r] = ((r < 4 ? b.x : b.y) >> (8 * (r & 3))) & 255u;
            } else if constexpr (BITS == 4) {
                const uint32_t w = *reinterpret_cast<const uint32_t*>(half + 4 * (q & 1));
#pragma unroll
                for (int r = 0; r < 8; ++r) bv[r] = (w >> (8 * (r & 3) + 4 * (r >> 2))) & 15u;
            } else {
                const uint32_t b = half[q & 1];
#pragma unroll
                for (int r = 0; r < 8; ++r) bv[r] = (b >> r) & 1u;
            }
            uint4 l = level == 0 ? make_uint4(0u, 0u, 0u, 0u)
                                 : reinterpret_cast<const uint4*>(leaf)[q];
            uint32_t lw[4] = {l.x, l.y, l.z, l.w};
#pragma unroll
            for (int r = 0; r < 8; ++r)
                if ((int)bv[r] > k) lw[r >> 1] |= bit << (16 * (r & 1));
            reinterpret_cast<uint4*>(leaf)[q] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
        }
        for (int64_t i = n8 * 8 + tid; i < n; i += stride) {
            const uint32_t old = level == 0 ? 0u : leaf[i];
            const uint32_t bv = seg_bin<BITS>(col + (i >> 4) * sstride, (int)(i & 15));
            leaf[i] = (uint16_t)(old | (((int)bv > k) ? bit : 0u));
        }
    } else {
        for (int64_t i = tid; i < n; i += stride) {
            const uint32_t old = level == 0 ? 0u : leaf[i];
            const uint32_t bv = seg_bin<BITS>(col + (i >> 4) * sstride, (int)(i & 15));
            leaf[i] = (uint16_t)(old | (((int)bv > k) ? bit : 0u));
        }
    }
}

// Packed bins from byte bins (cbh_pack_bins): one thread per (feature,
// 16-row segment); rows past n pack as 0.
template <int BITS>
__global__ __launch_bounds__(256) void pack_bins_kernel(const uint8_t* const* __restrict__ bins,
                                                        const int64_t* __restrict__ seg,
                                                        uint8_t* const* __restrict__ out,
                                                        int32_t F, int64_t n, int64_t n_seg,
                                                        uint32_t* __restrict__ flags) {
    const int64_t total = n_seg * F;
    for (int64_t t = int64_t(blockIdx.x) * 256 + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * 256) {
        const int f = (int)(t / n_seg);
        const int64_t sg = t - int64_t(f) * n_seg;
        const uint8_t* src = bins[f] + sg * seg_stride_of(seg, f);
        const int rows = (int)min<int64_t>(16, n - sg * 16);
        uint32_t v[16];
        bool over = false;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            v[r] = r < rows ? (uint32_t)src[r] : 0u;
            over |= v[r] >= (1u << BITS);
            v[r] &= (1u << BITS) - 1u;
        }
        if (over) atomicOr(flags, FLAG_PACK_RANGE);
        // byte stores: the output columns need no alignment
        uint8_t* dst = out[f] + sg * seg_bytes<BITS>();
        if constexpr (BITS == 4) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    dst[4 * k + j] = (uint8_t)(v[8 * k + j] | (v[8 * k + 4 + j] << 4));
        } else {
            uint32_t b = 0u;
#pragma unroll
            for (int r = 0; r < 16; ++r) b |= v[r] << r;
            dst[0] = (uint8_t)b;
            dst[1] = (uint8_t)(b >> 8);
        }
    }
}

// One wave per (final leaf, class).
__global__ __launch_bounds__(256) void leaf_solve_kernel(SolveArgs a) {
    const int64_t t = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (t >= (int64_t(1) << a.depth) * a.K) return;
    leaf_solve_one(a, t, threadIdx.x & 63);
}

template <int LOSS>
__global__ __launch_bounds__(256) void update_kernel(UpdArgs a) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < a.n;
         i += int64_t(gridDim.x) * 256)
        update_row<LOSS>(a, i);
}

__global__ void zero_i64_kernel(int64_t* p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0;
}

// Rows per final leaf: LDS counters per block, one global add per leaf.
__global__ __launch_bounds__(256) void leaf_count_kernel(const uint16_t* __restrict__ leaf,
                                                         int64_t n, int32_t leaves,
                                                         unsigned long long* __restrict__ out) {
    extern __shared__ uint32_t cnt[];
    for (int i = threadIdx.x; i < leaves; i += 256) cnt[i] = 0u;
    __syncthreads();
    const uint32_t m = (uint32_t)leaves - 1u;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256)
        atomicAdd(&cnt[leaf[i] & m], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i < leaves; i += 256)
        if (cnt[i]) atomicAdd(&out[i], (unsigned long long)cnt[i]);
}

static int grid_rows(const cbh_ctx* ctx, int64_t n, int per_thread = 1) {
    int64_t g = (n + 256LL * per_thread - 1) / (256LL * per_thread);
    if (g < 1) g = 1;
    const int64_t cap = int64_t(ctx->num_cus) * 8;
    return (int)(g < cap ? g : cap);
}

int launch_apply(const cbh_ctx* ctx, const cbh_problem* p, int32_t level, const cbh_split* best,
                 hipStream_t s) {
    const unsigned g = grid_rows(ctx, p->n, 8);
    if (p->bin_bits == 4)
        apply_split_kernel<4><<<g, 256, 0, s>>>(p->bins, p->seg_stride, p->n_features, best,
                                                p->leaf, p->n, level);
    else if (p->bin_bits == 1)
        apply_split_kernel<1><<<g, 256, 0, s>>>(p->bins, p->seg_stride, p->n_features, best,
                                                p->leaf, p->n, level);
    else
        apply_split_kernel<8><<<g, 256, 0, s>>>(p->bins, p->seg_stride, p->n_features, best,
                                                p->leaf, p->n, level);
    CBH_LAUNCHED();
    return CBH_OK;
}

int launch_update(const cbh_ctx* ctx, const cbh_problem* p, const void* hist_last,
                  int32_t precision, const cbh_split* last, double lr, double l2,
                  double* leaf_values, int64_t* leaf_counts, hipStream_t s) {
    const int64_t leaves = int64_t(1) << p->depth;
    if (hist_last) {
        SolveArgs sa;
        sa.hist = hist_last;
        sa.split = last;
        sa.grad_scale = p->grad_scale;
        sa.values = leaf_values;
        sa.depth = p->depth;
        sa.F = p->n_features;
        sa.B = p->max_bins;
        sa.K = p->K;
        sa.rmse = count_stat(p);
        sa.precision = out_prec(precision);
        sa.l2 = l2;
        const int64_t work = leaves * p->K;
        leaf_solve_kernel<<<(unsigned)((work + 3) / 4), 256, 0, s>>>(sa);
        CBH_LAUNCHED();
    }
    UpdArgs ua;
    ua.leaf = p->leaf;
    ua.values = leaf_values;
    ua.label = p->label;
    ua.weight = p->weight;
    ua.approx = p->approx;
    ua.g = p->g;
    ua.h = p->h;
    ua.n = p->n;
    ua.K = p->K;
    ua.loss = p->loss;
    ua.add = hist_last != nullptr;
    ua.lmask = (uint16_t)(leaves - 1);
    ua.lr = lr;
    const int gr = grid_rows(ctx, p->n);
    switch (p->loss) {
        case CBH_LOSS_RMSE: update_kernel<CBH_LOSS_RMSE><<<gr, 256, 0, s>>>(ua); break;
        case CBH_LOSS_LOGLOSS: update_kernel<CBH_LOSS_LOGLOSS><<<gr, 256, 0, s>>>(ua); break;
        default: update_kernel<CBH_LOSS_MULTICLASS><<<gr, 256, 0, s>>>(ua); break;
    }
    CBH_LAUNCHED();
    if (leaf_counts) {
        zero_i64_kernel<<<(unsigned)((leaves + 255) / 256), 256, 0, s>>>(leaf_counts, leaves);
        leaf_count_kernel<<<grid_rows(ctx, p->n, 16), 256, (size_t)leaves * 4, s>>>(
            p->leaf, p->n, (int32_t)leaves, (unsigned long long*)leaf_counts);
        CBH_LAUNCHED();
    }
    return CBH_OK;
}

}  // namespace cbh

namespace cbh {

// Model apply (Sec. 4, "Fast scorer"): tree t's leaf for a row is the
// binary vector sum_i 2^i [bin_{f(t,i)} > k(t,i)], and the row's approx gains
// lr * v[t][leaf][c], tree after tree in model order (the additions of the
// model updates that built the trees, in the same order and precision).
// The model goes through in chunks of trees, two launches per chunk:
//   model_leaves_kernel  one block per (row block, tree of the chunk): each thread
//                        finds the leaves of 4 consecutive rows (one 32-bit
//                        load per level gives their 4 bins; the tree's splits
//                        are the same for the whole block, so they and the
//                        column pointers come through scalar loads) and
//                        stores them as [tree][row] (uint8 up to depth 8,
//                        else uint16);
//   model_sum_kernel     one thread per row adds the chunk's trees in order,
//                        16 (one class) or 8 trees' leaves and values loaded
//                        before their adds.
// Every (tree, row) leaf is independent, so the first launch has T x n / 4
// threads of work where a single pass over the rows would have n / 4, each
// walking the whole model.
struct ApplyArgs {
    const uint8_t* const* bins;
    const int64_t* seg;
    int64_t n;
    int32_t F, K, d, t0, nt;
    const int32_t* feat;
    const int32_t* border;
    const double* values;
    double lr;
    double* approx;
    void* leaves;                  // [nt][n] of LT: uint8 for depth <= 8, else uint16
    uint32_t* flags;
};

// Block b runs on XCD b mod 8. Row block rb (1024 rows) goes to XCD rb mod
// 8 with all the chunk's trees in turn, so its bins of every feature (1 KB
// per feature) stay in that XCD's L2 while the trees read them.
template <typename LT>
__global__ __launch_bounds__(256) void model_leaves_kernel(ApplyArgs a) {
    const int64_t j = blockIdx.x >> 3;
    const int64_t rb = (j / a.nt) * 8 + (blockIdx.x & 7);
    const int tl = (int)(j % a.nt);
    const int64_t i0 = (rb * 256 + threadIdx.x) * 4;
    if (i0 >= a.n) return;
    const int nr = (int)min<int64_t>(4, a.n - i0);
    const int64_t t = a.t0 + tl;
    uint32_t lf[4] = {0u, 0u, 0u, 0u};
    bool bad = false;
    for (int l = 0; l < a.d; ++l) {
        const int f = a.feat[t * a.d + l];
        const int k = a.border[t * a.d + l];
        if ((unsigned)f >= (unsigned)a.F) {
            bad = true;
            continue;
        }
        const uint8_t* col = a.bins[f];
        const int64_t st = a.seg ? a.seg[f] : 16;
        const uint8_t* p = col + (i0 >> 4) * st + (i0 & 15);
        uint32_t w = 0u;
        if (nr == 4 && ((reinterpret_cast<uintptr_t>(p) & 3) == 0)) {
            w = gld_u32(p);
        } else {
            for (int r = 0; r < nr; ++r) w |= gld_u8(seg_ptr(col, st, i0 + r)) << (8 * r);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) lf[r] |= ((int)((w >> (8 * r)) & 255u) > k ? 1u : 0u) << l;
    }
    LT* out = reinterpret_cast<LT*>(a.leaves) + int64_t(tl) * a.n + i0;
    if (nr == 4 && ((reinterpret_cast<uintptr_t>(out) & (4 * sizeof(LT) - 1)) == 0)) {
        if constexpr (sizeof(LT) == 1)
            *reinterpret_cast<uint32_t*>(out) = lf[0] | (lf[1] << 8) | (lf[2] << 16) | (lf[3] << 24);
        else
            *reinterpret_cast<uint2*>(out) = make_uint2(lf[0] | (lf[1] << 16), lf[2] | (lf[3] << 16));
    } else {
        for (int r = 0; r < nr; ++r) out[r] = (LT)lf[r];
    }
    if (bad && threadIdx.x == 0 && rb == 0) atomicOr(a.flags, FLAG_BAD_SPLIT);
}

template <typename LT, int KC>
__global__ __launch_bounds__(256) void model_sum_kernel(ApplyArgs a) {
    const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (i >= a.n) return;
    const int K = KC == 1 ? 1 : a.K;
    const int64_t nl = int64_t(1) << a.d;
    double acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = c < K ? a.approx[int64_t(c) * a.n + i] : 0.0;
    const LT* leaves = reinterpret_cast<const LT*>(a.leaves);
    constexpr int U = KC == 1 ? 16 : 8;
    int tl = 0;
    for (; tl + U <= a.nt; tl += U) {
        uint32_t lf[U];
#pragma unroll
        for (int u = 0; u < U; ++u) lf[u] = leaves[int64_t(tl + u) * a.n + i];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double* v = a.values + ((int64_t(a.t0 + tl + u) * nl) + lf[u]) * K;
#pragma unroll
            for (int c = 0; c < KC; ++c)
                if (c < K) acc[c] = acc[c] + a.lr * v[c];
        }
    }
    for (; tl < a.nt; ++tl) {
        const uint32_t lf = leaves[int64_t(tl) * a.n + i];
        const double* v = a.values + ((int64_t(a.t0 + tl) * nl) + lf) * K;
#pragma unroll
        for (int c = 0; c < KC; ++c)
            if (c < K) acc[c] = acc[c] + a.lr * v[c];
    }
#pragma unroll
    for (int c = 0; c < KC; ++c)
        if (c < K) a.approx[int64_t(c) * a.n + i] = acc[c];
}

// ------------------------------------------------- binarized model apply
// The scorer of Sec. 4 in its two steps. First every binary feature the
// model uses, (feature bf[j], border bk[j]), is evaluated once for every row
// into a bit vector: bits[j][w] bit r = [bin of row 32 w + r > bk[j]]
// (binarize_kernel). Then a tree's leaf index of a row is the binary vector
// sum_l 2^l B(row, s(t, l)) read from those bits (model_leaves_bits_kernel),
// and the leaves are summed as in cbh_apply_model.
constexpr int kBinJ = 8;   // binary features per binarize block

// One thread per 32-row word, kBinJ consecutive binary features per block:
// a feature's 32 bins are loaded once for the run of its binary features
// among the block's kBinJ (features given next to each other share loads).
__global__ __launch_bounds__(256) void binarize_kernel(
    const uint8_t* const* __restrict__ bins, const int64_t* __restrict__ seg, int64_t n,
    int32_t F, int32_t nb, const int32_t* __restrict__ bf, const int32_t* __restrict__ bk,
    int64_t nw, int64_t wblocks, uint32_t* __restrict__ bits, uint32_t* flags) {
    const int64_t jb = int64_t(blockIdx.x) / wblocks;
    const int64_t w = (int64_t(blockIdx.x) % wblocks) * 256 + threadIdx.x;
    if (w >= nw) return;
    const int64_t i0 = w * 32;
    const int nr = (int)min<int64_t>(32, n - i0);
    int prev = -1;
    uint32_t v[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};   // the 32 bins, 4 per word
    bool bad = false;
    for (int jj = 0; jj < kBinJ; ++jj) {
        const int64_t j = jb * kBinJ + jj;
        if (j >= nb) break;
        const int f = bf[j];
        const int k = bk[j];
        uint32_t word = 0u;
        if ((unsigned)f >= (unsigned)F) {
            bad = true;
        } else {
            if (f != prev) {
                const uint8_t* col = bins[f];
                const int64_t st = seg ? seg[f] : 16;
                const uint8_t* p0 = col + (i0 >> 4) * st;
                const uint8_t* p1 = p0 + st;
                if (nr == 32 && ((reinterpret_cast<uintptr_t>(col) | (uintptr_t)st) & 15) == 0) {
                    const uint4 a = gld_u4(p0), b = gld_u4(p1);
                    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
                    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
                } else {
#pragma unroll
                    for (int q = 0; q < 8; ++q) v[q] = 0u;
                    for (int r = 0; r < nr; ++r)
                        v[r >> 2] |= gld_u8((r < 16 ? p0 : p1) + (r & 15)) << (8 * (r & 3));
                }
                prev = f;
            }
#pragma unroll
            for (int r = 0; r < 32; ++r)
                word |= (((int)((v[r >> 2] >> (8 * (r & 3))) & 255u) > k) ? 1u : 0u) << r;
            if (nr < 32) word &= (1u << nr) - 1u;
        }
        bits[j * nw + w] = word;
    }
    if (bad && threadIdx.x == 0) atomicOr(flags, FLAG_BAD_SPLIT);
}

// One thread per (tree of the chunk, 32-row word): the tree's depth bit
// words of the word's rows give its 32 leaf indices, stored [tree][row].
struct ApplyBitsArgs {
    const uint32_t* bits;
    int64_t n, nw;
    int32_t nb, d, t0, nt;
    int64_t wblocks;
    const int32_t* split;     // [tree][depth] binary feature index
    void* leaves;
    uint32_t* flags;
};

template <typename LT>
__global__ __launch_bounds__(256) void model_leaves_bits_kernel(ApplyBitsArgs a) {
    const int tl = (int)(int64_t(blockIdx.x) / a.wblocks);
    const int64_t w = (int64_t(blockIdx.x) % a.wblocks) * 256 + threadIdx.x;
    if (w >= a.nw) return;
    const int64_t t = a.t0 + tl;
    uint32_t wd[CBH_MAX_DEPTH];
    bool bad = false;
#pragma unroll
    for (int l = 0; l < CBH_MAX_DEPTH; ++l) {
        wd[l] = 0u;
        if (l < a.d) {
            const int j = a.split[t * a.d + l];
            if ((unsigned)j >= (unsigned)a.nb) bad = true;
            else wd[l] = a.bits[int64_t(j) * a.nw + w];
        }
    }
    const int64_t i0 = w * 32;
    const int nr = (int)min<int64_t>(32, a.n - i0);
    LT* out = reinterpret_cast<LT*>(a.leaves) + int64_t(tl) * a.n + i0;
    if constexpr (sizeof(LT) == 1) {
        uint32_t o[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            uint32_t x = 0u;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int r = 4 * q + b;
                uint32_t lf = 0u;
#pragma unroll
                for (int l = 0; l < 8; ++l) lf |= ((wd[l] >> r) & 1u) << l;
                x |= lf << (8 * b);
            }
            o[q] = x;
        }
        if (nr == 32 && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
            reinterpret_cast<uint4*>(out)[0] = make_uint4(o[0], o[1], o[2], o[3]);
            reinterpret_cast<uint4*>(out)[1] = make_uint4(o[4], o[5], o[6], o[7]);
        } else {
            for (int r = 0; r < nr; ++r) out[r] = (LT)((o[r >> 2] >> (8 * (r & 3))) & 255u);
        }
    } else {
        for (int r = 0; r < nr; ++r) {
            uint32_t lf = 0u;
#pragma unroll
            for (int l = 0; l < CBH_MAX_DEPTH; ++l) lf |= ((wd[l] >> r) & 1u) << l;
            out[r] = (LT)lf;
        }
    }
    if (bad && threadIdx.x == 0) atomicOr(a.flags, FLAG_BAD_SPLIT);
}

}  // namespace cbh

using namespace cbh;

extern "C" {

int cbh_apply_model(cbh_ctx* ctx, const uint8_t* const* bins, const int64_t* seg_stride,
                    int64_t n, int32_t n_features, int32_t K, int32_t n_trees, int32_t depth,
                    const int32_t* split_feature, const int32_t* split_border,
                    const double* leaf_values, double lr, double* approx, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0 && n < (int64_t(1) << 40), "n must be in [0, 2^40)");
    CBH_ARG(n_features >= 1, "n_features must be >= 1");
    CBH_REQUIRE(K >= 1 && K <= CBH_MAX_K, CBH_EUNSUPPORTED, "K must be in [1, 16] (got %d)", K);
    CBH_ARG(n_trees >= 0, "n_trees must be >= 0");
    CBH_REQUIRE(depth >= 1 && depth <= CBH_MAX_DEPTH, CBH_EUNSUPPORTED,
                "depth must be in [1, 16] (got %d)", depth);
    CBH_ARG(std::isfinite(lr), "lr must be finite");
    if (n == 0 || n_trees == 0) return CBH_OK;
    CBH_ARG(bins && split_feature && split_border && leaf_values && approx, "NULL argument");
    // one thread per row in the summing launch: the grid must stay below 2^31
    CBH_REQUIRE(n < (int64_t(1) << 38), CBH_EUNSUPPORTED, "n must be < 2^38");
    // trees per chunk: their leaves ([chunk][n], one byte each up to depth 8,
    // else two) stay within 256 MB of workspace
    const int64_t lb = depth <= 8 ? 1 : 2;
    const int64_t per = std::max<int64_t>(1, (int64_t(256) << 20) / (lb * n));
    // the leaf launch has one block per (1024-row block, tree), row blocks
    // padded to a multiple of 8: at most 2^31 - 1 blocks
    const int64_t rblocks = align_up((n + 1023) / 1024, 8);
    const int64_t per_grid = std::max<int64_t>(1, int64_t(INT32_MAX) / rblocks);
    const int32_t chunk =
        (int32_t)std::min<int64_t>({int64_t(n_trees), per, per_grid, 65535});
    int rc = ensure_ws(ctx, int64_t(chunk) * n * lb, stream);
    if (rc) return rc;
    ApplyArgs a;
    a.bins = bins;
    a.seg = seg_stride;
    a.n = n;
    a.F = n_features;
    a.K = K;
    a.d = depth;
    a.feat = split_feature;
    a.border = split_border;
    a.values = leaf_values;
    a.lr = lr;
    a.approx = approx;
    a.leaves = ctx->ws;
    a.flags = ctx->d_flags;
    hipStream_t s = (hipStream_t)stream;
    for (int32_t t0 = 0; t0 < n_trees; t0 += chunk) {
        a.t0 = t0;
        a.nt = std::min(chunk, n_trees - t0);
        const unsigned lg = (unsigned)(rblocks * a.nt);
        const unsigned grid = (unsigned)((n + 255) / 256);
        if (lb == 1) {
            model_leaves_kernel<uint8_t><<<lg, 256, 0, s>>>(a);
            CBH_LAUNCHED();
            if (K == 1) model_sum_kernel<uint8_t, 1><<<grid, 256, 0, s>>>(a);
            else model_sum_kernel<uint8_t, CBH_MAX_K><<<grid, 256, 0, s>>>(a);
        } else {
            model_leaves_kernel<uint16_t><<<lg, 256, 0, s>>>(a);
            CBH_LAUNCHED();
            if (K == 1) model_sum_kernel<uint16_t, 1><<<grid, 256, 0, s>>>(a);
            else model_sum_kernel<uint16_t, CBH_MAX_K><<<grid, 256, 0, s>>>(a);
        }
        CBH_LAUNCHED();
    }
    return CBH_OK;
}

int cbh_binarize(cbh_ctx* ctx, const uint8_t* const* bins, const int64_t* seg_stride, int64_t n,
                 int32_t n_features, int32_t n_binary, const int32_t* bin_feature,
                 const int32_t* bin_border, uint32_t* bits_out, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0 && n < (int64_t(1) << 40), "n must be in [0, 2^40)");
    CBH_ARG(n_features >= 1, "n_features must be >= 1");
    CBH_ARG(n_binary >= 0, "n_binary must be >= 0");
    if (n == 0 || n_binary == 0) return CBH_OK;
    CBH_ARG(bins && bin_feature && bin_border && bits_out, "NULL argument");
    const int64_t nw = (n + 31) / 32;
    const int64_t wblocks = (nw + 255) / 256;
    const int64_t blocks = wblocks * ((n_binary + kBinJ - 1) / kBinJ);
    CBH_REQUIRE(blocks <= INT32_MAX, CBH_EUNSUPPORTED, "too many (binary feature, row) words");
    binarize_kernel<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(
        bins, seg_stride, n, n_features, n_binary, bin_feature, bin_border, nw, wblocks, bits_out,
        ctx->d_flags);
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_apply_model_binarized(cbh_ctx* ctx, const uint32_t* bits, int64_t n, int32_t n_binary,
                              int32_t K, int32_t n_trees, int32_t depth,
                              const int32_t* split_binary, const double* leaf_values, double lr,
                              double* approx, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0 && n < (int64_t(1) << 38), "n must be in [0, 2^38)");
    CBH_ARG(n_binary >= 1, "n_binary must be >= 1");
    CBH_REQUIRE(K >= 1 && K <= CBH_MAX_K, CBH_EUNSUPPORTED, "K must be in [1, 16] (got %d)", K);
    CBH_ARG(n_trees >= 0, "n_trees must be >= 0");
    CBH_REQUIRE(depth >= 1 && depth <= CBH_MAX_DEPTH, CBH_EUNSUPPORTED,
                "depth must be in [1, 16] (got %d)", depth);
    CBH_ARG(std::isfinite(lr), "lr must be finite");
    if (n == 0 || n_trees == 0) return CBH_OK;
    CBH_ARG(bits && split_binary && leaf_values && approx, "NULL argument");
    const int64_t lb = depth <= 8 ? 1 : 2;
    const int64_t nw = (n + 31) / 32;
    const int64_t wblocks = (nw + 255) / 256;
    const int64_t per = std::max<int64_t>(1, (int64_t(256) << 20) / (lb * n));
    const int64_t per_grid = std::max<int64_t>(1, int64_t(INT32_MAX) / wblocks);
    const int32_t chunk =
        (int32_t)std::min<int64_t>({int64_t(n_trees), per, per_grid, 65535});
    int rc = ensure_ws(ctx, int64_t(chunk) * n * lb, stream);
    if (rc) return rc;
    ApplyBitsArgs b;
    b.bits = bits;
    b.n = n;
    b.nw = nw;
    b.nb = n_binary;
    b.d = depth;
    b.wblocks = wblocks;
    b.split = split_binary;
    b.leaves = ctx->ws;
    b.flags = ctx->d_flags;
    ApplyArgs a;   // the summing launch's arguments (bins and splits unused)
    a.bins = nullptr;
    a.seg = nullptr;
    a.n = n;
    a.F = 0;
    a.K = K;
    a.d = depth;
    a.feat = nullptr;
    a.border = nullptr;
    a.values = leaf_values;
    a.lr = lr;
    a.approx = approx;
    a.leaves = ctx->ws;
    a.flags = ctx->d_flags;
    hipStream_t s = (hipStream_t)stream;
    for (int32_t t0 = 0; t0 < n_trees; t0 += chunk) {
        b.t0 = a.t0 = t0;
        b.nt = a.nt = std::min(chunk, n_trees - t0);
        const unsigned lg = (unsigned)(wblocks * b.nt);
        const unsigned grid = (unsigned)((n + 255) / 256);
        if (lb == 1) {
            model_leaves_bits_kernel<uint8_t><<<lg, 256, 0, s>>>(b);
            CBH_LAUNCHED();
            if (K == 1) model_sum_kernel<uint8_t, 1><<<grid, 256, 0, s>>>(a);
            else model_sum_kernel<uint8_t, CBH_MAX_K><<<grid, 256, 0, s>>>(a);
        } else {
            model_leaves_bits_kernel<uint16_t><<<lg, 256, 0, s>>>(b);
            CBH_LAUNCHED();
            if (K == 1) model_sum_kernel<uint16_t, 1><<<grid, 256, 0, s>>>(a);
            else model_sum_kernel<uint16_t, CBH_MAX_K><<<grid, 256, 0, s>>>(a);
        }
        CBH_LAUNCHED();
    }
    return CBH_OK;
}

int cbh_pack_bins(cbh_ctx* ctx, const uint8_t* const* bins, const int64_t* seg_stride,
                  int32_t n_features, int64_t n, int32_t bits, uint8_t* const* packed,
                  void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr && bins != nullptr && packed != nullptr, "NULL argument");
    CBH_ARG(n >= 1 && n_features >= 1, "n and n_features must be >= 1");
    CBH_ARG(bits == 4 || bits == 1, "bits must be 4 or 1 (got %d)", bits);
    const int64_t n_seg = (n + 15) / 16;
    const int64_t total = n_seg * n_features;
    const unsigned g = (unsigned)std::max<int64_t>(
        1, std::min<int64_t>((total + 255) / 256, int64_t(ctx->num_cus) * 16));
    hipStream_t s = (hipStream_t)stream;
    if (bits == 4)
        pack_bins_kernel<4><<<g, 256, 0, s>>>(bins, seg_stride, packed, n_features, n, n_seg,
                                              ctx->d_flags);
    else
        pack_bins_kernel<1><<<g, 256, 0, s>>>(bins, seg_stride, packed, n_features, n, n_seg,
                                              ctx->d_flags);
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_apply_split(cbh_ctx* ctx, const cbh_problem* prob, int32_t level, const cbh_split* best,
                    void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    int rc = validate_problem(prob);
    if (rc) return rc;
    CBH_ARG(level >= 0 && level < prob->depth, "level %d outside [0, depth)", level);
    CBH_ARG(best != nullptr, "best is NULL");
    return launch_apply(ctx, prob, level, best, (hipStream_t)stream);
}

int cbh_update_approx(cbh_ctx* ctx, const cbh_problem* prob, const void* hist_last,
                      int32_t precision, const cbh_split* last, double lr, double l2,
                      double* leaf_values_out, int64_t* leaf_counts_out, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    int rc = validate_problem(prob);
    if (rc) return rc;
    if (hist_last) {
        rc = validate_precision(prob, precision);
        if (rc) return rc;
        CBH_ARG(last != nullptr && leaf_values_out != nullptr,
                "last and leaf_values_out are required with hist_last");
        CBH_ARG(std::isfinite(lr), "lr must be finite");
        CBH_ARG(l2 >= 0 && std::isfinite(l2), "l2 must be finite and >= 0");
        CBH_REQUIRE(prob->depth <= 13 || leaf_counts_out == nullptr, CBH_EUNSUPPORTED,
                    "leaf counts need depth <= 13");
    } else {
        CBH_ARG(last == nullptr && leaf_values_out == nullptr && leaf_counts_out == nullptr,
                "without hist_last, last / leaf_values_out / leaf_counts_out must be NULL");
    }
    return launch_update(ctx, prob, hist_last, precision, last, lr, l2, leaf_values_out,
                         leaf_counts_out, (hipStream_t)stream);
}

}  // extern "C"
