// Ordered boosting (Sec. 3): the supporting approximations of one
// permutation, kept as about log2(n) models instead of one per position.
//
// Model m (m = 0..M-1) learns from the positions below T_m (T_0 = 0,
// T_m = 2^(m-1)) and is kept for the positions below min(n, 2^m). The
// gradient that chooses the next tree structure is taken, for the row at
// position p, at model m(p) = bit length of p (0 for p = 0): that model
// learned from the positions below 2^floor(log2 p) <= p only. Every model
// shares the tree structure and takes its own Newton leaf values from its
// own gradients over its learning positions. The model that is kept for
// prediction (the second phase of Sec. 3) takes its leaf values from its own
// gradients over all rows.
//
// Layout: support [K][S], model m's values from offset off_m = sum over
// m' < m of min(n, 2^m'), in position order; S = off_M < 4n. With
// mc = bit length of n, models below mc hold 2^m values (off_m = 2^m - 1)
// and the rest hold n each.
//
// Launches of one update:
//   ord_gather_kernel  leaf and label of every position (one gather through
//                      perm), so that the later passes read both in position
//                      order;
//   ord_sums_kernel    per (leaf, class) (G, H) of every model: each block
//                      takes kOrdChunk learning entries of one model, sums in
//                      FP64 LDS (one copy per wave when that fits) and writes
//                      its partial;
//   ord_solve_kernel   one wave per (model, leaf, class): the partials of the
//                      model's blocks in a fixed lane order, then -G/(H + l2);
//   ord_apply_kernel   every row of the kept model and every kept entry of
//                      every supporting model gains lr * its leaf's value;
//                      an entry that its position reads also writes that
//                      row's g and h for the next tree.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace cbh {

constexpr int kOrdThreads = 256;
constexpr int64_t kOrdChunk = 2048;        // learning entries per sums block
constexpr int kOrdMaxSeg = 48;             // kept model + supporting models (n < 2^40)
constexpr int64_t kOrdMaxCells = 4096;     // leaves x classes
constexpr int64_t kOrdWaveLds = 32 * 1024; // per-wave copies when they fit in this

__host__ __device__ inline int ord_bitlen(uint64_t x) {
    return x ? 64 - __builtin_clzll(x) : 0;
}
__host__ __device__ inline int32_t ord_models(int64_t n) {
    return n <= 1 ? 1 : ord_bitlen((uint64_t)(n - 1)) + 1;
}
__host__ __device__ inline int64_t ord_learn(int m) { return m ? int64_t(1) << (m - 1) : 0; }
__host__ __device__ inline int64_t ord_offset(int64_t n, int m) {
    const int mc = ord_bitlen((uint64_t)n);   // 2^(mc-1) <= n < 2^mc
    if (m <= mc) return (int64_t(1) << m) - 1;
    return ((int64_t(1) << mc) - 1) + int64_t(m - mc) * n;
}

struct OrdArgs {
    int64_t n, S;
    int32_t M, K, cells, copies;
    uint32_t lmask;
    const int32_t* perm;
    const uint16_t* leaf;      // row order
    const float* label;        // row order
    double* approx;            // kept model [K][n]
    double* support;           // [K][S]
    float* g;                  // [K][n] row order
    float* h;                  // [K][n] row order, NULL for RMSE (h = 1)
    uint16_t* lpos;            // leaf by position
    float* ypos;               // label by position
    double* part;              // [blocks][cells][2]
    double* vals;              // [1 + M][cells]: kept model, then supporting model m
    uint32_t* flags;
    int32_t keep;              // the kept model is updated too
    double lr, l2;
    // segment s's first sums block: s = 0 the kept model (n rows), s = 1 + m
    // supporting model m (its T_m learning positions)
    int64_t blk_off[kOrdMaxSeg + 1];
};

template <int LOSS>
__device__ inline void ord_derivs(const double* a, double y, int K, double* g, double* h) {
    if constexpr (LOSS == CBH_LOSS_RMSE) {
        g[0] = a[0] - y;
        h[0] = 1.0;
    } else if constexpr (LOSS == CBH_LOSS_LOGLOSS) {
        const double p = 1.0 / (1.0 + exp(-a[0]));
        g[0] = p - y;
        h[0] = p * (1.0 - p);
    } else {
        double mx = a[0];
        for (int c = 1; c < K; ++c) mx = a[c] > mx ? a[c] : mx;
        double z = 0.0;
        for (int c = 0; c < K; ++c) z += exp(a[c] - mx);
        const int yc = (int)y;
        for (int c = 0; c < K; ++c) {
            const double p = exp(a[c] - mx) / z;
            g[c] = p - (c == yc ? 1.0 : 0.0);
            h[c] = p * (1.0 - p);
        }
    }
}

__global__ __launch_bounds__(kOrdThreads) void ord_gather_kernel(OrdArgs a) {
    for (int64_t p = int64_t(blockIdx.x) * kOrdThreads + threadIdx.x; p < a.n;
         p += int64_t(gridDim.x) * kOrdThreads) {
        const int32_t r = a.perm[p];
        if (r < 0 || r >= a.n) {
            atomicOr(a.flags, FLAG_BAD_INDEX);
            a.lpos[p] = 0;
            a.ypos[p] = 0.f;
            continue;
        }
        a.lpos[p] = (uint16_t)(a.leaf[r] & a.lmask);
        a.ypos[p] = a.label[r];
    }
}

template <int LOSS>
__global__ __launch_bounds__(kOrdThreads) void ord_sums_kernel(OrdArgs a) {
    extern __shared__ double sh[];   // [copies][cells][2]
    constexpr bool MC = LOSS == CBH_LOSS_MULTICLASS;
    const int K = MC ? a.K : 1;
    int s = 0;
    while (s < a.M && a.blk_off[s + 1] <= (int64_t)blockIdx.x) ++s;
    const int64_t cnt = s == 0 ? a.n : ord_learn(s - 1);
    const int64_t i0 = (int64_t(blockIdx.x) - a.blk_off[s]) * kOrdChunk;
    const int64_t i1 = i0 + kOrdChunk < cnt ? i0 + kOrdChunk : cnt;
    const int words = a.cells * 2;
    for (int i = threadIdx.x; i < a.copies * words; i += kOrdThreads) sh[i] = 0.0;
    __syncthreads();
    double* mine = sh + (a.copies > 1 ? (threadIdx.x >> 6) * words : 0);
    const int64_t off = s == 0 ? 0 : ord_offset(a.n, s - 1);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kOrdThreads) {
        int L;
        double y, av[MC ? CBH_MAX_K : 1], gg[MC ? CBH_MAX_K : 1], hh[MC ? CBH_MAX_K : 1];
        if (s == 0) {
            L = (int)(a.leaf[i] & a.lmask);
            y = (double)a.label[i];
            for (int c = 0; c < K; ++c) av[c] = a.approx[int64_t(c) * a.n + i];
        } else {
            L = a.lpos[i];
            y = (double)a.ypos[i];
            for (int c = 0; c < K; ++c) av[c] = a.support[int64_t(c) * a.S + off + i];
        }
        ord_derivs<LOSS>(av, y, K, gg, hh);
        for (int c = 0; c < K; ++c) {
            double* cell = mine + (L * K + c) * 2;
            __hip_atomic_fetch_add(cell, gg[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(cell + 1, hh[c], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();
    double* out = a.part + int64_t(blockIdx.x) * words;
    for (int i = threadIdx.x; i < words; i += kOrdThreads) {
        double v = 0.0;
        for (int c = 0; c < a.copies; ++c) v += sh[c * words + i];
        out[i] = v;
    }
}

__global__ __launch_bounds__(256) void ord_solve_kernel(OrdArgs a, double* leaf_values,
                                                        double* support_values) {
    const int64_t w = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (w >= int64_t(a.M + 1) * a.cells) return;
    const int s = (int)(w / a.cells), cell = (int)(w % a.cells);
    double G = 0.0, H = 0.0;
    for (int64_t b = a.blk_off[s] + lane; b < a.blk_off[s + 1]; b += 64) {
        G += a.part[(b * a.cells + cell) * 2];
        H += a.part[(b * a.cells + cell) * 2 + 1];
    }
    for (int d = 32; d >= 1; d >>= 1) {
        G += __shfl_xor(G, d, 64);
        H += __shfl_xor(H, d, 64);
    }
    if (lane != 0) return;
    const double den = H + a.l2;
    const double v = den == 0.0 ? 0.0 : -G / den;
    a.vals[w] = v;
    if (s == 0) {
        if (leaf_values) leaf_values[cell] = v;
    } else if (support_values) support_values[int64_t(s - 1) * a.cells + cell] = v;
}

template <int LOSS>
__global__ __launch_bounds__(256) void ord_apply_kernel(OrdArgs a) {
    constexpr bool MC = LOSS == CBH_LOSS_MULTICLASS;
    const int K = MC ? a.K : 1;
    const int mc = ord_bitlen((uint64_t)a.n);
    const int64_t full = (int64_t(1) << mc) - 1;   // entries of the models below mc
    for (int64_t t = (a.keep ? 0 : a.n) + int64_t(blockIdx.x) * 256 + threadIdx.x; t < a.n + a.S;
         t += int64_t(gridDim.x) * 256) {
        if (t < a.n) {   // the kept model, row t
            const double* v = a.vals + int64_t(a.leaf[t] & a.lmask) * K;
            for (int c = 0; c < K; ++c) a.approx[int64_t(c) * a.n + t] += a.lr * v[c];
            continue;
        }
        const int64_t e = t - a.n;
        int m;
        int64_t j;
        if (e < full) {
            m = ord_bitlen((uint64_t)(e + 1)) - 1;
            j = e - ((int64_t(1) << m) - 1);
        } else {
            const int64_t q = (e - full) / a.n;
            m = mc + (int)q;
            j = e - full - q * a.n;
        }
        const double* v = a.vals + int64_t(1 + m) * a.cells + int64_t(a.lpos[j]) * K;
        double av[MC ? CBH_MAX_K : 1], gg[MC ? CBH_MAX_K : 1], hh[MC ? CBH_MAX_K : 1];
        for (int c = 0; c < K; ++c) {
            const double x = a.support[int64_t(c) * a.S + e] + a.lr * v[c];
            a.support[int64_t(c) * a.S + e] = x;
            av[c] = x;
        }
        if (ord_bitlen((uint64_t)j) != m) continue;   // position j reads another model
        const int32_t r = a.perm[j];
        if (r < 0 || r >= a.n) continue;              // flagged by the gather
        ord_derivs<LOSS>(av, (double)a.ypos[j], K, gg, hh);
        for (int c = 0; c < K; ++c) {
            a.g[int64_t(c) * a.n + r] = (float)gg[c];
            if (a.h) a.h[int64_t(c) * a.n + r] = (float)hh[c];
        }
    }
}

// Gradients for the next tree straight from the support (no update).
template <int LOSS>
__global__ __launch_bounds__(256) void ord_grad_kernel(OrdArgs a) {
    constexpr bool MC = LOSS == CBH_LOSS_MULTICLASS;
    const int K = MC ? a.K : 1;
    for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < a.n;
         p += int64_t(gridDim.x) * 256) {
        const int32_t r = a.perm[p];
        if (r < 0 || r >= a.n) {
            atomicOr(a.flags, FLAG_BAD_INDEX);
            continue;
        }
        const int64_t e = ord_offset(a.n, ord_bitlen((uint64_t)p)) + p;
        double av[MC ? CBH_MAX_K : 1], gg[MC ? CBH_MAX_K : 1], hh[MC ? CBH_MAX_K : 1];
        for (int c = 0; c < K; ++c) av[c] = a.support[int64_t(c) * a.S + e];
        ord_derivs<LOSS>(av, (double)a.label[r], K, gg, hh);
        for (int c = 0; c < K; ++c) {
            a.g[int64_t(c) * a.n + r] = (float)gg[c];
            if (a.h) a.h[int64_t(c) * a.n + r] = (float)hh[c];
        }
    }
}

int validate_ordered(const cbh_ctx* ctx, const cbh_ordered* ord, const cbh_problem* p) {
    CBH_ARG(ctx != nullptr && ord != nullptr, "NULL argument");
    int rc = validate_problem(p);
    if (rc) return rc;
    CBH_ARG(ord->n == p->n, "ordered n (%lld) differs from the problem's n (%lld)",
            (long long)ord->n, (long long)p->n);
    CBH_ARG(ord->perm != nullptr && ord->support != nullptr, "perm / support is NULL");
    CBH_REQUIRE(p->weight == nullptr, CBH_EUNSUPPORTED,
                "ordered boosting takes no row weights");
    CBH_REQUIRE((int64_t(1) << p->depth) * p->K <= kOrdMaxCells, CBH_EUNSUPPORTED,
                "ordered boosting needs 2^depth * K <= %lld (got %lld)",
                (long long)kOrdMaxCells, (long long)((int64_t(1) << p->depth) * p->K));
    return CBH_OK;
}

static OrdArgs ord_args(cbh_ctx* ctx, const cbh_ordered* ord, const cbh_problem* p) {
    OrdArgs a{};
    a.n = p->n;
    a.M = ord_models(p->n);
    a.S = ord_offset(p->n, a.M);
    a.K = p->K;
    a.cells = (int32_t)((int64_t(1) << p->depth) * p->K);
    a.lmask = (uint32_t)((1u << p->depth) - 1);
    a.perm = ord->perm;
    a.leaf = p->leaf;
    a.label = p->label;
    a.approx = p->approx;
    a.support = ord->support;
    a.g = p->g;
    a.h = count_stat(p) ? nullptr : p->h;
    a.flags = ctx->d_flags;
    return a;
}

template <template <int> class KernelOf>
static void launch_by_loss(int loss, dim3 g, dim3 b, size_t lds, hipStream_t s, const OrdArgs& a) {
    switch (loss) {
        case CBH_LOSS_RMSE: KernelOf<CBH_LOSS_RMSE>::run(g, b, lds, s, a); break;
        case CBH_LOSS_LOGLOSS: KernelOf<CBH_LOSS_LOGLOSS>::run(g, b, lds, s, a); break;
        default: KernelOf<CBH_LOSS_MULTICLASS>::run(g, b, lds, s, a); break;
    }
}
template <int L> struct SumsK {
    static void run(dim3 g, dim3 b, size_t lds, hipStream_t s, const OrdArgs& a) {
        ord_sums_kernel<L><<<g, b, lds, s>>>(a);
    }
};
template <int L> struct ApplyK {
    static void run(dim3 g, dim3 b, size_t lds, hipStream_t s, const OrdArgs& a) {
        ord_apply_kernel<L><<<g, b, lds, s>>>(a);
    }
};
template <int L> struct GradK {
    static void run(dim3 g, dim3 b, size_t lds, hipStream_t s, const OrdArgs& a) {
        ord_grad_kernel<L><<<g, b, lds, s>>>(a);
    }
};

static unsigned ord_grid(const cbh_ctx* ctx, int64_t items) {
    const int64_t cap = int64_t(ctx->num_cus) * 16;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cap, (items + 255) / 256));
}

int ordered_update(cbh_ctx* ctx, const cbh_ordered* ord, const cbh_problem* p, double lr,
                   double l2, double* leaf_values, double* support_values, hipStream_t s) {
    OrdArgs a = ord_args(ctx, ord, p);
    a.lr = lr;
    a.l2 = l2;
    a.keep = leaf_values != nullptr;
    // sums blocks per segment (none for the kept model when it is not updated)
    a.blk_off[0] = 0;
    for (int sg = 0; sg <= a.M; ++sg) {
        const int64_t cnt = sg == 0 ? (a.keep ? a.n : 0) : ord_learn(sg - 1);
        a.blk_off[sg + 1] = a.blk_off[sg] + (cnt + kOrdChunk - 1) / kOrdChunk;
    }
    const int64_t blocks = a.blk_off[a.M + 1];
    const int64_t lpos_b = align_up(a.n * 2, 256), ypos_b = align_up(a.n * 4, 256);
    const int64_t part_b = align_up(blocks * a.cells * 2 * 8, 256);
    const int64_t vals_b = align_up(int64_t(a.M + 1) * a.cells * 8, 256);
    int rc = ensure_ws(ctx, lpos_b + ypos_b + part_b + vals_b, s);
    if (rc) return rc;
    char* ws = (char*)ctx->ws;
    a.lpos = (uint16_t*)ws;
    a.ypos = (float*)(ws + lpos_b);
    a.part = (double*)(ws + lpos_b + ypos_b);
    a.vals = (double*)(ws + lpos_b + ypos_b + part_b);
    const int64_t words = int64_t(a.cells) * 2 * 8;
    a.copies = words * 4 <= kOrdWaveLds ? 4 : 1;
    ord_gather_kernel<<<ord_grid(ctx, a.n), kOrdThreads, 0, s>>>(a);
    CBH_LAUNCHED();
    if (blocks > 0) {
        launch_by_loss<SumsK>(p->loss, dim3((unsigned)blocks), dim3(kOrdThreads),
                              (size_t)(a.copies * words), s, a);
        CBH_LAUNCHED();
    }
    const int64_t waves = int64_t(a.M + 1) * a.cells;
    ord_solve_kernel<<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(a, leaf_values, support_values);
    CBH_LAUNCHED();
    launch_by_loss<ApplyK>(p->loss, dim3(ord_grid(ctx, (a.keep ? a.n : 0) + a.S)), dim3(256), 0,
                           s, a);
    CBH_LAUNCHED();
    return CBH_OK;
}

}  // namespace cbh

using namespace cbh;

extern "C" {

int32_t cbh_ordered_models(int64_t n) { return n < 1 ? 0 : ord_models(n); }

int64_t cbh_ordered_offset(int64_t n, int32_t m) {
    if (n < 1 || m < 0 || m > ord_models(n)) return -1;
    return ord_offset(n, m);
}

int64_t cbh_ordered_support_size(int64_t n) {
    return n < 1 ? 0 : ord_offset(n, ord_models(n));
}

int cbh_ordered_gradients(cbh_ctx* ctx, const cbh_ordered* ord, const cbh_problem* prob,
                          void* stream) {
    clear_error();
    int rc = validate_ordered(ctx, ord, prob);
    if (rc) return rc;
    const OrdArgs a = ord_args(ctx, ord, prob);
    launch_by_loss<GradK>(prob->loss, dim3(ord_grid(ctx, a.n)), dim3(256), 0,
                          (hipStream_t)stream, a);
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_ordered_update(cbh_ctx* ctx, const cbh_ordered* ord, const cbh_problem* prob,
                       double lr, double l2, double* leaf_values, double* support_values,
                       void* stream) {
    clear_error();
    int rc = validate_ordered(ctx, ord, prob);
    if (rc) return rc;
    CBH_ARG(std::isfinite(lr) && l2 >= 0 && std::isfinite(l2), "lr / l2 out of range");
    return ordered_update(ctx, ord, prob, lr, l2, leaf_values, support_values,
                          (hipStream_t)stream);
}

}  // extern "C"
