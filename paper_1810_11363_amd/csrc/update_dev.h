// Leaf solve and approx update of one tree (the second phase of a tree,
// Sec. 3: leaf values -G / (H + l2) from the last level's histogram at the
// chosen split, then approx += lr * value and the loss derivatives at the new
// approx), as device functions for the single-problem and the batched kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace cbh {

struct SolveArgs {
    const void* hist;
    const cbh_split* split;
    const float* grad_scale;
    double* values;
    int32_t depth, F, B, K, rmse, precision;
    double l2;
};

// Leaf value of (final leaf, class) t = Lf * K + c by one wave: lanes sum the
// bins of the chosen side in double, then a wave reduction in a fixed order;
// lane 0 writes -G / (H + l2).
__device__ __forceinline__ void leaf_solve_one(const SolveArgs& a, int64_t t, int lane) {
    const int64_t leaves = int64_t(1) << a.depth;
    const int64_t Lf = t / a.K;
    const int c = (int)(t % a.K);
    const int64_t half = leaves >> 1;
    const int64_t L = Lf & (half - 1);
    const bool right = (Lf & half) != 0;
    int f = a.split->feature;
    int k = a.split->border;
    if (f < 0 || f >= a.F) {  // no split: every row stayed left
        f = 0;
        k = a.B - 1;
    }
    const int b_lo = right ? k + 1 : 0;
    const int b_hi = right ? a.B : k + 1;
    const int64_t cell0 = (L * a.F + f) * a.B;
    double G = 0.0, H = 0.0;
    for (int b = b_lo + lane; b < b_hi; b += 64) {
        const int64_t e = (cell0 + b) * 2 * a.K + 2 * c;
        if (a.precision == CBH_PREC_FP32) {
            G += (double)reinterpret_cast<const float*>(a.hist)[e];
            H += a.rmse ? (double)reinterpret_cast<const uint32_t*>(a.hist)[e + 1]
                        : (double)reinterpret_cast<const float*>(a.hist)[e + 1];
        } else if (a.precision == CBH_PREC_TWOFLOAT) {
            const float2 gg = reinterpret_cast<const float2*>(a.hist)[e];
            const float2 hh = reinterpret_cast<const float2*>(a.hist)[e + 1];
            G += (double)gg.x + (double)gg.y;
            H += a.rmse ? (double)__float_as_uint(hh.x) : (double)hh.x + (double)hh.y;
        } else {
            G += (double)reinterpret_cast<const int64_t*>(a.hist)[e];
            H += (double)reinterpret_cast<const int64_t*>(a.hist)[e + 1];
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        G += __shfl_xor(G, d, 64);
        H += __shfl_xor(H, d, 64);
    }
    if (lane != 0) return;
    if (a.precision == CBH_PREC_INT16) {
        G *= (double)a.grad_scale[2 * c];
        if (!a.rmse) H *= (double)a.grad_scale[2 * c + 1];
    }
    const double d = H + a.l2;
    a.values[Lf * a.K + c] = d == 0.0 ? 0.0 : -G / d;
}

struct UpdArgs {
    const uint16_t* leaf;
    const double* values;
    const float* label;
    const float* weight;      // row weights or NULL
    double* approx;
    float* g;
    float* h;
    int64_t n;
    int32_t K, loss, add;
    uint16_t lmask;
    double lr;
};

// Row i: approx += lr * value of its final leaf (when add), then the loss
// derivatives at the new approx.
template <int LOSS>
__device__ __forceinline__ void update_row(const UpdArgs& a, int64_t i) {
    const int K = a.K;
    const double y = (double)a.label[i];
    const int64_t Lf = a.add ? (a.leaf[i] & a.lmask) : 0;
    // with row weights the loss of row i counts w times: so do g and h
    // (RMSE: h = w, the second statistic becomes the sum of weights)
    const double w = a.weight ? (double)a.weight[i] : 1.0;
    if constexpr (LOSS != CBH_LOSS_MULTICLASS) {
        double ap = a.approx[i];
        if (a.add) {
            ap = ap + a.lr * a.values[Lf];
            a.approx[i] = ap;
        }
        if constexpr (LOSS == CBH_LOSS_RMSE) {
            if (a.weight) {
                a.g[i] = (float)(w * (ap - y));
                a.h[i] = (float)w;
            } else {
                a.g[i] = (float)(ap - y);
            }
        } else {
            const double p = 1.0 / (1.0 + exp(-ap));
            if (a.weight) {
                a.g[i] = (float)(w * (p - y));
                a.h[i] = (float)(w * (p * (1.0 - p)));
            } else {
                a.g[i] = (float)(p - y);
                a.h[i] = (float)(p * (1.0 - p));
            }
        }
    } else {
        // the K approx values loaded before any store (unrolled to the
        // largest K, so the values stay in registers)
        double av[CBH_MAX_K];
#pragma unroll
        for (int c = 0; c < CBH_MAX_K; ++c) av[c] = c < K ? a.approx[int64_t(c) * a.n + i] : 0.0;
        double mx = -INFINITY;
#pragma unroll
        for (int c = 0; c < CBH_MAX_K; ++c) {
            if (c >= K) continue;
            if (a.add) {
                av[c] = av[c] + a.lr * a.values[Lf * K + c];
                a.approx[int64_t(c) * a.n + i] = av[c];
            }
            mx = av[c] > mx ? av[c] : mx;
        }
        double z = 0.0;
#pragma unroll
        for (int c = 0; c < CBH_MAX_K; ++c)
            if (c < K) z += exp(av[c] - mx);
        const int yc = (int)y;
#pragma unroll
        for (int c = 0; c < CBH_MAX_K; ++c) {
            if (c >= K) continue;
            const double p = exp(av[c] - mx) / z;
            const double gc = p - (c == yc ? 1.0 : 0.0), hc = p * (1.0 - p);
            a.g[int64_t(c) * a.n + i] = (float)(a.weight ? w * gc : gc);
            a.h[int64_t(c) * a.n + i] = (float)(a.weight ? w * hc : hc);
        }
    }
}

}  // namespace cbh
