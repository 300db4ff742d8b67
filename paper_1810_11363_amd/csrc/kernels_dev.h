// Device building blocks shared by the single-problem launches and the
// batched launches: the LDS histogram tile, the partial-tile merge and the
// per-feature split scoring.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "cbhip.h"

namespace cbh {

// ------------------------------------------------------------ histogram tile
// One block accumulates rows [r0, r1) of features [f0, f0 + nf) for leaves
// [l0, l0 + lt) into an LDS tile [lt][fb][B][wpc words], then writes the tile
// into `part`, the chunk's partial histogram laid out as [L][F][B][wpc].
struct TileArgs {
    const uint8_t* const* bins;
    const float* g;
    const float* h;
    const uint32_t* gq;
    const uint16_t* leaf;
    uint32_t* part;
    int64_t n, r0, r1;
    int32_t F, B, K, L;
    int32_t fb, lt, wpc, rmse;
    int32_t f0, nf;
    uint32_t l0;
};

template <int PREC>
__device__ __forceinline__ void add_row(uint32_t* lds, uint32_t w, int c, float gv, float hv,
                                        uint32_t qv, bool rmse) {
    if constexpr (PREC == CBH_PREC_FP32) {
        __hip_atomic_fetch_add((float*)&lds[w + 2 * c], gv, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        if (rmse)
            __hip_atomic_fetch_add(&lds[w + 2 * c + 1], 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            __hip_atomic_fetch_add((float*)&lds[w + 2 * c + 1], hv, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    } else if constexpr (PREC == CBH_PREC_TWOFLOAT) {
        // TwoSum on the value the atomic returned: fl(old + v) is what the LDS
        // now holds, err is the exact rounding error of that addition, and the
        // "lo" word collects the errors, so hi + lo tracks the exact sum.
        const float old = __hip_atomic_fetch_add((float*)&lds[w + 4 * c], gv, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        const float s = old + gv;
        const float bp = s - old;
        const float err = (old - (s - bp)) + (gv - bp);
        if (err != 0.0f)
            __hip_atomic_fetch_add((float*)&lds[w + 4 * c + 1], err, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        if (rmse) {
            __hip_atomic_fetch_add(&lds[w + 4 * c + 2], 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            const float oh = __hip_atomic_fetch_add((float*)&lds[w + 4 * c + 2], hv,
                                                    __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_WORKGROUP);
            const float sh = oh + hv;
            const float bh = sh - oh;
            const float eh = (oh - (sh - bh)) + (hv - bh);
            if (eh != 0.0f)
                __hip_atomic_fetch_add((float*)&lds[w + 4 * c + 3], eh, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    } else {
        // (g code << 32) + h code: with <= 65536 rows per tile neither half
        // overflows, so one 64-bit LDS add updates both sums exactly.
        const int64_t gcode = (int16_t)(qv & 0xffffu);
        const uint64_t hcode = (qv >> 16) & 0x7fffu;
        const uint64_t packed = ((uint64_t)gcode << 32) + hcode;
        __hip_atomic_fetch_add((unsigned long long*)&lds[w + 2 * c], (unsigned long long)packed,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

template <int PREC, int KT>
__device__ __forceinline__ void hist_tile(const TileArgs& a, uint32_t* lds) {
    const int K = KT > 0 ? KT : a.K;
    const uint32_t lmask = (uint32_t)a.L - 1u;
    const uint32_t ltn = (uint32_t)a.lt;
    const uint32_t Bm1 = (uint32_t)a.B - 1u;
    const int wpc = a.wpc;
    const int tile_words = a.lt * a.fb * a.B * wpc;
    for (int i = threadIdx.x; i < tile_words; i += blockDim.x) lds[i] = 0u;
    __syncthreads();
    const bool rmse = a.rmse != 0;
    const bool vec = (a.n & 3) == 0 || K == 1;
    const int64_t ngroups = (a.r1 - a.r0) >> 2;
    for (int64_t q = threadIdx.x; q < ngroups; q += blockDim.x) {
        const int64_t i = a.r0 + 4 * q;
        const uint2 lf = a.L == 1 ? make_uint2(0u, 0u)
                                  : *reinterpret_cast<const uint2*>(a.leaf + i);
        uint32_t lv[4] = {lf.x & 0xffffu, lf.x >> 16, lf.y & 0xffffu, lf.y >> 16};
#pragma unroll
        for (int r = 0; r < 4; ++r) lv[r] = (lv[r] & lmask) - a.l0;  // >= lt: not in tile
        for (int c = 0; c < K; ++c) {
            float gv[4] = {0.f, 0.f, 0.f, 0.f}, hv[4] = {1.f, 1.f, 1.f, 1.f};
            uint32_t qv[4] = {0u, 0u, 0u, 0u};
            const int64_t ci = int64_t(c) * a.n + i;
            if constexpr (PREC == CBH_PREC_INT16) {
                if (vec) {
                    const uint4 t = *reinterpret_cast<const uint4*>(a.gq + ci);
                    qv[0] = t.x; qv[1] = t.y; qv[2] = t.z; qv[3] = t.w;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) qv[r] = a.gq[ci + r];
                }
            } else {
                if (vec) {
                    const float4 t = *reinterpret_cast<const float4*>(a.g + ci);
                    gv[0] = t.x; gv[1] = t.y; gv[2] = t.z; gv[3] = t.w;
                    if (!rmse) {
                        const float4 u = *reinterpret_cast<const float4*>(a.h + ci);
                        hv[0] = u.x; hv[1] = u.y; hv[2] = u.z; hv[3] = u.w;
                    }
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        gv[r] = a.g[ci + r];
                        if (!rmse) hv[r] = a.h[ci + r];
                    }
                }
            }
            for (int j = 0; j < a.nf; ++j) {
                const uint32_t b4 = *reinterpret_cast<const uint32_t*>(a.bins[a.f0 + j] + i);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (lv[r] < ltn) {
                        const uint32_t bin = min((b4 >> (8 * r)) & 255u, Bm1);
                        const uint32_t w = ((lv[r] * a.fb + j) * a.B + bin) * wpc;
                        add_row<PREC>(lds, w, c, gv[r], hv[r], qv[r], rmse);
                    }
                }
            }
        }
    }
    // rows of the chunk after the last full group of 4
    const int64_t tail0 = a.r0 + 4 * ngroups;
    if (threadIdx.x < a.r1 - tail0) {
        const int64_t i = tail0 + threadIdx.x;
        const uint32_t l = ((a.L == 1 ? 0u : (uint32_t)a.leaf[i]) & lmask) - a.l0;
        if (l < ltn) {
            for (int c = 0; c < K; ++c) {
                const int64_t ci = int64_t(c) * a.n + i;
                float gv = 0.f, hv = 1.f;
                uint32_t qv = 0u;
                if constexpr (PREC == CBH_PREC_INT16) {
                    qv = a.gq[ci];
                } else {
                    gv = a.g[ci];
                    if (!rmse) hv = a.h[ci];
                }
                for (int j = 0; j < a.nf; ++j) {
                    const uint32_t bin = min((uint32_t)a.bins[a.f0 + j][i], Bm1);
                    const uint32_t w = ((l * a.fb + j) * a.B + bin) * wpc;
                    add_row<PREC>(lds, w, c, gv, hv, qv, rmse);
                }
            }
        }
    }
    __syncthreads();
    const int row_words = a.B * wpc;
    for (int idx = threadIdx.x; idx < tile_words; idx += blockDim.x) {
        const int s = idx % row_words;
        const int rest = idx / row_words;
        const int j = rest % a.fb;
        const int ll = rest / a.fb;
        if (j < a.nf)
            a.part[((int64_t)(a.l0 + ll) * a.F + (a.f0 + j)) * row_words + s] = lds[idx];
    }
}

// ------------------------------------------------------------ partial merge
// Merge cell `cell` (all 2K statistics) over n_chunks partial histograms of
// `cells` cells each, in chunk order, into the output layout of the precision.
template <int PREC>
__device__ __forceinline__ void merge_cell(const uint32_t* __restrict__ part, int64_t cells,
                                           int K, int n_chunks, bool rmse, void* __restrict__ out,
                                           int64_t cell) {
    const int wpc = PREC == CBH_PREC_TWOFLOAT ? 4 * K : 2 * K;
    const int64_t cw = cells * wpc;
    for (int c = 0; c < K; ++c) {
        if constexpr (PREC == CBH_PREC_FP32) {
            const int64_t j = cell * wpc + 2 * c;
            float g = 0.f;
            for (int ch = 0; ch < n_chunks; ++ch) g += __uint_as_float(part[ch * cw + j]);
            reinterpret_cast<float*>(out)[j] = g;
            if (rmse) {
                uint32_t cnt = 0;
                for (int ch = 0; ch < n_chunks; ++ch) cnt += part[ch * cw + j + 1];
                reinterpret_cast<uint32_t*>(out)[j + 1] = cnt;
            } else {
                float hh = 0.f;
                for (int ch = 0; ch < n_chunks; ++ch) hh += __uint_as_float(part[ch * cw + j + 1]);
                reinterpret_cast<float*>(out)[j + 1] = hh;
            }
        } else if constexpr (PREC == CBH_PREC_TWOFLOAT) {
            for (int st = 0; st < 2; ++st) {
                const int64_t j = cell * wpc + 4 * c + 2 * st;
                float2 r;
                if (st == 1 && rmse) {
                    uint32_t cnt = 0;
                    for (int ch = 0; ch < n_chunks; ++ch) cnt += part[ch * cw + j];
                    r = make_float2(__uint_as_float(cnt), 0.f);
                } else {
                    float S = 0.f, E = 0.f;
                    for (int ch = 0; ch < n_chunks; ++ch) {
                        const float hi = __uint_as_float(part[ch * cw + j]);
                        const float lo = __uint_as_float(part[ch * cw + j + 1]);
                        const float t = S + hi;
                        const float bp = t - S;
                        const float e = (S - (t - bp)) + (hi - bp);
                        S = t;
                        E += e + lo;
                    }
                    const float hs = S + E;
                    r = make_float2(hs, E - (hs - S));
                }
                reinterpret_cast<float2*>(out)[cell * 2 * K + 2 * c + st] = r;
            }
        } else {
            const uint64_t* P64 = reinterpret_cast<const uint64_t*>(part);
            const int64_t slot = cell * K + c;
            int64_t gs = 0, hs = 0;
            for (int ch = 0; ch < n_chunks; ++ch) {
                const uint64_t v = P64[ch * (cw / 2) + slot];
                hs += (int64_t)(uint32_t)(v & 0xffffffffull);
                gs += (int64_t)(int32_t)(uint32_t)(v >> 32);
            }
            reinterpret_cast<int64_t*>(out)[2 * slot] = gs;
            reinterpret_cast<int64_t*>(out)[2 * slot + 1] = hs;
        }
    }
}

// ---------------------------------------------------------------- scoring
struct FeatBest {
    float s1;     // best score of the feature
    int32_t k1;   // its border (-1: no candidate)
    float s2;     // best score of any other border of the feature
    int32_t pad;
};

__device__ __forceinline__ float side_term(float G, float H, float l2) {
    const float d = H + l2;
    return d == 0.0f ? 0.0f : (G * G) / d;
}

// top-2 merge: larger score wins, ties go to the smaller index
__device__ __forceinline__ void top2_merge(float& s1, int& i1, float& s2, float t1, int j1,
                                           float t2) {
    const bool take = (j1 >= 0) && (i1 < 0 || t1 > s1 || (t1 == s1 && j1 < i1));
    if (take) {
        s2 = fmaxf(fmaxf(s2, t2), i1 >= 0 ? s1 : -INFINITY);
        s1 = t1;
        i1 = j1;
    } else {
        s2 = fmaxf(fmaxf(s2, t2), j1 >= 0 ? t1 : -INFINITY);
    }
}

struct F2 {
    float hi, lo;
};
__device__ __forceinline__ F2 f2_add(F2 a, F2 b) {
    const float s = a.hi + b.hi;
    const float bp = s - a.hi;
    const float e = (a.hi - (s - bp)) + (b.hi - bp) + a.lo + b.lo;
    const float hi = s + e;
    return F2{hi, e - (hi - s)};
}
__device__ __forceinline__ F2 f2_neg(F2 a) { return F2{-a.hi, -a.lo}; }

struct ScoreRow {
    const void* hist;
    const float* grad_scale;
    int32_t F, B, K, rmse;
    float l2;
};

// Terms of one histogram row (leaf L, feature f, class c) for the 4 borders
// 4*lane .. 4*lane+3, added into acc. Prefix sums over bins are formed in the
// accumulator type of the precision (float, two-float or exact int64).
template <int PREC>
__device__ void row_terms(const ScoreRow& a, int L, int f, int c, int lane, int kmax,
                          float acc[4]) {
    const int64_t cell0 = (int64_t(L) * a.F + f) * a.B;
    const int b0 = 4 * lane;
    if constexpr (PREC == CBH_PREC_FP32) {
        const float* hs = reinterpret_cast<const float*>(a.hist);
        const uint32_t* hu = reinterpret_cast<const uint32_t*>(a.hist);
        float G[4], H[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = b0 + j;
            G[j] = 0.f;
            H[j] = 0.f;
            if (b < a.B) {
                const int64_t e = (cell0 + b) * 2 * a.K + 2 * c;
                G[j] = hs[e];
                H[j] = a.rmse ? (float)hu[e + 1] : hs[e + 1];
            }
        }
#pragma unroll
        for (int j = 1; j < 4; ++j) {
            G[j] += G[j - 1];
            H[j] += H[j - 1];
        }
        float g = G[3], h = H[3];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const float gu = __shfl_up(g, d, 64), hu2 = __shfl_up(h, d, 64);
            if (lane >= d) {
                g += gu;
                h += hu2;
            }
        }
        const float gt = __shfl(g, 63, 64), ht = __shfl(h, 63, 64);
        const float ge = g - G[3], he = h - H[3];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (b0 + j < kmax) {
                const float gl = ge + G[j], hl = he + H[j];
                acc[j] += side_term(gl, hl, a.l2) + side_term(gt - gl, ht - hl, a.l2);
            }
        }
    } else if constexpr (PREC == CBH_PREC_TWOFLOAT) {
        const float2* hs = reinterpret_cast<const float2*>(a.hist);
        F2 G[4], H[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = b0 + j;
            G[j] = F2{0.f, 0.f};
            H[j] = F2{0.f, 0.f};
            if (b < a.B) {
                const int64_t e = (cell0 + b) * 2 * a.K + 2 * c;
                const float2 gg = hs[e];
                const float2 hh = hs[e + 1];
                G[j] = F2{gg.x, gg.y};
                H[j] = a.rmse ? F2{(float)__float_as_uint(hh.x), 0.f} : F2{hh.x, hh.y};
            }
        }
#pragma unroll
        for (int j = 1; j < 4; ++j) {
            G[j] = f2_add(G[j], G[j - 1]);
            H[j] = f2_add(H[j], H[j - 1]);
        }
        F2 g = G[3], h = H[3];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const F2 gu{__shfl_up(g.hi, d, 64), __shfl_up(g.lo, d, 64)};
            const F2 hu2{__shfl_up(h.hi, d, 64), __shfl_up(h.lo, d, 64)};
            if (lane >= d) {
                g = f2_add(gu, g);
                h = f2_add(hu2, h);
            }
        }
        const F2 gt{__shfl(g.hi, 63, 64), __shfl(g.lo, 63, 64)};
        const F2 ht{__shfl(h.hi, 63, 64), __shfl(h.lo, 63, 64)};
        const F2 ge = f2_add(g, f2_neg(G[3])), he = f2_add(h, f2_neg(H[3]));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (b0 + j < kmax) {
                const F2 gl = f2_add(ge, G[j]), hl = f2_add(he, H[j]);
                const F2 gr = f2_add(gt, f2_neg(gl)), hr = f2_add(ht, f2_neg(hl));
                acc[j] += side_term(gl.hi + gl.lo, hl.hi + hl.lo, a.l2) +
                          side_term(gr.hi + gr.lo, hr.hi + hr.lo, a.l2);
            }
        }
    } else {
        const int64_t* hs = reinterpret_cast<const int64_t*>(a.hist);
        const double sg = (double)a.grad_scale[2 * c];
        const double sh = a.rmse ? 1.0 : (double)a.grad_scale[2 * c + 1];
        int64_t G[4], H[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = b0 + j;
            G[j] = 0;
            H[j] = 0;
            if (b < a.B) {
                const int64_t e = (cell0 + b) * 2 * a.K + 2 * c;
                G[j] = hs[e];
                H[j] = hs[e + 1];
            }
        }
#pragma unroll
        for (int j = 1; j < 4; ++j) {
            G[j] += G[j - 1];
            H[j] += H[j - 1];
        }
        int64_t g = G[3], h = H[3];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t gu = __shfl_up(g, d, 64), hu2 = __shfl_up(h, d, 64);
            if (lane >= d) {
                g += gu;
                h += hu2;
            }
        }
        const int64_t gt = __shfl(g, 63, 64), ht = __shfl(h, 63, 64);
        const int64_t ge = g - G[3], he = h - H[3];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (b0 + j < kmax) {
                const int64_t gl = ge + G[j], hl = he + H[j];
                const float fgl = (float)((double)gl * sg), fhl = (float)((double)hl * sh);
                const float fgr = (float)((double)(gt - gl) * sg);
                const float fhr = (float)((double)(ht - hl) * sh);
                acc[j] += side_term(fgl, fhl, a.l2) + side_term(fgr, fhr, a.l2);
            }
        }
    }
}

// Whole-block scoring of feature f over all leaves and classes; writes the
// per-border scores (optional) and the feature's best/second-best. Needs a
// block of 256 threads.
template <int PREC>
__device__ void score_feature(const ScoreRow& a, int L, int f, int n_bins_f, float* scores,
                              FeatBest* out) {
    __shared__ float part[4][256];
    __shared__ float rs1[4], rs2[4];
    __shared__ int ri1[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kmax = min(n_bins_f, a.B) - 1;  // candidates k < kmax
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (kmax > 0) {
        const int items = L * a.K;
        for (int it = wave; it < items; it += 4) row_terms<PREC>(a, it / a.K, f, it % a.K, lane,
                                                                  kmax, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) part[wave][4 * lane + j] = acc[j];
    __syncthreads();
    const int k = threadIdx.x;  // thread k owns border k
    float s = -INFINITY;
    if (k < kmax) {
        s = part[0][k] + part[1][k];
        s += part[2][k];
        s += part[3][k];
        if (s != s) s = -INFINITY;
    }
    if (scores && k < a.B - 1) scores[int64_t(f) * (a.B - 1) + k] = s;
    float s1 = s, s2 = -INFINITY;
    int i1 = k < kmax ? k : -1;
    if (i1 < 0) s1 = -INFINITY;
    for (int d = 32; d >= 1; d >>= 1) {
        const float t1 = __shfl_xor(s1, d, 64), t2 = __shfl_xor(s2, d, 64);
        const int j1 = __shfl_xor(i1, d, 64);
        top2_merge(s1, i1, s2, t1, j1, t2);
    }
    if (lane == 0) {
        rs1[wave] = s1;
        rs2[wave] = s2;
        ri1[wave] = i1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float b1 = rs1[0], b2 = rs2[0];
        int j = ri1[0];
        for (int w = 1; w < 4; ++w) top2_merge(b1, j, b2, rs1[w], ri1[w], rs2[w]);
        *out = FeatBest{b1, j, b2, 0};
    }
}

// Reduce F per-feature winners (block of 256) to the level's split.
__device__ inline void argmax_features(const FeatBest* __restrict__ fb, int F, int Bm1,
                                       cbh_split* __restrict__ out) {
    float s1 = -INFINITY, s2 = -INFINITY;
    int i1 = -1;
    for (int f = threadIdx.x; f < F; f += 256) {
        const FeatBest e = fb[f];
        top2_merge(s1, i1, s2, e.s1, e.k1 >= 0 ? f * Bm1 + e.k1 : -1, e.s2);
    }
    __shared__ float rs1[4], rs2[4];
    __shared__ int ri1[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = 32; d >= 1; d >>= 1) {
        const float t1 = __shfl_xor(s1, d, 64), t2 = __shfl_xor(s2, d, 64);
        const int j1 = __shfl_xor(i1, d, 64);
        top2_merge(s1, i1, s2, t1, j1, t2);
    }
    if (lane == 0) {
        rs1[wave] = s1;
        rs2[wave] = s2;
        ri1[wave] = i1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float b1 = rs1[0], b2 = rs2[0];
        int j = ri1[0];
        for (int w = 1; w < 4; ++w) top2_merge(b1, j, b2, rs1[w], ri1[w], rs2[w]);
        cbh_split r;
        if (j < 0) {
            r.feature = -1;
            r.border = -1;
            r.score = 0.f;
            r.margin = 0.f;
        } else {
            r.feature = j / Bm1;
            r.border = j % Bm1;
            r.score = b1;
            r.margin = (b2 == -INFINITY) ? INFINITY : b1 - b2;
        }
        *out = r;
    }
}

// leaf |= [bin > k] << level for rows [i0, i1) (level 0 overwrites); a
// missing split (f < 0) leaves the bit clear.
__device__ __forceinline__ void apply_rows(const uint8_t* const* bins, int F, cbh_split sp,
                                           uint16_t* leaf, int64_t i0, int64_t i1, int level) {
    int f = sp.feature, k = sp.border;
    if (f < 0 || f >= F) {
        if (level != 0) return;
        f = 0;
        k = 255;
    }
    const uint8_t* col = bins[f];
    const uint32_t bit = 1u << level;
    for (int64_t i = i0; i < i1; ++i) {
        const uint32_t old = level == 0 ? 0u : leaf[i];
        leaf[i] = (uint16_t)(old | (((int)col[i] > k) ? bit : 0u));
    }
}

}  // namespace cbh
