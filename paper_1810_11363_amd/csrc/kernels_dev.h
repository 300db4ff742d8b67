// Device building blocks shared by the single-problem launches and the
// batched launches: the LDS histogram tile, the partial-tile merge and the
// per-feature split scoring.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "cbhip.h"

namespace cbh {

// ------------------------------------------------------------ global loads
// Loads through pointers the compiler cannot place in global memory (bin
// columns reached through a pointer table, fields of device-resident problem
// descriptors) otherwise become flat loads. A flat load counts against both
// the vector-memory and the LDS counters, so every later wait has to drain
// both: a load issued early for the next segment then blocks the LDS updates
// of the current one. These helpers load through the global address space.
typedef unsigned int gv4u __attribute__((ext_vector_type(4)));
typedef unsigned int gv2u __attribute__((ext_vector_type(2)));
typedef float gv4f __attribute__((ext_vector_type(4)));
#define CBH_GLOBAL(T) const __attribute__((address_space(1))) T*
__device__ __forceinline__ uint4 gld_u4(const void* p) {
    const gv4u v = *(CBH_GLOBAL(gv4u))(p);
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint2 gld_u2(const void* p) {
    const gv2u v = *(CBH_GLOBAL(gv2u))(p);
    return make_uint2(v.x, v.y);
}
__device__ __forceinline__ float4 gld_f4(const void* p) {
    const gv4f v = *(CBH_GLOBAL(gv4f))(p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ uint32_t gld_u32(const void* p) { return *(CBH_GLOBAL(uint32_t))(p); }
__device__ __forceinline__ uint32_t gld_u16(const void* p) { return *(CBH_GLOBAL(uint16_t))(p); }
__device__ __forceinline__ uint32_t gld_u8(const void* p) { return *(CBH_GLOBAL(uint8_t))(p); }
__device__ __forceinline__ float gld_f32(const void* p) { return *(CBH_GLOBAL(float))(p); }
#undef CBH_GLOBAL

// ------------------------------------------------- precision forms
// Output format of a precision: the float64-accumulated form writes the same
// (hi, lo) float pairs as the compensated form, so every step after the
// histogram (merge, subtraction, score, leaf solve) takes it as TWOFLOAT.
__host__ __device__ constexpr int out_prec(int p) {
    return p == CBH_PREC_F64 ? CBH_PREC_TWOFLOAT : p;
}

// Float32 accumulation in LDS. The LDS float32 atomic add of gfx950 is not
// pipelined (measured 0.33 updates per clock per CU, with or without
// denormal flushing, against 7.6 for the float64 add and 14.8 for the u32
// add), so the float32 forms update a cell by compare-and-swap: read it, add
// in float32 (FP32) or by TwoSum into a (hi, lo) pair (TWOFLOAT), and swap
// the new bits in if the cell still holds the bits that were read; otherwise
// the add is redone on the value found. Every addition is then one float32
// addition (or one TwoSum) in some order, as with an atomic add.
__device__ __forceinline__ uint32_t lds_cas32(uint32_t* p, uint32_t cmp, uint32_t val) {
    __hip_atomic_compare_exchange_strong(p, &cmp, val, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    return cmp;   // the bits found: equal to the bits compared iff the swap happened
}
__device__ __forceinline__ uint64_t lds_cas64(uint64_t* p, uint64_t cmp, uint64_t val) {
    __hip_atomic_compare_exchange_strong(p, &cmp, val, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
    return cmp;
}
__device__ __forceinline__ uint32_t lds_load32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t lds_load64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint64_t pack_f2(float lo_word, float hi_word) {
    return (uint64_t)__float_as_uint(lo_word) | ((uint64_t)__float_as_uint(hi_word) << 32);
}
// float32 add of x to the float in the word's low half and y to the high half
__device__ __forceinline__ uint64_t add_pair_word(uint64_t w, float x, float y) {
    return pack_f2(__uint_as_float((uint32_t)w) + x, __uint_as_float((uint32_t)(w >> 32)) + y);
}
// TwoSum of x into the pair (hi = low half, lo = high half): hi + x = s + e
// exactly (Knuth's TwoSum; needs round-to-nearest and no contraction), and e
// is added to lo in float32.
__device__ __forceinline__ uint64_t twosum_word(uint64_t w, float x) {
    const float hi = __uint_as_float((uint32_t)w), lo = __uint_as_float((uint32_t)(w >> 32));
    const float s = hi + x, bp = s - hi;
    const float e = (hi - (s - bp)) + (x - bp);
    return pack_f2(s, lo + e);
}
// (hi, lo) with hi the float nearest to hi + lo (TwoSum renormalisation)
__device__ __forceinline__ float2 renorm_pair(float hi, float lo) {
    const float s = hi + lo, bp = s - hi;
    return make_float2(s, (hi - (s - bp)) + (lo - bp));
}
// Pair additions by compare-and-swap, one cell: retried until the swap holds.
__device__ __forceinline__ void cas_add_f32(uint32_t* p, float x) {
    uint32_t old = lds_load32(p);
    for (;;) {
        const uint32_t got = lds_cas32(p, old, __float_as_uint(__uint_as_float(old) + x));
        if (got == old) break;
        old = got;
    }
}
__device__ __forceinline__ void cas_twosum(uint64_t* p, float x) {
    uint64_t old = lds_load64(p);
    for (;;) {
        const uint64_t got = lds_cas64(p, old, twosum_word(old, x));
        if (got == old) break;
        old = got;
    }
}

// ------------------------------------------------------------ histogram tile
// One block accumulates rows [r0, r1) of features [f0, f0 + nf) for leaves
// [l0, l0 + lt) into an LDS tile, then writes the tile into `part`, the
// chunk's partial histogram laid out as [L][F][B][wpc words] in the output
// format of the precision.
//
// The tile has 8-byte elements for every form: F64 accumulates with the
// float64 LDS atomic, FP32 keeps a float in the element's low half (updated by
// compare-and-swap), TWOFLOAT a (hi, lo) float pair (TwoSum by 64-bit
// compare-and-swap); counts use u32 atomics and the int16 form one u64 atomic
// of packed codes. A "cell" is one (leaf, feature) pair of the tile,
// cell = leaf_in_tile * fb + feature_in_block.
//   float forms, K classes, h statistic:   8 B [cells][K][2][B]
//   float forms, RMSE (K = 1, count):      8 B [cells][B], then u32 [cells][B]
//   INT16:                                 u64 [cells][K][B]
// Each thread streams 8 or 16 consecutive rows per step: one 8- or 16-byte
// load of bins per feature (a wave reads 512 B or 1 KB contiguous per
// feature), and loads for 4 features are issued before their LDS updates so
// that memory latency overlaps.
// Bin of row i of a feature whose 16-row segments start `stride` bytes apart
// (16 for a plain column).
__device__ __forceinline__ const uint8_t* seg_ptr(const uint8_t* base, int64_t stride,
                                                   int64_t i) {
    return base + (i >> 4) * stride + (i & 15);
}
// Packed bins (cbh_problem.bin_bits 4 or 1; Sec. 5 stores features of at most
// 15 bins in 4 bits and binary ones in 1 bit): a 16-row segment of a feature
// is 2 * BITS bytes. 4 bits: 32-bit word k (k = 0, 1) of the segment holds
// rows 8k..8k+3 in the low nibbles of its bytes 0..3 and rows 8k+4..8k+7 in
// the high nibbles, so two masks give four rows per byte lane; 1 bit: bit r
// of the segment's little-endian 16-bit word is row r.
template <int BITS>
constexpr int seg_bytes() { return 2 * BITS; }

// 4 bits x -> bytes 0..3 holding bit 0..3 of x (x < 16: the four shifted
// copies x, x << 7, x << 14, x << 21 do not overlap)
__device__ __forceinline__ uint32_t spread4(uint32_t x) {
    return __umul24(x, 0x204081u) & 0x01010101u;
}

// The 16 bins of the segment at p, row r in byte r.
template <int BITS>
__device__ __forceinline__ uint4 load_seg16(const uint8_t* p) {
    if constexpr (BITS == 8) {
        return gld_u4(p);
    } else if constexpr (BITS == 4) {
        const uint2 w = gld_u2(p);
        return make_uint4(w.x & 0x0f0f0f0fu, (w.x >> 4) & 0x0f0f0f0fu, w.y & 0x0f0f0f0fu,
                          (w.y >> 4) & 0x0f0f0f0fu);
    } else {
        const uint32_t b = gld_u16(p);
        return make_uint4(spread4(b & 15u), spread4((b >> 4) & 15u), spread4((b >> 8) & 15u),
                          spread4((b >> 12) & 15u));
    }
}

// Bin of row r (0..15) of the segment at p.
template <int BITS>
__device__ __forceinline__ uint32_t seg_bin(const uint8_t* p, int r) {
    if constexpr (BITS == 8) {
        return gld_u8(p + r);
    } else if constexpr (BITS == 4) {
        const int q = r & 7;
        return (gld_u8(p + 4 * (r >> 3) + (q & 3)) >> (4 * (q >> 2))) & 15u;
    } else {
        return (gld_u8(p + (r >> 3)) >> (r & 7)) & 1u;
    }
}

__device__ __forceinline__ int64_t seg_stride_of(const int64_t* seg, int f) {
    return seg ? seg[f] : 16;
}

struct TileArgs {
    const uint8_t* const* bins;
    const int64_t* seg = nullptr;   // per-feature segment strides, NULL = columns
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
    // Histogram subtraction: when `side` is set, the tile is indexed by the
    // parent leaf p = leaf & (L - 1) (L = number of parents) and only rows of
    // the child whose bit `sub_shift` equals side[p] are accumulated.
    const uint8_t* side = nullptr;
    uint32_t sub_shift = 0;
    // LDS replicas per cell (power of two): lane l updates replica l % rep, so
    // lanes of a wave that hit the same bin of the same cell mostly update
    // different words; the flush adds the replicas.
    int32_t rep = 1;
};

// Tile leaf slot of a row with leaf value v (>= lt: not in this tile).
__device__ __forceinline__ uint32_t tile_slot(const TileArgs& a, uint32_t v, uint32_t lmask) {
    if (a.side) {
        const uint32_t p = v & lmask;
        if (((v >> a.sub_shift) & 1u) != (uint32_t)a.side[p]) return 0xffffffffu;
        return p - a.l0;
    }
    return (v & lmask) - a.l0;
}

// Bins per cell row in LDS: padded to an odd count so that consecutive cells
// (and replicas) start in different banks.
__host__ __device__ inline int32_t lds_stride(int32_t B) { return B | 1; }

// LDS bytes of a tile of `cells` cells (replicas counted as cells).
__host__ __device__ inline int64_t tile_lds_bytes(int precision, int rmse, int K, int B,
                                                  int64_t cells) {
    const int64_t Bs = lds_stride(B);
    if (precision == CBH_PREC_INT16) return cells * K * Bs * 8;
    if (rmse) return cells * Bs * 12;
    return cells * K * 2 * Bs * 8;
}

// LDS element of (plane row, bin, replica): replicas innermost, so the lanes
// of a half-wave (replica = lane % rep with rep = 32) fall in distinct banks.
__device__ __forceinline__ uint32_t lds_elem(uint32_t plane_row, uint32_t Bs, uint32_t bin,
                                             uint32_t rep, uint32_t replica) {
    return (plane_row * Bs + bin) * rep + replica;
}

// Add one row's statistics of class c to (cell, bin). Plane rows:
//   INT16: cell * K + c (u64); FP RMSE: cell (f64) and, after all f64 planes,
//   cell (u32 count); FP otherwise: (cell * K + c) * 2 + t (f64, t = 0 g, 1 h).
template <int PREC, int RM>
__device__ __forceinline__ void add_row(uint32_t* lds, uint32_t ncells, uint32_t cell,
                                        uint32_t Bs, uint32_t bin, int c, int K, uint32_t rep,
                                        uint32_t replica, float gv, float hv, uint32_t qv) {
    if constexpr (PREC == CBH_PREC_INT16) {
        // (g code << 32) + h code: with <= 65536 rows per tile neither half
        // overflows, so one 64-bit LDS add updates both sums exactly.
        const int64_t gcode = (int16_t)(qv & 0xffffu);
        const uint64_t hcode = (qv >> 16) & 0x7fffu;
        const uint64_t packed = ((uint64_t)gcode << 32) + hcode;
        unsigned long long* l64 = reinterpret_cast<unsigned long long*>(lds);
        __hip_atomic_fetch_add(l64 + lds_elem(cell * K + c, Bs, bin, rep, replica),
                               (unsigned long long)packed, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
        // 8-byte element e of the g (and h) planes
        const auto add_elem = [&](uint32_t e, float v) {
            if constexpr (PREC == CBH_PREC_F64) {
                __hip_atomic_fetch_add(reinterpret_cast<double*>(lds) + e, (double)v,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } else if constexpr (PREC == CBH_PREC_FP32) {
                cas_add_f32(lds + 2 * e, v);
            } else {
                cas_twosum(reinterpret_cast<uint64_t*>(lds) + e, v);
            }
        };
        if constexpr (RM != 0) {
            const uint32_t e = lds_elem(cell, Bs, bin, rep, replica);
            add_elem(e, gv);
            __hip_atomic_fetch_add(lds + 2 * ncells * Bs * rep + e, 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            const uint32_t pr = (cell * K + c) * 2;
            add_elem(lds_elem(pr, Bs, bin, rep, replica), gv);
            add_elem(lds_elem(pr + 1, Bs, bin, rep, replica), hv);
        }
    }
}

// ROWS (8 or 16) bins of rows i.. of one column (any alignment of the column),
// in .x .y (.z .w) little-endian order.
template <int ROWS>
__device__ __forceinline__ uint4 load_bins(const uint8_t* col, int64_t stride, int64_t i) {
    // i is a multiple of ROWS (8 or 16), so the ROWS rows share one segment
    const uint8_t* p = seg_ptr(col, stride, i);
    if constexpr (ROWS == 16) {
        if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) return *reinterpret_cast<const uint4*>(p);
    } else {
        if ((reinterpret_cast<uintptr_t>(p) & 7) == 0) {
            const uint2 v = *reinterpret_cast<const uint2*>(p);
            return make_uint4(v.x, v.y, 0u, 0u);
        }
    }
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int k = 0; k < ROWS / 4; ++k)
        w[k] = (uint32_t)p[4 * k] | ((uint32_t)p[4 * k + 1] << 8) |
               ((uint32_t)p[4 * k + 2] << 16) | ((uint32_t)p[4 * k + 3] << 24);
    return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ uint32_t byte_of(const uint4& v, int r) {
    const uint32_t w = r < 4 ? v.x : r < 8 ? v.y : r < 12 ? v.z : v.w;
    return (w >> (8 * (r & 3))) & 255u;
}

template <int PREC, int ROWS>
__device__ __forceinline__ void load_grad(const TileArgs& a, int c, int64_t i, bool vec,
                                          bool rmse, float gv[ROWS], float hv[ROWS],
                                          uint32_t qv[ROWS]) {
    const int64_t ci = int64_t(c) * a.n + i;
    if constexpr (PREC == CBH_PREC_INT16) {
        if (vec) {
#pragma unroll
            for (int k = 0; k < ROWS / 4; ++k) {
                const uint4 t = *reinterpret_cast<const uint4*>(a.gq + ci + 4 * k);
                qv[4 * k] = t.x; qv[4 * k + 1] = t.y; qv[4 * k + 2] = t.z; qv[4 * k + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) qv[r] = a.gq[ci + r];
        }
    } else {
        if (vec) {
#pragma unroll
            for (int k = 0; k < ROWS / 4; ++k) {
                const float4 t = *reinterpret_cast<const float4*>(a.g + ci + 4 * k);
                gv[4 * k] = t.x; gv[4 * k + 1] = t.y; gv[4 * k + 2] = t.z; gv[4 * k + 3] = t.w;
                if (!rmse) {
                    const float4 u = *reinterpret_cast<const float4*>(a.h + ci + 4 * k);
                    hv[4 * k] = u.x; hv[4 * k + 1] = u.y; hv[4 * k + 2] = u.z;
                    hv[4 * k + 3] = u.w;
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                gv[r] = a.g[ci + r];
                if (!rmse) hv[r] = a.h[ci + r];
            }
        }
    }
}

// Rows per thread per step: 16 for the int16 form (one u64 atomic per row and
// feature, few live registers), 8 for the float forms, whose float64 LDS
// updates need twice the registers per row.
template <int PREC>
constexpr int rows_per_step() { return PREC == CBH_PREC_INT16 ? 16 : 8; }

template <int PREC, int KT, int RM>
__device__ __forceinline__ void hist_tile(const TileArgs& a, uint32_t* lds) {
    constexpr int ROWS = rows_per_step<PREC>();
    constexpr int LOG_ROWS = ROWS == 16 ? 4 : 3;
    const int K = KT > 0 ? KT : a.K;
    const int nthr = blockDim.x;
    const uint32_t lmask = (uint32_t)a.L - 1u;
    const uint32_t ltn = (uint32_t)a.lt;
    const uint32_t B = (uint32_t)a.B;
    const uint32_t Bs = (uint32_t)lds_stride(a.B);
    const uint32_t Bm1 = B - 1u;
    const uint32_t rep = (uint32_t)a.rep;
    const uint32_t ncells = (uint32_t)(a.lt * a.fb);
    const int tile_words = (int)(tile_lds_bytes(PREC, RM, K, a.B, ncells * rep) / 4);
    for (int i = threadIdx.x; i < tile_words; i += nthr) lds[i] = 0u;
    __syncthreads();
    constexpr bool rmse = RM != 0;
    const bool vec = ((a.n & 3) == 0 || K == 1) &&
                     ((reinterpret_cast<uintptr_t>(a.g) | reinterpret_cast<uintptr_t>(a.h) |
                       reinterpret_cast<uintptr_t>(a.gq)) & 15) == 0;
    const bool leaf_vec = (reinterpret_cast<uintptr_t>(a.leaf) & 15) == 0;
    const int64_t nq = (a.r1 - a.r0) >> LOG_ROWS;
    constexpr uint32_t kSkip = 0xffffffffu;
    float gv[ROWS], hv[ROWS];
    uint32_t qv[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        gv[r] = 0.f;
        hv[r] = 1.f;
        qv[r] = 0u;
    }
    const uint32_t fbu = (uint32_t)a.fb;            // cells per tile leaf
    const uint32_t replica = (uint32_t)threadIdx.x & (rep - 1u);
    for (int64_t q = threadIdx.x; q < nq; q += nthr) {
        const int64_t i = a.r0 + (int64_t)ROWS * q;
        // lb[r]: first cell of row r's leaf in the tile, kSkip if outside it
        uint32_t lb[ROWS];
        if (a.L == 1 && !a.side) {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) lb[r] = 0u;
        } else if (leaf_vec) {
            uint32_t w[ROWS / 2];
#pragma unroll
            for (int k = 0; k < ROWS / 8; ++k) {
                const uint4 x = *reinterpret_cast<const uint4*>(a.leaf + i + 8 * k);
                w[4 * k] = x.x; w[4 * k + 1] = x.y; w[4 * k + 2] = x.z; w[4 * k + 3] = x.w;
            }
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const uint32_t l = tile_slot(a, (w[r >> 1] >> (16 * (r & 1))) & 0xffffu, lmask);
                lb[r] = l < ltn ? l * fbu : kSkip;
            }
        } else {
#pragma unroll
            for (int r = 0; r < ROWS; ++r) {
                const uint32_t l = tile_slot(a, (uint32_t)a.leaf[i + r], lmask);
                lb[r] = l < ltn ? l * fbu : kSkip;
            }
        }
        if constexpr (KT == 1) load_grad<PREC, ROWS>(a, 0, i, vec, rmse, gv, hv, qv);
        for (int j0 = 0; j0 < a.nf; j0 += 4) {
            uint4 bb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                bb[u] = (j0 + u < a.nf)
                            ? load_bins<ROWS>(a.bins[a.f0 + j0 + u],
                                              seg_stride_of(a.seg, a.f0 + j0 + u), i)
                            : make_uint4(0u, 0u, 0u, 0u);
            for (int c = 0; c < K; ++c) {
                if constexpr (KT != 1) load_grad<PREC, ROWS>(a, c, i, vec, rmse, gv, hv, qv);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (j0 + u < a.nf) {
#pragma unroll
                        for (int r = 0; r < ROWS; ++r) {
                            if (lb[r] != kSkip) {
                                const uint32_t bin = min(byte_of(bb[u], r), Bm1);
                                add_row<PREC, RM>(lds, ncells, lb[r] + (uint32_t)(j0 + u), Bs,
                                                  bin, c, K, rep, replica, gv[r], hv[r], qv[r]);
                            }
                        }
                    }
                }
            }
        }
    }
    // rows after the last full group (only in the last chunk)
    const int64_t tail0 = a.r0 + (int64_t)ROWS * nq;
    if (threadIdx.x < a.r1 - tail0) {
        const int64_t i = tail0 + threadIdx.x;
        const uint32_t l = (a.L == 1 && !a.side) ? 0u - a.l0 : tile_slot(a, a.leaf[i], lmask);
        if (l < ltn) {
            for (int c = 0; c < K; ++c) {
                const int64_t ci = int64_t(c) * a.n + i;
                float g1 = 0.f, h1 = 1.f;
                uint32_t q1 = 0u;
                if constexpr (PREC == CBH_PREC_INT16) {
                    q1 = a.gq[ci];
                } else {
                    g1 = a.g[ci];
                    if (!rmse) h1 = a.h[ci];
                }
                for (int j = 0; j < a.nf; ++j) {
                    const uint32_t bin = min(
                        (uint32_t)*seg_ptr(a.bins[a.f0 + j], seg_stride_of(a.seg, a.f0 + j), i),
                        Bm1);
                    add_row<PREC, RM>(lds, ncells, l * fbu + (uint32_t)j, Bs, bin, c, K, rep,
                                      replica, g1, h1, q1);
                }
            }
        }
    }
    __syncthreads();
    // write the tile in the partial's [L][F][B][wpc] order (coalesced stores),
    // converting to the output format: FP32 copies its float sums (replicas
    // added in float), TWOFLOAT its (hi, lo) pairs (replicas added by TwoSum),
    // F64 splits each sum into (hi, lo) floats, counts and INT16 sums are copied
    const int wpc = a.wpc;
    const int row_words = a.B * wpc;
    const int out_words = a.lt * a.nf * row_words;
    const double* l64 = reinterpret_cast<const double*>(lds);
    const uint64_t* u64 = reinterpret_cast<const uint64_t*>(lds);
    const uint32_t* cnt = lds + 2 * ncells * Bs * rep;      // RMSE count planes
    for (int idx = threadIdx.x; idx < out_words; idx += nthr) {
        const int s = idx % wpc;
        const int bin = (idx / wpc) % a.B;
        const int rest = idx / row_words;
        const int j = rest % a.nf;
        const int ll = rest / a.nf;
        const uint32_t cell = (uint32_t)(ll * a.fb + j);
        uint32_t v;
        if constexpr (PREC == CBH_PREC_INT16) {
            // the two 32-bit halves of the packed sum, replicas added as u64
            const uint32_t e0 = lds_elem(cell * K + (s >> 1), Bs, bin, rep, 0);
            uint64_t t = 0;
            for (uint32_t rp = 0; rp < rep; ++rp) t += u64[e0 + rp];
            v = (s & 1) ? (uint32_t)(t >> 32) : (uint32_t)t;
        } else {
            // statistic t (0 g, 1 h or count) of class c; TWOFLOAT has (hi, lo) parts
            const int c = PREC == CBH_PREC_FP32 ? (s >> 1) : (s >> 2);
            const int t = PREC == CBH_PREC_FP32 ? (s & 1) : ((s >> 1) & 1);
            const int hi_lo = PREC == CBH_PREC_FP32 ? 0 : (s & 1);
            if (rmse && t == 1) {
                const uint32_t e0 = lds_elem(cell, Bs, bin, rep, 0);
                uint32_t tc = 0;
                for (uint32_t rp = 0; rp < rep; ++rp) tc += cnt[e0 + rp];
                v = hi_lo ? 0u : tc;
            } else {
                const uint32_t e0 = rmse ? lds_elem(cell, Bs, bin, rep, 0)
                                         : lds_elem((cell * K + c) * 2 + t, Bs, bin, rep, 0);
                if constexpr (PREC == CBH_PREC_F64) {
                    double d = 0.0;
                    for (uint32_t rp = 0; rp < rep; ++rp) d += l64[e0 + rp];
                    const float hi = (float)d;
                    v = __float_as_uint(hi_lo ? (float)(d - (double)hi) : hi);
                } else if constexpr (PREC == CBH_PREC_FP32) {
                    float f = 0.f;
                    for (uint32_t rp = 0; rp < rep; ++rp) f += __uint_as_float(lds[2 * (e0 + rp)]);
                    v = __float_as_uint(f);
                } else {
                    float S = 0.f, E = 0.f;
                    for (uint32_t rp = 0; rp < rep; ++rp) {
                        const uint64_t w = u64[e0 + rp];
                        const float hi = __uint_as_float((uint32_t)w);
                        const float t2 = S + hi, bp = t2 - S;
                        E += ((S - (t2 - bp)) + (hi - bp)) + __uint_as_float((uint32_t)(w >> 32));
                        S = t2;
                    }
                    const float2 r = renorm_pair(S, E);
                    v = __float_as_uint(hi_lo ? r.y : r.x);
                }
            }
        }
        a.part[((int64_t)(a.l0 + ll) * a.F + (a.f0 + j)) * row_words + bin * wpc + s] = v;
    }
}

// ------------------------------------------------------------ partial merge
// Merge cell `cell` (all 2K statistics) over n_chunks partial histograms of
// `cells` cells each, in chunk order, into cell `dst` of the output layout of
// the precision. With a parent histogram (a build by subtraction: the partials
// hold the smaller child of each parent, cell = parent cell), cell `sib` of
// the output gets parent cell `cell` minus the merged value.
template <int PREC>
__device__ __forceinline__ void merge_cell(const uint32_t* __restrict__ part, int64_t cells,
                                           int K, int n_chunks, bool rmse, void* __restrict__ out,
                                           int64_t cell, int64_t dst, int64_t sib = -1,
                                           const void* __restrict__ parent = nullptr) {
    static_assert(PREC != CBH_PREC_F64, "F64 histograms are merged as TWOFLOAT");
    const int wpc = PREC == CBH_PREC_TWOFLOAT ? 4 * K : 2 * K;
    const int64_t cw = cells * wpc;
    for (int c = 0; c < K; ++c) {
        if constexpr (PREC == CBH_PREC_FP32) {
            const int64_t j = cell * wpc + 2 * c;
            const int64_t jd = dst * wpc + 2 * c, js = sib * wpc + 2 * c;
            float g = 0.f;
            for (int ch = 0; ch < n_chunks; ++ch) g += __uint_as_float(part[ch * cw + j]);
            reinterpret_cast<float*>(out)[jd] = g;
            if (sib >= 0)
                reinterpret_cast<float*>(out)[js] = reinterpret_cast<const float*>(parent)[j] - g;
            if (rmse) {
                uint32_t cnt = 0;
                for (int ch = 0; ch < n_chunks; ++ch) cnt += part[ch * cw + j + 1];
                reinterpret_cast<uint32_t*>(out)[jd + 1] = cnt;
                if (sib >= 0)
                    reinterpret_cast<uint32_t*>(out)[js + 1] =
                        reinterpret_cast<const uint32_t*>(parent)[j + 1] - cnt;
            } else {
                float hh = 0.f;
                for (int ch = 0; ch < n_chunks; ++ch) hh += __uint_as_float(part[ch * cw + j + 1]);
                reinterpret_cast<float*>(out)[jd + 1] = hh;
                if (sib >= 0)
                    reinterpret_cast<float*>(out)[js + 1] =
                        reinterpret_cast<const float*>(parent)[j + 1] - hh;
            }
        } else if constexpr (PREC == CBH_PREC_TWOFLOAT) {
            for (int st = 0; st < 2; ++st) {
                const int64_t j = cell * wpc + 4 * c + 2 * st;
                const int64_t o = 2 * c + st;          // float2 index within a cell
                float2 r;
                if (st == 1 && rmse) {
                    uint32_t cnt = 0;
                    for (int ch = 0; ch < n_chunks; ++ch) cnt += part[ch * cw + j];
                    r = make_float2(__uint_as_float(cnt), 0.f);
                    if (sib >= 0) {
                        const uint32_t pc = __float_as_uint(
                            reinterpret_cast<const float2*>(parent)[cell * 2 * K + o].x);
                        reinterpret_cast<float2*>(out)[sib * 2 * K + o] =
                            make_float2(__uint_as_float(pc - cnt), 0.f);
                    }
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
                    if (sib >= 0) {
                        // (P_hi, P_lo) - (hs, lo), TwoSum on the leading parts
                        const float2 Pv = reinterpret_cast<const float2*>(parent)[cell * 2 * K + o];
                        const float t = Pv.x - r.x;
                        const float bp = t - Pv.x;
                        const float e = ((Pv.x - (t - bp)) + (-r.x - bp)) + (Pv.y - r.y);
                        const float dh = t + e;
                        reinterpret_cast<float2*>(out)[sib * 2 * K + o] =
                            make_float2(dh, e - (dh - t));
                    }
                }
                reinterpret_cast<float2*>(out)[dst * 2 * K + o] = r;
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
            const int64_t sd = dst * K + c;
            reinterpret_cast<int64_t*>(out)[2 * sd] = gs;
            reinterpret_cast<int64_t*>(out)[2 * sd + 1] = hs;
            if (sib >= 0) {
                const int64_t* Pv = reinterpret_cast<const int64_t*>(parent);
                const int64_t ss = sib * K + c;
                reinterpret_cast<int64_t*>(out)[2 * ss] = Pv[2 * slot] - gs;
                reinterpret_cast<int64_t*>(out)[2 * ss + 1] = Pv[2 * slot + 1] - hs;
            }
        }
    }
}

// Smaller child of parent leaf p at the parent level's split (feature f,
// border k), judged by the parent histogram's second statistic (row count for
// RMSE, sum of h otherwise) on the split feature, summed by one wave: 1 if the
// bit-set child is the smaller one. With no split every row stayed on the
// clear side, so the set side is empty.
template <int PREC>
__device__ __forceinline__ uint8_t parent_side(const void* __restrict__ parent, int64_t p, int f,
                                               int k, int32_t F, int32_t B, int32_t K,
                                               int32_t rmse, int lane) {
    static_assert(PREC != CBH_PREC_F64, "F64 histograms are read as TWOFLOAT");
    if (f < 0 || f >= F) return 1;
    double left = 0.0, right = 0.0;
    for (int b = lane; b < B; b += 64) {
        const int64_t e = ((p * F + f) * B + b) * 2 * K + 1;   // statistic 1 of class 0
        double v;
        if constexpr (PREC == CBH_PREC_FP32)
            v = rmse ? (double)reinterpret_cast<const uint32_t*>(parent)[e]
                     : (double)reinterpret_cast<const float*>(parent)[e];
        else if constexpr (PREC == CBH_PREC_TWOFLOAT)
            v = rmse ? (double)__float_as_uint(reinterpret_cast<const float2*>(parent)[e].x)
                     : (double)reinterpret_cast<const float2*>(parent)[e].x;
        else
            v = (double)reinterpret_cast<const int64_t*>(parent)[e];
        if (b <= k) left += v; else right += v;
    }
    for (int d = 32; d >= 1; d >>= 1) {
        left += __shfl_xor(left, d, 64);
        right += __shfl_xor(right, d, 64);
    }
    return right < left ? 1 : 0;
}

// ---------------------------------------------------------------- scoring
struct FeatBest {
    float s1;     // best score of the feature
    int32_t k1;   // its border (-1: no candidate)
    float s2;     // best score of any other border of the feature
    int32_t pad;
};

// One side's term G^2 / (H + l2), in double: a feature's score adds up to
// 2^level * K * 2 terms (C5's deepest level: 10240), and a float sum of that
// many terms could be off by more than the 1e-5 relative margin that decides
// which of two close splits wins.
__device__ __forceinline__ double side_term(double G, double H, double l2) {
    const double d = H + l2;
    return d == 0.0 ? 0.0 : (G * G) / d;
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
    double l2;
};

// Terms of one histogram row (leaf L, feature f, class c) for the 4 borders
// 4*lane .. 4*lane+3, added into acc. Prefix sums over bins are formed in the
// accumulator type of the precision (float, two-float or exact int64).
template <int PREC>
__device__ void row_terms(const ScoreRow& a, int L, int f, int c, int lane, int kmax,
                          double acc[4]) {
    static_assert(PREC != CBH_PREC_F64, "F64 histograms are scored as TWOFLOAT");
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
                acc[j] += side_term((double)gl.hi + (double)gl.lo, (double)hl.hi + (double)hl.lo,
                                    a.l2) +
                          side_term((double)gr.hi + (double)gr.lo, (double)hr.hi + (double)hr.lo,
                                    a.l2);
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
                acc[j] += side_term((double)gl * sg, (double)hl * sh, a.l2) +
                          side_term((double)(gt - gl) * sg, (double)(ht - hl) * sh, a.l2);
            }
        }
    }
}

// LDS of score_feature: per-wave partial scores and per-wave winners.
template <int NW>
struct ScoreLds {
    double part[NW][256];
    float rs1[NW], rs2[NW];
    int ri1[NW];
};

// Whole-block scoring of feature f over all leaves and classes; writes the
// per-border scores (optional) and the feature's best/second-best. Needs a
// block of 64 NW threads (NW >= 4); wave w takes the (leaf, class) rows
// w, w + NW, ..., and the waves' partial scores are added in wave order.
// `sh`: the block's LDS for it (a kernel whose dynamic LDS serves other work
// passes a part of it).
template <int PREC, int NW>
__device__ void score_feature_in(const ScoreRow& a, int L, int f, int n_bins_f, float* scores,
                                 FeatBest* out, ScoreLds<NW>* sh) {
    double (&part)[NW][256] = sh->part;
    float (&rs1)[NW] = sh->rs1;
    float (&rs2)[NW] = sh->rs2;
    int (&ri1)[NW] = sh->ri1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int kmax = min(n_bins_f, a.B) - 1;  // candidates k < kmax
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (kmax > 0) {
        const int items = L * a.K;
        for (int it = wave; it < items; it += NW) row_terms<PREC>(a, it / a.K, f, it % a.K, lane,
                                                                   kmax, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) part[wave][4 * lane + j] = acc[j];
    __syncthreads();
    const int k = threadIdx.x;  // thread k < 256 owns border k
    float s = -INFINITY;
    if (k < kmax) {
        double sd = part[0][k] + part[1][k];
#pragma unroll
        for (int w = 2; w < NW; ++w) sd += part[w][k];
        s = (float)sd;
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
        // borders live in the first four waves only
        float b1 = rs1[0], b2 = rs2[0];
        int j = ri1[0];
        for (int w = 1; w < 4; ++w) top2_merge(b1, j, b2, rs1[w], ri1[w], rs2[w]);
        *out = FeatBest{b1, j, b2, 0};
    }
}

template <int PREC, int NW = 4>
__device__ void score_feature(const ScoreRow& a, int L, int f, int n_bins_f, float* scores,
                              FeatBest* out) {
    __shared__ ScoreLds<NW> sh;
    score_feature_in<PREC, NW>(a, L, f, n_bins_f, scores, out, &sh);
}

// Reduce F per-feature winners (one block, its first 256 threads) to the
// level's split.
__device__ inline void argmax_features(const FeatBest* __restrict__ fb, int F, int Bm1,
                                       cbh_split* __restrict__ out) {
    float s1 = -INFINITY, s2 = -INFINITY;
    int i1 = -1;
    for (int f = threadIdx.x; f < F && threadIdx.x < 256; f += 256) {
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
    if (lane == 0 && wave < 4) {
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

// bytes per (slot, bin, feature) over all stats
template <int PREC>
__host__ __device__ constexpr uint32_t lpf_cell_bytes() { return PREC == CBH_PREC_INT16 ? 8u : 16u; }

// Bytes of one (slot, bin) record of the tile (W features x all stats). For
// narrow groups (W * CS <= 128) several lanes share a feature, and their bins
// decide the bank: an 8-byte pad makes the record an odd number of 8-byte
// words, so different bins fall on different banks.
__host__ __device__ constexpr uint32_t lpf_record_bytes(uint32_t W, uint32_t CS) {
    return W * CS <= 128 ? W * CS + 8 : W * CS;
}

// Arguments of one lanes-over-features block, shared by the single-problem
// and the batched launches.
struct LpfBlock {
    const uint8_t* const* bins;
    const int64_t* seg;          // per-feature segment strides, NULL = columns
    const float* g;              // this class's statistics
    const float* h;
    const uint32_t* gq;
    const uint16_t* rowcode;     // per-row slot codes (MODE != 0)
    int32_t F, B;
    int32_t wpc;                 // words per output cell (all classes)
    int32_t coff;                // words before this class within a cell
};

// ------------------------------------------- lanes-over-features variant
// For one class (K = 1). Lane l of a wave owns feature f0 + l % W of the
// block's group of W features and the 16-row segment l / W of the wave's
// current group of 64 / W segments. The LDS tile is [slot][bin][stat][W] of
// 8-byte elements (one stat, the packed int16 codes; or two: the g sum (a
// float64, a (hi, lo) pair or a float) and then the count or the h sum in
// the same form; FP32 with h keeps the (g, h) float pair in the first), so
// in one LDS instruction the lanes with distinct features touch distinct
// banks whatever their bins are, with no replicas. With the bins in
// the tiled layout the W segments of one row group are adjacent in memory and
// a wave's bin load is fully coalesced; plain columns work too.
// LDS byte offset, in slot 0, of the first stat of (bin of row r of the
// segment's words, this lane's feature): bin * W * CS + lane_off, where
// lane_off = 8 * feature; the second stat is W * 8 bytes further.
template <int W, int CS>
__device__ __forceinline__ uint32_t lpf_addr(const uint32_t (&bw)[4], int r, uint32_t lane_off) {
    const uint32_t word = bw[r >> 2];
    if constexpr (W * CS == 256) {
        // byte 1 <- bin, byte 0 <- lane_off (< 256), bytes 2 and 3 <- 0
        return __builtin_amdgcn_perm(word, lane_off, 0x0c0c0000u | ((4u + (r & 3)) << 8));
    } else if constexpr (W * CS == 512) {
        return __builtin_amdgcn_perm(word, lane_off >> 1, 0x0c0c0000u | ((4u + (r & 3)) << 8))
               << 1;
    } else {
        return ((word >> (8 * (r & 3))) & 255u) * lpf_record_bytes(W, CS) + lane_off;
    }
}

// Add rows r0 .. r0+7 of one 16-row segment (bins in bw) to the tile.
// off[k]: slot byte offset of row r0 + k, or kLpfSkip; CHECK = false when every
// row is known to be valid.
constexpr uint32_t kLpfSkip = 0xffffffffu;

// Float32 forms (cells updated by compare-and-swap, see lds_cas32): the
// eight rows' cells are read, all eight swaps are issued back to back, and
// only the rows whose swap found the cell changed (another row of this lane
// on the same bin, or another wave) are redone one at a time. Cell layout
// (8 bytes each at `ad` and `ad + W * 8`):
//   FP32, RMSE:      float g sum at ad, u32 count at ad + W * 8
//   FP32, h:         (g, h) float pair at ad, one 64-bit swap for both
//   TWOFLOAT, RMSE:  (g hi, g lo) at ad, u32 count at ad + W * 8
//   TWOFLOAT, h:     (g hi, g lo) at ad, (h hi, h lo) at ad + W * 8
// FP32 with an h statistic: the (g, h) pair of a cell is one 64-bit word,
// updated by compare-and-swap. A lane's rows that land in one cell are
// first added in float32 in row order onto the first of them, which then
// makes the one compare-and-swap for the cell: compare-and-swaps of one lane
// on one address would otherwise fail one after the other (each retry a full
// LDS round trip). The sums stay float32 additions. (Measured: this pays
// where many rows of a segment share a bin, as with the statistic columns
// of the many-class workload, and costs more than it saves elsewhere, so
// the count form and the compensated form keep one swap per row.)
template <int W>
__device__ __forceinline__ void lpf_rows8_pair_f32(char* tile, const uint32_t (&ad)[8],
                                                   const bool (&ok)[8], const float (&gv)[8],
                                                   const float (&hv)[8]) {
    float ag[8], ah[8];
    bool lead[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        ag[k] = gv[k];
        ah[k] = hv[k];
        lead[k] = ok[k];
    }
#pragma unroll
    for (int k = 1; k < 8; ++k) {
#pragma unroll
        for (int j = 0; j < k; ++j) {
            if (lead[j] && lead[k] && ad[j] == ad[k]) {
                ag[j] = ag[j] + ag[k];
                ah[j] = ah[j] + ah[k];
                lead[k] = false;
            }
        }
    }
    uint64_t old[8], got[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        old[k] = lead[k] ? lds_load64(reinterpret_cast<uint64_t*>(tile + ad[k])) : 0ull;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        got[k] = lead[k] ? lds_cas64(reinterpret_cast<uint64_t*>(tile + ad[k]), old[k],
                                     add_pair_word(old[k], ag[k], ah[k]))
                         : 0ull;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        while (got[k] != old[k]) {
            old[k] = got[k];
            got[k] = lds_cas64(reinterpret_cast<uint64_t*>(tile + ad[k]), old[k],
                               add_pair_word(old[k], ag[k], ah[k]));
        }
    }
}

template <int PREC, int RM, int W, bool CHECK>
__device__ __forceinline__ void lpf_rows8_cas(char* tile, const uint32_t (&bw)[4], int r0,
                                              uint32_t lane_off, const uint32_t (&off)[8],
                                              const float (&gv)[8], const float (&hv)[8]) {
    constexpr uint32_t CS = lpf_cell_bytes<PREC>();
    uint32_t ad[8];
    bool ok[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        ok[k] = !CHECK || off[k] != kLpfSkip;
        ad[k] = ok[k] ? lpf_addr<W, CS>(bw, r0 + k, lane_off) + off[k] : 0u;
    }
    if constexpr (PREC == CBH_PREC_FP32 && RM == 0) {
        lpf_rows8_pair_f32<W>(tile, ad, ok, gv, hv);
        return;
    }
    if constexpr (PREC == CBH_PREC_FP32 && RM != 0) {
        uint32_t old[8], got[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            old[k] = ok[k] ? lds_load32(reinterpret_cast<uint32_t*>(tile + ad[k])) : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            got[k] = ok[k] ? lds_cas32(reinterpret_cast<uint32_t*>(tile + ad[k]), old[k],
                                       __float_as_uint(__uint_as_float(old[k]) + gv[k]))
                           : 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (ok[k])
                __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(tile + ad[k] + W * 8), 1u,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            while (got[k] != old[k]) {
                old[k] = got[k];
                got[k] = lds_cas32(reinterpret_cast<uint32_t*>(tile + ad[k]), old[k],
                                   __float_as_uint(__uint_as_float(old[k]) + gv[k]));
            }
        }
    } else {
        // the 64-bit word at ad: (g, h) pair (FP32) or the (hi, lo) g pair
        const auto upd = [&](uint64_t w, int k) -> uint64_t {
            if constexpr (PREC == CBH_PREC_FP32) return add_pair_word(w, gv[k], hv[k]);
            else return twosum_word(w, gv[k]);
        };
        uint64_t old[8], got[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            old[k] = ok[k] ? lds_load64(reinterpret_cast<uint64_t*>(tile + ad[k])) : 0ull;
#pragma unroll
        for (int k = 0; k < 8; ++k)
            got[k] = ok[k] ? lds_cas64(reinterpret_cast<uint64_t*>(tile + ad[k]), old[k],
                                       upd(old[k], k))
                           : 0ull;
        if constexpr (PREC == CBH_PREC_TWOFLOAT) {
            if constexpr (RM != 0) {
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (ok[k])
                        __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(tile + ad[k] + W * 8),
                                               1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
                uint64_t oh[8], gh[8];
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    oh[k] = ok[k] ? lds_load64(reinterpret_cast<uint64_t*>(tile + ad[k] + W * 8))
                                  : 0ull;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    gh[k] = ok[k] ? lds_cas64(reinterpret_cast<uint64_t*>(tile + ad[k] + W * 8),
                                              oh[k], twosum_word(oh[k], hv[k]))
                                  : 0ull;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    while (gh[k] != oh[k]) {
                        oh[k] = gh[k];
                        gh[k] = lds_cas64(reinterpret_cast<uint64_t*>(tile + ad[k] + W * 8),
                                          oh[k], twosum_word(oh[k], hv[k]));
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            while (got[k] != old[k]) {
                old[k] = got[k];
                got[k] = lds_cas64(reinterpret_cast<uint64_t*>(tile + ad[k]), old[k],
                                   upd(old[k], k));
            }
        }
    }
}

// One row of a float32 form (the ragged tail), same cells as lpf_rows8_cas.
template <int PREC, int RM, int W>
__device__ __forceinline__ void lpf_row1_cas(char* tile, uint32_t ad, float g, float h) {
    if constexpr (PREC == CBH_PREC_FP32 && RM != 0) {
        cas_add_f32(reinterpret_cast<uint32_t*>(tile + ad), g);
    } else if constexpr (PREC == CBH_PREC_FP32) {
        uint64_t* p = reinterpret_cast<uint64_t*>(tile + ad);
        uint64_t old = lds_load64(p);
        for (;;) {
            const uint64_t got = lds_cas64(p, old, add_pair_word(old, g, h));
            if (got == old) break;
            old = got;
        }
    } else {
        cas_twosum(reinterpret_cast<uint64_t*>(tile + ad), g);
        if constexpr (RM == 0) cas_twosum(reinterpret_cast<uint64_t*>(tile + ad + W * 8), h);
    }
    if constexpr (RM != 0)
        __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(tile + ad + W * 8), 1u,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

template <int PREC, int RM, int W, bool CHECK>
__device__ __forceinline__ void lpf_rows8(char* tile, const uint32_t (&bw)[4], int r0,
                                          uint32_t lane_off, const uint32_t (&off)[8],
                                          const float (&gv)[8], const float (&hv)[8],
                                          const uint32_t (&qv)[8]) {
    constexpr uint32_t CS = lpf_cell_bytes<PREC>();
    if constexpr (PREC == CBH_PREC_FP32 || PREC == CBH_PREC_TWOFLOAT) {
        lpf_rows8_cas<PREC, RM, W, CHECK>(tile, bw, r0, lane_off, off, gv, hv);
        return;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        if (CHECK && off[k] == kLpfSkip) continue;
        const uint32_t ad = lpf_addr<W, CS>(bw, r0 + k, lane_off) + off[k];
        if constexpr (PREC == CBH_PREC_INT16) {
            // (g code << 32) + h code: both halves stay exact for <= 65536
            // rows per chunk. The h code (high half of the word) is in
            // [0, 32767]; the g code (low half) is sign-extended.
            const uint32_t hq = qv[k] >> 16;
            const uint32_t gq = (uint32_t)((int32_t)(qv[k] << 16) >> 16);
            const uint64_t packed = ((uint64_t)gq << 32) | hq;
            __hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(tile + ad),
                                   (unsigned long long)packed, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            __hip_atomic_fetch_add(reinterpret_cast<double*>(tile + ad), (double)gv[k],
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if constexpr (RM != 0)
                __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(tile + ad + W * 8), 1u,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            else
                __hip_atomic_fetch_add(reinterpret_cast<double*>(tile + ad + W * 8),
                                       (double)hv[k], __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
}

// One 16-row segment of the lanes-over-features kernel: its bins (this
// lane's feature), row codes and gradient statistics, loaded with 16-byte
// loads; add() puts its rows into the tile, 8 at a time.
// s_waitcnt immediate that waits until at most n vector-memory loads are
// outstanding and leaves the export and LDS counters alone (gfx9 encoding:
// vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
constexpr int vm_wait_imm(int n) {
    return (n & 15) | (7 << 4) | (15 << 8) | (((n >> 4) & 3) << 14);
}

template <int PREC, int RM, int MODE, int BITS = 8>
struct LpfSeg {
    // 16-byte loads per segment (bins, row codes, statistics)
    static constexpr int kLoads =
        1 + (MODE != 0 ? 2 : 0) + 4 + ((PREC != CBH_PREC_INT16 && RM == 0) ? 4 : 0);
    uint4 b;
    uint4 c[2];      // row codes (MODE != 0)
    uint4 q[4];      // int16 codes
    float4 g[4], h[4];
    __device__ __forceinline__ void load(const uint8_t* col, int64_t sstride,
                                         const uint16_t* rowcode, const LpfBlock& a, int64_t t) {
        const int64_t i = t << 4;
        b = load_seg16<BITS>(col + t * sstride);
        if constexpr (MODE != 0) {
            c[0] = gld_u4(rowcode + i);
            c[1] = gld_u4(rowcode + i + 8);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if constexpr (PREC == CBH_PREC_INT16) {
                q[k] = gld_u4(a.gq + i + 4 * k);
            } else {
                g[k] = gld_f4(a.g + i + 4 * k);
                if constexpr (RM == 0) h[k] = gld_f4(a.h + i + 4 * k);
            }
        }
    }
    // Wait for this segment's loads while the other register set's kLoads
    // loads, issued after them, stay in flight. Called on every path before
    // add(): the compiler's own waits, merged over add()'s branches, would
    // otherwise drain the next segment's loads too.
    __device__ __forceinline__ static void wait_mine() {
        __builtin_amdgcn_s_waitcnt(vm_wait_imm(kLoads));
    }
    template <int W>
    __device__ __forceinline__ void add(char* tile, uint32_t lane_off, uint32_t s0, uint32_t ns,
                                        uint32_t slot_bytes) const {
        const uint32_t bw[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
            uint32_t off[8];
            float gv[8], hv[8];
            uint32_t qv[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                off[k] = 0u;
                if constexpr (MODE != 0) {
                    const uint4 cc = c[h2];
                    const uint32_t lw[4] = {cc.x, cc.y, cc.z, cc.w};
                    const uint32_t code = (lw[k >> 1] >> (16 * (k & 1))) & 0xffffu;
                    const uint32_t sl = code - s0;
                    // slot offsets stay below the LDS size: 24-bit products
                    // (full rate, where a 32-bit multiply is quarter rate)
                    off[k] = MODE == 1 ? __umul24(code, slot_bytes)
                                       : (sl < ns ? __umul24(sl, slot_bytes) : kLpfSkip);
                }
                const int r = 8 * h2 + k;
                if constexpr (PREC == CBH_PREC_INT16) {
                    const uint4 qq = q[r >> 2];
                    const uint32_t qw[4] = {qq.x, qq.y, qq.z, qq.w};
                    qv[k] = qw[r & 3];
                    gv[k] = hv[k] = 0.f;
                } else {
                    const float4 gg = g[r >> 2];
                    const float gw[4] = {gg.x, gg.y, gg.z, gg.w};
                    gv[k] = gw[r & 3];
                    hv[k] = 0.f;
                    if constexpr (RM == 0) {
                        const float4 hh = h[r >> 2];
                        const float hw[4] = {hh.x, hh.y, hh.z, hh.w};
                        hv[k] = hw[r & 3];
                    }
                    qv[k] = 0u;
                }
            }
            lpf_rows8<PREC, RM, W, MODE == 2>(tile, bw, 8 * h2, lane_off, off, gv, hv, qv);
        }
    }
};

// MODE 0: one slot (level 0, direct): no per-row reads, no checks.
// MODE 1: all slots of a direct build in one tile: slot = row code (the leaf).
// MODE 2: subtraction and/or several slot tiles: slot = row code - first slot
//         of the tile, rows outside the tile (or with code 0xffff) skipped.
// One block's tile, in three phases (lpf_block runs them in turn; a caller
// may accumulate several row ranges, in different modes, into one tile):
//   lpf_zero        clears the tile of ns slots;
//   lpf_accumulate  adds rows [r0, r1) (r0 a multiple of 16) of feature
//                   group fg (W features) for slots [s0, s0 + ns) (ns <= 64);
//   lpf_flush       writes the tile to the block's partial histogram `part`,
//                   [slot - part_slot0][F][B][wpc] words, this class at word
//                   coff of each cell.
// lds holds the block's dynamic LDS; the phases are separated by barriers.
template <int PREC, int W>
__device__ __forceinline__ void lpf_zero(int B, uint32_t ns, uint32_t* lds) {
    constexpr uint32_t CS = lpf_cell_bytes<PREC>();
    const uint32_t tile_words = ns * (uint32_t)B * lpf_record_bytes(W, CS) / 4;
    for (uint32_t i = threadIdx.x; i < tile_words; i += blockDim.x) lds[i] = 0u;
}

template <int PREC, int RM, int W, int MODE, int BITS = 8>
__device__ __forceinline__ void lpf_accumulate(const LpfBlock& a, int64_t r0, int64_t r1, int fg,
                                               uint32_t s0, uint32_t ns, uint32_t* lds) {
    constexpr uint32_t CS = lpf_cell_bytes<PREC>();
    constexpr int RG = 64 / W;                  // segments per wave step
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    const int fl = lane & (W - 1), rq = lane / W;
    const int f0 = fg * W;
    const int nf = min(W, a.F - f0);
    const bool fok = fl < nf;
    const int f = f0 + (fok ? fl : 0);
    const uint8_t* col = a.bins[f];
    const int64_t sstride = a.seg ? a.seg[f] : seg_bytes<BITS>();
    const uint32_t slot_bytes = (uint32_t)a.B * lpf_record_bytes(W, CS);
    char* tile = reinterpret_cast<char*>(lds);
    const int64_t t_full = r1 >> 4;            // segments before this one are full
    const uint32_t lane_off = (uint32_t)fl * 8u;
    const uint16_t* rowcode = a.rowcode;
    const bool vec = ((reinterpret_cast<uintptr_t>(col) & (seg_bytes<BITS>() - 1)) |
                      ((reinterpret_cast<uintptr_t>(a.g) | reinterpret_cast<uintptr_t>(a.h) |
                        reinterpret_cast<uintptr_t>(a.gq) | reinterpret_cast<uintptr_t>(rowcode)) &
                       15)) == 0;
    int64_t t = (r0 >> 4) + int64_t(wave) * RG + rq;
    const int64_t step = int64_t(nwaves) * RG;
    if (vec && t < t_full) {
        // software pipeline: the loads of the next segment are issued before
        // the atomics of the current one (two register sets, A and B). The
        // loads are unconditional (past the end they re-read the last full
        // segment and are not used): a load under a branch would make the
        // compiler's wait before the atomics drain it too.
        const int64_t t_last = t_full - 1;
        LpfSeg<PREC, RM, MODE, BITS> A, B;
        A.load(col, sstride, rowcode, a, t);
        for (;;) {
            int64_t tn = t + step;
            B.load(col, sstride, rowcode, a, min(tn, t_last));
            LpfSeg<PREC, RM, MODE, BITS>::wait_mine();
            if (fok) A.template add<W>(tile, lane_off, s0, ns, slot_bytes);
            t = tn;
            if (t >= t_full) break;
            tn = t + step;
            A.load(col, sstride, rowcode, a, min(tn, t_last));
            LpfSeg<PREC, RM, MODE, BITS>::wait_mine();
            if (fok) B.template add<W>(tile, lane_off, s0, ns, slot_bytes);
            t = tn;
            if (t >= t_full) break;
        }
    }
    // the ragged last segment, and everything when a pointer is unaligned:
    // one row at a time
    for (; t < ((r1 + 15) >> 4); t += int64_t(nwaves) * RG) {
        const int64_t i = t << 4;
        const uint8_t* pb = col + t * sstride;
        for (int r = 0; r < 16 && i + r < r1; ++r) {
            const uint32_t bwr[4] = {seg_bin<BITS>(pb, r), 0u, 0u, 0u};
            uint32_t o1[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
            float g1[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            float h1[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            uint32_t q1[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
            if constexpr (MODE != 0) {
                const uint32_t code = gld_u16(rowcode + i + r);
                const uint32_t sl = code - s0;
                o1[0] = MODE == 1 ? code * slot_bytes : (sl < ns ? sl * slot_bytes : kLpfSkip);
            }
            if constexpr (PREC == CBH_PREC_INT16) {
                q1[0] = gld_u32(a.gq + i + r);
            } else {
                g1[0] = gld_f32(a.g + i + r);
                if constexpr (RM == 0) h1[0] = gld_f32(a.h + i + r);
            }
            if (fok && o1[0] != kLpfSkip) {
                // one row: use the per-row routine on a segment holding only this bin
                constexpr uint32_t CSz = lpf_cell_bytes<PREC>();
                const uint32_t ad = lpf_addr<W, CSz>(bwr, 0, lane_off) + o1[0];
                if constexpr (PREC == CBH_PREC_INT16) {
                    const uint64_t packed =
                        ((uint64_t)(int64_t)(int16_t)(q1[0] & 0xffffu) << 32) +
                        ((q1[0] >> 16) & 0x7fffu);
                    __hip_atomic_fetch_add(reinterpret_cast<unsigned long long*>(tile + ad),
                                           (unsigned long long)packed, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                } else if constexpr (PREC != CBH_PREC_F64) {
                    lpf_row1_cas<PREC, RM, W>(tile, ad, g1[0], h1[0]);
                } else {
                    __hip_atomic_fetch_add(reinterpret_cast<double*>(tile + ad), (double)g1[0],
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if constexpr (RM != 0)
                        __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(tile + ad + W * 8), 1u,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    else
                        __hip_atomic_fetch_add(reinterpret_cast<double*>(tile + ad + W * 8),
                                               (double)h1[0], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            }
        }
    }
}

template <int PREC, int RM, int W>
__device__ __forceinline__ void lpf_flush(const LpfBlock& a, int fg, uint32_t s0, uint32_t ns,
                                          uint32_t* part, uint32_t part_slot0,
                                          const uint32_t* lds) {
    constexpr uint32_t CS = lpf_cell_bytes<PREC>();
    const int f0 = fg * W;
    const int nf = min(W, a.F - f0);
    const char* tile = reinterpret_cast<const char*>(lds);
    // write the tile in the partial's [L][F][B][wpc] order; consecutive threads
    // take consecutive features of one (slot, bin), so the LDS reads are
    // conflict-free and every thread writes one whole cell
    const uint32_t cells = ns * (uint32_t)a.B * W;
    for (uint32_t c = threadIdx.x; c < cells; c += blockDim.x) {
        const uint32_t cfl = c & (W - 1);
        if ((int)cfl >= nf) continue;
        const uint32_t sb = c / W;                 // slot * B + bin
        const uint32_t bin = sb % (uint32_t)a.B, sl = sb / (uint32_t)a.B;
        // first stat; the second is W * 8 bytes further
        const char* cell = tile + (size_t)sb * lpf_record_bytes(W, CS) + cfl * 8u;
        const int64_t o =
            ((int64_t(s0 + sl - part_slot0) * a.F + f0 + cfl) * a.B + bin) * a.wpc + a.coff;
        if constexpr (PREC == CBH_PREC_INT16) {
            *reinterpret_cast<uint2*>(part + o) = *reinterpret_cast<const uint2*>(cell);
        } else if constexpr (PREC == CBH_PREC_FP32) {
            const uint2 w = *reinterpret_cast<const uint2*>(cell);
            const uint32_t w1 = RM != 0 ? *reinterpret_cast<const uint32_t*>(cell + W * 8) : w.y;
            *reinterpret_cast<uint2*>(part + o) = make_uint2(w.x, w1);
        } else if constexpr (PREC == CBH_PREC_TWOFLOAT) {
            const uint2 gw = *reinterpret_cast<const uint2*>(cell);
            const float2 gr = renorm_pair(__uint_as_float(gw.x), __uint_as_float(gw.y));
            uint32_t w1, hlo = 0u;
            if constexpr (RM != 0) {
                w1 = *reinterpret_cast<const uint32_t*>(cell + W * 8);
            } else {
                const uint2 hw = *reinterpret_cast<const uint2*>(cell + W * 8);
                const float2 hr = renorm_pair(__uint_as_float(hw.x), __uint_as_float(hw.y));
                w1 = __float_as_uint(hr.x);
                hlo = __float_as_uint(hr.y);
            }
            *reinterpret_cast<uint4*>(part + o) =
                make_uint4(__float_as_uint(gr.x), __float_as_uint(gr.y), w1, hlo);
        } else {
            const double gs = *reinterpret_cast<const double*>(cell);
            const float ghi = (float)gs;
            uint32_t w1;                               // count or h, as stored in the output
            float hlo = 0.f;
            if constexpr (RM != 0) {
                w1 = *reinterpret_cast<const uint32_t*>(cell + W * 8);
            } else {
                const double hs = *reinterpret_cast<const double*>(cell + W * 8);
                const float hhi = (float)hs;
                hlo = (float)(hs - (double)hhi);
                w1 = __float_as_uint(hhi);
            }
            const float glo = (float)(gs - (double)ghi);
            *reinterpret_cast<uint4*>(part + o) =
                make_uint4(__float_as_uint(ghi), __float_as_uint(glo), w1,
                           RM != 0 ? 0u : __float_as_uint(hlo));
        }
    }
}

template <int PREC, int RM, int W, int MODE, int BITS = 8>
__device__ __forceinline__ void lpf_block(const LpfBlock& a, int64_t r0, int64_t r1, int fg,
                                          uint32_t s0, uint32_t ns, uint32_t* part,
                                          uint32_t part_slot0, uint32_t* lds) {
    lpf_zero<PREC, W>(a.B, ns, lds);
    __syncthreads();
    lpf_accumulate<PREC, RM, W, MODE, BITS>(a, r0, r1, fg, s0, ns, lds);
    __syncthreads();
    lpf_flush<PREC, RM, W>(a, fg, s0, ns, part, part_slot0, lds);
}

}  // namespace cbh
