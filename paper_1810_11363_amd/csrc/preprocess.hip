// Feature binarization and ordered target statistics.
//
// Binarization (Sec. 5, "Dense numerical features"): bin = number of borders
// strictly below the value, found by a branch-free binary search over the
// borders staged in LDS.
//
// Ordered statistics (Sec. 2, Eq. 1; GPU method of Sec. 5, "Categorical
// features": group rows by category with a radix sort, then prefix-sum the
// statistic inside every group with a segmented scan):
//   1. key[p] = category of the row at permutation position p, payload = row;
//   2. stable LSD radix sort on the 32-bit key, 8 bits per pass, so rows of a
//      category stay in permutation order;
//   3. segment heads are positions where the key changes; an exclusive
//      segmented scan of 1 gives den, of the target numerator gives num
//      (operator transformation of Sengupta, Harris and Garland: pairs
//      (head flag, sum) combined as (f1|f2, f2 ? v2 : v1+v2));
//   4. results are scattered back to row order together with the statistic
//      value and its bin.
// The scan is reduce-then-scan over 4096-element tiles (three launches), so no
// block ever waits on another.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace cbh {

// ------------------------------------------------------------------ quantize
__global__ __launch_bounds__(256) void quantize_kernel(const float* __restrict__ x, int64_t n,
                                                       const float* __restrict__ borders,
                                                       int32_t nb, uint8_t* __restrict__ out,
                                                       uint32_t* __restrict__ flags) {
    __shared__ float sb[256];
    for (int i = threadIdx.x; i < 256; i += 256) sb[i] = i < nb ? borders[i] : INFINITY;
    __syncthreads();
    auto bin_of = [&](float v) -> uint32_t {
        uint32_t pos = 0;
#pragma unroll
        for (uint32_t step = 128; step >= 1; step >>= 1)
            if (sb[pos + step - 1] < v) pos += step;
        return pos;
    };
    bool nan_seen = false;
    const int64_t n4 = n / 4;
    const bool vec = ((reinterpret_cast<uintptr_t>(x) & 15) == 0) &&
                     ((reinterpret_cast<uintptr_t>(out) & 3) == 0);
    const int64_t tid = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t stride = int64_t(gridDim.x) * 256;
    if (vec) {
        for (int64_t q = tid; q < n4; q += stride) {
            float4 v = reinterpret_cast<const float4*>(x)[q];
            nan_seen |= (v.x != v.x) | (v.y != v.y) | (v.z != v.z) | (v.w != v.w);
            uint32_t w = bin_of(v.x) | (bin_of(v.y) << 8) | (bin_of(v.z) << 16) |
                         (bin_of(v.w) << 24);
            reinterpret_cast<uint32_t*>(out)[q] = w;
        }
        for (int64_t i = n4 * 4 + tid; i < n; i += stride) {
            float v = x[i];
            nan_seen |= (v != v);
            out[i] = (uint8_t)bin_of(v);
        }
    } else {
        for (int64_t i = tid; i < n; i += stride) {
            float v = x[i];
            nan_seen |= (v != v);
            out[i] = (uint8_t)bin_of(v);
        }
    }
    if (nan_seen) atomicOr(flags, FLAG_NAN_INPUT);
}

// ------------------------------------------------------------- radix sort
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kTile = kSortThreads * kSortItems;  // 4096 keys per block

// Per-tile digit counts, stored digit-major: counts[d * n_tiles + tile].
// OR of all keys, as kOrParts per-block partial ORs (no zeroing needed): a
// sort pass whose 8 digit bits are zero in every key is the identity.
constexpr int kOrParts = 1024;

__global__ __launch_bounds__(256) void key_or_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                                     uint32_t* __restrict__ parts) {
    __shared__ uint32_t wor[4];
    uint32_t v = 0u;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256)
        v |= keys[i];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v |= __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0) wor[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) parts[blockIdx.x] = wor[0] | wor[1] | wor[2] | wor[3];
}

// Whether the pass at `shift` sorts anything: some key has a nonzero digit
// there (always, without the partial ORs). Uniform over the block.
// (256 threads, 4 parts each.)
__device__ __forceinline__ bool pass_active(const uint32_t* parts, int shift) {
    static_assert(kOrParts == 4 * kSortThreads, "four partial ORs per thread");
    if (!parts) return true;
    const uint4 q = reinterpret_cast<const uint4*>(parts)[threadIdx.x];
    const uint32_t v = q.x | q.y | q.z | q.w;
    return __syncthreads_or(((v >> shift) & 255u) != 0u) != 0;
}

// Digit counts of one tile of kTile keys (zeros for an identity pass).
__global__ __launch_bounds__(kSortThreads) void radix_count_kernel(
    const uint32_t* __restrict__ keys, int64_t n, int shift, int64_t n_tiles,
    int64_t* __restrict__ counts, const uint32_t* __restrict__ or_parts = nullptr) {
    __shared__ uint32_t c[256];
    if (!pass_active(or_parts, shift)) {
        counts[int64_t(threadIdx.x) * n_tiles + blockIdx.x] = 0;
        return;
    }
    c[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * kTile;
#pragma unroll 4
    for (int j = 0; j < kSortItems; ++j) {
        int64_t i = base + j * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&c[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    counts[int64_t(threadIdx.x) * n_tiles + blockIdx.x] = c[threadIdx.x];
}

// Scatter with stable in-tile ranks. Keys of a tile are visited in 16 rounds
// of 256 (round-major, thread-minor), so rank order equals input order. An
// identity pass copies the tile.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t* __restrict__ keys, const int32_t* __restrict__ vals, int64_t n, int shift,
    int64_t n_tiles, const int64_t* __restrict__ offsets, uint32_t* __restrict__ keys_out,
    int32_t* __restrict__ vals_out, const uint32_t* __restrict__ or_parts = nullptr) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[4][256];
    const int64_t base = int64_t(blockIdx.x) * kTile;
    if (!pass_active(or_parts, shift)) {
        for (int j = 0; j < kSortItems; ++j) {
            const int64_t i = base + j * kSortThreads + threadIdx.x;
            if (i < n) {
                keys_out[i] = keys[i];
                vals_out[i] = vals[i];
            }
        }
        return;
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    run[threadIdx.x] = 0;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int64_t goff = offsets[int64_t(threadIdx.x) * n_tiles + blockIdx.x];
    __shared__ int64_t gbase[256];
    gbase[threadIdx.x] = goff;
    for (int j = 0; j < kSortItems; ++j) {
        for (int w = 0; w < 4; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        const int64_t i = base + j * kSortThreads + threadIdx.x;
        const bool act = i < n;
        uint32_t key = act ? keys[i] : 0u;
        int32_t val = act ? vals[i] : 0;
        uint32_t d = (key >> shift) & 255u;
        uint64_t same = __ballot(act);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t m = __ballot(((d >> b) & 1u) != 0u);
            same &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank_w = __popcll(same & lt_mask);
        // the lowest lane of each digit group publishes the group size
        if (act && rank_w == 0) wcnt[wave][d] = __popcll(same);
        __syncthreads();
        if (act) {
            uint32_t before = run[d];
            for (int w = 0; w < wave; ++w) before += wcnt[w][d];
            const int64_t dst = gbase[d] + before + rank_w;
            if (dst >= 0 && dst < n) {   // always true when the offsets are consistent
                keys_out[dst] = key;
                vals_out[dst] = val;
            }
        }
        __syncthreads();
        run[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] + wcnt[2][threadIdx.x] +
                            wcnt[3][threadIdx.x];
        __syncthreads();
    }
}

__global__ void gather_keys_kernel(const int32_t* __restrict__ cat,
                                   const int32_t* __restrict__ perm, int64_t n,
                                   uint32_t* __restrict__ keys, int32_t* __restrict__ vals,
                                   uint32_t* __restrict__ flags) {
    bool bad = false;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n;
         p += int64_t(gridDim.x) * blockDim.x) {
        int32_t r = perm[p];
        if (r < 0 || r >= n) {   // not a permutation: report, and keep every access in bounds
            bad = true;
            r = 0;
        }
        keys[p] = (uint32_t)cat[r];
        vals[p] = r;
    }
    if (bad) atomicOr(flags, FLAG_BAD_INDEX);
}

// ---------------------------------------------------------- segmented scan
// Element i contributes (head_i, v_i). Modes:
//   0: v = values[i] (plain values array), head = (i == 0)
//   1: v = 1, head = key change
//   2: v = y[vals[i]], head = key change
//   3: v = 1, head = heads[i]
//   4: v = y[vals[i]], head = heads[i]
//   5: v = values[i], head = heads[i]
struct ScanSrc {
    int mode;
    const int64_t* values;
    const uint32_t* keys;
    const int32_t* vals;
    const int64_t* y;
    const uint8_t* heads = nullptr;
};

struct SegPair {
    int64_t v;
    int f;
};

__device__ __forceinline__ SegPair seg_op(SegPair a, SegPair b) {
    return SegPair{b.f ? b.v : a.v + b.v, a.f | b.f};
}

__device__ __forceinline__ SegPair load_elem(const ScanSrc& s, int64_t i) {
    if (s.mode == 0) return SegPair{s.values[i], i == 0};
    int head = s.mode >= 3 ? (int)s.heads[i] : ((i == 0) || (s.keys[i] != s.keys[i - 1]));
    int64_t v = (s.mode == 1 || s.mode == 3) ? 1 : (s.mode == 5 ? s.values[i] : s.y[s.vals[i]]);
    return SegPair{v, head};
}

__device__ __forceinline__ SegPair shfl_up_pair(SegPair p, int d) {
    SegPair q;
    q.v = __shfl_up(p.v, d, 64);
    q.f = __shfl_up(p.f, d, 64);
    return q;
}

// Inclusive block scan of one pair per thread (thread order); returns the
// inclusive value of this thread; *total gets the block aggregate.
__device__ SegPair block_scan(SegPair x, SegPair* total) {
    __shared__ SegPair wsum[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        SegPair y = shfl_up_pair(x, d);
        if (lane >= d) x = seg_op(y, x);
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    SegPair pre{0, 0};
    for (int w = 0; w < wave; ++w) pre = seg_op(pre, wsum[w]);
    if (wave > 0) x = seg_op(pre, x);
    SegPair tot{0, 0};
    for (int w = 0; w < 4; ++w) tot = seg_op(tot, wsum[w]);
    *total = tot;
    __syncthreads();
    return x;
}

// Inclusive segmented scan over the 64 lanes of a wave (lane order).
__device__ __forceinline__ SegPair wave_incl_scan(SegPair x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        SegPair y = shfl_up_pair(x, d);
        if (lane >= d) x = seg_op(y, x);
    }
    return x;
}

__device__ __forceinline__ SegPair lane63(SegPair x) {
    return SegPair{__shfl(x.v, 63, 64), __shfl(x.f, 63, 64)};
}

// A tile of kTile elements: wave w takes the w-th quarter, 64 consecutive
// elements per step (one per lane, so every load is coalesced), 16 steps.
constexpr int kScanSteps = kTile / (4 * 64);

__global__ __launch_bounds__(256) void seg_reduce_kernel(ScanSrc src, int64_t n,
                                                         SegPair* __restrict__ agg) {
    __shared__ SegPair wagg[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t wbase = int64_t(blockIdx.x) * kTile + int64_t(wave) * (kTile / 4);
    SegPair run{0, 0};
    for (int j = 0; j < kScanSteps; ++j) {
        const int64_t i = wbase + j * 64 + lane;
        const SegPair x = wave_incl_scan(i < n ? load_elem(src, i) : SegPair{0, 0});
        run = seg_op(run, lane63(x));
    }
    if (lane == 0) wagg[wave] = run;
    __syncthreads();
    if (threadIdx.x == 0)
        agg[blockIdx.x] = seg_op(seg_op(seg_op(wagg[0], wagg[1]), wagg[2]), wagg[3]);
}

// Exclusive scan of the tile aggregates by one block; carry[t] is the value
// carried into tile t.
__global__ __launch_bounds__(256) void seg_carry_kernel(const SegPair* __restrict__ agg,
                                                        int64_t n_tiles,
                                                        int64_t* __restrict__ carry) {
    const int64_t per = (n_tiles + 255) / 256;
    const int64_t b0 = int64_t(threadIdx.x) * per;
    SegPair acc{0, 0};
    for (int64_t t = b0; t < b0 + per && t < n_tiles; ++t) acc = seg_op(acc, agg[t]);
    SegPair tot;
    SegPair inc = block_scan(acc, &tot);
    // exclusive prefix for this thread's range
    SegPair ex = shfl_up_pair(inc, 1);
    __shared__ SegPair last[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 63) last[wave] = inc;
    __syncthreads();
    if (lane == 0) ex = (wave == 0) ? SegPair{0, 0} : last[wave - 1];
    SegPair run = ex;
    for (int64_t t = b0; t < b0 + per && t < n_tiles; ++t) {
        carry[t] = run.v;
        run = seg_op(run, agg[t]);
    }
}

// Exclusive segmented scan written in sorted order (0 at a segment head),
// the tile laid out over the waves as in seg_reduce_kernel: each step's
// inclusive wave scan stays in registers until the prefix of the tile's
// earlier elements (the carry, then the earlier waves) is known.
__global__ __launch_bounds__(256) void seg_scan_kernel(ScanSrc src, int64_t n,
                                                       const int64_t* __restrict__ carry,
                                                       int64_t* __restrict__ out) {
    __shared__ SegPair wagg[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t wbase = int64_t(blockIdx.x) * kTile + int64_t(wave) * (kTile / 4);
    SegPair inc[kScanSteps];
    uint32_t heads = 0u;
    SegPair run{0, 0};
#pragma unroll
    for (int j = 0; j < kScanSteps; ++j) {
        const int64_t i = wbase + j * 64 + lane;
        const SegPair x = i < n ? load_elem(src, i) : SegPair{0, 0};
        heads |= uint32_t(x.f != 0) << j;
        inc[j] = wave_incl_scan(x);
        run = seg_op(run, lane63(inc[j]));
    }
    if (lane == 0) wagg[wave] = run;
    __syncthreads();
    SegPair pre{carry[blockIdx.x], 0};
    for (int w = 0; w < wave; ++w) pre = seg_op(pre, wagg[w]);
#pragma unroll
    for (int j = 0; j < kScanSteps; ++j) {
        const int64_t i = wbase + j * 64 + lane;
        SegPair ex = shfl_up_pair(inc[j], 1);
        if (lane == 0) ex = SegPair{0, 0};
        const SegPair before = seg_op(pre, ex);
        if (i < n) out[i] = ((heads >> j) & 1u) ? 0 : before.v;
        pre = seg_op(pre, lane63(inc[j]));
    }
}

// Scatter num/den back to row order, with the statistic value and its bin.
__global__ __launch_bounds__(256) void ts_scatter_kernel(
    const int32_t* __restrict__ rows, const int64_t* __restrict__ den_sorted,
    const int64_t* __restrict__ num_sorted, int64_t n, int32_t y_shift, double a, double ap,
    const double* __restrict__ tsb, int32_t ntsb, int64_t* __restrict__ num_out,
    int32_t* __restrict__ den_out, uint8_t* __restrict__ bin_out, double* __restrict__ ts_out) {
    __shared__ double sb[256];
    for (int i = threadIdx.x; i < 256; i += 256) sb[i] = (i < ntsb) ? tsb[i] : INFINITY;
    __syncthreads();
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        const int32_t r = rows[i];
        if (r < 0 || r >= n) continue;
        const int64_t den = den_sorted[i];
        if (den_out) den_out[r] = (int32_t)den;
        if (!num_sorted) continue;
        const int64_t num = num_sorted[i];
        if (num_out) num_out[r] = num;
        if (ts_out || bin_out) {
            // (num * 2^-e + a * P) / (den + a), operation order fixed, no contraction
            const double t = (ldexp((double)num, -y_shift) + ap) / ((double)den + a);
            if (ts_out) ts_out[r] = t;
            if (bin_out) {
                uint32_t pos = 0;
#pragma unroll
                for (uint32_t step = 128; step >= 1; step >>= 1)
                    if (sb[pos + step - 1] < t) pos += step;
                bin_out[r] = (uint8_t)pos;
            }
        }
    }
}

// ------------------------------------------------------------- tile bins
// Unit u = (column c, segment t), t fastest, so a wave reads one column
// contiguously; each unit writes its 16 bytes to out + (t * n_cols + c) * 16.
__global__ __launch_bounds__(256) void tile_bins_kernel(const uint8_t* const* __restrict__ cols,
                                                        int32_t n_cols, int64_t n, int64_t T,
                                                        uint8_t* __restrict__ out) {
    const int64_t units = T * n_cols;
    for (int64_t u = int64_t(blockIdx.x) * 256 + threadIdx.x; u < units;
         u += int64_t(gridDim.x) * 256) {
        const int32_t c = (int32_t)(u / T);
        const int64_t t = u - int64_t(c) * T;
        const uint8_t* src = cols[c] + 16 * t;
        uint4 v;
        if (16 * t + 16 <= n && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
            v = *reinterpret_cast<const uint4*>(src);
        } else {
            uint32_t w[4] = {0u, 0u, 0u, 0u};
            for (int r = 0; r < 16; ++r)
                if (16 * t + r < n) w[r >> 2] |= (uint32_t)src[r] << (8 * (r & 3));
            v = make_uint4(w[0], w[1], w[2], w[3]);
        }
        *reinterpret_cast<uint4*>(out + (t * n_cols + c) * 16) = v;
    }
}

// Dense ids of category pairs, the perfect hash the paper applies to
// combinations of categorical features (Sec. 2, "Feature combinations": the
// values of a combination get ids on the fly; Sec. 5, "Categorical
// features": perfect hashes built with a radix sort). The combination's
// ordered statistics are then computed like those of one feature. Rows are sorted by (a, b) as unsigned 32-bit values with two
// rounds of the stable LSD radix sort (by b, then by a), a row starts a new
// id where its pair differs from the previous row's, and an exclusive scan
// of those starts numbers the ids in increasing pair order.
__global__ void pair_first_keys_kernel(const int32_t* __restrict__ b, int64_t n,
                                       uint32_t* __restrict__ keys, int32_t* __restrict__ rows) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        keys[i] = (uint32_t)b[i];
        rows[i] = (int32_t)i;
    }
}

__global__ void pair_second_keys_kernel(const int32_t* __restrict__ a,
                                        const int32_t* __restrict__ rows, int64_t n,
                                        uint32_t* __restrict__ keys) {
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n;
         p += int64_t(gridDim.x) * blockDim.x)
        keys[p] = (uint32_t)a[rows[p]];
}

// A row starts a new id where its pair differs from the previous row's: a
// comes sorted from the second sort; b is gathered once per row, and the
// previous row's b comes from the neighbouring lane (first lane of a wave:
// a second gather).
__global__ __launch_bounds__(256) void pair_heads_kernel(const uint32_t* __restrict__ a_sorted,
                                                         const int32_t* __restrict__ b,
                                                         const int32_t* __restrict__ rows,
                                                         int64_t n, int64_t* __restrict__ head) {
    const int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const bool act = p < n;
    const int32_t bp = act ? b[rows[p]] : 0;
    int32_t bq = __shfl_up(bp, 1, 64);
    if (act && p > 0 && (threadIdx.x & 63) == 0) bq = b[rows[p - 1]];
    if (act) head[p] = (p == 0 || a_sorted[p] != a_sorted[p - 1] || bp != bq) ? 1 : 0;
}

__global__ void pair_ids_kernel(const int32_t* __restrict__ rows, const int64_t* __restrict__ head,
                                const int64_t* __restrict__ excl, int64_t n,
                                int32_t* __restrict__ ids, int64_t* __restrict__ n_distinct) {
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n;
         p += int64_t(gridDim.x) * blockDim.x) {
        ids[rows[p]] = (int32_t)(excl[p] + head[p] - 1);
        if (p == n - 1) *n_distinct = excl[p] + head[p];
    }
}

// The counter statistic (Sec. 2: a category, or a combination of
// categories, replaced by its number of appearances in the dataset): per
// dense id, the number of rows that carry it, then that count per row.
__global__ void zero_i32_kernel(int32_t* __restrict__ p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0;
}

// Frequent ids (a Zipf-distributed category) would serialise many atomics
// on one address: the lanes of a wave that share the id of its first
// pending lane add their count with one atomic, up to four ids per wave
// step; the rest add one each.
__global__ void id_count_kernel(const int32_t* __restrict__ ids, int64_t n,
                                int32_t* __restrict__ cnt, uint32_t* __restrict__ flags) {
    bool bad = false;
    const int lane = threadIdx.x & 63;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int32_t v = ids[i];
        bool pending = true;
        if (v < 0 || v >= n) {
            bad = true;
            pending = false;
        }
        for (int it = 0; it < 4; ++it) {
            const uint64_t act = __ballot(pending);
            if (act == 0) break;
            const int leader = __ffsll((unsigned long long)act) - 1;
            const int32_t lv = __shfl(v, leader, 64);
            const bool mine = pending && v == lv;
            const uint64_t same = __ballot(mine);
            if (mine) {
                if (lane == leader) atomicAdd(&cnt[lv], (int32_t)__popcll(same));
                pending = false;
            }
        }
        if (pending) atomicAdd(&cnt[v], 1);
    }
    if (bad) atomicOr(flags, FLAG_BAD_INDEX);
}

__global__ void id_count_gather_kernel(const int32_t* __restrict__ ids, int64_t n,
                                       const int32_t* __restrict__ cnt,
                                       int32_t* __restrict__ out) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int32_t v = ids[i];
        out[i] = (v >= 0 && v < n) ? cnt[v] : 0;
    }
}

// ------------------------------------------------ crossings of categories
// A row starts a new category where its sorted key differs from the previous.
__global__ void key_heads_kernel(const uint32_t* __restrict__ keys, int64_t n,
                                 int64_t* __restrict__ head) {
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n;
         p += int64_t(gridDim.x) * blockDim.x)
        head[p] = (p == 0 || keys[p] != keys[p - 1]) ? 1 : 0;
}

// Crossing k (blockIdx.y) of n rows: element j = k n + i takes row order[k][i]
// (the rows in order of (category of crossing k, position)); its key is
// (e[row] << k_bits) | k, so a stable sort on the key orders the elements by
// (e, crossing, category, position): every (crossing, e, category) group is
// contiguous and in position order. With e in the high bits, the passes over
// e's unused high digits (a one-bit split value) find only zeros.
__global__ void cross_keys_kernel(const int32_t* __restrict__ e, int32_t e_bits, int32_t k_bits,
                                  const int32_t* const* __restrict__ order, int64_t n,
                                  uint32_t* __restrict__ keys, int32_t* __restrict__ rows,
                                  uint32_t* __restrict__ flags) {
    const int k = blockIdx.y;
    const int32_t* ord = order[k];
    const uint32_t emax = e_bits >= 32 ? 0xffffffffu : ((1u << e_bits) - 1u);
    bool bad = false;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        int32_t r = ord[i];
        if (r < 0 || r >= n) {
            bad = true;
            r = 0;
        }
        uint32_t v = (uint32_t)e[r];
        if (v > emax) {
            bad = true;
            v &= emax;
        }
        const int64_t j = int64_t(k) * n + i;
        keys[j] = (v << k_bits) | (uint32_t)k;
        rows[j] = r;
    }
    if (bad) atomicOr(flags, FLAG_BAD_INDEX);
}

// A sorted element starts a new group where its key (crossing, e) or its
// category in that crossing differs from the previous element's. Each thread
// gathers its own element's category once; the previous element's comes
// from LDS (from global memory for a block's first element).
__global__ __launch_bounds__(256) void cross_heads_kernel(
    const uint32_t* __restrict__ keys, const int32_t* __restrict__ rows,
    const int32_t* const* __restrict__ cids, int32_t k_bits, int64_t N,
    uint8_t* __restrict__ head) {
    const uint32_t kmask = (1u << k_bits) - 1u;
    __shared__ int32_t sc[256];
    __shared__ uint32_t sk[256];
    for (int64_t base = int64_t(blockIdx.x) * 256; base < N; base += int64_t(gridDim.x) * 256) {
        const int64_t p = base + threadIdx.x;
        uint32_t key = 0u;
        int32_t c = 0;
        if (p < N) {
            key = keys[p];
            c = cids[key & kmask][rows[p]];
        }
        sk[threadIdx.x] = key;
        sc[threadIdx.x] = c;
        __syncthreads();
        if (p < N) {
            bool h = p == 0;
            if (!h) {
                uint32_t pk;
                int32_t pc;
                if (threadIdx.x > 0) {
                    pk = sk[threadIdx.x - 1];
                    pc = sc[threadIdx.x - 1];
                } else {
                    pk = keys[p - 1];
                    pc = pk == key ? cids[pk & kmask][rows[p - 1]] : c;
                }
                h = pk != key || pc != c;
            }
            head[p] = h ? 1 : 0;
        }
        __syncthreads();
    }
}

struct CrossPriors {
    double ap[8];     // a * prior of every prior of the target
};

// Statistic bins of every sorted element for target t and each prior q:
// ts = (num 2^-y_shift + a P_q) / (den + a), in this order, its bin the
// number of borders strictly below it. They go to the element's record of
// stride bytes, rec[(k n + row) stride + t Q + q], so that the bytes of one
// element land in one cache line (the rows are in random order here: one
// byte per column would cost a partial line write each). With counters
// (size_at_start != NULL, on the last target) the record's byte counter_col
// gets the counter bin of the element's group: floor(log2(size)) capped at
// counter_bins - 1, the group starting at p - den[p]. WHOLE: this pass
// fills the whole record (one target), written as 32-bit words (the stride
// a multiple of 4, at most 12 bytes).
template <bool WHOLE>
__global__ __launch_bounds__(256) void cross_scatter_kernel(
    const uint32_t* __restrict__ keys, const int32_t* __restrict__ rows,
    const int64_t* __restrict__ den_s, const int64_t* __restrict__ num_s, int64_t N, int64_t n,
    int32_t k_bits, int32_t y_shift, double a, CrossPriors pri, int32_t Q, int32_t t,
    const double* __restrict__ tsb, int32_t ntsb, const uint32_t* __restrict__ size_at_start,
    int32_t counter_bins, int32_t counter_col, uint8_t* __restrict__ rec, int32_t stride) {
    __shared__ double sb[256];
    sb[threadIdx.x] = (int32_t(threadIdx.x) < ntsb) ? tsb[threadIdx.x] : INFINITY;
    __syncthreads();
    for (int64_t p = int64_t(blockIdx.x) * 256 + threadIdx.x; p < N;
         p += int64_t(gridDim.x) * 256) {
        const int k = (int)(keys[p] & ((1u << k_bits) - 1u));
        const int32_t r = rows[p];
        const int64_t d = den_s[p];
        const double num = ldexp((double)num_s[p], -y_shift);
        const double den = (double)d + a;
        uint8_t* o = rec + (int64_t(k) * n + r) * stride;
        uint32_t wd[3] = {0u, 0u, 0u};
        for (int q = 0; q < Q; ++q) {
            const double ts = (num + pri.ap[q]) / den;
            uint32_t pos = 0;
#pragma unroll
            for (uint32_t step = 128; step >= 1; step >>= 1)
                if (sb[pos + step - 1] < ts) pos += step;
            if constexpr (WHOLE) {
                const int c = t * Q + q;
                wd[c >> 2] |= pos << (8 * (c & 3));
            } else {
                o[t * Q + q] = (uint8_t)pos;
            }
        }
        if (size_at_start) {
            const uint32_t c = size_at_start[p - d];
            const int b = min(c ? 31 - __clz(c) : 0, counter_bins - 1);
            if constexpr (WHOLE)
                wd[counter_col >> 2] |= uint32_t(b) << (8 * (counter_col & 3));
            else
                o[counter_col] = (uint8_t)b;
        }
        if constexpr (WHOLE) {
            uint32_t* ow = reinterpret_cast<uint32_t*>(o);
            for (int j = 0; j < (stride >> 2); ++j) ow[j] = wd[j];
        }
    }
}

// The counter statistic of every crossing's groups (Sec. 2): the group
// of sorted element p starts at p - den[p] (den: its exclusive index in the
// group); the group's last element records the group's size at the start.
__global__ void cross_group_size_kernel(const uint8_t* __restrict__ head,
                                        const int64_t* __restrict__ den_s, int64_t N,
                                        uint32_t* __restrict__ size_at_start) {
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < N;
         p += int64_t(gridDim.x) * blockDim.x) {
        if (p == N - 1 || head[p + 1]) size_at_start[p - den_s[p]] = (uint32_t)(den_s[p] + 1);
    }
}

// The target of every sorted element in sorted order, ys[p] = y[rows[p]]:
// one random gather, so that both passes of the segmented scan read ys
// contiguously.
__global__ void cross_gather_y_kernel(const int32_t* __restrict__ rows,
                                      const int64_t* __restrict__ y, int64_t N,
                                      int64_t* __restrict__ ys) {
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < N;
         p += int64_t(gridDim.x) * blockDim.x)
        ys[p] = y[rows[p]];
}

// Records to columns: out[k][c ld + row] = rec[(k n + row) stride + c] for
// the cpc columns; one thread per row of crossing k = blockIdx.y, so every
// column's writes are consecutive bytes.
__global__ __launch_bounds__(256) void cross_unpack_kernel(const uint8_t* __restrict__ rec,
                                                           int64_t n, int32_t cpc,
                                                           int32_t stride,
                                                           uint8_t* const* __restrict__ out,
                                                           int64_t ld) {
    const int k = blockIdx.y;
    uint8_t* ok = out[k];
    const uint8_t* rk = rec + int64_t(k) * n * stride;
    for (int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x; r < n;
         r += int64_t(gridDim.x) * 256) {
        const uint8_t* src = rk + r * stride;
        for (int c = 0; c < cpc; ++c) ok[int64_t(c) * ld + r] = src[c];
    }
}

static int grid_for(int64_t n, int per_block, int cap = 16384) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace cbh

using namespace cbh;

extern "C" {

int cbh_quantize(cbh_ctx* ctx, const float* x, int64_t n, const float* borders,
                 int32_t n_borders, uint8_t* bins_out, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0, "n must be >= 0");
    CBH_REQUIRE(n_borders >= 0 && n_borders <= 255, CBH_EUNSUPPORTED,
                "n_borders must be in [0, 255] (got %d)", n_borders);
    if (n == 0) return CBH_OK;
    CBH_ARG(x && bins_out, "x / bins_out is NULL");
    CBH_ARG(n_borders == 0 || borders, "borders is NULL");
    hipStream_t s = (hipStream_t)stream;
    quantize_kernel<<<grid_for((n + 3) / 4, 256, ctx->num_cus * 8), 256, 0, s>>>(
        x, n, borders, n_borders, bins_out, ctx->d_flags);
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_tile_bins(cbh_ctx* ctx, const uint8_t* const* cols, int32_t n_cols, int64_t n,
                  uint8_t* out, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(cols && out, "cols / out is NULL");
    CBH_ARG(n >= 1, "n must be >= 1");
    CBH_ARG(n_cols >= 1 && n_cols <= 65535, "n_cols must be in [1, 65535] (got %d)", n_cols);
    CBH_ARG((reinterpret_cast<uintptr_t>(out) & 15) == 0, "out must be 16-byte aligned");
    const int64_t T = (n + 15) / 16;
    tile_bins_kernel<<<grid_for(T * n_cols, 256, ctx->num_cus * 8), 256, 0,
                       (hipStream_t)stream>>>(cols, n_cols, n, T, out);
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_compute_ordered_ts(cbh_ctx* ctx, const int32_t* cat, const int32_t* perm, int64_t n,
                           const int64_t* y_num, int32_t n_targets, int32_t y_shift,
                           int64_t y_abs_max, double a, const double* priors,
                           const double* ts_borders, int32_t n_ts_borders, int64_t* num_out,
                           int32_t* den_out, uint8_t* ts_bin_out, double* ts_out,
                           void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0 && n < (int64_t(1) << 31), "n must be in [0, 2^31)");
    CBH_ARG(n_targets >= 1 && n_targets <= 16, "n_targets must be in [1, 16]");
    CBH_ARG(y_shift >= 0 && y_shift <= 62, "y_shift must be in [0, 62]");
    CBH_ARG(y_abs_max >= 0, "y_abs_max must be >= 0");
    CBH_ARG(a > 0 && std::isfinite(a), "prior weight a must be finite and > 0");
    CBH_ARG(priors != nullptr, "priors is NULL");
    for (int t = 0; t < n_targets; ++t) CBH_ARG(std::isfinite(priors[t]), "prior not finite");
    CBH_REQUIRE(n_ts_borders >= 0 && n_ts_borders <= 255, CBH_EUNSUPPORTED,
                "n_ts_borders must be in [0, 255]");
    CBH_ARG(ts_bin_out == nullptr || n_ts_borders == 0 || ts_borders != nullptr,
            "ts_borders is NULL");
    CBH_REQUIRE(y_abs_max == 0 || (double)n * (double)y_abs_max < 4.611686018427387904e18,
                CBH_EOVERFLOW, "n * y_abs_max must be < 2^62 for exact int64 sums");
    if (n == 0) return CBH_OK;
    CBH_ARG(cat && perm && y_num, "cat / perm / y_num is NULL");
    const bool need_num = num_out || ts_bin_out || ts_out;

    const int64_t n_tiles = (n + kTile - 1) / kTile;
    const int64_t cnt_elems = 256 * n_tiles;
    const int64_t cnt_tiles = (cnt_elems + kTile - 1) / kTile;
    const int64_t max_tiles = std::max(n_tiles, cnt_tiles);
    // workspace: keys x2, vals x2, den, num, counts, aggregates, carries
    int64_t off = 0;
    auto take = [&](int64_t bytes) { int64_t o = off; off += align_up(bytes, 256); return o; };
    const int64_t o_k0 = take(4 * n), o_k1 = take(4 * n), o_v0 = take(4 * n),
                  o_v1 = take(4 * n), o_den = take(8 * n), o_num = take(8 * n),
                  o_cnt = take(8 * cnt_elems), o_off = take(8 * cnt_elems),
                  o_agg = take(sizeof(SegPair) * max_tiles), o_car = take(8 * max_tiles);
    int rc = ensure_ws(ctx, off, stream);
    if (rc != CBH_OK) return rc;
    char* w = (char*)ctx->ws;
    uint32_t* keys[2] = {(uint32_t*)(w + o_k0), (uint32_t*)(w + o_k1)};
    int32_t* vals[2] = {(int32_t*)(w + o_v0), (int32_t*)(w + o_v1)};
    int64_t* den_s = (int64_t*)(w + o_den);
    int64_t* num_s = (int64_t*)(w + o_num);
    int64_t* counts = (int64_t*)(w + o_cnt);
    int64_t* offs = (int64_t*)(w + o_off);
    SegPair* agg = (SegPair*)(w + o_agg);
    int64_t* car = (int64_t*)(w + o_car);
    hipStream_t s = (hipStream_t)stream;

    auto scan = [&](ScanSrc src, int64_t len, int64_t* out) -> int {
        const int64_t tiles = (len + kTile - 1) / kTile;
        seg_reduce_kernel<<<(unsigned)tiles, 256, 0, s>>>(src, len, agg);
        seg_carry_kernel<<<1, 256, 0, s>>>(agg, tiles, car);
        seg_scan_kernel<<<(unsigned)tiles, 256, 0, s>>>(src, len, car, out);
        CBH_LAUNCHED();
        return CBH_OK;
    };

    gather_keys_kernel<<<grid_for(n, 256, ctx->num_cus * 8), 256, 0, s>>>(cat, perm, n, keys[0],
                                                                           vals[0], ctx->d_flags);
    CBH_LAUNCHED();
    int cur = 0;
    for (int shift = 0; shift < 32; shift += 8) {
        radix_count_kernel<<<(unsigned)n_tiles, kSortThreads, 0, s>>>(keys[cur], n, shift,
                                                                      n_tiles, counts);
        CBH_LAUNCHED();
        rc = scan(ScanSrc{0, counts, nullptr, nullptr, nullptr}, cnt_elems, offs);
        if (rc != CBH_OK) return rc;
        radix_scatter_kernel<<<(unsigned)n_tiles, kSortThreads, 0, s>>>(
            keys[cur], vals[cur], n, shift, n_tiles, offs, keys[cur ^ 1], vals[cur ^ 1]);
        CBH_LAUNCHED();
        cur ^= 1;
    }
    const uint32_t* sk = keys[cur];
    const int32_t* sv = vals[cur];
    rc = scan(ScanSrc{1, nullptr, sk, sv, nullptr}, n, den_s);
    if (rc != CBH_OK) return rc;
    const int gs = grid_for(n, 256, ctx->num_cus * 8);
    if (!need_num) {
        ts_scatter_kernel<<<gs, 256, 0, s>>>(sv, den_s, nullptr, n, 0, a, 0.0, nullptr, 0,
                                             nullptr, den_out, nullptr, nullptr);
        CBH_LAUNCHED();
        return CBH_OK;
    }
    for (int t = 0; t < n_targets; ++t) {
        rc = scan(ScanSrc{2, nullptr, sk, sv, y_num + int64_t(t) * n}, n, num_s);
        if (rc != CBH_OK) return rc;
        const double ap = a * priors[t];
        ts_scatter_kernel<<<gs, 256, 0, s>>>(
            sv, den_s, num_s, n, y_shift, a, ap, ts_borders, ts_bin_out ? n_ts_borders : 0,
            num_out ? num_out + int64_t(t) * n : nullptr, t == 0 ? den_out : nullptr,
            ts_bin_out ? ts_bin_out + int64_t(t) * n : nullptr,
            ts_out ? ts_out + int64_t(t) * n : nullptr);
        CBH_LAUNCHED();
    }
    return CBH_OK;
}

int cbh_combine_categories(cbh_ctx* ctx, const int32_t* cat_a, const int32_t* cat_b, int64_t n,
                           int32_t* ids_out, int64_t* n_distinct_out, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0 && n <= int64_t(INT32_MAX), "n must be in [0, 2^31 - 1]");
    if (n == 0) return CBH_OK;
    CBH_ARG(cat_a && cat_b && ids_out && n_distinct_out, "NULL argument");
    const int64_t n_tiles = (n + kTile - 1) / kTile;
    const int64_t cnt_elems = 256 * n_tiles;
    const int64_t cnt_tiles = (cnt_elems + kTile - 1) / kTile;
    const int64_t max_tiles = std::max(n_tiles, cnt_tiles);
    int64_t off = 0;
    auto take = [&](int64_t bytes) { int64_t o = off; off += align_up(bytes, 256); return o; };
    const int64_t o_k0 = take(4 * n), o_k1 = take(4 * n), o_v0 = take(4 * n),
                  o_v1 = take(4 * n), o_head = take(8 * n), o_excl = take(8 * n),
                  o_cnt = take(8 * cnt_elems), o_off = take(8 * cnt_elems),
                  o_agg = take(sizeof(SegPair) * max_tiles), o_car = take(8 * max_tiles),
                  o_or = take(4 * kOrParts);
    int rc = ensure_ws(ctx, off, stream);
    if (rc != CBH_OK) return rc;
    char* w = (char*)ctx->ws;
    uint32_t* keys[2] = {(uint32_t*)(w + o_k0), (uint32_t*)(w + o_k1)};
    int32_t* rows[2] = {(int32_t*)(w + o_v0), (int32_t*)(w + o_v1)};
    uint32_t* or_parts = (uint32_t*)(w + o_or);
    int64_t* head = (int64_t*)(w + o_head);
    int64_t* excl = (int64_t*)(w + o_excl);
    int64_t* counts = (int64_t*)(w + o_cnt);
    int64_t* offs = (int64_t*)(w + o_off);
    SegPair* agg = (SegPair*)(w + o_agg);
    int64_t* car = (int64_t*)(w + o_car);
    hipStream_t s = (hipStream_t)stream;
    auto scan = [&](const int64_t* values, int64_t len, int64_t* out) -> int {
        const int64_t tiles = (len + kTile - 1) / kTile;
        const ScanSrc src{0, values, nullptr, nullptr, nullptr};
        seg_reduce_kernel<<<(unsigned)tiles, 256, 0, s>>>(src, len, agg);
        seg_carry_kernel<<<1, 256, 0, s>>>(agg, tiles, car);
        seg_scan_kernel<<<(unsigned)tiles, 256, 0, s>>>(src, len, car, out);
        CBH_LAUNCHED();
        return CBH_OK;
    };
    int cur = 0;
    // passes over digits that are zero in every key (small category ids,
    // a one-bit split value) copy instead of sorting
    auto sort32 = [&]() -> int {
        key_or_kernel<<<kOrParts, 256, 0, s>>>(keys[cur], n, or_parts);
        CBH_LAUNCHED();
        for (int shift = 0; shift < 32; shift += 8) {
            radix_count_kernel<<<(unsigned)n_tiles, kSortThreads, 0, s>>>(
                keys[cur], n, shift, n_tiles, counts, or_parts);
            CBH_LAUNCHED();
            int r = scan(counts, cnt_elems, offs);
            if (r != CBH_OK) return r;
            radix_scatter_kernel<<<(unsigned)n_tiles, kSortThreads, 0, s>>>(
                keys[cur], rows[cur], n, shift, n_tiles, offs, keys[cur ^ 1], rows[cur ^ 1],
                or_parts);
            CBH_LAUNCHED();
            cur ^= 1;
        }
        return CBH_OK;
    };
    const int gs = grid_for(n, 256, ctx->num_cus * 8);
    pair_first_keys_kernel<<<gs, 256, 0, s>>>(cat_b, n, keys[0], rows[0]);
    CBH_LAUNCHED();
    rc = sort32();                       // rows by b
    if (rc != CBH_OK) return rc;
    pair_second_keys_kernel<<<gs, 256, 0, s>>>(cat_a, rows[cur], n, keys[cur]);
    CBH_LAUNCHED();
    rc = sort32();                       // then stably by a: rows by (a, b)
    if (rc != CBH_OK) return rc;
    pair_heads_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(keys[cur], cat_b, rows[cur],
                                                                   n, head);
    CBH_LAUNCHED();
    rc = scan(head, n, excl);
    if (rc != CBH_OK) return rc;
    pair_ids_kernel<<<gs, 256, 0, s>>>(rows[cur], head, excl, n, ids_out, n_distinct_out);
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_category_counts(cbh_ctx* ctx, const int32_t* ids, int64_t n, int32_t* counts_out,
                        void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0 && n <= int64_t(INT32_MAX), "n must be in [0, 2^31 - 1]");
    if (n == 0) return CBH_OK;
    CBH_ARG(ids && counts_out, "NULL argument");
    int rc = ensure_ws(ctx, 4 * n, stream);
    if (rc != CBH_OK) return rc;
    int32_t* cnt = (int32_t*)ctx->ws;
    hipStream_t s = (hipStream_t)stream;
    const int gs = grid_for(n, 256, ctx->num_cus * 8);
    zero_i32_kernel<<<gs, 256, 0, s>>>(cnt, n);
    CBH_LAUNCHED();
    id_count_kernel<<<gs, 256, 0, s>>>(ids, n, cnt, ctx->d_flags);
    CBH_LAUNCHED();
    id_count_gather_kernel<<<gs, 256, 0, s>>>(ids, n, cnt, counts_out);
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_category_order(cbh_ctx* ctx, const int32_t* cat, const int32_t* perm, int64_t n,
                       int32_t* order_out, int32_t* ids_out, int64_t* n_distinct_out,
                       void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0 && n <= int64_t(INT32_MAX), "n must be in [0, 2^31 - 1]");
    if (n == 0) return CBH_OK;
    CBH_ARG(cat && (order_out || ids_out), "NULL argument");
    const int64_t n_tiles = (n + kTile - 1) / kTile;
    const int64_t cnt_elems = 256 * n_tiles;
    const int64_t cnt_tiles = (cnt_elems + kTile - 1) / kTile;
    const int64_t max_tiles = std::max(n_tiles, cnt_tiles);
    int64_t off = 0;
    auto take = [&](int64_t bytes) { int64_t o = off; off += align_up(bytes, 256); return o; };
    const int64_t o_k0 = take(4 * n), o_k1 = take(4 * n), o_v0 = take(4 * n),
                  o_v1 = take(4 * n), o_head = take(8 * n), o_excl = take(8 * n),
                  o_cnt = take(8 * cnt_elems), o_off = take(8 * cnt_elems),
                  o_agg = take(sizeof(SegPair) * max_tiles), o_car = take(8 * max_tiles),
                  o_nd = take(8);
    int rc = ensure_ws(ctx, off, stream);
    if (rc != CBH_OK) return rc;
    char* w = (char*)ctx->ws;
    uint32_t* keys[2] = {(uint32_t*)(w + o_k0), (uint32_t*)(w + o_k1)};
    int32_t* rows[2] = {(int32_t*)(w + o_v0), (int32_t*)(w + o_v1)};
    int64_t* head = (int64_t*)(w + o_head);
    int64_t* excl = (int64_t*)(w + o_excl);
    int64_t* counts = (int64_t*)(w + o_cnt);
    int64_t* offs = (int64_t*)(w + o_off);
    SegPair* agg = (SegPair*)(w + o_agg);
    int64_t* car = (int64_t*)(w + o_car);
    hipStream_t s = (hipStream_t)stream;
    const int gs = grid_for(n, 256, ctx->num_cus * 8);
    if (perm) gather_keys_kernel<<<gs, 256, 0, s>>>(cat, perm, n, keys[0], rows[0], ctx->d_flags);
    else pair_first_keys_kernel<<<gs, 256, 0, s>>>(cat, n, keys[0], rows[0]);
    CBH_LAUNCHED();
    int cur = 0;
    for (int shift = 0; shift < 32; shift += 8) {
        radix_count_kernel<<<(unsigned)n_tiles, kSortThreads, 0, s>>>(keys[cur], n, shift,
                                                                      n_tiles, counts);
        CBH_LAUNCHED();
        const int64_t tiles = (cnt_elems + kTile - 1) / kTile;
        const ScanSrc src{0, counts, nullptr, nullptr, nullptr};
        seg_reduce_kernel<<<(unsigned)tiles, 256, 0, s>>>(src, cnt_elems, agg);
        seg_carry_kernel<<<1, 256, 0, s>>>(agg, tiles, car);
        seg_scan_kernel<<<(unsigned)tiles, 256, 0, s>>>(src, cnt_elems, car, offs);
        radix_scatter_kernel<<<(unsigned)n_tiles, kSortThreads, 0, s>>>(
            keys[cur], rows[cur], n, shift, n_tiles, offs, keys[cur ^ 1], rows[cur ^ 1]);
        CBH_LAUNCHED();
        cur ^= 1;
    }
    if (order_out)
        CBH_HIP(hipMemcpyAsync(order_out, rows[cur], 4 * n, hipMemcpyDeviceToDevice, s));
    if (ids_out || n_distinct_out) {
        key_heads_kernel<<<gs, 256, 0, s>>>(keys[cur], n, head);
        const ScanSrc src{0, head, nullptr, nullptr, nullptr};
        seg_reduce_kernel<<<(unsigned)n_tiles, 256, 0, s>>>(src, n, agg);
        seg_carry_kernel<<<1, 256, 0, s>>>(agg, n_tiles, car);
        seg_scan_kernel<<<(unsigned)n_tiles, 256, 0, s>>>(src, n, car, excl);
        // without ids_out the ids go to the sort's free key buffer
        int32_t* ids = ids_out ? ids_out : (int32_t*)keys[cur ^ 1];
        int64_t* nd = n_distinct_out ? n_distinct_out : (int64_t*)(w + o_nd);
        pair_ids_kernel<<<gs, 256, 0, s>>>(rows[cur], head, excl, n, ids, nd);
        CBH_LAUNCHED();
    }
    return CBH_OK;
}

int cbh_ordered_ts_crossings(cbh_ctx* ctx, const int32_t* e_ids, int32_t e_bits,
                             int32_t n_cross, const int32_t* const* c_order,
                             const int32_t* const* c_ids, int64_t n, const int64_t* y_num,
                             int32_t n_targets, int32_t y_shift, int64_t y_abs_max, double a,
                             int32_t n_priors, const double* priors, const double* ts_borders,
                             int32_t n_ts_borders, int32_t counter_bins,
                             uint8_t* const* ts_bin_out, int64_t ld, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0 && n <= int64_t(INT32_MAX), "n must be in [0, 2^31 - 1]");
    CBH_ARG(n_cross >= 1 && n_cross <= 4096, "n_cross must be in [1, 4096]");
    CBH_ARG(e_bits >= 0 && e_bits <= 32, "e_bits must be in [0, 32]");
    int k_bits = 0;
    while ((1 << k_bits) < n_cross) ++k_bits;
    CBH_REQUIRE(e_bits + k_bits <= 32, CBH_EUNSUPPORTED,
                "e_bits + bits of the crossing index must be <= 32 (got %d + %d)", e_bits,
                k_bits);
    CBH_REQUIRE(n == 0 || int64_t(n_cross) * n <= int64_t(INT32_MAX), CBH_EUNSUPPORTED,
                "n_cross * n must be < 2^31");
    CBH_ARG(n_targets >= 1 && n_targets <= 16, "n_targets must be in [1, 16]");
    CBH_ARG(n_priors >= 1 && n_priors <= 8, "n_priors must be in [1, 8]");
    CBH_ARG(y_shift >= 0 && y_shift <= 62, "y_shift must be in [0, 62]");
    CBH_ARG(y_abs_max >= 0, "y_abs_max must be >= 0");
    CBH_ARG(a > 0 && std::isfinite(a), "prior weight a must be finite and > 0");
    CBH_REQUIRE(n_ts_borders >= 0 && n_ts_borders <= 255, CBH_EUNSUPPORTED,
                "n_ts_borders must be in [0, 255]");
    CBH_REQUIRE(y_abs_max == 0 || (double)n * (double)y_abs_max < 4.611686018427387904e18,
                CBH_EOVERFLOW, "n * y_abs_max must be < 2^62 for exact int64 sums");
    CBH_ARG(ld >= n, "ld must be >= n");
    CBH_ARG(counter_bins >= 0 && counter_bins <= 256, "counter_bins must be in [0, 256]");
    if (n == 0) return CBH_OK;
    CBH_ARG(e_ids && c_order && c_ids && y_num && priors && ts_bin_out, "NULL argument");
    CBH_ARG(n_ts_borders == 0 || ts_borders, "ts_borders is NULL");
    for (int i = 0; i < n_targets * n_priors; ++i)
        CBH_ARG(std::isfinite(priors[i]), "prior not finite");
    const int64_t N = int64_t(n_cross) * n;
    const int64_t n_tiles = (N + kTile - 1) / kTile;
    const int64_t cnt_elems = 256 * n_tiles;
    const int64_t cnt_tiles = (cnt_elems + kTile - 1) / kTile;
    const int64_t max_tiles = std::max(n_tiles, cnt_tiles);
    int64_t off = 0;
    auto take = [&](int64_t bytes) { int64_t o = off; off += align_up(bytes, 256); return o; };
    const int64_t o_k0 = take(4 * N), o_k1 = take(4 * N), o_v0 = take(4 * N),
                  o_v1 = take(4 * N), o_head = take(N), o_den = take(8 * N),
                  o_num = take(8 * N), o_cnt = take(8 * cnt_elems), o_off = take(8 * cnt_elems),
                  o_agg = take(sizeof(SegPair) * max_tiles), o_car = take(8 * max_tiles);
    const int32_t cpc = n_targets * n_priors + (counter_bins > 0 ? 1 : 0);
    // one target fills a record at once: 32-bit words (at most 9 bytes)
    const bool whole = n_targets == 1;
    const int32_t stride = whole ? (cpc + 3) / 4 * 4 : cpc;
    const int64_t o_rec = take(int64_t(stride) * N), o_ys = take(8 * N),
                  o_or = take(4 * kOrParts);
    int rc = ensure_ws(ctx, off, stream);
    if (rc != CBH_OK) return rc;
    char* w = (char*)ctx->ws;
    uint32_t* keys[2] = {(uint32_t*)(w + o_k0), (uint32_t*)(w + o_k1)};
    int32_t* rows[2] = {(int32_t*)(w + o_v0), (int32_t*)(w + o_v1)};
    uint8_t* head = (uint8_t*)(w + o_head);
    int64_t* den_s = (int64_t*)(w + o_den);
    int64_t* num_s = (int64_t*)(w + o_num);
    uint8_t* rec = (uint8_t*)(w + o_rec);
    int64_t* ys = (int64_t*)(w + o_ys);
    uint32_t* or_parts = (uint32_t*)(w + o_or);
    int64_t* counts = (int64_t*)(w + o_cnt);
    int64_t* offs = (int64_t*)(w + o_off);
    SegPair* agg = (SegPair*)(w + o_agg);
    int64_t* car = (int64_t*)(w + o_car);
    hipStream_t s = (hipStream_t)stream;
    auto scan = [&](ScanSrc src, int64_t len, int64_t* out) -> int {
        const int64_t tiles = (len + kTile - 1) / kTile;
        seg_reduce_kernel<<<(unsigned)tiles, 256, 0, s>>>(src, len, agg);
        seg_carry_kernel<<<1, 256, 0, s>>>(agg, tiles, car);
        seg_scan_kernel<<<(unsigned)tiles, 256, 0, s>>>(src, len, car, out);
        CBH_LAUNCHED();
        return CBH_OK;
    };
    const int gsx = grid_for(n, 256, std::max(1, ctx->num_cus * 8 / n_cross));
    cross_keys_kernel<<<dim3(gsx, n_cross), 256, 0, s>>>(e_ids, e_bits, k_bits, c_order, n,
                                                         keys[0], rows[0], ctx->d_flags);
    CBH_LAUNCHED();
    int cur = 0;
    const int key_bits = e_bits + k_bits;
    // e values of a one-bit split leave the upper digits of e zero: those
    // passes copy
    key_or_kernel<<<kOrParts, 256, 0, s>>>(keys[0], N, or_parts);
    CBH_LAUNCHED();
    for (int shift = 0; shift < key_bits; shift += 8) {
        radix_count_kernel<<<(unsigned)n_tiles, kSortThreads, 0, s>>>(keys[cur], N, shift,
                                                                      n_tiles, counts, or_parts);
        CBH_LAUNCHED();
        rc = scan(ScanSrc{0, counts, nullptr, nullptr, nullptr}, cnt_elems, offs);
        if (rc != CBH_OK) return rc;
        radix_scatter_kernel<<<(unsigned)n_tiles, kSortThreads, 0, s>>>(
            keys[cur], rows[cur], N, shift, n_tiles, offs, keys[cur ^ 1], rows[cur ^ 1],
            or_parts);
        CBH_LAUNCHED();
        cur ^= 1;
    }
    const int gs = grid_for(N, 256, ctx->num_cus * 8);
    cross_heads_kernel<<<gs, 256, 0, s>>>(keys[cur], rows[cur], c_ids, k_bits, N, head);
    CBH_LAUNCHED();
    ScanSrc dsrc{3, nullptr, keys[cur], rows[cur], nullptr};
    dsrc.heads = head;
    rc = scan(dsrc, N, den_s);
    if (rc != CBH_OK) return rc;
    uint32_t* size_at_start = nullptr;
    if (counter_bins > 0) {
        size_at_start = keys[cur ^ 1];     // free after the sort
        cross_group_size_kernel<<<gs, 256, 0, s>>>(head, den_s, N, size_at_start);
        CBH_LAUNCHED();
    }
    for (int t = 0; t < n_targets; ++t) {
        cross_gather_y_kernel<<<gs, 256, 0, s>>>(rows[cur], y_num + int64_t(t) * n, N, ys);
        CBH_LAUNCHED();
        ScanSrc nsrc{5, ys, nullptr, nullptr, nullptr};
        nsrc.heads = head;
        rc = scan(nsrc, N, num_s);
        if (rc != CBH_OK) return rc;
        CrossPriors pri;
        for (int q = 0; q < 8; ++q) pri.ap[q] = q < n_priors ? a * priors[t * n_priors + q] : 0.0;
        const bool last = t == n_targets - 1;
        auto kern = whole ? cross_scatter_kernel<true> : cross_scatter_kernel<false>;
        kern<<<gs, 256, 0, s>>>(keys[cur], rows[cur], den_s, num_s, N, n, k_bits, y_shift, a,
                                pri, n_priors, t, ts_borders, n_ts_borders,
                                last ? size_at_start : nullptr, counter_bins,
                                n_targets * n_priors, rec, stride);
        CBH_LAUNCHED();
    }
    const dim3 ug(grid_for(n, 256, std::max(1, ctx->num_cus * 8 / n_cross)), n_cross);
    cross_unpack_kernel<<<ug, 256, 0, s>>>(rec, n, cpc, stride, ts_bin_out, ld);
    CBH_LAUNCHED();
    return CBH_OK;
}

}  // extern "C"
