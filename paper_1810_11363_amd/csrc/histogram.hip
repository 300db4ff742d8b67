// Per-leaf gradient histograms over binned features (Sec. 5, "Dense numerical
// features": the histogram of feature j sums the gradient of every row whose
// bin of j is b; here additionally split by the row's current leaf, with a
// second statistic h, the row count for RMSE).
//
// MI355X design. The paper's kernel keeps per-warp copies in shared memory and
// rotates lanes over features to avoid atomics. On CDNA4 the LDS has native
// 64-bit atomics (ds_add_f64, ds_add_u64) and ds_add_u32 at full rate, while
// ds_add_f32 is not pipelined (measured 0.33 lane-ops per clock per CU
// against 7.6 for ds_add_f64), and a CU has 160 KB of LDS. A copy of a
// B-bin histogram per lane, as the paper's rotation needs, holds only 5
// waves per CU at B = 128 and, waiting on each read-add-write, reached 0.9
// updates per clock per CU. So one LDS tile per block is updated with LDS
// atomics (or compare-and-swap for the float32 forms), and no global atomics
// are used anywhere:
//   - a block owns (row chunk, feature group, leaf tile); every thread streams
//     ROWS consecutive rows per step (16 for int16 codes, 8 for float forms):
//     ROWS bins of each of its features (coalesced, feature-major columns),
//     the rows' gradient statistics and, from level 1 on, their leaf indices;
//   - the tile is [leaf][feature][stat][bin][replica] in LDS with the bin
//     stride padded to an odd number of words; spare LDS holds up to 32
//     replicas of every cell, replica = lane mod rep, so lanes that hit one
//     bin mostly update different words;
//   - the block sums the replicas and writes its tile to a partial buffer; a
//     second launch merges the partial tiles of all row chunks in a fixed
//     order (deterministic merge);
//   - block ids map to work XCD-contiguously: consecutive work items (same row
//     chunk, different feature groups) land on one XCD and share its L2.
// Precision variants:
//   FP32      float32 sums: compare-and-swap of the float g (RMSE, with a
//             ds_add_u32 count) or of the (g, h) float pair; chunk partials
//             are added in float;
//   TWOFLOAT  compensated float32: TwoSum of each value into a (hi, lo)
//             float pair by a 64-bit compare-and-swap (h the same way, or a
//             u32 count); chunk partials are added with TwoSum;
//   F64       ds_add_f64 for g (and h), ds_add_u32 for RMSE counts; each
//             tile sum is split into a (hi, lo) float pair (TWOFLOAT's
//             output layout); chunk partials are added with TwoSum;
//   INT16     one ds_add_u64 per row, feature and class of the packed word
//             (g code << 32) + h code; at most 65536 rows per chunk keep
//             both halves exact; partials are decoded and summed in int64.
// Histogram subtraction (levels >= 1, optional): only the smaller child of
// every parent leaf is accumulated; its sibling is the parent minus it.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "kernels_dev.h"

namespace cbh {

int words_per_cell(int32_t precision, int32_t K) {
    return out_prec(precision) == CBH_PREC_TWOFLOAT ? 4 * K : 2 * K;
}

int64_t hist_elems(int32_t n_leaves, int32_t F, int32_t B, int32_t K) {
    return int64_t(n_leaves) * F * B * 2 * K;
}

int64_t hist_elem_bytes(int32_t precision) {
    return precision == CBH_PREC_FP32 ? 4 : 8;
}

HistKnobs knobs_for(const cbh_ctx* ctx, int32_t F, int32_t B, int32_t K, int32_t level,
                    int32_t precision, int64_t n, int32_t sub) {
    if (ctx->force_knobs) return ctx->forced;
    int32_t nb = 0;
    while ((int64_t(1) << (nb + 1)) <= n) ++nb;
    auto it = ctx->tuned.find(TuneKey{F, B, K, level, precision, nb, sub});
    if (it != ctx->tuned.end()) return it->second;
    return ctx->knobs;
}

// Plan of the lanes-over-features kernel: the widest lane group W (at most
// the requested one) whose tile of all slots fits the LDS budget; if even
// W = 4 does not fit, the slots are split into tiles (rows re-read per tile).
// With K classes every class is a block of its own (same tile size). Chunks
// as for the other kernel.
static HistPlan plan_lpf(const HistKnobs& kn, int64_t n, int32_t F, int32_t B, int32_t K,
                         int32_t n_slots, int32_t precision, int max_lds) {
    HistPlan p;
    p.kind = 1;
    p.words_per_cell = words_per_cell(precision, K);
    const uint32_t cs = precision == CBH_PREC_INT16 ? 8 : 16;
    // with several classes the whole LDS: wider lane groups mean fewer
    // feature groups re-reading every row's statistics (5*10^7 rows, 10
    // classes, 255 bins: the one-slot build 62 -> 56 ms with 32 features per
    // group instead of 16, one block per CU instead of two)
    const int64_t budget = K > 1 ? int64_t(max_lds) : std::min<int64_t>(kn.lds_budget, max_lds);
    int32_t W = kn.lpf_w > 0 ? std::min(kn.lpf_w, 32) : 32;
    while (W > 4 && int64_t(n_slots) * B * lpf_record_bytes(W, cs) > budget) W /= 2;
    p.fb = W;
    const int64_t slot_bytes = int64_t(B) * lpf_record_bytes(W, cs);
    // slots per tile: all if they fit, at most 64
    int32_t lt = std::min<int32_t>(n_slots, 64);
    while (lt > 1 && lt * slot_bytes > std::max<int64_t>(budget, slot_bytes)) lt = (lt + 1) / 2;
    p.lt = lt;
    p.n_ltiles = (n_slots + lt - 1) / lt;
    p.n_fgroups = (F + W - 1) / W;
    const int64_t tiles = int64_t(p.n_fgroups) * p.n_ltiles * K;   // blocks per chunk
    const int64_t part_per_chunk = int64_t(n_slots) * F * B * p.words_per_cell * 4;
    const int64_t c_part = std::max<int64_t>(1, (int64_t(kn.partial_pct) * n * F / 100) /
                                                    std::max<int64_t>(1, part_per_chunk));
    const int64_t c_rows = std::max<int64_t>(1, n / std::max<int64_t>(1, kn.min_rows));
    // the K class blocks of one (chunk, group, tile) read the same bins, which
    // stay in L2 only if their row range is short: with several classes, 8
    // times as many blocks
    const int64_t target = int64_t(kn.target_blocks) * (K > 1 ? 8 : 1);
    const int64_t c_fill = std::max<int64_t>(1, (target + tiles - 1) / tiles);
    const int64_t chunks = std::min(std::min(c_part, c_rows), c_fill);
    int64_t rows = align_up((n + chunks - 1) / chunks, 16);
    if (precision == CBH_PREC_INT16) rows = std::min<int64_t>(rows, 65536);
    p.rows_per_chunk = rows;
    p.n_chunks = (int32_t)((n + rows - 1) / rows);
    p.rep = 1;
    p.lds_bytes = lt * slot_bytes;
    p.n_blocks = int64_t(p.n_chunks) * tiles;
    return p;
}

// Launch plan of one histogram level.
//   leaves per tile lt: all leaves if one leaf row per feature fits the LDS
//     budget, else the largest power of two that does (extra tiles re-read
//     the rows from cache, not from HBM);
//   chunks C (row ranges): bounded by the rows a block needs to be efficient
//     (min_rows) and by the partial-tile volume C * L * F * B * wpc * 4, kept
//     under partial_pct % of the n * F bin bytes;
//   feature groups: as many as needed to reach target_blocks, at least enough
//     to respect the LDS bound on features per block.
HistPlan plan_hist(const HistKnobs& kn, int64_t n, int32_t F, int32_t B, int32_t K,
                   int32_t n_leaves, int32_t precision, int32_t rmse, int max_lds) {
    if (kn.kernel == 1) return plan_lpf(kn, n, F, B, K, n_leaves, precision, max_lds);
    HistPlan p;
    p.words_per_cell = words_per_cell(precision, K);
    const int64_t cell_bytes = tile_lds_bytes(precision, rmse, K, B, 1);   // LDS per cell
    const int64_t out_cell_bytes = int64_t(B) * p.words_per_cell * 4;     // partial per cell
    const int64_t budget = std::max<int64_t>(cell_bytes, std::min<int64_t>(kn.lds_budget, max_lds));
    int64_t fb_max;
    if (int64_t(n_leaves) * cell_bytes <= budget) {
        p.lt = n_leaves;
        // reserve room for rep_target replicas of every cell where possible
        int64_t want = std::max<int32_t>(1, std::min(kn.rep_target, kn.max_rep));
        while (want > 1 && int64_t(n_leaves) * cell_bytes * want > budget) want /= 2;
        fb_max = budget / (int64_t(n_leaves) * cell_bytes * want);
    } else {
        int32_t lt = 1;
        while (int64_t(lt) * 2 * cell_bytes <= budget && lt * 2 <= n_leaves) lt *= 2;
        p.lt = lt;
        fb_max = 1;
    }
    fb_max = std::max<int64_t>(1, std::min<int64_t>(fb_max, std::min<int64_t>(F, kn.max_fb)));
    p.n_ltiles = (n_leaves + p.lt - 1) / p.lt;
    const int64_t g_min = (F + fb_max - 1) / fb_max;
    const int64_t tiles = p.n_ltiles;
    const int64_t part_per_chunk = int64_t(n_leaves) * F * out_cell_bytes;
    const int64_t c_part = std::max<int64_t>(1, (int64_t(kn.partial_pct) * n * F / 100) /
                                                    std::max<int64_t>(1, part_per_chunk));
    const int64_t c_rows = std::max<int64_t>(1, n / std::max<int64_t>(1, kn.min_rows));
    const int64_t c_fill = std::max<int64_t>(1, (kn.target_blocks + g_min * tiles - 1) /
                                                    (g_min * tiles));
    int64_t chunks = std::min(std::min(c_part, c_rows), c_fill);
    int64_t rows = align_up((n + chunks - 1) / chunks, 16);
    if (precision == CBH_PREC_INT16) rows = std::min<int64_t>(rows, 65536);
    p.rows_per_chunk = rows;
    p.n_chunks = (int32_t)((n + rows - 1) / rows);
    int64_t groups = std::max<int64_t>(
        g_min, (kn.target_blocks + int64_t(p.n_chunks) * tiles - 1) / (int64_t(p.n_chunks) * tiles));
    groups = std::min<int64_t>(groups, F);
    p.fb = (int32_t)((F + groups - 1) / groups);
    p.n_fgroups = (F + p.fb - 1) / p.fb;
    // spare LDS goes to replicas of every cell
    const int64_t cells = int64_t(p.lt) * p.fb;
    p.rep = 1;
    while (p.rep * 2 <= kn.max_rep &&
           tile_lds_bytes(precision, rmse, K, B, cells * p.rep * 2) <= budget)
        p.rep *= 2;
    p.lds_bytes = tile_lds_bytes(precision, rmse, K, B, cells * p.rep);
    p.n_blocks = int64_t(p.n_chunks) * p.n_fgroups * p.n_ltiles;
    return p;
}

struct HistArgs {
    const uint8_t* const* bins;
    const int64_t* seg;
    const float* g;
    const float* h;
    const uint32_t* gq;
    const uint16_t* leaf;
    uint32_t* partials;
    int64_t n;
    int64_t rows_per_chunk;
    int64_t n_blocks;
    int32_t F, B, K, L;
    int32_t fb, lt, n_fgroups, n_ltiles;
    int32_t wpc;
    int32_t rmse;
    const uint8_t* side;    // subtraction mode (see TileArgs), else NULL
    uint32_t sub_shift;
    int32_t rep;
    // lanes-over-features kernel: per-row slot codes (the leaf in a direct
    // build; the parent, or 0xffff for the larger child's rows, in subtraction)
    const uint16_t* rowcode;
    int32_t bits;           // bins per byte layout: 8, or packed 4 / 1 (lanes-over-features only)
};

template <int PREC, int KT, int RM>
__global__ __launch_bounds__(kHistThreads) void hist_kernel(HistArgs a) {
    extern __shared__ __align__(16) uint32_t lds[];
    // XCD-contiguous work: hardware deals consecutive block ids to the 8 XCDs in
    // turn, so block b works on item (b % 8) * per_xcd + b / 8.
    const int64_t per_xcd = (a.n_blocks + 7) / 8;
    int64_t item = int64_t(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (item >= a.n_blocks) return;
    const int lt_i = (int)(item % a.n_ltiles);
    item /= a.n_ltiles;
    const int fg = (int)(item % a.n_fgroups);
    const int64_t chunk = item / a.n_fgroups;
    TileArgs t;
    t.bins = a.bins;
    t.seg = a.seg;
    t.g = a.g;
    t.h = a.h;
    t.gq = a.gq;
    t.leaf = a.leaf;
    t.part = a.partials + chunk * (int64_t(a.L) * a.F * a.B * a.wpc);
    t.n = a.n;
    t.r0 = chunk * a.rows_per_chunk;
    t.r1 = min(a.n, t.r0 + a.rows_per_chunk);
    t.F = a.F;
    t.B = a.B;
    t.K = a.K;
    t.L = a.L;
    t.fb = a.fb;
    t.lt = a.lt;
    t.wpc = a.wpc;
    t.rmse = a.rmse;
    t.f0 = fg * a.fb;
    t.nf = min(a.fb, a.F - t.f0);
    t.l0 = (uint32_t)lt_i * a.lt;
    t.side = a.side;
    t.sub_shift = a.sub_shift;
    t.rep = a.rep;
    hist_tile<PREC, KT, RM>(t, lds);
}

// Merge the partial tiles of all chunks. A block takes 64 consecutive output
// units (a word for FP32, a (hi, lo) pair for TWOFLOAT, a packed u64 for
// INT16); wave w sums chunks w, w + 4, w + 8, ... and the four slice sums are
// added in slice order, so the result does not depend on scheduling.
//
// Subtraction mode (parent != NULL): the partials hold, for every parent leaf
// p < half, the histogram of its smaller child (bit side[p]); the merged value
// is written to that child and parent - value to its sibling: exact for
// integer sums and counts, a two-float difference for TWOFLOAT.
struct SubArgs {
    const void* parent;     // level-1 histogram in the output format, or NULL
    const uint8_t* side;    // [half] child whose rows were accumulated
    int64_t fb_cells;       // F * B
    int64_t half;           // number of parents
};

template <int PREC>
__global__ __launch_bounds__(256) void hist_reduce_kernel(const uint32_t* __restrict__ part,
                                                          int64_t cells, int32_t K,
                                                          int32_t n_chunks, int32_t rmse,
                                                          void* __restrict__ out, SubArgs sub) {
    __shared__ int64_t acc_a[4][64];
    __shared__ int64_t acc_b[4][64];
    const int lane = threadIdx.x & 63, slice = threadIdx.x >> 6;
    const int wpc = PREC == CBH_PREC_TWOFLOAT ? 4 * K : 2 * K;
    const int64_t cw = cells * wpc;     // words per chunk partial
    const int64_t upc = PREC == CBH_PREC_INT16 ? K : 2 * K;   // units per cell
    const int64_t units = cells * upc;
    for (int64_t u0 = int64_t(blockIdx.x) * 64; u0 < units; u0 += int64_t(gridDim.x) * 64) {
        const int64_t u = u0 + lane;
        const bool ok = u < units;
        // destination units: the merged value and, in subtraction mode, its sibling
        int64_t u_small = u, u_big = -1;
        if (sub.parent && ok) {
            const int64_t cell = u / upc, within = u % upc;
            const int64_t p = cell / sub.fb_cells, rest = cell % sub.fb_cells;
            const int64_t sd = sub.side[p];
            u_small = ((p + sd * sub.half) * sub.fb_cells + rest) * upc + within;
            u_big = ((p + (1 - sd) * sub.half) * sub.fb_cells + rest) * upc + within;
        }
        if constexpr (PREC == CBH_PREC_FP32) {
            const bool is_count = rmse && (u & 1);
            float fs = 0.f;
            uint32_t cs = 0;
            if (ok) {
                int ch = slice;
                for (; ch + 12 < n_chunks; ch += 16) {
                    uint32_t v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = part[(ch + 4 * q) * cw + u];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (is_count) cs += v[q]; else fs += __uint_as_float(v[q]);
                    }
                }
                for (; ch < n_chunks; ch += 4) {
                    const uint32_t v = part[ch * cw + u];
                    if (is_count) cs += v; else fs += __uint_as_float(v);
                }
            }
            acc_a[slice][lane] = is_count ? (int64_t)cs : (int64_t)__float_as_uint(fs);
            __syncthreads();
            if (slice == 0 && ok) {
                if (is_count) {
                    uint32_t t = 0;
                    for (int sl = 0; sl < 4; ++sl) t += (uint32_t)acc_a[sl][lane];
                    reinterpret_cast<uint32_t*>(out)[u_small] = t;
                    if (u_big >= 0)
                        reinterpret_cast<uint32_t*>(out)[u_big] =
                            reinterpret_cast<const uint32_t*>(sub.parent)[u] - t;
                } else {
                    float t = 0.f;
                    for (int sl = 0; sl < 4; ++sl) t += __uint_as_float((uint32_t)acc_a[sl][lane]);
                    reinterpret_cast<float*>(out)[u_small] = t;
                    if (u_big >= 0)
                        reinterpret_cast<float*>(out)[u_big] =
                            reinterpret_cast<const float*>(sub.parent)[u] - t;
                }
            }
        } else if constexpr (PREC == CBH_PREC_TWOFLOAT) {
            const bool is_count = rmse && (u & 1);
            float S = 0.f, E = 0.f;
            uint32_t cs = 0;
            if (ok) {
                // this slice's chunks in order, four chunks' words loaded
                // before their adds (the adds keep the order)
                auto add1 = [&](uint32_t hi_w, uint32_t lo_w) {
                    if (is_count) {
                        cs += hi_w;
                        return;
                    }
                    const float hi = __uint_as_float(hi_w);
                    const float lo = __uint_as_float(lo_w);
                    const float t = S + hi;
                    const float bp = t - S;
                    E += ((S - (t - bp)) + (hi - bp)) + lo;
                    S = t;
                };
                int ch = slice;
                for (; ch + 12 < n_chunks; ch += 16) {
                    uint2 w[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        w[q] = *reinterpret_cast<const uint2*>(part + (ch + 4 * q) * cw + 2 * u);
#pragma unroll
                    for (int q = 0; q < 4; ++q) add1(w[q].x, w[q].y);
                }
                for (; ch < n_chunks; ch += 4) {
                    const uint2 w = *reinterpret_cast<const uint2*>(part + ch * cw + 2 * u);
                    add1(w.x, w.y);
                }
            }
            acc_a[slice][lane] = is_count ? (int64_t)cs : (int64_t)__float_as_uint(S);
            acc_b[slice][lane] = (int64_t)__float_as_uint(E);
            __syncthreads();
            if (slice == 0 && ok) {
                float2 r;
                if (is_count) {
                    uint32_t t = 0;
                    for (int sl = 0; sl < 4; ++sl) t += (uint32_t)acc_a[sl][lane];
                    r = make_float2(__uint_as_float(t), 0.f);
                    if (u_big >= 0) {
                        const uint32_t pc =
                            __float_as_uint(reinterpret_cast<const float2*>(sub.parent)[u].x);
                        reinterpret_cast<float2*>(out)[u_big] = make_float2(__uint_as_float(pc - t), 0.f);
                    }
                } else {
                    float S2 = 0.f, E2 = 0.f;
                    for (int sl = 0; sl < 4; ++sl) {
                        const float hi = __uint_as_float((uint32_t)acc_a[sl][lane]);
                        const float lo = __uint_as_float((uint32_t)acc_b[sl][lane]);
                        const float t = S2 + hi;
                        const float bp = t - S2;
                        E2 += ((S2 - (t - bp)) + (hi - bp)) + lo;
                        S2 = t;
                    }
                    const float hs = S2 + E2;
                    r = make_float2(hs, E2 - (hs - S2));
                    if (u_big >= 0) {
                        // (P_hi, P_lo) - (hs, lo) with TwoSum on the leading parts
                        const float2 P = reinterpret_cast<const float2*>(sub.parent)[u];
                        const float t = P.x - r.x;
                        const float bp = t - P.x;
                        const float e = ((P.x - (t - bp)) + (-r.x - bp)) + (P.y - r.y);
                        const float dh = t + e;
                        reinterpret_cast<float2*>(out)[u_big] = make_float2(dh, e - (dh - t));
                    }
                }
                reinterpret_cast<float2*>(out)[u_small] = r;
            }
        } else {
            const uint64_t* P64 = reinterpret_cast<const uint64_t*>(part);
            int64_t gs = 0, hs = 0;
            if (ok) {
                int ch = slice;
                for (; ch + 12 < n_chunks; ch += 16) {
                    uint64_t v[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = P64[(ch + 4 * q) * (cw / 2) + u];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        hs += (int64_t)(uint32_t)(v[q] & 0xffffffffull);
                        gs += (int64_t)(int32_t)(uint32_t)(v[q] >> 32);
                    }
                }
                for (; ch < n_chunks; ch += 4) {
                    const uint64_t v = P64[ch * (cw / 2) + u];
                    hs += (int64_t)(uint32_t)(v & 0xffffffffull);
                    gs += (int64_t)(int32_t)(uint32_t)(v >> 32);
                }
            }
            acc_a[slice][lane] = gs;
            acc_b[slice][lane] = hs;
            __syncthreads();
            if (slice == 0 && ok) {
                int64_t tg = 0, th = 0;
                for (int sl = 0; sl < 4; ++sl) {
                    tg += acc_a[sl][lane];
                    th += acc_b[sl][lane];
                }
                int64_t* o = reinterpret_cast<int64_t*>(out);
                o[2 * u_small] = tg;
                o[2 * u_small + 1] = th;
                if (u_big >= 0) {
                    const int64_t* P = reinterpret_cast<const int64_t*>(sub.parent);
                    o[2 * u_big] = P[2 * u] - tg;
                    o[2 * u_big + 1] = P[2 * u + 1] - th;
                }
            }
        }
        __syncthreads();
    }
}

// side[p] of every parent p of a build by subtraction (see parent_side).
template <int PREC>
__global__ __launch_bounds__(256) void sub_side_kernel(const void* __restrict__ parent,
                                                       const cbh_split* __restrict__ split,
                                                       int64_t half, int32_t F, int32_t B,
                                                       int32_t K, int32_t rmse,
                                                       uint8_t* __restrict__ side) {
    // one wave per parent leaf, lanes over bins
    const int64_t p = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= half) return;
    const uint8_t sd = parent_side<PREC>(parent, p, split->feature, split->border, F, B, K, rmse,
                                         lane);
    if (lane == 0) side[p] = sd;
}

// Sides and row codes in one launch (lanes-over-features builds by
// subtraction with few parents): every block first derives the side of every
// parent into LDS (block 0 also stores them for the merge), then writes
// code[i] = p = leaf & (half - 1) for rows on the parent's accumulated side,
// 0xffff otherwise. APPLY: the leaf array does not hold the parent level's
// bit yet; the kernel takes it from the split feature's bin (as
// cbh_apply_split does, overwriting the leaf when the parent is level 0)
// and stores the updated leaf.
template <int PREC, bool APPLY>
__global__ __launch_bounds__(256) void side_code_kernel(const void* __restrict__ parent,
                                                        const cbh_split* __restrict__ split,
                                                        int64_t half, int32_t F, int32_t B,
                                                        int32_t K, int32_t rmse,
                                                        uint16_t* __restrict__ leaf, int64_t n,
                                                        int64_t rows_per_block, uint32_t shift,
                                                        uint8_t* __restrict__ side,
                                                        uint16_t* __restrict__ code,
                                                        const uint8_t* const* __restrict__ bins,
                                                        const int64_t* __restrict__ seg) {
    extern __shared__ uint8_t sd[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int f = split->feature, k = split->border;
    for (int64_t p = wave; p < half; p += 4) {
        const uint8_t v = parent_side<PREC>(parent, p, f, k, F, B, K, rmse, lane);
        if (lane == 0) {
            sd[p] = v;
            if (blockIdx.x == 0) side[p] = v;
        }
    }
    __syncthreads();
    const bool has_split = f >= 0 && f < F;
    const uint8_t* col = (APPLY && has_split) ? bins[f] : nullptr;
    const int64_t st = (APPLY && has_split) ? seg_stride_of(seg, f) : 16;
    const uint32_t lmask = (uint32_t)half - 1u;
    const int64_t i0 = int64_t(blockIdx.x) * rows_per_block;
    const int64_t i1 = min(n, i0 + rows_per_block);
    // 8 rows per thread and step where the block's rows are 8-aligned
    const bool vec = ((reinterpret_cast<uintptr_t>(leaf) | reinterpret_cast<uintptr_t>(code) |
                       (APPLY ? reinterpret_cast<uintptr_t>(col) & 7 : 0)) & 15) == 0;
    int64_t i = i0;
    if (vec) {
        const int64_t i8 = i0 + ((i1 - i0) & ~int64_t(7));
        for (int64_t j = i0 + 8 * int64_t(threadIdx.x); j < i8; j += 8 * 256) {
            uint4 lv = *reinterpret_cast<const uint4*>(leaf + j);
            if constexpr (APPLY) {
                // level 0's bit overwrites what the previous tree left
                if (shift == 0) lv = make_uint4(0u, 0u, 0u, 0u);
                // the 8 rows' bins: 8 bytes of one 16-row segment
                uint2 bw = make_uint2(0u, 0u);
                if (col) bw = gld_u2(seg_ptr(col, st, j));
                const uint32_t bb[2] = {bw.x, bw.y};
                uint32_t lw2[4] = {lv.x, lv.y, lv.z, lv.w};
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const uint32_t bit = col && (int)((bb[r >> 2] >> (8 * (r & 3))) & 255u) > k;
                    lw2[r >> 1] |= (bit << shift) << (16 * (r & 1));
                }
                lv = make_uint4(lw2[0], lw2[1], lw2[2], lw2[3]);
                *reinterpret_cast<uint4*>(leaf + j) = lv;
            }
            const uint32_t lw[4] = {lv.x, lv.y, lv.z, lv.w};
            uint32_t cw[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t out = 0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const uint32_t v = (lw[q] >> (16 * h)) & 0xffffu;
                    const uint32_t pp = v & lmask;
                    const uint32_t c = (((v >> shift) & 1u) == (uint32_t)sd[pp]) ? pp : 0xffffu;
                    out |= c << (16 * h);
                }
                cw[q] = out;
            }
            *reinterpret_cast<uint4*>(code + j) = make_uint4(cw[0], cw[1], cw[2], cw[3]);
        }
        i = i8;
    }
    for (int64_t j = i + threadIdx.x; j < i1; j += 256) {
        uint32_t v = leaf[j];
        if constexpr (APPLY) {
            if (shift == 0) v = 0u;
            if (col && (int)*seg_ptr(col, st, j) > k) v |= 1u << shift;
            leaf[j] = (uint16_t)v;
        }
        const uint32_t pp = v & lmask;
        code[j] = (uint16_t)((((v >> shift) & 1u) == (uint32_t)sd[pp]) ? pp : 0xffffu);
    }
}

// Single-problem launch: block -> (class, slot tile, feature group, chunk),
// XCD-contiguous (the classes of one tile, group and chunk, which read the
// same bins, are neighbours).
template <int PREC, int RM, int W, int MODE, int BITS>
__global__ __launch_bounds__(kHistThreads) void hist_lpf_kernel(HistArgs a) {
    extern __shared__ __align__(16) uint32_t lds[];
    const int64_t per_xcd = (a.n_blocks + 7) / 8;
    int64_t item = int64_t(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (item >= a.n_blocks) return;
    const int c = (int)(item % a.K);
    item /= a.K;
    const int lt_i = (int)(item % a.n_ltiles);
    item /= a.n_ltiles;
    const int fg = (int)(item % a.n_fgroups);
    const int64_t chunk = item / a.n_fgroups;
    LpfBlock b;
    b.bins = a.bins;
    b.seg = a.seg;
    b.g = a.g + int64_t(c) * a.n;
    b.h = a.h ? a.h + int64_t(c) * a.n : nullptr;
    b.gq = a.gq ? a.gq + int64_t(c) * a.n : nullptr;
    b.rowcode = a.rowcode;
    b.F = a.F;
    b.B = a.B;
    b.wpc = a.wpc;
    b.coff = c * (a.wpc / a.K);
    const int64_t r0 = chunk * a.rows_per_chunk;
    const uint32_t s0 = (uint32_t)lt_i * (uint32_t)a.lt;
    lpf_block<PREC, RM, W, MODE, BITS>(b, r0, min(a.n, r0 + a.rows_per_chunk), fg, s0,
                                 min((uint32_t)a.lt, (uint32_t)a.L - s0),
                                 a.partials + chunk * (int64_t(a.L) * a.F * a.B * a.wpc), 0u,
                                 lds);
}

void hist_init_attrs(int max_lds) {
    const void* fns[] = {
        (const void*)hist_kernel<CBH_PREC_FP32, 1, 0>, (const void*)hist_kernel<CBH_PREC_FP32, 1, 1>,
        (const void*)hist_kernel<CBH_PREC_FP32, 0, 0>,
        (const void*)hist_kernel<CBH_PREC_TWOFLOAT, 1, 0>,
        (const void*)hist_kernel<CBH_PREC_TWOFLOAT, 1, 1>,
        (const void*)hist_kernel<CBH_PREC_TWOFLOAT, 0, 0>,
        (const void*)hist_kernel<CBH_PREC_INT16, 1, 0>, (const void*)hist_kernel<CBH_PREC_INT16, 1, 1>,
        (const void*)hist_kernel<CBH_PREC_INT16, 0, 0>,
        (const void*)hist_kernel<CBH_PREC_F64, 1, 0>, (const void*)hist_kernel<CBH_PREC_F64, 1, 1>,
        (const void*)hist_kernel<CBH_PREC_F64, 0, 0>};
    for (const void* f : fns)
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
#define CBH_LPF_ATTRB(P, R, M, BT)                                                           \
    {                                                                                        \
        const void* l[] = {(const void*)hist_lpf_kernel<P, R, 32, M, BT>,                    \
                           (const void*)hist_lpf_kernel<P, R, 16, M, BT>,                    \
                           (const void*)hist_lpf_kernel<P, R, 8, M, BT>,                     \
                           (const void*)hist_lpf_kernel<P, R, 4, M, BT>};                    \
        for (const void* f : l)                                                              \
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds); \
    }
#define CBH_LPF_ATTR(P, R, M) CBH_LPF_ATTRB(P, R, M, 8) CBH_LPF_ATTRB(P, R, M, 4) \
    CBH_LPF_ATTRB(P, R, M, 1)
#define CBH_LPF_ATTR3(P, R) CBH_LPF_ATTR(P, R, 0) CBH_LPF_ATTR(P, R, 1) CBH_LPF_ATTR(P, R, 2)
    CBH_LPF_ATTR3(CBH_PREC_FP32, 0)
    CBH_LPF_ATTR3(CBH_PREC_FP32, 1)
    CBH_LPF_ATTR3(CBH_PREC_TWOFLOAT, 0)
    CBH_LPF_ATTR3(CBH_PREC_TWOFLOAT, 1)
    CBH_LPF_ATTR3(CBH_PREC_INT16, 0)
    CBH_LPF_ATTR3(CBH_PREC_F64, 0)
    CBH_LPF_ATTR3(CBH_PREC_F64, 1)
#undef CBH_LPF_ATTR3
#undef CBH_LPF_ATTR
#undef CBH_LPF_ATTRB
}

// Row codes for a lanes-over-features build by subtraction: the parent
// p = leaf & lmask if the row is on the parent's accumulated side
// (bit `shift` of the leaf equals side[p]), else 0xffff.
__global__ __launch_bounds__(256) void slot_code_kernel(const uint16_t* __restrict__ leaf,
                                                        const uint8_t* __restrict__ side,
                                                        int64_t n, uint32_t lmask, uint32_t shift,
                                                        uint16_t* __restrict__ code) {
    const int64_t tid = int64_t(blockIdx.x) * 256 + threadIdx.x;
    const int64_t stride = int64_t(gridDim.x) * 256;
    for (int64_t i = tid; i < n; i += stride) {
        const uint32_t v = leaf[i];
        const uint32_t p = v & lmask;
        code[i] = (uint16_t)((((v >> shift) & 1u) == (uint32_t)side[p]) ? p : 0xffffu);
    }
}

template <int PREC, int RM, int MODE, int BITS>
static void launch_lpf_bits(const HistArgs& a, const HistPlan& plan, hipStream_t s) {
    const unsigned grid = (unsigned)(8 * ((plan.n_blocks + 7) / 8));
    const size_t lds = (size_t)plan.lds_bytes;
    switch (plan.fb) {
        case 32: hist_lpf_kernel<PREC, RM, 32, MODE, BITS><<<grid, kHistThreads, lds, s>>>(a); break;
        case 16: hist_lpf_kernel<PREC, RM, 16, MODE, BITS><<<grid, kHistThreads, lds, s>>>(a); break;
        case 8: hist_lpf_kernel<PREC, RM, 8, MODE, BITS><<<grid, kHistThreads, lds, s>>>(a); break;
        default: hist_lpf_kernel<PREC, RM, 4, MODE, BITS><<<grid, kHistThreads, lds, s>>>(a); break;
    }
}

template <int PREC, int RM, int MODE>
static void launch_lpf_mode(const HistArgs& a, const HistPlan& plan, hipStream_t s) {
    if (a.bits == 4) launch_lpf_bits<PREC, RM, MODE, 4>(a, plan, s);
    else if (a.bits == 1) launch_lpf_bits<PREC, RM, MODE, 1>(a, plan, s);
    else launch_lpf_bits<PREC, RM, MODE, 8>(a, plan, s);
}

template <int PREC, int RM>
static void launch_lpf(const HistArgs& a, const HistPlan& plan, hipStream_t s) {
    if (a.L == 1 && !a.side) launch_lpf_mode<PREC, RM, 0>(a, plan, s);
    else if (!a.side && plan.n_ltiles == 1) launch_lpf_mode<PREC, RM, 1>(a, plan, s);
    else launch_lpf_mode<PREC, RM, 2>(a, plan, s);
}

int64_t hist_code_bytes(const HistPlan& plan, int64_t n, bool sub) {
    return plan.kind == 1 && sub ? align_up(n * 2, 256) : 0;
}

template <int PREC>
static void launch_hist_prec(const HistArgs& a, const HistPlan& plan, int max_lds,
                             hipStream_t s) {
    const int64_t grid = 8 * ((plan.n_blocks + 7) / 8);
    (void)max_lds;
    if (plan.kind == 1) {
        if constexpr (PREC != CBH_PREC_INT16) {
            if (a.rmse) {
                launch_lpf<PREC, 1>(a, plan, s);
                return;
            }
        }
        launch_lpf<PREC, 0>(a, plan, s);
        return;
    }
    // MultiClass (K > 1) is never RMSE; K = 1 has an RMSE (count) and a
    // second-derivative form
    if (a.K > 1)
        hist_kernel<PREC, 0, 0><<<(unsigned)grid, kHistThreads, (size_t)plan.lds_bytes, s>>>(a);
    else if (a.rmse)
        hist_kernel<PREC, 1, 1><<<(unsigned)grid, kHistThreads, (size_t)plan.lds_bytes, s>>>(a);
    else
        hist_kernel<PREC, 1, 0><<<(unsigned)grid, kHistThreads, (size_t)plan.lds_bytes, s>>>(a);
}

template <int PREC>
static void launch_side_code(const void* parent, const cbh_split* split, int64_t half, int32_t F,
                             int32_t B, int32_t K, int32_t rmse, uint16_t* leaf, int64_t n,
                             uint32_t shift, uint8_t* side, uint16_t* codes, int num_cus,
                             hipStream_t s, const cbh_problem* apply) {
    // about four blocks per CU: each block first derives every parent's side
    // (a few KB of the parent histogram from L2), then streams its rows
    const int64_t rpb = std::max<int64_t>(2048, align_up((n + 4 * num_cus - 1) / (4 * num_cus), 8));
    const unsigned grid = (unsigned)((n + rpb - 1) / rpb);
    if (apply)
        side_code_kernel<PREC, true><<<grid, 256, (size_t)half, s>>>(
            parent, split, half, F, B, K, rmse, leaf, n, rpb, shift, side, codes, apply->bins,
            apply->seg_stride);
    else
        side_code_kernel<PREC, false><<<grid, 256, (size_t)half, s>>>(
            parent, split, half, F, B, K, rmse, leaf, n, rpb, shift, side, codes, nullptr,
            nullptr);
}

int launch_hist(cbh_ctx* ctx, const cbh_problem* p, int32_t level, int32_t precision,
                const HistPlan& plan, void* hist_out, void* partials, hipStream_t s,
                const void* parent, uint8_t* side, uint16_t* codes,
                const cbh_split* parent_split, bool apply_parent) {
    HistArgs a;
    a.rowcode = p->leaf;
    a.bits = packed_bins(p) ? p->bin_bits : 8;
    if (packed_bins(p) && plan.kind != 1) {
        set_error("internal: packed bins need the lanes-over-features histogram");
        return CBH_EINVAL;
    }
    if (parent) {
        const int64_t half = int64_t(1) << (level - 1);
        const int rmse = count_stat(p);
        // (the one-launch side/code pass sets the parent's leaf bit from byte
        // bins only; packed bins take the separate apply)
        const bool fused = plan.kind == 1 && half * p->max_bins <= 16384 &&
                           !(apply_parent && packed_bins(p));
        if (apply_parent && !fused) {
            // the parent level's leaf bit first, as cbh_apply_split
            const int rc = launch_apply(ctx, p, level - 1, parent_split, s);
            if (rc) return rc;
        }
        if (plan.kind == 1) {
            if (!codes) {
                set_error("internal: no row-code buffer for a build by subtraction");
                return CBH_EINVAL;
            }
            const uint32_t shift = (uint32_t)(level - 1);
            if (fused) {
                // few parents: sides and codes (and the parent's leaf bit) in one launch
                const cbh_problem* ap = apply_parent ? p : nullptr;
                switch (out_prec(precision)) {
                    case CBH_PREC_FP32:
                        launch_side_code<CBH_PREC_FP32>(parent, parent_split, half, p->n_features,
                                                        p->max_bins, p->K, rmse, p->leaf, p->n,
                                                        shift, side, codes, ctx->num_cus, s, ap);
                        break;
                    case CBH_PREC_TWOFLOAT:
                        launch_side_code<CBH_PREC_TWOFLOAT>(
                            parent, parent_split, half, p->n_features, p->max_bins, p->K, rmse,
                            p->leaf, p->n, shift, side, codes, ctx->num_cus, s, ap);
                        break;
                    default:
                        launch_side_code<CBH_PREC_INT16>(parent, parent_split, half,
                                                         p->n_features, p->max_bins, p->K, rmse,
                                                         p->leaf, p->n, shift, side, codes,
                                                         ctx->num_cus, s, ap);
                        break;
                }
                CBH_LAUNCHED();
            } else {
                const int rc = launch_side(parent, parent_split, half, p->n_features, p->max_bins,
                                           p->K, rmse, precision, side, s);
                if (rc) return rc;
                slot_code_kernel<<<(unsigned)std::min<int64_t>((p->n + 255) / 256,
                                                               int64_t(ctx->num_cus) * 8),
                                   256, 0, s>>>(p->leaf, side, p->n, (uint32_t)half - 1u, shift,
                                                codes);
                CBH_LAUNCHED();
            }
            a.rowcode = codes;
        } else {
            const int rc = launch_side(parent, parent_split, half, p->n_features, p->max_bins,
                                       p->K, rmse, precision, side, s);
            if (rc) return rc;
        }
    }
    a.bins = p->bins;
    a.seg = p->seg_stride;
    a.g = p->g;
    a.h = p->h;
    a.gq = reinterpret_cast<const uint32_t*>(p->gq);
    a.leaf = p->leaf;
    a.partials = (uint32_t*)partials;
    a.n = p->n;
    a.rows_per_chunk = plan.rows_per_chunk;
    a.n_blocks = plan.n_blocks;
    a.F = p->n_features;
    a.B = p->max_bins;
    a.K = p->K;
    // subtraction mode accumulates per parent leaf (half as many tile leaves)
    a.L = parent ? 1 << (level - 1) : 1 << level;
    a.side = parent ? side : nullptr;
    a.sub_shift = parent ? (uint32_t)(level - 1) : 0u;
    a.fb = plan.fb;
    a.lt = plan.lt;
    a.n_fgroups = plan.n_fgroups;
    a.n_ltiles = plan.n_ltiles;
    a.wpc = plan.words_per_cell;
    a.rmse = count_stat(p);
    a.rep = plan.rep;
    switch (precision) {
        case CBH_PREC_FP32: launch_hist_prec<CBH_PREC_FP32>(a, plan, ctx->max_lds, s); break;
        case CBH_PREC_TWOFLOAT:
            launch_hist_prec<CBH_PREC_TWOFLOAT>(a, plan, ctx->max_lds, s);
            break;
        case CBH_PREC_F64: launch_hist_prec<CBH_PREC_F64>(a, plan, ctx->max_lds, s); break;
        default: launch_hist_prec<CBH_PREC_INT16>(a, plan, ctx->max_lds, s); break;
    }
    CBH_LAUNCHED();
    const int64_t cells = int64_t(a.L) * a.F * a.B;
    const int64_t units = precision == CBH_PREC_INT16 ? cells * a.K : cells * 2 * a.K;
    const int grid = (int)std::min<int64_t>((units + 63) / 64, int64_t(ctx->num_cus) * 16);
    const SubArgs sub{parent, side, int64_t(a.F) * a.B, int64_t(a.L)};
    switch (out_prec(precision)) {
        case CBH_PREC_FP32:
            hist_reduce_kernel<CBH_PREC_FP32><<<grid, 256, 0, s>>>(
                (const uint32_t*)partials, cells, a.K, plan.n_chunks, a.rmse, hist_out, sub);
            break;
        case CBH_PREC_TWOFLOAT:
            hist_reduce_kernel<CBH_PREC_TWOFLOAT><<<grid, 256, 0, s>>>(
                (const uint32_t*)partials, cells, a.K, plan.n_chunks, a.rmse, hist_out, sub);
            break;
        default:
            hist_reduce_kernel<CBH_PREC_INT16><<<grid, 256, 0, s>>>(
                (const uint32_t*)partials, cells, a.K, plan.n_chunks, a.rmse, hist_out, sub);
            break;
    }
    CBH_LAUNCHED();
    return CBH_OK;
}

int launch_side(const void* parent_hist, const cbh_split* parent_split, int64_t half, int32_t F,
                int32_t B, int32_t K, int32_t rmse, int32_t precision, uint8_t* side,
                hipStream_t s) {
    const unsigned gs = (unsigned)((half + 3) / 4);
    switch (out_prec(precision)) {
        case CBH_PREC_FP32:
            sub_side_kernel<CBH_PREC_FP32><<<gs, 256, 0, s>>>(parent_hist, parent_split, half, F,
                                                              B, K, rmse, side);
            break;
        case CBH_PREC_TWOFLOAT:
            sub_side_kernel<CBH_PREC_TWOFLOAT><<<gs, 256, 0, s>>>(parent_hist, parent_split,
                                                                  half, F, B, K, rmse, side);
            break;
        default:
            sub_side_kernel<CBH_PREC_INT16><<<gs, 256, 0, s>>>(parent_hist, parent_split, half,
                                                               F, B, K, rmse, side);
            break;
    }
    CBH_LAUNCHED();
    return CBH_OK;
}

// ------------------------------------------------------ int16 gradient codes
__global__ __launch_bounds__(256) void grad_max_kernel(const float* __restrict__ g,
                                                       const float* __restrict__ h, int64_t n,
                                                       int32_t K, int32_t with_h,
                                                       uint32_t* __restrict__ maxbits) {
    __shared__ float wm[2][4];
    const int c = blockIdx.y;
    float mg = 0.f, mh = 0.f;
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        mg = fmaxf(mg, fabsf(g[int64_t(c) * n + i]));
        if (with_h) mh = fmaxf(mh, h[int64_t(c) * n + i]);
    }
    for (int d = 32; d >= 1; d >>= 1) {
        mg = fmaxf(mg, __shfl_xor(mg, d, 64));
        mh = fmaxf(mh, __shfl_xor(mh, d, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        wm[0][threadIdx.x >> 6] = mg;
        wm[1][threadIdx.x >> 6] = mh;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        mg = fmaxf(fmaxf(wm[0][0], wm[0][1]), fmaxf(wm[0][2], wm[0][3]));
        mh = fmaxf(fmaxf(wm[1][0], wm[1][1]), fmaxf(wm[1][2], wm[1][3]));
        // one atomic per block; non-negative floats order like their bit patterns
        atomicMax(&maxbits[2 * c], __float_as_uint(mg));
        atomicMax(&maxbits[2 * c + 1], __float_as_uint(mh));
    }
}

__global__ void zero_u32_kernel(uint32_t* p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

__global__ __launch_bounds__(256) void grad_code_kernel(const float* __restrict__ g,
                                                        const float* __restrict__ h, int64_t n,
                                                        int32_t K, int32_t with_h,
                                                        const uint32_t* __restrict__ maxbits,
                                                        uint32_t* __restrict__ codes,
                                                        float* __restrict__ scales) {
    const int c = blockIdx.y;
    const float sg = __uint_as_float(maxbits[2 * c]) / 32767.0f;
    const float sh = with_h ? __uint_as_float(maxbits[2 * c + 1]) / 32767.0f : 1.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        scales[2 * c] = sg;
        scales[2 * c + 1] = sh;
    }
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        const int64_t ci = int64_t(c) * n + i;
        const float qg = sg > 0.f ? rintf(g[ci] / sg) : 0.f;
        float qh = 1.f;
        if (with_h) qh = sh > 0.f ? rintf(h[ci] / sh) : 0.f;
        const uint32_t lo = (uint32_t)(uint16_t)(int16_t)qg;
        const uint32_t hi = (uint32_t)(uint16_t)(int16_t)qh;
        codes[ci] = lo | (hi << 16);
    }
}

}  // namespace cbh

using namespace cbh;

extern "C" {

int cbh_quantize_gradients(cbh_ctx* ctx, const cbh_problem* prob, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    int rc = validate_problem(prob);
    if (rc) return rc;
    CBH_ARG(prob->gq && prob->grad_scale, "gq / grad_scale is NULL");
    rc = ensure_ws(ctx, 8 * CBH_MAX_K, stream);
    if (rc) return rc;
    uint32_t* maxbits = (uint32_t*)ctx->ws;
    hipStream_t s = (hipStream_t)stream;
    const int with_h = !count_stat(prob);
    zero_u32_kernel<<<1, 64, 0, s>>>(maxbits, 2 * prob->K);
    const int gx = (int)std::min<int64_t>((prob->n + 255) / 256, ctx->num_cus * 4);
    const int gm = (int)std::min<int64_t>((prob->n + 255) / 256, ctx->num_cus);
    grad_max_kernel<<<dim3(gm, prob->K), 256, 0, s>>>(prob->g, prob->h, prob->n, prob->K,
                                                      with_h, maxbits);
    grad_code_kernel<<<dim3(gx, prob->K), 256, 0, s>>>(prob->g, prob->h, prob->n, prob->K,
                                                       with_h, maxbits,
                                                       (uint32_t*)prob->gq, prob->grad_scale);
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_build_histograms(cbh_ctx* ctx, const cbh_problem* prob, int32_t level,
                         int32_t precision, void* hist_out, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_precision(prob, precision);
    if (rc) return rc;
    CBH_ARG(level >= 0 && level < prob->depth, "level %d outside [0, depth)", level);
    CBH_ARG(hist_out != nullptr, "hist_out is NULL");
    const int L = 1 << level;
    HistKnobs kn = knobs_for(ctx, prob->n_features, prob->max_bins, prob->K, level,
                             precision, prob->n, 0);
    if (packed_bins(prob)) kn.kernel = 1;
    const int rmse = count_stat(prob);
    const HistPlan plan = plan_hist(kn, prob->n, prob->n_features, prob->max_bins, prob->K, L,
                                    precision, rmse, ctx->max_lds);
    CBH_REQUIRE(tile_lds_bytes(precision, rmse, prob->K, prob->max_bins, 1) <= ctx->max_lds,
                CBH_EUNSUPPORTED, "one (leaf, feature) tile of %d bins does not fit in LDS",
                prob->max_bins);
    const int64_t part_bytes =
        int64_t(plan.n_chunks) * L * prob->n_features * prob->max_bins * plan.words_per_cell * 4;
    rc = ensure_ws(ctx, part_bytes, stream);
    if (rc) return rc;
    return launch_hist(ctx, prob, level, precision, plan, hist_out, ctx->ws,
                       (hipStream_t)stream);
}

static int build_sub(cbh_ctx* ctx, const cbh_problem* prob, int32_t level, int32_t precision,
                     const void* parent_hist, const cbh_split* parent_split, void* hist_out,
                     void* stream, bool apply_parent) {
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_precision(prob, precision);
    if (rc) return rc;
    CBH_ARG(level >= 1 && level < prob->depth, "level %d outside [1, depth)", level);
    CBH_ARG(parent_hist && parent_split && hist_out, "NULL histogram or split");
    CBH_ARG(parent_hist != hist_out, "parent_hist and hist_out must not be the same buffer");
    const int half = 1 << (level - 1);
    HistKnobs kn = knobs_for(ctx, prob->n_features, prob->max_bins, prob->K, level,
                             precision, prob->n, 1);
    if (packed_bins(prob)) kn.kernel = 1;
    const int rmse = count_stat(prob);
    const HistPlan plan = plan_hist(kn, prob->n, prob->n_features, prob->max_bins, prob->K, half,
                                    precision, rmse, ctx->max_lds);
    CBH_REQUIRE(tile_lds_bytes(precision, rmse, prob->K, prob->max_bins, 1) <= ctx->max_lds,
                CBH_EUNSUPPORTED, "one (leaf, feature) tile of %d bins does not fit in LDS",
                prob->max_bins);
    const int64_t part_bytes = align_up(
        int64_t(plan.n_chunks) * half * prob->n_features * prob->max_bins * plan.words_per_cell * 4,
        256);
    const int64_t code_bytes = hist_code_bytes(plan, prob->n, true);
    rc = ensure_ws(ctx, part_bytes + align_up(half, 256) + code_bytes, stream);
    if (rc) return rc;
    uint8_t* side = (uint8_t*)ctx->ws + part_bytes;
    uint16_t* codes =
        code_bytes ? (uint16_t*)((uint8_t*)ctx->ws + part_bytes + align_up(half, 256)) : nullptr;
    hipStream_t s = (hipStream_t)stream;
    return launch_hist(ctx, prob, level, precision, plan, hist_out, ctx->ws, s, parent_hist, side,
                       codes, parent_split, apply_parent);
}

int cbh_build_histograms_sub(cbh_ctx* ctx, const cbh_problem* prob, int32_t level,
                             int32_t precision, const void* parent_hist,
                             const cbh_split* parent_split, void* hist_out, void* stream) {
    clear_error();
    return build_sub(ctx, prob, level, precision, parent_hist, parent_split, hist_out, stream,
                     false);
}

int cbh_apply_build_histograms_sub(cbh_ctx* ctx, const cbh_problem* prob, int32_t level,
                                   int32_t precision, const void* parent_hist,
                                   const cbh_split* parent_split, void* hist_out, void* stream) {
    clear_error();
    return build_sub(ctx, prob, level, precision, parent_hist, parent_split, hist_out, stream,
                     true);
}

}  // extern "C"
