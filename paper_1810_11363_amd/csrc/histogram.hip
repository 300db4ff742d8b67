// Per-leaf gradient histograms over binned features (Sec. 5, "Dense numerical
// features": the histogram of feature j sums the gradient of every row whose
// bin of j is b; here additionally split by the row's current leaf, with a
// second statistic h, the row count for RMSE).
//
// MI355X design. The paper's kernel keeps per-warp copies in shared memory and
// rotates lanes over features to avoid atomics; on CDNA4 the LDS has native
// float/int atomics (ds_add_f32, ds_add_u32, ds_add_u64) and 160 KB per CU,
// so one LDS tile per block is updated with LDS atomics and no global atomics
// are used anywhere:
//   - a block owns (row chunk, feature group, leaf tile); every thread streams
//     4 consecutive rows per step: one dword of bins per feature (coalesced,
//     feature-major columns), a float4 of g, a float4 of h and 8 bytes of leaf;
//   - the tile is [leaf][feature][bin][stat] in LDS;
//   - the block writes its tile to a partial buffer; a second launch merges
//     the partial tiles of all row chunks in chunk order (deterministic merge);
//   - block ids map to work XCD-contiguously: consecutive work items (same row
//     chunk, different feature groups) land on one XCD and share its L2.
// Precision variants:
//   FP32      ds_add_f32 for g (and h), ds_add_u32 for RMSE counts;
//   TWOFLOAT  ds_add_rtn_f32 returns the old value, from which the exact
//             rounding error of that addition is recomputed (TwoSum) and
//             added to a second, "lo" word; chunk partials are merged with
//             TwoSum as well;
//   INT16     one ds_add_u64 per row, feature and class of the packed word
//             (g code << 32) + h code; at most 65536 rows per chunk keep
//             both halves exact; partials are decoded and summed in int64.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "kernels_dev.h"

namespace cbh {

int words_per_cell(int32_t precision, int32_t K) {
    return precision == CBH_PREC_TWOFLOAT ? 4 * K : 2 * K;
}

int64_t hist_elems(int32_t n_leaves, int32_t F, int32_t B, int32_t K) {
    return int64_t(n_leaves) * F * B * 2 * K;
}

int64_t hist_elem_bytes(int32_t precision) {
    return precision == CBH_PREC_FP32 ? 4 : 8;
}

HistKnobs knobs_for(const cbh_ctx* ctx, int32_t F, int32_t B, int32_t K, int32_t level,
                    int32_t precision, int64_t n) {
    if (ctx->force_knobs) return ctx->forced;
    int32_t nb = 0;
    while ((int64_t(1) << (nb + 1)) <= n) ++nb;
    auto it = ctx->tuned.find(TuneKey{F, B, K, level, precision, nb});
    if (it != ctx->tuned.end()) return it->second;
    return ctx->knobs;
}

HistPlan plan_hist(const HistKnobs& kn, int64_t n, int32_t F, int32_t B, int32_t K,
                   int32_t n_leaves, int32_t precision, int max_lds) {
    HistPlan p;
    p.words_per_cell = words_per_cell(precision, K);
    const int64_t cell_bytes = int64_t(B) * p.words_per_cell * 4;
    const int64_t budget = std::min<int64_t>(kn.lds_budget, max_lds);
    if (int64_t(n_leaves) * cell_bytes <= budget) {
        p.lt = n_leaves;
        int64_t fb = budget / (int64_t(n_leaves) * cell_bytes);
        fb = std::min<int64_t>(fb, std::min<int64_t>(F, std::max(1, kn.max_fb)));
        p.fb = (int32_t)std::max<int64_t>(1, fb);
    } else {
        int32_t lt = 1;
        while (int64_t(lt) * 2 * cell_bytes <= budget && lt * 2 <= n_leaves) lt *= 2;
        p.lt = lt;
        p.fb = 1;
    }
    // balance features over groups so the last group is not nearly empty
    p.n_fgroups = (F + p.fb - 1) / p.fb;
    p.fb = (F + p.n_fgroups - 1) / p.n_fgroups;
    p.n_ltiles = (n_leaves + p.lt - 1) / p.lt;
    const int64_t base = int64_t(p.n_fgroups) * p.n_ltiles;
    int64_t chunks = std::max<int64_t>(1, (kn.target_blocks + base - 1) / base);
    int64_t rows = align_up((n + chunks - 1) / chunks, 16);
    rows = std::max<int64_t>(rows, align_up(std::min<int64_t>(kn.min_rows, n), 16));
    if (precision == CBH_PREC_INT16) rows = std::min<int64_t>(rows, 65536);
    p.rows_per_chunk = rows;
    p.n_chunks = (int32_t)((n + rows - 1) / rows);
    p.lds_bytes = int64_t(p.lt) * p.fb * cell_bytes;
    p.n_blocks = int64_t(p.n_chunks) * base;
    return p;
}

struct HistArgs {
    const uint8_t* const* bins;
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
};

template <int PREC, int KT>
__global__ __launch_bounds__(256) void hist_kernel(HistArgs a) {
    extern __shared__ uint32_t lds[];
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
    hist_tile<PREC, KT>(t, lds);
}

// Merge the partial tiles of all chunks in chunk order, one thread per cell.
template <int PREC>
__global__ __launch_bounds__(256) void hist_reduce_kernel(const uint32_t* __restrict__ partials,
                                                          int64_t cells, int32_t K,
                                                          int32_t n_chunks, int32_t rmse,
                                                          void* __restrict__ out) {
    for (int64_t cell = int64_t(blockIdx.x) * 256 + threadIdx.x; cell < cells;
         cell += int64_t(gridDim.x) * 256)
        merge_cell<PREC>(partials, cells, K, n_chunks, rmse != 0, out, cell);
}

void hist_init_attrs(int max_lds) {
    const void* fns[] = {(const void*)hist_kernel<CBH_PREC_FP32, 1>,
                         (const void*)hist_kernel<CBH_PREC_FP32, 0>,
                         (const void*)hist_kernel<CBH_PREC_TWOFLOAT, 1>,
                         (const void*)hist_kernel<CBH_PREC_TWOFLOAT, 0>,
                         (const void*)hist_kernel<CBH_PREC_INT16, 1>,
                         (const void*)hist_kernel<CBH_PREC_INT16, 0>};
    for (const void* f : fns)
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
}

template <int PREC>
static void launch_hist_prec(const HistArgs& a, const HistPlan& plan, int max_lds,
                             hipStream_t s) {
    const int64_t grid = 8 * ((plan.n_blocks + 7) / 8);
    (void)max_lds;
    if (a.K == 1)
        hist_kernel<PREC, 1><<<(unsigned)grid, 256, (size_t)plan.lds_bytes, s>>>(a);
    else
        hist_kernel<PREC, 0><<<(unsigned)grid, 256, (size_t)plan.lds_bytes, s>>>(a);
}

int launch_hist(cbh_ctx* ctx, const cbh_problem* p, int32_t level, int32_t precision,
                const HistPlan& plan, void* hist_out, void* partials, hipStream_t s) {
    HistArgs a;
    a.bins = p->bins;
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
    a.L = 1 << level;
    a.fb = plan.fb;
    a.lt = plan.lt;
    a.n_fgroups = plan.n_fgroups;
    a.n_ltiles = plan.n_ltiles;
    a.wpc = plan.words_per_cell;
    a.rmse = p->loss == CBH_LOSS_RMSE;
    switch (precision) {
        case CBH_PREC_FP32: launch_hist_prec<CBH_PREC_FP32>(a, plan, ctx->max_lds, s); break;
        case CBH_PREC_TWOFLOAT:
            launch_hist_prec<CBH_PREC_TWOFLOAT>(a, plan, ctx->max_lds, s);
            break;
        default: launch_hist_prec<CBH_PREC_INT16>(a, plan, ctx->max_lds, s); break;
    }
    CBH_LAUNCHED();
    const int64_t cells = int64_t(a.L) * a.F * a.B;
    const int grid = (int)std::min<int64_t>((cells + 255) / 256, int64_t(ctx->num_cus) * 16);
    switch (precision) {
        case CBH_PREC_FP32:
            hist_reduce_kernel<CBH_PREC_FP32><<<grid, 256, 0, s>>>(
                (const uint32_t*)partials, cells, a.K, plan.n_chunks, a.rmse, hist_out);
            break;
        case CBH_PREC_TWOFLOAT:
            hist_reduce_kernel<CBH_PREC_TWOFLOAT><<<grid, 256, 0, s>>>(
                (const uint32_t*)partials, cells, a.K, plan.n_chunks, a.rmse, hist_out);
            break;
        default:
            hist_reduce_kernel<CBH_PREC_INT16><<<grid, 256, 0, s>>>(
                (const uint32_t*)partials, cells, a.K, plan.n_chunks, a.rmse, hist_out);
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
        // non-negative floats order like their bit patterns
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
    rc = ensure_ws(ctx, 8 * CBH_MAX_K);
    if (rc) return rc;
    uint32_t* maxbits = (uint32_t*)ctx->ws;
    hipStream_t s = (hipStream_t)stream;
    const int with_h = prob->loss != CBH_LOSS_RMSE;
    zero_u32_kernel<<<1, 64, 0, s>>>(maxbits, 2 * prob->K);
    const int gx = (int)std::min<int64_t>((prob->n + 255) / 256, ctx->num_cus * 4);
    grad_max_kernel<<<dim3(gx, prob->K), 256, 0, s>>>(prob->g, prob->h, prob->n, prob->K,
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
    const HistKnobs kn = knobs_for(ctx, prob->n_features, prob->max_bins, prob->K, level,
                                   precision, prob->n);
    const HistPlan plan = plan_hist(kn, prob->n, prob->n_features, prob->max_bins, prob->K, L,
                                    precision, ctx->max_lds);
    CBH_REQUIRE(int64_t(prob->max_bins) * plan.words_per_cell * 4 <= ctx->max_lds,
                CBH_EUNSUPPORTED, "one leaf row of %d bins x %d words does not fit in LDS",
                prob->max_bins, plan.words_per_cell);
    const int64_t part_bytes =
        int64_t(plan.n_chunks) * L * prob->n_features * prob->max_bins * plan.words_per_cell * 4;
    rc = ensure_ws(ctx, part_bytes);
    if (rc) return rc;
    return launch_hist(ctx, prob, level, precision, plan, hist_out, ctx->ws,
                       (hipStream_t)stream);
}

}  // extern "C"
