// Split scoring and argmax (Sec. 3: the first phase scores candidate splits
// and keeps the best; Sec. 4: one split per level of an oblivious tree).
//
// Score of splitting every current leaf L by (f, k):
//   S(f, k) = sum_L sum_c  Gl^2 / (Hl + l2) + Gr^2 / (Hr + l2)
// (the paper gives no formula; this is the gain of the L2-regularised
// second-order objective, with the parent term, equal for all candidates,
// dropped). A side with H + l2 == 0 contributes 0.
//
// Kernel 1: one block per feature; each wave takes (leaf, class) rows of the
// histogram, one lane per 4 consecutive bins, forms bin prefixes with a wave
// scan (in the histogram's own type), and accumulates the per-border terms in
// double registers. The waves'
// partial scores are added in wave order (deterministic), then the block
// keeps its best and second-best border. The last block to finish (a
// device counter, reset by that block, so the launch needs no clearing and
// can be replayed from a graph) reduces the per-feature winners to the
// level's split with the tie rule "largest score, then smallest feature, then
// smallest border".
#include <cmath>

#include "common.h"
#include "kernels_dev.h"

namespace cbh {

// (leaf, class) rows in flight per feature: 16 waves once a feature has more
// than 4 rows, else 4 (a smaller block for the short early levels)
constexpr int kScoreWaves = 16;
constexpr int kScoreWavesSmall = 4;

template <int PREC, int NW>
__global__ __launch_bounds__(64 * NW) void score_split_kernel(
    ScoreRow r, const int32_t* n_bins, int32_t L, float* scores, FeatBest* fbest,
    uint32_t* __restrict__ counter, cbh_split* __restrict__ out) {
    const int f = blockIdx.x;
    score_feature<PREC, NW>(r, L, f, n_bins[f], scores, &fbest[f]);
    __shared__ uint32_t last;
    __syncthreads();
    if (threadIdx.x == 0) {
        // publish this block's winner, then count the block in
        __threadfence();
        last = atomicAdd(counter, 1u) == gridDim.x - 1 ? 1u : 0u;
    }
    __syncthreads();
    if (last) {
        __threadfence();
        argmax_features(fbest, r.F, r.B - 1, out);
        if (threadIdx.x == 0) atomicExch(counter, 0u);
    }
}

int64_t score_scratch_bytes(const cbh_problem* p) {
    return align_up(int64_t(p->n_features) * sizeof(FeatBest), 256);
}

// Scratch of cbh_score_splits_noalloc (the entry point for callers that
// cannot allocate device memory): the last-block counter in the first 256
// bytes, then one FeatBest per feature, for at most kStaticScoreFeatures
// features (1 MB). Every GPU holds its own copy until the process ends; in
// host code the array's name is not a device address, so the library keeps
// the address hipGetSymbolAddress returns for each device (in its context)
// and passes that to the kernels.
constexpr int64_t kStaticScoreFeatures = 65536;
constexpr int64_t kStaticScoreBytes = 256 + kStaticScoreFeatures * sizeof(FeatBest);
static __device__ __align__(256) unsigned char scratch[kStaticScoreBytes];

int score_static_init(cbh_ctx* ctx) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
        (void)hipGetLastError();
        set_error("hipGetSymbolAddress of the static score scratch failed: %s",
                  hipGetErrorString(e));
        return CBH_EDEVICE;
    }
    // the counter must start at zero; the kernel's last block resets it
    CBH_HIP(hipMemset(ptr, 0, 256));
    ctx->score_static = ptr;
    return CBH_OK;
}

int launch_score(cbh_ctx* ctx, const cbh_problem* p, int32_t level, const void* hist,
                 int32_t precision, double l2, cbh_split* best, float* scores, void* scratch,
                 hipStream_t s, uint32_t* counter_in) {
    ScoreRow r;
    r.hist = hist;
    r.grad_scale = p->grad_scale;
    r.F = p->n_features;
    r.B = p->max_bins;
    r.K = p->K;
    r.rmse = count_stat(p);
    r.l2 = l2;
    const int L = 1 << level;
    FeatBest* fb = (FeatBest*)scratch;
    uint32_t* counter = counter_in ? counter_in : ctx->d_flags + 1;
    const bool small = int64_t(L) * r.K <= kScoreWavesSmall;
#define CBH_SCORE(P)                                                                      \
    if (small)                                                                            \
        score_split_kernel<P, kScoreWavesSmall><<<r.F, 64 * kScoreWavesSmall, 0, s>>>(    \
            r, p->n_bins, L, scores, fb, counter, best);                                  \
    else                                                                                  \
        score_split_kernel<P, kScoreWaves><<<r.F, 64 * kScoreWaves, 0, s>>>(              \
            r, p->n_bins, L, scores, fb, counter, best);
    switch (out_prec(precision)) {
        case CBH_PREC_FP32: CBH_SCORE(CBH_PREC_FP32) break;
        case CBH_PREC_TWOFLOAT: CBH_SCORE(CBH_PREC_TWOFLOAT) break;
        default: CBH_SCORE(CBH_PREC_INT16) break;
    }
#undef CBH_SCORE
    CBH_LAUNCHED();
    return CBH_OK;
}

}  // namespace cbh

using namespace cbh;

extern "C" int cbh_score_splits(cbh_ctx* ctx, const cbh_problem* prob, int32_t level,
                                const void* hist, int32_t precision, double l2,
                                cbh_split* best_out, float* scores_out, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_precision(prob, precision);
    if (rc) return rc;
    CBH_ARG(level >= 0 && level < prob->depth, "level %d outside [0, depth)", level);
    CBH_ARG(hist && best_out, "hist / best_out is NULL");
    CBH_ARG(l2 >= 0 && std::isfinite(l2), "l2 must be finite and >= 0");
    rc = ensure_ws(ctx, score_scratch_bytes(prob), stream);
    if (rc) return rc;
    return launch_score(ctx, prob, level, hist, precision, l2, best_out, scores_out, ctx->ws,
                        (hipStream_t)stream);
}

extern "C" int cbh_score_splits_noalloc(cbh_ctx* ctx, const cbh_problem* prob, int32_t level,
                                        const void* hist, int32_t precision, double l2,
                                        cbh_split* best_out, float* scores_out, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    int rc = validate_problem(prob);
    if (rc) return rc;
    rc = validate_precision(prob, precision);
    if (rc) return rc;
    CBH_ARG(level >= 0 && level < prob->depth, "level %d outside [0, depth)", level);
    CBH_ARG(hist && best_out, "hist / best_out is NULL");
    CBH_ARG(l2 >= 0 && std::isfinite(l2), "l2 must be finite and >= 0");
    CBH_ARG(prob->n_features <= kStaticScoreFeatures,
            "cbh_score_splits_noalloc takes at most %lld features (got %d); use "
            "cbh_score_splits",
            (long long)kStaticScoreFeatures, prob->n_features);
    CBH_ARG(ctx->score_static != nullptr, "the context has no static score scratch");
    unsigned char* base = static_cast<unsigned char*>(ctx->score_static);
    return launch_score(ctx, prob, level, hist, precision, l2, best_out, scores_out, base + 256,
                        (hipStream_t)stream, reinterpret_cast<uint32_t*>(base));
}
