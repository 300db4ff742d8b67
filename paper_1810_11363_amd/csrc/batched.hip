// Batched levels over several independent problems and HIP-graph capture of a
// whole boosting iteration.
//
// The paper trains s permutations side by side (Sec. 3: several
// permutations, each with its own models) and its GPU code processes many
// histograms per launch (Sec. 5); batching independent problems, folds and
// permutations into shared launches is this library's MI355X design. A plan
// holds device copies of all descriptors; one level of all problems runs as
//   1. one histogram launch over the tiles of every problem (work list),
//   2. one merge launch over every problem's partial tiles,
//   3. one score launch over every (problem, feature),
//   4. one argmax launch (a block per problem),
//   5. one apply launch over the rows of every problem,
// so the launch count per level does not grow with the number of problems.
// With histogram subtraction (one class per problem), levels >= 1 start with
// a sixth launch over the rows of every problem that picks the smaller child
// of each parent and writes per-row slot codes; the histogram launch then
// accumulates only the smaller children and the merge launch writes both
// children (the larger one as parent minus smaller).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "kernels_dev.h"
#include "update_dev.h"

namespace cbh {

// Device descriptor of one problem inside a plan.
struct DevProb {
    const uint8_t* const* bins;
    const int32_t* n_bins;
    const float* g;
    const float* h;
    const uint32_t* gq;
    const float* grad_scale;
    uint16_t* leaf;
    void* hist;
    uint32_t* partials;      // this problem's partial tiles (workspace)
    int64_t n;
    int32_t F, B, K, rmse;
    const int64_t* seg;      // per-feature segment strides, NULL = columns
    const void* parent;      // subtraction: the previous level's histogram, else NULL
    uint8_t* side;           // subtraction: [half] smaller child of each parent
    uint16_t* codes;         // subtraction: [n] per-row slot codes
    const uint16_t* rowcode; // slot codes the histogram reads (codes, or the leaf)
};

// One histogram work item: (problem, chunk, feature group, leaf tile) and its plan.
struct DevTile {
    int32_t prob;
    int32_t fg;
    int32_t lt_i;
    int32_t chunk;
};

// The tiles of one row chunk of one problem (its feature groups and slot
// tiles, which read the same rows) and their work, rows x features x slot
// tiles.
struct TileGroup {
    int64_t work;
    int32_t prob, chunk, n_fgroups, n_ltiles;
};

// Work list of a level. The launches run the first eighth of the list on
// XCD 0, the next on XCD 1, and so on (block b runs on XCD b mod 8). Problems
// differ in size, so the groups are dealt out by work: largest first, each to
// the XCD with the least work so far; every XCD's share is then padded with
// empty tiles (prob = -1) to a common length. A group stays on one XCD, where
// its tiles share the rows' statistics and row codes in L2.
static void deal_tiles(std::vector<TileGroup>& groups, std::vector<DevTile>& tiles) {
    std::stable_sort(groups.begin(), groups.end(),
                     [](const TileGroup& a, const TileGroup& b) { return a.work > b.work; });
    std::vector<DevTile> share[8];
    int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (const TileGroup& gr : groups) {
        int x = 0;
        for (int k = 1; k < 8; ++k)
            if (load[k] < load[x]) x = k;
        load[x] += gr.work;
        for (int fg = 0; fg < gr.n_fgroups; ++fg)
            for (int lt = 0; lt < gr.n_ltiles; ++lt)
                share[x].push_back(DevTile{gr.prob, fg, lt, gr.chunk});
    }
    size_t len = 0;
    for (const auto& v : share) len = std::max(len, v.size());
    tiles.clear();
    tiles.reserve(8 * len);
    for (auto& v : share) {
        v.resize(len, DevTile{-1, 0, 0, 0});
        tiles.insert(tiles.end(), v.begin(), v.end());
    }
}

struct LevelPlan {
    std::vector<HistPlan> plans;       // per problem
    std::vector<int64_t> part_off;     // per problem, bytes into workspace
    int64_t part_bytes = 0;
    int64_t n_tiles = 0;
    DevTile* d_tiles = nullptr;        // device work list
    struct DevHP {
        int32_t fb, lt, n_fgroups, n_ltiles, n_chunks, wpc, rep, pad;
        int64_t rows_per_chunk, lds_bytes;
    }* d_plans = nullptr;              // per problem
    int64_t max_lds = 0;
    int32_t kind = 0;                  // 0 rows over lanes, 1 lanes over features
    int32_t W = 0;                     // lanes-over-features group width (all problems)
    int32_t mode = 0;                  // lanes-over-features slot mode (all problems)
    int64_t cells_total = 0;           // sum over problems of L*F*B
    int64_t* d_cell_off = nullptr;     // per problem prefix of cells (P+1)
    int64_t score_total = 0;           // sum of F
    int64_t* d_feat_off = nullptr;     // per problem prefix of features (P+1)
    int64_t rows_total = 0;
    int64_t* d_row_off = nullptr;      // per problem prefix of rows (P+1)
    int32_t sub = 0;                   // built by subtraction (levels >= 1)
    int64_t rb_total = 0;              // row blocks of the side/code launch
    int64_t* d_rb_off = nullptr;       // per problem prefix of row blocks (P+1)
    // the fused launch (kind 1): problem order of its merge, score, argmax
    // and apply items, their prefixes in that order, tiles per problem, and
    // the level's counters (bytes into the plan workspace)
    int32_t* d_order = nullptr;
    int32_t* d_hcount = nullptr;
    int64_t* d_goff = nullptr;
    int64_t* d_soff = nullptr;
    int64_t* d_xoff = nullptr;
    int64_t cnt_off = 0;
};

constexpr int64_t kSideRows = 16384;   // rows per block of the side/code launch
// LDS the fused launch keeps out of the histogram tile (its own small
// static arrays); the tile budget of a batched plan leaves this much free
constexpr int kFusedStaticLds = 1024;

}  // namespace cbh

struct cbh_batch {
    cbh_ctx* ctx = nullptr;
    int32_t P = 0;
    int32_t precision = 0;
    int32_t depth = 0;
    std::vector<cbh_problem> probs;
    std::vector<void*> hist;
    cbh_split* best = nullptr;      // device [P][depth]
    cbh::DevProb* d_probs = nullptr;
    std::vector<cbh::LevelPlan> levels;
    int64_t ws_need = 0;
    int64_t fbest_off = 0;
    int32_t sub = 0;                // levels >= 1 by subtraction
    int32_t fused = 0;              // one launch per level where the level allows it
    void* ws = nullptr;             // plan-owned partial tiles, feature winners and,
                                    // with subtraction, the second histogram of
                                    // every problem, sides and row codes
    // the tree's second phase for every problem in two launches: per-problem
    // leaf-solve and update arguments (leaf value pointers set per call) and
    // the block prefixes of the two launches
    cbh::SolveArgs* d_solve = nullptr;
    cbh::UpdArgs* d_upd = nullptr;
    int64_t* d_solve_off = nullptr;
    int64_t* d_upd_off = nullptr;
    int64_t solve_blocks = 0, upd_blocks = 0;
};


namespace cbh {

// ---------------------------------------------------------------- kernels
template <int PREC, int RM>
__global__ __launch_bounds__(kHistThreads) void bhist_kernel(const DevProb* __restrict__ probs,
                                                    const DevTile* __restrict__ tiles,
                                                    const LevelPlan::DevHP* __restrict__ plans,
                                                    int64_t n_tiles, int32_t L) {
    extern __shared__ __align__(16) uint32_t lds[];
    const int64_t per_xcd = (n_tiles + 7) / 8;
    const int64_t ti = int64_t(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (ti >= n_tiles) return;
    const DevTile tile = tiles[ti];
    if (tile.prob < 0) return;
    const DevProb pr = probs[tile.prob];
    const LevelPlan::DevHP hp = plans[tile.prob];
    TileArgs t;
    t.bins = pr.bins;
    t.seg = pr.seg;
    t.g = pr.g;
    t.h = pr.h;
    t.gq = pr.gq;
    t.leaf = pr.leaf;
    t.part = pr.partials + int64_t(tile.chunk) * (int64_t(L) * pr.F * pr.B * hp.wpc);
    t.n = pr.n;
    t.r0 = int64_t(tile.chunk) * hp.rows_per_chunk;
    t.r1 = min(pr.n, t.r0 + hp.rows_per_chunk);
    t.F = pr.F;
    t.B = pr.B;
    t.K = pr.K;
    t.L = L;
    t.fb = hp.fb;
    t.lt = hp.lt;
    t.wpc = hp.wpc;
    t.rmse = pr.rmse;
    t.f0 = tile.fg * hp.fb;
    t.nf = min(hp.fb, pr.F - t.f0);
    t.l0 = (uint32_t)tile.lt_i * hp.lt;
    t.side = nullptr;
    t.sub_shift = 0;
    t.rep = hp.rep;
    hist_tile<PREC, 0, RM>(t, lds);
}

// The same work list with the lanes-over-features tile: every problem of the
// level shares W and the slot mode; L is the number of slots (the leaves, or
// the parents in a build by subtraction).
template <int PREC, int RM, int W, int MODE>
__global__ __launch_bounds__(kHistThreads) void blpf_kernel(const DevProb* __restrict__ probs,
                                                   const DevTile* __restrict__ tiles,
                                                   const LevelPlan::DevHP* __restrict__ plans,
                                                   int64_t n_tiles, int32_t L) {
    extern __shared__ __align__(16) uint32_t lds[];
    const int64_t per_xcd = (n_tiles + 7) / 8;
    const int64_t ti = int64_t(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (ti >= n_tiles) return;
    const DevTile tile = tiles[ti];
    if (tile.prob < 0) return;
    const DevProb pr = probs[tile.prob];
    const LevelPlan::DevHP hp = plans[tile.prob];
    LpfBlock b;
    b.bins = pr.bins;
    b.seg = pr.seg;
    b.g = pr.g;
    b.h = pr.h;
    b.gq = pr.gq;
    b.rowcode = pr.rowcode;
    b.F = pr.F;
    b.B = pr.B;
    b.wpc = hp.wpc;
    b.coff = 0;
    const int64_t r0 = int64_t(tile.chunk) * hp.rows_per_chunk;
    const uint32_t s0 = (uint32_t)tile.lt_i * (uint32_t)hp.lt;
    lpf_block<PREC, RM, W, MODE>(b, r0, min(pr.n, r0 + hp.rows_per_chunk), tile.fg, s0,
                                 min((uint32_t)hp.lt, (uint32_t)L - s0),
                                 pr.partials + int64_t(tile.chunk) * (int64_t(L) * pr.F * pr.B * hp.wpc),
                                 0u, lds);
}

// Leaf bit of rows [i0, i1) under split sp (i1 - i0 <= 8, i0 a multiple of
// 8 from the problem's first row): eight rows of one half segment take one
// 8-byte bins load and one 16-byte leaf load and store where aligned.
__device__ __forceinline__ void apply_rows8(const uint8_t* const* bins, const int64_t* seg,
                                           int F, cbh_split sp, uint16_t* leaf, int64_t i0,
                                           int64_t i1, int level) {
    int f = sp.feature, k = sp.border;
    if (f < 0 || f >= F) {
        if (level != 0) return;
        f = 0;
        k = 255;
    }
    const uint8_t* col = bins[f];
    const int64_t stride = seg_stride_of(seg, f);
    const uint32_t bit = 1u << level;
    const uint8_t* half = seg_ptr(col, stride, i0);
    if (i1 - i0 == 8 && (i0 & 7) == 0 && (reinterpret_cast<uintptr_t>(half) & 7) == 0 &&
        (reinterpret_cast<uintptr_t>(leaf + i0) & 15) == 0) {
        // eight rows of one half segment: one 8-byte bins load, one 16-byte
        // leaf load and store
        const uint2 b = *reinterpret_cast<const uint2*>(half);
        uint4 l = level == 0 ? make_uint4(0u, 0u, 0u, 0u)
                             : *reinterpret_cast<const uint4*>(leaf + i0);
        uint32_t lw[4] = {l.x, l.y, l.z, l.w};
#pragma unroll
        for (int r = 0; r < 8; ++r)
            if ((int)(((r < 4 ? b.x : b.y) >> (8 * (r & 3))) & 255u) > k)
                lw[r >> 1] |= bit << (16 * (r & 1));
        *reinterpret_cast<uint4*>(leaf + i0) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
        return;
    }
    for (int64_t i = i0; i < i1; ++i) {
        const uint32_t old = level == 0 ? 0u : leaf[i];
        leaf[i] = (uint16_t)(old | (((int)*seg_ptr(col, stride, i) > k) ? bit : 0u));
    }
}

__device__ __forceinline__ int find_owner(const int64_t* __restrict__ off, int P, int64_t gi) {
    int lo = 0, hi = P - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= gi) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Merge partial tiles of every problem: one thread per (problem, cell).
template <int PREC>
__global__ __launch_bounds__(256) void breduce_kernel(const DevProb* __restrict__ probs,
                                                      const LevelPlan::DevHP* __restrict__ plans,
                                                      const int64_t* __restrict__ cell_off,
                                                      int32_t P, int64_t cells_total) {
    for (int64_t gi = int64_t(blockIdx.x) * 256 + threadIdx.x; gi < cells_total;
         gi += int64_t(gridDim.x) * 256) {
        const int p = find_owner(cell_off, P, gi);
        const DevProb pr = probs[p];
        const int64_t cells = cell_off[p + 1] - cell_off[p];
        const int64_t cell = gi - cell_off[p];
        if (pr.parent) {
            // cell = (parent, feature, bin); the partials hold the smaller child
            const int64_t fbc = int64_t(pr.F) * pr.B;
            const int64_t half = cells / fbc;
            const int64_t par = cell / fbc, rest = cell % fbc;
            const int64_t sd = pr.side[par];
            merge_cell<PREC>(pr.partials, cells, pr.K, plans[p].n_chunks, pr.rmse != 0, pr.hist,
                             cell, (par + sd * half) * fbc + rest,
                             (par + (1 - sd) * half) * fbc + rest, pr.parent);
        } else {
            merge_cell<PREC>(pr.partials, cells, pr.K, plans[p].n_chunks, pr.rmse != 0, pr.hist,
                             cell, cell);
        }
    }
}

// Build by subtraction, first launch: one block per kSideRows rows of a
// problem. Every block finds the smaller child of each of the problem's
// `half` parents (at the previous level's split) in LDS; block 0 of the
// problem stores them. Then each row gets the slot code of the histogram
// launch: its parent if it lies on the smaller side, else 0xffff (skipped).
template <int PREC>
__global__ __launch_bounds__(256) void bside_code_kernel(const DevProb* __restrict__ probs,
                                                         const int64_t* __restrict__ rb_off,
                                                         int32_t P, const cbh_split* __restrict__ best,
                                                         int32_t depth, int32_t level) {
    extern __shared__ uint8_t sd[];
    const int p = find_owner(rb_off, P, blockIdx.x);
    const DevProb pr = probs[p];
    const int64_t rb = int64_t(blockIdx.x) - rb_off[p];
    const int64_t half = int64_t(1) << (level - 1);
    const cbh_split sp = best[int64_t(p) * depth + level - 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t q = wave; q < half; q += 4) {
        const uint8_t v = parent_side<PREC>(pr.parent, q, sp.feature, sp.border, pr.F, pr.B,
                                            pr.K, pr.rmse, lane);
        if (lane == 0) {
            sd[q] = v;
            if (rb == 0) pr.side[q] = v;
        }
    }
    __syncthreads();
    const uint32_t lmask = (uint32_t)half - 1u, shift = (uint32_t)(level - 1);
    const int64_t i0 = rb * kSideRows, i1 = min(pr.n, i0 + kSideRows);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const uint32_t v = gld_u16(pr.leaf + i);
        const uint32_t pp = v & lmask;
        pr.codes[i] = (uint16_t)((((v >> shift) & 1u) == (uint32_t)sd[pp]) ? pp : 0xffffu);
    }
}

// One (problem, feature) per block.
template <int PREC>
__global__ __launch_bounds__(256) void bscore_kernel(const DevProb* __restrict__ probs,
                                                     const int64_t* __restrict__ feat_off,
                                                     int32_t P, int32_t L, double l2,
                                                     FeatBest* __restrict__ fbest) {
    const int64_t gf = blockIdx.x;
    const int p = find_owner(feat_off, P, gf);
    const DevProb pr = probs[p];
    const int f = (int)(gf - feat_off[p]);
    ScoreRow r;
    r.hist = pr.hist;
    r.grad_scale = pr.grad_scale;
    r.F = pr.F;
    r.B = pr.B;
    r.K = pr.K;
    r.rmse = pr.rmse;
    r.l2 = l2;
    score_feature<PREC>(r, L, f, pr.n_bins[f], nullptr, &fbest[gf]);
}

__global__ __launch_bounds__(256) void bargmax_kernel(const DevProb* __restrict__ probs,
                                                      const int64_t* __restrict__ feat_off,
                                                      const FeatBest* __restrict__ fbest,
                                                      cbh_split* __restrict__ best, int32_t depth,
                                                      int32_t level) {
    const int p = blockIdx.x;
    argmax_features(fbest + feat_off[p], probs[p].F, probs[p].B - 1,
                    &best[int64_t(p) * depth + level]);
}

// Apply every problem's split of this level; one thread per 8 rows.
__global__ __launch_bounds__(256) void bapply_kernel(const DevProb* __restrict__ probs,
                                                     const int64_t* __restrict__ row_off,
                                                     int32_t P, const cbh_split* __restrict__ best,
                                                     int32_t depth, int32_t level,
                                                     int64_t groups_total) {
    for (int64_t gq = int64_t(blockIdx.x) * 256 + threadIdx.x; gq < groups_total;
         gq += int64_t(gridDim.x) * 256) {
        const int p = find_owner(row_off, P, gq);
        const DevProb pr = probs[p];
        const int64_t i0 = (gq - row_off[p]) * 8;
        apply_rows8(pr.bins, pr.seg, pr.F, best[int64_t(p) * depth + level], pr.leaf, i0,
                   min(pr.n, i0 + 8), level);
    }
}

// ------------------------------------------- leaf solve and update, batched
// Rows per block of the batched update (4 per thread).
constexpr int64_t kUpdRows = 1024;

// Leaf value pointers of up to 32 problems, passed by value (a captured
// graph keeps the pointers it was captured with).
struct ValsChunk {
    double* v[32];
    int32_t first, count;
};

__global__ void bset_vals_kernel(SolveArgs* __restrict__ sa, UpdArgs* __restrict__ ua,
                                 ValsChunk c) {
    const int j = threadIdx.x;
    if (j < c.count) {
        sa[c.first + j].values = c.v[j];
        ua[c.first + j].values = c.v[j];
    }
}

// Every problem's leaf values: block b belongs to the problem whose block
// range holds it, one wave per (final leaf, class) as leaf_solve_kernel.
__global__ __launch_bounds__(256) void bleaf_solve_kernel(const SolveArgs* __restrict__ sa,
                                                          const int64_t* __restrict__ off,
                                                          int32_t P, double l2) {
    const int p = find_owner(off, P, blockIdx.x);
    SolveArgs a = sa[p];
    a.l2 = l2;
    const int64_t t = (int64_t(blockIdx.x) - off[p]) * 4 + (threadIdx.x >> 6);
    if (t >= (int64_t(1) << a.depth) * a.K) return;
    leaf_solve_one(a, t, threadIdx.x & 63);
}

// Every problem's approx update and loss derivatives: kUpdRows rows of one
// problem per block (add = 0: derivatives of the current approx only).
template <int LOSS>
__global__ __launch_bounds__(256) void bupdate_kernel(const UpdArgs* __restrict__ ua,
                                                      const int64_t* __restrict__ off, int32_t P,
                                                      double lr, int32_t add) {
    const int p = find_owner(off, P, blockIdx.x);
    UpdArgs a = ua[p];
    a.lr = lr;
    a.add = add;
    const int64_t r0 = (int64_t(blockIdx.x) - off[p]) * kUpdRows;
    const int64_t r1 = min(a.n, r0 + kUpdRows);
    for (int64_t i = r0 + threadIdx.x; i < r1; i += 256) update_row<LOSS>(a, i);
}

// ------------------------------------------------ one fused launch per level
// The whole level of every problem in one launch of persistent blocks, with
// no grid-wide barrier. The blocks claim work items in order from queues:
//   C  (subtraction only) per kSideRows rows of a problem: every parent's
//      smaller child and the rows' slot codes (as bside_code_kernel); every
//      block waits once for all of them before its histogram tiles;
//   H  histogram tiles, from 8 queues holding the dealt work list's 8 XCD
//      shares (block b takes queue b mod 8, the XCD it runs on);
//   G  then, from one queue: merge items (kFusedMergeCells cells of a
//      problem), score items (kFusedScoreFeatures features of a problem),
//      argmax items (one problem) and apply items (kFusedApplyRows rows of a
//      problem), the
//      problems in the order their histogram tiles finish in the dealt list.
// An item waits until every item it reads from is done: per-problem "done"
// counters, raised by each item after its writes are published, gate the
// stage that follows (a merge waits for its problem's H tiles, a score for
// its merges, the argmax for its scores, an apply for its argmax). Every
// item waited on was claimed earlier by a running block that
// waits only on still earlier items, so the earliest unfinished item can
// always run: the waits end. A wait is nonetheless bounded (it raises
// FLAG_FUSED_WAIT, reported by cbh_sync, and gives up). The last block to
// leave resets every counter for the next launch, so the launch replays from
// a graph with no clearing.
constexpr int kFusedMergeCells = 16384;
constexpr int64_t kFusedApplyRows = 65536;
constexpr int kFusedScoreFeatures = 8;    // features per score item
// counters: [0] C head, [1..8] H heads, [9] G head, [10] blocks out,
// [11] C items done, then 5 per problem (C, H, M, S, A done)
constexpr int kFusedCounters = 16;

struct FusedArgs {
    const DevProb* probs;
    const DevTile* tiles;
    const LevelPlan::DevHP* plans;
    const int64_t* cell_off;     // per problem prefix of merge cells (P+1)
    const int64_t* feat_off;     // per problem prefix of features (P+1)
    const int64_t* rb_off;       // per problem prefix of C items (P+1), or NULL
    const int64_t* g_off;        // per queue position: prefix of merge items (P+1)
    const int64_t* s_off;        // per queue position: prefix of score items (P+1), each
                                 // kFusedScoreFeatures features
    const int64_t* x_off;        // per queue position: prefix of apply items (P+1)
    const int32_t* order;        // problem at each queue position
    const int32_t* h_count;      // histogram tiles per problem
    FeatBest* fbest;
    cbh_split* best;
    uint32_t* cnt;               // this level's counters
    uint32_t* err;               // device error flags
    int64_t n_tiles;             // a multiple of 8
    int64_t rb_total;
    int32_t P, L, slots, depth, level;
    double l2;
};

template <int PREC, int RM, int W, int MODE>
__global__ __launch_bounds__(kHistThreads) void bfused_kernel(FusedArgs a) {
    constexpr int OP = out_prec(PREC);
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ int64_t s_item;
    const int P = a.P;
    uint32_t* done = a.cnt + kFusedCounters;            // [5][P]: C, H, M, S, A
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = blockDim.x >> 6;
    auto claim = [&](uint32_t* head) -> int64_t {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(head, 1u);
        __syncthreads();
        return s_item;
    };
    // One thread polls (relaxed, coherent at device scope) and then takes one
    // acquire fence for the block; the barrier orders the other waves' reads
    // after it. A signal: the barrier completes every wave's stores to L2,
    // then one release fence and the count.
    auto wait_for = [&](uint32_t* c, uint32_t target) {
        if (threadIdx.x == 0) {
            uint32_t spins = 0;
            while (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                __builtin_amdgcn_s_sleep(4);
                if (++spins == (1u << 24)) {
                    atomicOr(a.err, FLAG_FUSED_WAIT);
                    break;
                }
            }
            __threadfence();
        }
        __syncthreads();
    };
    auto signal = [&](uint32_t* c) {
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            atomicAdd(c, 1u);
        }
    };
    // ---- C: sides and row codes (levels >= 1 by subtraction)
    if (a.rb_total > 0) {
        const int64_t half = int64_t(1) << (a.level - 1);
        for (;;) {
            const int64_t i = claim(a.cnt + 0);
            if (i >= a.rb_total) break;
            const int p = find_owner(a.rb_off, P, i);
            const DevProb pr = a.probs[p];
            const int64_t rb = i - a.rb_off[p];
            const cbh_split sp = a.best[int64_t(p) * a.depth + a.level - 1];
            uint8_t* sd = reinterpret_cast<uint8_t*>(lds);
            for (int64_t q = wave; q < half; q += nwaves) {
                const uint8_t v = parent_side<OP>(pr.parent, q, sp.feature, sp.border, pr.F,
                                                  pr.B, pr.K, pr.rmse, lane);
                if (lane == 0) {
                    sd[q] = v;
                    if (rb == 0) pr.side[q] = v;
                }
            }
            __syncthreads();
            const uint32_t lmask = (uint32_t)half - 1u, shift = (uint32_t)(a.level - 1);
            const int64_t i0 = rb * kSideRows, i1 = min(pr.n, i0 + kSideRows);
            for (int64_t r = i0 + threadIdx.x; r < i1; r += blockDim.x) {
                const uint32_t v = gld_u16(pr.leaf + r);
                const uint32_t pp = v & lmask;
                pr.codes[r] =
                    (uint16_t)((((v >> shift) & 1u) == (uint32_t)sd[pp]) ? pp : 0xffffu);
            }
            signal(a.cnt + 11);
        }
        // every block claims C items before any H tile, so waiting once for
        // all of them costs one fence per block, not one per tile
        wait_for(a.cnt + 11, (uint32_t)a.rb_total);
    }
    // ---- H: histogram tiles of this block's XCD share
    {
        const int x = blockIdx.x & 7;
        const int64_t per = a.n_tiles / 8;
        for (;;) {
            const int64_t j = claim(a.cnt + 1 + x);
            if (j >= per) break;
            const DevTile tile = a.tiles[x * per + j];
            if (tile.prob < 0) continue;
            const int p = tile.prob;
            const DevProb pr = a.probs[p];
            const LevelPlan::DevHP hp = a.plans[p];
            LpfBlock b;
            b.bins = pr.bins;
            b.seg = pr.seg;
            b.g = pr.g;
            b.h = pr.h;
            b.gq = pr.gq;
            b.rowcode = pr.rowcode;
            b.F = pr.F;
            b.B = pr.B;
            b.wpc = hp.wpc;
            b.coff = 0;
            const int64_t r0 = int64_t(tile.chunk) * hp.rows_per_chunk;
            const uint32_t s0 = (uint32_t)tile.lt_i * (uint32_t)hp.lt;
            __syncthreads();
            lpf_block<PREC, RM, W, MODE>(
                b, r0, min(pr.n, r0 + hp.rows_per_chunk), tile.fg, s0,
                min((uint32_t)hp.lt, (uint32_t)a.slots - s0),
                pr.partials + int64_t(tile.chunk) * (int64_t(a.slots) * pr.F * pr.B * hp.wpc),
                0u, lds);
            signal(done + P + p);
        }
    }
    // ---- G: merges, scores, argmax and leaf bits, problem by problem
    const int64_t nM = a.g_off[P], nS = a.s_off[P], nX = a.x_off[P];
    const int64_t total = nM + nS + P + nX;
    for (;;) {
        const int64_t i = claim(a.cnt + 9);
        if (i >= total) break;
        if (i < nM) {
            const int k = find_owner(a.g_off, P, i);
            const int p = a.order[k];
            wait_for(done + P + p, (uint32_t)a.h_count[p]);
            const DevProb pr = a.probs[p];
            const int64_t cells = a.cell_off[p + 1] - a.cell_off[p];
            const int64_t c0 = (i - a.g_off[k]) * kFusedMergeCells;
            const int64_t c1 = min(cells, c0 + kFusedMergeCells);
            for (int64_t cell = c0 + threadIdx.x; cell < c1; cell += blockDim.x) {
                const int nch = a.plans[p].n_chunks;
                if (pr.parent) {
                    const int64_t fbc = int64_t(pr.F) * pr.B;
                    const int64_t half = cells / fbc;
                    const int64_t par = cell / fbc, rest = cell % fbc;
                    const int64_t sd = pr.side[par];
                    merge_cell<OP>(pr.partials, cells, pr.K, nch, pr.rmse != 0, pr.hist, cell,
                                   (par + sd * half) * fbc + rest,
                                   (par + (1 - sd) * half) * fbc + rest, pr.parent);
                } else {
                    merge_cell<OP>(pr.partials, cells, pr.K, nch, pr.rmse != 0, pr.hist, cell,
                                   cell);
                }
            }
            signal(done + 2 * P + p);
        } else if (i < nM + nS) {
            const int64_t si = i - nM;
            const int k = find_owner(a.s_off, P, si);
            const int p = a.order[k];
            wait_for(done + 2 * P + p, (uint32_t)(a.g_off[k + 1] - a.g_off[k]));
            const DevProb pr = a.probs[p];
            ScoreRow r;
            r.hist = pr.hist;
            r.grad_scale = pr.grad_scale;
            r.F = pr.F;
            r.B = pr.B;
            r.K = pr.K;
            r.rmse = pr.rmse;
            r.l2 = a.l2;
            const int f0 = (int)(si - a.s_off[k]) * kFusedScoreFeatures;
            const int f1 = min(pr.F, f0 + kFusedScoreFeatures);
            for (int f = f0; f < f1; ++f) {
                __syncthreads();
                score_feature_in<OP, 16>(r, a.L, f, pr.n_bins[f], nullptr,
                                         &a.fbest[a.feat_off[p] + f],
                                         reinterpret_cast<ScoreLds<16>*>(lds));
            }
            signal(done + 3 * P + p);
        } else if (i < nM + nS + P) {
            const int k = (int)(i - nM - nS);
            const int p = a.order[k];
            wait_for(done + 3 * P + p, (uint32_t)(a.s_off[k + 1] - a.s_off[k]));
            argmax_features(a.fbest + a.feat_off[p], a.probs[p].F, a.probs[p].B - 1,
                            &a.best[int64_t(p) * a.depth + a.level]);
            signal(done + 4 * P + p);
        } else {
            const int64_t xi = i - nM - nS - P;
            const int k = find_owner(a.x_off, P, xi);
            const int p = a.order[k];
            wait_for(done + 4 * P + p, 1u);
            const DevProb pr = a.probs[p];
            const cbh_split sp = a.best[int64_t(p) * a.depth + a.level];
            const int64_t x0 = (xi - a.x_off[k]) * kFusedApplyRows;
            const int64_t x1 = min(pr.n, x0 + kFusedApplyRows);
            for (int64_t i0 = x0 + int64_t(threadIdx.x) * 8; i0 < x1; i0 += int64_t(blockDim.x) * 8)
                apply_rows8(pr.bins, pr.seg, pr.F, sp, pr.leaf, i0, min(x1, i0 + 8), a.level);
        }
    }
    // the last block out resets the counters for the next launch
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(a.cnt + 10, 1u) == gridDim.x - 1) {
            for (int k = 0; k < kFusedCounters + 5 * P; ++k) a.cnt[k] = 0u;
            __threadfence();
        }
    }
}

void batch_init_attrs(int max_lds) {
    const void* fns[] = {
        (const void*)bhist_kernel<CBH_PREC_FP32, 0>, (const void*)bhist_kernel<CBH_PREC_FP32, 1>,
        (const void*)bhist_kernel<CBH_PREC_TWOFLOAT, 0>,
        (const void*)bhist_kernel<CBH_PREC_TWOFLOAT, 1>,
        (const void*)bhist_kernel<CBH_PREC_INT16, 0>, (const void*)bhist_kernel<CBH_PREC_INT16, 1>,
        (const void*)bhist_kernel<CBH_PREC_F64, 0>, (const void*)bhist_kernel<CBH_PREC_F64, 1>};
    for (const void* f : fns)
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
#define CBH_BLPF_ATTR(P, R, M)                                                               \
    {                                                                                        \
        const void* l[] = {(const void*)blpf_kernel<P, R, 32, M>,                            \
                           (const void*)blpf_kernel<P, R, 16, M>,                            \
                           (const void*)blpf_kernel<P, R, 8, M>,                             \
                           (const void*)blpf_kernel<P, R, 4, M>};                            \
        for (const void* f : l)                                                              \
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds); \
    }
#define CBH_BLPF_ATTR3(P, R) CBH_BLPF_ATTR(P, R, 0) CBH_BLPF_ATTR(P, R, 1) CBH_BLPF_ATTR(P, R, 2)
    CBH_BLPF_ATTR3(CBH_PREC_FP32, 0)
    CBH_BLPF_ATTR3(CBH_PREC_FP32, 1)
    CBH_BLPF_ATTR3(CBH_PREC_TWOFLOAT, 0)
    CBH_BLPF_ATTR3(CBH_PREC_TWOFLOAT, 1)
    CBH_BLPF_ATTR3(CBH_PREC_INT16, 0)
    CBH_BLPF_ATTR3(CBH_PREC_F64, 0)
    CBH_BLPF_ATTR3(CBH_PREC_F64, 1)
#undef CBH_BLPF_ATTR3
#undef CBH_BLPF_ATTR
#define CBH_FUSED_ATTR(P, R, M)                                                              \
    {                                                                                        \
        const void* l[] = {(const void*)bfused_kernel<P, R, 32, M>,                          \
                           (const void*)bfused_kernel<P, R, 16, M>,                          \
                           (const void*)bfused_kernel<P, R, 8, M>,                           \
                           (const void*)bfused_kernel<P, R, 4, M>};                          \
        for (const void* f : l)                                                              \
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,          \
                                      max_lds - kFusedStaticLds);                            \
    }
#define CBH_FUSED_ATTR3(P, R) CBH_FUSED_ATTR(P, R, 0) CBH_FUSED_ATTR(P, R, 1) CBH_FUSED_ATTR(P, R, 2)
    CBH_FUSED_ATTR3(CBH_PREC_FP32, 0)
    CBH_FUSED_ATTR3(CBH_PREC_FP32, 1)
    CBH_FUSED_ATTR3(CBH_PREC_TWOFLOAT, 0)
    CBH_FUSED_ATTR3(CBH_PREC_TWOFLOAT, 1)
    CBH_FUSED_ATTR3(CBH_PREC_INT16, 0)
    CBH_FUSED_ATTR3(CBH_PREC_F64, 0)
    CBH_FUSED_ATTR3(CBH_PREC_F64, 1)
#undef CBH_FUSED_ATTR3
#undef CBH_FUSED_ATTR
}

template <int PREC, int RM, int MODE>
static void launch_blpf_mode(const cbh_batch* b, const LevelPlan& lp, int L, dim3 grd,
                             size_t lds, hipStream_t s) {
    switch (lp.W) {
        case 32: blpf_kernel<PREC, RM, 32, MODE><<<grd, kHistThreads, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L); break;
        case 16: blpf_kernel<PREC, RM, 16, MODE><<<grd, kHistThreads, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L); break;
        case 8: blpf_kernel<PREC, RM, 8, MODE><<<grd, kHistThreads, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L); break;
        default: blpf_kernel<PREC, RM, 4, MODE><<<grd, kHistThreads, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L); break;
    }
}

template <int PREC, int RM>
static void launch_blpf(const cbh_batch* b, const LevelPlan& lp, int L, dim3 grd, size_t lds,
                        hipStream_t s) {
    if (lp.mode == 0) launch_blpf_mode<PREC, RM, 0>(b, lp, L, grd, lds, s);
    else if (lp.mode == 1) launch_blpf_mode<PREC, RM, 1>(b, lp, L, grd, lds, s);
    else launch_blpf_mode<PREC, RM, 2>(b, lp, L, grd, lds, s);
}

template <int PREC, int RM, int MODE>
static void launch_fused_mode(const FusedArgs& fa, int W, dim3 grd, size_t lds, hipStream_t s) {
    switch (W) {
        case 32: bfused_kernel<PREC, RM, 32, MODE><<<grd, kHistThreads, lds, s>>>(fa); break;
        case 16: bfused_kernel<PREC, RM, 16, MODE><<<grd, kHistThreads, lds, s>>>(fa); break;
        case 8: bfused_kernel<PREC, RM, 8, MODE><<<grd, kHistThreads, lds, s>>>(fa); break;
        default: bfused_kernel<PREC, RM, 4, MODE><<<grd, kHistThreads, lds, s>>>(fa); break;
    }
}

template <int PREC, int RM>
static void launch_fused(const FusedArgs& fa, const LevelPlan& lp, dim3 grd, size_t lds,
                         hipStream_t s) {
    if (lp.mode == 0) launch_fused_mode<PREC, RM, 0>(fa, lp.W, grd, lds, s);
    else if (lp.mode == 1) launch_fused_mode<PREC, RM, 1>(fa, lp.W, grd, lds, s);
    else launch_fused_mode<PREC, RM, 2>(fa, lp.W, grd, lds, s);
}

// The level as one persistent launch (bfused_kernel): as many blocks as the
// chip holds at once, a multiple of 8 (the XCD queues).
static int batch_level_fused(cbh_batch* b, int32_t level, double l2, hipStream_t s) {
    cbh_ctx* ctx = b->ctx;
    LevelPlan& lp = b->levels[level];
    const int L = 1 << level;
    FusedArgs fa;
    fa.probs = b->d_probs;
    fa.tiles = lp.d_tiles;
    fa.plans = lp.d_plans;
    fa.cell_off = lp.d_cell_off;
    fa.feat_off = lp.d_feat_off;
    fa.rb_off = lp.sub ? lp.d_rb_off : nullptr;
    fa.g_off = lp.d_goff;
    fa.s_off = lp.d_soff;
    fa.x_off = lp.d_xoff;
    fa.order = lp.d_order;
    fa.h_count = lp.d_hcount;
    fa.fbest = (FeatBest*)((char*)b->ws + b->fbest_off);
    fa.best = b->best;
    fa.cnt = (uint32_t*)((char*)b->ws + lp.cnt_off);
    fa.err = ctx->d_flags;
    fa.n_tiles = lp.n_tiles;
    fa.rb_total = lp.sub ? lp.rb_total : 0;
    fa.P = b->P;
    fa.L = L;
    fa.slots = lp.sub ? L / 2 : L;
    fa.depth = b->depth;
    fa.level = level;
    fa.l2 = l2;
    const int64_t lds = std::max<int64_t>({lp.max_lds, (int64_t)sizeof(ScoreLds<16>),
                                           int64_t(L / 2)});
    const int per_cu = lds + kFusedStaticLds <= ctx->max_lds / 2 ? 2 : 1;
    const dim3 grd((unsigned)(8 * ((int64_t(ctx->num_cus) * per_cu + 7) / 8)));
    const bool rm = count_stat(&b->probs[0]);
    switch (b->precision) {
        case CBH_PREC_FP32:
            if (rm) launch_fused<CBH_PREC_FP32, 1>(fa, lp, grd, (size_t)lds, s);
            else launch_fused<CBH_PREC_FP32, 0>(fa, lp, grd, (size_t)lds, s);
            break;
        case CBH_PREC_TWOFLOAT:
            if (rm) launch_fused<CBH_PREC_TWOFLOAT, 1>(fa, lp, grd, (size_t)lds, s);
            else launch_fused<CBH_PREC_TWOFLOAT, 0>(fa, lp, grd, (size_t)lds, s);
            break;
        case CBH_PREC_F64:
            if (rm) launch_fused<CBH_PREC_F64, 1>(fa, lp, grd, (size_t)lds, s);
            else launch_fused<CBH_PREC_F64, 0>(fa, lp, grd, (size_t)lds, s);
            break;
        default:
            launch_fused<CBH_PREC_INT16, 0>(fa, lp, grd, (size_t)lds, s);
            break;
    }
    CBH_LAUNCHED();
    return CBH_OK;
}

static int batch_level_launch(cbh_batch* b, int32_t level, double l2, hipStream_t s) {
    cbh_ctx* ctx = b->ctx;
    LevelPlan& lp = b->levels[level];
    if (b->fused && lp.kind == 1) return batch_level_fused(b, level, l2, s);
    const int L = 1 << level;
    const int slots = lp.sub ? L / 2 : L;      // histogram slots: parents or leaves
    const int64_t grid = 8 * ((lp.n_tiles + 7) / 8);
    const bool rm = count_stat(&b->probs[0]);
    const dim3 grd((unsigned)grid), blk(kHistThreads);
    const size_t lds = (size_t)lp.max_lds;
    if (lp.sub) {
        const dim3 sg((unsigned)lp.rb_total);
        const size_t half = (size_t)(L / 2);
        switch (out_prec(b->precision)) {
            case CBH_PREC_FP32:
                bside_code_kernel<CBH_PREC_FP32><<<sg, 256, half, s>>>(
                    b->d_probs, lp.d_rb_off, b->P, b->best, b->depth, level);
                break;
            case CBH_PREC_TWOFLOAT:
                bside_code_kernel<CBH_PREC_TWOFLOAT><<<sg, 256, half, s>>>(
                    b->d_probs, lp.d_rb_off, b->P, b->best, b->depth, level);
                break;
            default:
                bside_code_kernel<CBH_PREC_INT16><<<sg, 256, half, s>>>(
                    b->d_probs, lp.d_rb_off, b->P, b->best, b->depth, level);
                break;
        }
        CBH_LAUNCHED();
    }
    if (lp.kind == 1) {
        switch (b->precision) {
            case CBH_PREC_FP32:
                if (rm) launch_blpf<CBH_PREC_FP32, 1>(b, lp, slots, grd, lds, s);
                else launch_blpf<CBH_PREC_FP32, 0>(b, lp, slots, grd, lds, s);
                break;
            case CBH_PREC_TWOFLOAT:
                if (rm) launch_blpf<CBH_PREC_TWOFLOAT, 1>(b, lp, slots, grd, lds, s);
                else launch_blpf<CBH_PREC_TWOFLOAT, 0>(b, lp, slots, grd, lds, s);
                break;
            case CBH_PREC_F64:
                if (rm) launch_blpf<CBH_PREC_F64, 1>(b, lp, slots, grd, lds, s);
                else launch_blpf<CBH_PREC_F64, 0>(b, lp, slots, grd, lds, s);
                break;
            default:
                launch_blpf<CBH_PREC_INT16, 0>(b, lp, slots, grd, lds, s);
                break;
        }
    } else switch (b->precision) {
        case CBH_PREC_FP32:
            if (rm) bhist_kernel<CBH_PREC_FP32, 1><<<grd, blk, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L);
            else bhist_kernel<CBH_PREC_FP32, 0><<<grd, blk, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L);
            break;
        case CBH_PREC_TWOFLOAT:
            if (rm) bhist_kernel<CBH_PREC_TWOFLOAT, 1><<<grd, blk, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L);
            else bhist_kernel<CBH_PREC_TWOFLOAT, 0><<<grd, blk, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L);
            break;
        case CBH_PREC_F64:
            if (rm) bhist_kernel<CBH_PREC_F64, 1><<<grd, blk, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L);
            else bhist_kernel<CBH_PREC_F64, 0><<<grd, blk, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L);
            break;
        default:
            if (rm) bhist_kernel<CBH_PREC_INT16, 1><<<grd, blk, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L);
            else bhist_kernel<CBH_PREC_INT16, 0><<<grd, blk, lds, s>>>(b->d_probs, lp.d_tiles, lp.d_plans, lp.n_tiles, L);
            break;
    }
    CBH_LAUNCHED();
    const int rg = (int)std::min<int64_t>((lp.cells_total + 255) / 256, ctx->num_cus * 16);
    switch (out_prec(b->precision)) {
        case CBH_PREC_FP32:
            breduce_kernel<CBH_PREC_FP32><<<rg, 256, 0, s>>>(b->d_probs, lp.d_plans,
                                                            lp.d_cell_off, b->P, lp.cells_total);
            break;
        case CBH_PREC_TWOFLOAT:
            breduce_kernel<CBH_PREC_TWOFLOAT><<<rg, 256, 0, s>>>(
                b->d_probs, lp.d_plans, lp.d_cell_off, b->P, lp.cells_total);
            break;
        default:
            breduce_kernel<CBH_PREC_INT16><<<rg, 256, 0, s>>>(b->d_probs, lp.d_plans,
                                                             lp.d_cell_off, b->P, lp.cells_total);
            break;
    }
    CBH_LAUNCHED();
    FeatBest* fb = (FeatBest*)((char*)b->ws + b->fbest_off);
    const double fl2 = l2;
    switch (out_prec(b->precision)) {
        case CBH_PREC_FP32:
            bscore_kernel<CBH_PREC_FP32><<<(unsigned)lp.score_total, 256, 0, s>>>(
                b->d_probs, lp.d_feat_off, b->P, L, fl2, fb);
            break;
        case CBH_PREC_TWOFLOAT:
            bscore_kernel<CBH_PREC_TWOFLOAT><<<(unsigned)lp.score_total, 256, 0, s>>>(
                b->d_probs, lp.d_feat_off, b->P, L, fl2, fb);
            break;
        default:
            bscore_kernel<CBH_PREC_INT16><<<(unsigned)lp.score_total, 256, 0, s>>>(
                b->d_probs, lp.d_feat_off, b->P, L, fl2, fb);
            break;
    }
    bargmax_kernel<<<b->P, 256, 0, s>>>(b->d_probs, lp.d_feat_off, fb, b->best, b->depth, level);
    const int ag = (int)std::min<int64_t>((lp.rows_total + 255) / 256, ctx->num_cus * 8);
    bapply_kernel<<<ag, 256, 0, s>>>(b->d_probs, lp.d_row_off, b->P, b->best, b->depth, level,
                                     lp.rows_total);
    CBH_LAUNCHED();
    return CBH_OK;
}

static void free_levels(cbh_batch* b) {
    for (auto& lp : b->levels) {
        if (lp.d_tiles) (void)hipFree(lp.d_tiles);
        if (lp.d_plans) (void)hipFree(lp.d_plans);
        if (lp.d_cell_off) (void)hipFree(lp.d_cell_off);
        if (lp.d_feat_off) (void)hipFree(lp.d_feat_off);
        if (lp.d_row_off) (void)hipFree(lp.d_row_off);
        if (lp.d_rb_off) (void)hipFree(lp.d_rb_off);
        for (void* q : {(void*)lp.d_order, (void*)lp.d_hcount, (void*)lp.d_goff,
                        (void*)lp.d_soff, (void*)lp.d_xoff})
            if (q) (void)hipFree(q);
    }
    b->levels.clear();
}

template <typename T>
static int upload(T** dst, const std::vector<T>& v) {
    CBH_HIP(hipMalloc((void**)dst, std::max<size_t>(1, v.size()) * sizeof(T)));
    CBH_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return CBH_OK;
}

}  // namespace cbh

using namespace cbh;

extern "C" {

int cbh_batch_create(cbh_ctx* ctx, const cbh_problem* probs, int32_t P, int32_t precision,
                     int32_t subtract, void* const* hist, cbh_split* best, cbh_batch** out) {
    clear_error();
    CBH_ARG(ctx && probs && hist && best && out, "NULL argument");
    *out = nullptr;
    CBH_ARG(P >= 1 && P <= 65536, "P must be in [1, 65536]");
    for (int p = 0; p < P; ++p) {
        int rc = validate_problem(&probs[p]);
        if (rc) return rc;
        CBH_REQUIRE(!packed_bins(&probs[p]), CBH_EUNSUPPORTED,
                    "batched plans take byte bins (problem %d has packed bins)", p);
        if (rc) return rc;
        rc = validate_precision(&probs[p], precision);
        if (rc) return rc;
        CBH_ARG(probs[p].depth == probs[0].depth, "every problem needs the same depth");
        CBH_ARG(probs[p].loss == probs[0].loss, "every problem needs the same loss");
        CBH_ARG(count_stat(&probs[p]) == count_stat(&probs[0]),
                "either every RMSE problem has row weights or none has");
        CBH_ARG(hist[p] != nullptr, "hist[%d] is NULL", p);
        CBH_REQUIRE(tile_lds_bytes(precision, count_stat(&probs[p]), probs[p].K,
                                   probs[p].max_bins, 1) <= ctx->max_lds,
                    CBH_EUNSUPPORTED, "a (leaf, feature) tile of problem %d does not fit in LDS", p);
    }
    cbh_batch* b = new cbh_batch();
    b->ctx = ctx;
    b->P = P;
    b->precision = precision;
    b->depth = probs[0].depth;
    b->probs.assign(probs, probs + P);
    b->hist.assign(hist, hist + P);
    b->best = best;
    // subtraction needs one class per problem
    b->sub = subtract != 0 && b->depth > 1;
    for (int p = 0; p < P; ++p)
        if (probs[p].K != 1) b->sub = 0;
    // workspace layout: [per-level max partials][feature winners], and with
    // subtraction [second histogram per problem][sides per problem][row codes
    // per problem]
    int64_t max_part = 0, tot_feat = 0;
    for (int p = 0; p < P; ++p) tot_feat += probs[p].n_features;
    for (int lvl = 0; lvl < b->depth; ++lvl) {
        LevelPlan lp;
        const int L = 1 << lvl;
        std::vector<DevTile> tiles;
        std::vector<TileGroup> groups;
        std::vector<LevelPlan::DevHP> dplans;
        std::vector<int64_t> cell_off{0}, feat_off{0}, row_off{0};
        int64_t off = 0;
        // in a batch the problems share the chip: aim at a share of the blocks
        auto batch_knobs = [&](const cbh_problem& pr) {
            const HistKnobs kn =
                knobs_for(ctx, pr.n_features, pr.max_bins, pr.K, lvl, precision, pr.n, 0);
            HistKnobs kb = kn;
            kb.target_blocks = std::max<int32_t>(
                64, (int32_t)(int64_t(kn.target_blocks) * 1 / std::max(1, std::min(P, 8))));
            // the lanes-over-features tile needs no replicas: give it the whole
            // LDS, as the autotuner does (unless the knobs are forced)
            if (kb.kernel == 1 && !ctx->force_knobs) kb.lds_budget = ctx->max_lds - kFusedStaticLds;
            return kb;
        };
        // One histogram kernel serves the whole level: lanes over features
        // when every problem has one class and its knobs ask for that kernel,
        // with the narrowest group width any problem needs; else rows over
        // lanes.
        lp.kind = 1;
        lp.W = 32;
        for (int p = 0; p < P; ++p) {
            const HistKnobs kb = batch_knobs(probs[p]);
            if (probs[p].K != 1 || kb.kernel != 1) {
                lp.kind = 0;
                break;
            }
            const HistPlan hp = plan_hist(kb, probs[p].n, probs[p].n_features, probs[p].max_bins,
                                          1, L, precision, count_stat(&probs[p]),
                                          ctx->max_lds);
            lp.W = std::min(lp.W, hp.fb);
        }
        // a level >= 1 built by subtraction accumulates L/2 parent slots
        lp.sub = b->sub && lvl > 0 && lp.kind == 1;
        const int slots = lp.sub ? L / 2 : L;
        lp.mode = lp.sub ? 2 : (L == 1 ? 0 : 1);
        std::vector<int64_t> rb_off{0};
        for (int p = 0; p < P; ++p) {
            const cbh_problem& pr = probs[p];
            HistKnobs kb = batch_knobs(pr);
            kb.kernel = lp.kind;
            kb.lpf_w = lp.W;
            HistPlan hp = plan_hist(kb, pr.n, pr.n_features, pr.max_bins, pr.K, slots, precision,
                                    count_stat(&pr), ctx->max_lds);
            rb_off.push_back(rb_off.back() + (pr.n + kSideRows - 1) / kSideRows);
            if (lp.kind == 1 && hp.fb != lp.W) {
                set_error("batched group width %d differs from %d", hp.fb, lp.W);
                free_levels(b);
                delete b;
                return CBH_EUNSUPPORTED;
            }
            if (lp.kind == 1 && hp.n_ltiles > 1 && L > 1) lp.mode = 2;
            lp.plans.push_back(hp);
            lp.part_off.push_back(off);
            off += align_up(int64_t(hp.n_chunks) * slots * pr.n_features * pr.max_bins *
                                hp.words_per_cell * 4,
                            256);
            lp.max_lds = std::max(lp.max_lds, hp.lds_bytes);
            for (int ch = 0; ch < hp.n_chunks; ++ch) {
                const int64_t rows = std::min(hp.rows_per_chunk, pr.n - ch * hp.rows_per_chunk);
                groups.push_back(TileGroup{rows * pr.n_features * hp.n_ltiles, p, ch,
                                           hp.n_fgroups, hp.n_ltiles});
            }
            dplans.push_back(LevelPlan::DevHP{hp.fb, hp.lt, hp.n_fgroups, hp.n_ltiles,
                                              hp.n_chunks, hp.words_per_cell, hp.rep, 0,
                                              hp.rows_per_chunk, hp.lds_bytes});
            cell_off.push_back(cell_off.back() + int64_t(slots) * pr.n_features * pr.max_bins);
            feat_off.push_back(feat_off.back() + pr.n_features);
            row_off.push_back(row_off.back() + (pr.n + 7) / 8);
        }
        lp.part_bytes = off;
        max_part = std::max(max_part, off);
        deal_tiles(groups, tiles);
        lp.n_tiles = (int64_t)tiles.size();
        // fused launch: problems ordered by where their last tile sits in
        // the XCD shares (the earliest finished first), item prefixes in that order
        std::vector<int32_t> order(P), hcount(P, 0);
        std::vector<int64_t> last(P, -1), goff{0}, soff{0}, xoff{0};
        const int64_t per_x = lp.n_tiles / 8;
        for (int64_t ti = 0; ti < lp.n_tiles; ++ti) {
            const DevTile& t = tiles[ti];
            if (t.prob < 0) continue;
            ++hcount[t.prob];
            last[t.prob] = std::max(last[t.prob], per_x ? ti % per_x : ti);
        }
        for (int p = 0; p < P; ++p) order[p] = p;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return last[x] < last[y]; });
        for (int k = 0; k < P; ++k) {
            const int p = order[k];
            const int64_t cells = cell_off[p + 1] - cell_off[p];
            goff.push_back(goff.back() + (cells + kFusedMergeCells - 1) / kFusedMergeCells);
            soff.push_back(soff.back() +
                           (probs[p].n_features + kFusedScoreFeatures - 1) / kFusedScoreFeatures);
            xoff.push_back(xoff.back() + (probs[p].n + kFusedApplyRows - 1) / kFusedApplyRows);
        }
        lp.cells_total = cell_off.back();
        lp.score_total = feat_off.back();
        lp.rows_total = row_off.back();
        lp.rb_total = lp.sub ? rb_off.back() : 0;
        int rc = upload(&lp.d_tiles, tiles);
        if (!rc) rc = upload(&lp.d_plans, dplans);
        if (!rc) rc = upload(&lp.d_cell_off, cell_off);
        if (!rc) rc = upload(&lp.d_feat_off, feat_off);
        if (!rc) rc = upload(&lp.d_row_off, row_off);
        if (!rc && lp.sub) rc = upload(&lp.d_rb_off, rb_off);
        if (!rc && lp.kind == 1) rc = upload(&lp.d_order, order);
        if (!rc && lp.kind == 1) rc = upload(&lp.d_hcount, hcount);
        if (!rc && lp.kind == 1) rc = upload(&lp.d_goff, goff);
        if (!rc && lp.kind == 1) rc = upload(&lp.d_soff, soff);
        if (!rc && lp.kind == 1) rc = upload(&lp.d_xoff, xoff);
        b->levels.push_back(lp);
        if (rc) {
            free_levels(b);
            delete b;
            return rc;
        }
    }
    b->fbest_off = align_up(max_part, 256);
    b->ws_need = b->fbest_off + align_up(tot_feat * (int64_t)sizeof(FeatBest), 256);
    // counters of the fused launches, one set per level
    const int64_t cnt_bytes = align_up(int64_t(kFusedCounters + 5 * P) * 4, 256);
    const int64_t cnt_base = b->ws_need;
    for (int lvl = 0; lvl < b->depth; ++lvl) b->levels[lvl].cnt_off = cnt_base + lvl * cnt_bytes;
    b->ws_need += b->depth * cnt_bytes;
    // subtraction: level l writes hist[p] if depth-1-l is even, else the
    // second buffer, which therefore holds at most level depth-2
    std::vector<int64_t> hist2_off(P, 0), side_off(P, 0), code_off(P, 0);
    if (b->sub) {
        const int64_t esz = precision == CBH_PREC_FP32 ? 4 : 8;
        for (int p = 0; p < P; ++p) {
            hist2_off[p] = b->ws_need;
            b->ws_need += align_up((int64_t(1) << (b->depth - 2)) * probs[p].n_features *
                                       probs[p].max_bins * 2 * esz,
                                   256);
        }
        for (int p = 0; p < P; ++p) {
            side_off[p] = b->ws_need;
            b->ws_need += align_up(int64_t(1) << (b->depth - 2), 256);
        }
        for (int p = 0; p < P; ++p) {
            code_off[p] = b->ws_need;
            b->ws_need += align_up(probs[p].n * 2, 256);
        }
    }
    // the context workspace must exist before a capture (gradient codes use it)
    int rc = ensure_ws(ctx, 256, nullptr);
    if (!rc && b->ws_need > ctx->ws_limit) {
        set_error("batch workspace of %lld bytes exceeds the limit", (long long)b->ws_need);
        rc = CBH_ENOMEM;
    }
    if (!rc && hipMalloc(&b->ws, (size_t)b->ws_need) != hipSuccess) {
        (void)hipGetLastError();
        set_error("batch workspace allocation of %lld bytes failed", (long long)b->ws_need);
        rc = CBH_ENOMEM;
    }
    // the fused launches' counters start at zero (each launch leaves them so)
    if (!rc && hipMemset((char*)b->ws + cnt_base, 0, (size_t)(b->depth * cnt_bytes)) !=
                   hipSuccess) {
        (void)hipGetLastError();
        set_error("clearing the batch counters failed");
        rc = CBH_EDEVICE;
    }
    if (rc) {
        free_levels(b);
        delete b;
        return rc;
    }
    // device descriptors, one copy per level: the partial-tile offsets of the
    // problems differ between levels.
    std::vector<DevProb> dp(P);
    for (int p = 0; p < P; ++p) {
        const cbh_problem& pr = probs[p];
        dp[p] = DevProb{pr.bins, pr.n_bins, pr.g, pr.h, reinterpret_cast<const uint32_t*>(pr.gq),
                        pr.grad_scale, pr.leaf, hist[p], nullptr, pr.n, pr.n_features,
                        pr.max_bins, pr.K, count_stat(&pr), pr.seg_stride,
                        nullptr, nullptr, nullptr, pr.leaf};
    }
    std::vector<DevProb> all;
    all.reserve(size_t(P) * b->depth);
    char* wsb = (char*)b->ws;
    for (int lvl = 0; lvl < b->depth; ++lvl)
        for (int p = 0; p < P; ++p) {
            DevProb d = dp[p];
            d.partials = (uint32_t*)(wsb + b->levels[lvl].part_off[p]);
            if (b->sub) {
                // ping-pong: the last level lands in hist[p]
                auto out_of = [&](int l) -> void* {
                    return ((b->depth - 1 - l) % 2 == 0) ? hist[p] : (void*)(wsb + hist2_off[p]);
                };
                d.hist = out_of(lvl);
                if (b->levels[lvl].sub) {
                    d.parent = out_of(lvl - 1);
                    d.side = (uint8_t*)(wsb + side_off[p]);
                    d.codes = (uint16_t*)(wsb + code_off[p]);
                    d.rowcode = d.codes;
                }
            }
            all.push_back(d);
        }
    rc = upload(&b->d_probs, all);
    // the second phase: static arguments of every problem
    if (!rc) {
        std::vector<SolveArgs> sv(P);
        std::vector<UpdArgs> uv(P);
        std::vector<int64_t> soff{0}, uoff{0};
        for (int p = 0; p < P; ++p) {
            const cbh_problem& pr = probs[p];
            const int64_t leaves = int64_t(1) << pr.depth;
            sv[p] = SolveArgs{hist[p], best + int64_t(p) * b->depth + (b->depth - 1),
                              pr.grad_scale, nullptr, pr.depth, pr.n_features, pr.max_bins,
                              pr.K, (int32_t)count_stat(&pr), out_prec(precision), 0.0};
            uv[p] = UpdArgs{pr.leaf, nullptr, pr.label, pr.weight, pr.approx, pr.g, pr.h, pr.n,
                            pr.K, pr.loss, 1, (uint16_t)(leaves - 1), 0.0};
            soff.push_back(soff.back() + (leaves * pr.K + 3) / 4);
            uoff.push_back(uoff.back() + (pr.n + kUpdRows - 1) / kUpdRows);
        }
        b->solve_blocks = soff.back();
        b->upd_blocks = uoff.back();
        rc = upload(&b->d_solve, sv);
        if (!rc) rc = upload(&b->d_upd, uv);
        if (!rc) rc = upload(&b->d_solve_off, soff);
        if (!rc) rc = upload(&b->d_upd_off, uoff);
    }
    if (rc) {
        free_levels(b);
        for (void* q : {(void*)b->d_probs, (void*)b->d_solve, (void*)b->d_upd,
                        (void*)b->d_solve_off, (void*)b->d_upd_off})
            if (q) (void)hipFree(q);
        (void)hipFree(b->ws);
        delete b;
        return rc;
    }
    *out = b;
    return CBH_OK;
}

void cbh_batch_destroy(cbh_batch* b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    free_levels(b);
    for (void* q : {(void*)b->d_probs, (void*)b->d_solve, (void*)b->d_upd,
                    (void*)b->d_solve_off, (void*)b->d_upd_off})
        if (q) (void)hipFree(q);
    if (b->ws) (void)hipFree(b->ws);
    delete b;
}

int cbh_batch_level(cbh_ctx* ctx, cbh_batch* b, int32_t level, double l2, void* stream) {
    clear_error();
    CBH_ARG(ctx && b && b->ctx == ctx, "bad ctx / batch");
    CBH_ARG(level >= 0 && level < b->depth, "level outside [0, depth)");
    CBH_ARG(l2 >= 0 && std::isfinite(l2), "l2 must be finite and >= 0");
    const DevProb* saved = b->d_probs;
    b->d_probs = const_cast<DevProb*>(saved) + int64_t(level) * b->P;
    const int rc = batch_level_launch(b, level, l2, (hipStream_t)stream);
    b->d_probs = const_cast<DevProb*>(saved);
    return rc;
}

int cbh_batch_set_fused(cbh_batch* b, int32_t fused) {
    clear_error();
    CBH_ARG(b != nullptr, "batch is NULL");
    b->fused = fused != 0;
    return CBH_OK;
}

int cbh_batch_update(cbh_ctx* ctx, cbh_batch* b, double lr, double l2, double* const* leaf_values,
                     int32_t init, void* stream) {
    clear_error();
    CBH_ARG(ctx && b && b->ctx == ctx, "bad ctx / batch");
    CBH_ARG(init || leaf_values != nullptr, "leaf_values is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (!init) {
        for (int p = 0; p < b->P; ++p)
            CBH_ARG(leaf_values[p] != nullptr, "leaf_values[%d] is NULL", p);
        // the leaf value pointers (a graph captured here replays with these),
        // then every problem's leaf values in one launch
        for (int p0 = 0; p0 < b->P; p0 += 32) {
            ValsChunk c;
            c.first = p0;
            c.count = std::min(32, b->P - p0);
            for (int j = 0; j < 32; ++j) c.v[j] = j < c.count ? leaf_values[p0 + j] : nullptr;
            bset_vals_kernel<<<1, 64, 0, s>>>(b->d_solve, b->d_upd, c);
        }
        bleaf_solve_kernel<<<(unsigned)b->solve_blocks, 256, 0, s>>>(b->d_solve, b->d_solve_off,
                                                                      b->P, l2);
        CBH_LAUNCHED();
    }
    const unsigned ub = (unsigned)b->upd_blocks;
    const int32_t add = init ? 0 : 1;
    switch (b->probs[0].loss) {
        case CBH_LOSS_RMSE:
            bupdate_kernel<CBH_LOSS_RMSE><<<ub, 256, 0, s>>>(b->d_upd, b->d_upd_off, b->P, lr, add);
            break;
        case CBH_LOSS_LOGLOSS:
            bupdate_kernel<CBH_LOSS_LOGLOSS><<<ub, 256, 0, s>>>(b->d_upd, b->d_upd_off, b->P, lr,
                                                                add);
            break;
        default:
            bupdate_kernel<CBH_LOSS_MULTICLASS><<<ub, 256, 0, s>>>(b->d_upd, b->d_upd_off, b->P,
                                                                   lr, add);
            break;
    }
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_graph_capture_iteration(cbh_ctx* ctx, cbh_batch* b, double lr, double l2,
                                double* const* leaf_values, void* stream, cbh_graph** out) {
    clear_error();
    CBH_ARG(ctx && b && b->ctx == ctx && leaf_values && out, "NULL argument");
    CBH_ARG(stream != nullptr, "capture needs a non-default stream");
    *out = nullptr;
    for (int p = 0; p < b->P; ++p) CBH_ARG(leaf_values[p] != nullptr, "leaf_values[%d] NULL", p);
    hipStream_t s = (hipStream_t)stream;
    cbh_graph* g = new cbh_graph();
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        delete g;
        set_error("hipStreamBeginCapture failed: %s", hipGetErrorString(e));
        return CBH_EDEVICE;
    }
    int rc = CBH_OK;
    for (int p = 0; p < b->P && !rc; ++p)
        if (b->precision == CBH_PREC_INT16)
            rc = cbh_quantize_gradients(ctx, &b->probs[p], stream);
    for (int lvl = 0; lvl < b->depth && !rc; ++lvl) rc = cbh_batch_level(ctx, b, lvl, l2, stream);
    if (!rc) rc = cbh_batch_update(ctx, b, lr, l2, leaf_values, 0, stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (rc || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        delete g;
        if (!rc) set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
        return rc ? rc : CBH_EDEVICE;
    }
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete g;
        set_error("hipGraphInstantiate failed: %s", hipGetErrorString(e));
        return CBH_EDEVICE;
    }
    g->graph = graph;
    *out = g;
    return CBH_OK;
}

int cbh_graph_launch(cbh_graph* g, void* stream) {
    clear_error();
    CBH_ARG(g && g->exec, "graph is NULL");
    CBH_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return CBH_OK;
}

void cbh_graph_destroy(cbh_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
