// Internal declarations shared by the translation units of libcbhip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "cbhip.h"

namespace cbh {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

#define CBH_REQUIRE(cond, code, ...)            \
    do {                                        \
        if (!(cond)) {                          \
            ::cbh::set_error(__VA_ARGS__);      \
            return (code);                      \
        }                                       \
    } while (0)

#define CBH_ARG(cond, ...) CBH_REQUIRE(cond, CBH_EINVAL, __VA_ARGS__)

#define CBH_HIP(expr)                                                          \
    do {                                                                       \
        hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess) {                                                \
            ::cbh::set_error("%s failed: %s", #expr, hipGetErrorString(e_));   \
            return CBH_EDEVICE;                                                \
        }                                                                      \
    } while (0)

// Launch-error check after a kernel launch.
#define CBH_LAUNCHED()                                                         \
    do {                                                                       \
        hipError_t e_ = hipGetLastError();                                     \
        if (e_ != hipSuccess) {                                                \
            ::cbh::set_error("kernel launch failed: %s", hipGetErrorString(e_)); \
            return CBH_EDEVICE;                                                \
        }                                                                      \
    } while (0)

// Device-side error bits (ctx->d_flags[0]).
enum : uint32_t {
    FLAG_NAN_INPUT = 1u,
    FLAG_BAD_INDEX = 2u,
    FLAG_BAD_SPLIT = 4u,
    FLAG_FUSED_WAIT = 8u,
    FLAG_PACK_RANGE = 16u,
};

// ------------------------------------------------------- launch geometry
struct HistPlan {
    int32_t kind = 0;        // 0: rows over lanes with LDS replicas; 1: features over lanes
    int32_t fb = 1;          // features per block (kind 1: the lane group width W)
    int32_t lt = 1;          // leaves per LDS tile
    int32_t n_fgroups = 1;
    int32_t n_ltiles = 1;
    int32_t n_chunks = 1;
    int64_t rows_per_chunk = 0;  // multiple of 16
    int32_t words_per_cell = 2;  // 32-bit output words per (leaf, feature, bin)
    int32_t rep = 1;             // LDS replicas per (leaf, feature) cell
    int64_t lds_bytes = 0;
    int64_t n_blocks = 0;    // n_chunks * n_fgroups * n_ltiles
};

// Threads per histogram block (16 waves): one block per CU holds a large LDS
// tile while keeping enough waves resident to hide memory latency.
constexpr int kHistThreads = 1024;

// Tunable knobs of the histogram planner.
struct HistKnobs {
    int32_t lds_budget = 96 * 1024;  // bytes of LDS per block
    int32_t max_fb = 32;             // features per block at most
    int32_t target_blocks = 512;     // blocks aimed at per launch
    int64_t min_rows = 32768;        // rows per block at least (2 steps of 16 rows/thread)
    int32_t partial_pct = 25;        // partial tiles at most this % of the bin bytes
    int32_t max_rep = 32;            // LDS replicas per cell at most
    int32_t rep_target = 32;         // replicas the planner reserves LDS for first
    int32_t kernel = 1;              // 1: features over lanes where it applies (K == 1), 0: never
    int32_t lpf_w = 0;               // features per lane group for kernel 1, 0: widest that fits
};

// (F, B, K, level, precision, floor(log2 n), subtraction mode)
using TuneKey = std::tuple<int32_t, int32_t, int32_t, int32_t, int32_t, int32_t, int32_t>;

}  // namespace cbh

struct cbh_ctx {
    int device = 0;
    int num_cus = 256;
    int max_lds = 64 * 1024;
    void* ws = nullptr;
    int64_t ws_size = 0;
    // earlier, smaller workspaces: a graph captured over calls that used one
    // still points into it, so growth keeps them until cbh_destroy
    std::vector<void*> ws_retired;
    int64_t ws_limit = int64_t(64) << 30;
    uint32_t* d_flags = nullptr;  // [0] device error flags, [1] score blocks done (self-resetting)
    void* score_static = nullptr; // device address of the static score scratch on this device
    cbh::HistKnobs knobs;
    std::map<cbh::TuneKey, cbh::HistKnobs> tuned;
    std::map<cbh::TuneKey, std::string> tuned_note;   // chosen plan and its time, for the cache file
    bool force_knobs = false;
    cbh::HistKnobs forced;
};

// An instantiated HIP graph owned by the library (cbh_graph_capture_*).
struct cbh_graph {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

namespace cbh {

// Grow the workspace to at least `bytes` for a call on `stream`; returns
// CBH_OK / CBH_ENOMEM / CBH_EDEVICE, or CBH_EBUSY when growth would be needed
// while `stream` is being captured into a graph.
int ensure_ws(cbh_ctx* ctx, int64_t bytes, void* stream);

inline int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Ordered boosting (ordered.hip): argument checks, and the update of the kept
// model and the supporting approximations after a tree.
int validate_ordered(const cbh_ctx* ctx, const cbh_ordered* ord, const cbh_problem* p);
int ordered_update(cbh_ctx* ctx, const cbh_ordered* ord, const cbh_problem* p, double lr,
                   double l2, double* leaf_values, double* support_values, hipStream_t s);

// The histograms' second statistic is a row count (RMSE without row
// weights); otherwise it is the sum of h.
inline bool count_stat(const cbh_problem* p) {
    return p->loss == CBH_LOSS_RMSE && p->weight == nullptr;
}

// Bins packed below a byte per row (bin_bits 4 or 1).
inline bool packed_bins(const cbh_problem* p) { return p->bin_bits == 4 || p->bin_bits == 1; }

// Histogram planning (histogram.hip).
int words_per_cell(int32_t precision, int32_t K);
HistKnobs knobs_for(const cbh_ctx* ctx, int32_t F, int32_t B, int32_t K, int32_t level,
                    int32_t precision, int64_t n, int32_t sub);
int launch_side(const void* parent_hist, const cbh_split* parent_split, int64_t half, int32_t F,
                int32_t B, int32_t K, int32_t rmse, int32_t precision, uint8_t* side,
                hipStream_t s);
int launch_apply(const cbh_ctx* ctx, const cbh_problem* p, int32_t level, const cbh_split* best,
                 hipStream_t s);
HistPlan plan_hist(const HistKnobs& kn, int64_t n, int32_t F, int32_t B, int32_t K,
                   int32_t n_leaves, int32_t precision, int32_t rmse, int max_lds);
int64_t hist_elems(int32_t n_leaves, int32_t F, int32_t B, int32_t K);
int64_t hist_elem_bytes(int32_t precision);

int validate_problem(const cbh_problem* p);
int validate_precision(const cbh_problem* p, int32_t precision);

// Launchers used by several entry points (same stream semantics as the API).
// parent / side: subtraction mode (level >= 1), else NULL.
// codes: n uint16 of scratch, needed (hist_code_bytes) by the lanes-over-features
// kernel in subtraction mode.
// Subtraction mode (parent != NULL): the call derives the smaller child of
// every parent from `parent` and `parent_split` into `side` (2^(level-1)
// bytes) before the build; apply_parent: the leaf array does not hold the
// parent level's bit yet and the call sets it first (fused into the row-code
// pass where that pass runs).
int launch_hist(cbh_ctx* ctx, const cbh_problem* p, int32_t level, int32_t precision,
                const HistPlan& plan, void* hist_out, void* partials, hipStream_t s,
                const void* parent = nullptr, uint8_t* side = nullptr,
                uint16_t* codes = nullptr, const cbh_split* parent_split = nullptr,
                bool apply_parent = false);
int64_t hist_code_bytes(const HistPlan& plan, int64_t n, bool sub);
// counter: the self-resetting last-block counter (NULL: the context's)
int launch_score(cbh_ctx* ctx, const cbh_problem* p, int32_t level, const void* hist,
                 int32_t precision, double l2, cbh_split* best, float* scores,
                 void* scratch, hipStream_t s, uint32_t* counter = nullptr);
// Device address of score.hip's static scratch on the context's device (at
// cbh_create, with that device current).
int score_static_init(cbh_ctx* ctx);
int64_t score_scratch_bytes(const cbh_problem* p);

// Allow the dynamic-LDS kernels the device's full LDS (called by cbh_create).
void hist_init_attrs(int max_lds);
void batch_init_attrs(int max_lds);
void part_init_attrs(int max_lds);

}  // namespace cbh
