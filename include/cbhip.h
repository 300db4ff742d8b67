/*
 * cbhip — split search for oblivious gradient-boosted trees and ordered
 * target statistics on AMD Instinct MI355X (gfx950).
 *
 * The operations follow "CatBoost: gradient boosting with categorical
 * features support" (arXiv:1810.11363):
 *   - numeric features are discretized into a fixed number of bins, at most
 *     255 per feature (Sec. 5, "Dense numerical features");
 *   - categorical features are replaced by ordered target statistics over a
 *     permutation, with prior P and prior weight a (Sec. 2, Eq. 1); grouping
 *     by category uses a radix sort and a segmented scan (Sec. 5,
 *     "Categorical features");
 *   - trees are oblivious: one split per level, and the split at depth i sets
 *     bit i of the leaf index (Sec. 4);
 *   - splits are found from per-bin gradient histograms (Sec. 5), scored and
 *     the best one kept (Sec. 3, first phase of tree building); leaf values are
 *     then set by the ordinary boosting step and the tree is added to the
 *     model (Sec. 3, second phase; Algorithm 1 adds each tree to the model).
 * Where the paper is silent (score formula, regulariser, losses, border rule)
 * the readings are stated at the call that uses them.
 *
 * Conventions for every call:
 *   - Return value: CBH_OK or a negative status. cbh_last_error() returns a
 *     thread-local message for the last failing call on this thread.
 *   - Arguments are validated on the host before anything is enqueued; a
 *     call that fails validation enqueues nothing.
 *   - Pointers documented as "device" are device memory owned by the caller;
 *     the library never frees them and never keeps them past the call (except
 *     inside a batch plan or captured graph, see below). "host" pointers are
 *     read during the call only.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream). All
 *     device work is asynchronous on that stream; nothing in the per-level
 *     calls synchronizes the host. Device-side input errors (NaN inputs) and
 *     asynchronous faults are reported by cbh_sync().
 *   - A context owns a scratch workspace that calls on it reuse; use one
 *     context per concurrently used stream. See cbh_reserve_workspace for
 *     how the workspace behaves under graph capture.
 *   - Arrays written [A][B] are row-major with the last index fastest.
 */
#ifndef CBHIP_H
#define CBHIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CBH_OK 0
#define CBH_EINVAL (-1)        /* null pointer, bad shape or out-of-range argument */
#define CBH_ENOMEM (-2)        /* workspace allocation failed or exceeds the limit */
#define CBH_EDEVICE (-3)       /* HIP runtime error or device-reported input error */
#define CBH_EOVERFLOW (-4)     /* an integer accumulator could overflow */
#define CBH_EUNSUPPORTED (-5)  /* K > 16, more than 256 bins, depth > 16, ... */
#define CBH_EBUSY (-6)         /* the workspace would have to grow while the call's
                                  stream is being captured into a graph */

/* ---- losses (the paper uses Logloss and mentions regression; the
 *      derivative formulas are the standard ones, see cbh_update_approx) ---- */
#define CBH_LOSS_RMSE 0
#define CBH_LOSS_LOGLOSS 1
#define CBH_LOSS_MULTICLASS 2

/* ---- histogram precision -----------------------------------------------
 * How the per-bin sums of cbh_build_histograms are accumulated (the paper's
 * histograms sum float statistics, Sec. 5; the variants are this library's):
 *   CBH_PREC_FP32      every addition is a float32 addition (LDS
 *                      compare-and-swap updates; chunk partials added in
 *                      float32); output float
 *   CBH_PREC_TWOFLOAT  compensated float32: every addition is a TwoSum whose
 *                      rounding error is carried in a second float (the
 *                      (hi, lo) pair is updated by one 64-bit
 *                      compare-and-swap); partials merged with TwoSum; output
 *                      float2 (hi, lo)
 *   CBH_PREC_INT16     int16 gradient codes, exact integer sums; output int64
 *   CBH_PREC_F64       float64 LDS accumulation (the fastest float path on
 *                      gfx950, whose LDS has a pipelined float64 adder but
 *                      not a float32 one), each sum split into (hi, lo) when
 *                      written; output float2 (hi, lo), the TWOFLOAT layout,
 *                      and every call taking a TWOFLOAT histogram takes it */
#define CBH_PREC_FP32 0
#define CBH_PREC_TWOFLOAT 1
#define CBH_PREC_INT16 2
#define CBH_PREC_F64 3

#define CBH_MAX_K 16
#define CBH_MAX_BINS 256
#define CBH_MAX_DEPTH 16

typedef struct cbh_ctx cbh_ctx;

/* One boosting problem as seen by the per-level calls. The struct itself is
 * host memory; the pointers inside are device memory owned by the caller.
 *
 *   n           rows (>= 1)
 *   n_features  F, histogram features (numeric bins and statistic bins)
 *   max_bins    B, the bin stride of histograms: 2 <= B <= 256 and
 *               n_bins[f] <= B for every f; a stored bin >= B is counted in
 *               bin B-1
 *   bins        device array of F device pointers; bins[f] points at the
 *               uint8 bins of feature f. Rows are grouped in segments of 16
 *               consecutive rows: the bin of row i is the byte at
 *               bins[f] + (i / 16) * seg_stride[f] + i % 16. With seg_stride
 *               NULL every stride is 16, i.e. bins[f] is a plain column of
 *               n bytes in row order. Bins should be 16-byte aligned for full
 *               bandwidth.
 *   n_bins      device int32 [F]: number of bins of feature f (borders + 1);
 *               candidate borders are k = 0 .. n_bins[f]-2
 *   K           approx width: 1 (RMSE, Logloss) or the class count
 *               (MultiClass, 2 <= K <= 16)
 *   loss        CBH_LOSS_*
 *   depth       tree depth d, 1 <= d <= 16
 *   bin_bits    0 or 8: a byte per bin (bins as described above); 4 or 1:
 *               packed bins (Sec. 5 stores features of at most 15 bins in 4
 *               bits and binary features in 1 bit). Packed: every feature of
 *               the problem has that width (n_bins[f] <= 2^bin_bits, so
 *               max_bins <= 16 or 2), bins[f] is a plain column of
 *               ceil(n/16) segments of 2 * bin_bits bytes (8-byte aligned
 *               for 4 bits, 2-byte for 1 bit; cbh_pack_bins writes it) and
 *               seg_stride must be NULL. 4 bits: 32-bit word k (k = 0, 1) of
 *               a segment holds rows 8k..8k+3 of the segment in the low
 *               nibbles of its bytes 0..3 and rows 8k+4..8k+7 in the high
 *               nibbles; 1 bit: bit r of the segment's little-endian 16-bit
 *               word is row r. The histogram, subtraction, score, split,
 *               update, whole-tree and ordered calls take packed problems;
 *               the leaf-ordered (cbh_part_*), batched (cbh_batch_*) and
 *               autotuning calls return CBH_EUNSUPPORTED for them.
 *   label       device float [n]: target (RMSE), 0/1 (Logloss) or class index
 *               (MultiClass)
 *   g, h        device float [K][n]: first and second derivatives of the
 *               loss at approx. h is not read for RMSE (h = 1, the second
 *               statistic becomes the row count) and may be NULL there.
 *   gq          device int16 [K][n][2]: (g code, h code) pairs for
 *               CBH_PREC_INT16, written by cbh_quantize_gradients; else NULL
 *   grad_scale  device float [K][2]: per-class (g scale, h scale) for
 *               CBH_PREC_INT16; else NULL
 *   leaf        device uint16 [n]: leaf index of every row; bit i is the
 *               split of depth i (Sec. 4). Its contents are ignored at
 *               level 0, and cbh_apply_split at level 0 overwrites it, so a
 *               new tree needs no reset.
 *   approx      device double [K][n]: current model value of every row
 *   seg_stride  device int64 [F] or NULL: bytes between consecutive 16-row
 *               segments of feature f (a multiple of 16, at least 16; bins[f]
 *               16-byte aligned when it is not 16). A tiled matrix
 *               [ceil(n/16)][F][16] (see cbh_tile_bins) has bins[f] = base +
 *               16 f and seg_stride[f] = 16 F: then the 16-row segments of
 *               consecutive features are adjacent, which the histogram
 *               kernel that gives lanes of a wave different features reads
 *               with full coalescing. The values are not checked.
 *   weight      device float [n] or NULL: row weights w_i >= 0 (row i's loss
 *               counts w_i times). cbh_update_approx then writes w_i g_i and
 *               w_i h_i, and for RMSE h_i = w_i, so the second statistic of
 *               the histograms is the sum of weights instead of the row
 *               count (every call then treats RMSE like the h-carrying
 *               losses: h must be given). A cross-validation fold is the
 *               whole problem with weight 0 on its held-out rows: the folds
 *               read the same rows and bins (nothing is gathered or copied),
 *               and the held-out rows' approx are the fold model's
 *               predictions for them. Leaf counts still count every row.  */
typedef struct cbh_problem {
    int64_t n;
    int32_t n_features;
    int32_t max_bins;
    const uint8_t* const* bins;
    const int32_t* n_bins;
    int32_t K;
    int32_t loss;
    int32_t depth;
    int32_t bin_bits;
    const float* label;
    float* g;
    float* h;
    int16_t* gq;
    float* grad_scale;
    uint16_t* leaf;
    double* approx;
    const int64_t* seg_stride;
    const float* weight;
} cbh_problem;

/* Result of the split search of one level (device memory).
 * feature, border: the chosen split (rows with bin > border go right and get
 *                  the level's bit); -1, -1 if no feature has two bins.
 * score:           its score (see cbh_score_splits).
 * margin:          best score minus the best score of any other candidate
 *                  (0 for an exact tie).                                    */
typedef struct cbh_split {
    int32_t feature;
    int32_t border;
    float score;
    float margin;
} cbh_split;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device` (it becomes current on this thread). */
int cbh_create(int device, cbh_ctx** out);
/* Destroy a context and free its workspace. NULL is ignored. Waits for the
 * device to finish work that may still use the workspace. */
void cbh_destroy(cbh_ctx* ctx);
/* Thread-local message of the last failing call ("" if none). */
const char* cbh_last_error(void);
/* Cap on the workspace the context may allocate (bytes, > 0). A call that
 * would need more returns CBH_ENOMEM without enqueuing anything. */
int cbh_set_workspace_limit(cbh_ctx* ctx, int64_t bytes);
/* Current workspace size in bytes. */
int64_t cbh_workspace_size(const cbh_ctx* ctx);
/* Grow the workspace to at least `bytes` now (within the limit), so that
 * calls captured into a graph later find it large enough.
 * Workspace rules for graphs: a call that needs more workspace than the
 * context holds allocates a larger buffer; the earlier buffer is kept (not
 * freed) until cbh_destroy, so a graph captured over earlier calls stays
 * valid. A call whose stream is being captured never allocates: if it would
 * have to grow the workspace it returns CBH_EBUSY and enqueues nothing.
 * Errors: CBH_EINVAL (NULL, bytes < 0), CBH_ENOMEM. */
int cbh_reserve_workspace(cbh_ctx* ctx, int64_t bytes);
/* Wait for `stream`, then report asynchronous HIP errors and device-side input
 * errors (NaN feature values, bin or leaf values out of range) raised since
 * the previous cbh_sync, and clear them. */
int cbh_sync(cbh_ctx* ctx, void* stream);

/* Instrumentation (not part of the method): write the device's constant-rate
 * clock (cbh_device_clock_khz ticks per millisecond) to *slot when the stream
 * reaches this point. Two stamps around other calls on the same stream time
 * them, also inside a captured graph, where events cannot be recorded.
 *   slot  device uint64 [1]
 * Errors: CBH_EINVAL on NULL. */
int cbh_device_timestamp(cbh_ctx* ctx, uint64_t* slot, void* stream);
int cbh_device_clock_khz(cbh_ctx* ctx, int64_t* khz);

/* Instrumentation (not part of the method): issue rates of the LDS updates
 * the histogram forms use, in lane updates per clock per CU at the device's
 * peak shader clock, with the 64 lanes of every wave on distinct banks (16
 * waves per CU, four 1024-thread blocks per CU launched):
 *   rates_out[0] ds_add_u32   [1] ds_add_f32   [2] ds_add_f64   [3] ds_add_u64
 *   [4] float32 add by 32-bit compare-and-swap (the FP32 form's g cell)
 *   [5] (float, float) pair add by 64-bit compare-and-swap (FP32 (g, h) cell,
 *       TWOFLOAT (hi, lo) cell)
 *   rates_out  host double [6]
 * Runs on the default stream and synchronizes the device. */
int cbh_probe_lds_rates(cbh_ctx* ctx, double* rates_out);

/* ---- preprocessing -------------------------------------------------------- */

/* Borders of one numeric feature (host computation; Sec. 5: a fixed number of
 * bins, at most 255 borders). The paper gives no rule; this one takes
 * value-at-rank quantiles: with the column sorted ascending as s[0..n-1], if
 * it has m <= max_bins distinct values the borders are its m-1 smallest
 * distinct values; otherwise candidate j = 1..max_bins-1 is s[floor(j*n/max_bins)-1],
 * kept unless equal to the previous kept border or to s[n-1].
 *   x_host          host float [n], no NaN
 *   max_bins        2..256
 *   borders_out     host float [max_bins-1] (capacity), strictly increasing
 *   n_borders_out   host int32: number of borders written
 * Errors: CBH_EINVAL on NULL, n < 0, max_bins out of range or a NaN value. */
int cbh_select_borders(const float* x_host, int64_t n, int32_t max_bins,
                       float* borders_out, int32_t* n_borders_out);

/* Uniform borders for ordered-statistic values (host computation): the paper
 * binarizes statistics like numeric features (Sec. 4) without a rule; here
 * border j-1 = lo + ((hi - lo) * j) / n_bins for j = 1 .. n_bins-1, in
 * double precision with that operation order.
 *   borders_out  host double [n_bins-1]
 * Errors: CBH_EINVAL on NULL, non-finite or hi < lo; CBH_EUNSUPPORTED unless
 * 2 <= n_bins <= 256. */
int cbh_uniform_borders(double lo, double hi, int32_t n_bins, double* borders_out);

/* Bin index of every value of one numeric feature: bin = number of borders
 * strictly below x (so split k sends x > borders[k] right).
 *   x          device float [n]
 *   borders    device float [n_borders], strictly increasing
 *   n_borders  0..255
 *   bins_out   device uint8 [n]
 * A NaN value gets bin 0 and raises a device error reported by cbh_sync. */
int cbh_quantize(cbh_ctx* ctx, const float* x, int64_t n, const float* borders,
                 int32_t n_borders, uint8_t* bins_out, void* stream);

/* Copy bin columns into the row-tiled layout (a data layout step of this
 * library, not of the method): segment t of column c, the bins of rows
 * 16t .. 16t+15, lands at out + (t * n_cols + c) * 16, so the segments of
 * all columns for the same 16 rows are adjacent.
 *   cols    device array of n_cols device pointers to uint8 columns of n
 *           bytes (row order)
 *   n_cols  1 .. 65535
 *   out     device uint8 [ceil(n/16)][n_cols][16]; the bytes of the last
 *           segment past row n-1 are set to 0
 * Feature c then reads as bins[c] = out + 16 c, seg_stride[c] = 16 n_cols.
 * Errors: CBH_EINVAL on NULL or n < 1 or n_cols out of range. */
int cbh_tile_bins(cbh_ctx* ctx, const uint8_t* const* cols, int32_t n_cols, int64_t n,
                  uint8_t* out, void* stream);

/* Ordered target statistics of one categorical feature for one permutation,
 * Sec. 2, Eq. (1). For the row sigma_p at position p, over the rows placed at
 * positions < p that share its category value:
 *   num = sum of their target numerators,  den = their count,
 *   ts  = (num * 2^-y_shift + a * prior) / (den + a)   (double, this order),
 *   bin = number of ts_borders strictly below ts.
 * Several targets (e.g. one per class for MultiClass) share the grouping.
 *   cat          device int32 [n]: raw category values (any int32)
 *   perm         device int32 [n]: perm[p] = row placed at position p; must be
 *                a permutation of 0..n-1 (not checked)
 *   y_num        device int64 [n_targets][n]: target numerators, value
 *                y_num * 2^-y_shift (0/1 counts for classification)
 *   n_targets    1..16
 *   y_shift      0..62
 *   y_abs_max    host bound on |y_num|; CBH_EOVERFLOW if n * y_abs_max >= 2^62
 *   a            prior weight, > 0
 *   priors       host double [n_targets]
 *   ts_borders   device double [n_ts_borders] increasing; may be NULL if
 *                ts_bin_out is NULL
 *   n_ts_borders 0..255
 *   num_out      device int64 [n_targets][n] or NULL
 *   den_out      device int32 [n] or NULL
 *   ts_bin_out   device uint8 [n_targets][n] or NULL
 *   ts_out       device double [n_targets][n] or NULL
 * Uses workspace of about 24 * n bytes. */
int cbh_compute_ordered_ts(cbh_ctx* ctx, const int32_t* cat, const int32_t* perm,
                           int64_t n, const int64_t* y_num, int32_t n_targets,
                           int32_t y_shift, int64_t y_abs_max, double a,
                           const double* priors, const double* ts_borders,
                           int32_t n_ts_borders, int64_t* num_out, int32_t* den_out,
                           uint8_t* ts_bin_out, double* ts_out, void* stream);

/* Dense ids of category pairs: the perfect hash the paper uses for
 * combinations of categorical features (Sec. 2, "Feature combinations": the
 * values of a combination are numbered on the fly; Sec. 5, "Categorical
 * features": the perfect hashes are built with a radix sort). The
 * combination's ordered statistics are then those of one categorical
 * feature, see cbh_compute_ordered_ts. Rows with equal (cat_a, cat_b) get equal ids,
 * rows with different pairs different ids; the ids are 0 .. n_distinct - 1
 * in increasing order of the pair compared as unsigned 32-bit values
 * ((uint32)cat_a first, then (uint32)cat_b). Combinations of more features
 * chain the call: combine(combine(a, b), c).
 *   cat_a, cat_b    device int32 [n]: raw category values (any int32)
 *   n               0 .. 2^31 - 1 (0: nothing to do)
 *   ids_out         device int32 [n]
 *   n_distinct_out  device int64 [1]: number of distinct pairs
 * Uses workspace of about 40 * n bytes. Errors: CBH_EINVAL on NULL or n out
 * of range. */
int cbh_combine_categories(cbh_ctx* ctx, const int32_t* cat_a, const int32_t* cat_b, int64_t n,
                           int32_t* ids_out, int64_t* n_distinct_out, void* stream);

/* The counter statistic (Sec. 2, "Feature combinations": a category, or a
 * combination, replaced by the number of its appearances in the dataset):
 *   counts_out[i] = #{ j : ids[j] == ids[i] }.
 *   ids         device int32 [n], dense ids in [0, n) (for instance from
 *               cbh_combine_categories); an id outside [0, n) is counted
 *               nowhere, gets count 0, and is reported by cbh_sync
 *   n           0 .. 2^31 - 1 (0: nothing to do)
 *   counts_out  device int32 [n]
 * Uses workspace of 4 * n bytes. Errors: CBH_EINVAL on NULL or n out of
 * range. */
int cbh_category_counts(cbh_ctx* ctx, const int32_t* ids, int64_t n, int32_t* counts_out,
                        void* stream);

/* Where a tree's split gets its categorical value per row, for greedy
 * feature combinations (Sec. 2, "Feature combinations": after a split, the
 * categorical features and combinations present in the tree are combined
 * with every categorical feature of the dataset, and every split on a
 * numeric feature counts as a categorical feature of two values). One entry
 * per histogram feature of the problem the split was chosen on:
 *   kind CBH_SOURCE_BINS    ptr is the feature's uint8 bins in the layout of
 *                           cbh_problem.bins (byte bins; bin of row i at
 *                           ptr + (i / 16) * seg_stride + i % 16); the value
 *                           is 1 if bin > border, else 0 (a numeric split)
 *   kind CBH_SOURCE_VALUES  ptr is an int32 [n] column of category values (the
 *                           categorical feature behind a statistic column);
 *                           the value is ptr[i]
 *   kind CBH_SOURCE_PAIR    ptr and ptr_b are int32 [n] columns: the value is
 *                           the pair (ptr[i], ptr_b[i]) (a combination of a
 *                           grouping and a categorical feature)            */
#define CBH_SOURCE_BINS 0
#define CBH_SOURCE_VALUES 1
#define CBH_SOURCE_PAIR 2
typedef struct cbh_split_source {
    const void* ptr;
    const void* ptr_b;
    int64_t seg_stride;
    int32_t kind;
    int32_t reserved;
} cbh_split_source;

/* The categorical value of every row under a chosen split (Sec. 2, "Feature
 * combinations"), read on the device so that no host round trip is needed
 * between a level's argmax and the next level's combinations, as a pair of
 * columns (a, b): rows with equal pairs share the value.
 *   (a_out[i], b_out[i]) = per sources[split->feature] (see
 *                          cbh_split_source; b = 0 for the one-column
 *                          kinds); (0, 0) for every row when
 *                          split->feature < 0 (no split).
 *   split       device cbh_split (as written by cbh_score_splits)
 *   sources     device cbh_split_source [n_sources]
 *   a_out, b_out  device int32 [n]
 * cbh_combine_categories(a_out, b_out) then numbers the values densely. A
 * feature index >= n_sources, an unknown kind or a NULL column writes
 * zeros and is reported by cbh_sync. Errors: CBH_EINVAL on NULL or n out of
 * [0, 2^31 - 1]. */
int cbh_split_values(cbh_ctx* ctx, const cbh_split* split, const cbh_split_source* sources,
                     int32_t n_sources, int64_t n, int32_t* a_out, int32_t* b_out,
                     void* stream);

/* Rows of a categorical column grouped by category (Sec. 5, "Categorical
 * features": the rows are grouped with a radix sort), in permutation order
 * inside every category, and the dense id of every row's category:
 *   order_out   device int32 [n] or NULL: the rows in order of (category,
 *               position in perm); categories in increasing unsigned value
 *   ids_out     device int32 [n] or NULL: rank of the row's category among
 *               the distinct values (0 .. n_distinct - 1)
 *   n_distinct_out  device int64 [1] or NULL
 *   perm        device int32 [n], perm[p] = row at position p, or NULL for
 *               the identity
 * Uses workspace of about 40 * n bytes. */
int cbh_category_order(cbh_ctx* ctx, const int32_t* cat, const int32_t* perm, int64_t n,
                       int32_t* order_out, int32_t* ids_out, int64_t* n_distinct_out,
                       void* stream);

/* Ordered target statistics (Eq. 1) of several combinations at once: all
 * the crossings one level of a combination tree adds (Sec. 2, "Feature
 * combinations"; Sec. 5: grouping by radix sort and a segmented scan).
 * Crossing k groups the rows by the pair (e_ids[i], category of row i in
 * categorical feature k); its statistic for target t and prior q, in
 * permutation order, is written to ts_bin_out[k][(t * n_priors + q) * ld + i]
 * as the bin of ts = (num * 2^-y_shift + a * prior) / (den + a) (double,
 * this order) among ts_borders: bit for bit cbh_compute_ordered_ts on any
 * dense numbering of the pairs. All crossings share one sort over
 * n_cross * n elements keyed by (e, k) on e_bits + ceil(log2 n_cross) bits,
 * the rows of each crossing taken in its feature's category order (sort
 * passes over digits that are zero in every key copy instead of sorting).
 *   e_ids       device int32 [n], each in [0, 2^e_bits) (a value out of range
 *               is masked and reported by cbh_sync)
 *   c_order     device array of n_cross device int32 [n]: feature k's rows in
 *               order of (category, position), from cbh_category_order with
 *               the same permutation
 *   c_ids       device array of n_cross device int32 [n]: feature k's dense
 *               category ids (cbh_category_order's ids_out)
 *   y_num       device int64 [n_targets][n]
 *   priors      host double [n_targets][n_priors], n_priors <= 8
 *   ts_bin_out  device array of n_cross device uint8 [n_targets * n_priors][ld]
 *   counter_bins  0, or the bins of a counter column written after the
 *               statistics of every crossing, at column n_targets * n_priors
 *               (the counter statistic of Sec. 2, also calculated for
 *               combinations: the number of rows of the row's group, as
 *               cbh_counter_bins bins it); ts_bin_out then holds
 *               n_targets * n_priors + 1 columns per crossing
 * Errors: CBH_EINVAL on bad arguments, CBH_EUNSUPPORTED when e_bits plus the
 * crossing index bits exceed 32 or n_cross * n >= 2^31, CBH_EOVERFLOW as
 * cbh_compute_ordered_ts. Uses workspace of about (41 + columns per crossing)
 * * n_cross * n bytes. */
int cbh_ordered_ts_crossings(cbh_ctx* ctx, const int32_t* e_ids, int32_t e_bits,
                             int32_t n_cross, const int32_t* const* c_order,
                             const int32_t* const* c_ids, int64_t n, const int64_t* y_num,
                             int32_t n_targets, int32_t y_shift, int64_t y_abs_max, double a,
                             int32_t n_priors, const double* priors, const double* ts_borders,
                             int32_t n_ts_borders, int32_t counter_bins,
                             uint8_t* const* ts_bin_out, int64_t ld, void* stream);

/* Bins of the counter statistic (Sec. 2: a category, or a combination,
 * replaced by its number of appearances in the dataset; counts from
 * cbh_category_counts): bin = floor(log2(count)), at most n_bins - 1, and 0
 * for a count below 1. The paper gives no binarization for it; the log2
 * scale spreads Zipf-like counts over the bins.
 *   counts    device int32 [n];  bins_out  device uint8 [n] */
int cbh_counter_bins(cbh_ctx* ctx, const int32_t* counts, int64_t n, int32_t n_bins,
                     uint8_t* bins_out, void* stream);

/* Ordered target statistic of a grouping for one more prior (Sec. 2: several
 * priors, a feature for each), from the numerators and counts that
 * cbh_compute_ordered_ts wrote (num_out, den_out) for that grouping:
 *   ts = (num * 2^-y_shift + a * prior) / (den + a)   (double, this order),
 *   bin = number of ts_borders strictly below ts.
 * Bit for bit what cbh_compute_ordered_ts writes when called with `prior`.
 *   num         device int64 [n]  (one target's numerators)
 *   den         device int32 [n]
 *   ts_borders  device double [n_ts_borders] increasing (NULL if no bins)
 *   ts_bin_out  device uint8 [n] or NULL
 *   ts_out      device double [n] or NULL (not both NULL)
 * Errors: CBH_EINVAL on NULL arguments, a <= 0, y_shift outside [0, 62] or
 * more than 255 borders. */
int cbh_ts_bins(cbh_ctx* ctx, const int64_t* num, const int32_t* den, int64_t n,
                int32_t y_shift, double a, double prior, const double* ts_borders,
                int32_t n_ts_borders, uint8_t* ts_bin_out, double* ts_out, void* stream);

/* Packed bins from byte bins (Sec. 5 feature packing; layout at
 * cbh_problem.bin_bits): feature f's bins (the byte layout of
 * cbh_problem.bins with seg_stride, n rows) are written to packed[f], a
 * device buffer of ceil(n/16) * 2 * bits bytes, rows past n as 0.
 *   bins, packed  device arrays of n_features device pointers
 *   bits          4 or 1
 * A bin value >= 2^bits is stored masked and reported by cbh_sync. */
int cbh_pack_bins(cbh_ctx* ctx, const uint8_t* const* bins, const int64_t* seg_stride,
                  int32_t n_features, int64_t n, int32_t bits, uint8_t* const* packed,
                  void* stream);

/* ---- per-tree and per-level calls (the split search) -------------------- */

/* int16 gradient codes for CBH_PREC_INT16: per class, s_g = max|g| / 32767
 * and s_h = max h / 32767 (float32), code = round-half-even(value / scale)
 * (float32 division), 0 when the scale is 0. RMSE stores an h code of 1
 * (the count). Writes prob->gq and prob->grad_scale. */
int cbh_quantize_gradients(cbh_ctx* ctx, const cbh_problem* prob, void* stream);

/* Histograms of level `level` (0 <= level < depth), Sec. 5:
 *   hist[L][f][b][2c]   = sum of g_c over rows with leaf L and bin_f = b
 *   hist[L][f][b][2c+1] = sum of h_c over the same rows (row count for RMSE)
 * for L < 2^level, f < F, b < B, c < K. Element type by precision:
 *   CBH_PREC_FP32      float; for RMSE the odd slots hold uint32 counts
 *   CBH_PREC_TWOFLOAT,
 *   CBH_PREC_F64       float2 (hi, lo) with hi + lo the compensated (or
 *                      float64) sum; for RMSE the odd slots hold
 *                      (uint32 count, 0)
 *   CBH_PREC_INT16     int64 sums of the int16 codes (exact)
 *   hist_out   device, 2^level * F * B * 2K elements
 * Every block accumulates a tile in LDS; tiles are merged in a fixed order
 * without global atomics. Uses workspace for the per-block partial tiles. */
int cbh_build_histograms(cbh_ctx* ctx, const cbh_problem* prob, int32_t level,
                         int32_t precision, void* hist_out, void* stream);

/* Histograms of level `level` >= 1 by subtraction: for every parent leaf p of
 * the previous level, only the rows of its smaller child (judged from the
 * parent histogram at the parent's split: row counts for RMSE, sums of h
 * otherwise) are accumulated; the sibling is the parent's histogram minus that
 * child. The output equals cbh_build_histograms exactly for CBH_PREC_INT16 and
 * RMSE counts; for CBH_PREC_TWOFLOAT the difference is taken in two-float
 * arithmetic (error about 2^-44 of the parent's sums); for CBH_PREC_FP32 it is
 * a float difference, so a bin whose mass sits mostly in the smaller child can
 * carry the parent's float rounding error (use it when that is acceptable).
 * Histogram subtraction is not described in the paper.
 *   parent_hist   level-1 output of either build call, same precision; must
 *                 not be hist_out
 *   parent_split  the split chosen at level-1 (device cbh_split)
 *   hist_out      as cbh_build_histograms for `level` */
int cbh_build_histograms_sub(cbh_ctx* ctx, const cbh_problem* prob, int32_t level,
                             int32_t precision, const void* parent_hist,
                             const cbh_split* parent_split, void* hist_out, void* stream);

/* cbh_apply_split(level - 1, parent_split) followed by
 * cbh_build_histograms_sub(level), with the leaf update done in the same pass
 * over the rows as the row codes of the build where that pass runs (the
 * lanes-over-features kernel with 2^(level-1) * max_bins <= 16384), else as
 * a launch of its own before the build. prob->leaf must hold the bits of
 * levels < level - 1 (the state after cbh_apply_split(level - 2)); on return
 * it holds bit level - 1 too. Same arguments and results as
 * cbh_build_histograms_sub. */
int cbh_apply_build_histograms_sub(cbh_ctx* ctx, const cbh_problem* prob, int32_t level,
                                   int32_t precision, const void* parent_hist,
                                   const cbh_split* parent_split, void* hist_out, void* stream);

/* Score every candidate split of the level and keep the best (Sec. 3, first
 * phase). The paper gives no formula; the score is the gain of the
 * L2-regularised second-order objective: splitting every current leaf L by
 * (f, k), with left = bins <= k and right = bins > k,
 *   S(f, k) = sum_L sum_c  G_left^2 / (H_left + l2) + G_right^2 / (H_right + l2)
 * where H is the row count for RMSE; a side with H + l2 == 0 contributes 0.
 * The best split is the largest S; among equal scores the smallest feature,
 * then the smallest border. Prefix sums over bins are formed in the
 * histogram's own type (float, two-float pair or int64); every term and the
 * sum over leaves and classes are evaluated in double, and the per-border
 * score is stored as float32.
 *   hist        output of cbh_build_histograms for the same level/precision
 *   l2          >= 0
 *   best_out    device cbh_split [1]
 *   scores_out  device float [F][B-1] or NULL; -inf where k >= n_bins[f]-1 */
int cbh_score_splits(cbh_ctx* ctx, const cbh_problem* prob, int32_t level,
                     const void* hist, int32_t precision, double l2,
                     cbh_split* best_out, float* scores_out, void* stream);

/* cbh_score_splits for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and results, bit for bit, with the per-feature winners and
 * the last-block counter kept in a static device array of the library
 * (1 MB per GPU, held until the process ends) instead of the context's
 * workspace, which this call never touches or grows. The call allocates
 * nothing and issues no memset: the counter is cleared once by cbh_create and
 * reset by every launch's last block.
 *   n_features  at most 65536 (else CBH_EINVAL, nothing enqueued)
 * Every call on a GPU, from any context, shares that GPU's array: calls that
 * overlap on one GPU (concurrent streams) race and must not be issued.
 * Otherwise as cbh_score_splits. */
int cbh_score_splits_noalloc(cbh_ctx* ctx, const cbh_problem* prob, int32_t level,
                             const void* hist, int32_t precision, double l2,
                             cbh_split* best_out, float* scores_out, void* stream);

/* Apply the chosen split: leaf[i] |= (bins[f][i] > k) << level for the split
 * read from device memory (Sec. 4); at level 0, leaf[i] = (bins[f][i] > k).
 * If best->feature < 0 the bit stays clear for every row. */
int cbh_apply_split(cbh_ctx* ctx, const cbh_problem* prob, int32_t level,
                    const cbh_split* best, void* stream);

/* Finish a tree and refresh the gradients (Sec. 3, second phase).
 * With hist_last != NULL (the level depth-1 histograms) and `last` (the split
 * of level depth-1, already applied to prob->leaf):
 *   for every final leaf L' and class c, G and H are the sums of the parent's
 *   histogram row of the chosen feature on the side of the border that L'
 *   lies on, accumulated in double; the leaf value is the Newton step
 *   v = -G / (H + l2) (0 if H + l2 == 0); then
 *   approx[c][i] += lr * v[leaf[i]][c] in double.
 * Then, always, g and h are recomputed from approx in double and stored as
 * float (the paper uses d Loss / d a, Algorithm 1):
 *   RMSE        g = a - y, h = 1 (h not written)
 *   Logloss     p = 1 / (1 + exp(-a)), g = p - y, h = p (1 - p)
 *   MultiClass  p = softmax(a) (max subtracted), g_c = p_c - [y == c],
 *               h_c = p_c (1 - p_c)
 * With hist_last == NULL only the gradients are computed (tree 0 starts from
 * approx = 0, as Algorithm 1 starts from the zero model); `last`,
 * leaf_values_out and leaf_counts_out must then be NULL.
 *   leaf_values_out  device double [2^depth][K] (required with hist_last)
 *   leaf_counts_out  device int64 [2^depth] or NULL: rows per final leaf     */
int cbh_update_approx(cbh_ctx* ctx, const cbh_problem* prob, const void* hist_last,
                      int32_t precision, const cbh_split* last, double lr, double l2,
                      double* leaf_values_out, int64_t* leaf_counts_out, void* stream);

/* Model apply, the scorer of Sec. 4 ("Fast scorer"): for a model of n_trees
 * oblivious trees of depth d, tree t's leaf for row i is the binary vector
 *   leaf_t(i) = sum_{l < d} 2^l [bin_{f(t,l)}(i) > k(t,l)],
 * and for every class c
 *   approx[c][i] += lr * leaf_values[t][leaf_t(i)][c]
 * in double, tree after tree in model order: exactly the additions that the
 * model updates (cbh_update_approx) made while the trees were grown, so
 * applying a trained model to its training rows reproduces the training
 * approx bit for bit.
 *   bins, seg_stride  as in cbh_problem: device array of n_features device
 *                     pointers to uint8 bins (16-row segments `seg_stride`
 *                     bytes apart; seg_stride NULL = plain columns)
 *   n                 rows (0: nothing to do)
 *   K                 classes, 1..16 (1 for RMSE and Logloss)
 *   n_trees, depth    T >= 0 (0: nothing to do), 1 <= d <= 16
 *   split_feature     device int32 [T][d]: f(t, l), in [0, n_features)
 *   split_border      device int32 [T][d]: k(t, l); any int32 (-1 sets the
 *                     bit on every row, 255 on none)
 *   leaf_values       device double [T][2^d][K]
 *   lr                finite scale of every leaf value (the learning rate
 *                     the values were trained with; 1 for values already
 *                     scaled)
 *   approx            device double [K][n], read and written
 * A split feature outside [0, n_features) is taken as a bit of 0 on every
 * row and reported by cbh_sync (the call itself cannot see device arrays).
 * The rows of a launch are independent; approx must not overlap the other
 * arrays. Uses workspace for one chunk of trees' leaves (at most 256 MB,
 * at least one tree: n bytes, or 2n from depth 9). Errors: CBH_EINVAL (NULL
 * pointers, n or n_trees < 0, lr not finite), CBH_EUNSUPPORTED (K or depth
 * out of range, n >= 2^38), CBH_ENOMEM (workspace).                        */
int cbh_apply_model(cbh_ctx* ctx, const uint8_t* const* bins, const int64_t* seg_stride,
                    int64_t n, int32_t n_features, int32_t K, int32_t n_trees, int32_t depth,
                    const int32_t* split_feature, const int32_t* split_border,
                    const double* leaf_values, double lr, double* approx, void* stream);

/* The scorer of Sec. 4 in its two steps: every binary feature the model
 * uses is evaluated once for every row into a vector of bits, and each
 * tree's leaf index of a row is then read from those bits.
 *
 * cbh_binarize: binary feature j = (bin_feature[j], bin_border[j]); for
 * every row i,
 *   bit (i % 32) of bits_out[j][i / 32] = [bin of row i of feature
 *                                          bin_feature[j] > bin_border[j]],
 * bits of rows >= n in the last word 0.
 *   bins, seg_stride  the layout of cbh_problem.bins (byte bins; seg_stride
 *                     NULL: plain columns)
 *   bin_feature, bin_border  device int32 [n_binary]; binary features of one
 *                     feature given next to each other share the loads of
 *                     its bins
 *   bits_out          device uint32 [n_binary][ceil(n / 32)]
 * A feature index outside [0, n_features) gives a word of zeros and is
 * reported by cbh_sync.
 *
 * cbh_apply_model_binarized: as cbh_apply_model, with the split of tree t
 * at level l given as the binary feature split_binary[t][l] (device int32
 * [n_trees][depth], an index into the binarized features of `bits`):
 *   approx[c][i] += lr * leaf_values[t][sum_l 2^l bit(split_binary[t][l], i)][c]
 * for t = 0 .. n_trees - 1 in order, in double. With the binary features
 * of the model's (feature, border) pairs this is bit for bit
 * cbh_apply_model's result. An index outside [0, n_binary) reads bit 0 and
 * is reported by cbh_sync. Uses workspace as cbh_apply_model. Errors:
 * CBH_EINVAL on NULL or out-of-range sizes, CBH_EUNSUPPORTED for K or depth
 * out of range. */
int cbh_binarize(cbh_ctx* ctx, const uint8_t* const* bins, const int64_t* seg_stride, int64_t n,
                 int32_t n_features, int32_t n_binary, const int32_t* bin_feature,
                 const int32_t* bin_border, uint32_t* bits_out, void* stream);
int cbh_apply_model_binarized(cbh_ctx* ctx, const uint32_t* bits, int64_t n, int32_t n_binary,
                              int32_t K, int32_t n_trees, int32_t depth,
                              const int32_t* split_binary, const double* leaf_values, double lr,
                              double* approx, void* stream);

/* ---- one whole tree --------------------------------------------------------- */

typedef struct cbh_part cbh_part;

/* One tree of Algorithm 1 in one call: every level's histograms, score,
 * argmax and row routing (Sec. 3 first phase, Sec. 4), then the leaf solve
 * and the approx/gradient update (Sec. 3 second phase), enqueued on `stream`
 * exactly as the per-level calls would be:
 *   - CBH_PREC_INT16: cbh_quantize_gradients first;
 *   - level 0: cbh_build_histograms; level l >= 1: with a partition,
 *     cbh_part_build_histograms_sub (subtract != 0) or
 *     cbh_part_build_histograms; without one, cbh_apply_build_histograms_sub
 *     (subtract != 0, which also sets level l-1's leaf bit) or
 *     cbh_build_histograms;
 *   - then cbh_score_splits into best[l], and the rows are routed by that
 *     split: cbh_part_split with a partition, else cbh_apply_split (with
 *     subtraction only at the last level, the others being set by the next
 *     build);
 *   - finally cbh_update_approx with the last level's histograms.
 *   part         a partition for prob's shape (cbh_part_create), or NULL for
 *                the original row order
 *   hist         host array [2] of device buffers, each large enough for the
 *                level depth-1 histograms; level l writes hist[l % 2]
 *   best         device cbh_split [depth]
 *   leaf_values  device double [2^depth][K]; leaf_counts: device int64
 *                [2^depth] or NULL
 *   stamps       device uint64 [2 depth] or NULL: instrumentation, the
 *                device clock (cbh_device_timestamp) before and after every
 *                level's histogram build
 * Errors as the calls it makes; a failing call stops the sequence (calls
 * before it stay enqueued). */
int cbh_fit_tree(cbh_ctx* ctx, const cbh_problem* prob, cbh_part* part, int32_t precision,
                 int32_t subtract, void* const* hist, cbh_split* best, double lr, double l2,
                 double* leaf_values, int64_t* leaf_counts, uint64_t* stamps, void* stream);

/* The same tree captured into a HIP graph that the library owns (launch it
 * with cbh_graph_launch on any stream, free it with cbh_graph_destroy). Grow
 * one tree of the same shape first, so that the context workspace has its
 * size: a call under capture does not allocate (CBH_EBUSY). The graph keeps
 * the problem's device pointers, the partition and the buffers. `stream`
 * must not be the default stream. */
typedef struct cbh_graph cbh_graph;
int cbh_graph_capture_tree(cbh_ctx* ctx, const cbh_problem* prob, cbh_part* part,
                           int32_t precision, int32_t subtract, void* const* hist,
                           cbh_split* best, double lr, double l2, double* leaf_values,
                           int64_t* leaf_counts, uint64_t* stamps, void* stream,
                           cbh_graph** out);

/* Capture any sequence of library calls into one library-owned graph:
 * cbh_graph_begin starts capturing `stream` (this thread only); every call
 * then issued on `stream` is recorded, not run; cbh_graph_end stops and
 * instantiates the graph, which cbh_graph_launch replays and
 * cbh_graph_destroy frees. The recorded calls keep the pointers they were
 * given (and the context workspace as it was: a call that would have to
 * grow it under capture fails with CBH_EBUSY, see cbh_reserve_workspace),
 * so the caller keeps those buffers alive while the graph exists. A call
 * that fails under capture leaves the capture to be ended: cbh_graph_end
 * then returns CBH_EDEVICE and no graph. Used for the level loops a caller
 * drives itself, such as trees with feature combinations. */
int cbh_graph_begin(cbh_ctx* ctx, void* stream);
int cbh_graph_end(cbh_ctx* ctx, void* stream, cbh_graph** out);

/* ---- ordered boosting (Sec. 3) ---------------------------------------------- */

/* The supporting approximations of one permutation (Sec. 3, Algorithm 1 and
 * its O(s n) relaxation). Algorithm 1 keeps for every position a model that
 * never learns from it; the relaxation keeps about log2(n) models, all with
 * the tree structures of the trees grown, and takes a row's gradient for
 * choosing the next tree structure from the one that did not learn from it.
 * Reading of the relaxation, with 0-based positions p (perm[p] = row at
 * position p):
 *   model m = 0..M-1 learns from the positions below T_m (T_0 = 0,
 *   T_m = 2^(m-1)) and is kept for the positions below min(n, 2^m);
 *   the row at position p takes its gradient at model m(p) = bit length of p
 *   (0 for p = 0), which learned from positions below 2^floor(log2 p) <= p;
 *   M = cbh_ordered_models(n) = 1 for n = 1, floor(log2(n-1)) + 2 otherwise.
 * After each tree every model takes the Newton leaf values -G/(H+l2) of its
 * own gradients summed over its learning positions, per leaf of the tree,
 * and adds lr times them at every position it is kept for. The model that is
 * kept for prediction (prob->approx; the second phase of Sec. 3) takes its
 * leaf values from its own gradients over all rows.
 * Several permutations (s in Sec. 3) are several cbh_ordered, each with its
 * own support: a tree grown on one permutation's gradients (and its TS
 * columns) is added to the supporting models of every permutation.
 *   n        positions, equal to the problem's n
 *   perm     device int32 [n], a permutation of 0..n-1 (an entry outside
 *            [0, n) is skipped and reported by cbh_sync)
 *   support  device double [K][S], S = cbh_ordered_support_size(n) (< 4n):
 *            model m's values from cbh_ordered_offset(n, m) on, in position
 *            order; all zero before the first tree (approx 0, Algorithm 1) */
typedef struct cbh_ordered {
    int64_t n;
    const int32_t* perm;
    double* support;
} cbh_ordered;

/* M, model m's offset (m = 0..M; offset M = S) and S; 0 / -1 / 0 for n < 1 or
 * an m outside [0, M]. Host only, no context needed. */
int32_t cbh_ordered_models(int64_t n);
int64_t cbh_ordered_offset(int64_t n, int32_t m);
int64_t cbh_ordered_support_size(int64_t n);

/* prob->g and prob->h (h not for RMSE without weights) of every row, in row
 * order, at the model its position reads: the gradients that choose the
 * next tree structure. The first tree calls this on a zero support.
 * Errors: CBH_EINVAL for a NULL argument or ord->n != prob->n;
 * CBH_EUNSUPPORTED for row weights or 2^depth * K > 4096. */
int cbh_ordered_gradients(cbh_ctx* ctx, const cbh_ordered* ord, const cbh_problem* prob,
                          void* stream);

/* After a tree's structure is fixed (prob->leaf holds every row's final
 * leaf): with leaf_values, the kept model's leaf values from prob->approx's
 * own gradients over all rows, and prob->approx += lr * value of the row's
 * leaf; every supporting model of `ord` takes its own leaf values and
 * update; then prob->g / prob->h for the next tree as cbh_ordered_gradients
 * for `ord`. With s permutations a tree is one call with leaf_values and
 * s - 1 calls without (prob->approx untouched), the next tree's permutation
 * last, so that its gradients are the ones left in prob->g / prob->h.
 *   leaf_values     device double [2^depth][K]: the kept model's values, or
 *                   NULL to leave the kept model alone
 *   support_values  device double [M][2^depth][K] or NULL: every supporting
 *                   model's values
 * Sums are in double (LDS) in an order that may vary between runs; the
 * values are exact up to that rounding. Uses the context workspace (about
 * 6 bytes per row plus 16 bytes per leaf and class per 2048 learning
 * entries). Errors as cbh_ordered_gradients. */
int cbh_ordered_update(cbh_ctx* ctx, const cbh_ordered* ord, const cbh_problem* prob,
                       double lr, double l2, double* leaf_values, double* support_values,
                       void* stream);

/* One tree of ordered boosting in one call: the levels exactly as
 * cbh_fit_tree (prob->g / prob->h must hold the ordered gradients, from
 * cbh_ordered_gradients before the first tree and from the previous call
 * after that), then cbh_ordered_update (with leaf_values, required here) in
 * place of cbh_update_approx. */
int cbh_fit_tree_ordered(cbh_ctx* ctx, const cbh_problem* prob, const cbh_ordered* ord,
                         cbh_part* part, int32_t precision, int32_t subtract,
                         void* const* hist, cbh_split* best, double lr, double l2,
                         double* leaf_values, double* support_values, void* stream);

/* ---- rows in leaf order (deep trees, many classes) ------------------------- */

/* Device buffers that keep a problem's rows sorted by leaf during a tree, so
 * that a level's histograms (Sec. 5) read every row once whatever the number
 * of leaves (this library's layout, not the paper's). Holds two copies
 * of the bins (16-row tiled layout), of the gradient statistics the
 * histogram reads, of the original row ids and of the leaf indices, all
 * ceil(n / 16) * 16 rows long, plus per-leaf offsets. The partition is
 * sized for `prob` (n, features, K, depth, loss) and can serve any problem
 * of that shape (e.g. every permutation's bins). Owned by the caller of
 * cbh_part_create; cbh_part_destroy synchronizes the device first.
 * Returns CBH_ENOMEM if the buffers do not fit. */
int cbh_part_create(cbh_ctx* ctx, const cbh_problem* prob, cbh_part** out);
void cbh_part_destroy(cbh_part* part);

/* After the split of `level` (device cbh_split, e.g. from cbh_score_splits)
 * instead of cbh_apply_split: moves the rows by a stable partition on the
 * new leaf bit [bin of the split feature > border] (bit 0 first), which with
 * rows already in leaf order below that bit leaves them sorted by the full
 * leaf index. Level 0 reads the problem's bins, statistics (float g/h, or the
 * int16 codes for CBH_PREC_INT16) and the identity row order; level l reads
 * what level l-1 wrote. At level depth-1 nothing is moved: the leaf index of
 * every row is written to prob->leaf (original row order), as
 * cbh_apply_split over all levels would have left it. Levels must run in
 * order within a tree; the statistics must be those of the tree (for int16,
 * quantized before level 0). */
int cbh_part_split(cbh_ctx* ctx, cbh_part* part, const cbh_problem* prob, int32_t level,
                   int32_t precision, const cbh_split* split, void* stream);

/* Histograms of level >= 1 from the rows cbh_part_split(level - 1) left in
 * leaf order (a direct build; same output layout and values as
 * cbh_build_histograms up to summation order): every slot tile of leaves
 * reads only its rows. Uses the lanes-over-features kernel (any K) and the
 * context workspace for partial tiles. */
int cbh_part_build_histograms(cbh_ctx* ctx, cbh_part* part, const cbh_problem* prob,
                              int32_t level, int32_t precision, void* hist_out, void* stream);

/* The same level by subtraction (not described in the paper): with the rows
 * in leaf order every child is one contiguous range, so for every parent p
 * of the previous level only its child with fewer rows (leaf p or
 * p + 2^(level-1)) is accumulated, and the other child is written as the
 * parent's histogram minus it: exactly for CBH_PREC_INT16 sums and RMSE
 * counts, as a two-float difference for CBH_PREC_TWOFLOAT and CBH_PREC_F64
 * (error about 2^-44 of the parent's sums), as a float difference for
 * CBH_PREC_FP32 (the parent's float rounding can then dominate a small
 * sibling bin). Reads about half the rows of a direct build.
 *   parent_hist  the level-1 histograms (either build call, same
 *                precision); must not be hist_out
 * Otherwise as cbh_part_build_histograms. */
int cbh_part_build_histograms_sub(cbh_ctx* ctx, cbh_part* part, const cbh_problem* prob,
                                  int32_t level, int32_t precision, const void* parent_hist,
                                  void* hist_out, void* stream);

/* ---- batched, fused levels ------------------------------------------------- */

typedef struct cbh_batch cbh_batch;

/* A plan for running tree levels of P independent problems together (for
 * example several permutations, folds or separate datasets; the batching of
 * the s permutations of Sec. 3 and of the many histograms per launch of
 * Sec. 5). The problem descriptors and the histogram buffers are copied to
 * device memory once; the device buffers they point to must stay valid while
 * the plan exists.
 *   probs     host array [P]; every problem must have the same depth and loss
 *   subtract  != 0: levels >= 1 build only the smaller child of every parent
 *             and take the other as parent minus child (as
 *             cbh_build_histograms_sub); applies when every problem has
 *             K = 1, else ignored. The plan then keeps a second histogram
 *             buffer per problem, the sides and the row codes in its own
 *             workspace.
 *   hist      host array [P] of device pointers; hist[p] must hold the level
 *             depth-1 histograms of problem p (size as cbh_build_histograms);
 *             after a level of the plan it holds that level's histograms if
 *             depth-1-level is even (else the plan's second buffer does)
 *   best      device cbh_split [P][depth]: split of every problem and level
 * Precision: any CBH_PREC_* form. */
int cbh_batch_create(cbh_ctx* ctx, const cbh_problem* probs, int32_t P,
                     int32_t precision, int32_t subtract, void* const* hist,
                     cbh_split* best, cbh_batch** out);
void cbh_batch_destroy(cbh_batch* batch);

/* One level of every problem of the plan: histograms, score, argmax and the
 * leaf update, with the split written to best[p][level].
 * When cbh_batch_set_fused turned it on, every problem has one class and the
 * level uses the lanes-over-features histogram (the default plan), the whole
 * level is one launch of persistent blocks: the blocks claim
 * work items in order, first (with subtraction) the row codes, then the
 * histogram tiles of the work list dealt to the 8 XCDs (block b takes XCD
 * b mod 8's share), then per problem the merges, the per-feature scores, the
 * argmax and the leaf-bit updates; per-problem counters make each item wait
 * for the items it reads (no grid-wide barrier: every awaited item was
 * claimed earlier by a running block). A wait that does not end within a few
 * seconds gives up and raises a device error that cbh_sync reports. The
 * launch leaves its counters cleared, so it replays from a graph.
 * Otherwise the level runs as five launches shared by all problems (histogram tiles of every problem from
 * one work list, partial merge, score of every (problem, feature), argmax per
 * problem, leaf-bit update over every row), plus, for a level >= 1 built by
 * subtraction, a first launch over every row that picks each parent's smaller
 * child and writes the rows' slot codes; the launch count does not grow with
 * P. When every problem has K = 1 the histogram launch uses the kernel that
 * spreads the features of a group over the lanes of a wave, with one group
 * width for all problems of the level; otherwise (or when the histogram knobs
 * ask for it) the kernel that spreads rows over lanes. Levels must run in
 * order 0, 1, ..., depth-1 (a level reads the previous level's histograms and
 * splits). */
int cbh_batch_level(cbh_ctx* ctx, cbh_batch* batch, int32_t level, double l2,
                    void* stream);
/* Level launches of the plan: fused != 0 runs every level that allows it as
 * the one persistent launch described at cbh_batch_level, 0 (the default) as
 * the separate launches. Results are the same (bit for bit for int16). The
 * persistent launch keeps one 1024-thread block per CU through the merge,
 * score and update stages, which the separate launches run as many smaller
 * blocks, so it only pays where a level's launches are short enough for the
 * gaps between them to dominate. */
int cbh_batch_set_fused(cbh_batch* batch, int32_t fused);
/* A one-call form, level(ctx, probs, P, level, precision, l2, best_out,
 * stream), is cbh_batch_create once for the set of problems (it copies their
 * descriptors to the device and sizes the plan's workspace: the allocation a
 * per-level call could not make under graph capture) and then this call per
 * level; the split of problem p at the level is best[p][level]. */

/* Finish the trees of every problem of the plan (as cbh_update_approx with the
 * level depth-1 histograms and splits); leaf_values is a host array [P] of
 * device pointers, each double [2^depth][K] (entries may not be NULL). With
 * init != 0 only the gradients are computed (tree 0). All problems go in two
 * launches (leaf values, then approx and derivatives); the leaf value
 * pointers are set on the device by small launches that carry them by value,
 * so a captured iteration replays with the pointers it was captured with. */
int cbh_batch_update(cbh_ctx* ctx, cbh_batch* batch, double lr, double l2,
                     double* const* leaf_values, int32_t init, void* stream);

/* Capture one whole boosting iteration of the plan (reset leaves, every
 * level, the leaf solve and the approx/gradient update) into a HIP graph and
 * return an executable graph that replays it on `stream`. */
int cbh_graph_capture_iteration(cbh_ctx* ctx, cbh_batch* batch, double lr, double l2,
                                double* const* leaf_values, void* stream,
                                cbh_graph** out);
int cbh_graph_launch(cbh_graph* graph, void* stream);
void cbh_graph_destroy(cbh_graph* graph);

/* ---- autotuning -------------------------------------------------------------- */

/* Launch knobs of the histogram planner for every later call of this context
 * (overriding the autotune table); all must be > 0, or pass lds_budget = 0 to
 * return to the defaults and the table.
 *   lds_budget     LDS bytes per block
 *   target_blocks  blocks aimed at per launch
 *   min_rows       rows per block at least
 *   partial_pct    partial tiles at most this % of the level's bin bytes
 *   max_rep        LDS replicas per (leaf, feature) cell at most (power of two)
 *   rep_target     replicas the planner reserves LDS for before adding features
 *   kernel         1: for K = 1 use the kernel that spreads the features of a
 *                  group over the lanes of a wave (conflict-free LDS tile, no
 *                  replicas); 0: always the kernel that spreads rows over lanes
 *                  (replicated LDS tile)
 *   lpf_w          features per lane group of kernel 1: 4, 8, 16 or 32 (the
 *                  widest whose tile fits if the tile does not), 0: widest that
 *                  fits                                                         */
int cbh_set_hist_knobs(cbh_ctx* ctx, int32_t lds_budget, int32_t target_blocks,
                       int64_t min_rows, int32_t partial_pct, int32_t max_rep,
                       int32_t rep_target, int32_t kernel, int32_t lpf_w);

/* Tune the histogram launch plan of every level of `prob`: one tree is grown
 * level by level from the problem's current gradients (prob->leaf is
 * overwritten); at each level every distinct plan reachable from a grid of
 * knobs (LDS bytes per block, blocks per launch, rows per block, partial-tile
 * volume, LDS replicas per cell) is timed in the mode the tree will use —
 * subtract != 0: levels >= 1 by cbh_build_histograms_sub — and the fastest is
 * kept per (F, B, K, level, precision, floor(log2 n), mode). The table is
 * saved as JSON at cache_path (may be NULL); later calls of this context use
 * it. Synchronizes the stream. */
int cbh_autotune(cbh_ctx* ctx, const cbh_problem* prob, int32_t precision, int32_t subtract,
                 const char* cache_path, void* stream);
/* Load a table written by cbh_autotune. */
int cbh_autotune_load(cbh_ctx* ctx, const char* cache_path);

#ifdef __cplusplus
}
#endif

#endif /* CBHIP_H */
