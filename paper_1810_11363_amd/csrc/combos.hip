// Greedy feature combinations and several priors (Sec. 2, "Feature
// combinations" and the prior discussion under Eq. 1): the categorical value
// a tree's split gives every row, and the ordered-statistic bins of a
// grouping for one more prior from its numerators and counts. (The
// crossings of a level in one sort are in preprocess.hip, beside the sort.)
#include "common.h"

using namespace cbh;

namespace {

int grid_for(int64_t n, int per_block, int cap) {
    const int64_t b = (n + per_block - 1) / per_block;
    return int(b < 1 ? 1 : (b > cap ? cap : b));
}

// Every row's value under the split `*split` as a pair (a, b): the split's
// column is looked up in `src` (device memory) once per thread; a bins
// column gives ([bin > border], 0), a values column (value, 0), a pair
// source its two columns, no split (0, 0).
__global__ __launch_bounds__(256) void split_values_kernel(
    const cbh_split* __restrict__ split, const cbh_split_source* __restrict__ src,
    int32_t n_src, int64_t n, int32_t* __restrict__ a_out, int32_t* __restrict__ b_out,
    uint32_t* __restrict__ flags) {
    const int32_t f = split->feature;
    const int32_t k = split->border;
    int32_t kind = -1;
    const void* ptr = nullptr;
    const void* ptr_b = nullptr;
    int64_t stride = 16;
    if (f >= 0 && f < n_src) {
        kind = src[f].kind;
        ptr = src[f].ptr;
        ptr_b = src[f].ptr_b;
        stride = src[f].seg_stride;
    }
    const bool bad = f >= n_src ||
                     (f >= 0 && ((kind != CBH_SOURCE_BINS && kind != CBH_SOURCE_VALUES &&
                                  kind != CBH_SOURCE_PAIR) ||
                                 !ptr || (kind == CBH_SOURCE_PAIR && !ptr_b)));
    if (bad) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(flags, FLAG_BAD_SPLIT);
        kind = -1;
    }
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        int32_t v = 0, w = 0;
        if (kind == CBH_SOURCE_BINS) {
            const uint8_t* b = static_cast<const uint8_t*>(ptr);
            v = int32_t(b[(i >> 4) * stride + (i & 15)]) > k ? 1 : 0;
        } else if (kind == CBH_SOURCE_VALUES) {
            v = static_cast<const int32_t*>(ptr)[i];
        } else if (kind == CBH_SOURCE_PAIR) {
            v = static_cast<const int32_t*>(ptr)[i];
            w = static_cast<const int32_t*>(ptr_b)[i];
        }
        a_out[i] = v;
        b_out[i] = w;
    }
}

// Eq. (1) with another prior: ts = (num * 2^-e + a * P) / (den + a), the
// operations in this order (the expression cbh_compute_ordered_ts
// evaluates), and its bin = number of borders strictly below ts.
__global__ __launch_bounds__(256) void ts_bins_kernel(
    const int64_t* __restrict__ num, const int32_t* __restrict__ den, int64_t n,
    int32_t y_shift, double a, double ap, const double* __restrict__ tsb, int32_t ntsb,
    uint8_t* __restrict__ bin_out, double* __restrict__ ts_out) {
    __shared__ double sb[256];
    sb[threadIdx.x] = (int32_t(threadIdx.x) < ntsb) ? tsb[threadIdx.x] : INFINITY;
    __syncthreads();
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        const double t = (ldexp((double)num[i], -y_shift) + ap) / ((double)den[i] + a);
        if (ts_out) ts_out[i] = t;
        if (bin_out) {
            uint32_t pos = 0;
#pragma unroll
            for (uint32_t step = 128; step >= 1; step >>= 1)
                if (sb[pos + step - 1] < t) pos += step;
            bin_out[i] = (uint8_t)pos;
        }
    }
}

// Counter bins: floor(log2(count)) capped at n_bins - 1; 0 for count < 1.
__global__ __launch_bounds__(256) void counter_bins_kernel(const int32_t* __restrict__ counts,
                                                           int64_t n, int32_t n_bins,
                                                           uint8_t* __restrict__ out) {
    for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * 256) {
        const int32_t c = counts[i];
        const int b = c > 0 ? 31 - __clz((uint32_t)c) : 0;
        out[i] = (uint8_t)min(b, n_bins - 1);
    }
}

}  // namespace

extern "C" {

int cbh_counter_bins(cbh_ctx* ctx, const int32_t* counts, int64_t n, int32_t n_bins,
                     uint8_t* bins_out, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0, "n must be >= 0");
    CBH_ARG(n_bins >= 1 && n_bins <= 256, "n_bins must be in [1, 256]");
    if (n == 0) return CBH_OK;
    CBH_ARG(counts && bins_out, "NULL argument");
    counter_bins_kernel<<<grid_for(n, 256, ctx->num_cus * 8), 256, 0, (hipStream_t)stream>>>(
        counts, n, n_bins, bins_out);
    CBH_LAUNCHED();
    return CBH_OK;
}


int cbh_split_values(cbh_ctx* ctx, const cbh_split* split, const cbh_split_source* sources,
                     int32_t n_sources, int64_t n, int32_t* a_out, int32_t* b_out,
                     void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0 && n <= int64_t(INT32_MAX), "n must be in [0, 2^31 - 1]");
    CBH_ARG(n_sources >= 0, "n_sources must be >= 0");
    if (n == 0) return CBH_OK;
    CBH_ARG(split && a_out && b_out && (sources || n_sources == 0), "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    split_values_kernel<<<grid_for(n, 256, ctx->num_cus * 8), 256, 0, s>>>(
        split, sources, n_sources, n, a_out, b_out, ctx->d_flags);
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_ts_bins(cbh_ctx* ctx, const int64_t* num, const int32_t* den, int64_t n,
                int32_t y_shift, double a, double prior, const double* ts_borders,
                int32_t n_ts_borders, uint8_t* ts_bin_out, double* ts_out, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(n >= 0, "n must be >= 0");
    CBH_ARG(y_shift >= 0 && y_shift <= 62, "y_shift must be in [0, 62]");
    CBH_ARG(a > 0.0, "a must be > 0");
    CBH_ARG(n_ts_borders >= 0 && n_ts_borders <= 255, "n_ts_borders must be in [0, 255]");
    if (n == 0) return CBH_OK;
    CBH_ARG(num && den, "NULL argument");
    CBH_ARG(ts_bin_out || ts_out, "nothing to write");
    CBH_ARG(!ts_bin_out || n_ts_borders == 0 || ts_borders, "ts_borders is NULL");
    hipStream_t s = (hipStream_t)stream;
    const double ap = a * prior;
    ts_bins_kernel<<<grid_for(n, 256, ctx->num_cus * 8), 256, 0, s>>>(
        num, den, n, y_shift, a, ap, ts_borders, ts_bin_out ? n_ts_borders : 0, ts_bin_out,
        ts_out);
    CBH_LAUNCHED();
    return CBH_OK;
}

}  // extern "C"
