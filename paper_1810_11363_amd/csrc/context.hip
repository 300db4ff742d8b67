// Context, errors, workspace and host-side border selection.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace cbh {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

// Every entry point starts here: the message is reset, and so is the HIP
// runtime's last-error state, so that a launch check after our own launches
// reports our launches only.
void clear_error() {
    g_err[0] = 0;
    (void)hipGetLastError();
}

int ensure_ws(cbh_ctx* ctx, int64_t bytes, void* stream) {
    bytes = align_up(std::max<int64_t>(bytes, 256), 1 << 20);
    if (bytes <= ctx->ws_size) return CBH_OK;
    CBH_REQUIRE(bytes <= ctx->ws_limit, CBH_ENOMEM,
                "workspace of %lld bytes exceeds the limit of %lld bytes",
                (long long)bytes, (long long)ctx->ws_limit);
    // A graph being captured would keep the new buffer's address; growing
    // (an allocation) is refused there: run the calls once before the
    // capture, or reserve the workspace with cbh_reserve_workspace.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    CBH_HIP(hipStreamIsCapturing((hipStream_t)stream, &cap));
    CBH_REQUIRE(cap == hipStreamCaptureStatusNone, CBH_EBUSY,
                "workspace must grow from %lld to %lld bytes while the stream is being "
                "captured; run the calls once before capturing or call "
                "cbh_reserve_workspace",
                (long long)ctx->ws_size, (long long)bytes);
    void* nw = nullptr;
    hipError_t e = hipMalloc(&nw, (size_t)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("workspace allocation of %lld bytes failed: %s", (long long)bytes,
                  hipGetErrorString(e));
        return CBH_ENOMEM;
    }
    // the old buffer is kept, not freed: graphs captured earlier may use it
    if (ctx->ws) ctx->ws_retired.push_back(ctx->ws);
    ctx->ws = nw;
    ctx->ws_size = bytes;
    return CBH_OK;
}

int validate_problem(const cbh_problem* p) {
    CBH_ARG(p != nullptr, "problem is NULL");
    CBH_ARG(p->n >= 1, "n must be >= 1 (got %lld)", (long long)p->n);
    CBH_ARG(p->n < (int64_t(1) << 40), "n too large");
    CBH_ARG(p->n_features >= 1, "n_features must be >= 1");
    CBH_REQUIRE(p->max_bins >= 2 && p->max_bins <= CBH_MAX_BINS, CBH_EUNSUPPORTED,
                "max_bins must be in [2, 256] (got %d)", p->max_bins);
    CBH_ARG(p->bins != nullptr && p->n_bins != nullptr, "bins / n_bins is NULL");
    CBH_REQUIRE(p->depth >= 1 && p->depth <= CBH_MAX_DEPTH, CBH_EUNSUPPORTED,
                "depth must be in [1, 16] (got %d)", p->depth);
    CBH_ARG(p->loss == CBH_LOSS_RMSE || p->loss == CBH_LOSS_LOGLOSS ||
                p->loss == CBH_LOSS_MULTICLASS,
            "unknown loss %d", p->loss);
    if (p->loss == CBH_LOSS_MULTICLASS) {
        CBH_REQUIRE(p->K >= 2 && p->K <= CBH_MAX_K, CBH_EUNSUPPORTED,
                    "MultiClass needs 2 <= K <= 16 (got %d)", p->K);
    } else {
        CBH_ARG(p->K == 1, "K must be 1 for RMSE and Logloss (got %d)", p->K);
    }
    CBH_ARG(p->label && p->g && p->leaf && p->approx, "label/g/leaf/approx is NULL");
    CBH_ARG(count_stat(p) || p->h != nullptr, "h is NULL (needed unless RMSE without weights)");
    CBH_ARG(p->bin_bits == 0 || p->bin_bits == 8 || p->bin_bits == 4 || p->bin_bits == 1,
            "bin_bits must be 0 or 8 (bytes), 4 or 1 (got %d)", p->bin_bits);
    if (packed_bins(p)) {
        CBH_REQUIRE(p->max_bins <= (1 << p->bin_bits), CBH_EUNSUPPORTED,
                    "max_bins %d does not fit in %d-bit bins", p->max_bins, p->bin_bits);
        CBH_ARG(p->seg_stride == nullptr, "packed bins are plain columns (seg_stride NULL)");
    }
    return CBH_OK;
}

int validate_precision(const cbh_problem* p, int32_t precision) {
    CBH_ARG(precision == CBH_PREC_FP32 || precision == CBH_PREC_TWOFLOAT ||
                precision == CBH_PREC_INT16 || precision == CBH_PREC_F64,
            "unknown precision %d", precision);
    if (precision == CBH_PREC_INT16)
        CBH_ARG(p->gq != nullptr && p->grad_scale != nullptr,
                "INT16 precision needs gq and grad_scale");
    return CBH_OK;
}

}  // namespace cbh

using namespace cbh;

namespace cbh {
// Device clock stamp (instrumentation).
__global__ void stamp_kernel(uint64_t* slot) {
    if (threadIdx.x == 0) *slot = wall_clock64();
}
}  // namespace cbh

extern "C" {

const char* cbh_last_error(void) { return g_err; }

int cbh_create(int device, cbh_ctx** out) {
    clear_error();
    CBH_ARG(out != nullptr, "out is NULL");
    *out = nullptr;
    int count = 0;
    CBH_HIP(hipGetDeviceCount(&count));
    CBH_ARG(device >= 0 && device < count, "device %d out of range (%d devices)", device,
            count);
    CBH_HIP(hipSetDevice(device));
    cbh_ctx* c = new cbh_ctx();
    c->device = device;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess)
        c->num_cus = v;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
        hipSuccess)
        c->max_lds = v;
    hipError_t e = hipMalloc(&c->d_flags, 64);
    if (e != hipSuccess) {
        delete c;
        set_error("hipMalloc of error flags failed: %s", hipGetErrorString(e));
        return CBH_EDEVICE;
    }
    e = hipMemset(c->d_flags, 0, 64);
    if (e != hipSuccess) {
        (void)hipFree(c->d_flags);
        delete c;
        set_error("hipMemset failed: %s", hipGetErrorString(e));
        return CBH_EDEVICE;
    }
    hist_init_attrs(c->max_lds);
    batch_init_attrs(c->max_lds);
    part_init_attrs(c->max_lds);
    const int rc = score_static_init(c);
    if (rc != CBH_OK) {
        (void)hipFree(c->d_flags);
        delete c;
        return rc;
    }
    *out = c;
    return CBH_OK;
}

void cbh_destroy(cbh_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->ws) (void)hipFree(ctx->ws);
    for (void* w : ctx->ws_retired) (void)hipFree(w);
    if (ctx->d_flags) (void)hipFree(ctx->d_flags);
    delete ctx;
}

int cbh_set_workspace_limit(cbh_ctx* ctx, int64_t bytes) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(bytes > 0, "limit must be > 0");
    ctx->ws_limit = bytes;
    return CBH_OK;
}

int64_t cbh_workspace_size(const cbh_ctx* ctx) { return ctx ? ctx->ws_size : 0; }

int cbh_reserve_workspace(cbh_ctx* ctx, int64_t bytes) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_ARG(bytes >= 0, "bytes must be >= 0");
    return ensure_ws(ctx, bytes, nullptr);
}

int cbh_device_timestamp(cbh_ctx* ctx, uint64_t* slot, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr && slot != nullptr, "NULL argument");
    stamp_kernel<<<1, 64, 0, (hipStream_t)stream>>>(slot);
    CBH_LAUNCHED();
    return CBH_OK;
}

int cbh_device_clock_khz(cbh_ctx* ctx, int64_t* khz) {
    clear_error();
    CBH_ARG(ctx != nullptr && khz != nullptr, "NULL argument");
    int v = 0;
    CBH_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, ctx->device));
    *khz = v;
    return CBH_OK;
}

int cbh_sync(cbh_ctx* ctx, void* stream) {
    clear_error();
    CBH_ARG(ctx != nullptr, "ctx is NULL");
    CBH_HIP(hipStreamSynchronize((hipStream_t)stream));
    CBH_HIP(hipGetLastError());
    uint32_t flags = 0;
    CBH_HIP(hipMemcpy(&flags, ctx->d_flags, sizeof(flags), hipMemcpyDeviceToHost));
    if (flags) {
        CBH_HIP(hipMemset(ctx->d_flags, 0, sizeof(flags)));
        std::string msg = "device reported:";
        if (flags & FLAG_NAN_INPUT) msg += " NaN feature value (binned as 0);";
        if (flags & FLAG_BAD_INDEX) msg += " permutation entry outside [0, n);";
        if (flags & FLAG_BAD_SPLIT) msg += " model split feature outside [0, F) (bit taken as 0);";
        if (flags & FLAG_PACK_RANGE)
            msg += " bin value too large for the packed width (stored masked);";
        if (flags & FLAG_FUSED_WAIT)
            msg += " a fused batched level gave up waiting for an earlier stage (results invalid);";
        set_error("%s", msg.c_str());
        return CBH_EDEVICE;
    }
    return CBH_OK;
}

// Value-at-rank quantile borders; see the header for the rule.
int cbh_select_borders(const float* x_host, int64_t n, int32_t max_bins, float* borders_out,
                       int32_t* n_borders_out) {
    clear_error();
    CBH_ARG(n_borders_out != nullptr && borders_out != nullptr, "output pointer is NULL");
    *n_borders_out = 0;
    CBH_ARG(n >= 0, "n must be >= 0");
    CBH_ARG(n == 0 || x_host != nullptr, "x_host is NULL");
    CBH_REQUIRE(max_bins >= 2 && max_bins <= CBH_MAX_BINS, CBH_EUNSUPPORTED,
                "max_bins must be in [2, 256] (got %d)", max_bins);
    if (n == 0) return CBH_OK;
    std::vector<float> s(x_host, x_host + n);
    for (float v : s) CBH_ARG(!std::isnan(v), "NaN value in feature column");
    std::sort(s.begin(), s.end());
    const float top = s[n - 1];
    int64_t distinct = 1;
    for (int64_t i = 1; i < n; ++i) distinct += (s[i] != s[i - 1]);
    int32_t nb = 0;
    if (distinct <= max_bins) {
        float prev = 0.f;
        for (int64_t i = 0; i < n && s[i] != top; ++i) {
            if (nb == 0 || s[i] != prev) {
                borders_out[nb++] = s[i];
                prev = s[i];
            }
        }
    } else {
        for (int64_t j = 1; j < max_bins; ++j) {
            const float c = s[(j * n) / max_bins - 1];
            if (c == top || (nb > 0 && c == borders_out[nb - 1])) continue;
            borders_out[nb++] = c;
        }
    }
    *n_borders_out = nb;
    return CBH_OK;
}

int cbh_uniform_borders(double lo, double hi, int32_t n_bins, double* borders_out) {
    clear_error();
    CBH_ARG(borders_out != nullptr, "borders_out is NULL");
    CBH_ARG(std::isfinite(lo) && std::isfinite(hi) && hi >= lo, "need finite lo <= hi");
    CBH_REQUIRE(n_bins >= 2 && n_bins <= CBH_MAX_BINS, CBH_EUNSUPPORTED,
                "n_bins must be in [2, 256] (got %d)", n_bins);
    for (int32_t j = 1; j < n_bins; ++j)
        borders_out[j - 1] = lo + ((hi - lo) * (double)j) / (double)n_bins;
    return CBH_OK;
}

}  // extern "C"
