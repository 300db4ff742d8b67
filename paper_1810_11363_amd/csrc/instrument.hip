// Instrumentation (not part of the method): the LDS update rates that bound
// the histogram build. Every lane of a 1024-thread block updates 4-byte or
// 8-byte LDS words on distinct banks (lane l of wave w: word w * 64 + l plus
// a step of 1024 words per update), so the rate is the LDS unit's issue rate
// for that operation, not a bank-conflict rate.
#include <algorithm>

#include "common.h"
#include "kernels_dev.h"

namespace cbh {

constexpr int kProbeWords = 4096;   // 32-bit words of the LDS array (16 KB)
constexpr int kProbeIter = 128;     // steps per thread
constexpr int kProbeUnroll = 8;     // updates per step

// OP: 0 ds_add_u32, 1 ds_add_f32, 2 ds_add_f64, 3 ds_add_u64,
//     4 float32 add by 32-bit compare-and-swap, 5 (float, float) pair add by
//     64-bit compare-and-swap (the float32 forms' cell updates)
template <int OP>
__global__ __launch_bounds__(1024) void lds_rate_kernel(float* __restrict__ out) {
    __shared__ uint64_t words[kProbeWords / 2];
    uint32_t* w32 = reinterpret_cast<uint32_t*>(words);
    for (int i = threadIdx.x; i < kProbeWords / 2; i += blockDim.x) words[i] = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int it = 0; it < kProbeIter; ++it) {
        uint32_t a[kProbeUnroll];
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u)
            a[u] = (wave * 64 + lane + (uint32_t)(it * kProbeUnroll + u) * 1024u);
        if constexpr (OP == 0) {
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u)
                __hip_atomic_fetch_add(w32 + (a[u] & (kProbeWords - 1)), 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if constexpr (OP == 1) {
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u)
                __hip_atomic_fetch_add(reinterpret_cast<float*>(w32) + (a[u] & (kProbeWords - 1)),
                                       1.0f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if constexpr (OP == 2) {
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u)
                __hip_atomic_fetch_add(
                    reinterpret_cast<double*>(words) + (a[u] & (kProbeWords / 2 - 1)), 1.0,
                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if constexpr (OP == 3) {
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u)
                __hip_atomic_fetch_add(words + (a[u] & (kProbeWords / 2 - 1)), (uint64_t)1,
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else if constexpr (OP == 4) {
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u)
                cas_add_f32(w32 + (a[u] & (kProbeWords - 1)), 1.0f);
        } else {
#pragma unroll
            for (int u = 0; u < kProbeUnroll; ++u) {
                uint64_t* p = words + (a[u] & (kProbeWords / 2 - 1));
                uint64_t old = lds_load64(p);
                for (;;) {
                    const uint64_t got = lds_cas64(p, old, add_pair_word(old, 1.0f, 1.0f));
                    if (got == old) break;
                    old = got;
                }
            }
        }
    }
    __syncthreads();
    // keep the updates: one word per thread to global memory
    out[blockIdx.x * blockDim.x + threadIdx.x] =
        __uint_as_float(w32[threadIdx.x & (kProbeWords - 1)]);
}

}  // namespace cbh

using namespace cbh;

extern "C" int cbh_probe_lds_rates(cbh_ctx* ctx, double* rates_out) {
    clear_error();
    CBH_ARG(ctx != nullptr && rates_out != nullptr, "NULL argument");
    int clock_khz = 0;
    CBH_HIP(hipDeviceGetAttribute(&clock_khz, hipDeviceAttributeClockRate, ctx->device));
    const int blocks = ctx->num_cus * 4;
    float* out = nullptr;
    CBH_HIP(hipMalloc(&out, (size_t)blocks * 1024 * sizeof(float)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = CBH_OK;
    auto run = [&](auto kernel, double* rate) -> int {
        kernel<<<blocks, 1024>>>(out);   // warm-up
        CBH_LAUNCHED();
        CBH_HIP(hipEventRecord(e0, nullptr));
        for (int r = 0; r < 3; ++r) kernel<<<blocks, 1024>>>(out);
        CBH_HIP(hipEventRecord(e1, nullptr));
        CBH_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        CBH_HIP(hipEventElapsedTime(&ms, e0, e1));
        const double updates = 3.0 * blocks * 1024.0 * kProbeIter * kProbeUnroll;
        *rate = updates / (ms * 1e-3) / (double(ctx->num_cus) * clock_khz * 1e3);
        return CBH_OK;
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        set_error("hipEventCreate failed");
        rc = CBH_EDEVICE;
    }
    if (!rc) rc = run(lds_rate_kernel<0>, rates_out + 0);
    if (!rc) rc = run(lds_rate_kernel<1>, rates_out + 1);
    if (!rc) rc = run(lds_rate_kernel<2>, rates_out + 2);
    if (!rc) rc = run(lds_rate_kernel<3>, rates_out + 3);
    if (!rc) rc = run(lds_rate_kernel<4>, rates_out + 4);
    if (!rc) rc = run(lds_rate_kernel<5>, rates_out + 5);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipDeviceSynchronize();
    (void)hipFree(out);
    return rc;
}
