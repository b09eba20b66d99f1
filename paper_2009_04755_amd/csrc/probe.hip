// VALU issue-rate probe: the denominators of the VALU-bound rooflines (the overlap and GMM
// kernels price a term in issue slots of FP32 FMA, v_exp_f32 and v_rcp_f32).  Each lane runs
// PROBE_CHAINS independent dependency chains of one instruction kind, so that the SIMDs issue
// back to back; the grid holds eight waves per SIMD of every CU.  The rate is instructions
// per second over all lanes, timed with HIP events around the launch.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace rk {
namespace {

constexpr int PROBE_CHAINS = 8;
constexpr int PROBE_UNROLL = 16;

enum { PROBE_FMA = 0, PROBE_EXP2 = 1, PROBE_RCP = 2 };

template <int KIND>
__global__ __launch_bounds__(256) void k_probe(float *__restrict__ sink, int iters, float seed)
{
    float a[PROBE_CHAINS];
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) a[c] = seed + 0.001f * (threadIdx.x + c);
    const float m = 0.999f, k = 0.0001f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; ++u)
#pragma unroll
            for (int c = 0; c < PROBE_CHAINS; ++c) {
                if (KIND == PROBE_FMA) a[c] = fmaf(a[c], m, k);                 // v_fma_f32
                if (KIND == PROBE_EXP2) a[c] = __builtin_amdgcn_exp2f(-a[c]);   // v_exp_f32, stays in [0.5, 1]
                if (KIND == PROBE_RCP) a[c] = __builtin_amdgcn_rcpf(a[c]);      // v_rcp_f32, alternates x, 1/x
            }
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < PROBE_CHAINS; ++c) s += a[c];
    if (s == 12345.678f) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;  // keeps the chains alive
}

template <int KIND>
rocket_status run(int grid, int iters, hipEvent_t e0, hipEvent_t e1, float *sink, double *rate)
{
    hipLaunchKernelGGL(k_probe<KIND>, dim3(grid), dim3(256), 0, nullptr, sink, 1, 0.5f);  // warm-up
    if (hipEventRecord(e0, nullptr) != hipSuccess) return ROCKET_E_HIP;
    hipLaunchKernelGGL(k_probe<KIND>, dim3(grid), dim3(256), 0, nullptr, sink, iters, 0.5f);
    if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return ROCKET_E_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.f) return ROCKET_E_HIP;
    *rate = (double)grid * 256 * iters * PROBE_UNROLL * PROBE_CHAINS / (ms * 1e-3);
    return ROCKET_OK;
}

}  // namespace
}  // namespace rk

extern "C" rocket_status rocket_probe_valu(int device, double *fma_per_s, double *exp2_per_s, double *rcp_per_s)
{
    if (!fma_per_s || !exp2_per_s || !rcp_per_s) return rk::fail(nullptr, ROCKET_E_INVALID, "NULL argument");
    if (hipSetDevice(device) != hipSuccess) return rk::fail(nullptr, ROCKET_E_HIP, "hipSetDevice failed");
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        return rk::fail(nullptr, ROCKET_E_HIP, "cannot read the CU count");
    const int grid = cus * 8;  // 256-thread workgroups: 4 waves each, 8 waves per SIMD
    float *sink = nullptr;
    if (hipMalloc(&sink, sizeof(float) * (size_t)grid * 256) != hipSuccess)
        return rk::fail(nullptr, ROCKET_E_OOM, "hipMalloc of the probe sink failed");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rocket_status st = ROCKET_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = ROCKET_E_HIP;
    if (st == ROCKET_OK) st = rk::run<rk::PROBE_FMA>(grid, 4096, e0, e1, sink, fma_per_s);
    if (st == ROCKET_OK) st = rk::run<rk::PROBE_EXP2>(grid, 1024, e0, e1, sink, exp2_per_s);
    if (st == ROCKET_OK) st = rk::run<rk::PROBE_RCP>(grid, 1024, e0, e1, sink, rcp_per_s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (st != ROCKET_OK) return rk::fail(nullptr, st, "VALU probe launch or timing failed");
    return ROCKET_OK;
}
