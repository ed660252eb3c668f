// On-device peak probes: the vector-ALU rates this GPU actually sustains
// for the instruction kinds the point kernels are made of.  Each kernel runs
// eight independent dependency chains per lane (enough work in flight to
// saturate issue) and writes one value per lane, so nothing is optimised away.
#include <hip/hip_runtime.h>

#include "probe.h"

namespace envpot {
namespace {

constexpr int kProbeIters = 2048;
constexpr int kProbeBlocks = 8192;
constexpr int kProbeThreads = 256;

__global__ __launch_bounds__(kProbeThreads) void k_probe_fma32(float* out, float a) {
    float x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = (float)(threadIdx.x + c);
    for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = __builtin_fmaf(x[c], a, 1.0f);
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += x[c];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_fma64(double* out, double a) {
    double x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = (double)(threadIdx.x + c);
    for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = __builtin_fma(x[c], a, 1.0);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += x[c];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

__global__ __launch_bounds__(kProbeThreads) void k_probe_rsq32(float* out, float a) {
    float x[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = (float)(threadIdx.x + c + 1);
    for (int i = 0; i < kProbeIters; ++i) {
#pragma unroll
        for (int c = 0; c < 8; ++c) x[c] = __builtin_amdgcn_rsqf(x[c]) + a;
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 8; ++c) s += x[c];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace

int run_peak_probe(double* ms_out) {
    const int64_t n = int64_t(kProbeBlocks) * kProbeThreads;
    void* buf = nullptr;
    if (hipMalloc(&buf, size_t(n) * sizeof(double)) != hipSuccess) return -1;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    if (hipStreamCreate(&st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess)
        rc = -1;
    for (int k = 0; k < 3 && rc == 0; ++k) {
        for (int rep = 0; rep < 2 && rc == 0; ++rep) {  // the second run is the one kept
            (void)hipEventRecord(e0, st);
            if (k == 0)
                hipLaunchKernelGGL(k_probe_fma32, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st,
                                   static_cast<float*>(buf), 0.999f);
            else if (k == 1)
                hipLaunchKernelGGL(k_probe_fma64, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st,
                                   static_cast<double*>(buf), 0.999);
            else
                hipLaunchKernelGGL(k_probe_rsq32, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st,
                                   static_cast<float*>(buf), 0.5f);
            (void)hipEventRecord(e1, st);
            float ms = 0.0f;
            if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = -1;
            ms_out[k] = ms;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    (void)hipFree(buf);
    return rc;
}

int64_t peak_probe_lane_ops() { return int64_t(kProbeBlocks) * kProbeThreads * kProbeIters * 8; }

}  // namespace envpot
