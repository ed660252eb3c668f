// Device helpers shared by the gfx950 kernels: address-space casts and the
// reciprocal square roots of the far-field and point-charge terms.
#pragma once

#include <hip/hip_runtime.h>

namespace envpot {

// Address spaces.  The pair records, segments, nuclei and Boys table are
// never written while a kernel runs, so they are read through the constant
// address space: wave-uniform loads through it become scalar loads even in
// the persistent kernel, whose work-queue atomics and output stores would
// otherwise count as possible clobbers.  Points are read through the global
// address space (per-lane vector loads).
#define GLB __attribute__((address_space(4)))
#define PTS __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ const GLB T* glb(const T* p) {
    return (const GLB T*)p;
}

template <typename T>
__device__ __forceinline__ const PTS T* gpts(const T* p) {
    return (const PTS T*)p;
}

// 1/sqrt(x) from v_rsq_f32 plus one Newton correction y + y (1 - x y^2) / 2.
__device__ __forceinline__ float rsqrt_refined(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    const float h = x * y;
    const float e = __builtin_fmaf(-h, y, 1.0f);
    return __builtin_fmaf(0.5f * e, y, y);
}

// 1/sqrt(x) from v_rsq_f32 alone, for the FP32C far field.  Over its input
// mantissas the instruction's relative error averages -7.36e-9 (-0.086 ulp;
// measured on gfx950 over 2^24 log-uniform inputs in [1, 4), two binades,
// which cover every pattern since rsq(4x) = rsq(x)/2); the error of a single
// value stays below 0.87 ulp.  The far-field kernels remove the mean from
// their FP64 tile sums (kRsqMeanFix), so what is left per term is the
// zero-mean part of the error instead of a systematic bias times the sum of
// the terms' magnitudes.
constexpr double kRsqMeanFix = 1.0 + 7.36e-9;
__device__ __forceinline__ float rsqrt_raw(float x) { return __builtin_amdgcn_rsqf(x); }

// 1/sqrt(x) for finite x > 0 (far-field distances): v_rsq_f64 plus the
// second-order correction y (1 + e/2 + 3e^2/8), e = 1 - x y^2, of the series
// of (1 - e)^(-1/2).
__device__ __forceinline__ double rsqrt_far(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double h = x * y;
    const double e = __builtin_fma(-h, y, 1.0);
    return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}

}  // namespace envpot
