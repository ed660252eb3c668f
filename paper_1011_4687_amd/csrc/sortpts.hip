// Spatial order of the evaluation points: a Morton (Z-order) key on a
// 0.25-bohr grid, a radix sort of the keys (hipCUB), a gather of the points
// in key order and, after the evaluation, a scatter of the values back to
// the caller's order.  Points that are close in space then share waves, so
// fewer waves meet a pair (or cluster) inside its far-field radius with only
// some of their lanes.
#include <hip/hip_runtime.h>

#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "sort_internal.h"

namespace envpot {
namespace {

constexpr int kSortBlock = 256;
constexpr double kInvCell = 4.0;  // grid cells per bohr

// The 10 low bits of v spread to every third bit.
__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t cell(double x) {
    double c = floor(x * kInvCell) + 512.0;  // the grid covers +-128 bohr; outside, the key saturates
    c = c < 0.0 ? 0.0 : (c > 1023.0 ? 1023.0 : c);
    return uint32_t(c);
}

__global__ __launch_bounds__(kSortBlock) void k_morton(const double* __restrict__ pts, int64_t n,
                                                       uint32_t* __restrict__ key, uint32_t* __restrict__ idx) {
    const int64_t i = int64_t(blockIdx.x) * kSortBlock + threadIdx.x;
    if (i >= n) return;
    const uint32_t x = cell(pts[3 * i]), y = cell(pts[3 * i + 1]), z = cell(pts[3 * i + 2]);
    key[i] = spread10(x) | (spread10(y) << 1) | (spread10(z) << 2);
    idx[i] = uint32_t(i);
}

__global__ __launch_bounds__(kSortBlock) void k_gather(const double* __restrict__ pts,
                                                       const uint32_t* __restrict__ order, int64_t n,
                                                       double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * kSortBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t j = order[i];
    out[3 * i] = pts[3 * j];
    out[3 * i + 1] = pts[3 * j + 1];
    out[3 * i + 2] = pts[3 * j + 2];
}

__global__ __launch_bounds__(kSortBlock) void k_scatter(const double* __restrict__ v,
                                                        const uint32_t* __restrict__ order, int64_t n,
                                                        double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * kSortBlock + threadIdx.x;
    if (i >= n) return;
    out[order[i]] = v[i];
}

__global__ __launch_bounds__(kSortBlock) void k_scatter4(const double* __restrict__ v,
                                                         const uint32_t* __restrict__ order, int64_t n,
                                                         double* __restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * kSortBlock + threadIdx.x;
    if (i >= n) return;
    const int64_t j = order[i];
#pragma unroll
    for (int c = 0; c < 4; ++c) out[4 * j + c] = v[4 * i + c];
}

__global__ __launch_bounds__(kSortBlock) void k_scatter_multi(const ScatterDesc* __restrict__ d) {
    const ScatterDesc q = d[blockIdx.y];
    const int64_t i = int64_t(blockIdx.x) * kSortBlock + threadIdx.x;
    if (i >= q.n) return;
    q.out[q.order[i]] = q.v[i];
}

unsigned blocks(int64_t n) { return unsigned((n + kSortBlock - 1) / kSortBlock); }

}  // namespace

int sort_points(const double* pts, int64_t n, double* sorted, uint32_t* order, void* stream) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n <= 0 || n > int64_t(INT32_MAX)) return -1;
    uint32_t *key = nullptr, *key2 = nullptr, *idx = nullptr;
    void* tmp = nullptr;
    size_t tmp_bytes = 0;
    int rc = 0;
    if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, key, key2, idx, order, int(n), 0, 30, st) !=
        hipSuccess)
        return -1;
    if (hipMallocAsync(reinterpret_cast<void**>(&key), size_t(n) * 4, st) != hipSuccess) return -1;
    if (hipMallocAsync(reinterpret_cast<void**>(&key2), size_t(n) * 4, st) != hipSuccess) rc = -1;
    if (rc == 0 && hipMallocAsync(reinterpret_cast<void**>(&idx), size_t(n) * 4, st) != hipSuccess) rc = -1;
    if (rc == 0 && hipMallocAsync(&tmp, std::max<size_t>(tmp_bytes, 1), st) != hipSuccess) rc = -1;
    if (rc == 0) {
        hipLaunchKernelGGL(k_morton, dim3(blocks(n)), dim3(kSortBlock), 0, st, pts, n, key, idx);
        if (hipGetLastError() != hipSuccess) rc = -1;
    }
    if (rc == 0 && hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, key, key2, idx, order, int(n), 0, 30, st) !=
                       hipSuccess)
        rc = -1;
    if (rc == 0) {
        hipLaunchKernelGGL(k_gather, dim3(blocks(n)), dim3(kSortBlock), 0, st, pts, order, n, sorted);
        if (hipGetLastError() != hipSuccess) rc = -1;
    }
    (void)hipFreeAsync(tmp, st);
    (void)hipFreeAsync(idx, st);
    (void)hipFreeAsync(key2, st);
    (void)hipFreeAsync(key, st);
    return rc;
}

bool stream_capturing(void* stream) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (!stream) return false;  // the null stream is never captured here
    if (hipStreamIsCapturing(static_cast<hipStream_t>(stream), &cap) != hipSuccess) return true;
    return cap != hipStreamCaptureStatusNone;
}

int scatter_values(const double* v, const uint32_t* order, int64_t n, double* out, void* stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_scatter, dim3(blocks(n)), dim3(kSortBlock), 0, static_cast<hipStream_t>(stream), v, order,
                       n, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int scatter_values_multi(const ScatterDesc* d, int n_desc, int64_t max_n, void* stream) {
    if (n_desc <= 0 || max_n <= 0) return 0;
    hipLaunchKernelGGL(k_scatter_multi, dim3(blocks(max_n), unsigned(n_desc)), dim3(kSortBlock), 0,
                       static_cast<hipStream_t>(stream), d);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace envpot

namespace envpot {

int scatter_rows4(const double* v, const uint32_t* order, int64_t n, double* out, void* stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_scatter4, dim3(blocks(n)), dim3(kSortBlock), 0, static_cast<hipStream_t>(stream), v,
                       order, n, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace envpot
