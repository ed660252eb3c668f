// gfx950 kernels of the cell-sum environment: the paper's own form of the
// field (Sec. II.B, Eq. ElectrostaticField), nuclei plus M point-charge cells,
//     V(r) = sum_A Z_A / |r - R_A| - sum_m q_m / |r - r_m|.
//
// Batched mode (k_cells): the layout of the Gaussian kernel, with cells for
// pairs.  Every lane owns NP points; the wave walks its split's cells with
// wave-uniform scalar loads (one 8-word record feeds 64 NP points).  FP32C:
// the exact FP64 difference rounded once to FP32, a refined v_rsq_f32, FP32
// partial sums over 16 cells promoted to FP64; FP64: the same in FP64.
//
// Single-point mode (k_cells_one): one electron position for the whole GPU,
// the situation of the paper's QMC loop (one r_new per call, Sec. III).
// Consecutive threads take consecutive cells (the coalesced layout of the
// paper's Eq. coalease); wave partial sums by lane shuffles, workgroup sums
// through LDS, and the last workgroup to finish adds all workgroup partials
// in index order, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "cells_internal.h"
#include "device_math.h"
#include "env_potential.h"

namespace envpot {
namespace {

constexpr int kCellBlock = 256;

struct CellRec32 {
    double x, y, z;
    float q;
};

struct CellRec64 {
    double x, y, z, q;
};

__device__ __forceinline__ void load_cell(const GLB uint32_t* __restrict__ r, CellRec32& c) {
    const GLB double* d = reinterpret_cast<const GLB double*>(r);
    c.x = d[0];
    c.y = d[1];
    c.z = d[2];
    c.q = reinterpret_cast<const GLB float*>(r)[6];
}

__device__ __forceinline__ void load_cell(const GLB uint32_t* __restrict__ r, CellRec64& c) {
    const GLB double* d = reinterpret_cast<const GLB double*>(r);
    c.x = d[0];
    c.y = d[1];
    c.z = d[2];
    c.q = d[3];
}

template <int NP, bool F64>
__global__ __launch_bounds__(kCellBlock) void k_cells(CellArgs a) {
    const PTS double* __restrict__ pts = gpts(a.pts);
    const GLB uint32_t* __restrict__ cells = glb(a.cells);
    const GLB double* __restrict__ nuc = glb(a.nuc);
    const int64_t n = a.n;
    const int64_t base = (int64_t)blockIdx.x * (kCellBlock * NP) + threadIdx.x;
    double cx[NP], cy[NP], cz[NP], ve[NP], vn[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int64_t i = base + (int64_t)k * kCellBlock;
        const int64_t ic = i < n ? i : n - 1;  // ragged tail: recompute the last point
        cx[k] = pts[3 * ic];
        cy[k] = pts[3 * ic + 1];
        cz[k] = pts[3 * ic + 2];
        ve[k] = vn[k] = 0.0;
    }
    const int s = blockIdx.y;
    if (s == 0) {
        for (int q = 0; q < a.n_nuc; ++q) {
            const double qx = nuc[4 * q], qy = nuc[4 * q + 1], qz = nuc[4 * q + 2], qZ = nuc[4 * q + 3];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const double dx = cx[k] - qx, dy = cy[k] - qy, dz = cz[k] - qz;
                vn[k] += qZ * rsqrt(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)));
            }
        }
    }
    const GLB int32_t* __restrict__ split = glb(a.split);
    const int c0 = split[s], c1 = split[s + 1];
    if constexpr (F64) {
        CellRec64 cur, nxt;
        if (c0 < c1) load_cell(cells + (int64_t)c0 * kCellWords, cur);
        for (int m = c0; m < c1; ++m) {
            load_cell(cells + (int64_t)min(m + 1, c1 - 1) * kCellWords, nxt);
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const double X = cur.x - cx[k], Y = cur.y - cy[k], Z = cur.z - cz[k];
                const double r2 = __builtin_fma(X, X, __builtin_fma(Y, Y, Z * Z));
                ve[k] = __builtin_fma(cur.q, rsqrt_far(r2), ve[k]);
            }
            cur = nxt;
        }
    } else {
        CellRec32 cur, nxt;
        if (c0 < c1) load_cell(cells + (int64_t)c0 * kCellWords, cur);
        for (int m0 = c0; m0 < c1; m0 += kCellTile) {
            const int m1 = min(m0 + kCellTile, c1);
            float tile[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) tile[k] = 0.0f;
            for (int m = m0; m < m1; ++m) {
                load_cell(cells + (int64_t)min(m + 1, c1 - 1) * kCellWords, nxt);
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const float X = (float)(cur.x - cx[k]);
                    const float Y = (float)(cur.y - cy[k]);
                    const float Z = (float)(cur.z - cz[k]);
                    const float r2 = __builtin_fmaf(X, X, __builtin_fmaf(Y, Y, Z * Z));
                    tile[k] = __builtin_fmaf(cur.q, rsqrt_refined(r2), tile[k]);
                }
                cur = nxt;
            }
#pragma unroll
            for (int k = 0; k < NP; ++k) ve[k] += (double)tile[k];
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int64_t i = base + (int64_t)k * kCellBlock;
        if (i < n) a.out[(int64_t)s * n + i] = vn[k] - ve[k];
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum of v over the workgroup, in a fixed order (lane shuffles, then the
// four wave sums in wave order); the result is valid in every thread.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < kCellBlock / 64; ++k) t += sh[k];
    __syncthreads();
    return t;
}

// This workgroup's share of the cells at one point (every stride-th cell
// from its first; kOneUnroll loaded before any is used, so their memory
// latencies overlap), summed over the workgroup in fixed order.
template <bool F64>
__device__ __forceinline__ double cells_block_partial(const uint32_t* cells, int64_t m_total, double px, double py,
                                                      double pz, double* sh) {
    const PTS double* __restrict__ cd = gpts(reinterpret_cast<const double*>(cells));
    const int64_t stride = (int64_t)gridDim.x * kCellBlock;
    constexpr int kOneUnroll = 4;
    double acc = 0.0;
    for (int64_t m0 = (int64_t)blockIdx.x * kCellBlock + threadIdx.x; m0 < m_total; m0 += kOneUnroll * stride) {
        double cx[kOneUnroll], cy[kOneUnroll], cz[kOneUnroll], cq[kOneUnroll];
#pragma unroll
        for (int u = 0; u < kOneUnroll; ++u) {
            const int64_t m = m0 + u * stride;
            const bool ok = m < m_total;
            const PTS double* c = cd + (ok ? m : m0) * (kCellWords / 2);
            cx[u] = c[0];
            cy[u] = c[1];
            cz[u] = c[2];
            if constexpr (F64) cq[u] = ok ? c[3] : 0.0;
            else cq[u] = ok ? (double)reinterpret_cast<const PTS float*>(c)[6] : 0.0;
        }
        if constexpr (F64) {
#pragma unroll
            for (int u = 0; u < kOneUnroll; ++u) {
                const double X = cx[u] - px, Y = cy[u] - py, Z = cz[u] - pz;
                acc = __builtin_fma(cq[u], rsqrt_far(__builtin_fma(X, X, __builtin_fma(Y, Y, Z * Z))), acc);
            }
        } else {
            float tile = 0.0f;
#pragma unroll
            for (int u = 0; u < kOneUnroll; ++u) {
                const float X = (float)(cx[u] - px), Y = (float)(cy[u] - py), Z = (float)(cz[u] - pz);
                tile = __builtin_fmaf((float)cq[u], rsqrt_refined(__builtin_fmaf(X, X, __builtin_fmaf(Y, Y, Z * Z))),
                                      tile);
            }
            acc += (double)tile;
        }
    }
    return block_sum(acc, sh);
}

// Publish this workgroup's partial and take a ticket; true in every thread
// of the last workgroup to finish.
__device__ __forceinline__ bool cells_ticket(double bs, double* part, unsigned int* ticket, int* last) {
    if (threadIdx.x == 0) {
        // the partial goes to the device-coherent level, and the ticket's
        // release orders it before the increment (cheaper than a full fence:
        // measured 0.5-1 us of the 9-10 us launch)
        __hip_atomic_store(part + blockIdx.x, bs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned int t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        *last = (t == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    return *last != 0;
}

// The last workgroup: every workgroup partial in index order, minus from
// the nuclear sum; valid in thread 0.
__device__ __forceinline__ double cells_finish(const double* part, const double* nucp, int n_nuc, double px,
                                              double py, double pz, double* sh) {
    // every partial is written; read them past the caches
    __threadfence();
    double v = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kCellBlock)
        v += __hip_atomic_load(part + b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double total = block_sum(v, sh);
    double vn = 0.0;
    if (threadIdx.x == 0) {
        const GLB double* __restrict__ nuc = glb(nucp);
        for (int q = 0; q < n_nuc; ++q) {
            const double dx = px - nuc[4 * q], dy = py - nuc[4 * q + 1], dz = pz - nuc[4 * q + 2];
            vn += nuc[4 * q + 3] * rsqrt(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)));
        }
    }
    return vn - total;
}

template <bool F64>
__global__ __launch_bounds__(kCellBlock) void k_cells_one(CellOneArgs a) {
    __shared__ double sh[kCellBlock / 64];
    __shared__ int last;
    const GLB double* __restrict__ pt = glb(a.pt);
    const double px = pt[0], py = pt[1], pz = pt[2];
    const double bs = cells_block_partial<F64>(a.cells, a.m, px, py, pz, sh);
    if (!cells_ticket(bs, a.part, a.ticket, &last)) return;
    const double v = cells_finish(a.part, a.nuc, a.n_nuc, px, py, pz, sh);
    if (threadIdx.x == 0) {
        a.out[0] = v;
        __hip_atomic_store(a.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Resident single-point mode: the same rounds as k_cells_one, one per
// position the host posts, without a launch per position.  Workgroup 0's
// thread 0 alone polls the host mailbox (fine-grained host memory, system
// scope) and relays each position through device memory (agent scope) to
// every workgroup; the last workgroup of a round writes V and then the
// round's sequence number back into the mailbox.  Exit: the host's stop
// flag, or no position for idle_ticks of the 100 MHz real-time counter
// (workgroup 0 decides and relays; the others also give up a second after
// that on their own, so every wave ends).
template <bool F64>
__global__ __launch_bounds__(kCellBlock) void k_cells_resident(CellResidentArgs a) {
    __shared__ double sh[kCellBlock / 64];
    __shared__ int last;
    __shared__ double spt[3];
    __shared__ int scmd;
    CellMailbox* box = a.box;
    CellRelay* relay = a.relay;
    uint64_t seen = a.start_seq;
    for (;;) {
        if (threadIdx.x == 0) {
            int cmd = 0;
            uint64_t t0 = wall_clock64();
            if (blockIdx.x == 0) {
                // relaxed polls (an acquire per poll would invalidate the
                // caches every time); one acquire fence once a change is seen
                for (;;) {
                    const uint64_t r = __hip_atomic_load(&box->req_seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    const uint32_t stop = __hip_atomic_load(&box->stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    if (stop) break;
                    if (r != seen) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
                        for (int c = 0; c < 3; ++c) {
                            const double v = __hip_atomic_load(&box->point[c], __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_SYSTEM);
                            __hip_atomic_store(&relay->point[c], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                        cmd = 1;
                        seen = r;
                        break;
                    }
                    if (wall_clock64() - t0 > a.idle_ticks) break;
                    __builtin_amdgcn_s_sleep(2);
                }
                if (!cmd) __hip_atomic_store(&box->running, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&relay->cmd, (uint32_t)cmd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&relay->seq, cmd ? seen : ~0ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                for (;;) {
                    const uint64_t r = __hip_atomic_load(&relay->seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (r != seen) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        cmd = (int)__hip_atomic_load(&relay->cmd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        seen = r;
                        break;
                    }
                    if (wall_clock64() - t0 > a.idle_ticks + a.grace_ticks) break;
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            if (cmd)
                for (int c = 0; c < 3; ++c)
                    spt[c] = __hip_atomic_load(&relay->point[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            scmd = cmd;
        }
        __syncthreads();
        if (!scmd) return;
        const double px = spt[0], py = spt[1], pz = spt[2];
        const double bs = cells_block_partial<F64>(a.cells, a.m, px, py, pz, sh);
        if (cells_ticket(bs, a.part, a.ticket, &last)) {
            const double v = cells_finish(a.part, a.nuc, a.n_nuc, px, py, pz, sh);
            if (threadIdx.x == 0) {
                __hip_atomic_store(a.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&box->value, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                __hip_atomic_store(&box->done_seq, seen, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
        __syncthreads();
    }
}

}  // namespace

int launch_cells(const CellArgs& a, int S, int precision, int np, void* stream) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t per = (int64_t)kCellBlock * np;
    const dim3 grid((unsigned)((a.n + per - 1) / per), (unsigned)S);
    if (precision == ENV_PREC_FP64) {
        if (np == 1) hipLaunchKernelGGL((k_cells<1, true>), grid, dim3(kCellBlock), 0, st, a);
        else hipLaunchKernelGGL((k_cells<2, true>), grid, dim3(kCellBlock), 0, st, a);
    } else {
        if (np == 1) hipLaunchKernelGGL((k_cells<1, false>), grid, dim3(kCellBlock), 0, st, a);
        else if (np == 2) hipLaunchKernelGGL((k_cells<2, false>), grid, dim3(kCellBlock), 0, st, a);
        else hipLaunchKernelGGL((k_cells<4, false>), grid, dim3(kCellBlock), 0, st, a);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_cells_resident(const CellResidentArgs& a, int grid, int precision, void* stream) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (precision == ENV_PREC_FP64)
        hipLaunchKernelGGL((k_cells_resident<true>), dim3(grid), dim3(kCellBlock), 0, st, a);
    else
        hipLaunchKernelGGL((k_cells_resident<false>), dim3(grid), dim3(kCellBlock), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_cells_one(const CellOneArgs& a, int grid, int precision, void* stream) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (precision == ENV_PREC_FP64)
        hipLaunchKernelGGL((k_cells_one<true>), dim3(grid), dim3(kCellBlock), 0, st, a);
    else
        hipLaunchKernelGGL((k_cells_one<false>), dim3(grid), dim3(kCellBlock), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace envpot
