// gfx950 kernels of the environment potential.
//
// Work unit: one point x one primitive shell pair.  The paper's GPU kernel
// (Sec. III, Eq. blockSum) gave a whole block of threads one electron
// position (in constant memory) and split the environment terms across the
// threads.  Here the roles are inverted: every lane owns NP electron
// positions in VGPRs and the whole wavefront walks the same pair list, so the
// pair record is wave-uniform and is fetched with scalar loads into SGPRs
// (the modern counterpart of the paper's broadcast constant-memory operand),
// read once per wave and reused by 64*NP points.  Lanes of a wave read
// consecutive points (the coalesced layout of the paper's Eq. coalease).
//
// Per point-pair (FP32C path):
//   X = (float)(P - C) in FP64 (exact difference, one rounding),
//   T = p |X|^2,
//   Boys G_n: far field (T >= tfar[L]) G_n = (-1)^n (2n-1)!! |X|^{-2n-1}
//   from a refined v_rsq_f32; near field a 6-term Taylor step from the
//   tabulated F_n(k/8) held in LDS, scaled by 2 sqrt(p/pi) (-2p)^n,
//   McMurchie-Davidson R_tuv recursion and contraction with the pair's
//   Hermite density (hermite_gen.h),
//   FP32 sums over tiles of kTile pairs, promoted to FP64 per tile.
// The nuclear term and the per-fragment (nuclear - electronic) sums are FP64.
// With a split factor S > 1 the pair list is cut into S cost-balanced ranges
// (grid dimension y) whose FP64 partials a second kernel adds in fixed order,
// so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "envpot_internal.h"
#include "hermite_gen.h"

namespace envpot {
namespace {

constexpr int kTile = 8;  // pairs per FP32 partial sum

template <int L, typename T>
__device__ __forceinline__ T hermite_dot(const T* G, T X, T Y, T Z, const T* __restrict__ D) {
    if constexpr (L == 0) return hermite_dot_L0<T>(G, X, Y, Z, D);
    else if constexpr (L == 1) return hermite_dot_L1<T>(G, X, Y, Z, D);
    else if constexpr (L == 2) return hermite_dot_L2<T>(G, X, Y, Z, D);
    else if constexpr (L == 3) return hermite_dot_L3<T>(G, X, Y, Z, D);
    else return hermite_dot_L4<T>(G, X, Y, Z, D);
}

// 1/sqrt(x) from v_rsq_f32 plus one Newton correction y + y (1 - x y^2) / 2.
__device__ __forceinline__ float rsqrt_refined(float x) {
    const float y = __builtin_amdgcn_rsqf(x);
    const float h = x * y;
    const float e = __builtin_fmaf(-h, y, 1.0f);
    return __builtin_fmaf(0.5f * e, y, y);
}

template <int L, int NP>
__device__ __forceinline__ void pairs_f32(const uint32_t* __restrict__ rec, int npairs,
                                          const double* cx, const double* cy, const double* cz,
                                          const float* tab, float tfar, double* ele) {
    constexpr int RW = rec32_words(L);
    for (int i0 = 0; i0 < npairs; i0 += kTile) {
        float tile[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) tile[k] = 0.0f;
        const int m = min(kTile, npairs - i0);
        for (int j = 0; j < m; ++j) {
            const uint32_t* r = rec + (int64_t)(i0 + j) * RW;
            const double* rd = reinterpret_cast<const double*>(r);
            const float* rf = reinterpret_cast<const float*>(r + 6);
            const double Px = rd[0], Py = rd[1], Pz = rd[2];
            const float p = rf[0], c1 = rf[1];
            const float* D = rf + 2;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const float X = (float)(Px - cx[k]);
                const float Y = (float)(Py - cy[k]);
                const float Z = (float)(Pz - cz[k]);
                const float r2 = __builtin_fmaf(X, X, __builtin_fmaf(Y, Y, Z * Z));
                const float T = p * r2;
                float G[L + 1];
                if (T < tfar) {
                    const int kk = (int)__builtin_fmaf(T, (float)kBoysGridInv, 0.5f);
                    const float d = __builtin_fmaf((float)kk, -1.0f / kBoysGridInv, T);
                    const float* f = tab + kk * kBoysRowF32;
                    const float d2 = 0.5f * d, d3 = d * (1.0f / 3.0f), d4 = 0.25f * d, d5 = 0.2f * d;
                    const float m2p = -2.0f * p;
                    float s = c1;
#pragma unroll
                    for (int n = 0; n <= L; ++n) {
                        float F = __builtin_fmaf(-d5, f[n + 5], f[n + 4]);
                        F = __builtin_fmaf(-d4, F, f[n + 3]);
                        F = __builtin_fmaf(-d3, F, f[n + 2]);
                        F = __builtin_fmaf(-d2, F, f[n + 1]);
                        F = __builtin_fmaf(-d, F, f[n]);
                        G[n] = s * F;
                        s *= m2p;
                    }
                } else {
                    const float ri = rsqrt_refined(r2);
                    const float ri2 = ri * ri;
                    G[0] = ri;
#pragma unroll
                    for (int n = 1; n <= L; ++n) G[n] = (G[n - 1] * ri2) * (float)(1 - 2 * n);
                }
                tile[k] += hermite_dot<L, float>(G, X, Y, Z, D);
            }
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) ele[k] += (double)tile[k];
    }
}

template <int L, int NP>
__device__ __forceinline__ void pairs_f64(const uint32_t* __restrict__ rec, int npairs,
                                          const double* cx, const double* cy, const double* cz,
                                          const double* __restrict__ tab, double tfar,
                                          double* ele) {
    constexpr int RW = rec64_words(L);
    for (int i = 0; i < npairs; ++i) {
        const double* rd = reinterpret_cast<const double*>(rec + (int64_t)i * RW);
        const double Px = rd[0], Py = rd[1], Pz = rd[2], p = rd[3], c1 = rd[4];
        const double* D = rd + 5;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const double X = Px - cx[k], Y = Py - cy[k], Z = Pz - cz[k];
            const double r2 = __builtin_fma(X, X, __builtin_fma(Y, Y, Z * Z));
            const double T = p * r2;
            double G[L + 1];
            if (T < tfar) {
                const int kk = (int)__builtin_fma(T, (double)kBoysGridInv, 0.5);
                const double d = __builtin_fma((double)kk, -1.0 / kBoysGridInv, T);
                const double* f = tab + kk * kBoysRowF64;
                double dj[kBoysTaylorF64];
#pragma unroll
                for (int j = 1; j < kBoysTaylorF64; ++j) dj[j] = d * (1.0 / j);
                const double m2p = -2.0 * p;
                double s = c1;
#pragma unroll
                for (int n = 0; n <= L; ++n) {
                    double F = f[n + kBoysTaylorF64 - 1];
#pragma unroll
                    for (int j = kBoysTaylorF64 - 1; j >= 1; --j) F = __builtin_fma(-dj[j], F, f[n + j - 1]);
                    G[n] = s * F;
                    s *= m2p;
                }
            } else {
                const double ri = rsqrt(r2);
                const double ri2 = ri * ri;
                G[0] = ri;
#pragma unroll
                for (int n = 1; n <= L; ++n) G[n] = (G[n - 1] * ri2) * (double)(1 - 2 * n);
            }
            ele[k] += hermite_dot<L, double>(G, X, Y, Z, D);
        }
    }
}

template <int NP, bool F64>
__global__ __launch_bounds__(kBlock) void k_potential(EvalArgs a) {
    __shared__ float tab32[F64 ? 1 : kBoysMaxRowsF32 * kBoysRowF32];
    if constexpr (!F64) {
        const float* g = static_cast<const float*>(a.boys);
        for (int i = threadIdx.x; i < a.bp.rows32 * kBoysRowF32; i += kBlock) tab32[i] = g[i];
        __syncthreads();
    }
    const int64_t base = (int64_t)blockIdx.x * (kBlock * NP) + threadIdx.x;
    double cx[NP], cy[NP], cz[NP], acc[NP], vn[NP], ve[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int64_t i = base + (int64_t)k * kBlock;
        const int64_t ic = i < a.n ? i : a.n - 1;  // ragged tail: recompute the last point
        cx[k] = a.pts[3 * ic];
        cy[k] = a.pts[3 * ic + 1];
        cz[k] = a.pts[3 * ic + 2];
        acc[k] = vn[k] = ve[k] = 0.0;
    }
    const int s = blockIdx.y;
    const int sb = a.split[s], se = a.split[s + 1];
    for (int g = sb; g < se; ++g) {
        const Segment sg = a.segs[g];
        for (int q = sg.nuc_begin; q < sg.nuc_end; ++q) {
            const double qx = a.nuc[4 * q], qy = a.nuc[4 * q + 1], qz = a.nuc[4 * q + 2],
                         qZ = a.nuc[4 * q + 3];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const double dx = cx[k] - qx, dy = cy[k] - qy, dz = cz[k] - qz;
                vn[k] += qZ * rsqrt(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)));
            }
        }
        const uint32_t* rec = a.rec + sg.rec_off;
        if constexpr (F64) {
            const double* tab = static_cast<const double*>(a.boys);
            switch (sg.L) {
                case 0: pairs_f64<0, NP>(rec, sg.n_pairs, cx, cy, cz, tab, a.bp.tfar64[0], ve); break;
                case 1: pairs_f64<1, NP>(rec, sg.n_pairs, cx, cy, cz, tab, a.bp.tfar64[1], ve); break;
                case 2: pairs_f64<2, NP>(rec, sg.n_pairs, cx, cy, cz, tab, a.bp.tfar64[2], ve); break;
                case 3: pairs_f64<3, NP>(rec, sg.n_pairs, cx, cy, cz, tab, a.bp.tfar64[3], ve); break;
                default: pairs_f64<4, NP>(rec, sg.n_pairs, cx, cy, cz, tab, a.bp.tfar64[4], ve); break;
            }
        } else {
            switch (sg.L) {
                case 0: pairs_f32<0, NP>(rec, sg.n_pairs, cx, cy, cz, tab32, a.bp.tfar32[0], ve); break;
                case 1: pairs_f32<1, NP>(rec, sg.n_pairs, cx, cy, cz, tab32, a.bp.tfar32[1], ve); break;
                case 2: pairs_f32<2, NP>(rec, sg.n_pairs, cx, cy, cz, tab32, a.bp.tfar32[2], ve); break;
                case 3: pairs_f32<3, NP>(rec, sg.n_pairs, cx, cy, cz, tab32, a.bp.tfar32[3], ve); break;
                default: pairs_f32<4, NP>(rec, sg.n_pairs, cx, cy, cz, tab32, a.bp.tfar32[4], ve); break;
            }
        }
        if (sg.flags & kSegEndGroup) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                acc[k] += vn[k] - ve[k];
                vn[k] = ve[k] = 0.0;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        acc[k] += vn[k] - ve[k];
        const int64_t i = base + (int64_t)k * kBlock;
        if (i < a.n) a.out[(int64_t)s * a.n + i] = acc[k];
    }
}

__global__ __launch_bounds__(kBlock) void k_sum_splits(const double* __restrict__ part, int S,
                                                       int64_t n, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < S; ++k) s += part[(int64_t)k * n + i];
    out[i] = s;
}

}  // namespace

int launch_potential(const EvalArgs& a, int S, int precision, int np, void* stream) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t per = (int64_t)kBlock * np;
    const dim3 grid((unsigned)((a.n + per - 1) / per), (unsigned)S);
    const dim3 block(kBlock);
    if (precision == ENV_PREC_FP64) {
        if (np == 2) hipLaunchKernelGGL((k_potential<2, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_potential<1, true>), grid, block, 0, st, a);
    } else {
        if (np == 1) hipLaunchKernelGGL((k_potential<1, false>), grid, block, 0, st, a);
        else if (np == 4) hipLaunchKernelGGL((k_potential<4, false>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_potential<2, false>), grid, block, 0, st, a);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_sum_splits(const double* partial, int S, int64_t n, double* out, void* stream) {
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_sum_splits, grid, dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                       partial, S, n, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace envpot
