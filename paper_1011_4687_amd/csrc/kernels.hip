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
//   far field (p |X|^2 >= tfar[L], where the Boys function equals its
//   asymptote to below 2^-28): the pair is an exact finite multipole,
//   evaluated as (1/R) sum h_abc x^a y^b z^c with x = X/R^2 (one refined
//   v_rsq_f32 and a Horner polynomial, hermite_gen.h);
//   near field: T = p |X|^2, Boys F_n by a 6-term Taylor step from the
//   tabulated F_n(k/8) held in LDS, G_n = 2 sqrt(p/pi) (-2p)^n F_n, the
//   McMurchie-Davidson R_tuv recursion and its contraction with the pair's
//   Hermite density (hermite_gen.h),
//   FP32 sums over tiles of kTile pairs, promoted to FP64 per tile.
// The nuclear term and the per-fragment (nuclear - electronic) sums are FP64.
// Pairs whose two shells sit on one atom share that atom as product centre;
// their far fields are merged per atom and radius band into one multipole
// ("cluster"), evaluated once per wave while no point is inside its radius.
// With a split factor S > 1 the pair list is cut into S cost-balanced ranges
// (grid dimension y) whose FP64 partials a second kernel adds in fixed order,
// so results are bitwise reproducible.  The point kernels ask for four waves
// per SIMD (128 VGPRs): the long-lived per-point state then spills to scratch
// once per segment, which costs less than the latency a third wave hides.
#include <hip/hip_runtime.h>

#include "device_math.h"
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

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int L, typename T>
__device__ __forceinline__ T far_poly(const T* __restrict__ h, T x, T y, T z) {
    if constexpr (L == 0) return far_poly_L0<T>(h, x, y, z);
    else if constexpr (L == 1) return far_poly_L1<T>(h, x, y, z);
    else if constexpr (L == 2) return far_poly_L2<T>(h, x, y, z);
    else if constexpr (L == 3) return far_poly_L3<T>(h, x, y, z);
    else return far_poly_L4<T>(h, x, y, z);
}

// The far-field polynomial at X = P - C with w = 1/|X|^2.  For L = 1 the
// degree-1 part is formed from X directly, h0 + w (hx X + hy Y + hz Z),
// which saves the three scalings X w, Y w, Z w.
template <int L, typename T>
__device__ __forceinline__ T far_value(const T* __restrict__ h, T X, T Y, T Z, T w) {
    if constexpr (L == 1) {
        // component order (0,0,0), (0,0,1), (0,1,0), (1,0,0)
        return fma_t(w, fma_t(h[1], Z, fma_t(h[2], Y, h[3] * X)), h[0]);
    } else {
        return far_poly<L, T>(h, X * w, Y * w, Z * w);
    }
}

// The part of a record every point needs: centre, far-field radius^2 and
// far-field coefficients.  The loop below loads pair i+1's head while it
// computes pair i, so the scalar-load latency overlaps the arithmetic.
template <int L, typename T>
struct Head {
    double px, py, pz;
    T r2far;
    T h[kNComp[L]];
};

// Prefetch the next head only while two heads fit comfortably in SGPRs
// (spilled SGPRs cost VALU writelane/readlane instructions).
template <int L, typename T>
constexpr bool kPipelined = (6 + (1 + kNComp[L]) * int(sizeof(T) / 4)) <= 20;

template <int L>
__device__ __forceinline__ void load_head32(const GLB uint32_t* __restrict__ r, Head<L, float>& o) {
    const GLB double* rd = reinterpret_cast<const GLB double*>(r);
    const GLB float* rf = reinterpret_cast<const GLB float*>(r + 6);
    o.px = rd[0];
    o.py = rd[1];
    o.pz = rd[2];
    o.r2far = rf[0];
#pragma unroll
    for (int c = 0; c < kNComp[L]; ++c) o.h[c] = rf[3 + c];
}

template <int L>
__device__ __forceinline__ void load_head64(const GLB uint32_t* __restrict__ r, Head<L, double>& o) {
    const GLB double* rd = reinterpret_cast<const GLB double*>(r);
    o.px = rd[0];
    o.py = rd[1];
    o.pz = rd[2];
    o.r2far = rd[3];
#pragma unroll
    for (int c = 0; c < kNComp[L]; ++c) o.h[c] = rd[kRec64Head + c];
}

// Near field of one point (FP32): Boys values from the LDS table by a 6-term
// Taylor step, then the Hermite recursion contracted with D.
template <int L>
__device__ __forceinline__ float near_f32(const GLB uint32_t* __restrict__ r, float X, float Y, float Z,
                                          float r2, const float* tab) {
    const GLB float* rf = reinterpret_cast<const GLB float*>(r + 6);
    const float p = rf[1], c1 = rf[2];
    float D[kNComp[L]];
#pragma unroll
    for (int c = 0; c < kNComp[L]; ++c) D[c] = rf[3 + kNComp[L] + c];
    const float T = p * r2;
    const int kk = (int)__builtin_fmaf(T, (float)kBoysGridInv, 0.5f);
    const float d = __builtin_fmaf((float)kk, -1.0f / kBoysGridInv, T);
    const float* f = tab + kk * kBoysRowF32;
    const float d2 = 0.5f * d, d3 = d * (1.0f / 3.0f), d4 = 0.25f * d, d5 = 0.2f * d;
    const float m2p = -2.0f * p;
    float s = c1;
    float G[L + 1];
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
    return hermite_dot<L, float>(G, X, Y, Z, D);
}

template <int L>
__device__ __forceinline__ double near_f64(const GLB uint32_t* __restrict__ r, double X, double Y,
                                           double Z, double r2, const GLB double* __restrict__ tab) {
    const GLB double* rd = reinterpret_cast<const GLB double*>(r);
    const double p = rd[4], c1 = rd[5];
    double D[kNComp[L]];
#pragma unroll
    for (int c = 0; c < kNComp[L]; ++c) D[c] = rd[kRec64Head + kNComp[L] + c];
    const double T = p * r2;
    const int kk = (int)__builtin_fma(T, (double)kBoysGridInv, 0.5);
    const double d = __builtin_fma((double)kk, -1.0 / kBoysGridInv, T);
    const GLB double* f = tab + kk * kBoysRowF64;
    double dj[kBoysTaylorF64];
#pragma unroll
    for (int j = 1; j < kBoysTaylorF64; ++j) dj[j] = d * (1.0 / j);
    const double m2p = -2.0 * p;
    double s = c1;
    double G[L + 1];
#pragma unroll
    for (int n = 0; n <= L; ++n) {
        double F = f[n + kBoysTaylorF64 - 1];
#pragma unroll
        for (int j = kBoysTaylorF64 - 1; j >= 1; --j) F = __builtin_fma(-dj[j], F, f[n + j - 1]);
        G[n] = s * F;
        s *= m2p;
    }
    return hermite_dot<L, double>(G, X, Y, Z, D);
}

// FP32C pairs of one L.  Record: P (3 doubles), r2far, p, c1, h[nc], D[nc].
// FAR: every point-pair is known to be in the far field, and every point C
// is at least 2|C - O| from each pair centre (segment box test), where O is
// the wave-uniform origin (ox, oy, oz).  The per-pair near test is left out
// and X = P - C is formed as fl32(P - O) - fl32(C - O): one FP64 difference
// per pair and coordinate for the whole wave instead of one per point.  Its
// error is at most 2^-24 (|P - O| + |C - O| + |X|) <= 3 * 2^-24 |X| per
// component (against 2^-24 |X| for the rounded exact difference).
template <int L, int NP, bool FAR>
__device__ __forceinline__ void pairs_f32(const GLB uint32_t* __restrict__ rec, int npairs,
                                          const double* cx, const double* cy, const double* cz,
                                          double ox, double oy, double oz,
                                          const float* tab, double* ele) {
    constexpr int RW = rec32_words(L);
    if (npairs <= 0) return;
    Head<L, float> cur;
    if constexpr (kPipelined<L, float>) load_head32<L>(rec, cur);
    float crx[NP], cry[NP], crz[NP];
    double oxv = ox, oyv = oy, ozv = oz;
    if constexpr (FAR) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            crx[k] = (float)(cx[k] - ox);
            cry[k] = (float)(cy[k] - oy);
            crz[k] = (float)(cz[k] - oz);
        }
        // the origin in vector registers for the loop: an FP64 add takes one
        // scalar operand, and the pair centre is already one (an empty asm
        // with register constraints only; it emits no instruction)
        asm("" : "+v"(oxv), "+v"(oyv), "+v"(ozv));
    }
    // tiles of kTile pairs: FP32 partial sums, promoted to FP64 per tile
    for (int i0 = 0; i0 < npairs; i0 += kTile) {
        const int i1 = min(i0 + kTile, npairs);
        float tile[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) tile[k] = 0.0f;
        int i = i0;
        while (i < i1) {
            float X[NP], Y[NP], Z[NP], r2[NP];
            Head<L, float> nxt;
            // far-field run: pairs whose far-field radius no point of the wave is inside
            for (; i < i1; ++i) {
                if constexpr (kPipelined<L, float>) load_head32<L>(rec + (int64_t)min(i + 1, npairs - 1) * RW, nxt);
                else load_head32<L>(rec + (int64_t)i * RW, cur);
                if constexpr (FAR) {
                    const float prx = (float)(cur.px - oxv), pry = (float)(cur.py - oyv),
                                prz = (float)(cur.pz - ozv);
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        X[k] = prx - crx[k];
                        Y[k] = pry - cry[k];
                        Z[k] = prz - crz[k];
                        r2[k] = __builtin_fmaf(X[k], X[k], __builtin_fmaf(Y[k], Y[k], Z[k] * Z[k]));
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < NP; ++k) {
                        X[k] = (float)(cur.px - cx[k]);
                        Y[k] = (float)(cur.py - cy[k]);
                        Z[k] = (float)(cur.pz - cz[k]);
                        r2[k] = __builtin_fmaf(X[k], X[k], __builtin_fmaf(Y[k], Y[k], Z[k] * Z[k]));
                    }
                }
                if constexpr (!FAR) {
                    float m = r2[0];
#pragma unroll
                    for (int k = 1; k < NP; ++k) m = fminf(m, r2[k]);
                    if (__builtin_expect(__builtin_amdgcn_ballot_w64(m < cur.r2far) != 0, 0)) break;
                }
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const float ri = rsqrt_raw(r2[k]);
                    const float w = ri * ri;
                    tile[k] = __builtin_fmaf(ri, far_value<L, float>(cur.h, X[k], Y[k], Z[k], w), tile[k]);
                }
                if constexpr (kPipelined<L, float>) cur = nxt;
            }
            if (i >= i1) break;
            // pair i has some point of the wave inside its far-field radius:
            // far form for the other points, then the near points of every
            // lane one per pass (a pass per near point of the busiest lane,
            // not one per point slot that has a near point in some lane)
            const GLB uint32_t* r = rec + (int64_t)i * RW;
            uint32_t nm = 0;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (r2[k] < cur.r2far) {
                    nm |= 1u << k;
                } else {
                    const float ri = rsqrt_raw(r2[k]);
                    const float w = ri * ri;
                    tile[k] = __builtin_fmaf(ri, far_value<L, float>(cur.h, X[k], Y[k], Z[k], w), tile[k]);
                }
            }
            while (__builtin_amdgcn_ballot_w64(nm != 0) != 0) {
                if (nm != 0) {
                    const int kn = __builtin_ctz(nm);
                    nm &= nm - 1;
                    float xn = X[0], yn = Y[0], zn = Z[0], qn = r2[0];
#pragma unroll
                    for (int k = 1; k < NP; ++k) {
                        if (kn == k) {
                            xn = X[k];
                            yn = Y[k];
                            zn = Z[k];
                            qn = r2[k];
                        }
                    }
                    const float v = near_f32<L>(r, xn, yn, zn, qn, tab);
#pragma unroll
                    for (int k = 0; k < NP; ++k)
                        if (kn == k) tile[k] += v;
                }
            }
            if constexpr (kPipelined<L, float>) cur = nxt;
            ++i;
        }
#pragma unroll
        for (int k = 0; k < NP; ++k) ele[k] = __builtin_fma((double)tile[k], kRsqMeanFix, ele[k]);
    }
}

// FP64 pairs of one L.  Record: P, r2far, p, c1 (doubles), h[nc], D[nc].
template <int L, int NP, bool FAR>
__device__ __forceinline__ void pairs_f64(const GLB uint32_t* __restrict__ rec, int npairs,
                                          const double* cx, const double* cy, const double* cz,
                                          const GLB double* __restrict__ tab, double* ele) {
    constexpr int RW = rec64_words(L);
    if (npairs <= 0) return;
    Head<L, double> cur;
    if constexpr (kPipelined<L, double>) load_head64<L>(rec, cur);
    for (int i = 0; i < npairs; ++i) {
        const GLB uint32_t* r = rec + (int64_t)i * RW;
        Head<L, double> nxt;
        if constexpr (kPipelined<L, double>) load_head64<L>(rec + (int64_t)min(i + 1, npairs - 1) * RW, nxt);
        else load_head64<L>(r, cur);
        double X[NP], Y[NP], Z[NP], r2[NP];
        bool nearp = false;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            X[k] = cur.px - cx[k];
            Y[k] = cur.py - cy[k];
            Z[k] = cur.pz - cz[k];
            r2[k] = __builtin_fma(X[k], X[k], __builtin_fma(Y[k], Y[k], Z[k] * Z[k]));
            nearp |= r2[k] < cur.r2far;
        }
        if (FAR || __builtin_amdgcn_ballot_w64(nearp) == 0) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                const double ri = rsqrt_far(r2[k]);
                const double w = ri * ri;
                ele[k] = __builtin_fma(ri, far_value<L, double>(cur.h, X[k], Y[k], Z[k], w),
                                       ele[k]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                double v;
                if (r2[k] < cur.r2far) {
                    v = near_f64<L>(r, X[k], Y[k], Z[k], r2[k], tab);
                } else {
                    const double ri = rsqrt_far(r2[k]);
                    const double w = ri * ri;
                    v = ri * far_value<L, double>(cur.h, X[k], Y[k], Z[k], w);
                }
                ele[k] += v;
            }
        }
        if constexpr (kPipelined<L, double>) cur = nxt;
    }
}

// Same-centre clusters of merged L = LC, from cluster i on: every cluster
// whose far-field radius no point of the wave is inside is evaluated once
// from its merged coefficients.  Stops at the first cluster with a point
// inside that radius and returns its index (n when there is none); the
// caller then evaluates that cluster's members pair by pair.  FAR: every
// cluster is known to be far for every point of the wave (segment box
// test), so the near test is left out.  X stays the rounded exact
// difference here: a cluster holds a whole atom's band of charge in one
// term, so the extra rounding of the wave-origin form (an independent
// 2^-24 |P - O| per cluster) would not average out over many small terms
// as it does for pairs.
template <int LC, int NP, bool FAR>
__device__ __forceinline__ int clusters_f32(const GLB uint32_t* __restrict__ rec, int i, int n,
                                            const double* cx, const double* cy, const double* cz,
                                            double* ele) {
    constexpr int CW = cl32_words(LC);
    float tile[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) tile[k] = 0.0f;
    int done = 0;
    for (; i < n; ++i) {
        const GLB uint32_t* r = rec + (int64_t)i * CW;
        const GLB double* rd = reinterpret_cast<const GLB double*>(r);
        const GLB float* rf = reinterpret_cast<const GLB float*>(r);
        const double px = rd[0], py = rd[1], pz = rd[2];
        const float r2far = rf[6];
        float h[kNComp[LC]];
#pragma unroll
        for (int c = 0; c < kNComp[LC]; ++c) h[c] = rf[kClHead32 + c];
        float X[NP], Y[NP], Z[NP], r2[NP];
        bool nearp = false;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            X[k] = (float)(px - cx[k]);
            Y[k] = (float)(py - cy[k]);
            Z[k] = (float)(pz - cz[k]);
            r2[k] = __builtin_fmaf(X[k], X[k], __builtin_fmaf(Y[k], Y[k], Z[k] * Z[k]));
            nearp |= r2[k] < r2far;
        }
        if (!FAR && __builtin_amdgcn_ballot_w64(nearp) != 0) break;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const float ri = rsqrt_raw(r2[k]);
            const float w = ri * ri;
            tile[k] = __builtin_fmaf(ri, far_value<LC, float>(h, X[k], Y[k], Z[k], w), tile[k]);
        }
        if ((++done & (kTile - 1)) == 0) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                ele[k] = __builtin_fma((double)tile[k], kRsqMeanFix, ele[k]);
                tile[k] = 0.0f;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) ele[k] = __builtin_fma((double)tile[k], kRsqMeanFix, ele[k]);
    return i;
}

template <int LC, int NP, bool FAR>
__device__ __forceinline__ int clusters_f64(const GLB uint32_t* __restrict__ rec, int i, int n,
                                            const double* cx, const double* cy, const double* cz,
                                            double* ele) {
    constexpr int CW = cl64_words(LC);
    for (; i < n; ++i) {
        const GLB double* rd = reinterpret_cast<const GLB double*>(rec + (int64_t)i * CW);
        const double px = rd[0], py = rd[1], pz = rd[2], r2far = rd[3];
        double h[kNComp[LC]];
#pragma unroll
        for (int c = 0; c < kNComp[LC]; ++c) h[c] = rd[kClHead64 + c];
        double X[NP], Y[NP], Z[NP], r2[NP];
        bool nearp = false;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            X[k] = px - cx[k];
            Y[k] = py - cy[k];
            Z[k] = pz - cz[k];
            r2[k] = __builtin_fma(X[k], X[k], __builtin_fma(Y[k], Y[k], Z[k] * Z[k]));
            nearp |= r2[k] < r2far;
        }
        if (!FAR && __builtin_amdgcn_ballot_w64(nearp) != 0) break;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const double ri = rsqrt_far(r2[k]);
            const double w = ri * ri;
            ele[k] = __builtin_fma(ri, far_value<LC, double>(h, X[k], Y[k], Z[k], w), ele[k]);
        }
    }
    return i;
}

// The value of v in the first active lane, as a wave-uniform (scalar) value.
__device__ __forceinline__ double wave_uniform(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// One workgroup's share: points of point block `pblock` against the pair
// range of split `s` (all of it when S == 1).
template <int NP, bool F64>
__device__ __forceinline__ void block_work_impl(const PTS double* __restrict__ pts, int64_t n,
                                                const GLB Segment* __restrict__ segs,
                                                const GLB int32_t* __restrict__ split,
                                                const GLB uint32_t* __restrict__ recs,
                                                const GLB double* __restrict__ nuc,
                                                const GLB double* __restrict__ boys64,
                                                const GLB double* __restrict__ boxes,
                                                double* __restrict__ out,
                                                int64_t pblock, int s, const float* tab32) {
    const int64_t base = pblock * (kBlock * NP) + threadIdx.x;
    // the FP64 result of each point lives in LDS (thread-private slots,
    // touched once per fragment group): registers stay free for the loops
    __shared__ double acc[NP * kBlock];
    double cx[NP], cy[NP], cz[NP], ve[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int64_t i = base + (int64_t)k * kBlock;
        const int64_t ic = i < n ? i : n - 1;  // ragged tail: recompute the last point
        cx[k] = pts[3 * ic];
        cy[k] = pts[3 * ic + 1];
        cz[k] = pts[3 * ic + 2];
        acc[k * kBlock + threadIdx.x] = ve[k] = 0.0;
    }
    // wave-uniform origin of the FP32C far form: the wave's first point
    const double ox = wave_uniform(cx[0]), oy = wave_uniform(cy[0]), oz = wave_uniform(cz[0]);
    // Wave-uniform work loop over the segments of split s.  A cluster
    // segment is scanned cluster by cluster; a cluster with some point of
    // the wave inside its far-field radius hands its members (one run per L)
    // to the same pair dispatch as ordinary segments.
    const int sb = split[s], se = split[s + 1];
    int g = sb;
    bool fold = false;
    const GLB uint32_t* crec = recs;   // cluster segment in progress: clusters [ci, cn) of merged L lc
    int ci = 0, cn = 0, lc = 0;
    bool cfar = false;                 // ... and all its clusters far for every point of the wave
    const GLB uint32_t* mtab = recs;   // member table of the cluster being expanded
    uint32_t pend = 0;                 // its member runs (bit L) not yet evaluated
    for (;;) {
        int L, npairs;
        const GLB uint32_t* rec;
        bool all_far = false;  // member runs and clusters: tested pair by pair
        if (pend != 0) {
            L = __builtin_ctz(pend);
            pend &= pend - 1;
            rec = recs + mtab[2 * L];
            npairs = (int)mtab[2 * L + 1];
        } else if (ci < cn) {
            if constexpr (F64) {
                switch (lc) {
                    case 0: ci = cfar ? clusters_f64<0, NP, true>(crec, ci, cn, cx, cy, cz, ve)
                                        : clusters_f64<0, NP, false>(crec, ci, cn, cx, cy, cz, ve); break;
                    case 1: ci = cfar ? clusters_f64<1, NP, true>(crec, ci, cn, cx, cy, cz, ve)
                                        : clusters_f64<1, NP, false>(crec, ci, cn, cx, cy, cz, ve); break;
                    case 2: ci = cfar ? clusters_f64<2, NP, true>(crec, ci, cn, cx, cy, cz, ve)
                                        : clusters_f64<2, NP, false>(crec, ci, cn, cx, cy, cz, ve); break;
                    case 3: ci = cfar ? clusters_f64<3, NP, true>(crec, ci, cn, cx, cy, cz, ve)
                                        : clusters_f64<3, NP, false>(crec, ci, cn, cx, cy, cz, ve); break;
                    default: ci = cfar ? clusters_f64<4, NP, true>(crec, ci, cn, cx, cy, cz, ve)
                                        : clusters_f64<4, NP, false>(crec, ci, cn, cx, cy, cz, ve); break;
                }
                if (ci < cn) {
                    const GLB uint32_t* c = crec + (int64_t)ci * cl64_words(lc);
                    mtab = c + kClTable64;
                    pend = c[kClMask64];
                    ++ci;
                }
            } else {
                switch (lc) {
                    case 0: ci = cfar ? clusters_f32<0, NP, true>(crec, ci, cn, cx, cy, cz, ve)
                                        : clusters_f32<0, NP, false>(crec, ci, cn, cx, cy, cz, ve); break;
                    case 1: ci = cfar ? clusters_f32<1, NP, true>(crec, ci, cn, cx, cy, cz, ve)
                                        : clusters_f32<1, NP, false>(crec, ci, cn, cx, cy, cz, ve); break;
                    case 2: ci = cfar ? clusters_f32<2, NP, true>(crec, ci, cn, cx, cy, cz, ve)
                                        : clusters_f32<2, NP, false>(crec, ci, cn, cx, cy, cz, ve); break;
                    case 3: ci = cfar ? clusters_f32<3, NP, true>(crec, ci, cn, cx, cy, cz, ve)
                                        : clusters_f32<3, NP, false>(crec, ci, cn, cx, cy, cz, ve); break;
                    default: ci = cfar ? clusters_f32<4, NP, true>(crec, ci, cn, cx, cy, cz, ve)
                                        : clusters_f32<4, NP, false>(crec, ci, cn, cx, cy, cz, ve); break;
                }
                if (ci < cn) {
                    const GLB uint32_t* c = crec + (int64_t)ci * cl32_words(lc);
                    mtab = c + kClTable32;
                    pend = c[kClMask32];
                    ++ci;
                }
            }
            continue;
        } else {
            if (fold) {
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    acc[k * kBlock + threadIdx.x] -= ve[k];
                    ve[k] = 0.0;
                }
                fold = false;
            }
            if (g >= se) break;
            const GLB Segment* sp = segs + g;
            ++g;
            const int sL = sp->L, sn = sp->n_pairs, nb = sp->nuc_begin, ne = sp->nuc_end,
                      sf = sp->flags;
            const int64_t so = sp->rec_off;
            for (int q = nb; q < ne; ++q) {
                const double qx = nuc[4 * q], qy = nuc[4 * q + 1], qz = nuc[4 * q + 2],
                             qZ = nuc[4 * q + 3];
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const double dx = cx[k] - qx, dy = cy[k] - qy, dz = cz[k] - qz;
                    ve[k] -= qZ * rsqrt(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)));
                }
            }
            fold = (sf & kSegEndGroup) != 0;
            // segment box test: every point of the wave beyond the largest
            // far-field radius of the segment's pairs (or clusters), and for
            // the FP32C origin form of pair segments at least 2|C - O| from
            // the box
            const bool cl = (sf & kSegCluster) != 0;
            if (boxes && sn > 0) {
                const GLB double* bx = boxes + (int64_t)kSegBoxWords * sp->box;
                const double lim = bx[6] * (1.0 + 1e-6);
                bool nearp = false;
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const double gx = fmax(0.0, fmax(bx[0] - cx[k], cx[k] - bx[3]));
                    const double gy = fmax(0.0, fmax(bx[1] - cy[k], cy[k] - bx[4]));
                    const double gz = fmax(0.0, fmax(bx[2] - cz[k], cz[k] - bx[5]));
                    const double g2 = __builtin_fma(gx, gx, __builtin_fma(gy, gy, gz * gz));
                    nearp |= g2 < lim;
                    if (!F64 && !cl) {
                        const double ex = cx[k] - ox, ey = cy[k] - oy, ez = cz[k] - oz;
                        nearp |= g2 < 4.0 * __builtin_fma(ex, ex, __builtin_fma(ey, ey, ez * ez));
                    }
                }
                all_far = __builtin_amdgcn_ballot_w64(nearp) == 0;
            }
            if (cl) {
                crec = recs + so;
                ci = 0;
                cn = sn;
                lc = sL;
                cfar = all_far;
                all_far = false;
                continue;
            }
            L = sL;
            rec = recs + so;
            npairs = sn;
        }
        if constexpr (F64) {
            const GLB double* tab = boys64;
            if (all_far) {
                switch (L) {
                    case 0: pairs_f64<0, NP, true>(rec, npairs, cx, cy, cz, tab, ve); break;
                    case 1: pairs_f64<1, NP, true>(rec, npairs, cx, cy, cz, tab, ve); break;
                    case 2: pairs_f64<2, NP, true>(rec, npairs, cx, cy, cz, tab, ve); break;
                    case 3: pairs_f64<3, NP, true>(rec, npairs, cx, cy, cz, tab, ve); break;
                    default: pairs_f64<4, NP, true>(rec, npairs, cx, cy, cz, tab, ve); break;
                }
            } else {
                switch (L) {
                    case 0: pairs_f64<0, NP, false>(rec, npairs, cx, cy, cz, tab, ve); break;
                    case 1: pairs_f64<1, NP, false>(rec, npairs, cx, cy, cz, tab, ve); break;
                    case 2: pairs_f64<2, NP, false>(rec, npairs, cx, cy, cz, tab, ve); break;
                    case 3: pairs_f64<3, NP, false>(rec, npairs, cx, cy, cz, tab, ve); break;
                    default: pairs_f64<4, NP, false>(rec, npairs, cx, cy, cz, tab, ve); break;
                }
            }
        } else {
            if (all_far) {
                switch (L) {
                    case 0: pairs_f32<0, NP, true>(rec, npairs, cx, cy, cz, ox, oy, oz, tab32, ve); break;
                    case 1: pairs_f32<1, NP, true>(rec, npairs, cx, cy, cz, ox, oy, oz, tab32, ve); break;
                    case 2: pairs_f32<2, NP, true>(rec, npairs, cx, cy, cz, ox, oy, oz, tab32, ve); break;
                    case 3: pairs_f32<3, NP, true>(rec, npairs, cx, cy, cz, ox, oy, oz, tab32, ve); break;
                    default: pairs_f32<4, NP, true>(rec, npairs, cx, cy, cz, ox, oy, oz, tab32, ve); break;
                }
            } else {
                switch (L) {
                    case 0: pairs_f32<0, NP, false>(rec, npairs, cx, cy, cz, ox, oy, oz, tab32, ve); break;
                    case 1: pairs_f32<1, NP, false>(rec, npairs, cx, cy, cz, ox, oy, oz, tab32, ve); break;
                    case 2: pairs_f32<2, NP, false>(rec, npairs, cx, cy, cz, ox, oy, oz, tab32, ve); break;
                    case 3: pairs_f32<3, NP, false>(rec, npairs, cx, cy, cz, ox, oy, oz, tab32, ve); break;
                    default: pairs_f32<4, NP, false>(rec, npairs, cx, cy, cz, ox, oy, oz, tab32, ve); break;
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const double v = acc[k * kBlock + threadIdx.x] - ve[k];
        const int64_t i = base + (int64_t)k * kBlock;
        if (i < n) out[(int64_t)s * n + i] = v;
    }
}

// The buffers go in as separate restrict pointers: stores to `out` then
// provably do not clobber the pair records, which keeps the record loads
// scalar even when block_work runs in a loop (persistent kernel).
template <int NP, bool F64>
__device__ __forceinline__ void block_work(const EvalArgs& a, int64_t pblock, int s,
                                           const float* tab32) {
    block_work_impl<NP, F64>(gpts(a.pts), a.n, glb(a.segs), glb(a.split), glb(a.rec), glb(a.nuc),
                             glb(static_cast<const double*>(a.boys)), glb(a.boxes), a.out, pblock, s, tab32);
}

// Stage the FP32 Boys table into LDS (one copy per workgroup; the near
// field gathers from it by per-lane row).  The FP64 table is read through
// the caches: staged in LDS (45 KB, or 26 KB on a coarser grid with more
// Taylor terms) it measured slower or no faster.
template <bool F64>
__device__ __forceinline__ void load_boys_lds(const void* boys, int rows32, float* tab32) {
    if constexpr (!F64) {
        const float* g = static_cast<const float*>(boys);
        for (int i = threadIdx.x; i < rows32 * kBoysRowF32; i += kBlock) tab32[i] = g[i];
        __syncthreads();
    }
}

template <int NP, bool F64>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_potential(EvalArgs a) {
    __shared__ float tab32[F64 ? 1 : kBoysMaxRowsF32 * kBoysRowF32];
    load_boys_lds<F64>(a.boys, a.bp.rows32, tab32);
    block_work<NP, F64>(a, blockIdx.x, blockIdx.y, tab32);
}

// A copy of *p read word by word through the constant address space.
template <class T>
__device__ __forceinline__ T load_const(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "whole words");
    T v;
    const GLB uint32_t* src = glb(reinterpret_cast<const uint32_t*>(p));
    uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
    for (int i = 0; i < int(sizeof(T) / 4); ++i) dst[i] = src[i];
    return v;
}

// Persistent batched kernel: every workgroup takes work items (instance,
// point block, pair split) from a global counter until the queue is empty.
// Items are sorted by decreasing estimated cost, so the long ones start
// first.  Every workgroup reaches the exit test once the counter passes
// n_items, so the grid always drains.
template <int NP, bool F64>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_potential_persistent(BatchArgs b) {
    __shared__ float tab32[F64 ? 1 : kBoysMaxRowsF32 * kBoysRowF32];
    __shared__ unsigned long long item_sh;
    load_boys_lds<F64>(b.boys, b.rows32, tab32);
    for (;;) {
        if (threadIdx.x == 0) item_sh = atomicAdd(b.counter, 1ull);
        __syncthreads();
        const unsigned long long it_v = item_sh;
        __syncthreads();
        // wave-uniform copy, so the item and its instance are read with scalar loads
        const int64_t it = (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(it_v >> 32)) << 32) |
                                     (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)it_v));
        if (it >= b.n_items) break;
        // item and instance arguments through the constant address space:
        // scalar loads the compiler may repeat instead of holding the values
        const BatchItem w = load_const(b.items + it);
        const EvalArgs a = load_const(b.args + w.inst);
        block_work<NP, F64>(a, w.pblock, w.split, tab32);
    }
}

// Split factor 2^k of a device-sized evaluation of m points (host and
// device use this one rule, so both kernels agree on k).
__host__ __device__ __forceinline__ int devsized_k(int64_t m, int np, int64_t want_waves, int64_t part_cap) {
    const int64_t waves = (m + 64 * np - 1) / (64 * np);
    int k = 0;
    while (k < kMaxSplitLog2 && (waves << k) < want_waves && (m << (k + 1)) <= part_cap) ++k;
    return k;
}

// Persistent kernel of a device-sized evaluation: the items (point block,
// split) of the shape chosen from m are numbered it = pblock * 2^k + s and
// taken from the counter until it reaches their count; every workgroup
// reaches that exit test, so the grid drains (also for m = 0).
template <int NP, bool F64>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_potential_devsized(DevSizedArgs d) {
    __shared__ float tab32[F64 ? 1 : kBoysMaxRowsF32 * kBoysRowF32];
    __shared__ unsigned long long item_sh;
    load_boys_lds<F64>(d.a.boys, d.a.bp.rows32, tab32);
    const int64_t m = *d.m;
    const int k = devsized_k(m, NP, d.want_waves, d.part_cap);
    const int64_t n_items = ((m + (int64_t)kBlock * NP - 1) / ((int64_t)kBlock * NP)) << k;
    EvalArgs a = d.a;
    a.n = m;
    a.segs = d.segs_all + d.seg_off[k];
    a.split = d.split_all + d.split_off[k];
    for (;;) {
        if (threadIdx.x == 0) item_sh = atomicAdd(d.counter, 1ull);
        __syncthreads();
        const unsigned long long it_v = item_sh;
        __syncthreads();
        const int64_t it = (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(it_v >> 32)) << 32) |
                                     (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)it_v));
        if (it >= n_items) break;
        block_work<NP, F64>(a, it >> k, (int)(it & ((1 << k) - 1)), tab32);
    }
}

// Fixed-order sum of the 2^k partials of a device-sized evaluation into
// out[0, m); the grid covers the largest possible m.
__global__ __launch_bounds__(kBlock) void k_sum_devsized(const double* __restrict__ part, const int64_t* m_ptr,
                                                         int np, int64_t want_waves, int64_t part_cap,
                                                         double* __restrict__ out) {
    const int64_t m = *m_ptr;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    const int S = 1 << devsized_k(m, np, want_waves, part_cap);
    double s = 0.0;
    for (int k = 0; k < S; ++k) s += part[(int64_t)k * m + i];
    out[i] = s;
}

__global__ void k_reset_counter(unsigned long long* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0ull;
}

// Fixed-order sum of the split partials of several instances: grid.y is the
// instance, grid.x covers its points.
__global__ __launch_bounds__(kBlock) void k_sum_splits_multi(const SumDesc* __restrict__ d) {
    const SumDesc q = d[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= q.n) return;
    double s = 0.0;
    for (int k = 0; k < q.S; ++k) s += q.part[(int64_t)k * q.n + i];
    q.out[i] = s;
}

// Box of an unsplit segment (one workgroup per segment): the smallest and
// largest pair (or cluster) centre coordinates and the largest stored r2far
// (a cluster record stores the largest of its members').  Empty segments get
// r2far max = +inf (never all far).
__global__ __launch_bounds__(kBlock) void k_segment_boxes(const Segment* __restrict__ segs,
                                                          const uint32_t* __restrict__ rec, int fp64,
                                                          double* __restrict__ boxes) {
    __shared__ double red[7][kBlock];
    const Segment sg = segs[blockIdx.x];
    const bool pairs = sg.n_pairs > 0;
    const bool cl = (sg.flags & kSegCluster) != 0;
    double v[7] = {HUGE_VAL, HUGE_VAL, HUGE_VAL, -HUGE_VAL, -HUGE_VAL, -HUGE_VAL, 0.0};
    if (pairs) {
        // centre: doubles 0-2 of every record; r2far: double 3 (FP64) or
        // float word 6 (FP32C), in pair and cluster records alike
        const int rw = cl ? (fp64 ? cl64_words(sg.L) : cl32_words(sg.L)) : (fp64 ? rec64_words(sg.L) : rec32_words(sg.L));
        for (int i = threadIdx.x; i < sg.n_pairs; i += kBlock) {
            const uint32_t* r = rec + sg.rec_off + (int64_t)i * rw;
            const double* rd = reinterpret_cast<const double*>(r);
            const double r2f = fp64 ? rd[3] : (double)reinterpret_cast<const float*>(r)[6];
            for (int d = 0; d < 3; ++d) {
                v[d] = fmin(v[d], rd[d]);
                v[3 + d] = fmax(v[3 + d], rd[d]);
            }
            v[6] = fmax(v[6], r2f);
        }
    }
    for (int d = 0; d < 7; ++d) red[d][threadIdx.x] = v[d];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int d = 0; d < 3; ++d) red[d][threadIdx.x] = fmin(red[d][threadIdx.x], red[d][threadIdx.x + w]);
            for (int d = 3; d < 7; ++d) red[d][threadIdx.x] = fmax(red[d][threadIdx.x], red[d][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x < kSegBoxWords) {
        double o = 0.0;
        if (threadIdx.x < 6) o = red[threadIdx.x][0];
        else if (threadIdx.x == 6) o = pairs ? red[6][0] : HUGE_VAL;
        boxes[(int64_t)blockIdx.x * kSegBoxWords + threadIdx.x] = o;
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

int launch_persistent(const BatchArgs& b, int grid, int precision, int np, void* stream) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, b.counter);
    if (precision == ENV_PREC_FP64) {
        if (np == 2) hipLaunchKernelGGL((k_potential_persistent<2, true>), dim3(grid), dim3(kBlock), 0, st, b);
        else hipLaunchKernelGGL((k_potential_persistent<1, true>), dim3(grid), dim3(kBlock), 0, st, b);
    } else {
        if (np == 1) hipLaunchKernelGGL((k_potential_persistent<1, false>), dim3(grid), dim3(kBlock), 0, st, b);
        else if (np == 2) hipLaunchKernelGGL((k_potential_persistent<2, false>), dim3(grid), dim3(kBlock), 0, st, b);
        else hipLaunchKernelGGL((k_potential_persistent<4, false>), dim3(grid), dim3(kBlock), 0, st, b);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int devsized_klog(int64_t m, int np, int64_t want_waves, int64_t part_cap) {
    return devsized_k(m, np, want_waves, part_cap);
}

int devsized_grid(int precision, int cu_count) {
    int per_cu = 0;
    const hipError_t e =
        precision == ENV_PREC_FP64
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_potential_devsized<2, true>, kBlock, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_potential_devsized<4, false>, kBlock, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    return per_cu * cu_count;
}

int launch_potential_devsized(const DevSizedArgs& d, int grid, int precision, int np, void* stream) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(64), 0, st, d.counter);
    if (precision == ENV_PREC_FP64) {
        if (np != 2) return -1;
        hipLaunchKernelGGL((k_potential_devsized<2, true>), dim3(grid), dim3(kBlock), 0, st, d);
    } else {
        if (np != 4) return -1;
        hipLaunchKernelGGL((k_potential_devsized<4, false>), dim3(grid), dim3(kBlock), 0, st, d);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_sum_devsized(const DevSizedArgs& d, int np, int64_t n_max, double* out, void* stream) {
    if (n_max <= 0) return 0;
    const dim3 grid((unsigned)((n_max + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_sum_devsized, grid, dim3(kBlock), 0, static_cast<hipStream_t>(stream), d.a.out, d.m, np,
                       d.want_waves, d.part_cap, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int persistent_grid(int precision, int np, int cu_count) {
    int per_cu = 0;
    hipError_t e;
    if (precision == ENV_PREC_FP64)
        e = np == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_potential_persistent<2, true>, kBlock, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_potential_persistent<1, true>, kBlock, 0);
    else
        e = np == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_potential_persistent<1, false>, kBlock, 0)
          : np == 2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_potential_persistent<2, false>, kBlock, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_potential_persistent<4, false>, kBlock, 0);
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    return per_cu * cu_count;
}

int launch_sum_multi(const SumDesc* d, int n_desc, int64_t max_n, void* stream) {
    if (n_desc <= 0) return 0;
    const dim3 grid((unsigned)((max_n + kBlock - 1) / kBlock), (unsigned)n_desc);
    hipLaunchKernelGGL(k_sum_splits_multi, grid, dim3(kBlock), 0, static_cast<hipStream_t>(stream), d);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_segment_boxes(const Segment* segs, int n_segs, const uint32_t* rec, int fp64, double* boxes,
                         void* stream) {
    if (n_segs <= 0) return 0;
    hipLaunchKernelGGL(k_segment_boxes, dim3((unsigned)n_segs), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                       segs, rec, fp64, boxes);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_sum_splits(const double* partial, int S, int64_t n, double* out, void* stream) {
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_sum_splits, grid, dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                       partial, S, n, out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace envpot
