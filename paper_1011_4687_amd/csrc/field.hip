// gfx950 kernel of the environment's electric field E = -grad V together
// with V, on the potential's pair records, clusters and segments.
//
// With X = P - C the Hermite integrals R_tuv are derivatives with respect to
// the pair centre P, so the gradient of a pair's potential with respect to
// the point C is minus (R_{t+1,u,v}, R_{t,u+1,v}, R_{t,u,v+1}) contracted with
// the pair's Hermite density: the same recursion run one order further, with
// Boys values F_0 .. F_{L+1}.  In the far field the pair is the finite
// multipole (1/R) H(x), x = X/R^2, and its gradient follows from H and dH:
//     d/dX_i [H(x)/R] = (w/R) (dH/dx_i - X_i (H + 2 x.dH)),   w = 1/R^2
// (x.dH = sum_k k H_k by Euler's theorem on the homogeneous parts H_k, and
// sum_k (2k+1) H_k = H + 2 x.dH).  The far radius of the field is the one
// where the Boys asymptote holds for F_0 .. F_{L+1}, the pair's potential
// radius times a fixed ratio per L.
//
// Layout of the work as in the potential kernel: every lane owns NP points,
// the wave walks the pair list of its split with scalar loads, same-centre
// clusters are evaluated once per wave while no point is inside their
// radius, and per fragment group the (electronic - nuclear) sums of V and
// of the gradient are folded into the FP64 result.  FP32C: X rounded once
// from the exact FP64 difference, FP32 arithmetic, FP32 sums over tiles of
// pairs promoted to FP64.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_math.h"
#include "envpot_internal.h"
#include "field_gen.h"
#include "field_internal.h"

namespace envpot {
namespace {

constexpr int kFTile = 8;  // pairs per FP32 partial sum

template <int L, typename T>
__device__ __forceinline__ void near_dot(const T* G, T X, T Y, T Z, const T* __restrict__ D, T* o) {
    if constexpr (L == 0) hermite_field_L0<T>(G, X, Y, Z, D, o);
    else if constexpr (L == 1) hermite_field_L1<T>(G, X, Y, Z, D, o);
    else if constexpr (L == 2) hermite_field_L2<T>(G, X, Y, Z, D, o);
    else if constexpr (L == 3) hermite_field_L3<T>(G, X, Y, Z, D, o);
    else hermite_field_L4<T>(G, X, Y, Z, D, o);
}

template <int L, typename T>
__device__ __forceinline__ void far_poly(const T* __restrict__ h, T x, T y, T z, T* o) {
    if constexpr (L == 0) far_field_L0<T>(h, x, y, z, o);
    else if constexpr (L == 1) far_field_L1<T>(h, x, y, z, o);
    else if constexpr (L == 2) far_field_L2<T>(h, x, y, z, o);
    else if constexpr (L == 3) far_field_L3<T>(h, x, y, z, o);
    else far_field_L4<T>(h, x, y, z, o);
}

__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Far-field potential and gradient (with respect to X) at X = P - C, added
// to a[0..3]; ri = 1/R.  With t = ri w and W = H + 2 x.dH:
//     a0 += ri H,   a_i += t dH_i - t W X_i.
// L = 0: dH = 0, W = H = h0.  L = 1: H = h0 + w s with s = h.X (the degree-1
// coefficients), dH = those coefficients, x.dH = w s, so W = h0 + 3 w s and
// no scaled coordinates are needed.
template <int L, typename T>
__device__ __forceinline__ void far_acc(const T* __restrict__ h, T X, T Y, T Z, T ri, T* a) {
    const T w = ri * ri;
    const T t = ri * w;
    if constexpr (L == 0) {
        a[0] = fmat(ri, h[0], a[0]);
        const T tw = t * h[0];
        a[1] = fmat(-tw, X, a[1]);
        a[2] = fmat(-tw, Y, a[2]);
        a[3] = fmat(-tw, Z, a[3]);
    } else if constexpr (L == 1) {
        // component order (0,0,0), (0,0,1), (0,1,0), (1,0,0)
        const T ws = w * fmat(h[1], Z, fmat(h[2], Y, h[3] * X));
        const T tw = t * fmat(T(3), ws, h[0]);
        a[0] = fmat(ri, h[0] + ws, a[0]);
        a[1] = fmat(-tw, X, fmat(t, h[3], a[1]));
        a[2] = fmat(-tw, Y, fmat(t, h[2], a[2]));
        a[3] = fmat(-tw, Z, fmat(t, h[1], a[3]));
    } else {
        const T x = X * w, y = Y * w, z = Z * w;
        T f[4];
        far_poly<L, T>(h, x, y, z, f);
        const T tw = t * fmat(T(2), fmat(x, f[1], fmat(y, f[2], z * f[3])), f[0]);
        a[0] = fmat(ri, f[0], a[0]);
        a[1] = fmat(-tw, X, fmat(t, f[1], a[1]));
        a[2] = fmat(-tw, Y, fmat(t, f[2], a[2]));
        a[3] = fmat(-tw, Z, fmat(t, f[3], a[3]));
    }
}

// Near field (FP32): Boys F_0..F_{L+1} by a 6-term Taylor step from the
// field table in LDS, then the recursion to order L+1.
template <int L>
__device__ __forceinline__ void near_f32(const GLB uint32_t* __restrict__ r, float X, float Y, float Z,
                                         float r2, const float* tab, float* o) {
    const GLB float* rf = reinterpret_cast<const GLB float*>(r + 6);
    const float p = rf[1], c1 = rf[2];
    float D[kNComp[L]];
#pragma unroll
    for (int c = 0; c < kNComp[L]; ++c) D[c] = rf[3 + kNComp[L] + c];
    const float T = p * r2;
    const int kk = (int)__builtin_fmaf(T, (float)kBoysGridInv, 0.5f);
    const float d = __builtin_fmaf((float)kk, -1.0f / kBoysGridInv, T);
    const float* f = tab + kk * kFieldRowF32;
    const float d2 = 0.5f * d, d3 = d * (1.0f / 3.0f), d4 = 0.25f * d, d5 = 0.2f * d;
    const float m2p = -2.0f * p;
    float s = c1;
    float G[L + 2];
#pragma unroll
    for (int n = 0; n <= L + 1; ++n) {
        float F = __builtin_fmaf(-d5, f[n + 5], f[n + 4]);
        F = __builtin_fmaf(-d4, F, f[n + 3]);
        F = __builtin_fmaf(-d3, F, f[n + 2]);
        F = __builtin_fmaf(-d2, F, f[n + 1]);
        F = __builtin_fmaf(-d, F, f[n]);
        G[n] = s * F;
        s *= m2p;
    }
    near_dot<L, float>(G, X, Y, Z, D, o);
}

template <int L>
__device__ __forceinline__ void near_f64(const GLB uint32_t* __restrict__ r, double X, double Y, double Z,
                                         double r2, const GLB double* __restrict__ tab, double* o) {
    const GLB double* rd = reinterpret_cast<const GLB double*>(r);
    const double p = rd[4], c1 = rd[5];
    double D[kNComp[L]];
#pragma unroll
    for (int c = 0; c < kNComp[L]; ++c) D[c] = rd[kRec64Head + kNComp[L] + c];
    const double T = p * r2;
    const int kk = (int)__builtin_fma(T, (double)kBoysGridInv, 0.5);
    const double d = __builtin_fma((double)kk, -1.0 / kBoysGridInv, T);
    const GLB double* f = tab + kk * kFieldRowF64;
    double dj[kBoysTaylorF64];
#pragma unroll
    for (int j = 1; j < kBoysTaylorF64; ++j) dj[j] = d * (1.0 / j);
    const double m2p = -2.0 * p;
    double s = c1;
    double G[L + 2];
#pragma unroll
    for (int n = 0; n <= L + 1; ++n) {
        double F = f[n + kBoysTaylorF64 - 1];
#pragma unroll
        for (int j = kBoysTaylorF64 - 1; j >= 1; --j) F = __builtin_fma(-dj[j], F, f[n + j - 1]);
        G[n] = s * F;
        s *= m2p;
    }
    near_dot<L, double>(G, X, Y, Z, D, o);
}

// FP32C pairs of one L; ge[k] += (v, g) of every pair at point k.
// The part of a pair record the far field needs.
template <int L>
struct FHead {
    double px, py, pz;
    float r2far;
    float h[kNComp[L]];
};

template <int L>
__device__ __forceinline__ void load_fhead(const GLB uint32_t* __restrict__ r, FHead<L>& o) {
    const GLB double* rd = reinterpret_cast<const GLB double*>(r);
    const GLB float* rf = reinterpret_cast<const GLB float*>(r + 6);
    o.px = rd[0];
    o.py = rd[1];
    o.pz = rd[2];
    o.r2far = rf[0];
#pragma unroll
    for (int c = 0; c < kNComp[L]; ++c) o.h[c] = rf[3 + c];
}

// Prefetch the next head while two heads fit in SGPRs (L <= 2).
template <int L>
constexpr bool kFPipelined = L <= 2;

// FAR: every point-pair of the run is in the field's far region (segment
// box test): no near test.  X stays the rounded exact difference: at two
// points per lane the potential kernel's wave-origin form would cost as many
// instructions per pair as it saves.
template <int L, int NP, bool FAR>
__device__ __forceinline__ void pairs_f32(const GLB uint32_t* __restrict__ rec, int npairs, const double* cx,
                                          const double* cy, const double* cz, const float* tab, float ratio,
                                          double (*ge)[4]) {
    constexpr int RW = rec32_words(L);
    if (npairs <= 0) return;
    FHead<L> cur;
    if constexpr (kFPipelined<L>) load_fhead<L>(rec, cur);
    for (int i0 = 0; i0 < npairs; i0 += kFTile) {
        const int i1 = min(i0 + kFTile, npairs);
        float t[NP][4];
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) t[k][c] = 0.0f;
        for (int i = i0; i < i1; ++i) {
            const GLB uint32_t* r = rec + (int64_t)i * RW;
            FHead<L> nxt;
            if constexpr (kFPipelined<L>) load_fhead<L>(rec + (int64_t)min(i + 1, npairs - 1) * RW, nxt);
            else load_fhead<L>(r, cur);
            const double px = cur.px, py = cur.py, pz = cur.pz;
            const float r2f = cur.r2far * ratio;
            const float* h = cur.h;
            float X[NP], Y[NP], Z[NP], r2[NP];
            bool nearp = false;
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                X[k] = (float)(px - cx[k]);
                Y[k] = (float)(py - cy[k]);
                Z[k] = (float)(pz - cz[k]);
                r2[k] = __builtin_fmaf(X[k], X[k], __builtin_fmaf(Y[k], Y[k], Z[k] * Z[k]));
                nearp |= r2[k] < r2f;
            }
            if (FAR || __builtin_amdgcn_ballot_w64(nearp) == 0) {
#pragma unroll
                for (int k = 0; k < NP; ++k) far_acc<L, float>(h, X[k], Y[k], Z[k], rsqrt_refined(r2[k]), t[k]);
            } else {
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    if (r2[k] < r2f) {
                        float o[4];
                        near_f32<L>(r, X[k], Y[k], Z[k], r2[k], tab, o);
#pragma unroll
                        for (int c = 0; c < 4; ++c) t[k][c] += o[c];
                    } else {
                        far_acc<L, float>(h, X[k], Y[k], Z[k], rsqrt_refined(r2[k]), t[k]);
                    }
                }
            }
            if constexpr (kFPipelined<L>) cur = nxt;
        }
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) ge[k][c] += (double)t[k][c];
    }
}

template <int L>
struct FHead64 {
    double px, py, pz, r2far;
    double h[kNComp[L]];
};

template <int L>
__device__ __forceinline__ void load_fhead64(const GLB uint32_t* __restrict__ r, FHead64<L>& o) {
    const GLB double* rd = reinterpret_cast<const GLB double*>(r);
    o.px = rd[0];
    o.py = rd[1];
    o.pz = rd[2];
    o.r2far = rd[3];
#pragma unroll
    for (int c = 0; c < kNComp[L]; ++c) o.h[c] = rd[kRec64Head + c];
}

// FAR: every point-pair of the run is in the field's far region (segment
// box test): no near test.
template <int L, int NP, bool FAR>
__device__ __forceinline__ void pairs_f64(const GLB uint32_t* __restrict__ rec, int npairs, const double* cx,
                                          const double* cy, const double* cz, const GLB double* __restrict__ tab,
                                          double ratio, double (*ge)[4]) {
    constexpr int RW = rec64_words(L);
    constexpr bool kPipe = L <= 1;  // two FP64 heads fit in SGPRs
    if (npairs <= 0) return;
    FHead64<L> cur;
    if constexpr (kPipe) load_fhead64<L>(rec, cur);
    for (int i = 0; i < npairs; ++i) {
        const GLB uint32_t* r = rec + (int64_t)i * RW;
        FHead64<L> nxt;
        if constexpr (kPipe) load_fhead64<L>(rec + (int64_t)min(i + 1, npairs - 1) * RW, nxt);
        else load_fhead64<L>(r, cur);
        const double px = cur.px, py = cur.py, pz = cur.pz;
        const double r2f = cur.r2far * ratio;
        const double* h = cur.h;
        double X[NP], Y[NP], Z[NP], r2[NP];
        bool nearp = false;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            X[k] = px - cx[k];
            Y[k] = py - cy[k];
            Z[k] = pz - cz[k];
            r2[k] = __builtin_fma(X[k], X[k], __builtin_fma(Y[k], Y[k], Z[k] * Z[k]));
            nearp |= r2[k] < r2f;
        }
        if (FAR || __builtin_amdgcn_ballot_w64(nearp) == 0) {
#pragma unroll
            for (int k = 0; k < NP; ++k) far_acc<L, double>(h, X[k], Y[k], Z[k], rsqrt_far(r2[k]), ge[k]);
        } else {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                if (r2[k] < r2f) {
                    double o[4];
                    near_f64<L>(r, X[k], Y[k], Z[k], r2[k], tab, o);
#pragma unroll
                    for (int c = 0; c < 4; ++c) ge[k][c] += o[c];
                } else {
                    far_acc<L, double>(h, X[k], Y[k], Z[k], rsqrt_far(r2[k]), ge[k]);
                }
            }
        }
        if constexpr (kPipe) cur = nxt;
    }
}

// Same-centre clusters of merged L = LC from cluster i on, while no point of
// the wave is inside a cluster's field radius; returns the index of the
// first cluster with a point inside (n when none).
template <int LC, int NP, bool F64>
__device__ __forceinline__ int clusters(const GLB uint32_t* __restrict__ rec, int i, int n, const double* cx,
                                        const double* cy, const double* cz, double ratio, double (*ge)[4]) {
    using T = typename std::conditional<F64, double, float>::type;
    constexpr int CW = F64 ? cl64_words(LC) : cl32_words(LC);
    // FP32: partial sums over kFTile clusters, promoted to FP64
    T tile[NP][4];
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) tile[k][c] = T(0);
    int done = 0;
    for (; i < n; ++i) {
        const GLB uint32_t* r = rec + (int64_t)i * CW;
        const GLB double* rd = reinterpret_cast<const GLB double*>(r);
        const double px = rd[0], py = rd[1], pz = rd[2];
        T r2f;
        T h[kNComp[LC]];
        if constexpr (F64) {
            r2f = rd[3] * ratio;
#pragma unroll
            for (int c = 0; c < kNComp[LC]; ++c) h[c] = rd[kClHead64 + c];
        } else {
            const GLB float* rf = reinterpret_cast<const GLB float*>(r);
            r2f = rf[6] * (float)ratio;
#pragma unroll
            for (int c = 0; c < kNComp[LC]; ++c) h[c] = rf[kClHead32 + c];
        }
        T X[NP], Y[NP], Z[NP], r2[NP];
        bool nearp = false;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            X[k] = (T)(px - cx[k]);
            Y[k] = (T)(py - cy[k]);
            Z[k] = (T)(pz - cz[k]);
            r2[k] = fmat(X[k], X[k], fmat(Y[k], Y[k], Z[k] * Z[k]));
            nearp |= r2[k] < r2f;
        }
        if (__builtin_amdgcn_ballot_w64(nearp) != 0) break;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            if constexpr (F64) far_acc<LC, double>(h, X[k], Y[k], Z[k], rsqrt_far(r2[k]), tile[k]);
            else far_acc<LC, float>(h, X[k], Y[k], Z[k], rsqrt_refined(r2[k]), tile[k]);
        }
        if ((++done & (kFTile - 1)) == 0) {
#pragma unroll
            for (int k = 0; k < NP; ++k)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    ge[k][c] += (double)tile[k][c];
                    tile[k][c] = T(0);
                }
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int c = 0; c < 4; ++c) ge[k][c] += (double)tile[k][c];
    return i;
}

template <int NP, bool F64>
__device__ __forceinline__ int clusters_any(int lc, const GLB uint32_t* __restrict__ rec, int i, int n,
                                            const double* cx, const double* cy, const double* cz, double ratio,
                                            double (*ge)[4]) {
    switch (lc) {
        case 0: return clusters<0, NP, F64>(rec, i, n, cx, cy, cz, ratio, ge);
        case 1: return clusters<1, NP, F64>(rec, i, n, cx, cy, cz, ratio, ge);
        case 2: return clusters<2, NP, F64>(rec, i, n, cx, cy, cz, ratio, ge);
        case 3: return clusters<3, NP, F64>(rec, i, n, cx, cy, cz, ratio, ge);
        default: return clusters<4, NP, F64>(rec, i, n, cx, cy, cz, ratio, ge);
    }
}

// One workgroup's share: the points of point block `pblock` against the
// pair range of split `s`.
template <int NP, bool F64>
__device__ __forceinline__ void field_block(const PTS double* __restrict__ pts, int64_t n,
                                            const GLB Segment* __restrict__ segs,
                                            const GLB int32_t* __restrict__ split,
                                            const GLB uint32_t* __restrict__ recs,
                                            const GLB double* __restrict__ nuc,
                                            const GLB double* __restrict__ boys64,
                                            const GLB double* __restrict__ boxes, const FieldParams& fp,
                                            double* __restrict__ out, int64_t pblock, int s, const float* tab32) {
    const int64_t base = pblock * (kBlock * NP) + threadIdx.x;
    double cx[NP], cy[NP], cz[NP], acc[NP][4], ge[NP][4];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int64_t i = base + (int64_t)k * kBlock;
        const int64_t ic = i < n ? i : n - 1;  // ragged tail: recompute the last point
        cx[k] = pts[3 * ic];
        cy[k] = pts[3 * ic + 1];
        cz[k] = pts[3 * ic + 2];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[k][c] = ge[k][c] = 0.0;
    }
    const double cl_ratio = F64 ? fp.cl_ratio64 : (double)fp.cl_ratio32;
    const int sb = split[s], se = split[s + 1];
    int g = sb;
    bool fold = false;
    const GLB uint32_t* crec = recs;  // cluster segment in progress: clusters [ci, cn) of merged L lc
    int ci = 0, cn = 0, lc = 0;
    const GLB uint32_t* mtab = recs;  // member table of the cluster being expanded
    uint32_t pend = 0;                // its member runs (bit L) not yet evaluated
    for (;;) {
        int L, npairs;
        const GLB uint32_t* rec;
        bool all_far = false;  // member runs: tested pair by pair
        if (pend != 0) {
            L = __builtin_ctz(pend);
            pend &= pend - 1;
            rec = recs + mtab[2 * L];
            npairs = (int)mtab[2 * L + 1];
        } else if (ci < cn) {
            ci = clusters_any<NP, F64>(lc, crec, ci, cn, cx, cy, cz, cl_ratio, ge);
            if (ci < cn) {
                const GLB uint32_t* c = crec + (int64_t)ci * (F64 ? cl64_words(lc) : cl32_words(lc));
                mtab = c + (F64 ? kClTable64 : kClTable32);
                pend = c[F64 ? kClMask64 : kClMask32];
                ++ci;
            }
            continue;
        } else {
            if (fold) {
#pragma unroll
                for (int k = 0; k < NP; ++k)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        acc[k][c] -= ge[k][c];
                        ge[k][c] = 0.0;
                    }
                fold = false;
            }
            if (g >= se) break;
            const GLB Segment* sp = segs + g;
            ++g;
            const int sL = sp->L, sn = sp->n_pairs, nb = sp->nuc_begin, ne = sp->nuc_end, sf = sp->flags;
            const int64_t so = sp->rec_off;
            // nuclei: ge collects (electronic - nuclear) of V and of the gradient
            for (int q = nb; q < ne; ++q) {
                const double qx = nuc[4 * q], qy = nuc[4 * q + 1], qz = nuc[4 * q + 2], qZ = nuc[4 * q + 3];
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const double dx = cx[k] - qx, dy = cy[k] - qy, dz = cz[k] - qz;
                    const double ri = rsqrt(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)));
                    const double zr = qZ * ri, f = zr * ri * ri;
                    ge[k][0] -= zr;
                    ge[k][1] -= f * dx;
                    ge[k][2] -= f * dy;
                    ge[k][3] -= f * dz;
                }
            }
            fold = (sf & kSegEndGroup) != 0;
            if (sf & kSegCluster) {
                crec = recs + so;
                ci = 0;
                cn = sn;
                lc = sL;
                continue;
            }
            L = sL;
            rec = recs + so;
            npairs = sn;
            // segment box test: every point of the wave beyond the largest
            // field radius of the segment's pairs (r2far max times the
            // field's ratio for L)
            if (boxes && npairs > 0) {
                const GLB double* bx = boxes + (int64_t)kSegBoxWords * sp->box;
                const double lim = bx[6] * (F64 ? fp.ratio64[L] : (double)fp.ratio32[L]) * (1.0 + 1e-6);
                bool nearp = false;
#pragma unroll
                for (int k = 0; k < NP; ++k) {
                    const double gx = fmax(0.0, fmax(bx[0] - cx[k], cx[k] - bx[3]));
                    const double gy = fmax(0.0, fmax(bx[1] - cy[k], cy[k] - bx[4]));
                    const double gz = fmax(0.0, fmax(bx[2] - cz[k], cz[k] - bx[5]));
                    nearp |= __builtin_fma(gx, gx, __builtin_fma(gy, gy, gz * gz)) < lim;
                }
                all_far = __builtin_amdgcn_ballot_w64(nearp) == 0;
            }
        }
        if constexpr (F64) {
            if (all_far) {
                switch (L) {
                    case 0: pairs_f64<0, NP, true>(rec, npairs, cx, cy, cz, boys64, fp.ratio64[0], ge); break;
                    case 1: pairs_f64<1, NP, true>(rec, npairs, cx, cy, cz, boys64, fp.ratio64[1], ge); break;
                    case 2: pairs_f64<2, NP, true>(rec, npairs, cx, cy, cz, boys64, fp.ratio64[2], ge); break;
                    case 3: pairs_f64<3, NP, true>(rec, npairs, cx, cy, cz, boys64, fp.ratio64[3], ge); break;
                    default: pairs_f64<4, NP, true>(rec, npairs, cx, cy, cz, boys64, fp.ratio64[4], ge); break;
                }
            } else {
                switch (L) {
                    case 0: pairs_f64<0, NP, false>(rec, npairs, cx, cy, cz, boys64, fp.ratio64[0], ge); break;
                    case 1: pairs_f64<1, NP, false>(rec, npairs, cx, cy, cz, boys64, fp.ratio64[1], ge); break;
                    case 2: pairs_f64<2, NP, false>(rec, npairs, cx, cy, cz, boys64, fp.ratio64[2], ge); break;
                    case 3: pairs_f64<3, NP, false>(rec, npairs, cx, cy, cz, boys64, fp.ratio64[3], ge); break;
                    default: pairs_f64<4, NP, false>(rec, npairs, cx, cy, cz, boys64, fp.ratio64[4], ge); break;
                }
            }
        } else {
            if (all_far) {
                switch (L) {
                    case 0: pairs_f32<0, NP, true>(rec, npairs, cx, cy, cz, tab32, fp.ratio32[0], ge); break;
                    case 1: pairs_f32<1, NP, true>(rec, npairs, cx, cy, cz, tab32, fp.ratio32[1], ge); break;
                    case 2: pairs_f32<2, NP, true>(rec, npairs, cx, cy, cz, tab32, fp.ratio32[2], ge); break;
                    case 3: pairs_f32<3, NP, true>(rec, npairs, cx, cy, cz, tab32, fp.ratio32[3], ge); break;
                    default: pairs_f32<4, NP, true>(rec, npairs, cx, cy, cz, tab32, fp.ratio32[4], ge); break;
                }
            } else {
                switch (L) {
                    case 0: pairs_f32<0, NP, false>(rec, npairs, cx, cy, cz, tab32, fp.ratio32[0], ge); break;
                    case 1: pairs_f32<1, NP, false>(rec, npairs, cx, cy, cz, tab32, fp.ratio32[1], ge); break;
                    case 2: pairs_f32<2, NP, false>(rec, npairs, cx, cy, cz, tab32, fp.ratio32[2], ge); break;
                    case 3: pairs_f32<3, NP, false>(rec, npairs, cx, cy, cz, tab32, fp.ratio32[3], ge); break;
                    default: pairs_f32<4, NP, false>(rec, npairs, cx, cy, cz, tab32, fp.ratio32[4], ge); break;
                }
            }
        }
    }
    // V = nuclear - electronic; E = -grad V = nuclear field - (electronic gradient)
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int64_t i = base + (int64_t)k * kBlock;
        if (i < n) {
            double* o = out + ((int64_t)s * n + i) * 4;
#pragma unroll
            for (int c = 0; c < 4; ++c) o[c] = acc[k][c] - ge[k][c];
        }
    }
}

// Four waves per SIMD (128 VGPRs): the per-point state and the near-field
// recursion spill to scratch, which costs less than the latency that two
// or three resident waves leave exposed.
template <int NP, bool F64>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_field(FieldArgs a) {
    __shared__ float tab32[F64 ? 1 : kFieldMaxRowsF32 * kFieldRowF32];
    if constexpr (!F64) {
        const float* g = static_cast<const float*>(a.boys);
        for (int i = threadIdx.x; i < a.fp.rows32 * kFieldRowF32; i += kBlock) tab32[i] = g[i];
        __syncthreads();
    }
    field_block<NP, F64>(gpts(a.pts), a.n, glb(a.segs), glb(a.split), glb(a.rec), glb(a.nuc),
                         glb(static_cast<const double*>(a.boys)), glb(a.boxes), a.fp, a.out, blockIdx.x,
                         blockIdx.y, tab32);
}

}  // namespace

int launch_field(const FieldArgs& a, int S, int precision, int np, void* stream) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t per = (int64_t)kBlock * np;
    const dim3 grid((unsigned)((a.n + per - 1) / per), (unsigned)S);
    const dim3 block(kBlock);
    if (precision == ENV_PREC_FP64) {
        if (np == 2) hipLaunchKernelGGL((k_field<2, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_field<1, true>), grid, block, 0, st, a);
    } else {
        if (np == 2) hipLaunchKernelGGL((k_field<2, false>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((k_field<1, false>), grid, block, 0, st, a);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace envpot
