// gfx950 kernels of the incremental density update: every pair's Hermite
// density D (McMurchie-Davidson fold of the density block with the
// primitives' normalised coefficients and the Hermite expansion
// coefficients E^{ij}_t of the Gaussian product), its far-field
// coefficients h = M_L D, and the same-centre clusters' merged h, written
// into the handle's records in place.  One thread per pair (or cluster).
#include <hip/hip_runtime.h>

#include "envpot_internal.h"
#include "update_internal.h"

namespace envpot {
namespace {

constexpr int kUpdBlock = 256;

// Hermite expansion coefficients of one direction,
//   x_A^i x_B^j exp(-a x_A^2 - b x_B^2) = sum_t E[i][j][t] Lambda_t(x; p, P),
// raised first in j along i = 0, then in i:
//   E^{i,j+1}_t = E^{ij}_{t-1}/(2p) + X_PB E^{ij}_t + (t+1) E^{ij}_{t+1}   (likewise i with X_PA)
struct Edir {
    double v[3][3][5];
};

__device__ __forceinline__ double eget(const Edir& E, int i, int j, int t) {
    return (t < 0 || t > i + j) ? 0.0 : E.v[i][j][t];
}

__device__ void hermite_E(int li, int lj, double a, double b, double A, double B, Edir& E) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int t = 0; t < 5; ++t) E.v[i][j][t] = 0.0;
    const double p = a + b, P = (a * A + b * B) / p;
    const double xpa = P - A, xpb = P - B, h = 0.5 / p, dab = A - B;
    E.v[0][0][0] = exp(-(a * b / p) * dab * dab);
    for (int j = 0; j < lj; ++j)
        for (int t = 0; t <= j + 1; ++t)
            E.v[0][j + 1][t] = h * eget(E, 0, j, t - 1) + xpb * eget(E, 0, j, t) + (t + 1) * eget(E, 0, j, t + 1);
    for (int i = 0; i < li; ++i)
        for (int j = 0; j <= lj; ++j)
            for (int t = 0; t <= i + j + 1; ++t)
                E.v[i + 1][j][t] = h * eget(E, i, j, t - 1) + xpa * eget(E, i, j, t) + (t + 1) * eget(E, i, j, t + 1);
}

// Cartesian exponents of component c of a shell of angular momentum l
// (x-major: p = x, y, z; d = xx, xy, xz, yy, yz, zz).
__device__ __forceinline__ void cart(int l, int c, int e[3]) {
    const int tab[10][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                            {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
    const int base = l == 0 ? 0 : (l == 1 ? 1 : 4);
    for (int d = 0; d < 3; ++d) e[d] = tab[base + c][d];
}

// Index of Hermite component (t, u, v) among t + u + v <= L (t, then u, then v ascending).
__device__ __forceinline__ int hidx(int L, int t, int u, int v) {
    int idx = 0;
    for (int a = 0; a < t; ++a) {
        const int m = L - a;
        idx += (m + 1) * (m + 2) / 2;
    }
    const int m = L - t;
    for (int b = 0; b < u; ++b) idx += m - b + 1;
    return idx + v;
}

struct PairGeo {
    int lI, lJ, nI, nJ;
    double a, b, p, w2;
    const double* na;  // c N per component of primitive ia
    const double* nb;
    const double* W;   // the block's nI x nJ weights
    Edir Ex, Ey, Ez;
};

__device__ void pair_geometry(const UpdateArgs& A, const UpdPair& q, PairGeo& g) {
    const int I = A.blk[2 * q.blk], J = A.blk[2 * q.blk + 1];
    const UpdShell& SI = A.shells[I];
    const UpdShell& SJ = A.shells[J];
    g.lI = SI.l;
    g.lJ = SJ.l;
    g.nI = (g.lI + 1) * (g.lI + 2) / 2;
    g.nJ = (g.lJ + 1) * (g.lJ + 2) / 2;
    g.a = A.exps[SI.poff + q.ia];
    g.b = A.exps[SJ.poff + q.ib];
    g.p = g.a + g.b;
    g.w2 = (I == J && q.ia != q.ib) ? 2.0 : 1.0;
    g.na = A.cnorm + SI.noff + int64_t(q.ia) * g.nI;
    g.nb = A.cnorm + SJ.noff + int64_t(q.ib) * g.nJ;
    g.W = A.W + A.woff[q.blk];
    hermite_E(g.lI, g.lJ, g.a, g.b, SI.A[0], SJ.A[0], g.Ex);
    hermite_E(g.lI, g.lJ, g.a, g.b, SI.A[1], SJ.A[1], g.Ey);
    hermite_E(g.lI, g.lJ, g.a, g.b, SI.A[2], SJ.A[2], g.Ez);
}

__device__ __forceinline__ double pp32(double p) {
    const double pp = 3.14159265358979323846 / p;
    return pp * sqrt(pp);
}

// D_tuv of one pair (unscaled by (pi/p)^{3/2}); returns L.
__device__ int fold_D(const PairGeo& g, double* D) {
    const int L = g.lI + g.lJ;
    const int nc = (L + 1) * (L + 2) * (L + 3) / 6;
    for (int k = 0; k < nc; ++k) D[k] = 0.0;
    for (int x = 0; x < g.nI; ++x) {
        int ei[3];
        cart(g.lI, x, ei);
        for (int y = 0; y < g.nJ; ++y) {
            const double pw = g.W[x * g.nJ + y];
            if (pw == 0.0) continue;
            int ej[3];
            cart(g.lJ, y, ej);
            const double f = g.w2 * pw * g.na[x] * g.nb[y];
            for (int t = 0; t <= ei[0] + ej[0]; ++t) {
                const double ft = f * g.Ex.v[ei[0]][ej[0]][t];
                for (int u = 0; u <= ei[1] + ej[1]; ++u) {
                    const double fu = ft * g.Ey.v[ei[1]][ej[1]][u];
                    for (int v = 0; v <= ei[2] + ej[2]; ++v) D[hidx(L, t, u, v)] += fu * g.Ez.v[ei[2]][ej[2]][v];
                }
            }
        }
    }
    return L;
}

// Electron count of a pair: the t = u = v = 0 part of the fold.
__global__ __launch_bounds__(kUpdBlock) void k_upd_charges(UpdateArgs A) {
    const int64_t i = int64_t(blockIdx.x) * kUpdBlock + threadIdx.x;
    if (i >= A.n_pairs + A.n_drop) return;
    PairGeo g;
    pair_geometry(A, A.pairs[i], g);
    double q = 0.0;
    for (int x = 0; x < g.nI; ++x) {
        int ei[3];
        cart(g.lI, x, ei);
        for (int y = 0; y < g.nJ; ++y) {
            const double pw = g.W[x * g.nJ + y];
            if (pw == 0.0) continue;
            int ej[3];
            cart(g.lJ, y, ej);
            q += g.w2 * pw * g.na[x] * g.nb[y] * g.Ex.v[ei[0]][ej[0]][0] * g.Ey.v[ei[1]][ej[1]][0] *
                 g.Ez.v[ei[2]][ej[2]][0];
        }
    }
    A.charge[i] = q * pp32(g.p);
}

// D and h of a pair, scaled by (pi/p)^{3/2} and its group's factor.
__device__ int pair_Dh(const UpdateArgs& A, const UpdPair& q, double* D, double* h) {
    PairGeo g;
    pair_geometry(A, q, g);
    const int L = fold_D(g, D);
    const int nc = (L + 1) * (L + 2) * (L + 3) / 6;
    const double sc = pp32(g.p), s = A.scale[q.group];
    for (int k = 0; k < nc; ++k) D[k] = (D[k] * sc) * s;
    const double* M = A.M + kFarMatOff[L];
    for (int i = 0; i < nc; ++i) {
        double acc = 0.0;
        for (int j = 0; j < nc; ++j) acc += M[i * nc + j] * D[j];
        h[i] = acc;
    }
    return L;
}

__global__ __launch_bounds__(kUpdBlock) void k_upd_pairs(UpdateArgs A) {
    const int64_t i = int64_t(blockIdx.x) * kUpdBlock + threadIdx.x;
    if (i >= A.n_pairs) return;
    const UpdPair q = A.pairs[i];
    double D[35], h[35];
    const int L = pair_Dh(A, q, D, h);
    const int nc = (L + 1) * (L + 2) * (L + 3) / 6;
    uint32_t* r = A.rec + q.word;
    if (A.fp64) {
        double* rd = reinterpret_cast<double*>(r);
        for (int c = 0; c < nc; ++c) rd[kRec64Head + c] = h[c];
        for (int c = 0; c < nc; ++c) rd[kRec64Head + nc + c] = D[c];
    } else {
        float* f = reinterpret_cast<float*>(r + 6);
        for (int c = 0; c < nc; ++c) f[3 + c] = float(h[c]);
        for (int c = 0; c < nc; ++c) f[3 + nc + c] = float(D[c]);
    }
}

// Far-field coefficients of every cluster member (FP64), for the merge.
__global__ __launch_bounds__(kUpdBlock) void k_upd_members(UpdateArgs A) {
    const int64_t m = int64_t(blockIdx.x) * kUpdBlock + threadIdx.x;
    if (m >= A.n_members) return;
    double D[35], h[35];
    const int L = pair_Dh(A, A.pairs[A.members[m]], D, h);
    const int nc = (L + 1) * (L + 2) * (L + 3) / 6;
    double* o = A.hm + A.moff[m];
    for (int i = 0; i < nc; ++i) o[i] = h[i];
}

// Merged far-field coefficients of a cluster: the members' h summed in FP64
// in member order at the cluster's L (same exponents (a, b, c), re-indexed).
__global__ __launch_bounds__(kUpdBlock) void k_upd_clusters(UpdateArgs A) {
    const int64_t c = int64_t(blockIdx.x) * kUpdBlock + threadIdx.x;
    if (c >= A.n_clusters) return;
    const UpdCluster cl = A.clusters[c];
    const int Lc = cl.L, ncc = (Lc + 1) * (Lc + 2) * (Lc + 3) / 6;
    double hsum[35];
    for (int k = 0; k < ncc; ++k) hsum[k] = 0.0;
    for (int64_t m = cl.begin; m < cl.end; ++m) {
        const int Lm = A.pairs[A.members[m]].L;
        const double* h = A.hm + A.moff[m];
        int im = 0;
        for (int a = 0; a <= Lm; ++a)
            for (int b = 0; b <= Lm - a; ++b)
                for (int cc = 0; cc <= Lm - a - b; ++cc, ++im) hsum[hidx(Lc, a, b, cc)] += h[im];
    }
    uint32_t* r = A.rec + cl.word;
    if (A.fp64) {
        double* rd = reinterpret_cast<double*>(r);
        for (int k = 0; k < ncc; ++k) rd[kClHead64 + k] = hsum[k];
    } else {
        float* f = reinterpret_cast<float*>(r + kClHead32);
        for (int k = 0; k < ncc; ++k) f[k] = float(hsum[k]);
    }
}

unsigned blocks_for(int64_t n) { return unsigned((n + kUpdBlock - 1) / kUpdBlock); }

// One thread per stored element of a CSR density (ParseArgs).
__global__ __launch_bounds__(kUpdBlock) void k_parse_csr(ParseArgs a) {
    const int64_t k = (int64_t)blockIdx.x * kUpdBlock + threadIdx.x;
    if (k >= a.nnz) return;
    int lo = 0, hi = a.nbf;  // the row: row_ptr[lo] <= k < row_ptr[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (a.row_ptr[mid] <= k) lo = mid;
        else hi = mid;
    }
    const int mu = lo, nu = a.col[k];
    const double v = a.val[k];
    if (nu < 0 || nu >= a.nbf || !isfinite(v)) {
        atomicOr(a.err, 1);
        return;
    }
    if (v == 0.0) return;
    const int I = a.shell_of_bf[mu], J = a.shell_of_bf[nu];
    const int x = mu - a.bf0[I], y = nu - a.bf0[J];
    int64_t b0 = a.adj_begin[I], b1 = a.adj_begin[I + 1];  // first partner >= J
    const int64_t end = b1;
    while (b0 < b1) {
        const int64_t mid = (b0 + b1) >> 1;
        if (a.adj_J[mid] < J) b0 = mid + 1;
        else b1 = mid;
    }
    if (b0 == end || a.adj_J[b0] != J) {
        atomicOr(a.err, 2);
        return;
    }
    const int b = a.adj_blk[b0];
    const int lJ = a.shell_l[a.blk[2 * b + 1]];
    const int nJb = (lJ + 1) * (lJ + 2) / 2;
    if (a.adj_tr[b0]) atomicAdd(&a.Wt[a.woff[b] + y * nJb + x], v);  // element (J, I) of block (I, J)
    else atomicAdd(&a.Wd[a.woff[b] + x * nJb + y], v);
}

// One thread per block weight: symmetry against the transposed element,
// then W = f P s_x s_y (f = 2 off the diagonal blocks).
__global__ __launch_bounds__(kUpdBlock) void k_block_weights(ParseArgs a) {
    const int64_t total = a.woff[a.n_blocks];
    const int64_t e = (int64_t)blockIdx.x * kUpdBlock + threadIdx.x;
    if (e >= total) return;
    int64_t lo = 0, hi = a.n_blocks;  // the block: woff[lo] <= e < woff[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (a.woff[mid] <= e) lo = mid;
        else hi = mid;
    }
    const int b = (int)lo;
    const int I = a.blk[2 * b], J = a.blk[2 * b + 1];
    const int lJ = a.shell_l[J];
    const int nJ = (lJ + 1) * (lJ + 2) / 2;
    const int64_t r = e - a.woff[b];
    const int x = (int)(r / nJ), y = (int)(r % nJ);
    const double p = a.Wd[e];
    const double q = (I == J) ? a.Wd[a.woff[b] + y * nJ + x] : a.Wt[e];
    if (fabs(p - q) > 1e-10 * (fabs(p) + fabs(q))) atomicOr(a.err, 4);
    const double f = (I == J) ? 1.0 : 2.0;
    a.W[e] = f * p * a.cscale[a.bf0[I] + x] * a.cscale[a.bf0[J] + y];
}

// One workgroup per fragment group: its kept and its dropped pairs'
// charges, each summed by strided threads and then a fixed LDS tree.
__global__ __launch_bounds__(kUpdBlock) void k_group_charges(const double* __restrict__ charge,
                                                             const int64_t* __restrict__ gpb,
                                                             const int64_t* __restrict__ dropb, int64_t n_pairs,
                                                             double* __restrict__ gq) {
    __shared__ double sk[kUpdBlock], sd[kUpdBlock];
    const int g = blockIdx.x, t = threadIdx.x;
    double a = 0.0, d = 0.0;
    for (int64_t k = gpb[g] + t; k < gpb[g + 1]; k += kUpdBlock) a += charge[k];
    for (int64_t j = dropb[g] + t; j < dropb[g + 1]; j += kUpdBlock) d += charge[n_pairs + j];
    sk[t] = a;
    sd[t] = d;
    __syncthreads();
    for (int s = kUpdBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
            sk[t] += sk[t + s];
            sd[t] += sd[t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        gq[2 * g] = sk[0];
        gq[2 * g + 1] = sd[0];
    }
}

}  // namespace

int launch_group_charges(const double* charge, const int64_t* gpb, const int64_t* dropb, int64_t n_pairs,
                         int n_groups, double* gq, void* stream) {
    if (n_groups <= 0) return 0;
    hipLaunchKernelGGL(k_group_charges, dim3(n_groups), dim3(kUpdBlock), 0, static_cast<hipStream_t>(stream), charge,
                       gpb, dropb, n_pairs, gq);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_parse_csr(const ParseArgs& a, void* stream) {
    if (a.nnz <= 0) return 0;
    hipLaunchKernelGGL(k_parse_csr, dim3(blocks_for(a.nnz)), dim3(kUpdBlock), 0, static_cast<hipStream_t>(stream), a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_block_weights(const ParseArgs& a, int64_t total, void* stream) {
    if (total <= 0) return 0;
    hipLaunchKernelGGL(k_block_weights, dim3(blocks_for(total)), dim3(kUpdBlock), 0,
                       static_cast<hipStream_t>(stream), a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_update_charges(const UpdateArgs& a, void* stream) {
    const int64_t n = a.n_pairs + a.n_drop;
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_upd_charges, dim3(blocks_for(n)), dim3(kUpdBlock), 0, static_cast<hipStream_t>(stream), a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_update_pairs(const UpdateArgs& a, void* stream) {
    if (a.n_pairs <= 0) return 0;
    hipLaunchKernelGGL(k_upd_pairs, dim3(blocks_for(a.n_pairs)), dim3(kUpdBlock), 0,
                       static_cast<hipStream_t>(stream), a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_update_members(const UpdateArgs& a, void* stream) {
    if (a.n_members <= 0) return 0;
    hipLaunchKernelGGL(k_upd_members, dim3(blocks_for(a.n_members)), dim3(kUpdBlock), 0,
                       static_cast<hipStream_t>(stream), a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_update_clusters(const UpdateArgs& a, void* stream) {
    if (a.n_clusters <= 0) return 0;
    hipLaunchKernelGGL(k_upd_clusters, dim3(blocks_for(a.n_clusters)), dim3(kUpdBlock), 0,
                       static_cast<hipStream_t>(stream), a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace envpot
