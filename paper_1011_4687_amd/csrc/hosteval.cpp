// CPU evaluation of a handle created with ENV_FORCE_CPU: the paper's switch
// back to the CPU subroutine (Sec. I: the user can return to the original CPU
// code), here over the library's own screened pair list.
//
// The arithmetic is the FP64 path of the gfx950 kernel written for one host
// thread per point range: per fragment group the FP64 nuclear term and the
// pair sum, then nuclear minus electronic added to the point's result; per
// point-pair X = P - C, the exact far-field multipole (1/R) sum h x^a y^b z^c
// with x = X/R^2 when p R^2 reaches the FP64 threshold, else the Boys values
// from the FP64 table by a Taylor step and the generated Hermite recursion
// contracted with the pair's Hermite density.  Pairs are taken one by one in
// the pair list's order (no same-centre clusters); results agree with the
// FP64 device path to rounding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <thread>
#include <vector>

#include "handle.h"
#include "hermite_gen.h"

namespace envpot {

namespace {

constexpr double kPi = 3.14159265358979323846;

template <int L>
double near_pair(const double* D, double p, double X, double Y, double Z, double r2, const double* tab) {
    const double T = p * r2;
    const int kk = int(std::fma(T, double(kBoysGridInv), 0.5));
    const double d = std::fma(double(kk), -1.0 / kBoysGridInv, T);
    const double* f = tab + size_t(kk) * kBoysRowF64;
    const double m2p = -2.0 * p;
    double s = 2.0 * std::sqrt(p / kPi);
    double G[L + 1];
    for (int n = 0; n <= L; ++n) {
        // F_n(T) = sum_j F_{n+j}(T_k) (-d)^j / j!
        double F = f[n + kBoysTaylorF64 - 1];
        for (int j = kBoysTaylorF64 - 1; j >= 1; --j) F = std::fma(-(d * (1.0 / j)), F, f[n + j - 1]);
        G[n] = s * F;
        s *= m2p;
    }
    if constexpr (L == 0) return hermite_dot_L0<double>(G, X, Y, Z, D);
    else if constexpr (L == 1) return hermite_dot_L1<double>(G, X, Y, Z, D);
    else if constexpr (L == 2) return hermite_dot_L2<double>(G, X, Y, Z, D);
    else if constexpr (L == 3) return hermite_dot_L3<double>(G, X, Y, Z, D);
    else return hermite_dot_L4<double>(G, X, Y, Z, D);
}

template <int L>
double far_pair(const double* h, double X, double Y, double Z, double r2) {
    const double ri = 1.0 / std::sqrt(r2);
    const double w = ri * ri;
    const double x = X * w, y = Y * w, z = Z * w;
    double v;
    if constexpr (L == 0) v = far_poly_L0<double>(h, x, y, z);
    else if constexpr (L == 1) v = far_poly_L1<double>(h, x, y, z);
    else if constexpr (L == 2) v = far_poly_L2<double>(h, x, y, z);
    else if constexpr (L == 3) v = far_poly_L3<double>(h, x, y, z);
    else v = far_poly_L4<double>(h, x, y, z);
    return ri * v;
}

template <int L>
double pair_value(const HostEval& he, const PairList& pl, int64_t k, double cx, double cy, double cz) {
    const double X = pl.center[3 * k] - cx, Y = pl.center[3 * k + 1] - cy, Z = pl.center[3 * k + 2] - cz;
    const double r2 = std::fma(X, X, std::fma(Y, Y, Z * Z));
    const double p = pl.p[k];
    if (r2 >= he.tfar[L] / p) return far_pair<L>(&he.h[pl.d_off[k]], X, Y, Z, r2);
    return near_pair<L>(&pl.D[pl.d_off[k]], p, X, Y, Z, r2, he.boys.data());
}

double point_value(const HostEval& he, const PairList& pl, double cx, double cy, double cz) {
    double acc = 0.0;
    for (int g = 0; g < pl.n_groups; ++g) {
        double ve = 0.0;
        for (int q = pl.group_nuc_begin[g]; q < pl.group_nuc_end[g]; ++q) {
            const double dx = cx - pl.nuc[4 * q], dy = cy - pl.nuc[4 * q + 1], dz = cz - pl.nuc[4 * q + 2];
            ve -= pl.nuc[4 * q + 3] / std::sqrt(std::fma(dx, dx, std::fma(dy, dy, dz * dz)));
        }
        for (int64_t k = pl.group_pair_begin[g]; k < pl.group_pair_begin[g + 1]; ++k) {
            switch (pl.L[k]) {
                case 0: ve += pair_value<0>(he, pl, k, cx, cy, cz); break;
                case 1: ve += pair_value<1>(he, pl, k, cx, cy, cz); break;
                case 2: ve += pair_value<2>(he, pl, k, cx, cy, cz); break;
                case 3: ve += pair_value<3>(he, pl, k, cx, cy, cz); break;
                default: ve += pair_value<4>(he, pl, k, cx, cy, cz); break;
            }
        }
        acc -= ve;
    }
    return acc;
}

int host_threads() {
    const char* e = std::getenv("ENVPOT_THREADS");
    int t = e ? std::atoi(e) : 0;
    if (t <= 0) t = int(std::thread::hardware_concurrency());
    return std::max(1, std::min(t, 256));
}

}  // namespace

void host_prepare(env_potential* h, const std::vector<double>& t64) {
    HostEval& he = h->hosteval;
    const PairList& pl = h->host;
    he.boys = t64;
    for (int L = 0; L <= kLMax; ++L) he.tfar[L] = h->bp.tfar64[L];
    he.h.assign(pl.D.size(), 0.0);
    for (size_t k = 0; k < pl.L.size(); ++k) far_coefs(pl.L[k], &pl.D[pl.d_off[k]], &he.h[pl.d_off[k]]);
}

env_status host_eval(const env_potential* h, const double* points, int64_t n, double* out) {
    const HostEval& he = h->hosteval;
    const PairList& pl = h->host;
    const int64_t nt = std::min<int64_t>(host_threads(), n);
    auto work = [&](int64_t t) {
        for (int64_t i = t; i < n; i += nt)
            out[i] = point_value(he, pl, points[3 * i], points[3 * i + 1], points[3 * i + 2]);
    };
    std::vector<std::thread> pool;
    try {
        for (int64_t t = 1; t < nt; ++t) pool.emplace_back(work, t);
    } catch (...) {
        for (auto& th : pool) th.join();
        return ENV_E_NOMEM;
    }
    work(0);
    for (auto& th : pool) th.join();
    return ENV_OK;
}

}  // namespace envpot
