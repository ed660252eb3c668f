// Host-side builder of the screened primitive-pair list (runs once per
// environment, like the paper's one-time upload of the read-only field data,
// Sec. III).  For every pair of primitives a in shell I and b in shell J of a
// nonzero density block it forms the Gaussian product (exponent p = a + b,
// centre P = (a A + b B)/p) and folds the density-matrix block, the
// normalisation and the three 1-D Hermite expansion coefficients E^{ij}_t
// into one Hermite density D_tuv (McMurchie-Davidson), so that the pair's
// share of the electronic potential at C is
//     (2 pi / p) sum_{t+u+v <= L} D_tuv R_tuv(p, P - C).
// D is stored scaled by (pi/p)^{3/2}: then D_000 is the pair's electron
// count and the far field of the pair is sum_tuv D_tuv d^t d^u d^v (1/R).
#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <xmmintrin.h>

#include "envpot_internal.h"
#include "screen_math.h"
#include "update_internal.h"

namespace envpot {
namespace {

constexpr double kPi = 3.14159265358979323846;

int ncart(int l) { return (l + 1) * (l + 2) / 2; }

// Cartesian exponents of component c of a shell of angular momentum l,
// x-major order: p = x, y, z; d = xx, xy, xz, yy, yz, zz.
void cart(int l, int c, int e[3]) {
    static const int8_t tab[3][6][3] = {
        {{0, 0, 0}},
        {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
        {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}}};
    for (int d = 0; d < 3; ++d) e[d] = tab[l][c][d];
}

double odd_fact(int n) {  // (n)!! for odd n >= -1
    double r = 1.0;
    while (n > 1) { r *= n; n -= 2; }
    return r;
}

// Normalisation of x^i y^j z^k exp(-a r^2).
double prim_norm(double a, const int e[3]) {
    const int l = e[0] + e[1] + e[2];
    return std::pow(2.0 * a / kPi, 0.75) * std::pow(4.0 * a, 0.5 * l) /
           std::sqrt(odd_fact(2 * e[0] - 1) * odd_fact(2 * e[1] - 1) * odd_fact(2 * e[2] - 1));
}

// 1/sqrt(self-overlap) of a contracted component.
double contraction_scale(int nprim, const double* ex, const double* co, const int e[3]) {
    double s = 0.0;
    for (int a = 0; a < nprim; ++a)
        for (int b = 0; b < nprim; ++b) {
            const double p = ex[a] + ex[b];
            double m = std::pow(kPi / p, 1.5);
            for (int d = 0; d < 3; ++d) m *= odd_fact(2 * e[d] - 1) / std::pow(2.0 * p, e[d]);
            s += co[a] * co[b] * prim_norm(ex[a], e) * prim_norm(ex[b], e) * m;
        }
    return 1.0 / std::sqrt(s);
}

// Hermite expansion coefficients of one direction:
//   x_A^i x_B^j exp(-a x_A^2 - b x_B^2) = sum_t E[i][j][t] Lambda_t(x; p, P).
// First the column i = 0 is raised in j, then every column is raised in i:
//   E^{i,j+1}_t = E^{ij}_{t-1}/(2p) + X_PB E^{ij}_t + (t+1) E^{ij}_{t+1}
//   E^{i+1,j}_t = E^{ij}_{t-1}/(2p) + X_PA E^{ij}_t + (t+1) E^{ij}_{t+1}
struct Ecoef { double v[3][3][5]; };

void hermite_coefs(int li, int lj, double a, double b, double A, double B, Ecoef& E) {
    std::memset(&E, 0, sizeof(E));
    const double p = a + b, P = (a * A + b * B) / p;
    const double xpa = P - A, xpb = P - B, h = 0.5 / p, dab = A - B;
    E.v[0][0][0] = std::exp(-(a * b / p) * dab * dab);
    auto get = [&](int i, int j, int t) -> double {
        return (t < 0 || t > i + j) ? 0.0 : E.v[i][j][t];
    };
    for (int j = 0; j < lj; ++j)
        for (int t = 0; t <= j + 1; ++t)
            E.v[0][j + 1][t] = h * get(0, j, t - 1) + xpb * get(0, j, t) + (t + 1) * get(0, j, t + 1);
    for (int i = 0; i < li; ++i)
        for (int j = 0; j <= lj; ++j)
            for (int t = 0; t <= i + j + 1; ++t)
                E.v[i + 1][j][t] = h * get(i, j, t - 1) + xpa * get(i, j, t) + (t + 1) * get(i, j, t + 1);
}

struct Block {   // one unordered shell pair I <= J with its density block
    int I, J;
    int64_t woff;     // its weights P_IJ x contraction scales x (2 if I != J): nI x nJ from here
    double maxabs;
};

struct Bucket {  // pairs of one group and one L, appended in build order
    std::vector<double> rec;  // per pair: Px, Py, Pz, p, D[ncomp(L)]
    std::vector<int32_t> atom;  // per pair: the atom of both shells, or -1 (two centres)
    std::vector<int32_t> src;   // per pair (when sources are kept): block, ia, ib
    int64_t n = 0;
};

struct GroupOut {
    Bucket b[kLMax + 1];
    int64_t n_unscreened = 0;
    double screened_bound = 0.0;
    double dropped_charge = 0.0;  // electron count of screened-out pairs
    std::vector<int32_t> drop;    // screened-out pairs (when sources are kept): block, ia, ib
};

bool finite(double x) { return std::isfinite(x); }

// hermite_index as a lookup table for the hot loops.
struct HIndex {
    int8_t v[kLMax + 1][kLMax + 1][kLMax + 1][kLMax + 1];
    HIndex() {
        for (int L = 0; L <= kLMax; ++L)
            for (int t = 0; t <= kLMax; ++t)
                for (int u = 0; u <= kLMax; ++u)
                    for (int w = 0; w <= kLMax; ++w) v[L][t][u][w] = int8_t(hermite_index(L, t, u, w));
    }
};
const HIndex& hidx() {
    static const HIndex h;
    return h;
}

}  // namespace

env_status build_pair_list(const env_nucleus* nuclei, int32_t n_nuclei,
                           const env_shell* shells, int32_t n_shells,
                           const env_density* P, const env_options& opt, PairList& out) {
    return build_pair_list(nuclei, n_nuclei, shells, n_shells, P, opt, out, nullptr);
}

env_status build_pair_list(const env_nucleus* nuclei, int32_t n_nuclei,
                           const env_shell* shells, int32_t n_shells,
                           const env_density* P, const env_options& opt, PairList& out,
                           PairSources* src, BlockPlan* plan) {
    const char* tenv = std::getenv("ENVPOT_TIMING");
    const bool timing = tenv && *tenv && *tenv != '0';
    auto tlast = std::chrono::steady_clock::now();
    auto lap = [&](const char* what) {
        if (!timing) return;
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[envpot build] %-22s %8.3f s\n", what,
                     std::chrono::duration<double>(now - tlast).count());
        tlast = now;
    };
    out = PairList();
    if (n_nuclei < 0 || n_shells < 0 || !P) return ENV_E_ARG;
    if ((n_nuclei > 0 && !nuclei) || (n_shells > 0 && !shells)) return ENV_E_ARG;
    for (int a = 0; a < n_nuclei; ++a) {
        const env_nucleus& q = nuclei[a];
        if (!finite(q.xyz[0]) || !finite(q.xyz[1]) || !finite(q.xyz[2]) || !finite(q.Z))
            return ENV_E_ARG;
        if (q.fragment < -1 || q.reserved != 0) return ENV_E_ARG;
    }
    std::vector<int> bf0(n_shells + 1, 0);
    for (int s = 0; s < n_shells; ++s) {
        const env_shell& sh = shells[s];
        if (sh.atom < 0 || sh.atom >= n_nuclei || sh.nprim < 1 || sh.reserved != 0 ||
            !sh.exponents || !sh.coefs || sh.l < 0)
            return ENV_E_ARG;
        if (sh.l > 2) return ENV_E_UNSUPPORTED;
        for (int k = 0; k < sh.nprim; ++k)
            if (!(sh.exponents[k] > 0.0) || !finite(sh.exponents[k]) || !finite(sh.coefs[k]))
                return ENV_E_ARG;
        bf0[s + 1] = bf0[s] + ncart(sh.l);
    }
    const int nbf = bf0[n_shells];
    if (P->nbf != nbf) return ENV_E_ARG;
    if (P->format != ENV_DENSITY_DENSE && P->format != ENV_DENSITY_CSR) return ENV_E_ARG;
    if (nbf > 0 && !P->values) return ENV_E_ARG;
    if (P->format == ENV_DENSITY_CSR && (!P->row_ptr || (nbf > 0 && !P->col))) return ENV_E_ARG;
    const double thr = opt.screen_threshold;
    if (!(thr >= 0.0) || !finite(thr)) return ENV_E_ARG;
    const bool screen = !(opt.flags & ENV_NO_SCREENING) && thr > 0.0;
    out.nbf = nbf;

    // fragment groups: sorted fragment ids (-1 included), cross group last
    std::vector<int> ids;
    for (int a = 0; a < n_nuclei; ++a) ids.push_back(nuclei[a].fragment);
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
    auto group_of_atom = [&](int a) {
        return int(std::lower_bound(ids.begin(), ids.end(), nuclei[a].fragment) - ids.begin());
    };
    const int n_frag_groups = int(ids.size());

    std::vector<int> shell_of_bf(nbf);
    for (int s = 0; s < n_shells; ++s)
        for (int k = bf0[s]; k < bf0[s + 1]; ++k) shell_of_bf[k] = s;

    // contraction scales per shell component
    std::vector<double> cscale(nbf);
    for (int s = 0; s < n_shells; ++s)
        for (int c = 0; c < ncart(shells[s].l); ++c) {
            int e[3];
            cart(shells[s].l, c, e);
            cscale[bf0[s] + c] = contraction_scale(shells[s].nprim, shells[s].exponents,
                                                   shells[s].coefs, e);
        }

    // per shell: coefficient x primitive normalisation of every component, and
    // the s-type normalisation (2a/pi)^{3/4} used by the screening bound
    std::vector<int64_t> noff(n_shells + 1, 0);
    for (int s = 0; s < n_shells; ++s) noff[s + 1] = noff[s] + int64_t(shells[s].nprim) * ncart(shells[s].l);
    std::vector<double> cnorm(noff[n_shells]);
    std::vector<int64_t> poff(n_shells + 1, 0);
    for (int s = 0; s < n_shells; ++s) poff[s + 1] = poff[s] + shells[s].nprim;
    std::vector<double> n0(poff[n_shells]);
    for (int s = 0; s < n_shells; ++s) {
        const int nc = ncart(shells[s].l);
        for (int k = 0; k < shells[s].nprim; ++k) {
            const double a = shells[s].exponents[k];
            n0[poff[s] + k] = std::pow(2.0 * a / kPi, 0.75);
            for (int c = 0; c < nc; ++c) {
                int e[3];
                cart(shells[s].l, c, e);
                cnorm[noff[s] + int64_t(k) * nc + c] = shells[s].coefs[k] * prim_norm(a, e);
            }
        }
    }

    lap("validate, norms");
    // density blocks of ordered shell pairs, numbered in order of first
    // touch; rows arrive in order, so the rows of one shell I are
    // consecutive and slot[J] holds the block (I, J) while they last
    std::vector<double> rawv;                // per block nI x nJ elements, row-major
    std::vector<int64_t> roff;               // per block: first element in rawv
    std::vector<std::pair<int, int>> rawkey;
    std::vector<int> slot(size_t(std::max(n_shells, 1)), -1), touched;
    int cur_I = -1;
    auto put = [&](int mu, int nu, double v) -> bool {
        if (!finite(v)) return false;
        if (v == 0.0) return true;
        const int I = shell_of_bf[mu], J = shell_of_bf[nu];
        if (I != cur_I) {
            for (int j : touched) slot[j] = -1;
            touched.clear();
            cur_I = I;
        }
        const int nJ = bf0[J + 1] - bf0[J];
        int k = slot[J];
        if (k < 0) {
            k = int(rawkey.size());
            roff.push_back(int64_t(rawv.size()));
            rawv.resize(rawv.size() + size_t(bf0[I + 1] - bf0[I]) * size_t(nJ), 0.0);
            rawkey.emplace_back(I, J);
            slot[J] = k;
            touched.push_back(J);
        }
        rawv[size_t(roff[k] + int64_t(mu - bf0[I]) * nJ + (nu - bf0[J]))] += v;
        return true;
    };
    if (P->format == ENV_DENSITY_DENSE) {
        for (int mu = 0; mu < nbf; ++mu)
            for (int nu = 0; nu < nbf; ++nu)
                if (!put(mu, nu, P->values[(size_t)mu * nbf + nu])) return ENV_E_ARG;
    } else {
        if (P->row_ptr[0] != 0) return ENV_E_ARG;
        for (int mu = 0; mu < nbf; ++mu) {
            if (P->row_ptr[mu + 1] < P->row_ptr[mu]) return ENV_E_ARG;
            for (int64_t k = P->row_ptr[mu]; k < P->row_ptr[mu + 1]; ++k) {
                const int nu = P->col[k];
                if (nu < 0 || nu >= nbf) return ENV_E_ARG;
                if (!put(mu, nu, P->values[k])) return ENV_E_ARG;
            }
        }
    }
    lap("density blocks");
    // symmetry: block (I,J) must equal the transpose of block (J,I); each
    // shell's blocks sorted by partner shell for the lookup
    std::vector<int64_t> rbeg(size_t(n_shells) + 1, 0);
    for (const auto& key : rawkey) ++rbeg[size_t(key.first) + 1];
    for (int sI = 0; sI < n_shells; ++sI) rbeg[sI + 1] += rbeg[sI];
    std::vector<std::pair<int, int>> rlist(rawkey.size());  // (J, block), grouped by I
    {
        std::vector<int64_t> fill(rbeg.begin(), rbeg.end() - 1);
        for (size_t k = 0; k < rawkey.size(); ++k) rlist[size_t(fill[rawkey[k].first]++)] = {rawkey[k].second, int(k)};
        for (int sI = 0; sI < n_shells; ++sI) std::sort(rlist.begin() + rbeg[sI], rlist.begin() + rbeg[sI + 1]);
    }
    auto blk = [&](int I, int J) -> const double* {
        const auto b = rlist.begin() + rbeg[I], e = rlist.begin() + rbeg[I + 1];
        const auto it = std::lower_bound(b, e, std::make_pair(J, -1));
        return (it != e && it->first == J) ? rawv.data() + roff[size_t(it->second)] : nullptr;
    };
    static const double zero36[36] = {0};
    std::vector<Block> blocks;
    std::vector<double> bw;   // block weights, nI x nJ per block
    std::vector<int> block_group;
    for (size_t k = 0; k < rawkey.size(); ++k) {
        const int I = rawkey[k].first, J = rawkey[k].second;
        const double* a = rawv.data() + roff[k];
        const double* b = blk(J, I);
        if (!b) b = zero36;
        const int nI = ncart(shells[I].l), nJ = ncart(shells[J].l);
        for (int x = 0; x < nI; ++x)
            for (int y = 0; y < nJ; ++y) {
                const double u = a[x * nJ + y], v = b[y * nI + x];
                if (std::fabs(u - v) > 1e-10 * (std::fabs(u) + std::fabs(v))) return ENV_E_ARG;
            }
        if (I > J) continue;
        Block B;
        B.I = I;
        B.J = J;
        B.maxabs = 0.0;
        B.woff = int64_t(bw.size());
        bw.resize(bw.size() + size_t(nI) * size_t(nJ));
        const double f = (I == J) ? 1.0 : 2.0;
        for (int x = 0; x < nI; ++x)
            for (int y = 0; y < nJ; ++y) {
                const double wv = f * a[x * nJ + y] * cscale[bf0[I] + x] * cscale[bf0[J] + y];
                bw[size_t(B.woff + x * nJ + y)] = wv;
                B.maxabs = std::max(B.maxabs, std::fabs(wv));
            }
        const int gI = group_of_atom(shells[I].atom), gJ = group_of_atom(shells[J].atom);
        blocks.push_back(B);
        block_group.push_back(gI == gJ ? gI : n_frag_groups);
        if (gI != gJ) out.has_cross = true;
    }
    if (out.has_cross && (opt.flags & ENV_NEUTRALIZE)) return ENV_E_UNSUPPORTED;
    const int n_groups = n_frag_groups + (out.has_cross ? 1 : 0);
    out.n_groups = n_groups;

    // blocks of each group in (I, J) order: deterministic pair order
    std::vector<std::vector<int>> gblocks(n_groups);
    {
        std::vector<int> order(blocks.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = int(k);
        std::sort(order.begin(), order.end(), [&](int x, int y) {
            if (blocks[x].I != blocks[y].I) return blocks[x].I < blocks[y].I;
            return blocks[x].J < blocks[y].J;
        });
        for (int k : order) gblocks[block_group[k]].push_back(k);
    }

    lap("symmetry, grouping");
    // nuclei by group (Z == 0 centres carry basis functions only)
    std::vector<double> zg(n_groups, 0.0);
    out.group_nuc_begin.assign(n_groups, 0);
    out.group_nuc_end.assign(n_groups, 0);
    for (int g = 0; g < n_frag_groups; ++g) {
        out.group_nuc_begin[g] = int(out.nuc.size() / 4);
        for (int a = 0; a < n_nuclei; ++a) {
            if (group_of_atom(a) != g || nuclei[a].Z == 0.0) continue;
            out.nuc.push_back(nuclei[a].xyz[0]);
            out.nuc.push_back(nuclei[a].xyz[1]);
            out.nuc.push_back(nuclei[a].xyz[2]);
            out.nuc.push_back(nuclei[a].Z);
            zg[g] += nuclei[a].Z;
            out.nuclear_charge += nuclei[a].Z;
        }
        out.group_nuc_end[g] = int(out.nuc.size() / 4);
    }
    if (out.has_cross) {
        out.group_nuc_begin[n_frag_groups] = out.group_nuc_end[n_frag_groups] = int(out.nuc.size() / 4);
    }

    lap("nuclei");
    const bool neutralize = (opt.flags & ENV_NEUTRALIZE) != 0;
    // basis and blocks for the density update tables (and the device build)
    auto fill_sources = [&]() {
        src->neutralize = neutralize;
        src->blk_I.resize(blocks.size());
        src->blk_J.resize(blocks.size());
        for (size_t k = 0; k < blocks.size(); ++k) {
            src->blk_I[k] = blocks[k].I;
            src->blk_J[k] = blocks[k].J;
        }
        src->shell_l.resize(n_shells);
        src->shell_atom.resize(n_shells);
        src->bf0.assign(bf0.begin(), bf0.end());
        for (int s2 = 0; s2 < n_shells; ++s2) {
            src->shell_l[s2] = shells[s2].l;
            src->shell_atom[s2] = shells[s2].atom;
        }
        src->poff.assign(poff.begin(), poff.end());
        src->noff.assign(noff.begin(), noff.end());
        src->cscale = cscale;
        src->cnorm = cnorm;
        src->exps.resize(poff[n_shells]);
        for (int s2 = 0; s2 < n_shells; ++s2)
            for (int k = 0; k < shells[s2].nprim; ++k) src->exps[poff[s2] + k] = shells[s2].exponents[k];
        src->atom_xyz.resize(3 * size_t(n_nuclei));
        for (int a = 0; a < n_nuclei; ++a)
            for (int c = 0; c < 3; ++c) src->atom_xyz[3 * size_t(a) + c] = nuclei[a].xyz[c];
        src->group_charge = zg;
    };
    if (plan) {  // the device build takes over from here
        if (!src) return ENV_E_ARG;
        fill_sources();
        *plan = BlockPlan();
        plan->thr = thr;
        plan->screen = screen;
        plan->blk_maxabs.resize(blocks.size());
        for (size_t k = 0; k < blocks.size(); ++k) plan->blk_maxabs[k] = blocks[k].maxabs;
        plan->shell_nprim.resize(n_shells);
        for (int s2 = 0; s2 < n_shells; ++s2) plan->shell_nprim[s2] = shells[s2].nprim;
        plan->coefs.resize(poff[n_shells]);
        plan->n0 = n0;
        for (int s2 = 0; s2 < n_shells; ++s2)
            for (int k = 0; k < shells[s2].nprim; ++k) plan->coefs[poff[s2] + k] = shells[s2].coefs[k];
        int64_t u = 0;
        for (int g = 0; g < n_groups; ++g)
            for (int bk : gblocks[g]) {
                const int64_t nI = shells[blocks[bk].I].nprim, nJ = shells[blocks[bk].J].nprim;
                plan->enum_blk.push_back(bk);
                plan->enum_group.push_back(g);
                plan->enum_first.push_back(u);
                u += blocks[bk].I == blocks[bk].J ? nI * (nI + 1) / 2 : nI * nJ;
            }
        plan->enum_first.push_back(u);
        out.n_unscreened = u;
        out.group_pair_begin.assign(n_groups + 1, 0);
        lap("block plan");
        return ENV_OK;
    }
    std::vector<GroupOut> gout(n_groups);
    // the fold into D (and the charges of screened-out pairs) is left to the
    // device: D stays zero here
    const bool device_fold = src && src->device_fold;
    const HIndex& HX = hidx();
    auto work = [&](int g) {
        GroupOut& go = gout[g];
        Ecoef Ex, Ey, Ez;
        double D[35];
        for (int bk : gblocks[g]) {
            const Block& B = blocks[bk];
            const env_shell& SI = shells[B.I];
            const env_shell& SJ = shells[B.J];
            const double* A = nuclei[SI.atom].xyz;
            const double* Bc = nuclei[SJ.atom].xyz;
            const int lI = SI.l, lJ = SJ.l, L = lI + lJ, nc = kNComp[L];
            const int nI = ncart(lI), nJ = ncart(lJ);
            const double rab2 = sm::dist2(A, Bc);
            const bool one_centre = SI.atom == SJ.atom;
            int eI[6][3], eJ[6][3];
            for (int c = 0; c < nI; ++c) cart(lI, c, eI[c]);
            for (int c = 0; c < nJ; ++c) cart(lJ, c, eJ[c]);
            for (int ia = 0; ia < SI.nprim; ++ia) {
                for (int ib = (B.I == B.J ? ia : 0); ib < SJ.nprim; ++ib) {
                    const double a = SI.exponents[ia], b = SJ.exponents[ib];
                    const double ca = SI.coefs[ia], cb = SJ.coefs[ib];
                    const double p = a + b;
                    const double w = (B.I == B.J && ia != ib) ? 2.0 : 1.0;
                    const double pp = kPi / p, pp32 = pp * std::sqrt(pp);
                    const double* na_c = &cnorm[noff[B.I] + int64_t(ia) * nI];  // c_a N_a per component
                    const double* nb_c = &cnorm[noff[B.J] + int64_t(ib) * nJ];
                    ++go.n_unscreened;
                    const double bound = sm::screen_bound(ca, cb, n0[poff[B.I] + ia], n0[poff[B.J] + ib], a, b, rab2);
                    const bool drop = screen && bound < thr;
                    if (drop) go.screened_bound += w * B.maxabs * bound;
                    if (drop && !neutralize) continue;
                    if (drop && src) go.drop.insert(go.drop.end(), {int32_t(bk), int32_t(ia), int32_t(ib)});
                    if (drop && device_fold) continue;
                    if (!device_fold) {
                        hermite_coefs(lI, lJ, a, b, A[0], Bc[0], Ex);
                        hermite_coefs(lI, lJ, a, b, A[1], Bc[1], Ey);
                        hermite_coefs(lI, lJ, a, b, A[2], Bc[2], Ez);
                    }
                    if (drop) {  // only its charge: sum P c N c N E_0 E_0 E_0 (pi/p)^{3/2}
                        double q = 0.0;
                        for (int x = 0; x < nI; ++x)
                            for (int y = 0; y < nJ; ++y)
                                q += bw[size_t(B.woff + x * nJ + y)] * na_c[x] * nb_c[y] * Ex.v[eI[x][0]][eJ[y][0]][0] *
                                     Ey.v[eI[x][1]][eJ[y][1]][0] * Ez.v[eI[x][2]][eJ[y][2]][0];
                        go.dropped_charge += w * q * pp32;
                        continue;
                    }
                    for (int k = 0; k < nc; ++k) D[k] = 0.0;
                    for (int x = 0; x < (device_fold ? 0 : nI); ++x) {
                        for (int y = 0; y < nJ; ++y) {
                            const double pw = bw[size_t(B.woff + x * nJ + y)];
                            if (pw == 0.0) continue;
                            const double f = w * pw * na_c[x] * nb_c[y];
                            const int ix = eI[x][0], jx = eJ[y][0], iy = eI[x][1], jy = eJ[y][1],
                                      iz = eI[x][2], jz = eJ[y][2];
                            for (int t = 0; t <= ix + jx; ++t) {
                                const double ft = f * Ex.v[ix][jx][t];
                                for (int u = 0; u <= iy + jy; ++u) {
                                    const double fu = ft * Ey.v[iy][jy][u];
                                    const int8_t* hx = HX.v[L][t][u];
                                    for (int v = 0; v <= iz + jz; ++v) D[hx[v]] += fu * Ez.v[iz][jz][v];
                                }
                            }
                        }
                    }
                    const double sc = pp32;
                    Bucket& bu = go.b[L];
                    if (one_centre) {  // the product centre is the atom itself, exactly
                        bu.rec.push_back(A[0]);
                        bu.rec.push_back(A[1]);
                        bu.rec.push_back(A[2]);
                    } else {
                        bu.rec.push_back(sm::prod_centre(a, A[0], b, Bc[0], p));
                        bu.rec.push_back(sm::prod_centre(a, A[1], b, Bc[1], p));
                        bu.rec.push_back(sm::prod_centre(a, A[2], b, Bc[2], p));
                    }
                    bu.atom.push_back(one_centre ? SI.atom : -1);
                    if (src) bu.src.insert(bu.src.end(), {int32_t(bk), int32_t(ia), int32_t(ib)});
                    bu.rec.push_back(p);
                    for (int k = 0; k < nc; ++k) bu.rec.push_back(D[k] * sc);
                    ++bu.n;
                }
            }
        }
    };
    {
        unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        nt = std::min<unsigned>(nt, std::max(1, n_groups));
        std::vector<std::thread> th;
        std::atomic<int> next{0};
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&]() {
                // flush denormals to zero: products of vanishing Gaussian overlaps
                // (exp(-mu R^2) ~ 1e-300) otherwise take the slow denormal path
                _mm_setcsr(_mm_getcsr() | 0x8040);
                for (;;) {
                    const int g = next.fetch_add(1);
                    if (g >= n_groups) break;
                    work(g);
                }
            });
        for (auto& t : th) t.join();
    }

    lap("primitive pairs");
    // neutralise: scale the Hermite densities of each group so that its
    // electron count tr(P_f S_f) (screened-out pairs included) equals its
    // nuclear charge
    if (neutralize) {
        for (int g = 0; g < n_groups; ++g) {
            double q = gout[g].dropped_charge;
            for (int L = 0; L <= kLMax; ++L) {
                const Bucket& bu = gout[g].b[L];
                const int rw = 4 + kNComp[L];
                for (int64_t k = 0; k < bu.n; ++k) q += bu.rec[k * rw + 4];
            }
            if (q == 0.0) continue;
            const double s = zg[g] / q;
            for (int L = 0; L <= kLMax; ++L) {
                Bucket& bu = gout[g].b[L];
                const int rw = 4 + kNComp[L];
                for (int64_t k = 0; k < bu.n; ++k)
                    for (int c = 0; c < kNComp[L]; ++c) bu.rec[k * rw + 4 + c] *= s;
            }
        }
    }

    lap("neutralise");
    // final order: group, then L; every output sized once, groups filled in parallel
    out.group_pair_begin.assign(n_groups + 1, 0);
    std::vector<int64_t> gd(n_groups + 1, 0);  // first D word of each group
    for (int g = 0; g < n_groups; ++g) {
        int64_t np = 0, nd = 0;
        for (int L = 0; L <= kLMax; ++L) {
            np += gout[g].b[L].n;
            nd += gout[g].b[L].n * kNComp[L];
        }
        out.group_pair_begin[g + 1] = out.group_pair_begin[g] + np;
        gd[g + 1] = gd[g] + nd;
        out.n_unscreened += gout[g].n_unscreened;
        out.screened_bound += gout[g].screened_bound;
    }
    const int64_t npairs = out.group_pair_begin[n_groups];
    lap("count");
    out.L.resize(npairs);
    out.group.resize(npairs);
    out.center.resize(3 * size_t(npairs));
    out.p.resize(npairs);
    out.atom1.resize(npairs);
    out.d_off.resize(npairs + 1);
    out.D.resize(gd[n_groups]);
    out.d_off[npairs] = gd[n_groups];
    std::vector<double> qg(n_groups, 0.0);
    if (src) {
        src->pair_blk.resize(npairs);
        src->pair_ia.resize(npairs);
        src->pair_ib.resize(npairs);
    }
    lap("allocate");
    {
        std::atomic<int> next{0};
        std::vector<std::thread> th;
        const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&]() {
                for (;;) {
                    const int g = next.fetch_add(1);
                    if (g >= n_groups) break;
                    int64_t k = out.group_pair_begin[g], d = gd[g];
                    double q = 0.0;
                    for (int L = 0; L <= kLMax; ++L) {
                        Bucket& bu = gout[g].b[L];
                        const int rw = 4 + kNComp[L];
                        for (int64_t j = 0; j < bu.n; ++j, ++k) {
                            const double* r = &bu.rec[j * rw];
                            out.L[k] = L;
                            out.group[k] = g;
                            out.center[3 * k] = r[0];
                            out.center[3 * k + 1] = r[1];
                            out.center[3 * k + 2] = r[2];
                            out.p[k] = r[3];
                            out.atom1[k] = bu.atom[j];
                            out.d_off[k] = d;
                            if (src) {
                                src->pair_blk[k] = bu.src[3 * j];
                                src->pair_ia[k] = bu.src[3 * j + 1];
                                src->pair_ib[k] = bu.src[3 * j + 2];
                            }
                            for (int c = 0; c < kNComp[L]; ++c) out.D[d + c] = r[4 + c];
                            d += kNComp[L];
                            q += r[4];
                        }
                        std::vector<double>().swap(bu.rec);
                        std::vector<int32_t>().swap(bu.atom);
                        std::vector<int32_t>().swap(bu.src);
                    }
                    qg[g] = q;
                }
            });
        for (auto& t : th) t.join();
    }
    for (int g = 0; g < n_groups; ++g) out.electrons += qg[g];
    if (src) {
        fill_sources();
        for (int g = 0; g < n_groups; ++g) {
            const std::vector<int32_t>& dr = gout[g].drop;
            for (size_t j = 0; j + 2 < dr.size(); j += 3) {
                src->drop_blk.push_back(dr[j]);
                src->drop_ia.push_back(dr[j + 1]);
                src->drop_ib.push_back(dr[j + 2]);
                src->drop_group.push_back(g);
            }
        }
    }
    lap("order");
    return ENV_OK;
}

namespace {

// Coefficients of the homogeneous polynomials P_tuv with
//   d^t_X d^u_Y d^v_Z (1/R) = P_tuv(X, Y, Z) / R^{2k+1},  k = t + u + v,
// built by P_{t+1,u,v} = R^2 dP/dX - (2k+1) X P (likewise for Y and Z).
// Polynomials are dense arrays over exponents [a][b][c], a, b, c <= 4.
struct Poly { double c[5][5][5]; };
struct PolyTable { Poly t[5][5][5]; };

PolyTable make_poly_table() {
    PolyTable T;
    std::memset(&T, 0, sizeof(T));
    T.t[0][0][0].c[0][0][0] = 1.0;
    for (int k = 1; k <= kLMax; ++k)
        for (int tt = 0; tt <= k; ++tt)
            for (int uu = 0; uu <= k - tt; ++uu) {
                const int vv = k - tt - uu;
                int dir, pt = tt, pu = uu, pv = vv;
                if (tt > 0) { dir = 0; --pt; }
                else if (uu > 0) { dir = 1; --pu; }
                else { dir = 2; --pv; }
                const Poly& P = T.t[pt][pu][pv];
                Poly& Q = T.t[tt][uu][vv];
                for (int a = 0; a <= 4; ++a)
                    for (int b = 0; b <= 4 - a; ++b)
                        for (int c = 0; c <= 4 - a - b; ++c) {
                            const double co = P.c[a][b][c];
                            if (co == 0.0) continue;
                            const int e[3] = {a, b, c};
                            if (e[dir] > 0) {  // R^2 dP/d(dir)
                                for (int s = 0; s < 3; ++s) {
                                    int f[3] = {a, b, c};
                                    f[dir] -= 1;
                                    f[s] += 2;
                                    if (f[0] + f[1] + f[2] <= 4) Q.c[f[0]][f[1]][f[2]] += e[dir] * co;
                                }
                            }
                            int f[3] = {a, b, c};  // -(2k-1) X_dir P
                            f[dir] += 1;
                            if (f[0] + f[1] + f[2] <= 4) Q.c[f[0]][f[1]][f[2]] -= (2 * k - 1) * co;
                        }
            }
    return T;
}

const Poly& derivative_poly(int t, int u, int v) {
    static const PolyTable table = make_poly_table();  // thread-safe one-time init
    return table.t[t][u][v];
}

}  // namespace

void far_coefs(int L, const double* D, double* h) {
    const HIndex& HX = hidx();
    for (int k = 0; k < kNComp[L]; ++k) h[k] = 0.0;
    for (int t = 0; t <= L; ++t)
        for (int u = 0; u <= L - t; ++u)
            for (int v = 0; v <= L - t - u; ++v) {
                const double d = D[HX.v[L][t][u][v]];
                if (d == 0.0) continue;
                const Poly& P = derivative_poly(t, u, v);
                const int k = t + u + v;
                for (int a = 0; a <= k; ++a)
                    for (int b = 0; b <= k - a; ++b) {
                        const int c = k - a - b;
                        h[HX.v[L][a][b][c]] += d * P.c[a][b][c];
                    }
            }
}


// ------------------------------------------------------------ Boys tables

// F_n(T), n = 0..nmax, in long double: F_N for a high order N by its power
// series, then the stable downward recursion F_n = (2T F_{n+1} + e^{-T})/(2n+1).
void boys_ld(int nmax, long double T, long double* F) {
    const int N = nmax + 30;
    long double term = 1.0L / (2 * N + 1), sum = term;
    for (int i = 1; i < 4000; ++i) {
        term *= 2.0L * T / (2 * N + 2 * i + 1);
        sum += term;
        if (term < 1e-22L * sum) break;
    }
    const long double e = expl(-T);
    long double f = e * sum;
    for (int n = N - 1; n >= 0; --n) {
        f = (2.0L * T * f + e) / (2 * n + 1);
        if (n <= nmax) F[n] = f;
    }
}

long double boys_asym(int n, long double T) {
    long double df = 1.0L;
    for (int k = 2 * n - 1; k > 1; k -= 2) df *= k;
    return df / powl(2.0L, n + 1) * sqrtl(3.14159265358979323846264338327950288L / powl(T, 2 * n + 1));
}

// Smallest grid T (multiple of 1/8) beyond which the asymptotic form of
// F_0..F_L is within eps (relative) of the exact value.
double far_threshold(int L, long double eps) {
    long double F[16];
    int last_bad = 0;
    for (int k = 1; k <= 8 * 120; ++k) {
        const long double T = k / 8.0L;
        boys_ld(L, T, F);
        for (int n = 0; n <= L; ++n)
            if (fabsl(F[n] - boys_asym(n, T)) > eps * F[n]) last_bad = k;
    }
    return (last_bad + 1) / 8.0;
}

void build_boys_tables(std::vector<float>& t32, std::vector<double>& t64, BoysParams& bp) {
    std::memset(&bp, 0, sizeof(bp));
    double max32 = 0.0, max64 = 0.0;
    for (int L = 0; L <= kLMax; ++L) {
        bp.tfar32[L] = float(far_threshold(L, 0x1p-28L));
        bp.tfar64[L] = far_threshold(L, 0x1p-56L);
        max32 = std::max(max32, double(bp.tfar32[L]));
        max64 = std::max(max64, bp.tfar64[L]);
    }
    bp.rows32 = int(max32 * kBoysGridInv) + 2;
    bp.rows64 = int(max64 * kBoysGridInv) + 2;
    t32.assign(size_t(bp.rows32) * kBoysRowF32, 0.0f);
    t64.assign(size_t(bp.rows64) * kBoysRowF64, 0.0);
    long double F[16];
    for (int k = 0; k < bp.rows32; ++k) {
        boys_ld(kLMax + kBoysTaylorF32 - 1, k / (long double)kBoysGridInv, F);
        for (int n = 0; n < kLMax + kBoysTaylorF32; ++n) t32[size_t(k) * kBoysRowF32 + n] = float(F[n]);
    }
    for (int k = 0; k < bp.rows64; ++k) {
        boys_ld(kLMax + kBoysTaylorF64 - 1, k / (long double)kBoysGridInv, F);
        for (int n = 0; n < kLMax + kBoysTaylorF64; ++n) t64[size_t(k) * kBoysRowF64 + n] = double(F[n]);
    }
}

}  // namespace envpot
