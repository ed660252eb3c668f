// Device image of a pair list: pair records, same-centre clusters and the
// segment tables of every split factor.
//
// Records of one fragment group are laid out as
//   [pairs L=0] ... [pairs L=4] [clusters by merged L] [cluster members]
// where every run of equal-size records is one segment.  Cluster members are
// ordinary pair records reached only through their cluster's member table.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdlib>
#include <cmath>
#include <limits>
#include <map>
#include <thread>
#include <utility>

#include "envpot_internal.h"
#include "screen_math.h"
#include "update_internal.h"

namespace envpot {

// Estimated relative cost of one point-pair by L and of one point-nucleus.
const double kCost32[kLMax + 1] = {1.0, 1.5, 2.6, 4.4, 7.5};
const double kCost64[kLMax + 1] = {1.0, 1.4, 2.3, 3.8, 6.3};
const double kCostNuc = 0.6;
// Extra cost of a cluster per unit of member cost: the share of waves that
// have some point inside the cluster's far-field radius.
const double kClusterNearShare = 0.1;

namespace {

double pair_r2far(const PairList& pl, int64_t k, bool fp64, const BoysParams& bp) {
    const int L = pl.L[k];
    return sm::rec_r2far(fp64 ? bp.tfar64[L] : double(bp.tfar32[L]), pl.p[k], fp64);  // as stored in the record
}

void append_pair(const PairList& pl, int64_t k, bool fp64, const BoysParams& bp, std::vector<uint32_t>& rec) {
    double h[35];
    const int L = pl.L[k], nc = kNComp[L];
    const double p = pl.p[k];
    const double c1 = sm::rec_c1(p);
    const double* D = &pl.D[pl.d_off[k]];
    far_coefs(L, D, h);
    const size_t o = rec.size();
    if (fp64) {
        rec.resize(o + rec64_words(L), 0u);
        double* r = reinterpret_cast<double*>(&rec[o]);
        r[0] = pl.center[3 * k];
        r[1] = pl.center[3 * k + 1];
        r[2] = pl.center[3 * k + 2];
        r[3] = sm::rec_r2far(bp.tfar64[L], p, true);
        r[4] = p;
        r[5] = c1;
        for (int c = 0; c < nc; ++c) r[kRec64Head + c] = h[c];
        for (int c = 0; c < nc; ++c) r[kRec64Head + nc + c] = D[c];
    } else {
        rec.resize(o + rec32_words(L), 0u);
        double* r = reinterpret_cast<double*>(&rec[o]);
        r[0] = pl.center[3 * k];
        r[1] = pl.center[3 * k + 1];
        r[2] = pl.center[3 * k + 2];
        float* f = reinterpret_cast<float*>(&rec[o + 6]);
        f[0] = float(sm::rec_r2far(double(bp.tfar32[L]), p, false));
        f[1] = float(p);
        f[2] = float(c1);
        for (int c = 0; c < nc; ++c) f[3 + c] = float(h[c]);
        for (int c = 0; c < nc; ++c) f[3 + nc + c] = float(D[c]);
    }
}

struct Cluster {
    std::vector<int64_t> members;  // pair indices, sorted by (L, index)
    int L = 0;                     // largest member L
};

// Records, segments and clusters of one fragment group, with word offsets
// relative to the group's first record (the merge adds the group's base).
struct GroupPack {
    std::vector<uint32_t> rec;
    std::vector<Segment> base;
    std::vector<double> unit_cost;
    std::vector<std::pair<int64_t, int64_t>> pair_word;  // (pair, local word)
    std::vector<int64_t> cl_word;                        // local
    std::vector<int32_t> cl_L;
    std::vector<int64_t> cl_members;
    std::vector<int64_t> cl_count;
    int64_t n_clusters = 0, n_members = 0;
};

void pack_group(const PairList& pl, int g, bool fp64, const BoysParams& bp, bool merge, const double* edges,
                int bands, bool want_map, GroupPack& gp) {
    const double* w = fp64 ? kCost64 : kCost32;
    const int64_t b = pl.group_pair_begin[g], e = pl.group_pair_begin[g + 1];
    std::vector<int64_t> ord;
    std::vector<Cluster> clusters;
    {
        std::map<std::pair<int, int>, std::vector<int64_t>> by_key;  // (atom, band)
        for (int64_t k = b; k < e; ++k) {
            if (merge && pl.atom1[k] >= 0) {
                const int band = sm::band_of(pair_r2far(pl, k, fp64, bp), edges, bands);
                by_key[{pl.atom1[k], band}].push_back(k);
            } else {
                ord.push_back(k);
            }
        }
        for (auto& kv : by_key) {
            Cluster c;
            c.members = kv.second;
            double cost = 0.0;
            for (int64_t k : c.members) {
                c.L = std::max(c.L, pl.L[k]);
                cost += w[pl.L[k]];
            }
            // worth it only if the merged evaluation is clearly cheaper than the members
            if (c.members.size() >= 2 && cost > 1.25 * w[c.L]) {
                std::stable_sort(c.members.begin(), c.members.end(),
                                 [&](int64_t x, int64_t y) { return pl.L[x] < pl.L[y]; });
                clusters.push_back(std::move(c));
            } else {
                ord.insert(ord.end(), c.members.begin(), c.members.end());
            }
        }
    }
    {
        // order by (L, index): mark the group's ordinary pairs, then one
        // pass per L in index order
        std::vector<uint8_t> in_ord(size_t(e - b), 0);
        for (int64_t k : ord) in_ord[size_t(k - b)] = 1;
        ord.clear();
        for (int L = 0; L <= kLMax; ++L)
            for (int64_t k = b; k < e; ++k)
                if (in_ord[size_t(k - b)] && pl.L[k] == L) ord.push_back(k);
    }
    std::stable_sort(clusters.begin(), clusters.end(),
                     [](const Cluster& x, const Cluster& y) { return x.L < y.L; });

    std::vector<uint32_t>& rec = gp.rec;
    // ordinary pairs, one segment per L
    for (size_t i = 0; i < ord.size();) {
        size_t j = i;
        while (j < ord.size() && pl.L[ord[j]] == pl.L[ord[i]]) ++j;
        Segment sg{};
        sg.L = pl.L[ord[i]];
        sg.n_pairs = int32_t(j - i);
        sg.rec_off = int64_t(rec.size());
        for (size_t q = i; q < j; ++q) {
            if (want_map) gp.pair_word.push_back({ord[q], int64_t(rec.size())});
            append_pair(pl, ord[q], fp64, bp, rec);
        }
        gp.base.push_back(sg);
        gp.unit_cost.push_back(w[sg.L]);
        i = j;
    }
    // clusters, one segment per merged L; their members follow all of them
    if (!clusters.empty()) {
        int64_t cl_words = 0;
        for (const Cluster& c : clusters) cl_words += fp64 ? cl64_words(c.L) : cl32_words(c.L);
        int64_t member_word = int64_t(rec.size()) + cl_words;
        std::vector<int64_t> member_off(clusters.size());
        for (size_t i = 0; i < clusters.size(); ++i) {
            member_off[i] = member_word;
            for (int64_t k : clusters[i].members) member_word += fp64 ? rec64_words(pl.L[k]) : rec32_words(pl.L[k]);
        }
        for (size_t i = 0; i < clusters.size();) {
            size_t j = i;
            while (j < clusters.size() && clusters[j].L == clusters[i].L) ++j;
            Segment sg{};
            sg.L = clusters[i].L;
            sg.n_pairs = int32_t(j - i);
            sg.rec_off = int64_t(rec.size());
            sg.flags = kSegCluster;
            double cost = 0.0;
            for (size_t q = i; q < j; ++q) {
                const Cluster& c = clusters[q];
                const int Lc = c.L, nc = kNComp[Lc];
                double hsum[35] = {0.0}, hm[35];
                double r2far = 0.0;
                int64_t off[kLMax + 1] = {0}, cnt[kLMax + 1] = {0};
                int64_t word = member_off[q];
                double mcost = 0.0;
                for (int64_t k : c.members) {
                    const int Lm = pl.L[k];
                    if (cnt[Lm] == 0) off[Lm] = word;
                    ++cnt[Lm];
                    word += fp64 ? rec64_words(Lm) : rec32_words(Lm);
                    r2far = std::max(r2far, pair_r2far(pl, k, fp64, bp));
                    mcost += w[Lm];
                    far_coefs(Lm, &pl.D[pl.d_off[k]], hm);
                    // same (a, b, c) exponents, re-indexed from L = Lm to L = Lc
                    for (int a = 0, im = 0; a <= Lm; ++a)
                        for (int bb = 0; bb <= Lm - a; ++bb)
                            for (int cc = 0; cc <= Lm - a - bb; ++cc, ++im)
                                hsum[hermite_index(Lc, a, bb, cc)] += hm[im];
                }
                cost += sm::cluster_term(w[Lc], kClusterNearShare, mcost);
                uint32_t mask = 0;
                for (int L = 0; L <= kLMax; ++L) mask |= cnt[L] ? (1u << L) : 0u;
                const int64_t k0 = c.members[0];
                const size_t o = rec.size();
                if (want_map) {
                    gp.cl_word.push_back(int64_t(o));
                    gp.cl_L.push_back(Lc);
                    gp.cl_members.insert(gp.cl_members.end(), c.members.begin(), c.members.end());
                    gp.cl_count.push_back(int64_t(c.members.size()));
                }
                // member-table offsets are local here (the merge adds the group's base)
                if (fp64) {
                    rec.resize(o + cl64_words(Lc), 0u);
                    double* r = reinterpret_cast<double*>(&rec[o]);
                    r[0] = pl.center[3 * k0];
                    r[1] = pl.center[3 * k0 + 1];
                    r[2] = pl.center[3 * k0 + 2];
                    r[3] = r2far;
                    rec[o + kClMask64] = mask;
                    for (int L = 0; L <= kLMax; ++L) {
                        rec[o + kClTable64 + 2 * L] = uint32_t(off[L]);
                        rec[o + kClTable64 + 2 * L + 1] = uint32_t(cnt[L]);
                    }
                    for (int t = 0; t < nc; ++t) r[kClHead64 + t] = hsum[t];
                } else {
                    rec.resize(o + cl32_words(Lc), 0u);
                    double* r = reinterpret_cast<double*>(&rec[o]);
                    r[0] = pl.center[3 * k0];
                    r[1] = pl.center[3 * k0 + 1];
                    r[2] = pl.center[3 * k0 + 2];
                    reinterpret_cast<float*>(&rec[o])[6] = float(r2far);  // exact: a stored float
                    rec[o + kClMask32] = mask;
                    for (int L = 0; L <= kLMax; ++L) {
                        rec[o + kClTable32 + 2 * L] = uint32_t(off[L]);
                        rec[o + kClTable32 + 2 * L + 1] = uint32_t(cnt[L]);
                    }
                    float* f = reinterpret_cast<float*>(&rec[o + kClHead32]);
                    for (int t = 0; t < nc; ++t) f[t] = float(hsum[t]);
                }
                ++gp.n_clusters;
                gp.n_members += int64_t(c.members.size());
            }
            gp.base.push_back(sg);
            gp.unit_cost.push_back(cost / double(sg.n_pairs));
            i = j;
        }
        for (const Cluster& c : clusters)
            for (int64_t k : c.members) {
                if (want_map) gp.pair_word.push_back({k, int64_t(rec.size())});
                append_pair(pl, k, fp64, bp, rec);
            }
    }
    const int nb = pl.group_nuc_begin[g], ne = pl.group_nuc_end[g];
    if (gp.base.empty() && ne > nb) {
        Segment sg{};
        sg.rec_off = int64_t(rec.size());
        gp.base.push_back(sg);
        gp.unit_cost.push_back(0.0);
    }
    if (!gp.base.empty()) {
        gp.base.front().nuc_begin = nb;
        gp.base.front().nuc_end = ne;
        gp.base.back().flags |= kSegEndGroup;
    }
}

}  // namespace

int radius_bands() {
    const char* e = std::getenv("ENVPOT_BANDS");
    const int v = e ? std::atoi(e) : 0;
    return (v >= 1 && v <= kMaxBands) ? v : 4;
}

void radius_band_edges(double vmin, double vmax, int bands, double* edges) {
    // log-uniform bands between the smallest and the largest r2far
    for (int j = 0; j < kMaxBands; ++j) edges[j] = 0.0;
    if (!(vmin > 0.0) || !(vmax >= vmin) || !std::isfinite(vmax)) return;
    const double lo = std::log(vmin), hi = std::log(vmax);
    const double w = (hi > lo) ? (hi - lo) / bands : 1.0;
    for (int j = 1; j < bands; ++j) edges[j] = std::exp(lo + j * w);
}

void pack_layout(const PairList& pl, bool fp64, const BoysParams& bp, bool merge, Layout& out) {
    pack_layout(pl, fp64, bp, merge, out, nullptr);
}

void pack_layout(const PairList& pl, bool fp64, const BoysParams& bp, bool merge, Layout& out,
                 LayoutMap* map) {
    out.rec.clear();
    out.base.clear();
    out.unit_cost.clear();
    out.n_clusters = out.n_members = 0;
    const int64_t npairs = int64_t(pl.L.size());

    // radius band edges over all one-centre pairs
    double vmin = std::numeric_limits<double>::infinity(), vmax = -vmin;
    if (merge) {
        for (int64_t k = 0; k < npairs; ++k) {
            if (pl.atom1[k] < 0) continue;
            const double v = pair_r2far(pl, k, fp64, bp);
            vmin = std::min(vmin, v);
            vmax = std::max(vmax, v);
        }
    }
    const int bands = radius_bands();
    double edges[kMaxBands];
    radius_band_edges(vmin, vmax, bands, edges);

    // groups in parallel, each with local offsets
    const int ng = pl.n_groups;
    std::vector<GroupPack> packs(ng);
    {
        std::atomic<int> next{0};
        const unsigned nt = std::max(1u, std::min({16u, std::thread::hardware_concurrency(), unsigned(std::max(ng, 1))}));
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&]() {
                for (;;) {
                    const int g = next.fetch_add(1);
                    if (g >= ng) break;
                    pack_group(pl, g, fp64, bp, merge, edges, bands, map != nullptr, packs[g]);
                }
            });
        for (auto& t : th) t.join();
    }
    std::vector<int64_t> gbase(size_t(ng) + 1, 0);
    for (int g = 0; g < ng; ++g) gbase[g + 1] = gbase[g] + int64_t(packs[g].rec.size());
    if (merge && gbase[ng] > int64_t(UINT32_MAX)) {  // member offsets are 32-bit words
        pack_layout(pl, fp64, bp, false, out, map);
        return;
    }
    out.rec.resize(size_t(gbase[ng]));
    if (map) {
        *map = LayoutMap();
        map->pair_word.assign(size_t(npairs), -1);
        map->cl_begin.push_back(0);
    }
    for (int g = 0; g < ng; ++g) {
        GroupPack& gp = packs[g];
        const int64_t base = gbase[g];
        std::copy(gp.rec.begin(), gp.rec.end(), out.rec.begin() + base);
        for (size_t i = 0; i < gp.base.size(); ++i) {
            Segment sg = gp.base[i];
            sg.rec_off += base;
            out.base.push_back(sg);
            out.unit_cost.push_back(gp.unit_cost[i]);
            if (sg.flags & kSegCluster) {  // member tables: local -> absolute offsets
                const int cw = fp64 ? cl64_words(sg.L) : cl32_words(sg.L);
                const int tab = fp64 ? kClTable64 : kClTable32, mk = fp64 ? kClMask64 : kClMask32;
                for (int c = 0; c < sg.n_pairs; ++c) {
                    uint32_t* r = &out.rec[size_t(sg.rec_off + int64_t(c) * cw)];
                    for (int L = 0; L <= kLMax; ++L)
                        if (r[mk] & (1u << L)) r[tab + 2 * L] = uint32_t(int64_t(r[tab + 2 * L]) + base);
                }
            }
        }
        out.n_clusters += gp.n_clusters;
        out.n_members += gp.n_members;
        if (map) {
            for (const auto& pw : gp.pair_word) map->pair_word[pw.first] = pw.second + base;
            size_t m = 0;
            for (size_t c = 0; c < gp.cl_word.size(); ++c) {
                map->cl_word.push_back(gp.cl_word[c] + base);
                map->cl_L.push_back(gp.cl_L[c]);
                map->cl_members.insert(map->cl_members.end(), gp.cl_members.begin() + m,
                                       gp.cl_members.begin() + m + gp.cl_count[c]);
                m += size_t(gp.cl_count[c]);
                map->cl_begin.push_back(int64_t(map->cl_members.size()));
            }
        }
        GroupPack().rec.swap(gp.rec);
    }
}

void split_layout(const Layout& lay, int S, bool fp64, std::vector<Segment>& segs,
                  std::vector<int32_t>& split) {
    auto unit_words = [&](const Segment& s) -> int64_t {
        if (s.flags & kSegCluster) return fp64 ? cl64_words(s.L) : cl32_words(s.L);
        return fp64 ? rec64_words(s.L) : rec32_words(s.L);
    };
    double total = 0.0;
    for (size_t i = 0; i < lay.base.size(); ++i) {
        const Segment& s = lay.base[i];
        total += s.n_pairs * lay.unit_cost[i] + (s.nuc_end - s.nuc_begin) * kCostNuc;
    }
    segs.clear();
    split.assign(1, 0);
    const double target = total / S;
    double acc = 0.0;
    int cur = 0;
    for (size_t i = 0; i < lay.base.size(); ++i) {
        Segment rem = lay.base[i];
        const double uc = lay.unit_cost[i];
        double nucc = (rem.nuc_end - rem.nuc_begin) * kCostNuc;
        for (;;) {
            const double cost = nucc + rem.n_pairs * uc;
            const double boundary = (cur + 1) * target;
            if (cur < S - 1 && rem.n_pairs > 0 && acc + cost > boundary) {
                int64_t k = uc > 0.0 ? int64_t(std::floor((boundary - acc - nucc) / uc)) : rem.n_pairs;
                k = std::max<int64_t>(0, std::min<int64_t>(k, rem.n_pairs));
                if (k > 0 || nucc > 0) {
                    Segment a = rem;
                    a.n_pairs = int32_t(k);
                    a.flags = rem.flags & kSegCluster;
                    segs.push_back(a);
                }
                acc += nucc + k * uc;
                rem.rec_off += k * unit_words(rem);
                rem.n_pairs -= int32_t(k);
                rem.nuc_begin = rem.nuc_end;
                nucc = 0.0;
                split.push_back(int32_t(segs.size()));
                ++cur;
                continue;
            }
            if (rem.n_pairs > 0 || rem.nuc_end > rem.nuc_begin || (rem.flags & kSegEndGroup))
                segs.push_back(rem);
            acc += cost;
            break;
        }
    }
    while (int(split.size()) < S + 1) split.push_back(int32_t(segs.size()));
}

}  // namespace envpot
