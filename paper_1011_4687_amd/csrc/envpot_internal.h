// Internal layout shared by the host pair-list builder, the launcher and the
// gfx950 kernels.  Nothing here is part of the C ABI.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "env_potential.h"

namespace envpot {

constexpr int kLMax = 4;                  // largest L = l_I + l_J (d-d pairs)
constexpr int kNComp[kLMax + 1] = {1, 4, 10, 20, 35};
constexpr int kMaxSplitLog2 = 8;          // split-pair factors 1, 2, 4, ..., 256
constexpr int kBlock = 256;               // threads per workgroup of the point kernels

// Boys tables: grid T_k = k / 8, k = 0..rows-1.
constexpr int kBoysGridInv = 8;
constexpr int kBoysRowF32 = 12;           // floats per row: F_0..F_9 (+2 pad)
constexpr int kBoysTaylorF32 = 6;         // Taylor terms j = 0..5, |dT| <= 1/16
constexpr int kBoysRowF64 = 14;           // doubles per row: F_0..F_13
constexpr int kBoysTaylorF64 = 10;        // Taylor terms j = 0..9
constexpr int kBoysMaxRowsF32 = 8 * 40 + 1;

// Index of Hermite component (t,u,v), t+u+v <= L, in the order t ascending,
// then u, then v (the order of the generated recursion and of D in a record).
constexpr int hermite_index(int L, int t, int u, int v) {
    int idx = 0;
    for (int a = 0; a <= L; ++a)
        for (int b = 0; b <= L - a; ++b)
            for (int c = 0; c <= L - a - b; ++c) {
                if (a == t && b == u && c == v) return idx;
                ++idx;
            }
    return -1;
}

// Pair-record sizes in 4-byte words.
//  FP32C record: Px, Py, Pz (double); r2far, p, c1 (float); h[ncomp], D[ncomp] (float)
//  FP64  record: Px, Py, Pz, r2far, p, c1 (double); h[ncomp], D[ncomp] (double)
// D is the Hermite density scaled by (pi/p)^{3/2}; c1 = 2 sqrt(p/pi);
// r2far = tfar[L]/p is the squared distance beyond which the far-field form
// applies; h are the far-field polynomial coefficients (see far_coefs).
// Records are padded to an even number of words (8-byte aligned doubles).
constexpr int rec32_words(int L) { return ((9 + 2 * kNComp[L]) + 1) & ~1; }
constexpr int rec64_words(int L) { return 2 * (6 + 2 * kNComp[L]); }
constexpr int kRec32Head = 9;   // words before h in an FP32C record
constexpr int kRec64Head = 6;   // doubles before h in an FP64 record

// Same-centre clusters.  A pair whose two shells sit on one atom has its
// product centre exactly at that atom, so in the far field such pairs are
// finite multipoles about one point and their polynomial coefficients h add
// up exactly.  A cluster record holds the merged coefficients (at the largest
// L of its members) and the largest far-field radius of its members; a wave
// whose points are all beyond that radius evaluates the cluster once, any
// other wave evaluates the members (ordinary pair records) one by one.
//  FP32C cluster: P (3 doubles); r2far (float); member mask (bit L set when
//                 there are members of that L); member table (word offset,
//                 count) for L = 0..4; h[ncomp(Lc)] (float)
//  FP64  cluster: P, r2far (doubles); mask, pad; member table; h (double)
constexpr int kClMask32 = 7, kClTable32 = 8, kClHead32 = 18;  // in words
constexpr int kClMask64 = 8, kClTable64 = 10, kClHead64 = 10; // words, words, doubles
constexpr int cl32_words(int L) { return ((kClHead32 + kNComp[L]) + 1) & ~1; }
constexpr int cl64_words(int L) { return 2 * (kClHead64 + kNComp[L]); }

// A run of pairs (or of clusters) of one L inside one fragment group, plus
// (on the group's first segment) the group's nuclei.
struct Segment {
    int32_t L;           // pair L, or the clusters' merged L
    int32_t n_pairs;     // pairs, or clusters when flags has kSegCluster
    int64_t rec_off;     // offset of the first record, in 4-byte words
    int32_t nuc_begin;   // nuclei [nuc_begin, nuc_end) of the device array
    int32_t nuc_end;
    int32_t flags;       // kSegEndGroup: fold nuclear-minus-electronic sum afterwards
    int32_t box;         // the unsplit segment it comes from: its box in EvalArgs::boxes
};

// Box of an unsplit segment, 8 doubles: the smallest and largest x, y, z of
// its pair (or cluster) centres, the largest r2far (as stored), and a pad.
// A wave whose every point is farther from the box than sqrt(r2far max)
// (with a margin of 1e-6 relative, more than the FP32 rounding of |X|^2)
// has all its point-pairs of the segment in the far field, so the kernels
// run them without the per-pair near test (FP32C: with X from the wave
// origin where every point is also at least 2|C - O| from the box).
// Empty segments get r2far max = +inf.
constexpr int kSegBoxWords = 8;
constexpr int32_t kSegEndGroup = 1;
constexpr int32_t kSegCluster = 2;

struct BoysParams {
    float tfar32[kLMax + 1];   // FP32 path: asymptotic form for T >= tfar32[L]
    int32_t rows32;
    double tfar64[kLMax + 1];  // FP64 path
    int32_t rows64;
    int32_t pad;
};

struct EvalArgs {
    const double* pts;      // n x 3
    int64_t n;
    const Segment* segs;    // segments of the chosen split factor
    const int32_t* split;   // S+1 offsets into segs
    const uint32_t* rec;    // pair records of the handle's precision
    const double* nuc;      // nuclei, 4 doubles each (x, y, z, Z)
    const void* boys;       // Boys table of the handle's precision
    double* out;            // S == 1: V; S > 1: partial sums [S][n]
    const double* boxes;    // per unsplit segment (Segment::box), or nullptr: test every pair
    BoysParams bp;
};

// One work item of the persistent batched kernel.
struct BatchItem {
    int32_t inst;     // instance (index into BatchArgs::args)
    int32_t split;    // pair split of that instance
    int64_t pblock;   // point block of that instance
};

struct BatchArgs {
    const EvalArgs* args;         // per instance (out = its partial buffer when S > 1)
    const BatchItem* items;       // sorted by decreasing cost
    int64_t n_items;
    unsigned long long* counter;  // queue head, zeroed by a kernel before each launch
    const void* boys;             // Boys table of the common precision
    int32_t rows32;
    int32_t pad;
};

// A single evaluation whose point count is known only on the device (the
// gated-out points of a surrogate evaluation).  The persistent kernel reads
// m, picks the split factor 2^k from it (the rule of the host launcher's
// default shape, capped so that 2^k * m partials fit part_cap), and drains
// the (point block, split) items of that shape through a work counter; the
// sum kernel recomputes the same k and adds the partials.
struct DevSizedArgs {
    EvalArgs a;                    // pts, rec, nuc, boys, bp; out = partials [2^k][m]; n ignored
    const int64_t* m;              // device: number of points
    const Segment* segs_all;       // every split factor's segment table
    const int32_t* split_all;
    int64_t seg_off[kMaxSplitLog2 + 1];
    int64_t split_off[kMaxSplitLog2 + 1];
    int64_t part_cap;              // float64 elements of a.out
    int64_t want_waves;            // waves the split factor aims for
    unsigned long long* counter;   // zeroed by a kernel before the launch
};

struct SumDesc {                  // fixed-order sum of S partials of one instance
    const double* part;
    double* out;
    int64_t n;
    int32_t S;
    int32_t pad;
};

// Host-side result of the pair-list build.
struct PairList {
    int nbf = 0;
    int n_groups = 0;
    bool has_cross = false;
    // pairs in final order (group, L), SoA over pairs
    std::vector<int32_t> L, group;
    std::vector<double> center;   // 3 per pair
    std::vector<double> p;
    std::vector<int32_t> atom1;   // per pair: atom of both shells (one-centre pair) or -1
    std::vector<double> D;        // ncomp(L) per pair, pair k starts at d_off[k]
    std::vector<int64_t> d_off;   // n_pairs + 1
    std::vector<double> nuc;      // 4 per nucleus, grouped
    std::vector<int32_t> group_nuc_begin, group_nuc_end;  // per group
    std::vector<int64_t> group_pair_begin;                // per group (+1)
    int64_t n_unscreened = 0;
    double screened_bound = 0.0;
    double electrons = 0.0;
    double nuclear_charge = 0.0;
};

// Build the screened, folded primitive-pair list.  Returns ENV_OK or an error.
env_status build_pair_list(const env_nucleus* nuclei, int32_t n_nuclei,
                           const env_shell* shells, int32_t n_shells,
                           const env_density* P, const env_options& opt, PairList& out);

// Device image of a pair list in one precision: records (pair records,
// cluster records and the clusters' member records) and the unsplit segments.
struct Layout {
    std::vector<uint32_t> rec;
    std::vector<Segment> base;
    std::vector<double> unit_cost;   // per base segment: estimated cost of one pair / cluster
    int64_t n_clusters = 0;
    int64_t n_members = 0;           // pairs inside clusters
};

// Pack the records of one precision; with merge, one-centre pairs are grouped
// into clusters by atom and far-field radius band.
void pack_layout(const PairList& pl, bool fp64, const BoysParams& bp, bool merge, Layout& out);

// Segment table for split factor S: segments (cut where needed) and S+1
// offsets, balancing the estimated cost of pairs, clusters and nuclei.
void split_layout(const Layout& lay, int S, bool fp64, std::vector<Segment>& segs,
                  std::vector<int32_t>& split);

// Far-field coefficients: for X = P - C with p |X|^2 >= tfar[L],
//   sum_tuv D_tuv d^t_X d^u_Y d^v_Z (1/|X|) = (1/|X|) sum_abc h_abc x^a y^b z^c,
//   x = X/|X|^2, y = Y/|X|^2, z = Z/|X|^2   (both in the hermite_index order).
void far_coefs(int L, const double* D, double* h);

// Boys tables (host FP64/long double) and the far-field thresholds.
void build_boys_tables(std::vector<float>& t32, std::vector<double>& t64, BoysParams& bp);

// Kernel launchers (kernels.hip).
int launch_potential(const EvalArgs& a, int S, int precision, int np, void* stream);
int launch_sum_splits(const double* partial, int S, int64_t n, double* out, void* stream);
// Boxes (kSegBoxWords doubles each) of the unsplit segments segs[0, n_segs),
// one workgroup per segment; empty segments get r2far max = +inf.
int launch_segment_boxes(const Segment* segs, int n_segs, const uint32_t* rec, int fp64, double* boxes,
                         void* stream);
int launch_persistent(const BatchArgs& b, int grid, int precision, int np, void* stream);
int launch_sum_multi(const SumDesc* d, int n_desc, int64_t max_n, void* stream);
int persistent_grid(int precision, int np, int cu_count);
int launch_potential_devsized(const DevSizedArgs& d, int grid, int precision, int np, void* stream);
int launch_sum_devsized(const DevSizedArgs& d, int np, int64_t n_max, double* out, void* stream);
int devsized_klog(int64_t m, int np, int64_t want_waves, int64_t part_cap);
int devsized_grid(int precision, int cu_count);

}  // namespace envpot
