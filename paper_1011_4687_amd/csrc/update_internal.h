// Incremental update of an environment's density on the device: the pair
// list (screening, order, clusters, segments) depends on the geometry, the
// basis and which density blocks are nonzero, not on the density values, so
// a new density with the same block pattern only changes every record's
// Hermite density D and far-field coefficients h (and the clusters' merged
// h).  The device refolds them from the pair's primitives and the new
// density blocks.  Not part of the C ABI.
#pragma once

#include <cstdint>
#include <vector>

#include "envpot_internal.h"

namespace envpot {

// Where the pairs of a PairList came from, and the basis data needed to
// fold a density block again (filled by build_pair_list on request).
struct PairSources {
    // density blocks (I <= J) of the build, in build order
    std::vector<int32_t> blk_I, blk_J;
    // per pair, PairList order: block index and primitives
    std::vector<int32_t> pair_blk, pair_ia, pair_ib;
    // screened-out pairs whose charges enter the neutral scaling (ENV_NEUTRALIZE)
    std::vector<int32_t> drop_blk, drop_ia, drop_ib, drop_group;
    // basis: per shell l, atom, first basis function, first primitive, first
    // normalised coefficient; per basis function the contraction scale; per
    // primitive the exponent; per (primitive, component) c N
    std::vector<int32_t> shell_l, shell_atom, bf0;
    std::vector<int64_t> poff, noff;
    std::vector<double> cscale, exps, cnorm, atom_xyz;
    std::vector<double> group_charge;  // nuclear charge per group
    bool neutralize = false;
    bool device_fold = false;  // set by the caller: leave D (and charges) to the device
};

// Where each pair's record sits in a Layout, and the clusters' members.
struct LayoutMap {
    std::vector<int64_t> pair_word;   // per pair: word offset of its record
    std::vector<int64_t> cl_word;     // per cluster: word offset of its record
    std::vector<int32_t> cl_L;        // per cluster: merged L
    std::vector<int64_t> cl_begin;    // per cluster + 1: range in cl_members
    std::vector<int64_t> cl_members;  // pair indices, in merge order
};

// The enumeration plan of a build, from the host's parse of the inputs
// (validation, density blocks, symmetry, fragment groups, nuclei): the
// device build enumerates, screens and orders the primitive pairs from it.
struct BlockPlan {
    // enumerated blocks: groups ascending, the blocks of a group by (I, J);
    // a block's primitive pairs in the order ia, then ib (ib >= ia when I == J)
    std::vector<int32_t> enum_blk;    // block index (build order, as in PairSources)
    std::vector<int32_t> enum_group;  // fragment group of the block
    std::vector<int64_t> enum_first;  // first primitive pair of the block; last entry: the total
    std::vector<double> blk_maxabs;   // per block: largest |weight|
    std::vector<int32_t> shell_nprim; // per shell
    std::vector<double> coefs, n0;    // per primitive: contraction coefficient, (2 alpha / pi)^{3/4}
    double thr = 0.0;
    bool screen = false;
};

// With plan != nullptr the build stops before the pairs: it fills plan, src
// and the pair list's fields that do not depend on pairs (nbf, groups,
// nuclei, n_unscreened) and leaves the pairs to the device build.
env_status build_pair_list(const env_nucleus* nuclei, int32_t n_nuclei, const env_shell* shells,
                           int32_t n_shells, const env_density* P, const env_options& opt, PairList& out,
                           PairSources* src, BlockPlan* plan = nullptr);

void pack_layout(const PairList& pl, bool fp64, const BoysParams& bp, bool merge, Layout& out,
                 LayoutMap* map);

// Far-field radius bands of the same-centre clusters: the number of bands
// (ENVPOT_BANDS, 1..kMaxBands, default 4) and their edges, log-uniform between
// the smallest and the largest r2far of the one-centre pairs (edges[1] ..
// edges[bands-1]; a pair's band is sm::band_of).
constexpr int kMaxBands = 8;
int radius_bands();
void radius_band_edges(double vmin, double vmax, int bands, double* edges);

// Estimated relative cost of one point-pair by L, of one point-nucleus, and
// the share of a cluster's member cost that its segment is charged.
extern const double kCost32[kLMax + 1];
extern const double kCost64[kLMax + 1];
extern const double kCostNuc;
extern const double kClusterNearShare;

// Device records of one pair and one cluster for the fold kernels.
struct UpdPair {
    int32_t blk;
    int16_t ia, ib;
    int32_t group;
    int32_t L;
    int64_t word;
};
struct UpdShell {
    double A[3];
    int32_t l;
    int32_t pad;
    int64_t poff, noff;
};
struct UpdCluster {
    int64_t word;
    int64_t begin, end;   // range in the member list
    int32_t L;
    int32_t pad;
};

struct UpdateArgs {
    const UpdPair* pairs;       // pairs (kept), then screened-out ones (charges only)
    int64_t n_pairs;
    int64_t n_drop;
    const UpdShell* shells;
    const int32_t* blk;         // per block: I, J
    const int64_t* woff;        // per block: first weight (nI x nJ weights, row-major)
    const double* exps;
    const double* cnorm;
    const double* W;            // block weights of the new density
    const double* scale;        // per group
    const double* M;            // far-field matrices h = M_L D, L = 0..4
    const UpdCluster* clusters;
    const int64_t* members;     // pair indices
    const int64_t* moff;        // per member + 1: first word of its h in hm
    double* hm;                 // members' far-field coefficients (FP64)
    int64_t n_members;
    int64_t n_clusters;
    uint32_t* rec;              // the handle's records (updated in place)
    double* charge;             // per pair and dropped pair: electron count
    int32_t fp64;
    int32_t pad;
};

struct UpdateState {
    int64_t n_pairs = 0, n_drop = 0, n_clusters = 0, n_members = 0;
    int n_groups = 0, nbf = 0, n_shells = 0;
    bool neutralize = false;
    std::vector<int32_t> shell_l, bf0, shell_of_bf;
    std::vector<double> cscale, group_charge;
    std::vector<int64_t> group_pair_begin;
    std::vector<int32_t> drop_group;
    // per shell I: the blocks it takes part in, by partner shell J ascending
    // (adj_tr: the block is (J, I), its weights transposed)
    std::vector<int64_t> adj_begin;
    std::vector<int32_t> adj_J, adj_blk;
    std::vector<uint8_t> adj_tr;
    std::vector<int32_t> blk_I, blk_J;
    std::vector<int64_t> woff;        // per block + 1
    int64_t n_blocks = 0;
    // device
    UpdPair* d_pairs = nullptr;
    UpdShell* d_shells = nullptr;
    int32_t* d_blk = nullptr;
    int64_t* d_woff = nullptr;
    double* d_exps = nullptr;
    double* d_cnorm = nullptr;
    double* d_W = nullptr;
    double* d_scale = nullptr;
    double* d_M = nullptr;
    UpdCluster* d_clusters = nullptr;
    int64_t* d_members = nullptr;
    int64_t* d_moff = nullptr;
    double* d_hm = nullptr;
    double* d_charge = nullptr;
    // device parse of a CSR density (ParseArgs): the basis and block lists
    int32_t* d_shell_of_bf = nullptr;
    int32_t* d_bf0 = nullptr;
    int32_t* d_shell_l = nullptr;
    int64_t* d_adj_begin = nullptr;
    int32_t* d_adj_J = nullptr;
    int32_t* d_adj_blk = nullptr;
    uint8_t* d_adj_tr = nullptr;
    double* d_cscale = nullptr;
    double* d_Wd = nullptr;   // the density's elements by block, as given and transposed
    double* d_Wt = nullptr;
    int32_t* d_err = nullptr;
    // per-group electron counts on the device: pair and dropped-pair ranges
    // of every group, and the two sums per group
    int64_t* d_gpb = nullptr;     // per group + 1 (group_pair_begin)
    int64_t* d_dropb = nullptr;   // per group + 1 (dropped pairs are group-major)
    double* d_gq = nullptr;       // per group: kept, dropped
    int64_t device_bytes = 0;
};

// A CSR density parsed on the device into the block weights W: one thread
// per stored element finds its block through the row shell's block list
// (binary search by partner shell) and adds the value at its place, as
// given (Wd) or transposed (Wt; a stored element occurs once, so the sum
// is the value itself); then one thread per weight checks the symmetry
// against the transposed element and forms f P s_x s_y.  err collects
// bit 1 (column out of range or non-finite value), bit 2 (an element of a
// block the build did not see), bit 4 (asymmetric).
struct ParseArgs {
    const int64_t* row_ptr;   // nbf + 1
    const int32_t* col;       // nnz
    const double* val;        // nnz
    int64_t nnz;
    int32_t nbf;
    int32_t pad;
    const int32_t* shell_of_bf;
    const int32_t* bf0;       // per shell + 1
    const int32_t* shell_l;
    const int64_t* adj_begin; // per shell + 1
    const int32_t* adj_J;
    const int32_t* adj_blk;
    const uint8_t* adj_tr;
    const int32_t* blk;       // per block: I, J
    const int64_t* woff;      // per block + 1
    int64_t n_blocks;
    const double* cscale;     // per basis function
    double* Wd;
    double* Wt;
    double* W;
    int32_t* err;
};
int launch_parse_csr(const ParseArgs& a, void* stream);
int launch_block_weights(const ParseArgs& a, int64_t total, void* stream);  // total = woff[n_blocks]

// Offsets of the far-field matrices M_L (ncomp x ncomp, row-major) in d_M.
constexpr int kFarMatOff[kLMax + 2] = {0, 1, 17, 117, 517, 1742};

// Device tables of the update for a handle just built (current device);
// nullptr with *st == ENV_OK when the input does not fit them.
UpdateState* make_update_state(const PairList& pl, const PairSources& src, const LayoutMap& map,
                               env_status* st);
struct DevBuild;
// The same for a device-built pair list (takes over db's fold tables).
UpdateState* make_update_state_device(const PairList& meta, const PairSources& src, DevBuild& db,
                                      env_status* st);
void free_update_state(UpdateState* u);

int launch_update_charges(const UpdateArgs& a, void* stream);
// Per group g: gq[2g] = sum of the kept pairs' charges, gq[2g+1] = sum of
// the dropped pairs' charges, each in a fixed order (one workgroup per group).
int launch_group_charges(const double* charge, const int64_t* gpb, const int64_t* dropb, int64_t n_pairs,
                         int n_groups, double* gq, void* stream);
int launch_update_pairs(const UpdateArgs& a, void* stream);
int launch_update_members(const UpdateArgs& a, void* stream);
int launch_update_clusters(const UpdateArgs& a, void* stream);

}  // namespace envpot
