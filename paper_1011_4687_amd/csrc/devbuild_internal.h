// Device build of a handle's pair list and layout (not part of the C ABI).
//
// From the host's block plan the device enumerates every primitive pair of
// the nonzero density blocks, screens it, orders the kept pairs by (fragment
// group, L, enumeration order), forms the same-centre clusters (one-centre
// pairs by atom and far-field radius band), places every record and writes
// the records with their density terms zero, together with the tables of the
// density fold.  The host computes only per-group tables: segment offsets
// and costs from per-(group, L) counts.  Every decision takes the same bits
// as the host packer (screen_math.h), so the records equal the host packer's
// bit for bit once the same density fold has run.
#pragma once

#include <cstdint>
#include <vector>

#include "envpot_internal.h"
#include "update_internal.h"

namespace envpot {

// What the device build leaves behind.  Device arrays are owned by the
// caller afterwards (hipFree); host vectors describe the layout.
struct DevBuild {
    uint32_t* d_rec = nullptr;        // records, words
    int64_t words = 0;
    std::vector<Segment> base;        // unsplit segments
    std::vector<double> unit_cost;    // per base segment
    int64_t n_pairs = 0, n_unscreened = 0, n_clusters = 0, n_members = 0, n_drop = 0;
    int64_t n_pairs_by_L[kLMax + 1] = {};
    double screened_bound = 0.0;
    std::vector<int64_t> group_pair_begin;  // per group + 1
    std::vector<int32_t> drop_group;        // per dropped pair kept for the charges
    // density-fold tables (the layout of UpdateState)
    UpdPair* d_pairs = nullptr;       // n_pairs kept pairs, then n_drop dropped pairs
    UpdCluster* d_clusters = nullptr; // n_clusters
    int64_t* d_members = nullptr;     // n_members pair indices, in cluster order
    int64_t* d_moff = nullptr;        // n_members + 1: first h word of each member
    int64_t hm_words = 0;             // moff's last entry
    int64_t device_bytes = 0;
};

// Whether the device build can take the plan (index widths of its sorts and
// records); otherwise the host packer builds the pairs.
bool device_build_fits(const BlockPlan& plan, const PairList& meta, int n_nuclei);

// Run the device build on the current device (synchronous).  meta holds the
// pair list's fields that do not depend on pairs; the pair-dependent ones
// are returned in out.
env_status device_build(const BlockPlan& plan, const PairSources& src, const PairList& meta, bool fp64,
                        const BoysParams& bp, bool merge, DevBuild& out);

void free_device_build(DevBuild& b);

}  // namespace envpot
