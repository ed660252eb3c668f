// The opaque handle of the C ABI and helpers shared by the ABI files.
#pragma once

#include <hip/hip_runtime.h>

#include "envpot_internal.h"
#include "field_internal.h"
#include "update_internal.h"

namespace envpot {

// What a handle created with ENV_FORCE_CPU needs besides its pair list: the
// FP64 Boys table and far-field thresholds, and every pair's far-field
// coefficients (same offsets as the pair list's D).
struct HostEval {
    std::vector<double> boys;
    std::vector<double> h;
    double tfar[kLMax + 1] = {};
};

}  // namespace envpot

struct env_potential {
    int device = -1;
    int precision = ENV_PREC_FP32C;
    bool on_device = false;
    bool on_host = false;               // ENV_FORCE_CPU: evaluated by host threads
    uint64_t density_gen = 0;           // bumped whenever a density fold rewrites the records
    int cu_count = 256;
    env_info info{};
    envpot::PairList host;              // kept for ENV_BUILD_ONLY and ENV_FORCE_CPU handles
    envpot::HostEval hosteval;          // ENV_FORCE_CPU only
    envpot::BoysParams bp{};
    // device buffers
    uint32_t* d_rec = nullptr;
    envpot::Segment* d_segs = nullptr;
    double* d_boxes = nullptr;          // per unsplit segment (Segment::box)
    bool use_boxes = true;              // ENVPOT_NO_FARBOX=1 at create: test every pair
    int32_t* d_split = nullptr;
    double* d_nuc = nullptr;
    void* d_boys = nullptr;
    void* d_boys_field = nullptr;       // Boys table of the field (one order more)
    envpot::FieldParams fp{};
    envpot::UpdateState* upd = nullptr;  // density update tables (device)
    int64_t rec_words = 0;              // words of d_rec
    int64_t n_segs_all = 0;             // segments of d_segs (every split factor)
    int64_t seg_off[envpot::kMaxSplitLog2 + 1] = {};    // per split factor 2^k: first segment
    int64_t split_off[envpot::kMaxSplitLog2 + 1] = {};  // per split factor 2^k: first offset
    int64_t device_bytes = 0;
    // kernel timing (env_potential_kernel_timing): event pairs around each
    // potential-kernel launch, in call order
    bool ktime = false;
    std::vector<hipEvent_t> kev;
    size_t kev_used = 0;
    // tuned launch shapes: (point count, points per lane, split log2)
    struct Tuned { int64_t n; int np; int klog; };
    std::vector<Tuned> tuned;
};

namespace envpot {

struct DeviceGuard {  // restores the caller's current device
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (dev >= 0 && dev != prev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Launch shape of a single evaluation of h at n points.
void choose_shape(const env_potential* h, int64_t n, int* np, int* klog);

// Host evaluation of an ENV_FORCE_CPU handle (hosteval.cpp): tables at
// create, then V at n host points into host memory.
void host_prepare(env_potential* h, const std::vector<double>& t64);
env_status host_eval(const env_potential* h, const double* points, int64_t n, double* out);

// Exact evaluation of h at the first *m of n_max device points (count known
// only on the device) into out[0, *m), asynchronous: one persistent launch
// plus the fixed-order split sum.  part: part_cap float64 elements (at least
// n_max) for the split partials; counter: one device word.
env_status eval_devsized(env_potential* h, const double* points, const int64_t* m, int64_t n_max, double* out,
                         double* part, int64_t part_cap, unsigned long long* counter, void* stream);

// Arguments of one evaluation (out = V when S == 1, partials otherwise).
EvalArgs make_args(const env_potential* h, const double* points, int64_t n, double* out, int klog);

}  // namespace envpot
