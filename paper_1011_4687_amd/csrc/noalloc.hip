// env_potential_eval_noalloc: the evaluation of env_potential_eval for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).  The only scratch memory
// of an evaluation is the split-pair partial sums [S][n] (float64); here they
// live in one file-scope device array of fixed size, so the call allocates
// nothing.  Each device that runs this call holds its own copy of the array
// until the process ends; every call on one device uses that device's copy.
#include <hip/hip_runtime.h>

#include <mutex>

#include "handle.h"

using namespace envpot;

namespace {

// 2^23 float64 = 64 MiB of split partials per device.
constexpr int64_t kScratchDoubles = int64_t(1) << 23;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (the current device), looked
// up once per device.  The host-side name `scratch` is not a device address
// and is never passed to a kernel or a copy.
env_status scratch_address(int device, double** out) {
    if (device < 0 || device >= kMaxDevices) return ENV_E_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ENV_E_DEVICE;
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[device];
    return ENV_OK;
}

}  // namespace

extern "C" {

int64_t env_potential_noalloc_max_points(void) { return kScratchDoubles; }

env_status env_potential_eval_noalloc(env_potential* h, const double* points, int64_t n, double* out,
                                      void* stream) {
    if (!h || n < 0) return ENV_E_ARG;
    if (n == 0) return ENV_OK;
    if (!points || !out || n > kScratchDoubles) return ENV_E_ARG;
    if (!h->on_device) return ENV_E_STATE;
    DeviceGuard g(h->device);
    double* part = nullptr;
    env_status rc = scratch_address(h->device, &part);
    if (rc != ENV_OK) return rc;
    // the launch shape of env_potential_eval, with the split factor lowered
    // until the partials fit the array
    int np = 0, k = 0;
    choose_shape(h, n, &np, &k);
    while (k > 0 && (int64_t(1) << k) * n > kScratchDoubles) --k;
    const int S = 1 << k;
    if (S == 1) return launch_potential(make_args(h, points, n, out, 0), 1, h->precision, np, stream) == 0
                           ? ENV_OK
                           : ENV_E_DEVICE;
    // every (split, point) partial is written by the potential kernel before
    // the fixed-order sum reads it, so nothing needs clearing between calls
    if (launch_potential(make_args(h, points, n, part, k), S, h->precision, np, stream) != 0 ||
        launch_sum_splits(part, S, n, out, stream) != 0)
        return ENV_E_DEVICE;
    return ENV_OK;
}

}  // extern "C"
