// C ABI of the environment-potential library (include/env_potential.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "envpot_internal.h"

using namespace envpot;

struct env_potential {
    int device = -1;
    int precision = ENV_PREC_FP32C;
    bool on_device = false;
    int cu_count = 256;
    env_info info{};
    PairList host;                      // kept only for ENV_BUILD_ONLY handles
    BoysParams bp{};
    // device buffers
    uint32_t* d_rec = nullptr;
    Segment* d_segs = nullptr;
    int32_t* d_split = nullptr;
    double* d_nuc = nullptr;
    void* d_boys = nullptr;
    int64_t seg_off[kMaxSplitLog2 + 1] = {};    // per split factor 2^k: first segment
    int64_t split_off[kMaxSplitLog2 + 1] = {};  // per split factor 2^k: first offset
    int64_t device_bytes = 0;
};

namespace {

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

template <typename T>
env_status upload(const std::vector<T>& v, T** dst, int64_t& bytes) {
    const size_t nb = std::max<size_t>(v.size(), 1) * sizeof(T);
    if (hipMalloc(reinterpret_cast<void**>(dst), nb) != hipSuccess) return ENV_E_NOMEM;
    bytes += int64_t(nb);
    if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return ENV_E_DEVICE;
    return ENV_OK;
}

void free_device(env_potential* h) {
    if (!h->on_device) return;
    DeviceGuard g(h->device);
    (void)hipFree(h->d_rec);
    (void)hipFree(h->d_segs);
    (void)hipFree(h->d_split);
    (void)hipFree(h->d_nuc);
    (void)hipFree(h->d_boys);
    h->d_rec = nullptr;
    h->d_segs = nullptr;
    h->d_split = nullptr;
    h->d_nuc = nullptr;
    h->d_boys = nullptr;
    h->on_device = false;
}

int env_int(const char* name, int dflt) {
    const char* s = std::getenv(name);
    if (!s || !*s) return dflt;
    return std::atoi(s);
}

}  // namespace

extern "C" {

void env_options_default(env_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = ENV_PREC_FP32C;
    o->device = -1;
    o->screen_threshold = 1e-12;
    o->flags = 0;
}

const char* env_status_string(env_status s) {
    switch (s) {
        case ENV_OK: return "ok";
        case ENV_E_ARG: return "invalid argument";
        case ENV_E_UNSUPPORTED: return "unsupported input or option";
        case ENV_E_NOMEM: return "out of memory";
        case ENV_E_DEVICE: return "device error";
        case ENV_E_STATE: return "handle cannot do this";
    }
    return "unknown status";
}

env_status env_potential_create(const env_nucleus* nuclei, int32_t n_nuclei,
                                const env_shell* shells, int32_t n_shells,
                                const env_density* P, const env_options* opts,
                                env_potential** out) {
    if (!out) return ENV_E_ARG;
    *out = nullptr;
    env_options opt;
    if (opts) opt = *opts;
    else env_options_default(&opt);
    if (opt.precision != ENV_PREC_FP64 && opt.precision != ENV_PREC_FP32C) return ENV_E_ARG;
    if (opt.reserved[0] || opt.reserved[1] || opt.reserved[2]) return ENV_E_ARG;
    if (opt.flags & ~(ENV_BUILD_ONLY | ENV_NEUTRALIZE | ENV_NO_SCREENING)) return ENV_E_ARG;
    const bool build_only = (opt.flags & ENV_BUILD_ONLY) != 0;

    int device = opt.device;
    if (!build_only) {
        int ndev = 0;
        if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return ENV_E_DEVICE;
        if (device < 0 && hipGetDevice(&device) != hipSuccess) return ENV_E_DEVICE;
        if (device >= ndev) return ENV_E_ARG;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) != hipSuccess) return ENV_E_DEVICE;
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return ENV_E_DEVICE;
    }

    env_potential* h = new (std::nothrow) env_potential();
    if (!h) return ENV_E_NOMEM;
    h->device = device;
    h->precision = opt.precision;
    env_status st;
    try {
        st = build_pair_list(nuclei, n_nuclei, shells, n_shells, P, opt, h->host);
    } catch (const std::bad_alloc&) {
        st = ENV_E_NOMEM;
    } catch (...) {
        st = ENV_E_ARG;
    }
    if (st != ENV_OK) {
        delete h;
        return st;
    }
    const PairList& pl = h->host;
    env_info& in = h->info;
    in.nbf = pl.nbf;
    in.n_nuclei = int32_t(pl.nuc.size() / 4);
    in.n_groups = pl.n_groups;
    in.n_pairs = int64_t(pl.L.size());
    for (int L : pl.L) in.n_pairs_by_L[L]++;
    in.n_pairs_unscreened = pl.n_unscreened;
    in.electrons = pl.electrons;
    in.nuclear_charge = pl.nuclear_charge;
    in.screened_bound = pl.screened_bound;
    in.precision = h->precision;

    std::vector<float> t32;
    std::vector<double> t64;
    build_boys_tables(t32, t64, h->bp);
    if (h->bp.rows32 > kBoysMaxRowsF32) {
        delete h;
        return ENV_E_DEVICE;
    }
    const bool fp64 = h->precision == ENV_PREC_FP64;
    std::vector<Segment> allsegs;
    std::vector<int32_t> allsplit;
    for (int k = 0; k <= kMaxSplitLog2; ++k) {
        std::vector<Segment> segs;
        std::vector<int32_t> split;
        build_segments(pl, 1 << k, fp64, segs, split);
        h->seg_off[k] = int64_t(allsegs.size());
        h->split_off[k] = int64_t(allsplit.size());
        allsegs.insert(allsegs.end(), segs.begin(), segs.end());
        allsplit.insert(allsplit.end(), split.begin(), split.end());
        if (k == 0) in.n_segments = int32_t(segs.size());
    }
    if (build_only) {
        *out = h;
        return ENV_OK;
    }
    std::vector<uint32_t> rec;
    pack_records(pl, fp64, h->bp, rec);
    {
        DeviceGuard g(device);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) h->cu_count = prop.multiProcessorCount;
        h->on_device = true;
        st = upload(rec, &h->d_rec, h->device_bytes);
        if (st == ENV_OK) st = upload(allsegs, &h->d_segs, h->device_bytes);
        if (st == ENV_OK) st = upload(allsplit, &h->d_split, h->device_bytes);
        if (st == ENV_OK) st = upload(pl.nuc, &h->d_nuc, h->device_bytes);
        if (st == ENV_OK) {
            if (fp64) st = upload(t64, reinterpret_cast<double**>(&h->d_boys), h->device_bytes);
            else st = upload(t32, reinterpret_cast<float**>(&h->d_boys), h->device_bytes);
        }
    }
    if (st != ENV_OK) {
        free_device(h);
        delete h;
        return st;
    }
    in.device_bytes = h->device_bytes;
    in.built_on_device = 1;
    h->host = PairList();  // the device copy is the one that is used
    *out = h;
    return ENV_OK;
}

env_status env_potential_eval(env_potential* h, const double* points, int64_t n, double* out,
                              void* stream) {
    if (!h || n < 0) return ENV_E_ARG;
    if (n == 0) return ENV_OK;
    if (!points || !out) return ENV_E_ARG;
    if (!h->on_device) return ENV_E_STATE;
    DeviceGuard g(h->device);
    const bool fp64 = h->precision == ENV_PREC_FP64;
    int np = env_int("ENVPOT_NP", fp64 ? 2 : 4);
    if (np != 1 && np != 2 && np != 4) np = fp64 ? 2 : 4;
    if (fp64 && np == 4) np = 2;
    // split factor: enough waves to keep ~24 per SIMD in flight over the run
    const int64_t waves = (n + 64 * np - 1) / (64 * np);
    const int64_t want = int64_t(h->cu_count) * 4 * 24;
    int k = 0;
    while (k < kMaxSplitLog2 && waves * (int64_t(1) << k) < want) ++k;
    const int forced = env_int("ENVPOT_SPLIT_LOG2", -1);
    if (forced >= 0 && forced <= kMaxSplitLog2) k = forced;
    const int S = 1 << k;

    EvalArgs a;
    a.pts = points;
    a.n = n;
    a.segs = h->d_segs + h->seg_off[k];
    a.split = h->d_split + h->split_off[k];
    a.rec = h->d_rec;
    a.nuc = h->d_nuc;
    a.boys = h->d_boys;
    a.bp = h->bp;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (S == 1) {
        a.out = out;
        return launch_potential(a, 1, h->precision, np, stream) == 0 ? ENV_OK : ENV_E_DEVICE;
    }
    double* part = nullptr;
    if (hipMallocAsync(reinterpret_cast<void**>(&part), size_t(S) * size_t(n) * sizeof(double), st) !=
        hipSuccess)
        return ENV_E_NOMEM;
    a.out = part;
    int rc = launch_potential(a, S, h->precision, np, stream);
    if (rc == 0) rc = launch_sum_splits(part, S, n, out, stream);
    (void)hipFreeAsync(part, st);
    return rc == 0 ? ENV_OK : ENV_E_DEVICE;
}

env_status env_potential_eval_batched(env_potential* const* hs, int32_t n_inst,
                                      const double* const* points, const int64_t* n,
                                      double* const* out, void* stream) {
    if (n_inst < 0) return ENV_E_ARG;
    if (n_inst == 0) return ENV_OK;
    if (!hs || !points || !n || !out) return ENV_E_ARG;
    for (int i = 0; i < n_inst; ++i) {
        if (!hs[i] || n[i] < 0) return ENV_E_ARG;
        if (hs[i]->device != hs[0]->device || hs[i]->precision != hs[0]->precision)
            return ENV_E_ARG;
    }
    for (int i = 0; i < n_inst; ++i) {
        const env_status s = env_potential_eval(hs[i], points[i], n[i], out[i], stream);
        if (s != ENV_OK) return s;
    }
    return ENV_OK;
}

env_status env_potential_info(const env_potential* h, env_info* info) {
    if (!h || !info) return ENV_E_ARG;
    *info = h->info;
    return ENV_OK;
}

env_status env_potential_export_pairs(const env_potential* h, int64_t cap, int32_t* L,
                                      int32_t* group, double* center, double* p, double* D) {
    if (!h) return ENV_E_ARG;
    if (h->on_device) return ENV_E_STATE;
    const PairList& pl = h->host;
    const int64_t n = int64_t(pl.L.size());
    if (cap < n) return ENV_E_ARG;
    if (L) std::copy(pl.L.begin(), pl.L.end(), L);
    if (group) std::copy(pl.group.begin(), pl.group.end(), group);
    if (center) std::copy(pl.center.begin(), pl.center.end(), center);
    if (p) std::copy(pl.p.begin(), pl.p.end(), p);
    if (D) std::copy(pl.D.begin(), pl.D.end(), D);
    return ENV_OK;
}

void env_potential_destroy(env_potential* h) {
    if (!h) return;
    free_device(h);
    delete h;
}

}  // extern "C"
