// C ABI of the environment-potential library (include/env_potential.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "devbuild_internal.h"
#include "handle.h"
#include "probe.h"
#include "sort_internal.h"

using namespace envpot;

namespace {

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
    (void)hipFree(h->d_boxes);
    (void)hipFree(h->d_split);
    (void)hipFree(h->d_nuc);
    (void)hipFree(h->d_boys);
    (void)hipFree(h->d_boys_field);
    h->d_boys_field = nullptr;
    free_update_state(h->upd);
    h->upd = nullptr;
    h->d_rec = nullptr;
    h->d_segs = nullptr;
    h->d_boxes = nullptr;
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

// Far-field boxes of the unsplit segments, from the records on the device
// (the same for the host packer's and the device build's records).
env_status segment_boxes(env_potential* h, const std::vector<Segment>& base, bool fp64) {
    h->use_boxes = env_int("ENVPOT_NO_FARBOX", 0) != 1;
    const int64_t nb = std::max<int64_t>(int64_t(base.size()), 1) * kSegBoxWords * int64_t(sizeof(double));
    if (hipMalloc(reinterpret_cast<void**>(&h->d_boxes), size_t(nb)) != hipSuccess) return ENV_E_NOMEM;
    h->device_bytes += nb;
    if (base.empty()) return ENV_OK;
    Segment* tmp = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&tmp), base.size() * sizeof(Segment)) != hipSuccess) return ENV_E_NOMEM;
    env_status st = ENV_OK;
    if (hipMemcpy(tmp, base.data(), base.size() * sizeof(Segment), hipMemcpyHostToDevice) != hipSuccess ||
        launch_segment_boxes(tmp, int(base.size()), h->d_rec, fp64 ? 1 : 0, h->d_boxes, nullptr) != 0 ||
        hipStreamSynchronize(nullptr) != hipSuccess)
        st = ENV_E_DEVICE;
    (void)hipFree(tmp);
    return st;
}

}  // namespace

namespace envpot {

// Waves per SIMD that a single call's split factor aims for (both
// precisions; the device-sized launch uses the same target).
constexpr int64_t kWantWavesPerSimd = 48;

void choose_shape(const env_potential* h, int64_t n, int* np_out, int* k_out) {
    const bool fp64 = h->precision == ENV_PREC_FP64;
    // a tuned shape for a point count within a factor 2 of n wins
    const env_potential::Tuned* best = nullptr;
    double bestd = 1e300;
    for (const auto& t : h->tuned) {
        const double d = std::fabs(std::log(double(t.n) / double(n)));
        if (d < bestd) { bestd = d; best = &t; }
    }
    int np, k = 0;
    if (best && bestd <= std::log(2.0)) {
        np = best->np;
        k = best->klog;
    } else {
        np = fp64 ? 2 : 4;
        // split factor: enough waves to keep ~48 per SIMD in flight over the
        // run (mid, Morton order: FP32C 18.7 ms with 128 splits against
        // 19.2 ms with 64 and 20.1 ms with 32; FP64 33.6 ms with 64 or 128
        // against 34.5 ms with 32)
        const int64_t waves = (n + 64 * np - 1) / (64 * np);
        const int64_t want = int64_t(h->cu_count) * 4 * kWantWavesPerSimd;
        while (k < kMaxSplitLog2 && waves * (int64_t(1) << k) < want) ++k;
        // long pair lists: split further while one split holds more than 2^17
        // pairs, within 2^27 partial sums (1 GiB) (5000 atoms, 1,048,576
        // points: 128 splits 3.230 s FP32C / 5.914 s FP64 against 3.248 /
        // 6.271 s with 64 and 3.288 / 6.444 s with 32)
        while (k < kMaxSplitLog2 && (h->info.n_pairs >> k) > (int64_t(1) << 17) &&
               (n << (k + 1)) <= (int64_t(1) << 27))
            ++k;
    }
    const int fnp = env_int("ENVPOT_NP", -1);
    if (fnp == 1 || fnp == 2 || (fnp == 4 && !fp64)) np = fnp;
    const int fk = env_int("ENVPOT_SPLIT_LOG2", -1);
    if (fk >= 0 && fk <= kMaxSplitLog2) k = fk;
    *np_out = np;
    *k_out = k;
}

EvalArgs make_args(const env_potential* h, const double* points, int64_t n, double* out, int k) {
    EvalArgs a;
    a.pts = points;
    a.n = n;
    a.segs = h->d_segs + h->seg_off[k];
    a.split = h->d_split + h->split_off[k];
    a.rec = h->d_rec;
    a.nuc = h->d_nuc;
    a.boys = h->d_boys;
    a.boxes = h->use_boxes ? h->d_boxes : nullptr;
    a.out = out;
    a.bp = h->bp;
    return a;
}

env_status eval_devsized(env_potential* h, const double* points, const int64_t* m, int64_t n_max, double* out,
                         double* part, int64_t part_cap, unsigned long long* counter, void* stream) {
    if (!h->on_device) return ENV_E_STATE;
    if (n_max <= 0) return ENV_OK;
    if (part_cap < n_max) return ENV_E_ARG;
    const bool fp64 = h->precision == ENV_PREC_FP64;
    const int np = fp64 ? 2 : 4;
    DevSizedArgs d;
    d.a = make_args(h, points, 0, part, 0);
    d.m = m;
    d.segs_all = h->d_segs;
    d.split_all = h->d_split;
    for (int k = 0; k <= kMaxSplitLog2; ++k) {
        d.seg_off[k] = h->seg_off[k];
        d.split_off[k] = h->split_off[k];
    }
    d.part_cap = part_cap;
    d.want_waves = int64_t(h->cu_count) * 4 * kWantWavesPerSimd;  // the rule of choose_shape
    d.counter = counter;
    DeviceGuard g(h->device);
    if (launch_potential_devsized(d, devsized_grid(h->precision, h->cu_count), h->precision, np, stream) != 0 ||
        launch_sum_devsized(d, np, n_max, out, stream) != 0)
        return ENV_E_DEVICE;
    return ENV_OK;
}

}  // namespace envpot

namespace {
env_status eval_core(env_potential* h, const double* points, int64_t n, double* out, void* stream);
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
    // any int may arrive through the C ABI; an out-of-range value must not be
    // read as an env_status, so the bytes are read as an int
    static_assert(sizeof(env_status) == sizeof(int32_t), "env_status is int-sized");
    int32_t v;
    std::memcpy(&v, &s, sizeof v);
    switch (v) {
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
    if (opt.flags &
        ~(ENV_BUILD_ONLY | ENV_NEUTRALIZE | ENV_NO_SCREENING | ENV_NO_MERGE | ENV_FORCE_CPU | ENV_HOST_PACK))
        return ENV_E_ARG;
    const bool force_cpu = (opt.flags & ENV_FORCE_CPU) != 0;
    if (force_cpu && (opt.flags & ENV_BUILD_ONLY)) return ENV_E_ARG;
    if (force_cpu && opt.precision != ENV_PREC_FP64) return ENV_E_UNSUPPORTED;
    // host handles: the pair list and its D stay on the host (host fold)
    const bool build_only = (opt.flags & ENV_BUILD_ONLY) != 0 || force_cpu;

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

    const char* tenv = std::getenv("ENVPOT_TIMING");
    const bool timing = tenv && *tenv && *tenv != '0';
    auto tlast = std::chrono::steady_clock::now();
    auto lap = [&](const char* what) {
        if (!timing) return;
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[envpot create] %-22s %8.3f s\n", what,
                     std::chrono::duration<double>(now - tlast).count());
        tlast = now;
    };
    env_potential* h = new (std::nothrow) env_potential();
    if (!h) return ENV_E_NOMEM;
    h->device = device;
    h->precision = opt.precision;
    env_status st;
    PairSources src;  // kept for the density update tables of device handles
    // device handles fold the density on the device (the update kernels)
    // unless a shell has more primitives than the update tables index
    bool fits = true;
    for (int32_t s = 0; s < n_shells && shells; ++s) fits = fits && shells[s].nprim <= 32767;
    src.device_fold = !build_only && fits;
    const bool merge = (opt.flags & ENV_NO_MERGE) == 0;
    // device handles also enumerate, screen, order and lay out their pairs on
    // the device (the host parses the inputs into density blocks), unless
    // ENV_HOST_PACK asks for the host packer
    bool dev_build = src.device_fold && (opt.flags & ENV_HOST_PACK) == 0;
    BlockPlan plan;
    auto host_list = [&]() -> env_status {
        try {
            return build_pair_list(nuclei, n_nuclei, shells, n_shells, P, opt, h->host, build_only ? nullptr : &src,
                                   dev_build ? &plan : nullptr);
        } catch (const std::bad_alloc&) {
            return ENV_E_NOMEM;
        } catch (...) {
            return ENV_E_ARG;
        }
    };
    auto host_again = [&]() {  // the host packer after all
        dev_build = false;
        h->host = PairList();
        const bool df = src.device_fold;
        src = PairSources();
        src.device_fold = df;
        return host_list();
    };
    st = host_list();
    if (st == ENV_OK && dev_build && !device_build_fits(plan, h->host, n_nuclei)) st = host_again();
    if (st != ENV_OK) {
        delete h;
        return st;
    }
    lap(dev_build ? "block plan" : "pair list");
    env_info& in = h->info;
    in.precision = h->precision;

    std::vector<float> t32;
    std::vector<double> t64;
    build_boys_tables(t32, t64, h->bp);
    std::vector<float> tf32;
    std::vector<double> tf64;
    build_field_tables(h->bp, tf32, tf64, h->fp);
    if (h->bp.rows32 > kBoysMaxRowsF32 || h->fp.rows32 > kFieldMaxRowsF32) {
        delete h;
        return ENV_E_DEVICE;
    }
    lap("Boys tables");
    const bool fp64 = h->precision == ENV_PREC_FP64;
    Layout lay;
    LayoutMap lmap;
    DevBuild db;
    if (dev_build) {
        {
            DeviceGuard g(device);
            try {
                st = device_build(plan, src, h->host, fp64, h->bp, merge, db);
            } catch (const std::bad_alloc&) {
                st = ENV_E_NOMEM;
            }
        }
        if (st == ENV_E_UNSUPPORTED) {  // cluster tables beyond 32-bit words: the host packer drops the clusters
            free_device_build(db);
            st = host_again();
        }
        if (st != ENV_OK) {
            free_device_build(db);
            delete h;
            return st;
        }
    }
    const PairList& pl = h->host;
    in.nbf = pl.nbf;
    in.n_nuclei = int32_t(pl.nuc.size() / 4);
    in.n_groups = pl.n_groups;
    in.nuclear_charge = pl.nuclear_charge;
    in.electrons = pl.electrons;
    if (dev_build) {
        lay.base = db.base;
        lay.unit_cost = db.unit_cost;
        lay.n_clusters = db.n_clusters;
        lay.n_members = db.n_members;
        in.n_pairs = db.n_pairs;
        for (int L = 0; L <= kLMax; ++L) in.n_pairs_by_L[L] = db.n_pairs_by_L[L];
        in.n_pairs_unscreened = db.n_unscreened;
        in.screened_bound = db.screened_bound;
        h->host.group_pair_begin = db.group_pair_begin;
        lap("device build");
    } else {
        in.n_pairs = int64_t(pl.L.size());
        for (int L : pl.L) in.n_pairs_by_L[L]++;
        in.n_pairs_unscreened = pl.n_unscreened;
        in.screened_bound = pl.screened_bound;
        try {
            pack_layout(pl, fp64, h->bp, merge, lay, build_only ? nullptr : &lmap);
        } catch (const std::bad_alloc&) {
            delete h;
            return ENV_E_NOMEM;
        }
        lap("layout");
    }
    in.n_clusters = lay.n_clusters;
    in.n_cluster_members = lay.n_members;
    in.pairs_built_on_device = dev_build ? 1 : 0;
    for (size_t i = 0; i < lay.base.size(); ++i) lay.base[i].box = int32_t(i);
    std::vector<Segment> allsegs;
    std::vector<int32_t> allsplit;
    for (int k = 0; k <= kMaxSplitLog2; ++k) {
        std::vector<Segment> segs;
        std::vector<int32_t> split;
        split_layout(lay, 1 << k, fp64, segs, split);
        h->seg_off[k] = int64_t(allsegs.size());
        h->split_off[k] = int64_t(allsplit.size());
        allsegs.insert(allsegs.end(), segs.begin(), segs.end());
        allsplit.insert(allsplit.end(), split.begin(), split.end());
        if (k == 0) in.n_segments = int32_t(segs.size());
    }
    lap("splits");
    if (force_cpu) {
        try {
            host_prepare(h, t64);
        } catch (const std::bad_alloc&) {
            delete h;
            return ENV_E_NOMEM;
        }
        h->on_host = true;
        in.on_host = 1;
    }
    if (build_only) {
        *out = h;
        return ENV_OK;
    }
    std::vector<uint32_t>& rec = lay.rec;
    {
        DeviceGuard g(device);
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) h->cu_count = prop.multiProcessorCount;
        h->on_device = true;
        h->rec_words = dev_build ? db.words : int64_t(rec.size());
        h->n_segs_all = int64_t(allsegs.size());
        if (dev_build) {
            h->d_rec = db.d_rec;
            db.d_rec = nullptr;
            h->device_bytes += std::max<int64_t>(db.words, 1) * 4;
            st = ENV_OK;
        } else {
            st = upload(rec, &h->d_rec, h->device_bytes);
        }
        if (st == ENV_OK) st = upload(allsegs, &h->d_segs, h->device_bytes);
        if (st == ENV_OK) st = upload(allsplit, &h->d_split, h->device_bytes);
        if (st == ENV_OK) st = segment_boxes(h, lay.base, fp64);
        if (st == ENV_OK) st = upload(pl.nuc, &h->d_nuc, h->device_bytes);
        if (st == ENV_OK) {
            if (fp64) st = upload(t64, reinterpret_cast<double**>(&h->d_boys), h->device_bytes);
            else st = upload(t32, reinterpret_cast<float**>(&h->d_boys), h->device_bytes);
        }
        if (st == ENV_OK) {
            if (fp64) st = upload(tf64, reinterpret_cast<double**>(&h->d_boys_field), h->device_bytes);
            else st = upload(tf32, reinterpret_cast<float**>(&h->d_boys_field), h->device_bytes);
        }
        lap("upload");
        if (st == ENV_OK) {
            try {
                h->upd = dev_build ? make_update_state_device(pl, src, db, &st)
                                   : make_update_state(pl, src, lmap, &st);
            } catch (const std::bad_alloc&) {
                st = ENV_E_NOMEM;
            }
            if (h->upd) h->device_bytes += h->upd->device_bytes;
            else if (st == ENV_OK && src.device_fold) st = ENV_E_DEVICE;
        }
        lap("update tables");
        // the first fold of the density, on the device
        if (st == ENV_OK && src.device_fold) st = env_potential_update_density(h, P, nullptr);
        lap("device fold");
    }
    free_device_build(db);
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
    if (h->on_host) return host_eval(h, points, n, out);
    if (!h->on_device) return ENV_E_STATE;
    DeviceGuard g(h->device);
    if (n < kSortMinPoints || n > int64_t(INT32_MAX) || env_int("ENVPOT_NO_SORT", 0) != 0 ||
        stream_capturing(stream))
        return eval_core(h, points, n, out, stream);
    // large calls: evaluate the points in Morton order, then restore the caller's order
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *spts = nullptr, *sout = nullptr;
    uint32_t* order = nullptr;
    if (hipMallocAsync(reinterpret_cast<void**>(&spts), size_t(n) * 3 * sizeof(double), st) != hipSuccess)
        return ENV_E_NOMEM;
    env_status rc = ENV_OK;
    if (hipMallocAsync(reinterpret_cast<void**>(&sout), size_t(n) * sizeof(double), st) != hipSuccess ||
        hipMallocAsync(reinterpret_cast<void**>(&order), size_t(n) * sizeof(uint32_t), st) != hipSuccess)
        rc = ENV_E_NOMEM;
    if (rc == ENV_OK && sort_points(points, n, spts, order, stream) != 0) rc = ENV_E_DEVICE;
    if (rc == ENV_OK) rc = eval_core(h, spts, n, sout, stream);
    if (rc == ENV_OK && scatter_values(sout, order, n, out, stream) != 0) rc = ENV_E_DEVICE;
    (void)hipFreeAsync(order, st);
    (void)hipFreeAsync(sout, st);
    (void)hipFreeAsync(spts, st);
    return rc;
}

}  // extern "C"

namespace {

// The next event of the kernel-timing list (created on first use), or null.
hipEvent_t next_event(env_potential* h) {
    if (!h->ktime || h->kev_used >= 4096) return nullptr;
    if (h->kev_used == h->kev.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->kev.push_back(e);
    }
    return h->kev[h->kev_used++];
}

// The potential kernel, with a pair of timing events around it when on.
int timed_launch(env_potential* h, const EvalArgs& a, int S, int np, void* stream) {
    hipEvent_t e0 = next_event(h), e1 = e0 ? next_event(h) : nullptr;
    if (e0 && !e1) --h->kev_used;
    const bool on = e0 && e1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (on && hipEventRecord(e0, st) != hipSuccess) return -1;
    const int rc = launch_potential(a, S, h->precision, np, stream);
    if (on && rc == 0 && hipEventRecord(e1, st) != hipSuccess) return -1;
    return rc;
}

env_status eval_core(env_potential* h, const double* points, int64_t n, double* out, void* stream) {
    int np, k;
    choose_shape(h, n, &np, &k);
    const int S = 1 << k;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (S == 1) {
        const EvalArgs a = make_args(h, points, n, out, 0);
        return timed_launch(h, a, 1, np, stream) == 0 ? ENV_OK : ENV_E_DEVICE;
    }
    double* part = nullptr;
    if (hipMallocAsync(reinterpret_cast<void**>(&part), size_t(S) * size_t(n) * sizeof(double), st) !=
        hipSuccess)
        return ENV_E_NOMEM;
    const EvalArgs a = make_args(h, points, n, part, k);
    int rc = timed_launch(h, a, S, np, stream);
    if (rc == 0) rc = launch_sum_splits(part, S, n, out, stream);
    (void)hipFreeAsync(part, st);
    return rc == 0 ? ENV_OK : ENV_E_DEVICE;
}

}  // namespace

extern "C" {

env_status env_potential_autotune(env_potential* h, const double* points, int64_t n, void* stream) {
    if (!h || n <= 0 || !points) return ENV_E_ARG;
    if (!h->on_device) return ENV_E_STATE;
    DeviceGuard g(h->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    double* out = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&out), size_t(n) * sizeof(double)) != hipSuccess)
        return ENV_E_NOMEM;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(out);
        return ENV_E_DEVICE;
    }
    const bool fp64 = h->precision == ENV_PREC_FP64;
    const int nps32[] = {2, 4}, nps64[] = {1, 2};
    const int* nps = fp64 ? nps64 : nps32;
    float best = 1e30f;
    env_potential::Tuned bestc{n, fp64 ? 2 : 4, 0};
    env_status rc = ENV_OK;
    // drop an earlier entry for this size, then time every candidate shape
    h->tuned.erase(std::remove_if(h->tuned.begin(), h->tuned.end(),
                                  [&](const env_potential::Tuned& t) { return t.n == n; }),
                   h->tuned.end());
    for (int a = 0; a < 2 && rc == ENV_OK; ++a) {
        for (int k = 0; k <= kMaxSplitLog2 && rc == ENV_OK; ++k) {
            const int64_t waves = ((n + 64 * nps[a] - 1) / (64 * nps[a])) << k;
            if (waves < int64_t(h->cu_count) * 4 || (k > 0 && waves > int64_t(h->cu_count) * 4 * 96))
                continue;
            h->tuned.push_back({n, nps[a], k});
            float ms = 0.0f;
            for (int rep = 0; rep < 3 && rc == ENV_OK; ++rep) {  // first run warms up
                if (hipEventRecord(e0, st) != hipSuccess) rc = ENV_E_DEVICE;
                if (rc == ENV_OK) rc = env_potential_eval(h, points, n, out, stream);
                if (rc == ENV_OK && hipEventRecord(e1, st) != hipSuccess) rc = ENV_E_DEVICE;
                if (rc == ENV_OK && hipEventSynchronize(e1) != hipSuccess) rc = ENV_E_DEVICE;
                float t = 0.0f;
                if (rc == ENV_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = ENV_E_DEVICE;
                if (rep > 0) ms += t;
            }
            h->tuned.pop_back();
            if (rc == ENV_OK && ms < best) {
                best = ms;
                bestc = {n, nps[a], k};
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (rc == ENV_OK) h->tuned.push_back(bestc);
    return rc;
}

env_status env_potential_kernel_timing(env_potential* h, int32_t on) {
    if (!h) return ENV_E_ARG;
    if (!h->on_device) return ENV_E_STATE;
    h->ktime = on != 0;
    h->kev_used = 0;
    return ENV_OK;
}

env_status env_potential_kernel_times(env_potential* h, float* ms, int32_t cap, int32_t* count) {
    if (!h || cap < 0 || (cap > 0 && !ms)) return ENV_E_ARG;
    if (!h->on_device) return ENV_E_STATE;
    DeviceGuard g(h->device);
    const int32_t pairs = int32_t(h->kev_used / 2);
    for (int32_t i = 0; i < pairs && i < cap; ++i) {
        if (hipEventSynchronize(h->kev[2 * i + 1]) != hipSuccess ||
            hipEventElapsedTime(&ms[i], h->kev[2 * i], h->kev[2 * i + 1]) != hipSuccess)
            return ENV_E_DEVICE;
    }
    if (count) *count = pairs;
    return ENV_OK;
}

env_status env_potential_info(const env_potential* h, env_info* info) {
    if (!h || !info) return ENV_E_ARG;
    *info = h->info;
    return ENV_OK;
}

env_status env_peak_probe(int32_t device, env_peak* out) {
    if (!out) return ENV_E_ARG;
    int dev = device;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return ENV_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return ENV_E_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return ENV_E_DEVICE;
    DeviceGuard g(dev);
    double ms[3] = {0.0, 0.0, 0.0};
    if (run_peak_probe(ms) != 0) return ENV_E_DEVICE;
    const double ops = double(peak_probe_lane_ops());
    out->fp32_fma_tflops = 2.0 * ops / (ms[0] * 1e-3) / 1e12;
    out->fp64_fma_tflops = 2.0 * ops / (ms[1] * 1e-3) / 1e12;
    out->rsq_f32_per_s = ops / (ms[2] * 1e-3);
    for (int k = 0; k < 3; ++k) out->ms[k] = ms[k];
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
    if (D) {
        std::fill(D, D + 35 * n, 0.0);
        for (int64_t k = 0; k < n; ++k)
            std::copy(pl.D.begin() + pl.d_off[k], pl.D.begin() + pl.d_off[k + 1], D + 35 * k);
    }
    return ENV_OK;
}

env_status env_potential_export_image(const env_potential* h, uint32_t* rec, int64_t rec_cap,
                                      int64_t* rec_words, uint32_t* segs, int64_t seg_cap,
                                      int64_t* seg_words) {
    if (!h) return ENV_E_ARG;
    if (!h->on_device) return ENV_E_STATE;
    static_assert(sizeof(Segment) == 32, "8 words per segment");
    const int64_t rw = h->rec_words, sw = 8 * h->n_segs_all;
    if (rec_words) *rec_words = rw;
    if (seg_words) *seg_words = sw;
    if ((rec && rec_cap < rw) || (segs && seg_cap < sw)) return ENV_E_ARG;
    DeviceGuard g(h->device);
    if (hipDeviceSynchronize() != hipSuccess) return ENV_E_DEVICE;
    if (rec && rw > 0 && hipMemcpy(rec, h->d_rec, size_t(rw) * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return ENV_E_DEVICE;
    if (segs && sw > 0 && hipMemcpy(segs, h->d_segs, size_t(sw) * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return ENV_E_DEVICE;
    return ENV_OK;
}

void env_potential_destroy(env_potential* h) {
    if (!h) return;
    if (!h->kev.empty()) {
        DeviceGuard g(h->device);
        for (hipEvent_t e : h->kev) (void)hipEventDestroy(e);
    }
    free_device(h);
    delete h;
}

}  // extern "C"
