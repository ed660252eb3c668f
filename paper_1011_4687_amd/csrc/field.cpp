// Field E = -grad V of the environment (C ABI entry point and host tables).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <vector>

#include "field_internal.h"
#include "handle.h"
#include "sort_internal.h"

namespace envpot {

void build_field_tables(const BoysParams& bp, std::vector<float>& t32, std::vector<double>& t64,
                        FieldParams& fp) {
    fp = FieldParams{};
    double max32 = 0.0, max64 = 0.0;
    for (int L = 0; L <= kLMax; ++L) {
        // the far form of the field needs the asymptote of F_0 .. F_{L+1}
        const double f32 = double(float(far_threshold(L + 1, 0x1p-28L)));
        const double f64 = far_threshold(L + 1, 0x1p-56L);
        fp.ratio32[L] = float(f32 / double(bp.tfar32[L]));
        fp.ratio64[L] = f64 / bp.tfar64[L];
        // never below 1: the field radius contains the potential's
        fp.ratio32[L] = std::max(fp.ratio32[L], 1.0f);
        fp.ratio64[L] = std::max(fp.ratio64[L], 1.0);
        fp.cl_ratio32 = std::max(fp.cl_ratio32, fp.ratio32[L]);
        fp.cl_ratio64 = std::max(fp.cl_ratio64, fp.ratio64[L]);
        max32 = std::max(max32, double(bp.tfar32[L]) * fp.ratio32[L]);
        max64 = std::max(max64, bp.tfar64[L] * fp.ratio64[L]);
    }
    // rows up to the largest field threshold, plus the rounding margin of
    // the nearest-row index
    fp.rows32 = int(max32 * kBoysGridInv) + 2;
    fp.rows64 = int(max64 * kBoysGridInv) + 2;
    t32.assign(size_t(fp.rows32) * kFieldRowF32, 0.0f);
    t64.assign(size_t(fp.rows64) * kFieldRowF64, 0.0);
    long double F[kFieldRowF64];
    for (int k = 0; k < fp.rows32; ++k) {
        boys_ld(kFieldRowF32 - 1, k / (long double)kBoysGridInv, F);
        for (int n = 0; n < kFieldRowF32; ++n) t32[size_t(k) * kFieldRowF32 + n] = float(F[n]);
    }
    for (int k = 0; k < fp.rows64; ++k) {
        boys_ld(kFieldRowF64 - 1, k / (long double)kBoysGridInv, F);
        for (int n = 0; n < kFieldRowF64; ++n) t64[size_t(k) * kFieldRowF64 + n] = double(F[n]);
    }
}

}  // namespace envpot

using namespace envpot;

namespace {
env_status field_core(env_potential* h, const double* points, int64_t n, double* out, void* stream);
}  // namespace

extern "C" {

env_status env_potential_eval_field(env_potential* h, const double* points, int64_t n, double* out,
                                    void* stream) {
    if (!h || n < 0) return ENV_E_ARG;
    if (n == 0) return ENV_OK;
    if (!points || !out) return ENV_E_ARG;
    if (!h->on_device) return ENV_E_STATE;
    DeviceGuard g(h->device);
    const char* ns = std::getenv("ENVPOT_NO_SORT");
    if (n < kSortMinPoints || n > int64_t(INT32_MAX) || (ns && std::atoi(ns) != 0) || stream_capturing(stream))
        return field_core(h, points, n, out, stream);
    // large calls: evaluate the points in Morton order, then restore the caller's order
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *spts = nullptr, *sout = nullptr;
    uint32_t* order = nullptr;
    if (hipMallocAsync(reinterpret_cast<void**>(&spts), size_t(n) * 3 * sizeof(double), st) != hipSuccess)
        return ENV_E_NOMEM;
    env_status rc = ENV_OK;
    if (hipMallocAsync(reinterpret_cast<void**>(&sout), size_t(n) * 4 * sizeof(double), st) != hipSuccess ||
        hipMallocAsync(reinterpret_cast<void**>(&order), size_t(n) * sizeof(uint32_t), st) != hipSuccess)
        rc = ENV_E_NOMEM;
    if (rc == ENV_OK && sort_points(points, n, spts, order, stream) != 0) rc = ENV_E_DEVICE;
    if (rc == ENV_OK) rc = field_core(h, spts, n, sout, stream);
    if (rc == ENV_OK && scatter_rows4(sout, order, n, out, stream) != 0) rc = ENV_E_DEVICE;
    (void)hipFreeAsync(order, st);
    (void)hipFreeAsync(sout, st);
    (void)hipFreeAsync(spts, st);
    return rc;
}

}  // extern "C"

namespace {

env_status field_core(env_potential* h, const double* points, int64_t n, double* out, void* stream) {
    // two points per lane at four waves per SIMD (mid workload: FP32C 46 ms
    // against 53 ms with one; FP64 79 against 81 ms)
    int np = 2;
    if (const char* e = std::getenv("ENVPOT_FIELD_NP")) {  // tuning override
        const int v = std::atoi(e);
        if (v == 1 || v == 2) np = v;
    }
    // split factor: enough waves to keep ~48 per SIMD in flight over the run
    // (mid: FP32C 41.2 ms with 64 splits against 42.2 ms with 32, FP64 71.8
    // against 73.1 ms)
    const int64_t waves = (n + 64 * np - 1) / (64 * np);
    const int64_t want = int64_t(h->cu_count) * 4 * 48;
    int k = 0;
    while (k < kMaxSplitLog2 && waves * (int64_t(1) << k) < want) ++k;
    if (const char* e = std::getenv("ENVPOT_FIELD_SPLIT_LOG2")) {  // tuning override
        const int v = std::atoi(e);
        if (v >= 0 && v <= kMaxSplitLog2) k = v;
    }
    const int S = 1 << k;
    FieldArgs a;
    a.pts = points;
    a.n = n;
    a.segs = h->d_segs + h->seg_off[k];
    a.split = h->d_split + h->split_off[k];
    a.rec = h->d_rec;
    a.nuc = h->d_nuc;
    a.boys = h->d_boys_field;
    a.boxes = h->use_boxes ? h->d_boxes : nullptr;
    a.fp = h->fp;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (S == 1) {
        a.out = out;
        return launch_field(a, 1, h->precision, np, stream) == 0 ? ENV_OK : ENV_E_DEVICE;
    }
    double* part = nullptr;
    if (hipMallocAsync(reinterpret_cast<void**>(&part), size_t(S) * size_t(n) * 4 * sizeof(double), st) !=
        hipSuccess)
        return ENV_E_NOMEM;
    a.out = part;
    int rc = launch_field(a, S, h->precision, np, stream);
    if (rc == 0) rc = launch_sum_splits(part, S, 4 * n, out, stream);
    (void)hipFreeAsync(part, st);
    return rc == 0 ? ENV_OK : ENV_E_DEVICE;
}

}  // namespace
