// C ABI of the cell-sum environment (the paper's own form of the field:
// nuclei plus point-charge cells, Sec. II.B, Eq. ElectrostaticField).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>
#include <xmmintrin.h>

#include "cells_internal.h"
#include "envpot_internal.h"
#include "handle.h"

struct env_cells {
    int device = -1;
    int precision = ENV_PREC_FP32C;
    int cu_count = 256;
    int64_t m = 0;                 // cells
    int32_t n_nuc = 0;
    uint32_t* d_cells = nullptr;   // records, kCellWords each
    double* d_nuc = nullptr;
    int32_t* d_split = nullptr;    // split tables for S = 1, 2, ..., 64
    int64_t split_off[envpot::kMaxSplitLog2 + 1] = {};
    double* d_part = nullptr;      // single-point mode: one partial per workgroup
    unsigned int* d_ticket = nullptr;
    int one_grid = 128;            // workgroups of single-point mode 0
    // resident single-point mode
    envpot::CellMailbox* box = nullptr;  // pinned fine-grained host memory
    envpot::CellRelay* d_relay = nullptr;
    double* d_rpart = nullptr;
    unsigned int* d_rticket = nullptr;
    hipStream_t rstream = nullptr;       // the resident kernel's own stream
    bool resident = false;               // launched and not yet joined
    int rmode = 0;
    double ridle = 0.0;
    uint64_t seq = 0;                    // last posted position
};

namespace {

using envpot::DeviceGuard;

env_status resident_stop(env_cells* h);

void free_cells(env_cells* h) {
    DeviceGuard g(h->device);
    (void)resident_stop(h);
    if (h->rstream) (void)hipStreamDestroy(h->rstream);
    if (h->box) (void)hipHostFree(h->box);
    (void)hipFree(h->d_relay);
    (void)hipFree(h->d_rpart);
    (void)hipFree(h->d_rticket);
    (void)hipFree(h->d_cells);
    (void)hipFree(h->d_nuc);
    (void)hipFree(h->d_split);
    (void)hipFree(h->d_part);
    (void)hipFree(h->d_ticket);
}

// Ask the resident kernel to exit and join it (also after it left on its
// own for lack of positions).
env_status resident_stop(env_cells* h) {
    if (!h->resident) return ENV_OK;
    __atomic_store_n(&h->box->stop, 1u, __ATOMIC_RELEASE);
    const bool ok = hipStreamSynchronize(h->rstream) == hipSuccess;
    h->resident = false;
    return ok ? ENV_OK : ENV_E_DEVICE;
}

env_status resident_launch(env_cells* h) {
    const int grid = h->rmode == 0 ? h->one_grid : envpot::kCellsPaperGrid;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device) != hipSuccess || khz <= 0)
        return ENV_E_DEVICE;
    envpot::CellMailbox* b = h->box;
    b->stop = 0;
    b->running = 1;
    b->req_seq = h->seq;
    b->done_seq = h->seq;
    std::atomic_thread_fence(std::memory_order_seq_cst);
    envpot::CellRelay r{};
    r.seq = h->seq;
    if (hipMemcpyAsync(h->d_relay, &r, sizeof(r), hipMemcpyHostToDevice, h->rstream) != hipSuccess ||
        hipMemsetAsync(h->d_rticket, 0, sizeof(unsigned int), h->rstream) != hipSuccess ||
        hipStreamSynchronize(h->rstream) != hipSuccess)
        return ENV_E_DEVICE;
    envpot::CellResidentArgs a{};
    a.box = b;
    a.relay = h->d_relay;
    a.cells = h->d_cells;
    a.m = h->m;
    a.nuc = h->d_nuc;
    a.n_nuc = h->n_nuc;
    a.part = h->d_rpart;
    a.ticket = h->d_rticket;
    a.start_seq = h->seq;
    const double tps = double(khz) * 1e3;
    a.idle_ticks = uint64_t(h->ridle * tps);
    a.grace_ticks = uint64_t(tps);
    if (envpot::launch_cells_resident(a, grid, h->precision, h->rstream) != 0) {
        b->running = 0;
        return ENV_E_DEVICE;
    }
    h->resident = true;
    return ENV_OK;
}

template <typename T>
env_status to_device(const std::vector<T>& v, T** dst) {
    const size_t nb = std::max<size_t>(v.size(), 1) * sizeof(T);
    if (hipMalloc(reinterpret_cast<void**>(dst), nb) != hipSuccess) return ENV_E_NOMEM;
    if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return ENV_E_DEVICE;
    return ENV_OK;
}

// Points per lane and cell-split factor of a batched evaluation: enough
// waves in flight over the whole launch, about 24 per SIMD in FP32C and 48
// in FP64 (268,398 cells, 131,072 points: FP32C 11.0 ms with 64 splits,
// 11.1 ms median with 128; FP64 15.1 ms with 64 against 15.6 ms with 32).
void cells_shape(const env_cells* h, int64_t n, int* np, int* klog) {
    const bool fp64 = h->precision == ENV_PREC_FP64;
    *np = fp64 ? 2 : 4;
    const int64_t waves = (n + 64 * *np - 1) / (64 * *np);
    const int64_t want = int64_t(h->cu_count) * 4 * (fp64 ? 48 : 24);
    int k = 0;
    while (k < envpot::kMaxSplitLog2 && waves * (int64_t(1) << k) < want && (h->m >> (k + 1)) >= 64) ++k;
    if (const char* e = std::getenv("ENVPOT_CELLS_SPLIT_LOG2")) {  // tuning override
        const int v = std::atoi(e);
        if (v >= 0 && v <= envpot::kMaxSplitLog2 && (h->m >> v) >= 64) k = v;
    }
    *klog = k;
}

}  // namespace

extern "C" {

env_status env_cells_create(const env_nucleus* nuclei, int32_t n_nuclei, const double* cells,
                            int64_t n_cells, const env_options* options, env_cells** out) {
    if (!out) return ENV_E_ARG;
    *out = nullptr;
    if (n_nuclei < 0 || n_cells < 0 || n_cells > int64_t(INT32_MAX)) return ENV_E_ARG;
    if ((n_nuclei > 0 && !nuclei) || (n_cells > 0 && !cells)) return ENV_E_ARG;
    env_options opt;
    if (options) opt = *options;
    else env_options_default(&opt);
    if (opt.precision != ENV_PREC_FP64 && opt.precision != ENV_PREC_FP32C) return ENV_E_ARG;
    for (int32_t a = 0; a < n_nuclei; ++a)
        for (int c = 0; c < 3; ++c)
            if (!std::isfinite(nuclei[a].xyz[c]) || !std::isfinite(nuclei[a].Z)) return ENV_E_ARG;
    for (int64_t m = 0; m < 4 * n_cells; ++m)
        if (!std::isfinite(cells[m])) return ENV_E_ARG;
    int device = opt.device;
    if (device < 0 && hipGetDevice(&device) != hipSuccess) return ENV_E_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return ENV_E_DEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return ENV_E_DEVICE;

    env_cells* h = new (std::nothrow) env_cells;
    if (!h) return ENV_E_NOMEM;
    h->device = device;
    h->precision = opt.precision;
    h->cu_count = prop.multiProcessorCount;
    h->m = n_cells;
    h->one_grid = std::max(1, prop.multiProcessorCount / 2);  // latency optimum (measured)
    if (const char* e = std::getenv("ENVPOT_CELLS_GRID")) {  // tuning override
        const int g = std::atoi(e);
        if (g >= 1 && g <= 4 * prop.multiProcessorCount) h->one_grid = g;
    }
    env_status st = ENV_OK;
    try {
        // records
        std::vector<uint32_t> rec(size_t(std::max<int64_t>(n_cells, 1)) * envpot::kCellWords, 0u);
        for (int64_t m = 0; m < n_cells; ++m) {
            uint32_t* r = &rec[size_t(m) * envpot::kCellWords];
            double* d = reinterpret_cast<double*>(r);
            d[0] = cells[4 * m];
            d[1] = cells[4 * m + 1];
            d[2] = cells[4 * m + 2];
            if (h->precision == ENV_PREC_FP64) d[3] = cells[4 * m + 3];
            else reinterpret_cast<float*>(r)[6] = float(cells[4 * m + 3]);
        }
        std::vector<double> nuc;
        for (int32_t a = 0; a < n_nuclei; ++a) {
            if (nuclei[a].Z == 0.0) continue;
            nuc.insert(nuc.end(), {nuclei[a].xyz[0], nuclei[a].xyz[1], nuclei[a].xyz[2], nuclei[a].Z});
        }
        h->n_nuc = int32_t(nuc.size() / 4);
        // split tables: S equal cell ranges
        std::vector<int32_t> split;
        for (int k = 0; k <= envpot::kMaxSplitLog2; ++k) {
            const int S = 1 << k;
            h->split_off[k] = int64_t(split.size());
            for (int s = 0; s <= S; ++s) split.push_back(int32_t((n_cells * s) / S));
        }
        DeviceGuard g(device);
        st = to_device(rec, &h->d_cells);
        if (st == ENV_OK) st = to_device(nuc, &h->d_nuc);
        if (st == ENV_OK) st = to_device(split, &h->d_split);
        if (st == ENV_OK && hipMalloc(reinterpret_cast<void**>(&h->d_part),
                                      size_t(std::max(h->one_grid, envpot::kCellsPaperGrid)) * sizeof(double)) !=
                                hipSuccess)
            st = ENV_E_NOMEM;
        if (st == ENV_OK && hipMalloc(reinterpret_cast<void**>(&h->d_ticket), sizeof(unsigned int)) != hipSuccess)
            st = ENV_E_NOMEM;
        if (st == ENV_OK && hipMemset(h->d_ticket, 0, sizeof(unsigned int)) != hipSuccess) st = ENV_E_DEVICE;
    } catch (const std::bad_alloc&) {
        st = ENV_E_NOMEM;
    }
    if (st != ENV_OK) {
        free_cells(h);
        delete h;
        return st;
    }
    *out = h;
    return ENV_OK;
}

env_status env_cells_eval(env_cells* h, const double* points, int64_t n, double* out, void* stream) {
    if (!h || n < 0) return ENV_E_ARG;
    if (n == 0) return ENV_OK;
    if (!points || !out) return ENV_E_ARG;
    DeviceGuard g(h->device);
    int np, k;
    cells_shape(h, n, &np, &k);
    const int S = 1 << k;
    hipStream_t st = static_cast<hipStream_t>(stream);
    envpot::CellArgs a{};
    a.pts = points;
    a.n = n;
    a.cells = h->d_cells;
    a.split = h->d_split + h->split_off[k];
    a.nuc = h->d_nuc;
    a.n_nuc = h->n_nuc;
    if (S == 1) {
        a.out = out;
        return envpot::launch_cells(a, 1, h->precision, np, stream) == 0 ? ENV_OK : ENV_E_DEVICE;
    }
    double* part = nullptr;
    if (hipMallocAsync(reinterpret_cast<void**>(&part), size_t(S) * size_t(n) * sizeof(double), st) !=
        hipSuccess)
        return ENV_E_NOMEM;
    a.out = part;
    int rc = envpot::launch_cells(a, S, h->precision, np, stream);
    if (rc == 0) rc = envpot::launch_sum_splits(part, S, n, out, stream);
    (void)hipFreeAsync(part, st);
    return rc == 0 ? ENV_OK : ENV_E_DEVICE;
}

env_status env_cells_eval_single(env_cells* h, const double* point, double* out, int32_t mode,
                                 void* stream) {
    if (!h || !point || !out || (mode != 0 && mode != 1)) return ENV_E_ARG;
    DeviceGuard g(h->device);
    envpot::CellOneArgs a{};
    a.pt = point;
    a.cells = h->d_cells;
    a.m = h->m;
    a.nuc = h->d_nuc;
    a.n_nuc = h->n_nuc;
    a.part = h->d_part;
    a.ticket = h->d_ticket;
    a.out = out;
    const int grid = mode == 0 ? h->one_grid : envpot::kCellsPaperGrid;
    return envpot::launch_cells_one(a, grid, h->precision, stream) == 0 ? ENV_OK : ENV_E_DEVICE;
}

env_status env_cells_resident_start(env_cells* h, int32_t mode, double idle_s) {
    if (!h || (mode != 0 && mode != 1) || !(idle_s > 0.0) || !(idle_s <= 3600.0)) return ENV_E_ARG;
    DeviceGuard g(h->device);
    if (h->resident && __atomic_load_n(&h->box->running, __ATOMIC_ACQUIRE) != 0 && h->rmode == mode &&
        h->ridle == idle_s)
        return ENV_OK;
    if (resident_stop(h) != ENV_OK) return ENV_E_DEVICE;
    // buffers and stream on first use (each one retried if an earlier start failed)
    if (!h->box) {
        void* p = nullptr;
        if (hipHostMalloc(&p, sizeof(envpot::CellMailbox), hipHostMallocCoherent) != hipSuccess) return ENV_E_NOMEM;
        h->box = static_cast<envpot::CellMailbox*>(p);
        std::memset(h->box, 0, sizeof(envpot::CellMailbox));
    }
    const int gmax = std::max(h->one_grid, envpot::kCellsPaperGrid);
    if (!h->d_relay && hipMalloc(reinterpret_cast<void**>(&h->d_relay), sizeof(envpot::CellRelay)) != hipSuccess)
        return ENV_E_NOMEM;
    if (!h->d_rpart && hipMalloc(reinterpret_cast<void**>(&h->d_rpart), size_t(gmax) * sizeof(double)) != hipSuccess)
        return ENV_E_NOMEM;
    if (!h->d_rticket && hipMalloc(reinterpret_cast<void**>(&h->d_rticket), sizeof(unsigned int)) != hipSuccess)
        return ENV_E_NOMEM;
    if (!h->rstream && hipStreamCreateWithFlags(&h->rstream, hipStreamNonBlocking) != hipSuccess) {
        h->rstream = nullptr;
        return ENV_E_DEVICE;
    }
    h->rmode = mode;
    h->ridle = idle_s;
    return resident_launch(h);
}

env_status env_cells_resident_eval(env_cells* h, const double* point, double* out, double timeout_s) {
    if (!h || !point || !out || !(timeout_s > 0.0)) return ENV_E_ARG;
    if (!h->resident) return ENV_E_STATE;
    envpot::CellMailbox* b = h->box;
    if (__atomic_load_n(&b->running, __ATOMIC_ACQUIRE) == 0) {
        // the kernel left after idle_s without a position: start it again
        DeviceGuard g(h->device);
        if (resident_stop(h) != ENV_OK || resident_launch(h) != ENV_OK) return ENV_E_DEVICE;
    }
    for (int c = 0; c < 3; ++c) b->point[c] = point[c];
    const uint64_t k = ++h->seq;
    __atomic_store_n(&b->req_seq, k, __ATOMIC_RELEASE);
    const auto t0 = std::chrono::steady_clock::now();
    for (uint64_t it = 0;; ++it) {
        if (__atomic_load_n(&b->done_seq, __ATOMIC_ACQUIRE) == k) {
            *out = b->value;
            return ENV_OK;
        }
        if ((it & 1023) == 1023) {
            if (__atomic_load_n(&b->running, __ATOMIC_ACQUIRE) == 0 &&
                __atomic_load_n(&b->done_seq, __ATOMIC_ACQUIRE) != k) {
                // left for lack of positions just before this one arrived
                DeviceGuard g(h->device);
                h->seq = k - 1;
                if (resident_stop(h) != ENV_OK || resident_launch(h) != ENV_OK) return ENV_E_DEVICE;
                h->seq = k;
                __atomic_store_n(&b->req_seq, k, __ATOMIC_RELEASE);
            }
            if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > timeout_s) {
                DeviceGuard g(h->device);
                (void)resident_stop(h);
                return ENV_E_DEVICE;
            }
        }
        _mm_pause();
    }
}

env_status env_cells_resident_stop(env_cells* h) {
    if (!h) return ENV_E_ARG;
    DeviceGuard g(h->device);
    return resident_stop(h);
}

void env_cells_destroy(env_cells* h) {
    if (!h) return;
    free_cells(h);
    delete h;
}

}  // extern "C"
