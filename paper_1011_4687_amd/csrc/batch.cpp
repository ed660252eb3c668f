// Batched evaluation of many independent environments in one persistent
// launch (env_batch_*), replayed from a captured HIP graph while the caller
// keeps its buffers.  The paper's outlook (Sec. I, Sec. V) is a GPU shared by
// several host processes; here one process batches many QM/MM instances.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "handle.h"

using namespace envpot;

struct env_batch {
    int device = -1;
    int precision = ENV_PREC_FP32C;
    int np = 4;
    int grid = 0;
    int n_inst = 0;
    std::vector<env_potential*> hs;
    // work-queue shape (depends on the point counts)
    std::vector<int64_t> n;
    std::vector<int> klog;
    std::vector<int64_t> part_off;      // offset of each instance's partials, -1 if S == 1
    std::vector<BatchItem> items;
    // device side
    EvalArgs* d_args = nullptr;
    BatchItem* d_items = nullptr;
    SumDesc* d_sum = nullptr;
    unsigned long long* d_counter = nullptr;
    double* d_part = nullptr;
    int n_sum = 0;
    int64_t max_n_sum = 0;
    bool shape_valid = false;
    // pointers of the uploaded argument table
    std::vector<const double*> pts;
    std::vector<double*> out;
    bool args_valid = false;
    // captured graph
    hipGraphExec_t exec = nullptr;
    env_batch_stats stats{};
};

namespace {

const double kW32[kLMax + 1] = {1.0, 1.5, 2.6, 4.4, 7.5};
const double kW64[kLMax + 1] = {1.0, 1.4, 2.3, 3.8, 6.3};

void drop_graph(env_batch* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
}

void free_shape(env_batch* b) {
    (void)hipFree(b->d_items);
    (void)hipFree(b->d_part);
    (void)hipFree(b->d_sum);
    (void)hipFree(b->d_args);
    b->d_items = nullptr;
    b->d_part = nullptr;
    b->d_sum = nullptr;
    b->d_args = nullptr;
    b->shape_valid = false;
    b->args_valid = false;
    drop_graph(b);
}

// Work items for point counts n: per instance a split factor such that an
// item costs at most ~1/8 of a workgroup's fair share, items sorted by
// decreasing cost.
env_status build_shape(env_batch* b, const int64_t* n) {
    free_shape(b);
    const int per = kBlock * b->np;
    const double* w = b->precision == ENV_PREC_FP64 ? kW64 : kW32;
    std::vector<double> pcost(b->n_inst, 0.0);
    double total = 0.0;
    for (int i = 0; i < b->n_inst; ++i) {
        const env_info& in = b->hs[i]->info;
        for (int L = 0; L <= kLMax; ++L) pcost[i] += double(in.n_pairs_by_L[L]) * w[L];
        pcost[i] += 0.6 * in.n_nuclei + 1.0;
        total += double(n[i]) * pcost[i];
    }
    const double target = std::max(1.0, total / (8.0 * b->grid));
    b->n.assign(n, n + b->n_inst);
    b->klog.assign(b->n_inst, 0);
    b->part_off.assign(b->n_inst, -1);
    b->items.clear();
    std::vector<double> cost;
    int64_t part_words = 0;
    b->n_sum = 0;
    b->max_n_sum = 0;
    for (int i = 0; i < b->n_inst; ++i) {
        if (n[i] == 0) continue;
        int k = 0;
        while (k < kMaxSplitLog2 && double(per) * pcost[i] / double(1 << k) > target) ++k;
        b->klog[i] = k;
        const int S = 1 << k;
        if (S > 1) {
            b->part_off[i] = part_words;
            part_words += int64_t(S) * n[i];
            ++b->n_sum;
            b->max_n_sum = std::max(b->max_n_sum, n[i]);
        }
        const int64_t nb = (n[i] + per - 1) / per;
        for (int64_t pb = 0; pb < nb; ++pb) {
            const int64_t pts = std::min<int64_t>(per, n[i] - pb * per);
            for (int s = 0; s < S; ++s) {
                b->items.push_back({i, s, pb});
                cost.push_back(double(pts) * pcost[i] / S);
            }
        }
    }
    std::vector<size_t> order(b->items.size());
    std::iota(order.begin(), order.end(), size_t(0));
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    std::vector<BatchItem> sorted(b->items.size());
    for (size_t k = 0; k < order.size(); ++k) sorted[k] = b->items[order[k]];
    b->items.swap(sorted);
    const size_t ni = std::max<size_t>(b->items.size(), 1);
    if (hipMalloc(reinterpret_cast<void**>(&b->d_items), ni * sizeof(BatchItem)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&b->d_args), size_t(b->n_inst) * sizeof(EvalArgs)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&b->d_sum), size_t(std::max(b->n_sum, 1)) * sizeof(SumDesc)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&b->d_part), size_t(std::max<int64_t>(part_words, 1)) * sizeof(double)) != hipSuccess) {
        free_shape(b);
        return ENV_E_NOMEM;
    }
    if (!b->items.empty() &&
        hipMemcpy(b->d_items, b->items.data(), b->items.size() * sizeof(BatchItem), hipMemcpyHostToDevice) != hipSuccess) {
        free_shape(b);
        return ENV_E_DEVICE;
    }
    b->stats.n_items = int64_t(b->items.size());
    b->stats.grid = b->grid;
    b->shape_valid = true;
    return ENV_OK;
}

// Argument table and sum descriptors for the caller's pointers.
env_status upload_args(env_batch* b, const double* const* points, double* const* out) {
    std::vector<EvalArgs> args(b->n_inst);
    std::vector<SumDesc> sums;
    for (int i = 0; i < b->n_inst; ++i) {
        env_potential* h = b->hs[i];
        double* o = b->part_off[i] >= 0 ? b->d_part + b->part_off[i] : out[i];
        args[i] = make_args(h, points[i], b->n[i], o, b->klog[i]);
        if (b->part_off[i] >= 0) sums.push_back({b->d_part + b->part_off[i], out[i], b->n[i], 1 << b->klog[i], 0});
    }
    if (hipMemcpy(b->d_args, args.data(), args.size() * sizeof(EvalArgs), hipMemcpyHostToDevice) != hipSuccess)
        return ENV_E_DEVICE;
    if (!sums.empty() &&
        hipMemcpy(b->d_sum, sums.data(), sums.size() * sizeof(SumDesc), hipMemcpyHostToDevice) != hipSuccess)
        return ENV_E_DEVICE;
    b->pts.assign(points, points + b->n_inst);
    b->out.assign(out, out + b->n_inst);
    b->args_valid = true;
    drop_graph(b);
    return ENV_OK;
}

int launch_all(env_batch* b, void* stream) {
    BatchArgs a;
    a.args = b->d_args;
    a.items = b->d_items;
    a.n_items = int64_t(b->items.size());
    a.counter = b->d_counter;
    a.boys = b->hs[0]->d_boys;
    a.rows32 = b->hs[0]->bp.rows32;
    a.pad = 0;
    int rc = launch_persistent(a, b->grid, b->precision, b->np, stream);
    if (rc == 0) rc = launch_sum_multi(b->d_sum, b->n_sum, b->max_n_sum, stream);
    return rc;
}

}  // namespace

extern "C" {

env_status env_batch_create(env_potential* const* hs, int32_t n_inst, env_batch** out) {
    if (!out) return ENV_E_ARG;
    *out = nullptr;
    if (n_inst <= 0 || !hs) return ENV_E_ARG;
    for (int i = 0; i < n_inst; ++i) {
        if (!hs[i]) return ENV_E_ARG;
        if (!hs[i]->on_device) return ENV_E_STATE;
        if (hs[i]->device != hs[0]->device || hs[i]->precision != hs[0]->precision) return ENV_E_ARG;
    }
    env_batch* b = new (std::nothrow) env_batch();
    if (!b) return ENV_E_NOMEM;
    b->device = hs[0]->device;
    b->precision = hs[0]->precision;
    b->np = b->precision == ENV_PREC_FP64 ? 2 : 4;
    b->n_inst = n_inst;
    b->hs.assign(hs, hs + n_inst);
    DeviceGuard g(b->device);
    b->grid = persistent_grid(b->precision, b->np, hs[0]->cu_count);
    if (hipMalloc(reinterpret_cast<void**>(&b->d_counter), sizeof(unsigned long long)) != hipSuccess) {
        delete b;
        return ENV_E_NOMEM;
    }
    *out = b;
    return ENV_OK;
}

}  // extern "C"

namespace {

env_status batch_eval(env_batch* b, const double* const* points, const int64_t* n,
                      double* const* out, void* stream, bool allow_graph) {
    if (!b || !points || !n || !out) return ENV_E_ARG;
    for (int i = 0; i < b->n_inst; ++i) {
        if (n[i] < 0) return ENV_E_ARG;
        if (n[i] > 0 && (!points[i] || !out[i])) return ENV_E_ARG;
    }
    DeviceGuard g(b->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool same_n = b->shape_valid && std::equal(n, n + b->n_inst, b->n.begin());
    const bool same_ptr = same_n && b->args_valid && std::equal(points, points + b->n_inst, b->pts.begin()) &&
                          std::equal(out, out + b->n_inst, b->out.begin());
    if (!same_ptr) {
        // earlier launches on this stream may still read the tables being replaced
        if (hipStreamSynchronize(st) != hipSuccess) return ENV_E_DEVICE;
        if (!same_n) {
            const env_status s = build_shape(b, n);
            if (s != ENV_OK) return s;
        }
        const env_status s = upload_args(b, points, out);
        if (s != ENV_OK) return s;
    }
    if (b->items.empty()) return ENV_OK;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (st && hipStreamIsCapturing(st, &cap) != hipSuccess) return ENV_E_DEVICE;
    const char* ng = std::getenv("ENVPOT_NO_GRAPH");
    const bool use_graph = allow_graph && st != nullptr && cap == hipStreamCaptureStatusNone &&
                           !(ng && *ng && *ng != '0');
    if (!use_graph) {
        ++b->stats.launches;
        return launch_all(b, stream) == 0 ? ENV_OK : ENV_E_DEVICE;
    }
    if (!b->exec) {
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess) return ENV_E_DEVICE;
        const int rc = launch_all(b, stream);
        const hipError_t e = hipStreamEndCapture(st, &graph);
        if (rc != 0 || e != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return ENV_E_DEVICE;
        }
        const hipError_t ie = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ie != hipSuccess) {
            b->exec = nullptr;
            return ENV_E_DEVICE;
        }
        ++b->stats.captures;
    }
    if (hipGraphLaunch(b->exec, st) != hipSuccess) return ENV_E_DEVICE;
    ++b->stats.graph_launches;
    return ENV_OK;
}

}  // namespace

extern "C" {

env_status env_batch_eval(env_batch* b, const double* const* points, const int64_t* n,
                          double* const* out, void* stream) {
    return batch_eval(b, points, n, out, stream, true);
}

env_status env_batch_get_stats(const env_batch* b, env_batch_stats* s) {
    if (!b || !s) return ENV_E_ARG;
    *s = b->stats;
    return ENV_OK;
}

void env_batch_destroy(env_batch* b) {
    if (!b) return;
    DeviceGuard g(b->device);
    free_shape(b);
    (void)hipFree(b->d_counter);
    delete b;
}

env_status env_potential_eval_batched(env_potential* const* hs, int32_t n_inst,
                                      const double* const* points, const int64_t* n,
                                      double* const* out, void* stream) {
    if (n_inst < 0) return ENV_E_ARG;
    if (n_inst == 0) return ENV_OK;
    env_batch* b = nullptr;
    env_status s = env_batch_create(hs, n_inst, &b);
    if (s != ENV_OK) return s;
    s = batch_eval(b, points, n, out, stream, false);
    if (s == ENV_OK) {
        DeviceGuard g(b->device);
        if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) s = ENV_E_DEVICE;
    }
    env_batch_destroy(b);
    return s;
}

}  // extern "C"
