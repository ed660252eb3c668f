// Batched evaluation of many independent environments in one persistent
// launch (env_batch_*), replayed from a captured HIP graph while the caller
// keeps its buffers.  The paper's outlook (Sec. I, Sec. V) is a GPU shared by
// several host processes; here one process batches many QM/MM instances.
//
// Instances of 32,768 points or more are evaluated in Morton order, as a
// single evaluation is: before each launch their points are sorted into the
// plan's own buffers (outside any graph: the sort library may record
// memory-set nodes), the persistent kernel reads those buffers, and a scatter
// kernel inside the graph writes the values back in the caller's order.
// While the caller's stream is being captured the plan uses a second
// argument table that reads and writes the caller's buffers directly.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "handle.h"
#include "sort_internal.h"

using namespace envpot;

struct env_batch {
    int device = -1;
    int precision = ENV_PREC_FP32C;
    int np = 4;
    int gran = 16;      // items per workgroup's fair share of the work (split granularity;
                        // the autotuner's pick on the 64-instance workload)
    int grid = 0;
    int cu_count = 256;
    int n_inst = 0;
    std::vector<env_potential*> hs;
    // work-queue shape (depends on the point counts, np and gran)
    std::vector<int64_t> n;
    std::vector<int> klog;
    std::vector<int64_t> part_off;      // offset of each instance's partials, -1 if S == 1
    std::vector<int64_t> sort_off;      // offset of each instance's sorted points, -1 if unsorted
    std::vector<BatchItem> items;
    // device side
    EvalArgs* d_args = nullptr;         // sorted instances read the plan's buffers
    EvalArgs* d_args_direct = nullptr;  // every instance reads the caller's buffers
    BatchItem* d_items = nullptr;
    SumDesc* d_sum = nullptr;
    SumDesc* d_sum_direct = nullptr;
    ScatterDesc* d_scat = nullptr;
    unsigned long long* d_counter = nullptr;
    double* d_part = nullptr;
    double* d_spts = nullptr;           // sorted points (3 per point)
    double* d_sout = nullptr;           // values in sorted order
    uint32_t* d_order = nullptr;
    int n_sum = 0;
    int64_t max_n_sum = 0;
    int n_scat = 0;
    int64_t max_n_scat = 0;
    int64_t sorted_points = 0;
    bool shape_valid = false;
    // pointers of the uploaded argument tables
    std::vector<const double*> pts;
    std::vector<double*> out;
    bool args_valid = false;
    // captured graph (sorted table)
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
    for (void* p : {static_cast<void*>(b->d_items), static_cast<void*>(b->d_part), static_cast<void*>(b->d_sum),
                    static_cast<void*>(b->d_sum_direct), static_cast<void*>(b->d_args),
                    static_cast<void*>(b->d_args_direct), static_cast<void*>(b->d_scat),
                    static_cast<void*>(b->d_spts), static_cast<void*>(b->d_sout), static_cast<void*>(b->d_order)})
        (void)hipFree(p);
    b->d_items = nullptr;
    b->d_part = nullptr;
    b->d_sum = b->d_sum_direct = nullptr;
    b->d_args = b->d_args_direct = nullptr;
    b->d_scat = nullptr;
    b->d_spts = b->d_sout = nullptr;
    b->d_order = nullptr;
    b->shape_valid = false;
    b->args_valid = false;
    drop_graph(b);
}

// Instances evaluated in Morton order (the rule of a single evaluation,
// including its ENVPOT_NO_SORT switch).
bool sorts(int64_t n) {
    const char* ns = std::getenv("ENVPOT_NO_SORT");
    return n >= kSortMinPoints && n <= int64_t(INT32_MAX) && !(ns && *ns && std::atoi(ns) != 0);
}

// Work items for point counts n: per instance a split factor such that an
// item costs at most ~1/gran of a workgroup's fair share, items sorted by
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
    const double target = std::max(1.0, total / (double(b->gran) * b->grid));
    b->n.assign(n, n + b->n_inst);
    b->klog.assign(b->n_inst, 0);
    b->part_off.assign(b->n_inst, -1);
    b->sort_off.assign(b->n_inst, -1);
    b->items.clear();
    std::vector<double> cost;
    int64_t part_words = 0, sorted = 0;
    b->n_sum = 0;
    b->max_n_sum = 0;
    b->n_scat = 0;
    b->max_n_scat = 0;
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
        if (sorts(n[i])) {
            b->sort_off[i] = sorted;
            sorted += n[i];
            ++b->n_scat;
            b->max_n_scat = std::max(b->max_n_scat, n[i]);
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
    b->sorted_points = sorted;
    std::vector<size_t> order(b->items.size());
    std::iota(order.begin(), order.end(), size_t(0));
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return cost[x] > cost[y]; });
    std::vector<BatchItem> sorted_items(b->items.size());
    for (size_t k = 0; k < order.size(); ++k) sorted_items[k] = b->items[order[k]];
    b->items.swap(sorted_items);
    const size_t ni = std::max<size_t>(b->items.size(), 1);
    auto dm = [](auto** p, size_t bytes) {
        return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(bytes, 8)) == hipSuccess;
    };
    const size_t ns = size_t(std::max(b->n_sum, 1)), nsc = size_t(std::max(b->n_scat, 1));
    if (!dm(&b->d_items, ni * sizeof(BatchItem)) || !dm(&b->d_args, size_t(b->n_inst) * sizeof(EvalArgs)) ||
        !dm(&b->d_args_direct, size_t(b->n_inst) * sizeof(EvalArgs)) || !dm(&b->d_sum, ns * sizeof(SumDesc)) ||
        !dm(&b->d_sum_direct, ns * sizeof(SumDesc)) || !dm(&b->d_scat, nsc * sizeof(ScatterDesc)) ||
        !dm(&b->d_part, size_t(part_words) * sizeof(double)) || !dm(&b->d_spts, size_t(sorted) * 3 * sizeof(double)) ||
        !dm(&b->d_sout, size_t(sorted) * sizeof(double)) || !dm(&b->d_order, size_t(sorted) * sizeof(uint32_t))) {
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
    b->stats.np = b->np;
    b->stats.granularity = b->gran;
    b->stats.sorted_points = sorted;
    b->shape_valid = true;
    return ENV_OK;
}

// Argument tables, sum and scatter descriptors for the caller's pointers.
env_status upload_args(env_batch* b, const double* const* points, double* const* out) {
    std::vector<EvalArgs> args(b->n_inst), direct(b->n_inst);
    std::vector<SumDesc> sums, sums_direct;
    std::vector<ScatterDesc> scat;
    for (int i = 0; i < b->n_inst; ++i) {
        env_potential* h = b->hs[i];
        const bool split = b->part_off[i] >= 0, sorted = b->sort_off[i] >= 0;
        double* part = split ? b->d_part + b->part_off[i] : nullptr;
        const double* spts = sorted ? b->d_spts + 3 * b->sort_off[i] : points[i];
        double* sout = sorted ? b->d_sout + b->sort_off[i] : out[i];
        args[i] = make_args(h, spts, b->n[i], split ? part : sout, b->klog[i]);
        direct[i] = make_args(h, points[i], b->n[i], split ? part : out[i], b->klog[i]);
        if (split) {
            sums.push_back({part, sout, b->n[i], 1 << b->klog[i], 0});
            sums_direct.push_back({part, out[i], b->n[i], 1 << b->klog[i], 0});
        }
        if (sorted) scat.push_back({sout, b->d_order + b->sort_off[i], out[i], b->n[i]});
    }
    auto up = [](void* dst, const void* src, size_t bytes) {
        return bytes == 0 || hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up(b->d_args, args.data(), args.size() * sizeof(EvalArgs)) ||
        !up(b->d_args_direct, direct.data(), direct.size() * sizeof(EvalArgs)) ||
        !up(b->d_sum, sums.data(), sums.size() * sizeof(SumDesc)) ||
        !up(b->d_sum_direct, sums_direct.data(), sums_direct.size() * sizeof(SumDesc)) ||
        !up(b->d_scat, scat.data(), scat.size() * sizeof(ScatterDesc)))
        return ENV_E_DEVICE;
    b->pts.assign(points, points + b->n_inst);
    b->out.assign(out, out + b->n_inst);
    b->args_valid = true;
    drop_graph(b);
    return ENV_OK;
}

// Morton order of the sorted instances' points into the plan's buffers
// (stream-ordered, never inside a graph).
env_status sort_inputs(env_batch* b, void* stream) {
    for (int i = 0; i < b->n_inst; ++i) {
        if (b->sort_off[i] < 0) continue;
        if (sort_points(b->pts[i], b->n[i], b->d_spts + 3 * b->sort_off[i], b->d_order + b->sort_off[i], stream) != 0)
            return ENV_E_DEVICE;
    }
    return ENV_OK;
}

// The graph-safe part of an evaluation: persistent kernel, fixed-order
// split sums and (sorted table) the scatter back to the caller's order.
int launch_all(env_batch* b, void* stream, bool sorted) {
    BatchArgs a;
    a.args = sorted ? b->d_args : b->d_args_direct;
    a.items = b->d_items;
    a.n_items = int64_t(b->items.size());
    a.counter = b->d_counter;
    a.boys = b->hs[0]->d_boys;
    a.rows32 = b->hs[0]->bp.rows32;
    a.pad = 0;
    int rc = launch_persistent(a, b->grid, b->precision, b->np, stream);
    if (rc == 0) rc = launch_sum_multi(sorted ? b->d_sum : b->d_sum_direct, b->n_sum, b->max_n_sum, stream);
    if (rc == 0 && sorted) rc = scatter_values_multi(b->d_scat, b->n_scat, b->max_n_scat, stream);
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
    b->cu_count = hs[0]->cu_count;
    b->hs.assign(hs, hs + n_inst);
    DeviceGuard g(b->device);
    b->grid = persistent_grid(b->precision, b->np, b->cu_count);
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
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (st && hipStreamIsCapturing(st, &cap) != hipSuccess) return ENV_E_DEVICE;
    const bool capturing = cap != hipStreamCaptureStatusNone;
    const bool same_n = b->shape_valid && std::equal(n, n + b->n_inst, b->n.begin());
    const bool same_ptr = same_n && b->args_valid && std::equal(points, points + b->n_inst, b->pts.begin()) &&
                          std::equal(out, out + b->n_inst, b->out.begin());
    if (!same_ptr) {
        // a new table cannot be set up while the caller records a graph
        if (capturing) return ENV_E_STATE;
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
    if (capturing) {
        // recorded into the caller's graph: the direct table, no sort
        ++b->stats.launches;
        return launch_all(b, stream, false) == 0 ? ENV_OK : ENV_E_DEVICE;
    }
    if (b->n_scat > 0) {
        const env_status s = sort_inputs(b, stream);
        if (s != ENV_OK) return s;
        ++b->stats.sorts;
    }
    const char* ng = std::getenv("ENVPOT_NO_GRAPH");
    const bool use_graph = allow_graph && st != nullptr && !(ng && *ng && *ng != '0');
    if (!use_graph) {
        ++b->stats.launches;
        return launch_all(b, stream, true) == 0 ? ENV_OK : ENV_E_DEVICE;
    }
    if (!b->exec) {
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed) != hipSuccess) return ENV_E_DEVICE;
        const int rc = launch_all(b, stream, true);
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

// Set the launch shape (points per lane, split granularity) and rebuild the
// work queue and tables for the current counts and pointers.
env_status set_shape(env_batch* b, int np, int gran, const double* const* points, const int64_t* n,
                     double* const* out) {
    b->np = np;
    b->gran = gran;
    b->grid = persistent_grid(b->precision, np, b->cu_count);
    env_status s = build_shape(b, n);
    if (s == ENV_OK) s = upload_args(b, points, out);
    return s;
}

}  // namespace

extern "C" {

env_status env_batch_eval(env_batch* b, const double* const* points, const int64_t* n,
                          double* const* out, void* stream) {
    return batch_eval(b, points, n, out, stream, true);
}

env_status env_batch_autotune(env_batch* b, const double* const* points, const int64_t* n, double* const* out,
                              void* stream) {
    if (!b || !points || !n || !out) return ENV_E_ARG;
    for (int i = 0; i < b->n_inst; ++i) {
        if (n[i] < 0) return ENV_E_ARG;
        if (n[i] > 0 && (!points[i] || !out[i])) return ENV_E_ARG;
    }
    if (!stream) return ENV_E_ARG;  // the plan's graph needs a stream of the caller's
    DeviceGuard g(b->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipStreamSynchronize(st) != hipSuccess) return ENV_E_DEVICE;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return ENV_E_DEVICE;
    }
    const bool fp64 = b->precision == ENV_PREC_FP64;
    const int nps32[] = {2, 4}, nps64[] = {1, 2};
    const int* nps = fp64 ? nps64 : nps32;
    const int grans[] = {4, 8, 16};
    float best = 1e30f;
    int best_np = b->np, best_gran = b->gran;
    env_status rc = ENV_OK;
    for (int a = 0; a < 2 && rc == ENV_OK; ++a) {
        for (int gi = 0; gi < 3 && rc == ENV_OK; ++gi) {
            rc = set_shape(b, nps[a], grans[gi], points, n, out);
            float ms = 0.0f;
            for (int rep = 0; rep < 3 && rc == ENV_OK; ++rep) {  // the first run captures and warms up
                if (hipEventRecord(e0, st) != hipSuccess) rc = ENV_E_DEVICE;
                if (rc == ENV_OK) rc = batch_eval(b, points, n, out, stream, true);
                if (rc == ENV_OK && hipEventRecord(e1, st) != hipSuccess) rc = ENV_E_DEVICE;
                if (rc == ENV_OK && hipEventSynchronize(e1) != hipSuccess) rc = ENV_E_DEVICE;
                float t = 0.0f;
                if (rc == ENV_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = ENV_E_DEVICE;
                if (rep > 0) ms += t;
            }
            if (rc == ENV_OK && ms < best) {
                best = ms;
                best_np = nps[a];
                best_gran = grans[gi];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == ENV_OK) rc = set_shape(b, best_np, best_gran, points, n, out);
    if (rc == ENV_OK) ++b->stats.autotunes;
    return rc;
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
