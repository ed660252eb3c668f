// Host driver of the coordinate-MLP surrogate (env_surrogate_*): training on
// samples of the exact kernel, a validated voxel gate, and gated evaluation
// that sends every point outside the gate to the exact kernel.  The learned
// model is an addition to the paper's method, which has none.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "handle.h"
#include "surrogate_internal.h"

using namespace envpot;

namespace {

struct Workspace {
    int64_t cap = 0;    // rows (multiple of 32)
    bool train = false;
    uint16_t* H[kLayers + 1] = {};
    float* Z[kLayers] = {};
    float* y = nullptr;
    float* dy = nullptr;
    uint16_t* dZb = nullptr;
    float* dH = nullptr;
    float* gpart = nullptr;     // per-workgroup partials of dW: (rows / 128) x 128 x 128
    float* colb = nullptr;      // per-block column sums (bias gradient)
    float* colo = nullptr;      // per-block column sums (output weights)
    double* losspart = nullptr;
    float* dypart = nullptr;    // per-block sums of dy
};


template <typename T>
bool dalloc(T** p, size_t n) {
    return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(n, 1) * sizeof(T)) == hipSuccess;
}

void ws_free(Workspace& w) {
    for (int l = 0; l <= kLayers; ++l) {
        (void)hipFree(w.H[l]);
        w.H[l] = nullptr;
    }
    for (int l = 0; l < kLayers; ++l) {
        (void)hipFree(w.Z[l]);
        w.Z[l] = nullptr;
    }
    (void)hipFree(w.y);
    (void)hipFree(w.dy);
    (void)hipFree(w.dZb);
    (void)hipFree(w.dH);
    (void)hipFree(w.gpart);
    (void)hipFree(w.colb);
    (void)hipFree(w.colo);
    (void)hipFree(w.losspart);
    (void)hipFree(w.dypart);
    w = Workspace();
}

bool ws_ensure(Workspace& w, int64_t rows, bool train) {
    if (w.cap >= rows && (w.train || !train)) return true;
    const int64_t cap = std::max(rows, w.cap);
    ws_free(w);
    w.cap = cap;
    w.train = train;
    bool ok = true;
    for (int l = 0; l <= kLayers; ++l) {
        ok = ok && dalloc(&w.H[l], size_t(cap) * kHidden);
    }
    for (int l = 0; l < kLayers; ++l) ok = ok && dalloc(&w.Z[l], size_t(cap) * kHidden);
    ok = ok && dalloc(&w.y, cap);
    if (train) {
        const int64_t nb = (cap + 127) / 128;   // workgroups of the backward layer kernel
        ok = ok && dalloc(&w.dy, cap) && dalloc(&w.dZb, size_t(cap) * kHidden) &&
             dalloc(&w.dH, size_t(cap) * kHidden) &&
             dalloc(&w.gpart, size_t((cap + 127) / 128) * kHidden * kHidden) && dalloc(&w.colb, size_t(nb) * kHidden) &&
             dalloc(&w.colo, size_t(nb) * kHidden) && dalloc(&w.losspart, size_t((cap + 255) / 256)) &&
             dalloc(&w.dypart, size_t((cap + 255) / 256));
    }
    if (!ok) ws_free(w);
    return ok;
}

std::vector<int8_t> monomials(int degree) {
    std::vector<int8_t> m;
    for (int k = 0; k <= degree; ++k)
        for (int a = k; a >= 0; --a)
            for (int b = k - a; b >= 0; --b) {
                m.push_back(int8_t(a));
                m.push_back(int8_t(b));
                m.push_back(int8_t(k - a - b));
            }
    return m;
}

int64_t round32(int64_t n) { return std::max<int64_t>(32, (n + 31) / 32 * 32); }

}  // namespace

struct env_surrogate {
    env_potential* fallback = nullptr;
    env_potential* near = nullptr;   // exactly evaluated part added to the network (may be null)
    uint64_t fallback_gen = 0;   // the fallback's density generation when the network was trained
    int device = -1;
    double radius = 6.0;
    int degree = 0;
    std::vector<int8_t> mono;
    std::vector<double> coef;
    double sigma = 1.0;
    // device
    double* d_B = nullptr;
    float* d_params = nullptr;
    float* d_grad = nullptr;
    float* d_m = nullptr;
    float* d_v = nullptr;
    uint16_t* d_W = nullptr;
    uint16_t* d_WT = nullptr;
    double* d_coef = nullptr;
    int8_t* d_mono = nullptr;
    uint8_t* d_pass = nullptr;
    int64_t* d_nfb = nullptr;              // gated-out count of the last evaluation
    unsigned long long* d_counter = nullptr;  // work counter of the fallback launch
    TrainState* d_tstate = nullptr;        // device step counter of training
    int G = 0;
    void* eval_stream = nullptr;           // stream of the last evaluation
    int64_t step = 0;
    Workspace ws;
    env_surrogate_info info{};
};

namespace {

env_status upload_baseline(env_surrogate* s) {
    (void)hipFree(s->d_coef);
    (void)hipFree(s->d_mono);
    s->d_coef = nullptr;
    s->d_mono = nullptr;
    if (!dalloc(&s->d_coef, s->coef.size()) || !dalloc(&s->d_mono, s->mono.size())) return ENV_E_NOMEM;
    if (hipMemcpy(s->d_coef, s->coef.data(), s->coef.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_mono, s->mono.data(), s->mono.size(), hipMemcpyHostToDevice) != hipSuccess)
        return ENV_E_DEVICE;
    return ENV_OK;
}

// Forward pass of rows [0, Np) whose first n are real points, storing what
// the backward pass reads (H and H^T of every layer, Z, y in ws.y); one launch.
void forward(env_surrogate* s, const double* pts, int64_t n, int64_t Np, void* st) {
    Workspace& w = s->ws;
    sg_forward_train(pts, n, Np, s->d_B, s->d_W, s->d_params, w.H, w.Z, w.y, st);
}

// Host copies of the intermediate tensors of one training step (see
// env_surrogate_trace_step); every copy is queued on the step's stream.
struct TraceCopies {
    env_surrogate_trace* tr = nullptr;
    int64_t n = 0;
    std::vector<uint16_t> dzb;   // staging of the BF16 dZ of every layer
    bool ok = true;
    void copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
        if (ok && dst && hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st) != hipSuccess) ok = false;
    }
};

// Loss partials and the full gradient into d_grad (forward must have run with train = true).
void backward(env_surrogate* s, const float* t, int64_t n, int64_t Np, void* st, TraceCopies* tc = nullptr) {
    Workspace& w = s->ws;
    hipStream_t hst = static_cast<hipStream_t>(st);
    sg_loss(w.y, t, n, Np, w.dy, w.losspart, w.dypart, st);
    if (tc) tc->copy(tc->tr->dy, w.dy, size_t(n) * sizeof(float), hst);
    for (int l = kLayers - 1; l >= 0; --l) {
        const bool top = l == kLayers - 1;
        if (tc && !top) tc->copy(tc->tr->dH ? tc->tr->dH + size_t(l) * n * kHidden : nullptr, w.dH,
                                 size_t(n) * kHidden * sizeof(float), hst);
        // dZ, the bias and output-weight column sums, dH of the layer below
        // (over w.dH) and the dW partials in one launch
        const int nb = sg_backward_layer(top, w.dH, w.dy, s->d_params + kOutOffset, w.Z[l], w.H[kLayers],
                                         s->d_WT + size_t(l) * kHidden * kHidden, w.H[l], Np, l > 0, w.dZb,
                                         w.gpart, w.colb, w.colo, st);
        if (tc && tc->tr->dZ)
            tc->copy(tc->dzb.data() + size_t(l) * n * kHidden, w.dZb, size_t(n) * kHidden * sizeof(uint16_t), hst);
        float* gl = s->d_grad + size_t(l) * kLayerStride;
        sg_reduce_rows(w.colb, nb, kHidden, gl + kHidden * kHidden, st);
        if (top) {
            sg_reduce_rows(w.colo, nb, kHidden, s->d_grad + kOutOffset, st);
            sg_reduce_rows(w.dypart, int((Np + 255) / 256), 1, s->d_grad + kOutOffset + kHidden, st);
        }
        sg_reduce_rows(w.gpart, nb, int64_t(kHidden) * kHidden, gl, st);
    }
}

// Surrogate values (baseline + network, plus add[i] when add is not null) at
// n points, in chunks.
env_status predict(env_surrogate* s, const double* pts, int64_t n, double* out, void* st,
                   const double* add = nullptr) {
    sg_infer(pts, n, s->d_B, s->d_W, s->d_params, s->d_coef, s->d_mono, int(s->mono.size() / 3), 1.0 / s->radius,
             s->sigma, add, out, st);
    return sg_last_error() == 0 ? ENV_OK : ENV_E_DEVICE;
}

// Least-squares fit of the polynomial baseline (normal equations, Cholesky, FP64).
bool fit_baseline(const std::vector<double>& P, const std::vector<double>& V, const std::vector<int8_t>& mono,
                  double R, std::vector<double>& coef, double& rms) {
    const size_t m = mono.size() / 3, n = V.size();
    std::vector<double> A(m * m, 0.0), b(m, 0.0), row(m);
    for (size_t i = 0; i < n; ++i) {
        const double u[3] = {P[3 * i] / R, P[3 * i + 1] / R, P[3 * i + 2] / R};
        for (size_t k = 0; k < m; ++k)
            row[k] = std::pow(u[0], mono[3 * k]) * std::pow(u[1], mono[3 * k + 1]) * std::pow(u[2], mono[3 * k + 2]);
        for (size_t a = 0; a < m; ++a) {
            b[a] += row[a] * V[i];
            for (size_t c = 0; c <= a; ++c) A[a * m + c] += row[a] * row[c];
        }
    }
    for (size_t a = 0; a < m; ++a) {  // Cholesky A = L L^T in place (lower)
        for (size_t c = 0; c <= a; ++c) {
            double sum = A[a * m + c];
            for (size_t k = 0; k < c; ++k) sum -= A[a * m + k] * A[c * m + k];
            if (a == c) {
                if (!(sum > 0.0)) return false;
                A[a * m + a] = std::sqrt(sum);
            } else {
                A[a * m + c] = sum / A[c * m + c];
            }
        }
    }
    coef.assign(m, 0.0);
    std::vector<double> z(m);
    for (size_t a = 0; a < m; ++a) {
        double sum = b[a];
        for (size_t k = 0; k < a; ++k) sum -= A[a * m + k] * z[k];
        z[a] = sum / A[a * m + a];
    }
    for (size_t a = m; a-- > 0;) {
        double sum = z[a];
        for (size_t k = a + 1; k < m; ++k) sum -= A[k * m + a] * coef[k];
        coef[a] = sum / A[a * m + a];
    }
    double ss = 0.0;
    for (size_t i = 0; i < n; ++i) {
        const double u[3] = {P[3 * i] / R, P[3 * i + 1] / R, P[3 * i + 2] / R};
        double v = 0.0;
        for (size_t k = 0; k < m; ++k)
            v += coef[k] * std::pow(u[0], mono[3 * k]) * std::pow(u[1], mono[3 * k + 1]) *
                 std::pow(u[2], mono[3 * k + 2]);
        ss += (V[i] - v) * (V[i] - v);
    }
    rms = std::sqrt(ss / std::max<size_t>(n, 1));
    return true;
}

void destroy(env_surrogate* s) {
    DeviceGuard g(s->device);
    ws_free(s->ws);
    (void)hipFree(s->d_B);
    (void)hipFree(s->d_params);
    (void)hipFree(s->d_grad);
    (void)hipFree(s->d_m);
    (void)hipFree(s->d_v);
    (void)hipFree(s->d_W);
    (void)hipFree(s->d_WT);
    (void)hipFree(s->d_coef);
    (void)hipFree(s->d_mono);
    (void)hipFree(s->d_pass);
    (void)hipFree(s->d_nfb);
    (void)hipFree(s->d_counter);
    (void)hipFree(s->d_tstate);
    delete s;
}

}  // namespace

extern "C" {

void env_train_opts_default(env_train_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->n_train = 2000000;
    o->epochs = 20;
    o->batch = 8192;
    o->lr = 2e-3;
    o->lr_final = 2e-5;
    o->seed = 12345;
    o->gate_grid = 24;
    o->gate_samples = 8;
    o->gate_tol = 5e-6;
    o->n_fit = 131072;
    o->poly_degree = 6;
}

env_status env_surrogate_create(env_potential* fallback, const env_surrogate_spec* spec, env_surrogate** out) {
    if (!out) return ENV_E_ARG;
    *out = nullptr;
    if (!fallback || !spec || !spec->B || !spec->params) return ENV_E_ARG;
    if (!fallback->on_device) return ENV_E_STATE;
    if (spec->n_freq != kFreq || spec->hidden != kHidden || spec->layers != kLayers) return ENV_E_UNSUPPORTED;
    if (!(spec->radius > 0.0) || spec->poly_degree < 0 || spec->poly_degree > kMaxPolyDegree) return ENV_E_ARG;
    if (spec->poly_degree > 0 && !spec->poly) return ENV_E_ARG;
    env_surrogate* s = new (std::nothrow) env_surrogate();
    if (!s) return ENV_E_NOMEM;
    s->fallback = fallback;
    s->device = fallback->device;
    s->radius = spec->radius;
    s->degree = spec->poly_degree;
    s->mono = monomials(s->degree);
    s->coef.assign(s->mono.size() / 3, 0.0);
    if (spec->poly) std::copy(spec->poly, spec->poly + s->coef.size(), s->coef.begin());
    s->sigma = spec->sigma > 0.0 ? spec->sigma : 1.0;
    DeviceGuard g(s->device);
    bool ok = dalloc(&s->d_B, 3 * kFreq) && dalloc(&s->d_params, kNParams) && dalloc(&s->d_grad, kNParams) &&
              dalloc(&s->d_m, kNParams) && dalloc(&s->d_v, kNParams) &&
              dalloc(&s->d_W, size_t(kLayers) * kHidden * kHidden) &&
              dalloc(&s->d_WT, size_t(kLayers) * kHidden * kHidden) && dalloc(&s->d_nfb, 1) &&
              dalloc(&s->d_counter, 1) && dalloc(&s->d_tstate, 1);
    if (!ok) {
        destroy(s);
        return ENV_E_NOMEM;
    }
    if (hipMemcpy(s->d_B, spec->B, 3 * kFreq * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->d_params, spec->params, kNParams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(s->d_m, 0, kNParams * sizeof(float)) != hipSuccess ||
        hipMemset(s->d_v, 0, kNParams * sizeof(float)) != hipSuccess ||
        hipMemset(s->d_nfb, 0, sizeof(int64_t)) != hipSuccess) {
        destroy(s);
        return ENV_E_DEVICE;
    }
    env_status st = upload_baseline(s);
    if (st != ENV_OK) {
        destroy(s);
        return st;
    }
    sg_pack(s->d_params, s->d_W, s->d_WT, nullptr);
    if (sg_last_error() != 0 || hipStreamSynchronize(nullptr) != hipSuccess) {
        destroy(s);
        return ENV_E_DEVICE;
    }
    s->info.n_params = kNParams;
    s->info.n_freq = kFreq;
    s->info.hidden = kHidden;
    s->info.layers = kLayers;
    s->info.poly_degree = s->degree;
    s->info.radius = s->radius;
    s->info.sigma = s->sigma;
    *out = s;
    return ENV_OK;
}

env_status env_surrogate_predict(env_surrogate* s, const double* points, int64_t n, double* out, void* stream) {
    if (!s || n < 0) return ENV_E_ARG;
    if (n == 0) return ENV_OK;
    if (!points || !out) return ENV_E_ARG;
    if (s->d_pass && s->fallback->density_gen != s->fallback_gen) return ENV_E_STATE;  // trained on an old density
    DeviceGuard g(s->device);
    return predict(s, points, n, out, stream);
}

env_status env_surrogate_loss_grad(env_surrogate* s, const double* points, const float* targets, int64_t n,
                                   float* grad_host, double* loss, void* stream) {
    if (!s || n <= 0 || !points || !targets) return ENV_E_ARG;
    DeviceGuard g(s->device);
    const int64_t Np = round32(n);
    if (!ws_ensure(s->ws, Np, true)) return ENV_E_NOMEM;
    hipStream_t st = static_cast<hipStream_t>(stream);
    forward(s, points, n, Np, stream);
    backward(s, targets, n, Np, stream);
    if (sg_last_error() != 0) return ENV_E_DEVICE;
    std::vector<double> lp((Np + 255) / 256);
    if (hipMemcpyAsync(lp.data(), s->ws.losspart, lp.size() * sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        (grad_host && hipMemcpyAsync(grad_host, s->d_grad, kNParams * sizeof(float), hipMemcpyDeviceToHost, st) !=
                          hipSuccess) ||
        hipStreamSynchronize(st) != hipSuccess)
        return ENV_E_DEVICE;
    double L = 0.0;
    for (double v : lp) L += v;
    if (loss) *loss = L / double(n);
    return ENV_OK;
}

env_status env_surrogate_trace_step(env_surrogate* s, const double* points, const float* targets, int64_t n,
                                    env_surrogate_trace* tr, void* stream) {
    if (!s || n <= 0 || !points || !targets || !tr) return ENV_E_ARG;
    DeviceGuard g(s->device);
    const int64_t Np = round32(n);
    if (!ws_ensure(s->ws, Np, true)) return ENV_E_NOMEM;
    hipStream_t st = static_cast<hipStream_t>(stream);
    Workspace& w = s->ws;
    TraceCopies tc;
    tc.tr = tr;
    tc.n = n;
    std::vector<uint16_t> hb(tr->H ? size_t(kLayers + 1) * n * kHidden : 0);
    if (tr->dZ) tc.dzb.assign(size_t(kLayers) * n * kHidden, 0);
    forward(s, points, n, Np, stream);
    for (int l = 0; l <= kLayers && tr->H; ++l)
        tc.copy(hb.data() + size_t(l) * n * kHidden, w.H[l], size_t(n) * kHidden * sizeof(uint16_t), st);
    for (int l = 0; l < kLayers && tr->Z; ++l)
        tc.copy(tr->Z + size_t(l) * n * kHidden, w.Z[l], size_t(n) * kHidden * sizeof(float), st);
    tc.copy(tr->y, w.y, size_t(n) * sizeof(float), st);
    backward(s, targets, n, Np, stream, &tc);
    tc.copy(tr->grad, s->d_grad, kNParams * sizeof(float), st);
    std::vector<double> lp((Np + 255) / 256);
    tc.copy(lp.data(), w.losspart, lp.size() * sizeof(double), st);
    if (sg_last_error() != 0 || !tc.ok || hipStreamSynchronize(st) != hipSuccess) return ENV_E_DEVICE;
    auto widen = [](uint16_t b) {
        const uint32_t u = uint32_t(b) << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return f;
    };
    for (size_t i = 0; i < hb.size(); ++i) tr->H[i] = widen(hb[i]);
    for (size_t i = 0; i < tc.dzb.size(); ++i) tr->dZ[i] = widen(tc.dzb[i]);
    if (tr->dH) {
        // dL/dH of the top layer is dy w_out^T, formed inside the SiLU backward
        std::vector<float> dy(n), wo(kHidden);
        if (hipMemcpy(dy.data(), w.dy, size_t(n) * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(wo.data(), s->d_params + kOutOffset, kHidden * sizeof(float), hipMemcpyDeviceToHost) !=
                hipSuccess)
            return ENV_E_DEVICE;
        float* top = tr->dH + size_t(kLayers - 1) * n * kHidden;
        for (int64_t r = 0; r < n; ++r)
            for (int c = 0; c < kHidden; ++c) top[r * kHidden + c] = dy[r] * wo[c];
    }
    double L = 0.0;
    for (double v : lp) L += v;
    tr->loss = L / double(n);
    return ENV_OK;
}

env_status env_surrogate_train(env_surrogate* s, env_potential* teacher, const env_train_opts* opts, void* stream) {
    if (!s || !teacher) return ENV_E_ARG;
    if (!teacher->on_device) return ENV_E_STATE;
    env_train_opts o;
    if (opts) o = *opts;
    else env_train_opts_default(&o);
    if (o.n_train < 1024 || o.batch < 32 || o.batch % 32 || o.epochs < 1 || !(o.lr > 0.0) ||
        o.gate_grid < 1 || o.gate_samples < 1 || o.poly_degree < 0 || o.poly_degree > kMaxPolyDegree ||
        o.n_fit < 1)
        return ENV_E_ARG;
    DeviceGuard g(s->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const auto t0 = std::chrono::steady_clock::now();
    const int64_t n = o.n_train;
    double* d_pts = nullptr;
    double* d_V = nullptr;
    float* d_t = nullptr;
    int32_t* d_perm = nullptr;
    double* d_pb = nullptr;
    float* d_tb = nullptr;
    env_status rc = ENV_OK;
    auto cleanup = [&]() {
        (void)hipStreamSynchronize(st);
        (void)hipFree(d_pts);
        (void)hipFree(d_V);
        (void)hipFree(d_t);
        (void)hipFree(d_perm);
        (void)hipFree(d_pb);
        (void)hipFree(d_tb);
    };
    if (!dalloc(&d_pts, 3 * size_t(n)) || !dalloc(&d_V, n) || !dalloc(&d_t, n) || !dalloc(&d_perm, n) ||
        !dalloc(&d_pb, 3 * size_t(o.batch)) || !dalloc(&d_tb, o.batch) || !ws_ensure(s->ws, o.batch, true)) {
        cleanup();
        return ENV_E_NOMEM;
    }
    // 1. training samples and their exact values
    sg_sample_ball(o.seed, n, s->radius, d_pts, stream);
    rc = env_potential_eval(teacher, d_pts, n, d_V, stream);
    if (rc != ENV_OK) {
        cleanup();
        return rc;
    }
    if (hipStreamSynchronize(st) != hipSuccess) {
        cleanup();
        return ENV_E_DEVICE;
    }
    const auto t1 = std::chrono::steady_clock::now();
    // 2. polynomial baseline on a subsample, residual targets
    const int64_t nf = std::min(n, o.n_fit);
    std::vector<double> hp(3 * size_t(nf)), hv(nf);
    if (hipMemcpy(hp.data(), d_pts, hp.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(hv.data(), d_V, hv.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) {
        cleanup();
        return ENV_E_DEVICE;
    }
    s->degree = o.poly_degree;
    s->mono = monomials(s->degree);
    double rms = 0.0;
    if (!fit_baseline(hp, hv, s->mono, s->radius, s->coef, rms)) {
        cleanup();
        return ENV_E_ARG;
    }
    s->sigma = rms > 0.0 ? rms : 1.0;
    rc = upload_baseline(s);
    if (rc != ENV_OK) {
        cleanup();
        return rc;
    }
    sg_residual(d_pts, d_V, n, s->d_coef, s->d_mono, int(s->mono.size() / 3), 1.0 / s->radius, 1.0 / s->sigma,
                d_t, stream);
    // 3. Adam on minibatches, cosine learning-rate decay.  One step (gather,
    // forward, backward, Adam, BF16 pack, step counter) is captured once as
    // a graph on a stream of the library's own and replayed for every step;
    // the step number, minibatch offset and learning rate live on the device.
    const int64_t steps_per_epoch = n / o.batch;
    const int64_t total = steps_per_epoch * o.epochs;
    std::mt19937_64 gen(o.seed ^ 0x5DEECE66Dull);
    double last_loss = 0.0;
    hipStream_t ts = nullptr;
    hipGraphExec_t step_exec = nullptr;
    // two pinned host permutations: the next epoch's is shuffled on the host
    // while the device runs the current one; the last minibatch's loss
    // partials of every epoch are kept on the device and read at the end
    const int64_t nlp = (o.batch + 255) / 256;
    int32_t* hperm[2] = {nullptr, nullptr};
    hipEvent_t copied[2] = {nullptr, nullptr};
    double* d_losshist = nullptr;
    auto release = [&]() {
        for (int b = 0; b < 2; ++b) {
            if (hperm[b]) (void)hipHostFree(hperm[b]);
            if (copied[b]) (void)hipEventDestroy(copied[b]);
        }
        (void)hipFree(d_losshist);
    };
    for (int b = 0; b < 2 && rc == ENV_OK; ++b)
        if (hipHostMalloc(reinterpret_cast<void**>(&hperm[b]), size_t(n) * sizeof(int32_t), hipHostMallocDefault) !=
                hipSuccess ||
            hipEventCreateWithFlags(&copied[b], hipEventDisableTiming) != hipSuccess)
            rc = ENV_E_NOMEM;
    if (rc == ENV_OK && !dalloc(&d_losshist, size_t(nlp) * o.epochs)) rc = ENV_E_NOMEM;
    auto shuffle_into = [&](int32_t* pv) {
        for (int64_t i = 0; i < n; ++i) pv[i] = int32_t(i);
        std::shuffle(pv, pv + n, gen);
    };
    if (rc == ENV_OK) shuffle_into(hperm[0]);
    const TrainState tstate0 = {s->step, s->step};
    if (hipStreamSynchronize(st) != hipSuccess || hipStreamCreateWithFlags(&ts, hipStreamNonBlocking) != hipSuccess ||
        hipMemcpy(s->d_tstate, &tstate0, sizeof(TrainState), hipMemcpyHostToDevice) != hipSuccess)
        rc = ENV_E_DEVICE;
    auto one_step = [&](void* sp) {
        sg_gather(d_pts, d_t, d_perm, s->d_tstate, steps_per_epoch, o.batch, d_pb, d_tb, sp);
        forward(s, d_pb, o.batch, o.batch, sp);
        backward(s, d_tb, o.batch, o.batch, sp);
        sg_adam(s->d_params, s->d_grad, s->d_m, s->d_v, kNParams, s->d_tstate, o.lr, o.lr_final, total, 0.9f, 0.999f,
                1e-8f, sp);
        sg_pack(s->d_params, s->d_W, s->d_WT, sp);
        sg_advance(s->d_tstate, sp);
    };
    const char* ng = std::getenv("ENVPOT_NO_GRAPH");   // plain launches (profilers, debugging)
    const bool use_graph = !(ng && *ng && *ng != '0');
    if (rc == ENV_OK && use_graph) {
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(ts, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = ENV_E_DEVICE;
        } else {
            one_step(ts);
            const hipError_t e = hipStreamEndCapture(ts, &graph);
            if (e != hipSuccess || !graph || sg_last_error() != 0 ||
                hipGraphInstantiate(&step_exec, graph, nullptr, nullptr, 0) != hipSuccess)
                rc = ENV_E_DEVICE;
            if (graph) (void)hipGraphDestroy(graph);
        }
    }
    for (int ep = 0; ep < o.epochs && rc == ENV_OK; ++ep) {
        const int b = ep & 1;
        // the epoch's permutation goes to the device after the previous
        // epoch's steps (stream order), from pinned memory
        if (hipMemcpyAsync(d_perm, hperm[b], size_t(n) * sizeof(int32_t), hipMemcpyHostToDevice, ts) !=
                hipSuccess ||
            hipEventRecord(copied[b], ts) != hipSuccess) {
            rc = ENV_E_DEVICE;
            break;
        }
        for (int64_t k = 0; k < steps_per_epoch && rc == ENV_OK; ++k) {
            if (!use_graph) one_step(ts);
            else if (hipGraphLaunch(step_exec, ts) != hipSuccess) rc = ENV_E_DEVICE;
        }
        s->step += steps_per_epoch;
        if (rc == ENV_OK && hipMemcpyAsync(d_losshist + size_t(ep) * nlp, s->ws.losspart, size_t(nlp) * sizeof(double),
                                           hipMemcpyDeviceToDevice, ts) != hipSuccess)
            rc = ENV_E_DEVICE;
        // next epoch's permutation, on the host while the device works; its
        // buffer's last copy (two epochs ago) must have finished
        if (rc == ENV_OK && ep + 1 < o.epochs) {
            if (hipEventSynchronize(copied[b ^ 1]) != hipSuccess) rc = ENV_E_DEVICE;
            else shuffle_into(hperm[b ^ 1]);
        }
    }
    if (rc == ENV_OK) {
        std::vector<double> lh(size_t(nlp) * o.epochs);
        if (hipMemcpyAsync(lh.data(), d_losshist, lh.size() * sizeof(double), hipMemcpyDeviceToHost, ts) !=
                hipSuccess ||
            hipStreamSynchronize(ts) != hipSuccess) {
            rc = ENV_E_DEVICE;
        } else {
            for (int ep = 0; ep < o.epochs; ++ep) {
                double l = 0.0;
                for (int64_t q = 0; q < nlp; ++q) l += lh[size_t(ep) * nlp + q];
                last_loss = l / double(o.batch);
                if (ep < int(sizeof(s->info.epoch_loss) / sizeof(double))) s->info.epoch_loss[ep] = last_loss;
            }
        }
    }
    if (ts) (void)hipStreamSynchronize(ts);
    if (step_exec) (void)hipGraphExecDestroy(step_exec);
    if (ts) (void)hipStreamDestroy(ts);
    release();
    const auto t2 = std::chrono::steady_clock::now();
    // 4. gate: m validation points per voxel of a G^3 grid over the ball
    if (rc == ENV_OK) {
        const int G = o.gate_grid, m = o.gate_samples;
        const int64_t nv = int64_t(G) * G * G, nvp = nv * m;
        double *d_vp = nullptr, *d_ve = nullptr, *d_vs = nullptr, *d_err = nullptr;
        if (!dalloc(&d_vp, 3 * size_t(nvp)) || !dalloc(&d_ve, nvp) || !dalloc(&d_vs, nvp) || !dalloc(&d_err, nv)) {
            rc = ENV_E_NOMEM;
        } else {
            sg_sample_voxels(o.seed ^ 0xA5A5A5A5ull, G, m, s->radius, d_vp, stream);
            rc = env_potential_eval(teacher, d_vp, nvp, d_ve, stream);
            if (rc == ENV_OK) rc = predict(s, d_vp, nvp, d_vs, stream);
            if (rc == ENV_OK) sg_voxel_maxerr(d_ve, d_vs, nv, m, d_err, stream);
            std::vector<double> err(nv);
            if (rc == ENV_OK &&
                (hipMemcpyAsync(err.data(), d_err, nv * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
                 hipStreamSynchronize(st) != hipSuccess))
                rc = ENV_E_DEVICE;
            if (rc == ENV_OK) {
                std::vector<uint8_t> pass(nv, 0);
                const double h = 2.0 * s->radius / G, R = s->radius;
                int64_t in_ball = 0, passed = 0;
                double vol_in = 0.0, vol_pass = 0.0, maxpass = 0.0;
                for (int64_t v = 0; v < nv; ++v) {
                    const int vx = int(v % G), vy = int((v / G) % G), vz = int(v / (int64_t(G) * G));
                    // nearest point of the voxel to the centre: does it touch the ball?
                    auto nearest = [&](int i) {
                        const double lo = -R + h * i, hi = lo + h;
                        return lo > 0 ? lo : (hi < 0 ? hi : 0.0);
                    };
                    const double dx = nearest(vx), dy = nearest(vy), dz = nearest(vz);
                    if (dx * dx + dy * dy + dz * dz > R * R) continue;
                    ++in_ball;
                    // volume weight: fraction of the voxel's corners inside the ball
                    int inside = 0;
                    for (int c = 0; c < 8; ++c) {
                        const double cx = -R + h * (vx + (c & 1)), cy = -R + h * (vy + ((c >> 1) & 1)),
                                     cz = -R + h * (vz + ((c >> 2) & 1));
                        inside += (cx * cx + cy * cy + cz * cz <= R * R);
                    }
                    const double wv = (inside + 1) / 9.0;
                    vol_in += wv;
                    if (err[v] <= o.gate_tol) {
                        pass[v] = 1;
                        ++passed;
                        vol_pass += wv;
                        maxpass = std::max(maxpass, err[v]);
                    }
                }
                (void)hipFree(s->d_pass);
                s->d_pass = nullptr;
                if (!dalloc(&s->d_pass, nv) ||
                    hipMemcpy(s->d_pass, pass.data(), nv, hipMemcpyHostToDevice) != hipSuccess) {
                    rc = ENV_E_DEVICE;
                } else {
                    s->G = G;
                    s->info.gate_grid = G;
                    s->info.gate_voxels_in_ball = in_ball;
                    s->info.gate_voxels_pass = passed;
                    s->info.gate_pass_volume_fraction = vol_in > 0 ? vol_pass / vol_in : 0.0;
                    s->info.gate_max_err_passed = maxpass;
                    s->info.gate_tol = o.gate_tol;
                }
            }
        }
        (void)hipStreamSynchronize(st);
        (void)hipFree(d_vp);
        (void)hipFree(d_ve);
        (void)hipFree(d_vs);
        (void)hipFree(d_err);
    }
    const auto t3 = std::chrono::steady_clock::now();
    cleanup();
    if (rc != ENV_OK) return rc;
    s->fallback_gen = s->fallback->density_gen;
    s->info.sigma = s->sigma;
    s->info.poly_degree = s->degree;
    s->info.baseline_rms = rms;
    s->info.train_steps = s->step;
    s->info.final_loss = last_loss;
    s->info.teacher_seconds = std::chrono::duration<double>(t1 - t0).count();
    s->info.train_seconds = std::chrono::duration<double>(t2 - t1).count();
    s->info.gate_seconds = std::chrono::duration<double>(t3 - t2).count();
    return ENV_OK;
}

env_status env_surrogate_set_near(env_surrogate* s, env_potential* near) {
    if (!s) return ENV_E_ARG;
    if (near && (!near->on_device || near->device != s->device)) return ENV_E_STATE;
    s->near = near;
    return ENV_OK;
}

env_status env_surrogate_eval(env_surrogate* s, const double* points, int64_t n, double* out,
                              uint8_t* used_fallback, void* stream) {
    if (!s || n < 0) return ENV_E_ARG;
    if (n == 0) return ENV_OK;
    if (!points || !out) return ENV_E_ARG;
    if (!s->d_pass) return ENV_E_STATE;  // no gate before training
    if (s->fallback->density_gen != s->fallback_gen) return ENV_E_STATE;  // trained on an old density
    if (s->near && (!s->near->on_device || s->near->device != s->device)) return ENV_E_STATE;
    DeviceGuard g(s->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nb = int((n + 255) / 256);
    // the gated-out count stays on the device: the compacted list is sized
    // for all n points and the fallback launch reads the count itself
    const int64_t part_cap = std::max<int64_t>(n, int64_t(1) << 23);
    uint8_t* flag = nullptr;
    int32_t* counts = nullptr;
    int64_t *offs = nullptr, *idx = nullptr;
    double *cpts = nullptr, *vals = nullptr, *part = nullptr, *add = nullptr;
    auto amalloc = [&](auto** p, size_t bytes) {
        return hipMallocAsync(reinterpret_cast<void**>(p), std::max<size_t>(bytes, 8), st) == hipSuccess;
    };
    bool ok = amalloc(&flag, size_t(n)) && amalloc(&counts, size_t(nb) * 4) && amalloc(&offs, size_t(nb) * 8) &&
              amalloc(&idx, size_t(n) * 8) && amalloc(&cpts, size_t(n) * 24) && amalloc(&vals, size_t(n) * 8) &&
              amalloc(&part, size_t(part_cap) * 8) && (!s->near || amalloc(&add, size_t(n) * 8));
    env_status rc = ok ? ENV_OK : ENV_E_NOMEM;
    if (rc == ENV_OK) {
        sg_gate_flags(points, n, s->d_pass, s->G, s->radius, flag, counts, stream);
        sg_scan_counts(counts, nb, offs, s->d_nfb, stream);
        if (s->near) rc = env_potential_eval(s->near, points, n, add, stream);
    }
    if (rc == ENV_OK) rc = predict(s, points, n, out, stream, add);
    if (rc == ENV_OK) {
        sg_compact(points, n, flag, offs, idx, cpts, stream);
        rc = eval_devsized(s->fallback, cpts, s->d_nfb, n, vals, part, part_cap, s->d_counter, stream);
    }
    if (rc == ENV_OK) sg_scatter(vals, idx, s->d_nfb, n, out, stream);
    if (rc == ENV_OK && used_fallback &&
        hipMemcpyAsync(used_fallback, flag, size_t(n), hipMemcpyDeviceToDevice, st) != hipSuccess)
        rc = ENV_E_DEVICE;
    if (rc == ENV_OK && sg_last_error() != 0) rc = ENV_E_DEVICE;
    for (void* p : {static_cast<void*>(flag), static_cast<void*>(counts), static_cast<void*>(offs),
                    static_cast<void*>(idx), static_cast<void*>(cpts), static_cast<void*>(vals),
                    static_cast<void*>(part), static_cast<void*>(add)})
        if (p) (void)hipFreeAsync(p, st);
    s->info.last_eval_n = n;
    s->eval_stream = stream;
    return rc;
}

env_status env_surrogate_get_params(const env_surrogate* s, float* params, double* poly, double* sigma) {
    if (!s) return ENV_E_ARG;
    DeviceGuard g(s->device);
    if (params && hipMemcpy(params, s->d_params, kNParams * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return ENV_E_DEVICE;
    if (poly) std::copy(s->coef.begin(), s->coef.end(), poly);
    if (sigma) *sigma = s->sigma;
    return ENV_OK;
}

env_status env_surrogate_get_info(const env_surrogate* s, env_surrogate_info* info) {
    if (!s || !info) return ENV_E_ARG;
    *info = s->info;
    if (s->info.last_eval_n > 0) {
        // the last evaluation's gated-out count, read once that call is done
        DeviceGuard g(s->device);
        int64_t m = 0;
        hipStream_t st = static_cast<hipStream_t>(s->eval_stream);
        if (hipStreamSynchronize(st) != hipSuccess ||
            hipMemcpy(&m, s->d_nfb, sizeof(m), hipMemcpyDeviceToHost) != hipSuccess)
            return ENV_E_DEVICE;
        info->last_eval_fallback = m;
    }
    return ENV_OK;
}

void env_surrogate_destroy(env_surrogate* s) {
    if (s) destroy(s);
}

}  // extern "C"
