// Internal interface of the surrogate kernels (surrogate.hip) for the host
// driver (surrogate.cpp).  Not part of the C ABI.
#pragma once

#include <cstdint>

namespace envpot {

constexpr int kHidden = 128;                 // width of every hidden layer
constexpr int kLayers = 4;                   // hidden layers
constexpr int kFreq = 64;                    // Fourier frequencies: 2 x 64 = 128 inputs
constexpr int kLayerStride = kHidden * kHidden + kHidden;   // W (out x in) then b
constexpr int kOutOffset = kLayers * kLayerStride;          // w_out (128) then b_out
constexpr int kNParams = kOutOffset + kHidden + 1;          // 66,177
constexpr int kMaxPolyDegree = 8;

void sg_reduce_rows(const float* part, int P, int64_t L, float* out, void* st);
void sg_loss(const float* y, const float* t, int64_t n, int64_t Np, float* dy, double* part, float* part_dy,
             void* st);
// Device state of a training run: Adam step count so far and its value at
// the start of the run (the minibatch index and the learning-rate schedule
// are derived from them on the device, so one captured step graph is
// replayed for every step).
struct TrainState {
    int64_t step;
    int64_t step0;
};

void sg_adam(float* p, const float* g, float* m, float* v, int64_t n, const TrainState* ts, double lr0,
             double lr1, int64_t total, float b1, float b2, float eps, void* st);
void sg_advance(TrainState* ts, void* st);
void sg_pack(const float* params, uint16_t* W, uint16_t* WT, void* st);
// The whole network at inference (features, four layers, output, baseline,
// optional exact part) in one launch: out[i] = poly + sigma y (+ add[i]).
void sg_infer(const double* pts, int64_t n, const double* B, const uint16_t* W, const float* params,
              const double* coef, const int8_t* mono, int nmono, double inv_r, double sigma, const double* add,
              double* out, void* st);
// The forward pass of a training step in one launch: H_0..H_4 (row-major
// [Np x 128], BF16), Z_0..Z_3 (FP32) and y for the first Np rows (rows >= n
// have zero features).
void sg_forward_train(const double* pts, int64_t n, int64_t Np, const double* B, const uint16_t* W,
                      const float* params, uint16_t* const* H, float* const* Z, float* y, void* st);
// One layer of the backward pass in one launch: BF16 dZ (to dZb), the
// per-workgroup column sums of dZ (and, top layer, of dy H_top), dH of the
// layer below written over dH (when `below`), and per-workgroup 128 x 128
// partials of dW; returns the number of workgroups (partials).  Np is a
// multiple of 32.
int sg_backward_layer(bool top, float* dH, const float* dy, const float* w_out, const float* Z, const uint16_t* Htop,
                      const uint16_t* WT, const uint16_t* H, int64_t Np, bool below, uint16_t* dZb, float* gpart,
                      float* colsum, float* colsum_out, void* st);
void sg_residual(const double* pts, const double* V, int64_t n, const double* coef, const int8_t* mono,
                 int nmono, double inv_r, double inv_sigma, float* t, void* st);
void sg_sample_ball(uint64_t seed, int64_t n, double R, double* pts, void* st);
void sg_sample_voxels(uint64_t seed, int G, int m, double R, double* pts, void* st);
void sg_gather(const double* pts, const float* t, const int32_t* perm, const TrainState* ts,
               int64_t steps_per_epoch, int64_t bs, double* pb, float* tb, void* st);
int sg_gate_flags(const double* pts, int64_t n, const uint8_t* pass, int G, double R, uint8_t* flag,
                  int32_t* counts, void* st);
void sg_scan_counts(const int32_t* counts, int nb, int64_t* offsets, int64_t* total, void* st);
void sg_compact(const double* pts, int64_t n, const uint8_t* flag, const int64_t* offsets, int64_t* idx,
                double* cpts, void* st);
void sg_scatter(const double* vals, const int64_t* idx, const int64_t* m, int64_t n_max, double* out, void* st);
void sg_voxel_maxerr(const double* a, const double* b, int64_t nv, int m, double* err, void* st);
int sg_last_error();

}  // namespace envpot
