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
constexpr int kRowsPerBlock = 64;            // rows per workgroup of k_dsilu
constexpr int kMaxPolyDegree = 8;

int sg_gemm_nt(const uint16_t* A, int lda, const uint16_t* Bt, int ldb, float* C, int ldc, int M, int N,
               int K, int ksplit, void* st);
void sg_reduce_rows(const float* part, int P, int64_t L, float* out, void* st);
void sg_features(const double* pts, int64_t n, int64_t Np, const double* B, int F, uint16_t* H,
                 uint16_t* HT, int64_t ldT, void* st);
void sg_bias_silu(float* Z, const float* bias, uint16_t* H, uint16_t* HT, int64_t Np, int64_t ldT, void* st);
void sg_out_fwd(const uint16_t* H, const float* w, const float* b, int64_t Np, float* y, void* st);
void sg_loss(const float* y, const float* t, int64_t n, int64_t Np, float* dy, double* part, float* part_dy,
             void* st);
void sg_dsilu(const float* dH, const float* dy, const float* w_out, const float* Z, const uint16_t* Htop,
              int64_t Np, uint16_t* dZb, uint16_t* dZT, int64_t ldT, float* colsum, float* colsum_out,
              void* st);
void sg_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
             float bc1, float bc2, void* st);
void sg_pack(const float* params, uint16_t* W, uint16_t* WT, void* st);
void sg_finish(const double* pts, const float* y, int64_t n, const double* coef, const int8_t* mono, int nmono,
               double inv_r, double sigma, const double* add, double* out, void* st);
void sg_residual(const double* pts, const double* V, int64_t n, const double* coef, const int8_t* mono,
                 int nmono, double inv_r, double inv_sigma, float* t, void* st);
void sg_sample_ball(uint64_t seed, int64_t n, double R, double* pts, void* st);
void sg_sample_voxels(uint64_t seed, int G, int m, double R, double* pts, void* st);
void sg_gather(const double* pts, const float* t, const int32_t* perm, int64_t start, int64_t bs, double* pb,
               float* tb, void* st);
int sg_gate_flags(const double* pts, int64_t n, const uint8_t* pass, int G, double R, uint8_t* flag,
                  int32_t* counts, void* st);
void sg_scan_counts(const int32_t* counts, int nb, int64_t* offsets, int64_t* total, void* st);
void sg_compact(const double* pts, int64_t n, const uint8_t* flag, const int64_t* offsets, int64_t* idx,
                double* cpts, void* st);
void sg_scatter(const double* vals, const int64_t* idx, const int64_t* m, int64_t n_max, double* out, void* st);
void sg_voxel_maxerr(const double* a, const double* b, int64_t nv, int m, double* err, void* st);
int sg_last_error();

}  // namespace envpot
