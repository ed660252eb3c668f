// gfx950 kernels of the coordinate-MLP surrogate of V(r) inside the QM region.
//
// Network: gamma(r) = [cos 2 pi B r, sin 2 pi B r] (BF16) -> 4 x (Linear 128 x 128
// in BF16 on the matrix cores with FP32 accumulation, bias, SiLU, BF16) ->
// Linear 128 -> 1 in FP32; V_hat = poly(r/R) + sigma * y.  Training: MSE,
// straight-through BF16 rounding, Adam on FP32 master weights.
//
// The forward pass (features, the four layers, the output) is one kernel,
// k_mlp, that keeps a workgroup's 128 rows in LDS; each layer of the backward
// pass is one kernel, k_mlp_bwd, likewise (dZ, dH of the layer below, the
// workgroup's dW partial, summed over workgroups in fixed order by
// k_reduce_rows).  Every product is C[M x N] = A[M x K] * Bt[N x K]^T with
// BF16 operands (K contiguous) staged in LDS, on v_mfma_f32_32x32x16_bf16.  Operand layout of the instruction (verified
// on the device): lane l, g = l / 32, r = l % 32 holds A[r][g*8 .. g*8+7] and
// Bt[r][g*8 .. g*8+7]; result register i holds C[(i/4)*8 + g*4 + i%4][r].
#include <hip/hip_runtime.h>

#include "surrogate_internal.h"

namespace envpot {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

constexpr double kTwoPi = 6.283185307179586476925286766559;

__device__ __forceinline__ uint16_t to_bf16(float x) {  // round to nearest even
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }

__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// out[j] = sum_{p < P} part[p * L + j] in FP64: four groups of consecutive
// partials summed in order by four waves, then the group sums added in group
// order (a fixed order, so the result is reproducible).  Block: 64 outputs.
__global__ __launch_bounds__(256) void k_reduce_rows(const float* __restrict__ part, int P, int64_t L,
                                                     float* __restrict__ out) {
    __shared__ double sh[4][64];
    const int jl = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + jl;
    const int chunk = (P + 3) / 4;
    double s = 0.0;
    if (j < L)
        for (int p = g * chunk; p < min(P, (g + 1) * chunk); ++p) s += part[(int64_t)p * L + j];
    sh[g][jl] = s;
    __syncthreads();
    if (g == 0 && j < L) out[j] = (float)(((sh[0][jl] + sh[1][jl]) + sh[2][jl]) + sh[3][jl]);
}

__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ t,
                                              int64_t n, int64_t Np, float* __restrict__ dy,
                                              double* __restrict__ part, float* __restrict__ part_dy) {
    __shared__ double sh[256];
    __shared__ float shd[256];
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double e2 = 0.0;
    float d = 0.0f;
    if (row < Np) {
        if (row < n) {
            const float e = y[row] - t[row];
            d = 2.0f * e / (float)n;
            e2 = (double)e * (double)e;
        }
        dy[row] = d;
    }
    sh[threadIdx.x] = e2;
    shd[threadIdx.x] = d;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sh[threadIdx.x] += sh[threadIdx.x + s];
            shd[threadIdx.x] += shd[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sh[0];
        part_dy[blockIdx.x] = shd[0];
    }
}

// Adam on the FP32 master weights.  The step number comes from the device
// training state (so one captured step graph serves every step): step =
// st->step + 1, learning rate by cosine decay from lr0 to lr1 over `total`
// steps, bias corrections 1 - b^step.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int64_t n,
                                              const TrainState* __restrict__ st, double lr0, double lr1,
                                              int64_t total, float b1, float b2, float eps) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t step = st->step + 1;
    const double frac = fmin(1.0, (double)(step - st->step0) / (double)(total > 0 ? total : 1));
    const float lr = (float)(lr1 + 0.5 * (lr0 - lr1) * (1.0 + cos(3.14159265358979323846 * frac)));
    const float bc1 = (float)(1.0 - pow((double)b1, (double)step));
    const float bc2 = (float)(1.0 - pow((double)b2, (double)step));
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// End of a training step: advance the device step counter.
__global__ void k_advance(TrainState* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) st->step += 1;
}

// BF16 copies of the four hidden weight matrices, as stored (out x in) and transposed.
__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ params, uint16_t* __restrict__ W,
                                              uint16_t* __restrict__ WT) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (int64_t)kLayers * kHidden * kHidden) return;
    const int l = (int)(idx / (kHidden * kHidden));
    const int e = (int)(idx % (kHidden * kHidden));
    const int o = e / kHidden, i = e % kHidden;
    const uint16_t b = to_bf16(params[(int64_t)l * kLayerStride + e]);
    W[idx] = b;
    WT[(int64_t)l * kHidden * kHidden + i * kHidden + o] = b;
}

// Phase 2 pi b_k . r of one Fourier feature (FP64).
__device__ __forceinline__ double feature_phase(const double* __restrict__ B, int k, double x, double y, double z) {
    return kTwoPi * (B[3 * k] * x + B[3 * k + 1] * y + B[3 * k + 2] * z);
}

// poly(r/R) + sigma * y (FP64) at one point.
__device__ __forceinline__ double finish_value(double x, double y, double z, float net,
                                               const double* __restrict__ coef, const int8_t* __restrict__ mono,
                                               int nmono, double inv_r, double sigma) {
    double px[kMaxPolyDegree + 1], py[kMaxPolyDegree + 1], pz[kMaxPolyDegree + 1];
    const double ux = x * inv_r, uy = y * inv_r, uz = z * inv_r;
    px[0] = py[0] = pz[0] = 1.0;
    for (int d = 1; d <= kMaxPolyDegree; ++d) {
        px[d] = px[d - 1] * ux;
        py[d] = py[d - 1] * uy;
        pz[d] = pz[d - 1] * uz;
    }
    double v = 0.0;
    for (int k = 0; k < nmono; ++k) v += coef[k] * px[mono[3 * k]] * py[mono[3 * k + 1]] * pz[mono[3 * k + 2]];
    return v + sigma * (double)net;
}

// The whole network in one kernel.  A workgroup takes 128 rows (four waves
// of 32), computes their Fourier features into LDS, then per layer stages
// the layer's BF16 weights in LDS and lets each wave multiply its own 32
// rows by them on the matrix cores (four 32 x 32 output tiles, K = 128 in
// steps of 16), adds the bias, applies SiLU and writes the BF16 activations
// back over its rows; then the FP32 output layer.  Inference (TRAIN false)
// finishes with the baseline and the optional exact part; training (TRAIN
// true) also stores what the backward pass reads: H_0..H_4 (row-major), the
// pre-activations Z_l and y, for the first Np rows.  LDS rows
// are padded to 136 elements (bank spread of the 16-byte row reads).
constexpr int kInferRows = 128;
constexpr int kLdsLd = kHidden + 8;

struct TrainStores {
    uint16_t* H[kLayers + 1];
    float* Z[kLayers];
    float* y;
    int64_t Np;     // rows stored (multiple of 32; rows >= n are padding with zero features)
};

template <bool TRAIN>
__global__ __launch_bounds__(256) void k_mlp(const double* __restrict__ pts, int64_t n,
                                             const double* __restrict__ B, const uint16_t* __restrict__ W,
                                             const float* __restrict__ params, const double* __restrict__ coef,
                                             const int8_t* __restrict__ mono, int nmono, double inv_r,
                                             double sigma, const double* __restrict__ add,
                                             double* __restrict__ out, TrainStores ts) {
    __shared__ __attribute__((aligned(16))) uint16_t sW[kHidden * kLdsLd];
    __shared__ __attribute__((aligned(16))) uint16_t sH[kInferRows * kLdsLd];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 5, r = lane & 31;
    const int64_t row0 = (int64_t)blockIdx.x * kInferRows;
    const int64_t nstore = TRAIN ? ts.Np : n;
    {   // features: thread t -> row t % 128, frequencies 32 (t / 128) .. + 31
        const int lr = tid & (kInferRows - 1);
        const int k0 = (tid >> 7) * (kFreq / 2);
        const int64_t row = row0 + lr;
        double x = 0.0, y = 0.0, z = 0.0;
        if (row < n) {
            x = pts[3 * row];
            y = pts[3 * row + 1];
            z = pts[3 * row + 2];
        }
        for (int k = k0; k < k0 + kFreq / 2; ++k) {
            uint16_t c = 0, sn = 0;
            if (row < n) {
                double sv, cv;
                sincos(feature_phase(B, k, x, y, z), &sv, &cv);
                c = to_bf16((float)cv);
                sn = to_bf16((float)sv);
            }
            sH[lr * kLdsLd + k] = c;
            sH[lr * kLdsLd + kFreq + k] = sn;
            if (TRAIN && row < nstore) {
                ts.H[0][row * kHidden + k] = c;
                ts.H[0][row * kHidden + kFreq + k] = sn;
            }
        }
    }
    for (int l = 0; l < kLayers; ++l) {
        {   // stage W_l (out x in) with padded rows: 128 rows x 16 chunks of 8 values
            const uint4* gW = reinterpret_cast<const uint4*>(W + (int64_t)l * kHidden * kHidden);
            for (int q = tid; q < kHidden * kHidden / 8; q += 256) {
                const int o = q >> 4, c = q & 15;
                *reinterpret_cast<uint4*>(sW + o * kLdsLd + c * 8) = gW[q];
            }
        }
        __syncthreads();  // W_l staged; the previous layer's activations written
        f32x16 acc[4] = {};
        const uint16_t* a = sH + (wave * 32 + r) * kLdsLd + g * 8;
        for (int k = 0; k < kHidden; k += 16) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(a + k);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8*>(sW + (t * 32 + r) * kLdsLd + g * 8 + k);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[t], 0, 0, 0);
            }
        }
        // this wave's rows are read; its new activations go over them (the
        // other waves read only their own rows)
        const float* bias = params + (int64_t)l * kLayerStride + kHidden * kHidden;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int col = t * 32 + r;
            const float bc = bias[col];
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int lr = wave * 32 + (i >> 2) * 8 + g * 4 + (i & 3);
                const float zv = acc[t][i] + bc;
                const uint16_t h = to_bf16(silu(zv));
                sH[lr * kLdsLd + col] = h;
                if (TRAIN) {
                    const int64_t row = row0 + lr;
                    if (row < nstore) {
                        ts.Z[l][row * kHidden + col] = zv;
                        ts.H[l + 1][row * kHidden + col] = h;
                    }
                }
            }
        }
        __syncthreads();  // every wave is done with W_l before it is replaced
    }
    if (tid < kInferRows) {
        const int64_t row = row0 + tid;
        if (row < nstore) {
            const float* w = params + kOutOffset;
            float s = 0.0f;
            const uint16_t* h = sH + tid * kLdsLd;
            for (int j = 0; j < kHidden; ++j) s = __builtin_fmaf(__uint_as_float((uint32_t)h[j] << 16), w[j], s);
            const float yv = s + w[kHidden];
            if (TRAIN) {
                ts.y[row] = yv;
            } else {
                const double v = finish_value(pts[3 * row], pts[3 * row + 1], pts[3 * row + 2], yv, coef, mono,
                                              nmono, inv_r, sigma);
                out[row] = add ? v + add[row] : v;
            }
        }
    }
}

// One layer of the backward pass in one kernel.  A workgroup takes 128 rows
// (four waves of 32):
//  1. dZ = dH * silu'(Z) (dH = dy w_out for the top layer) in FP32; BF16 dZ
//     into LDS (row-major and transposed) and to dZb; the workgroup's column
//     sums of the FP32 dZ (bias gradient) and, for the top layer, of
//     dy * H_top (output weights);
//  2. for a layer with one below it, dH of that layer = dZ W_l on the matrix
//     cores with W_l^T staged in LDS (the tiling of the forward layers),
//     written over dH: every row of dH is read and rewritten by the one
//     workgroup that owns it;
//  3. the workgroup's share of dW_l = dZ^T H_l (its rows only), with H_l^T
//     transposed into LDS from the row-major H_l: a 128 x 128 FP32 partial
//     per workgroup, summed over the workgroups in fixed order by
//     k_reduce_rows.
// Rows >= Np contribute zeros.  LDS: three padded 128 x 128 BF16 tiles.
template <bool TOP>
__global__ __launch_bounds__(256) void k_mlp_bwd(float* __restrict__ dH, const float* __restrict__ dy,
                                                 const float* __restrict__ w_out, const float* __restrict__ Z,
                                                 const uint16_t* __restrict__ Htop,
                                                 const uint16_t* __restrict__ WT, const uint16_t* __restrict__ H,
                                                 int64_t Np, bool below, uint16_t* __restrict__ dZb,
                                                 float* __restrict__ gpart, float* __restrict__ colsum,
                                                 float* __restrict__ colsum_out) {
    __shared__ __attribute__((aligned(16))) uint16_t sA[kInferRows * kLdsLd];  // dZ [row][o]
    __shared__ __attribute__((aligned(16))) uint16_t sB[kHidden * kLdsLd];     // dZ^T [o][row]
    __shared__ __attribute__((aligned(16))) uint16_t sC[kHidden * kLdsLd];     // W^T [i][o], then H^T [i][row]
    __shared__ float csh[2][kHidden], cosh_[2][kHidden];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g = lane >> 5, r = lane & 31;
    const int64_t row0 = (int64_t)blockIdx.x * kInferRows;
    {   // 1. thread -> column t % 128, rows 64 (t / 128) .. + 63
        const int col = tid & (kHidden - 1), half = tid >> 7;
        float cs = 0.0f, co = 0.0f;
        for (int rl = half * 64; rl < half * 64 + 64; ++rl) {
            const int64_t row = row0 + rl;
            uint16_t b = 0;
            if (row < Np) {
                const int64_t idx = row * kHidden + col;
                float gv;
                if (TOP) {
                    gv = dy[row] * w_out[col];
                    co = __builtin_fmaf(dy[row], __uint_as_float((uint32_t)Htop[idx] << 16), co);
                } else {
                    gv = dH[idx];
                }
                const float dz = gv * dsilu(Z[idx]);
                cs += dz;
                b = to_bf16(dz);
                dZb[idx] = b;
            }
            sA[rl * kLdsLd + col] = b;
            sB[col * kLdsLd + rl] = b;
        }
        csh[half][col] = cs;
        if (TOP) cosh_[half][col] = co;
    }
    __syncthreads();
    if (tid < kHidden) {
        colsum[(int64_t)blockIdx.x * kHidden + tid] = csh[0][tid] + csh[1][tid];
        if (TOP) colsum_out[(int64_t)blockIdx.x * kHidden + tid] = cosh_[0][tid] + cosh_[1][tid];
    }
    if (below) {   // 2. dH of the layer below = dZ W (Bt = W^T rows)
        const uint4* gW = reinterpret_cast<const uint4*>(WT);
        for (int q = tid; q < kHidden * kHidden / 8; q += 256) {
            const int i = q >> 4, c = q & 15;
            *reinterpret_cast<uint4*>(sC + i * kLdsLd + c * 8) = gW[q];
        }
        __syncthreads();
        f32x16 acc[4] = {};
        const uint16_t* a = sA + (wave * 32 + r) * kLdsLd + g * 8;
        for (int k = 0; k < kHidden; k += 16) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(a + k);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8*>(sC + (t * 32 + r) * kLdsLd + g * 8 + k);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int64_t row = row0 + wave * 32 + (i >> 2) * 8 + g * 4 + (i & 3);
                if (row < Np) dH[row * kHidden + t * 32 + r] = acc[t][i];
            }
        __syncthreads();   // sC is overwritten next
    }
    {   // 3. stage H^T [i][row] from the row-major H rows row0 .. row0 + 127
        //    (16-byte global reads, transposed into LDS; zero past Np)
        for (int q = tid; q < kHidden * kInferRows / 8; q += 256) {
            const int rl = q >> 4, c = q & 15;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (row0 + rl < Np) v = *reinterpret_cast<const uint4*>(H + (row0 + rl) * kHidden + c * 8);
            const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                sC[(c * 8 + 2 * j) * kLdsLd + rl] = (uint16_t)(w4[j] & 0xFFFFu);
                sC[(c * 8 + 2 * j + 1) * kLdsLd + rl] = (uint16_t)(w4[j] >> 16);
            }
        }
        __syncthreads();
        // wave w: output rows o = 32 w .. + 31, all 128 columns i
        f32x16 acc[4] = {};
        const uint16_t* a = sB + (wave * 32 + r) * kLdsLd + g * 8;
        for (int k = 0; k < kInferRows; k += 16) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(a + k);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bf16x8 bv = *reinterpret_cast<const bf16x8*>(sC + (t * 32 + r) * kLdsLd + g * 8 + k);
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[t], 0, 0, 0);
            }
        }
        float* gp = gpart + (int64_t)blockIdx.x * kHidden * kHidden;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                gp[(wave * 32 + (i >> 2) * 8 + g * 4 + (i & 3)) * kHidden + t * 32 + r] = acc[t][i];
    }
}

// Residual targets t = (V - poly(r/R)) / sigma.
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ pts, const double* __restrict__ V,
                                                  int64_t n, const double* __restrict__ coef,
                                                  const int8_t* __restrict__ mono, int nmono, double inv_r,
                                                  double inv_sigma, float* __restrict__ t) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double px[kMaxPolyDegree + 1], py[kMaxPolyDegree + 1], pz[kMaxPolyDegree + 1];
    const double ux = pts[3 * i] * inv_r, uy = pts[3 * i + 1] * inv_r, uz = pts[3 * i + 2] * inv_r;
    px[0] = py[0] = pz[0] = 1.0;
    for (int d = 1; d <= kMaxPolyDegree; ++d) {
        px[d] = px[d - 1] * ux;
        py[d] = py[d - 1] * uy;
        pz[d] = pz[d - 1] * uz;
    }
    double v = 0.0;
    for (int k = 0; k < nmono; ++k) v += coef[k] * px[mono[3 * k]] * py[mono[3 * k + 1]] * pz[mono[3 * k + 2]];
    t[i] = (float)((V[i] - v) * inv_sigma);
}

// SplitMix64 (Steele, Lea, Flood 2014): the counter-based generator of the
// training and gate sample points.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__device__ __forceinline__ double unif(uint64_t seed, uint64_t ctr) {
    return (double)(splitmix64(seed ^ splitmix64(ctr)) >> 11) * 0x1.0p-53;
}

// n points uniform in the ball of radius R, point i from counters 3i..3i+2.
__global__ __launch_bounds__(256) void k_sample_ball(uint64_t seed, int64_t n, double R, double* __restrict__ pts) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double u0 = unif(seed, 3 * (uint64_t)i), u1 = unif(seed, 3 * (uint64_t)i + 1),
                 u2 = unif(seed, 3 * (uint64_t)i + 2);
    const double r = R * cbrt(u0), ct = 2.0 * u1 - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
    const double ph = kTwoPi * u2;
    pts[3 * i] = r * st * cos(ph);
    pts[3 * i + 1] = r * st * sin(ph);
    pts[3 * i + 2] = r * ct;
}

// Gate validation points: per voxel v (of the G^3 grid over [-R, R]^3) m
// points uniform in the voxel, pulled radially into the ball when outside it.
__global__ __launch_bounds__(256) void k_sample_voxels(uint64_t seed, int G, int m, double R,
                                                       double* __restrict__ pts) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nv = (int64_t)G * G * G;
    if (i >= nv * m) return;
    const int64_t v = i / m;
    const int vx = (int)(v % G), vy = (int)((v / G) % G), vz = (int)(v / ((int64_t)G * G));
    const double h = 2.0 * R / G;
    double x = -R + h * (vx + unif(seed, 3 * (uint64_t)i));
    double y = -R + h * (vy + unif(seed, 3 * (uint64_t)i + 1));
    double z = -R + h * (vz + unif(seed, 3 * (uint64_t)i + 2));
    const double rr = sqrt(x * x + y * y + z * z);
    if (rr > R) {
        const double s = R * (1.0 - 1e-12) / rr;
        x *= s;
        y *= s;
        z *= s;
    }
    pts[3 * i] = x;
    pts[3 * i + 1] = y;
    pts[3 * i + 2] = z;
}

// Minibatch of a training step: rows ((step - step0) mod steps_per_epoch)
// * bs .. + bs of the epoch's permutation.
__global__ __launch_bounds__(256) void k_gather(const double* __restrict__ pts, const float* __restrict__ t,
                                                const int32_t* __restrict__ perm, const TrainState* __restrict__ st,
                                                int64_t steps_per_epoch, int64_t bs, double* __restrict__ pb,
                                                float* __restrict__ tb) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= bs) return;
    const int64_t start = ((st->step - st->step0) % steps_per_epoch) * bs;
    const int64_t j = perm[start + i];
    pb[3 * i] = pts[3 * j];
    pb[3 * i + 1] = pts[3 * j + 1];
    pb[3 * i + 2] = pts[3 * j + 2];
    tb[i] = t[j];
}

// Gate: flag[i] = 1 when point i must use the exact kernel (outside the
// ball or in a voxel that failed validation); per-block counts of flags.
__global__ __launch_bounds__(256) void k_gate_flags(const double* __restrict__ pts, int64_t n,
                                                    const uint8_t* __restrict__ pass, int G, double R,
                                                    uint8_t* __restrict__ flag, int32_t* __restrict__ counts) {
    __shared__ int32_t sh[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int f = 0;
    if (i < n) {
        const double x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
        f = 1;
        if (x * x + y * y + z * z <= R * R) {
            const double h = 2.0 * R / G;
            const int vx = min(G - 1, max(0, (int)floor((x + R) / h)));
            const int vy = min(G - 1, max(0, (int)floor((y + R) / h)));
            const int vz = min(G - 1, max(0, (int)floor((z + R) / h)));
            f = pass[((int64_t)vz * G + vy) * G + vx] ? 0 : 1;
        }
        flag[i] = (uint8_t)f;
    }
    sh[threadIdx.x] = f;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = sh[0];
}

// Exclusive scan of the block counts (one workgroup, sequential chunks).
__global__ __launch_bounds__(256) void k_scan_counts(const int32_t* __restrict__ counts, int nb,
                                                     int64_t* __restrict__ offsets, int64_t* __restrict__ total) {
    __shared__ int64_t sh[256];
    int64_t carry = 0;
    for (int base = 0; base < nb; base += 256) {
        const int i = base + threadIdx.x;
        const int64_t v = i < nb ? counts[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int s = 1; s < 256; s <<= 1) {  // inclusive Hillis-Steele scan
            const int64_t a = threadIdx.x >= s ? sh[threadIdx.x - s] : 0;
            __syncthreads();
            sh[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < nb) offsets[i] = carry + sh[threadIdx.x] - v;
        const int64_t last = sh[255];
        __syncthreads();
        carry += last;
    }
    if (threadIdx.x == 0) *total = carry;
}

// Stable compaction of the flagged points (order of the input kept).
__global__ __launch_bounds__(256) void k_compact(const double* __restrict__ pts, int64_t n,
                                                 const uint8_t* __restrict__ flag,
                                                 const int64_t* __restrict__ offsets,
                                                 int64_t* __restrict__ idx, double* __restrict__ cpts) {
    __shared__ int32_t sh[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int f = (i < n) ? flag[i] : 0;
    sh[threadIdx.x] = f;
    __syncthreads();
    for (int s = 1; s < 256; s <<= 1) {
        const int32_t a = threadIdx.x >= s ? sh[threadIdx.x - s] : 0;
        __syncthreads();
        sh[threadIdx.x] += a;
        __syncthreads();
    }
    if (f) {
        const int64_t o = offsets[blockIdx.x] + sh[threadIdx.x] - 1;
        idx[o] = i;
        cpts[3 * o] = pts[3 * i];
        cpts[3 * o + 1] = pts[3 * i + 1];
        cpts[3 * o + 2] = pts[3 * i + 2];
    }
}

// out[idx[k]] = vals[k] for k < *m (the count is read on the device; the
// grid covers the largest possible count).
__global__ __launch_bounds__(256) void k_scatter(const double* __restrict__ vals, const int64_t* __restrict__ idx,
                                                 const int64_t* __restrict__ m, double* __restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < *m) out[idx[k]] = vals[k];
}

// max |a - b| per voxel (m consecutive samples per voxel), FP64.
__global__ __launch_bounds__(256) void k_voxel_maxerr(const double* __restrict__ a, const double* __restrict__ b,
                                                      int64_t nv, int m, double* __restrict__ err) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= nv) return;
    double e = 0.0;
    for (int k = 0; k < m; ++k) e = fmax(e, fabs(a[v * m + k] - b[v * m + k]));
    err[v] = e;
}

inline unsigned blocks(int64_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }

}  // namespace

#define SG_LAUNCH(k, g, b, st, ...) hipLaunchKernelGGL(k, g, b, 0, static_cast<hipStream_t>(st), __VA_ARGS__)

void sg_reduce_rows(const float* part, int P, int64_t L, float* out, void* st) {
    SG_LAUNCH(k_reduce_rows, dim3(blocks(L, 64)), dim3(256), st, part, P, L, out);
}

void sg_loss(const float* y, const float* t, int64_t n, int64_t Np, float* dy, double* part, float* part_dy,
             void* st) {
    SG_LAUNCH(k_loss, dim3(blocks(Np)), dim3(256), st, y, t, n, Np, dy, part, part_dy);
}

void sg_adam(float* p, const float* g, float* m, float* v, int64_t n, const TrainState* ts, double lr0,
             double lr1, int64_t total, float b1, float b2, float eps, void* st) {
    SG_LAUNCH(k_adam, dim3(blocks(n)), dim3(256), st, p, g, m, v, n, ts, lr0, lr1, total, b1, b2, eps);
}

void sg_advance(TrainState* ts, void* st) { SG_LAUNCH(k_advance, dim3(1), dim3(64), st, ts); }

void sg_pack(const float* params, uint16_t* W, uint16_t* WT, void* st) {
    SG_LAUNCH(k_pack, dim3(blocks((int64_t)kLayers * kHidden * kHidden)), dim3(256), st, params, W, WT);
}

void sg_infer(const double* pts, int64_t n, const double* B, const uint16_t* W, const float* params,
              const double* coef, const int8_t* mono, int nmono, double inv_r, double sigma, const double* add,
              double* out, void* st) {
    if (n <= 0) return;
    TrainStores none = {};
    SG_LAUNCH(k_mlp<false>, dim3(blocks(n, kInferRows)), dim3(256), st, pts, n, B, W, params, coef, mono, nmono,
              inv_r, sigma, add, out, none);
}

void sg_forward_train(const double* pts, int64_t n, int64_t Np, const double* B, const uint16_t* W,
                      const float* params, uint16_t* const* H, float* const* Z, float* y, void* st) {
    if (Np <= 0) return;
    TrainStores ts;
    for (int l = 0; l <= kLayers; ++l) ts.H[l] = H[l];
    for (int l = 0; l < kLayers; ++l) ts.Z[l] = Z[l];
    ts.y = y;
    ts.Np = Np;
    SG_LAUNCH(k_mlp<true>, dim3(blocks(Np, kInferRows)), dim3(256), st, pts, n, B, W, params, nullptr, nullptr, 0,
              0.0, 0.0, nullptr, nullptr, ts);
}

int sg_backward_layer(bool top, float* dH, const float* dy, const float* w_out, const float* Z, const uint16_t* Htop,
                      const uint16_t* WT, const uint16_t* H, int64_t Np, bool below, uint16_t* dZb, float* gpart,
                      float* colsum, float* colsum_out, void* st) {
    const unsigned nb = blocks(Np, kInferRows);
    if (top)
        SG_LAUNCH(k_mlp_bwd<true>, dim3(nb), dim3(256), st, dH, dy, w_out, Z, Htop, WT, H, Np, below, dZb, gpart,
                  colsum, colsum_out);
    else
        SG_LAUNCH(k_mlp_bwd<false>, dim3(nb), dim3(256), st, dH, dy, w_out, Z, Htop, WT, H, Np, below, dZb, gpart,
                  colsum, colsum_out);
    return int(nb);
}

void sg_residual(const double* pts, const double* V, int64_t n, const double* coef, const int8_t* mono,
                 int nmono, double inv_r, double inv_sigma, float* t, void* st) {
    SG_LAUNCH(k_residual, dim3(blocks(n)), dim3(256), st, pts, V, n, coef, mono, nmono, inv_r, inv_sigma, t);
}

void sg_sample_ball(uint64_t seed, int64_t n, double R, double* pts, void* st) {
    SG_LAUNCH(k_sample_ball, dim3(blocks(n)), dim3(256), st, seed, n, R, pts);
}

void sg_sample_voxels(uint64_t seed, int G, int m, double R, double* pts, void* st) {
    SG_LAUNCH(k_sample_voxels, dim3(blocks((int64_t)G * G * G * m)), dim3(256), st, seed, G, m, R, pts);
}

void sg_gather(const double* pts, const float* t, const int32_t* perm, const TrainState* ts,
               int64_t steps_per_epoch, int64_t bs, double* pb, float* tb, void* st) {
    SG_LAUNCH(k_gather, dim3(blocks(bs)), dim3(256), st, pts, t, perm, ts, steps_per_epoch, bs, pb, tb);
}

int sg_gate_flags(const double* pts, int64_t n, const uint8_t* pass, int G, double R, uint8_t* flag,
                  int32_t* counts, void* st) {
    SG_LAUNCH(k_gate_flags, dim3(blocks(n)), dim3(256), st, pts, n, pass, G, R, flag, counts);
    return (int)blocks(n);
}

void sg_scan_counts(const int32_t* counts, int nb, int64_t* offsets, int64_t* total, void* st) {
    SG_LAUNCH(k_scan_counts, dim3(1), dim3(256), st, counts, nb, offsets, total);
}

void sg_compact(const double* pts, int64_t n, const uint8_t* flag, const int64_t* offsets, int64_t* idx,
                double* cpts, void* st) {
    SG_LAUNCH(k_compact, dim3(blocks(n)), dim3(256), st, pts, n, flag, offsets, idx, cpts);
}

void sg_scatter(const double* vals, const int64_t* idx, const int64_t* m, int64_t n_max, double* out, void* st) {
    if (n_max <= 0) return;
    SG_LAUNCH(k_scatter, dim3(blocks(n_max)), dim3(256), st, vals, idx, m, out);
}

void sg_voxel_maxerr(const double* a, const double* b, int64_t nv, int m, double* err, void* st) {
    SG_LAUNCH(k_voxel_maxerr, dim3(blocks(nv)), dim3(256), st, a, b, nv, m, err);
}

int sg_last_error() { return hipGetLastError() == hipSuccess ? 0 : -1; }

}  // namespace envpot
