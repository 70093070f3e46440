// Learned warm start: per-window count-histogram features, a 3-layer MLP
// trained on the GPU with hand-written BF16 MFMA GEMMs (FP32 accumulation,
// FP32 master weights, Adam), and the warm-start epilogue that turns the
// network's prediction into initial (mu, alpha, beta) and keeps the cold
// start wherever it has the higher likelihood.
//
// The paper fits every window from scratch; this component is a systems
// addition around its solver (the solver's likelihood decides whether a
// prediction is used).

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mdhp_device.h"

namespace mdhp {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }  // round to nearest even
__device__ __forceinline__ float from_bf16(__bf16 x) { return (float)x; }

// ---------------------------------------------------------------------------
// Features: x[w][m * bins + b] = log1p(count_{m,b} * bins / T_w), where the
// bin of an event is floor(t * bins / T) (clamped to bins - 1), in FP64.
// ---------------------------------------------------------------------------
__global__ void features_kernel(const int64_t* __restrict__ offsets, const double* __restrict__ t,
                                const int32_t* __restrict__ dim, const double* __restrict__ T,
                                int64_t W, int M, int bins, __bf16* __restrict__ x) {
  extern __shared__ int hist[];
  const int F = M * bins;
  for (int64_t w = blockIdx.x; w < W; w += gridDim.x) {
    for (int i = threadIdx.x; i < F; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int64_t b0 = offsets[w], b1 = offsets[w + 1];
    const double Tw = T[w];
    for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
      int b = (int)floor(t[i] * (double)bins / Tw);
      b = b < 0 ? 0 : (b >= bins ? bins - 1 : b);
      atomicAdd(&hist[dim[i] * bins + b], 1);
    }
    __syncthreads();
    const float scale = (float)((double)bins / Tw);
    for (int i = threadIdx.x; i < F; i += blockDim.x)
      x[w * F + i] = to_bf16(log1pf((float)hist[i] * scale));
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// BF16 GEMM on MFMA: C[i][j] = sum_k A(i, k) B(k, j), with A(i, k) at
// A[i * sai + k * sak] and B(k, j) at B[k * sbk + j * sbj] (so every
// transpose of row-major operands is a choice of strides).  FP32 accumulate;
// epilogue: + bias[j], ReLU, store FP32 (ldc) and/or BF16 (ldc).
// Tiles: 64 x 64 per workgroup of 4 waves (2 x 2), 32 x 32 per wave as 2 x 2
// v_mfma_f32_16x16x32_bf16 blocks, K staged in LDS 32 at a time.
// MFMA operand layout (lane l): A fragment = row l % 16, k = 8 (l / 16) .. +7;
// B fragment = column l % 16, same k; result r = row 4 (l / 16) + r,
// column l % 16.
// ---------------------------------------------------------------------------
constexpr int GB_M = 64, GB_N = 64, GB_K = 32, GB_KP = GB_K + 8;

struct GemmArgs {
  const __bf16* A;
  const __bf16* B;
  int64_t sai, sak, sbk, sbj;
  int Mr, Nc, K;
  const float* bias;  // [Nc] or null
  int relu;
  float* Cf;          // [Mr][ldc] or null
  __bf16* Cb;         // [Mr][ldc] or null
  int ldc;
};

__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[GB_M][GB_KP];  // [row][k]
  __shared__ __attribute__((aligned(16))) __bf16 Bs[GB_N][GB_KP];  // [col][k] (B transposed)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = blockIdx.y * GB_M, j0 = blockIdx.x * GB_N;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  // Staging of the 64 x 32 tiles: thread t owns row t / 4, k = 8 (t % 4) .. + 7
  // of each.  Where k is contiguous in memory and the 8 elements are in range
  // and 16-byte aligned they are one 16-byte load, else 8 element loads.
  const int sr = tid >> 2, sk = 8 * (tid & 3);
  auto stage = [&](const __bf16* P, int64_t sm, int64_t skk, int m, int mlim, int k0,
                   __bf16 (*T)[GB_KP]) {
    const __bf16* p = P + (int64_t)m * sm + (int64_t)(k0 + sk) * skk;
    const bool full = m < mlim && k0 + sk + 8 <= g.K;
    if (full && skk == 1 && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
      *reinterpret_cast<bf16x8*>(&T[sr][sk]) = *reinterpret_cast<const bf16x8*>(p);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        T[sr][sk + e] = (m < mlim && k0 + sk + e < g.K) ? p[e * skk] : to_bf16(0.f);
    }
  };
  for (int k0 = 0; k0 < g.K; k0 += GB_K) {
    // Stage A (64 x 32) and B^T (64 x 32): 2048 elements each, 8 per thread.
    stage(g.A, g.sai, g.sak, i0 + sr, g.Mr, k0, As);
    stage(g.B, g.sbj, g.sbk, j0 + sr, g.Nc, k0, Bs);
    __syncthreads();
    const int kf = 8 * (lane >> 4);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const bf16x8 af = *reinterpret_cast<const bf16x8*>(&As[wm + a * 16 + (lane & 15)][kf]);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const bf16x8 bfr = *reinterpret_cast<const bf16x8*>(&Bs[wn + b * 16 + (lane & 15)][kf]);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bfr, acc[a][b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wm + a * 16 + 4 * (lane >> 4) + r;
        const int gj = j0 + wn + b * 16 + (lane & 15);
        if (gi < g.Mr && gj < g.Nc) {
          float v = acc[a][b][r];
          if (g.bias) v += g.bias[gj];
          if (g.relu) v = fmaxf(v, 0.f);
          if (g.Cf) g.Cf[(int64_t)gi * g.ldc + gj] = v;
          if (g.Cb) g.Cb[(int64_t)gi * g.ldc + gj] = to_bf16(v);
        }
      }
}

// dZ = dH * (H > 0), BF16 in/out.
__global__ void relu_grad_kernel(const __bf16* __restrict__ dH, const __bf16* __restrict__ H,
                                 __bf16* __restrict__ dZ, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dZ[i] = from_bf16(H[i]) > 0.f ? dH[i] : to_bf16(0.f);
}

// db[j] = sum_i dZ[i][j]: one workgroup per 64 columns, wavefront w summing
// rows w, w + 4, ... (each row's 64 columns one 128-byte read), the four
// partial sums added in order.
constexpr int kColsumCols = 64;
__global__ __launch_bounds__(256) void colsum_kernel(const __bf16* __restrict__ dZ, int rows,
                                                     int cols, float* __restrict__ db) {
  __shared__ float part[4][kColsumCols];
  const int c = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * kColsumCols + c;
  float s = 0.f;
  if (j < cols) {
#pragma unroll 8
    for (int i = w; i < rows; i += 4) s += from_bf16(dZ[(int64_t)i * cols + j]);
  }
  part[w][c] = s;
  __syncthreads();
  if (w == 0 && j < cols) db[j] = ((part[0][c] + part[1][c]) + part[2][c]) + part[3][c];
}

// Mean squared error over B x O and its gradient 2 (y - t) / (B O) (BF16);
// the loss is reduced per block in FP64 and added atomically.
__global__ void mse_kernel(const float* __restrict__ y, const float* __restrict__ tgt, int64_t n,
                           __bf16* __restrict__ dy, double* loss) {
  __shared__ double red[256];
  double s = 0.0;
  const float scale = 2.f / (float)n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = y[i] - tgt[i];
    dy[i] = to_bf16(scale * d);
    s += (double)d * (double)d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] / (double)n);
}

__global__ void zero_double_kernel(double* p) { *p = 0.0; }

// Adam on FP32 master weights; BF16 shadow for the next forward pass.
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m1, float* __restrict__ m2,
                            __bf16* __restrict__ shadow, int64_t n, float lr, float b1, float b2,
                            float eps, float bc1, float bc2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    const float nw = w[i] - lr * (a / bc1) / (sqrtf(v / bc2) + eps);
    w[i] = nw;
    if (shadow) shadow[i] = to_bf16(nw);
  }
}

__global__ void to_bf16_kernel(const float* __restrict__ src, __bf16* __restrict__ dst, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = to_bf16(src[i]);
}

// Prediction -> parameters: y = pred * std + mean holds, per window,
// log(mu_m T / max(N_m, 0.5)), the branching entries alpha_mn / beta and
// log beta; mu and beta are clamped to the projection's floors.
__global__ void warm_params_kernel(const float* __restrict__ pred, const float* __restrict__ mean,
                                   const float* __restrict__ stdv,
                                   const int32_t* __restrict__ counts, const int32_t* __restrict__ n,
                                   const double* __restrict__ T, int64_t W, int M,
                                   float mu_floor_rel, float beta_floor_rel, float* __restrict__ mu,
                                   float* __restrict__ alpha, float* __restrict__ beta) {
  const int O = M + M * M + 1;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < W * O;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = i / O;
    const int o = (int)(i % O);
    const float rate = (float)((double)max(n[w], 1) / T[w]);
    const float yb = pred[w * O + O - 1] * stdv[O - 1] + mean[O - 1];
    const float b = fmaxf(expf(fminf(yb, 30.f)), beta_floor_rel * rate);
    const float y = pred[i] * stdv[o] + mean[o];
    if (o < M) {
      const float rm = (float)(fmax((double)counts[w * M + o], 0.5) / T[w]);
      mu[w * M + o] = fmaxf(expf(fminf(y, 30.f)) * rm, mu_floor_rel * rate);
    } else if (o < M + M * M) {
      alpha[w * M * M + (o - M)] = fmaxf(y, 0.f) * b;
    } else {
      beta[w] = b;
    }
  }
}

// Per window, keep the warm start unless the cold start has the higher (or
// a finite where the warm one is not) likelihood.
__global__ void choose_init_kernel(const double* __restrict__ ll_warm,
                                   const double* __restrict__ ll_cold, int64_t W, int M,
                                   const float* __restrict__ mu_c, const float* __restrict__ al_c,
                                   const float* __restrict__ be_c, float* __restrict__ mu,
                                   float* __restrict__ alpha, float* __restrict__ beta,
                                   int32_t* __restrict__ used_warm) {
  const int64_t w = blockIdx.x;
  if (w >= W) return;
  const double lw = ll_warm[w], lc = ll_cold[w];
  const bool warm = isfinite(lw) && !(lc > lw);
  if (threadIdx.x == 0) used_warm[w] = warm ? 1 : 0;
  if (warm) return;
  for (int e = threadIdx.x; e < M * M; e += blockDim.x) alpha[w * M * M + e] = al_c[w * M * M + e];
  for (int e = threadIdx.x; e < M; e += blockDim.x) mu[w * M + e] = mu_c[w * M + e];
  if (threadIdx.x == 0) beta[w] = be_c[w];
}

int grid_for(int64_t n, int block = 256) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + block - 1) / block, 8192));
}

hipError_t gemm(const __bf16* A, int64_t sai, int64_t sak, const __bf16* B, int64_t sbk,
                int64_t sbj, int Mr, int Nc, int K, const float* bias, int relu, float* Cf,
                __bf16* Cb, int ldc, hipStream_t s) {
  GemmArgs g{A, B, sai, sak, sbk, sbj, Mr, Nc, K, bias, relu, Cf, Cb, ldc};
  dim3 grid((Nc + GB_N - 1) / GB_N, (Mr + GB_M - 1) / GB_M);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace
}  // namespace mdhp

using namespace mdhp;

// Layer l maps din[l] -> dout[l]; weights W_l[dout][din] then b_l[dout],
// packed in order in one FP32 buffer.
struct mdhp_surrogate {
  int in_dim = 0, hidden = 0, out_dim = 0, max_batch = 0;
  int64_t n_params = 0;
  int64_t woff[3] = {0, 0, 0}, boff[3] = {0, 0, 0};
  int din[3] = {0, 0, 0}, dout[3] = {0, 0, 0};
  float* w = nullptr;   // master weights
  float* g = nullptr;   // gradients
  float* m1 = nullptr;
  float* m2 = nullptr;
  __bf16* wb = nullptr;  // BF16 shadow of the whole buffer (biases unused)
  __bf16* h1 = nullptr;  // [B][hidden]
  __bf16* h2 = nullptr;
  float* y = nullptr;    // [B][out]
  __bf16* dy = nullptr;  // [B][out]
  __bf16* dh = nullptr;  // [B][hidden]
  __bf16* dz = nullptr;  // [B][hidden]
  int64_t step = 0;
  uint32_t magic = 0;
};

namespace {
constexpr uint32_t kSurrogateMagic = 0x5355524fu;
// Checkpoint header (see mdhp_surrogate_save); 48 bytes, no padding.
constexpr char kCheckpointMagic[8] = {'M', 'D', 'H', 'P', 'S', 'U', 'R', '1'};
struct CheckpointHeader {
  char magic[8];
  int32_t version, in_dim, hidden, out_dim;
  int64_t n_params, step, n_extra;
};
static_assert(sizeof(CheckpointHeader) == 48, "checkpoint header layout");
bool sur_ok(const mdhp_surrogate* s) { return s && s->magic == kSurrogateMagic; }
void free_sur(mdhp_surrogate* s) {
  for (void* p : {(void*)s->w, (void*)s->g, (void*)s->m1, (void*)s->m2, (void*)s->wb,
                  (void*)s->h1, (void*)s->h2, (void*)s->y, (void*)s->dy, (void*)s->dh,
                  (void*)s->dz})
    (void)hipFree(p);
  s->magic = 0;
  delete s;
}
}  // namespace

extern "C" {

mdhp_status mdhp_features(const mdhp_batch* b, int32_t M, int32_t bins, uint16_t* x,
                          void* stream) {
  if (!b || !x || M < 1 || M > MDHP_MAX_M || bins < 1 || M * bins > 16384 || b->W < 0)
    return mdhp_fail(MDHP_E_INVAL, "features: invalid argument");
  if (b->W == 0) return MDHP_OK;
  if (!b->offsets || !b->T || (b->n_events > 0 && (!b->t || !b->dim)))
    return mdhp_fail(MDHP_E_INVAL, "features: null array");
  hipStream_t s = (hipStream_t)stream;
  const int grid = (int)std::min<int64_t>(b->W, 65536);
  hipLaunchKernelGGL(features_kernel, dim3(grid), dim3(256), M * bins * sizeof(int), s,
                     b->offsets, b->t, b->dim, b->T, b->W, M, bins, (__bf16*)x);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MDHP_OK : mdhp_hip_fail(e, "features");
}

mdhp_status mdhp_surrogate_create(int32_t in_dim, int32_t hidden, int32_t out_dim,
                                  int32_t max_batch, uint64_t seed, mdhp_surrogate** out) {
  if (!out) return mdhp_fail(MDHP_E_INVAL, "surrogate_create: out is NULL");
  *out = nullptr;
  if (in_dim < 1 || hidden < 1 || out_dim < 1 || max_batch < 1)
    return mdhp_fail(MDHP_E_INVAL, "surrogate_create: sizes must be positive");
  mdhp_surrogate* s = new mdhp_surrogate();
  s->in_dim = in_dim;
  s->hidden = hidden;
  s->out_dim = out_dim;
  s->max_batch = max_batch;
  const int din[3] = {in_dim, hidden, hidden}, dout[3] = {hidden, hidden, out_dim};
  int64_t off = 0;
  for (int l = 0; l < 3; ++l) {
    s->din[l] = din[l];
    s->dout[l] = dout[l];
    s->woff[l] = off;
    off += (int64_t)din[l] * dout[l];
    s->boff[l] = off;
    off += dout[l];
  }
  s->n_params = off;
  s->magic = kSurrogateMagic;
  const int64_t B = max_batch;
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  alloc((void**)&s->w, off * 4);
  alloc((void**)&s->g, off * 4);
  alloc((void**)&s->m1, off * 4);
  alloc((void**)&s->m2, off * 4);
  alloc((void**)&s->wb, off * 2);
  alloc((void**)&s->h1, B * hidden * 2);
  alloc((void**)&s->h2, B * hidden * 2);
  alloc((void**)&s->y, B * out_dim * 4);
  alloc((void**)&s->dy, B * out_dim * 2);
  alloc((void**)&s->dh, B * hidden * 2);
  alloc((void**)&s->dz, B * hidden * 2);
  if (e != hipSuccess) {
    free_sur(s);
    return mdhp_hip_fail(e, "surrogate_create: allocation");
  }
  // He-uniform weights (bound sqrt(6 / fan_in)), zero biases; SplitMix64.
  std::vector<float> h(off, 0.f);
  uint64_t st = seed;
  for (int l = 0; l < 3; ++l) {
    const float bound = std::sqrt(6.f / (float)din[l]);
    for (int64_t i = 0; i < (int64_t)din[l] * dout[l]; ++i) {
      const double u = (double)(splitmix(st) >> 11) * (1.0 / 9007199254740992.0);
      h[s->woff[l] + i] = (float)((2.0 * u - 1.0) * bound);
    }
  }
  std::vector<float> zeros(off, 0.f);
  e = hipMemcpy(s->w, h.data(), off * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->m1, zeros.data(), off * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->m2, zeros.data(), off * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(off)), dim3(256), 0, 0, s->w, s->wb, off);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    free_sur(s);
    return mdhp_hip_fail(e, "surrogate_create: init");
  }
  *out = s;
  return MDHP_OK;
}

void mdhp_surrogate_destroy(mdhp_surrogate* s) {
  if (!sur_ok(s)) return;
  (void)hipDeviceSynchronize();
  free_sur(s);
}

int64_t mdhp_surrogate_num_params(const mdhp_surrogate* s) { return sur_ok(s) ? s->n_params : 0; }

mdhp_status mdhp_surrogate_get_weights(mdhp_surrogate* s, float* dst, void* stream) {
  if (!sur_ok(s) || !dst) return mdhp_fail(MDHP_E_INVAL, "surrogate_get_weights: null");
  hipError_t e = hipMemcpyAsync(dst, s->w, s->n_params * 4, hipMemcpyDeviceToDevice,
                                (hipStream_t)stream);
  return e == hipSuccess ? MDHP_OK : mdhp_hip_fail(e, "surrogate_get_weights");
}

mdhp_status mdhp_surrogate_set_weights(mdhp_surrogate* s, const float* src, void* stream) {
  if (!sur_ok(s) || !src) return mdhp_fail(MDHP_E_INVAL, "surrogate_set_weights: null");
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(s->w, src, s->n_params * 4, hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(s->n_params)), dim3(256), 0, st, s->w, s->wb,
                       s->n_params);
    e = hipGetLastError();
  }
  return e == hipSuccess ? MDHP_OK : mdhp_hip_fail(e, "surrogate_set_weights");
}

mdhp_status mdhp_surrogate_get_gradients(mdhp_surrogate* s, float* dst, void* stream) {
  if (!sur_ok(s) || !dst) return mdhp_fail(MDHP_E_INVAL, "surrogate_get_gradients: null");
  hipError_t e = hipMemcpyAsync(dst, s->g, s->n_params * 4, hipMemcpyDeviceToDevice,
                                (hipStream_t)stream);
  return e == hipSuccess ? MDHP_OK : mdhp_hip_fail(e, "surrogate_get_gradients");
}

mdhp_status mdhp_surrogate_get_hidden(mdhp_surrogate* s, int32_t B, uint16_t* h1, uint16_t* h2,
                                      void* stream) {
  if (!sur_ok(s) || !h1 || !h2 || B < 0 || B > s->max_batch)
    return mdhp_fail(MDHP_E_INVAL, "surrogate_get_hidden");
  const size_t bytes = (size_t)B * s->hidden * 2;
  hipError_t e = hipMemcpyAsync(h1, s->h1, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h2, s->h2, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  return e == hipSuccess ? MDHP_OK : mdhp_hip_fail(e, "surrogate_get_hidden");
}

static mdhp_status forward(mdhp_surrogate* s, const __bf16* x, int32_t B, float* y,
                           hipStream_t st) {
  const int H = s->hidden, I = s->in_dim, O = s->out_dim;
  hipError_t e;
  // h1 = relu(x W1^T + b1): A = x [B][I], B(k, j) = W1[j][k].
  e = gemm(x, I, 1, s->wb + s->woff[0], 1, I, B, H, I, s->w + s->boff[0], 1, nullptr, s->h1, H,
           st);
  if (e == hipSuccess)
    e = gemm(s->h1, H, 1, s->wb + s->woff[1], 1, H, B, H, H, s->w + s->boff[1], 1, nullptr, s->h2,
             H, st);
  if (e == hipSuccess)
    e = gemm(s->h2, H, 1, s->wb + s->woff[2], 1, H, B, O, H, s->w + s->boff[2], 0, y, nullptr, O,
             st);
  return e == hipSuccess ? MDHP_OK : mdhp_hip_fail(e, "surrogate forward");
}

mdhp_status mdhp_surrogate_forward(mdhp_surrogate* s, const uint16_t* x, int32_t B, float* y,
                                   void* stream) {
  if (!sur_ok(s) || !x || !y) return mdhp_fail(MDHP_E_INVAL, "surrogate_forward: null");
  if (B < 0 || B > s->max_batch) return mdhp_fail(MDHP_E_INVAL, "surrogate_forward: batch size");
  if (B == 0) return MDHP_OK;
  return forward(s, (const __bf16*)x, B, y, (hipStream_t)stream);
}

mdhp_status mdhp_surrogate_backward(mdhp_surrogate* s, const uint16_t* xin, int32_t B,
                                    const float* target, double* loss, void* stream) {
  if (!sur_ok(s) || !xin || !target || !loss)
    return mdhp_fail(MDHP_E_INVAL, "surrogate_backward: null");
  if (B < 1 || B > s->max_batch) return mdhp_fail(MDHP_E_INVAL, "surrogate_backward: batch size");
  hipStream_t st = (hipStream_t)stream;
  const __bf16* x = (const __bf16*)xin;
  const int H = s->hidden, I = s->in_dim, O = s->out_dim;
  mdhp_status rc = forward(s, x, B, s->y, st);
  if (rc != MDHP_OK) return rc;
  hipLaunchKernelGGL(zero_double_kernel, dim3(1), dim3(1), 0, st, loss);
  const int64_t ny = (int64_t)B * O;
  hipLaunchKernelGGL(mse_kernel, dim3(grid_for(ny)), dim3(256), 0, st, s->y, target, ny, s->dy,
                     loss);
  float* g = s->g;
  hipError_t e = hipGetLastError();
  // Layer 3: dW3 = dy^T h2 [O][H]; db3 = colsum(dy); dh = dy W3 [B][H].
  if (e == hipSuccess)
    e = gemm(s->dy, 1, O, s->h2, H, 1, O, H, B, nullptr, 0, g + s->woff[2], nullptr, H, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(colsum_kernel, dim3((O + kColsumCols - 1) / kColsumCols), dim3(256), 0, st, s->dy, B, O,
                       g + s->boff[2]);
    e = gemm(s->dy, O, 1, s->wb + s->woff[2], H, 1, B, H, O, nullptr, 0, nullptr, s->dh, H, st);
  }
  const int64_t nh = (int64_t)B * H;
  // Layer 2.
  if (e == hipSuccess) {
    hipLaunchKernelGGL(relu_grad_kernel, dim3(grid_for(nh)), dim3(256), 0, st, s->dh, s->h2, s->dz,
                       nh);
    e = gemm(s->dz, 1, H, s->h1, H, 1, H, H, B, nullptr, 0, g + s->woff[1], nullptr, H, st);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(colsum_kernel, dim3((H + kColsumCols - 1) / kColsumCols), dim3(256), 0, st, s->dz, B, H,
                       g + s->boff[1]);
    e = gemm(s->dz, H, 1, s->wb + s->woff[1], H, 1, B, H, H, nullptr, 0, nullptr, s->dh, H, st);
  }
  // Layer 1.
  if (e == hipSuccess) {
    hipLaunchKernelGGL(relu_grad_kernel, dim3(grid_for(nh)), dim3(256), 0, st, s->dh, s->h1, s->dz,
                       nh);
    e = gemm(s->dz, 1, H, x, I, 1, H, I, B, nullptr, 0, g + s->woff[0], nullptr, I, st);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(colsum_kernel, dim3((H + kColsumCols - 1) / kColsumCols), dim3(256), 0, st, s->dz, B, H,
                       g + s->boff[0]);
    e = hipGetLastError();
  }
  return e == hipSuccess ? MDHP_OK : mdhp_hip_fail(e, "surrogate backward");
}

mdhp_status mdhp_surrogate_adam(mdhp_surrogate* s, float lr, float b1, float b2, float eps,
                                void* stream) {
  if (!sur_ok(s) || !(lr > 0.f)) return mdhp_fail(MDHP_E_INVAL, "surrogate_adam");
  s->step += 1;
  const float bc1 = 1.f - std::pow(b1, (float)s->step);
  const float bc2 = 1.f - std::pow(b2, (float)s->step);
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(s->n_params)), dim3(256), 0, (hipStream_t)stream,
                     s->w, s->g, s->m1, s->m2, s->wb, s->n_params, lr, b1, b2, eps, bc1, bc2);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MDHP_OK : mdhp_hip_fail(e, "surrogate_adam");
}

mdhp_status mdhp_surrogate_save(mdhp_surrogate* s, const char* path, const float* extra,
                                int64_t n_extra, void* stream) {
  if (!sur_ok(s) || !path || n_extra < 0 || (n_extra > 0 && !extra))
    return mdhp_fail(MDHP_E_INVAL, "surrogate_save: invalid argument");
  const int64_t n = s->n_params;
  std::vector<float> host((size_t)n * 3);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(host.data(), s->w, n * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(host.data() + n, s->m1, n * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(host.data() + 2 * n, s->m2, n * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return mdhp_hip_fail(e, "surrogate_save");
  CheckpointHeader h;
  std::memcpy(h.magic, kCheckpointMagic, 8);
  h.version = 1;
  h.in_dim = s->in_dim;
  h.hidden = s->hidden;
  h.out_dim = s->out_dim;
  h.n_params = n;
  h.step = s->step;
  h.n_extra = n_extra;
  FILE* f = std::fopen(path, "wb");
  if (!f) return mdhp_fail(MDHP_E_IO, std::string("surrogate_save: cannot open ") + path);
  bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 &&
            std::fwrite(host.data(), 4, host.size(), f) == host.size() &&
            (n_extra == 0 || std::fwrite(extra, 4, (size_t)n_extra, f) == (size_t)n_extra);
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return mdhp_fail(MDHP_E_IO, std::string("surrogate_save: write failed: ") + path);
  return MDHP_OK;
}

mdhp_status mdhp_surrogate_load(mdhp_surrogate* s, const char* path, float* extra,
                                int64_t extra_cap, int64_t* n_extra, void* stream) {
  if (!sur_ok(s) || !path || extra_cap < 0)
    return mdhp_fail(MDHP_E_INVAL, "surrogate_load: invalid argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return mdhp_fail(MDHP_E_IO, std::string("surrogate_load: cannot open ") + path);
  CheckpointHeader h;
  if (std::fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, kCheckpointMagic, 8) != 0 ||
      h.version != 1 || h.n_extra < 0) {
    std::fclose(f);
    return mdhp_fail(MDHP_E_IO, std::string("surrogate_load: not a surrogate checkpoint: ") + path);
  }
  if (h.in_dim != s->in_dim || h.hidden != s->hidden || h.out_dim != s->out_dim ||
      h.n_params != s->n_params) {
    std::fclose(f);
    return mdhp_fail(MDHP_E_INVAL, "surrogate_load: the checkpoint's network has another shape");
  }
  const int64_t n = s->n_params;
  std::vector<float> host((size_t)n * 3);
  std::vector<float> ext((size_t)h.n_extra);
  const bool ok = std::fread(host.data(), 4, host.size(), f) == host.size() &&
                  (h.n_extra == 0 || std::fread(ext.data(), 4, ext.size(), f) == ext.size());
  std::fclose(f);
  if (!ok) return mdhp_fail(MDHP_E_IO, std::string("surrogate_load: truncated file: ") + path);
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(s->w, host.data(), n * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(s->m1, host.data() + n, n * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->m2, host.data() + 2 * n, n * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, st, s->w, s->wb, n);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return mdhp_hip_fail(e, "surrogate_load");
  s->step = h.step;
  if (n_extra) *n_extra = h.n_extra;
  if (extra && h.n_extra > 0)
    std::memcpy(extra, ext.data(), (size_t)std::min<int64_t>(extra_cap, h.n_extra) * 4);
  return MDHP_OK;
}

mdhp_status mdhp_surrogate_train_step(mdhp_surrogate* s, const uint16_t* x, int32_t B,
                                      const float* target, float lr, double* loss,
                                      void* stream) {
  mdhp_status rc = mdhp_surrogate_backward(s, x, B, target, loss, stream);
  if (rc != MDHP_OK) return rc;
  return mdhp_surrogate_adam(s, lr, 0.9f, 0.999f, 1e-8f, stream);
}

}  // extern "C"

namespace mdhp {

hipError_t warm_params(const float* pred, const float* mean, const float* stdv,
                       const int32_t* counts, const int32_t* n, const double* T, int64_t W,
                       int M, float mu_floor_rel, float beta_floor_rel, float* mu, float* alpha,
                       float* beta, hipStream_t s) {
  const int64_t total = W * (int64_t)(M + M * M + 1);
  hipLaunchKernelGGL(warm_params_kernel, dim3(grid_for(total)), dim3(256), 0, s, pred, mean, stdv,
                     counts, n, T, W, M, mu_floor_rel, beta_floor_rel, mu, alpha, beta);
  return hipGetLastError();
}

hipError_t choose_init(const double* ll_warm, const double* ll_cold, int64_t W, int M,
                       const float* mu_c, const float* al_c, const float* be_c, float* mu,
                       float* alpha, float* beta, int32_t* used_warm, hipStream_t s) {
  if (W == 0) return hipSuccess;
  hipLaunchKernelGGL(choose_init_kernel, dim3((unsigned)W), dim3(256), 0, s, ll_warm, ll_cold, W,
                     M, mu_c, al_c, be_c, mu, alpha, beta, used_warm);
  return hipGetLastError();
}

}  // namespace mdhp
