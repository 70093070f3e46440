// The MDHP-LSTM layer (Sec. IV, "MDHP-LSTM", Eq. (7)) on the GPU, in FP32.
//
// For B sequences of L inputs x_t of width D, hidden width H, and each
// sequence's fitted window parameters (alpha, beta, theta = mu) and length
// T_span:
//   hks = tanh(A vec(alpha) - B (beta T_span) + C theta)        once per sequence
//   z_t = W x_t + U h_{t-1} + b; i, f, o = sigmoid and g = tanh of its blocks
//   c_t = hks * (f c_{t-1} + i g),  h_t = o tanh(c_t),  h_{-1} = c_{-1} = 0.
//
// Work split:
//  * the input products W x_t + b of all steps, and hks, are GEMMs before the
//    recurrence (gemm_f32_kernel);
//  * the recurrence (lstm_fwd_kernel): one workgroup per 16 sequences runs
//    all L steps; h_{t-1} U^T on the matrix cores (v_mfma_f32_16x16x4_f32)
//    with h_{t-1} in LDS and U streamed from L2 in a lane-packed layout, so
//    that every B operand of a wavefront is one contiguous 1 KB load; each
//    lane ends a step holding i, f, g, o of the same (sequence, unit) pairs
//    and updates their cells in registers;
//  * backward (lstm_bwd_kernel) runs the steps in reverse, with dz_{t+1} U on
//    the matrix cores, and writes the pre-activation gradients dz_t over the
//    saved gates, plus the hks gradient; the weight and input gradients then
//    are GEMMs over all steps: dX = dZ W, dW = dZ^T X,
//    dU = sum_t dz_t^T h_{t-1}, db = column sums of dZ, and the Hawkes-gate
//    weights from dpre = dhks (1 - hks^2).
//
// MFMA 16x16x4 FP32 operand layout (lane l): A[i = l % 16][k = l / 16],
// B[k = l / 16][j = l % 16]; result element r: row 4 (l / 16) + r, column
// l % 16.  The recurrent kernels take four k-steps per float4: in k-group
// ks lane l supplies k = 16 ks + 4 (l / 16) + s at step s, so that both its
// A values (one LDS row) and its B values (one row of U) are contiguous.

#include <cmath>

#include "mdhp_device.h"

namespace mdhp {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.f / (1.f + expf(-z)); }

// ----------------------------------------------------------------- GEMM
// C[i][j] = epilogue(sum_{z < Z} sum_{k < K} A(z, i, k) B(z, k, j)) with
// A(z, i, k) = A[z saz + i sai + k sak] and B(z, k, j) = B[z sbz + k sbk +
// j sbj].  With S > 1 workgroup slice s of the grid sums its share of z (Z
// > 1) or of k (Z = 1) into part[s][Mr][Nc], and gemm_reduce_kernel adds the
// slices in order and applies the epilogue (deterministic).  Epilogue:
// + bias[j], then tanh if act, then store or add to C.
// Tiles: 64 x 64 per workgroup of 4 waves (2 x 2 of 32 x 32), K staged in
// LDS 16 at a time.
constexpr int GT = 64, GK = 16, GLD = GT + 16;  // row stride 80: 4 k-rows in distinct banks

struct GemmF32 {
  const float* A;
  int64_t saz, sai, sak;
  const float* B;
  int64_t sbz, sbk, sbj;
  int64_t Z, K;
  int64_t Mr, Nc;
  float* C;
  int64_t ldc;
  float* part;
  const float* bias;
  int act, accumulate, S;
};

__device__ __forceinline__ void gemm_finish(const GemmF32& g, int64_t i, int64_t j, float v) {
  if (g.bias) v += g.bias[j];
  if (g.act) v = tanhf(v);
  float* dst = g.C + i * g.ldc + j;
  *dst = g.accumulate ? *dst + v : v;
}

__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmF32 g) {
  __shared__ float As[GK][GLD];  // As[k][i]
  __shared__ float Bs[GK][GLD];  // Bs[k][j]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * GT, j0 = (int64_t)blockIdx.x * GT;
  const int s = blockIdx.z;
  int64_t zb = 0, ze = g.Z, kb = 0, ke = g.K;
  if (g.S > 1) {
    if (g.Z > 1) {
      zb = g.Z * s / g.S;
      ze = g.Z * (s + 1) / g.S;
    } else {
      kb = g.K * s / g.S;
      ke = g.K * (s + 1) / g.S;
    }
  }
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const bool a_kc = g.sak == 1;  // stage A along k, else along i
  const bool b_jc = g.sbj == 1;  // stage B along j, else along k
  f32x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int64_t z = zb; z < ze; ++z) {
    const float* Az = g.A + z * g.saz;
    const float* Bz = g.B + z * g.sbz;
    for (int64_t k0 = kb; k0 < ke; k0 += GK) {
      float av[4], bv[4];
      int ai[4], ak[4], bj[4], bk[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int idx = tid + 256 * e;  // 0 .. 1023 over a 64 x 16 tile
        ai[e] = a_kc ? idx / GK : idx % GT;
        ak[e] = a_kc ? idx % GK : idx / GT;
        const int64_t gi = i0 + ai[e], gk = k0 + ak[e];
        av[e] = (gi < g.Mr && gk < ke) ? Az[gi * g.sai + gk * g.sak] : 0.f;
        bj[e] = b_jc ? idx % GT : idx / GK;
        bk[e] = b_jc ? idx / GT : idx % GK;
        const int64_t gj = j0 + bj[e], gk2 = k0 + bk[e];
        bv[e] = (gj < g.Nc && gk2 < ke) ? Bz[gk2 * g.sbk + gj * g.sbj] : 0.f;
      }
      __syncthreads();  // the previous chunk's LDS reads are done
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        As[ak[e]][ai[e]] = av[e];
        Bs[bk[e]][bj[e]] = bv[e];
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < GK; kk += 4) {
        const int kr = kk + (lane >> 4);
        float a[2], b[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) a[x] = As[kr][wm + 16 * x + (lane & 15)];
#pragma unroll
        for (int y = 0; y < 2; ++y) b[y] = Bs[kr][wn + 16 * y + (lane & 15)];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) acc[x][y] = mfma4(a[x], b[y], acc[x][y]);
      }
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wm + 16 * x + 4 * (lane >> 4) + r;
        const int64_t j = j0 + wn + 16 * y + (lane & 15);
        if (i < g.Mr && j < g.Nc) {
          if (g.S > 1) g.part[((int64_t)s * g.Mr + i) * g.Nc + j] = acc[x][y][r];
          else gemm_finish(g, i, j, acc[x][y][r]);
        }
      }
}

__global__ void gemm_reduce_kernel(GemmF32 g) {
  const int64_t n = g.Mr * g.Nc;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    float v = 0.f;
    for (int s = 0; s < g.S; ++s) v += g.part[s * n + e];
    gemm_finish(g, e / g.Nc, e % g.Nc, v);
  }
}

constexpr int kMaxSplit = 16;

// Splits so that tiles x splits reaches about 1,024 workgroups, each split
// keeping at least 256 of the reduction.
int gemm_splits(int64_t Mr, int64_t Nc, int64_t Z, int64_t K) {
  const int64_t tiles = ((Mr + GT - 1) / GT) * ((Nc + GT - 1) / GT);
  int64_t s = (1024 + tiles - 1) / tiles;
  const int64_t red = Z > 1 ? Z : K / 256;
  s = std::min<int64_t>(s, std::max<int64_t>(red, 1));
  return (int)std::max<int64_t>(1, std::min<int64_t>(s, kMaxSplit));
}

hipError_t gemm_f32(GemmF32 g, float* part, hipStream_t st) {
  g.S = part ? gemm_splits(g.Mr, g.Nc, g.Z, g.K) : 1;
  g.part = part;
  if (g.Mr == 0 || g.Nc == 0) return hipSuccess;
  const dim3 grid((unsigned)((g.Nc + GT - 1) / GT), (unsigned)((g.Mr + GT - 1) / GT),
                  (unsigned)g.S);
  hipLaunchKernelGGL(gemm_f32_kernel, grid, dim3(256), 0, st, g);
  if (g.S > 1) {
    const int64_t n = g.Mr * g.Nc;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(gemm_reduce_kernel, dim3(blocks), dim3(256), 0, st, g);
  }
  return hipGetLastError();
}

// ------------------------------------------------------ small elementwise
// feat[b] = (vec alpha, -beta T_span, theta): the Hawkes gate's input with
// the sign of the B block folded in, so that pre = [A | B | C] feat.
__global__ void lstm_features_kernel(int64_t Bn, int M, int Kb, const float* __restrict__ alpha,
                                     const float* __restrict__ beta,
                                     const float* __restrict__ T_span,
                                     const float* __restrict__ theta, float* __restrict__ feat) {
  const int M2 = M * M, Kf = M2 + Kb + M;
  const int64_t n = Bn * Kf;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / Kf;
    const int k = (int)(e % Kf);
    float v;
    if (k < M2) v = alpha[b * M2 + k];
    else if (k < M2 + Kb) v = -(beta[b * Kb + (k - M2)] * T_span[b]);
    else v = theta[b * M + (k - M2 - Kb)];
    feat[e] = v;
  }
}

// Lane-packed copies of U [4H][H] for the recurrent kernels.
//   Up [(nt KS + ks) 64 + l] = U[q H + 16 ut + l % 16][16 ks + 4 (l / 16) + s], s = 0..3,
//     nt = q (H / 16) + ut over the 4H gate columns, KS = H / 16 (forward: h U^T);
//   UpT[(nt KT + ks) 64 + l] = U[16 ks + 4 (l / 16) + s][16 nt + l % 16],
//     nt over the H units, KT = 4H / 16 (backward: dz U).
__global__ void lstm_pack_kernel(int H, const float* __restrict__ U, float4* __restrict__ Up,
                                 float4* __restrict__ UpT) {
  const int64_t n = (int64_t)H * H;  // float4 entries of each copy
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(e & 63);
    const int64_t tile = e >> 6;
    {
      const int KS = H / 16;
      const int nt = (int)(tile / KS), ks = (int)(tile % KS);
      const int q = nt / (H / 16), ut = nt % (H / 16);
      const float* row = U + (int64_t)(q * H + 16 * ut + (l & 15)) * H + 16 * ks + 4 * (l >> 4);
      Up[e] = make_float4(row[0], row[1], row[2], row[3]);
    }
    {
      const int KT = 4 * H / 16;
      const int nt = (int)(tile / KT), ks = (int)(tile % KT);
      const int k = 16 * ks + 4 * (l >> 4), col = 16 * nt + (l & 15);
      UpT[e] = make_float4(U[(int64_t)k * H + col], U[(int64_t)(k + 1) * H + col],
                           U[(int64_t)(k + 2) * H + col], U[(int64_t)(k + 3) * H + col]);
    }
  }
}

// dpre = dhks (1 - hks^2), in place.
__global__ void lstm_dpre_kernel(int64_t n, const float* __restrict__ hks, float* __restrict__ d) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const float k = hks[e];
    d[e] *= 1.f - k * k;
  }
}

// dfeat's beta T_span block: the GEMM gave the gradient with respect to
// -beta T_span.
__global__ void lstm_negate_block_kernel(int64_t Bn, int Kf, int c0, int nc, float* __restrict__ x) {
  const int64_t n = Bn * nc;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    x[(e / nc) * Kf + c0 + e % nc] *= -1.f;
}

// part[s][j] = sum of column j of X [rows][cols] over split s's rows.
__global__ void colsum_part_kernel(const float* __restrict__ X, int64_t rows, int cols, int S,
                                   float* __restrict__ part) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (j >= cols) return;
  const int64_t r0 = rows * s / S, r1 = rows * (s + 1) / S;
  float v = 0.f;
  for (int64_t r = r0; r < r1; ++r) v += X[r * cols + j];
  part[(int64_t)s * cols + j] = v;
}

__global__ void colsum_reduce_kernel(const float* __restrict__ part, int cols, int S,
                                     float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float v = 0.f;
  for (int s = 0; s < S; ++s) v += part[(int64_t)s * cols + j];
  out[j] = v;
}

constexpr int kColsumSplit = 256;

// ------------------------------------------------------------ recurrence
constexpr int kRows = 16;  // sequences per workgroup (one MFMA row tile)

// gates [B][L][4H]: on entry W x_t + b, on exit (i, f, g, o); c and h
// [B][L][H]; hks [B][H].
template <int H>
__global__ __launch_bounds__(256) void lstm_fwd_kernel(int64_t Bn, int L,
                                                       const float4* __restrict__ Up,
                                                       const float* __restrict__ hks,
                                                       float* __restrict__ gates,
                                                       float* __restrict__ cs,
                                                       float* __restrict__ hout) {
  constexpr int UT = H / 64;  // unit tiles per wave
  constexpr int NT = 4 * UT;  // gate-column tiles per wave
  constexpr int KS = H / 16;  // k-groups of 16
  constexpr int HS = H + 4;   // LDS row stride (float4-aligned)
  __shared__ __attribute__((aligned(16))) float hs[2][kRows][HS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  for (int e = tid; e < kRows * HS; e += 256) hs[0][e / HS][e % HS] = 0.f;
  float hk[UT][4], c[UT][4];
#pragma unroll
  for (int ut = 0; ut < UT; ++ut)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + 4 * lq + r;
      const int u = (wave * UT + ut) * 16 + lr;
      hk[ut][r] = row < Bn ? hks[row * H + u] : 0.f;
      c[ut][r] = 0.f;
    }
  __syncthreads();
  for (int t = 0; t < L; ++t) {
    const int cur = t & 1;
    f32x4 acc[NT];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int ut = 0; ut < UT; ++ut)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = r0 + 4 * lq + r;
          const int col = q * H + (wave * UT + ut) * 16 + lr;
          acc[q * UT + ut][r] = row < Bn ? gates[(row * L + t) * (4 * H) + col] : 0.f;
        }
    if (t > 0) {
#pragma unroll 2
      for (int ks = 0; ks < KS; ++ks) {
        const float4 a = *reinterpret_cast<const float4*>(&hs[cur][lr][16 * ks + 4 * lq]);
#pragma unroll
        for (int n = 0; n < NT; ++n) {
          const int q = n / UT, ut = n % UT;
          const int ntg = q * (H / 16) + wave * UT + ut;
          const float4 b = Up[((int64_t)ntg * KS + ks) * 64 + lane];
          acc[n] = mfma4(a.x, b.x, acc[n]);
          acc[n] = mfma4(a.y, b.y, acc[n]);
          acc[n] = mfma4(a.z, b.z, acc[n]);
          acc[n] = mfma4(a.w, b.w, acc[n]);
        }
      }
    }
#pragma unroll
    for (int ut = 0; ut < UT; ++ut)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + 4 * lq + r;
        const int u = (wave * UT + ut) * 16 + lr;
        const float i = sigmoidf(acc[0 * UT + ut][r]);
        const float f = sigmoidf(acc[1 * UT + ut][r]);
        const float g = tanhf(acc[2 * UT + ut][r]);
        const float o = sigmoidf(acc[3 * UT + ut][r]);
        const float cn = hk[ut][r] * (f * c[ut][r] + i * g);
        const float h = o * tanhf(cn);
        c[ut][r] = cn;
        hs[cur ^ 1][4 * lq + r][u] = row < Bn ? h : 0.f;
        if (row < Bn) {
          float* gp = gates + (row * L + t) * (4 * H) + u;
          gp[0] = i;
          gp[H] = f;
          gp[2 * H] = g;
          gp[3 * H] = o;
          cs[(row * L + t) * H + u] = cn;
          hout[(row * L + t) * H + u] = h;
        }
      }
    __syncthreads();
  }
}

// gates [B][L][4H]: on entry (i, f, g, o), on exit dz (the gradient with
// respect to the pre-activations); dh [B][L][H] the loss's gradient with
// respect to each h_t; dhks [B][H] out.
template <int H>
__global__ __launch_bounds__(256) void lstm_bwd_kernel(int64_t Bn, int L,
                                                       const float4* __restrict__ UpT,
                                                       const float* __restrict__ hks,
                                                       float* __restrict__ gates,
                                                       const float* __restrict__ cs,
                                                       const float* __restrict__ dh,
                                                       float* __restrict__ dhks) {
  constexpr int UT = H / 64;      // unit tiles per wave
  constexpr int KT = 4 * H / 16;  // k-groups over the gate columns
  constexpr int GS = 4 * H + 4;
  __shared__ __attribute__((aligned(16))) float dzs[kRows][GS];  // dz_{t+1}
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  float hk[UT][4], dc[UT][4], dk[UT][4];
#pragma unroll
  for (int ut = 0; ut < UT; ++ut)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + 4 * lq + r;
      const int u = (wave * UT + ut) * 16 + lr;
      hk[ut][r] = row < Bn ? hks[row * H + u] : 0.f;
      dc[ut][r] = 0.f;
      dk[ut][r] = 0.f;
    }
  for (int t = L - 1; t >= 0; --t) {
    f32x4 acc[UT];
#pragma unroll
    for (int ut = 0; ut < UT; ++ut) acc[ut] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (t < L - 1) {
#pragma unroll 2
      for (int ks = 0; ks < KT; ++ks) {
        const float4 a = *reinterpret_cast<const float4*>(&dzs[lr][16 * ks + 4 * lq]);
#pragma unroll
        for (int ut = 0; ut < UT; ++ut) {
          const int ntg = wave * UT + ut;
          const float4 b = UpT[((int64_t)ntg * KT + ks) * 64 + lane];
          acc[ut] = mfma4(a.x, b.x, acc[ut]);
          acc[ut] = mfma4(a.y, b.y, acc[ut]);
          acc[ut] = mfma4(a.z, b.z, acc[ut]);
          acc[ut] = mfma4(a.w, b.w, acc[ut]);
        }
      }
    }
    __syncthreads();  // every read of dz_{t+1} is done
#pragma unroll
    for (int ut = 0; ut < UT; ++ut)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + 4 * lq + r;
        const int u = (wave * UT + ut) * 16 + lr;
        float dzi = 0.f, dzf = 0.f, dzg = 0.f, dzo = 0.f;
        if (row < Bn) {
          float* gp = gates + (row * L + t) * (4 * H) + u;
          const float i = gp[0], f = gp[H], g = gp[2 * H], o = gp[3 * H];
          const float ct = cs[(row * L + t) * H + u];
          const float cp = t > 0 ? cs[(row * L + t - 1) * H + u] : 0.f;
          const float dht = dh[(row * L + t) * H + u] + acc[ut][r];
          const float tc = tanhf(ct);
          const float dct = dc[ut][r] + dht * o * (1.f - tc * tc);
          const float s = f * cp + i * g;  // c_t = hks s
          dk[ut][r] += dct * s;
          const float ds = dct * hk[ut][r];
          dzi = ds * g * i * (1.f - i);
          dzf = ds * cp * f * (1.f - f);
          dzg = ds * i * (1.f - g * g);
          dzo = dht * tc * o * (1.f - o);
          dc[ut][r] = ds * f;
          gp[0] = dzi;
          gp[H] = dzf;
          gp[2 * H] = dzg;
          gp[3 * H] = dzo;
        }
        float* zp = &dzs[4 * lq + r][u];
        zp[0] = dzi;
        zp[H] = dzf;
        zp[2 * H] = dzg;
        zp[3 * H] = dzo;
      }
    __syncthreads();
  }
#pragma unroll
  for (int ut = 0; ut < UT; ++ut)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + 4 * lq + r;
      if (row < Bn) dhks[row * H + (wave * UT + ut) * 16 + lr] = dk[ut][r];
    }
}

unsigned ew_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

struct Shape {
  int64_t B;
  int L, D, H, M, Kb, Kf;
};

mdhp_status lstm_shape(const mdhp_lstm_dims* d, Shape* s) {
  if (!d) return mdhp_fail(MDHP_E_INVAL, "lstm: null dims");
  if (d->B < 0 || d->L < 1 || d->D < 1 || (d->H != 64 && d->H != 128 && d->H != 256) ||
      d->M < 1 || d->M > 64 || (d->beta_mode != MDHP_BETA_SHARED && d->beta_mode != MDHP_BETA_PAIR))
    return mdhp_fail(MDHP_E_INVAL,
                     "lstm: need B >= 0, L >= 1, D >= 1, H in {64, 128, 256}, 1 <= M <= 64 and a "
                     "decay mode");
  s->B = d->B;
  s->L = d->L;
  s->D = d->D;
  s->H = d->H;
  s->M = d->M;
  s->Kb = d->beta_mode == MDHP_BETA_PAIR ? d->M * d->M : 1;
  s->Kf = d->M * d->M + s->Kb + d->M;
  return MDHP_OK;
}

// Saved-state layout (floats): gates [B][L][4H], c [B][L][H], hks [B][H],
// feat [B][Kf].
int64_t saved_floats(const Shape& s) {
  return s.B * s.L * 5 * (int64_t)s.H + s.B * (int64_t)s.H + s.B * (int64_t)s.Kf;
}
// Workspace layout (floats): Up [4H H], UpT [4H H], GEMM partials, dhks [B][H].
int64_t part_floats(const Shape& s) {
  const int64_t big = std::max<int64_t>(4 * (int64_t)s.H * std::max(s.D, s.H),
                                        (int64_t)s.H * s.Kf);
  return std::max<int64_t>(kMaxSplit * big, (int64_t)kColsumSplit * 4 * s.H);
}
int64_t work_floats(const Shape& s) {
  return 8 * (int64_t)s.H * s.H + part_floats(s) + s.B * (int64_t)s.H;
}

template <int H>
void launch_fwd(const Shape& s, const float4* Up, const float* hks, float* gates, float* cs,
                float* h, hipStream_t st) {
  hipLaunchKernelGGL(lstm_fwd_kernel<H>, dim3((unsigned)((s.B + kRows - 1) / kRows)), dim3(256),
                     0, st, s.B, s.L, Up, hks, gates, cs, h);
}
template <int H>
void launch_bwd(const Shape& s, const float4* UpT, const float* hks, float* gates, const float* cs,
                const float* dh, float* dhks, hipStream_t st) {
  hipLaunchKernelGGL(lstm_bwd_kernel<H>, dim3((unsigned)((s.B + kRows - 1) / kRows)), dim3(256),
                     0, st, s.B, s.L, UpT, hks, gates, cs, dh, dhks);
}

}  // namespace

}  // namespace mdhp

using namespace mdhp;

extern "C" {

mdhp_status mdhp_lstm_sizes(const mdhp_lstm_dims* d, int64_t* saved, int64_t* work) {
  Shape s;
  const mdhp_status e = lstm_shape(d, &s);
  if (e != MDHP_OK) return e;
  if (!saved || !work) return mdhp_fail(MDHP_E_INVAL, "lstm_sizes: null output");
  *saved = saved_floats(s);
  *work = work_floats(s);
  return MDHP_OK;
}

mdhp_status mdhp_lstm_forward(const mdhp_lstm_dims* d, const float* x, const float* W,
                              const float* U, const float* bias, const float* Whks,
                              const float* alpha, const float* beta, const float* T_span,
                              const float* theta, float* h, float* saved, float* work,
                              void* stream) {
  Shape s;
  mdhp_status e = lstm_shape(d, &s);
  if (e != MDHP_OK) return e;
  if (s.B == 0) return MDHP_OK;
  if (!x || !W || !U || !bias || !Whks || !alpha || !beta || !T_span || !theta || !h || !saved ||
      !work)
    return mdhp_fail(MDHP_E_INVAL, "lstm_forward: null pointer");
  hipStream_t st = (hipStream_t)stream;
  const int64_t H = s.H, G = 4 * H, BL = s.B * s.L;
  float* gates = saved;
  float* cs = gates + BL * G;
  float* hks = cs + BL * H;
  float* feat = hks + s.B * H;
  float4* Up = reinterpret_cast<float4*>(work);
  float4* UpT = Up + H * H;
  hipLaunchKernelGGL(lstm_features_kernel, dim3(ew_blocks(s.B * s.Kf)), dim3(256), 0, st, s.B,
                     s.M, s.Kb, alpha, beta, T_span, theta, feat);
  hipLaunchKernelGGL(lstm_pack_kernel, dim3(ew_blocks(H * H)), dim3(256), 0, st, s.H, U, Up, UpT);
  // hks = tanh(feat [B][Kf] Whks^T)
  GemmF32 g1{feat, 0, s.Kf, 1, Whks, 0, 1, s.Kf, 1, s.Kf, s.B, H, hks, H,
             nullptr, nullptr, 1, 0, 1};
  hipError_t he = gemm_f32(g1, nullptr, st);
  // gates = x [BL][D] W^T + b
  GemmF32 g2{x, 0, s.D, 1, W, 0, 1, s.D, 1, s.D, BL, G, gates, G, nullptr, bias, 0, 0, 1};
  if (he == hipSuccess) he = gemm_f32(g2, nullptr, st);
  if (he != hipSuccess) return mdhp_hip_fail(he, "lstm_forward");
  switch (s.H) {
    case 64: launch_fwd<64>(s, Up, hks, gates, cs, h, st); break;
    case 128: launch_fwd<128>(s, Up, hks, gates, cs, h, st); break;
    default: launch_fwd<256>(s, Up, hks, gates, cs, h, st); break;
  }
  he = hipGetLastError();
  return he == hipSuccess ? MDHP_OK : mdhp_hip_fail(he, "lstm_forward");
}

mdhp_status mdhp_lstm_backward(const mdhp_lstm_dims* d, const float* x, const float* W,
                               const float* U, const float* Whks, const float* h, float* saved,
                               const float* dh, float* dx, float* dW, float* dU, float* dbias,
                               float* dWhks, float* dfeat, float* work, void* stream) {
  Shape s;
  mdhp_status e = lstm_shape(d, &s);
  if (e != MDHP_OK) return e;
  // Arrays of B rows may be null for an empty batch (the weight gradients
  // are then zero).
  if (!W || !U || !Whks || !dW || !dU || !dbias || !dWhks || !work ||
      (s.B > 0 && (!x || !h || !saved || !dh || !dx || !dfeat)))
    return mdhp_fail(MDHP_E_INVAL, "lstm_backward: null pointer");
  hipStream_t st = (hipStream_t)stream;
  const int64_t H = s.H, G = 4 * H, BL = s.B * s.L;
  float* dz = saved;  // the gates, overwritten by their gradients
  const float* cs = dz + BL * G;
  const float* hks = cs + BL * H;
  const float* feat = hks + s.B * H;
  float4* Up = reinterpret_cast<float4*>(work);
  float4* UpT = Up + H * H;
  float* part = work + 8 * H * H;
  float* dpre = part + part_floats(s);
  if (s.B > 0) {
    hipLaunchKernelGGL(lstm_pack_kernel, dim3(ew_blocks(H * H)), dim3(256), 0, st, s.H, U, Up,
                       UpT);
    switch (s.H) {
      case 64: launch_bwd<64>(s, UpT, hks, dz, cs, dh, dpre, st); break;
      case 128: launch_bwd<128>(s, UpT, hks, dz, cs, dh, dpre, st); break;
      default: launch_bwd<256>(s, UpT, hks, dz, cs, dh, dpre, st); break;
    }
    hipLaunchKernelGGL(lstm_dpre_kernel, dim3(ew_blocks(s.B * H)), dim3(256), 0, st, s.B * H, hks,
                       dpre);
  }
  hipError_t he = hipGetLastError();
  // dx [BL][D] = dZ [BL][4H] W [4H][D]
  if (he == hipSuccess)
    he = gemm_f32(GemmF32{dz, 0, G, 1, W, 0, s.D, 1, 1, G, BL, s.D, dx, s.D, nullptr, nullptr,
                          0, 0, 1},
                  nullptr, st);
  // dW [4H][D] = dZ^T X
  if (he == hipSuccess)
    he = gemm_f32(GemmF32{dz, 0, 1, G, x, 0, s.D, 1, 1, BL, G, s.D, dW, s.D, nullptr, nullptr,
                          0, 0, 1},
                  part, st);
  // dU [4H][H] = sum over sequences b and steps t >= 1 of dz[b][t]^T h[b][t-1]
  if (he == hipSuccess)
    he = gemm_f32(GemmF32{dz + G, (int64_t)s.L * G, 1, G, h, (int64_t)s.L * H, H, 1, s.B,
                          s.L - 1, G, H, dU, H, nullptr, nullptr, 0, 0, 1},
                  part, st);
  // dWhks [H][Kf] = dpre^T feat (feat carries -beta T_span: this is dB itself)
  if (he == hipSuccess)
    he = gemm_f32(GemmF32{dpre, 0, 1, H, feat, 0, s.Kf, 1, 1, s.B, H, s.Kf, dWhks, s.Kf, nullptr,
                          nullptr, 0, 0, 1},
                  part, st);
  // dfeat [B][Kf] = dpre Whks, then the beta T_span block's sign
  if (he == hipSuccess)
    he = gemm_f32(GemmF32{dpre, 0, H, 1, Whks, 0, s.Kf, 1, 1, H, s.B, s.Kf, dfeat, s.Kf, nullptr,
                          nullptr, 0, 0, 1},
                  nullptr, st);
  if (he != hipSuccess) return mdhp_hip_fail(he, "lstm_backward");
  if (s.B > 0)
    hipLaunchKernelGGL(lstm_negate_block_kernel, dim3(ew_blocks(s.B * s.Kb)), dim3(256), 0, st,
                       s.B, s.Kf, s.M * s.M, s.Kb, dfeat);
  // db = column sums of dZ
  const int S = (int)std::max<int64_t>(1, std::min<int64_t>(kColsumSplit, BL / 64));
  hipLaunchKernelGGL(colsum_part_kernel, dim3((unsigned)((G + 255) / 256), (unsigned)S),
                     dim3(256), 0, st, dz, BL, (int)G, S, part);
  hipLaunchKernelGGL(colsum_reduce_kernel, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, st,
                     part, (int)G, S, dbias);
  he = hipGetLastError();
  return he == hipSuccess ? MDHP_OK : mdhp_hip_fail(he, "lstm_backward");
}

}  // extern "C"
