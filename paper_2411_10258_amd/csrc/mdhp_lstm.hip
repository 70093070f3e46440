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
//  * hks is a GEMM before the recurrence (gemm_f32_kernel); so are the input
//    products W x_t + b of all steps for inputs wider than kFusedMaxD,
//    while narrower inputs have them formed inside the recurrence
//    (lstm_fwd_fused_kernel);
//  * the recurrence (lstm_fwd_kernel): one workgroup per 16 sequences runs
//    all L steps; h_{t-1} U^T on the matrix cores (v_mfma_f32_16x16x4_f32)
//    with h_{t-1} in LDS and U streamed from L2 in a lane-packed layout, so
//    that every B operand of a wavefront is one contiguous 1 KB load; each
//    lane ends a step holding i, f, g, o of the same (sequence, unit) pairs
//    and updates their cells in registers;
//  * backward (lstm_bwd_kernel) runs the steps in reverse, with dz_{t+1} U on
//    the matrix cores, and writes the pre-activation gradients dz_t over the
//    saved gates, plus the hks gradient and each workgroup's column sums of
//    dz (db is their sum); the weight and input gradients then are GEMMs
//    over all steps: dX = dZ W, dW = dZ^T X, dU = sum_t dz_t^T h_{t-1}, and
//    the Hawkes-gate weights from dpre = dhks (1 - hks^2).
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
// j sbj].  With S > 1 grid row s sums its share of z (Z > 1) or of k (Z = 1)
// into part[s][Mr][Nc], and gemm_reduce_kernel adds the shares in order and
// applies the epilogue (deterministic).  Epilogue: + bias[j], then tanh if
// act, then store or add to C.
// Tiles: 128 x 128 per workgroup of 4 waves (2 x 2 of 64 x 64, 4 x 4 MFMA
// blocks each), K staged in LDS 32 at a time with k contiguous per row, so
// that a lane's A and B values for four k-steps are one float4 each (the
// k-permuted order of the recurrent kernels: in k-group kg lane l supplies
// k = 16 kg + 4 (l / 16) + s at step s); the next chunk's global loads are
// issued before the current chunk's products.  Tile order: the hardware
// deals consecutive workgroups round-robin to the 8 XCDs; each XCD is given
// a contiguous run of row-major tiles, so that the workgroups sharing an A
// row strip (and, for few column tiles, a B column strip) share one L2.
constexpr int GT = 128, GK = 32, GLD = GK + 4;  // row stride 36: 16 rows in distinct banks
constexpr int kXcds = 8;

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

// Tile (row, column) of dispatch id x among T = nI nJ tiles.
__device__ __forceinline__ void gemm_tile(int64_t x, int64_t nJ, int64_t T, int64_t* ti,
                                          int64_t* tj) {
  const int64_t q = T / kXcds, r = T % kXcds;
  const int64_t xcd = x % kXcds, slot = x / kXcds;
  const int64_t t = xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
  *ti = t / nJ;
  *tj = t % nJ;
}

// Staging of one operand's 128 x 32 tile: element (m, k) of the tile is
// P[m sm + k sk] (m the tile's row or column index).  With k contiguous
// (sk == 1) thread t loads 16 consecutive k of row t / 2; otherwise 16
// consecutive m of k-row t % 32 (so that a wavefront's transposing LDS
// stores spread over 32 banks).  v receives them; store() writes them to
// LDS as T[m][k].
struct TileStage {
  bool kc;
  __device__ __forceinline__ void load(const float* P, int64_t sm, int64_t sk, int64_t m0,
                                       int64_t mlim, int64_t k0, int64_t klim, int tid,
                                       float (&v)[16]) const {
    // The thread's 16 elements are p[e * step], e < n (n < 16 at the tile's
    // edges, 0 outside); a full, contiguous, 16-byte aligned run is read as
    // four float4.
    const float* p;
    int64_t step, n;
    if (kc) {
      const int64_t m = m0 + (tid >> 1), kb = k0 + 16 * (tid & 1);
      p = P + m * sm + kb;
      step = sk;
      n = m < mlim ? std::min<int64_t>(std::max<int64_t>(klim - kb, 0), 16) : 0;
    } else {
      const int64_t k = k0 + (tid & 31), mb = m0 + 16 * (tid >> 5);
      p = P + mb * sm + k * sk;
      step = sm;
      n = k < klim ? std::min<int64_t>(std::max<int64_t>(mlim - mb, 0), 16) : 0;
    }
    if (n == 16 && step == 1 && (reinterpret_cast<uintptr_t>(p) & 15) == 0) {
      const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float4 w = q[e];
        v[4 * e] = w.x;
        v[4 * e + 1] = w.y;
        v[4 * e + 2] = w.z;
        v[4 * e + 3] = w.w;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = e < n ? p[e * step] : 0.f;
    }
  }
  __device__ __forceinline__ void store(float (*T)[GLD], int tid, const float (&v)[16]) const {
    if (kc) {
      float* row = &T[tid >> 1][16 * (tid & 1)];
#pragma unroll
      for (int e = 0; e < 16; e += 4)
        *reinterpret_cast<float4*>(row + e) = make_float4(v[e], v[e + 1], v[e + 2], v[e + 3]);
    } else {
      const int k = tid & 31, mb = 16 * (tid >> 5);
#pragma unroll
      for (int e = 0; e < 16; ++e) T[mb + e][k] = v[e];
    }
  }
};

__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmF32 g) {
  // Two buffers: chunk c + 1 is stored while chunk c is read (one barrier
  // per chunk).
  __shared__ __attribute__((aligned(16))) float As[2][GT][GLD];  // As[.][i][k]
  __shared__ __attribute__((aligned(16))) float Bs[2][GT][GLD];  // Bs[.][j][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int64_t nI = (g.Mr + GT - 1) / GT, nJ = (g.Nc + GT - 1) / GT;
  int64_t ti, tj;
  gemm_tile(blockIdx.x, nJ, nI * nJ, &ti, &tj);
  const int64_t i0 = ti * GT, j0 = tj * GT;
  const int s = blockIdx.y;
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
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const TileStage sa{g.sak == 1}, sb{g.sbk == 1};
  f32x4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int64_t kchunks = ke > kb ? (ke - kb + GK - 1) / GK : 0;
  const int64_t nchunks = (ze - zb) * kchunks;
  float av[16], bv[16];
  auto fetch = [&](int64_t c) {
    const int64_t z = zb + c / kchunks;
    const int64_t k0 = kb + (c % kchunks) * GK;
    sa.load(g.A + z * g.saz, g.sai, g.sak, i0, g.Mr, k0, ke, tid, av);
    sb.load(g.B + z * g.sbz, g.sbj, g.sbk, j0, g.Nc, k0, ke, tid, bv);
  };
  if (nchunks > 0) {
    fetch(0);
    sa.store(As[0], tid, av);
    sb.store(Bs[0], tid, bv);
  }
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const int cb = (int)(c & 1);
    if (c + 1 < nchunks) fetch(c + 1);  // in flight during this chunk's products
#pragma unroll
    for (int kg = 0; kg < GK / 16; ++kg) {
      float4 a[4], b[4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
        a[x] = *reinterpret_cast<const float4*>(&As[cb][wm + 16 * x + lr][16 * kg + 4 * lq]);
#pragma unroll
      for (int y = 0; y < 4; ++y)
        b[y] = *reinterpret_cast<const float4*>(&Bs[cb][wn + 16 * y + lr][16 * kg + 4 * lq]);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
          acc[x][y] = mfma4(a[x].x, b[y].x, acc[x][y]);
          acc[x][y] = mfma4(a[x].y, b[y].y, acc[x][y]);
          acc[x][y] = mfma4(a[x].z, b[y].z, acc[x][y]);
          acc[x][y] = mfma4(a[x].w, b[y].w, acc[x][y]);
        }
    }
    // The other buffer was last read in chunk c - 1, before the barrier
    // that ended it.
    if (c + 1 < nchunks) {
      sa.store(As[cb ^ 1], tid, av);
      sb.store(Bs[cb ^ 1], tid, bv);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wm + 16 * x + 4 * lq + r;
        const int64_t j = j0 + wn + 16 * y + lr;
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

constexpr int kMaxSplit = 64;

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
  const int64_t tiles = ((g.Mr + GT - 1) / GT) * ((g.Nc + GT - 1) / GT);
  hipLaunchKernelGGL(gemm_f32_kernel, dim3((unsigned)tiles, (unsigned)g.S), dim3(256), 0, st, g);
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

// Lane-packed copy of W [4H][D] for the fused forward recurrence, zero-padded
// to Dp columns: Wp[(nt KSD + ks) 64 + l] = W[q H + 16 ut + l % 16][16 ks +
// 4 (l / 16) + s], s = 0..3, nt = q (H / 16) + ut, KSD = Dp / 16.
__global__ void lstm_pack_w_kernel(int H, int D, int Dp, const float* __restrict__ W,
                                   float4* __restrict__ Wp) {
  const int64_t n = (int64_t)H * Dp;  // float4 entries
  const int KSD = Dp / 16;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int l = (int)(e & 63);
    const int64_t tile = e >> 6;
    const int nt = (int)(tile / KSD), ks = (int)(tile % KSD);
    const int q = nt / (H / 16), ut = nt % (H / 16);
    const float* row = W + (int64_t)(q * H + 16 * ut + (l & 15)) * D;
    const int k = 16 * ks + 4 * (l >> 4);
    Wp[e] = make_float4(k < D ? row[k] : 0.f, k + 1 < D ? row[k + 1] : 0.f,
                        k + 2 < D ? row[k + 2] : 0.f, k + 3 < D ? row[k + 3] : 0.f);
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

// out[j] = sum over s of part[s][j], in order.
__global__ void lstm_zero_kernel(float* __restrict__ x, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = 0.f;
}

__global__ void colsum_reduce_kernel(const float* __restrict__ part, int cols, int S,
                                     float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  float v = 0.f;
  for (int s = 0; s < S; ++s) v += part[(int64_t)s * cols + j];
  out[j] = v;
}

// ------------------------------------------------------------ recurrence
// One workgroup per 16 sequences (one MFMA row tile) and one wavefront per
// 16 hidden units: H / 16 waves (4, 8 or 16), so that a SIMD holds several
// waves whose gate arithmetic and loads overlap the others' matrix-core
// work.  Lane l of wave w owns unit 16 w + l % 16 of sequences
// 4 (l / 16) .. + 3: the four result rows of its accumulators.
constexpr int kRows = 16;

// gates [B][L][4H]: on entry W x_t + b, on exit (i, f, g, o); c and h
// [B][L][H]; hks [B][H].
template <int H>
__global__ __launch_bounds__(4 * H) void lstm_fwd_kernel(int64_t Bn, int L,
                                                         const float4* __restrict__ Up,
                                                         const float* __restrict__ hks,
                                                         float* __restrict__ gates,
                                                         float* __restrict__ cs,
                                                         float* __restrict__ hout) {
  constexpr int KS = H / 16;  // k-groups of 16 over h
  constexpr int HS = H + 4;   // LDS row stride (float4-aligned)
  __shared__ __attribute__((aligned(16))) float hs[2][kRows][HS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int u = 16 * wave + lr;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  float hk[4], c[4];
  bool ok[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = r0 + 4 * lq + r;
    ok[r] = row < Bn;
    hk[r] = ok[r] ? hks[row * H + u] : 0.f;
    c[r] = 0.f;
  }
  // Step t + 1's pre-activations are loaded during step t.
  float nx[4][4];
  auto load_pre = [&](int t) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        nx[q][r] = ok[r] ? gates[((r0 + 4 * lq + r) * L + t) * (4 * H) + q * H + u] : 0.f;
  };
  load_pre(0);
  for (int t = 0; t < L; ++t) {
    const int cur = t & 1;
    f32x4 acc[4];  // gates i, f, g, o
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[q][r] = nx[q][r];
    if (t > 0) {
#pragma unroll 4
      for (int ks = 0; ks < KS; ++ks) {
        const float4 a = *reinterpret_cast<const float4*>(&hs[cur][lr][16 * ks + 4 * lq]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 b = Up[((int64_t)(q * (H / 16) + wave) * KS + ks) * 64 + lane];
          acc[q] = mfma4(a.x, b.x, acc[q]);
          acc[q] = mfma4(a.y, b.y, acc[q]);
          acc[q] = mfma4(a.z, b.z, acc[q]);
          acc[q] = mfma4(a.w, b.w, acc[q]);
        }
      }
    }
    // Issued after this step's last load of U: vector-memory loads complete
    // in order, so a prefetch issued earlier would hold up the first use of
    // U; here the gate arithmetic and the barrier cover its latency.
    if (t + 1 < L) load_pre(t + 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float i = sigmoidf(acc[0][r]);
      const float f = sigmoidf(acc[1][r]);
      const float g = tanhf(acc[2][r]);
      const float o = sigmoidf(acc[3][r]);
      const float cn = hk[r] * (f * c[r] + i * g);
      const float h = o * tanhf(cn);
      c[r] = cn;
      hs[cur ^ 1][4 * lq + r][u] = ok[r] ? h : 0.f;
      if (ok[r]) {
        const int64_t rt = (r0 + 4 * lq + r) * L + t;
        float* gp = gates + rt * (4 * H) + u;
        gp[0] = i;
        gp[H] = f;
        gp[2 * H] = g;
        gp[3 * H] = o;
        cs[rt * H + u] = cn;
        hout[rt * H + u] = h;
      }
    }
    __syncthreads();
  }
}

// The forward recurrence with the input products folded in (inputs of at
// most kFusedMaxD features): each step also forms x_t W^T + b on the matrix
// cores, x_t staged in LDS (double-buffered, zero-padded to Dp, a multiple
// of 16) and W read from L2 in the same lane-packed layout as U, so that
// the pre-activations are never written to or read from HBM.  Outputs as
// lstm_fwd_kernel's; `gates` is written only.
constexpr int kFusedMaxD = 256;

template <int H>
__global__ __launch_bounds__(4 * H) void lstm_fwd_fused_kernel(
    int64_t Bn, int L, int D, int Dp, const float* __restrict__ x, const float4* __restrict__ Wp,
    const float* __restrict__ bias, const float4* __restrict__ Up, const float* __restrict__ hks,
    float* __restrict__ gates, float* __restrict__ cs, float* __restrict__ hout) {
  constexpr int KS = H / 16;  // k-groups of 16 over h
  constexpr int HS = H + 4;   // LDS row stride (float4-aligned)
  constexpr int NT = 4 * H;   // threads
  // The 16 x Dp tile of x_t in float4 chunks: chunk c = tid + NT j is row
  // c / (Dp / 4), features 4 (c % (Dp / 4)) .. + 3 (fixed over the steps).
  constexpr int kMaxX = (kRows * kFusedMaxD / 4 + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) float hs[2][kRows][HS];
  extern __shared__ __attribute__((aligned(16))) float xs[];  // [2][kRows][Dp + 4]
  const int XS = Dp + 4, KSD = Dp / 16, QD = Dp / 4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int u = 16 * wave + lr;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  float hk[4], c[4], bq[4];
  bool ok[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = r0 + 4 * lq + r;
    ok[r] = row < Bn;
    hk[r] = ok[r] ? hks[row * H + u] : 0.f;
    c[r] = 0.f;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) bq[q] = bias[q * H + u];
  // Chunk j: its row's x at t = 0 from its first feature, the features in
  // range (0..4; 0 for a row past the batch) and its LDS offset in a buffer
  // (-1: no chunk).
  const float* xp[kMaxX];
  int xl[kMaxX], xn[kMaxX];
#pragma unroll
  for (int j = 0; j < kMaxX; ++j) {
    const int cidx = tid + NT * j;
    const int row = cidx / QD, d = 4 * (cidx % QD);
    const bool in = cidx < kRows * QD && r0 + row < Bn;
    xp[j] = in ? x + (r0 + row) * (int64_t)L * D + d : x;
    xn[j] = in ? min(max(D - d, 0), 4) : 0;
    xl[j] = cidx < kRows * QD ? row * XS + d : -1;
  }
  // rows of x are 16-byte aligned
  const bool vec = (D & 3) == 0 && (reinterpret_cast<uintptr_t>(x) & 15) == 0;
  float4 xv[kMaxX];
  auto load_x = [&](int t) {
#pragma unroll
    for (int j = 0; j < kMaxX; ++j) {
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      const float* p = xp[j] + (int64_t)t * D;
      if (xn[j] == 4 && vec) {
        v = *reinterpret_cast<const float4*>(p);
      } else if (xn[j] > 0) {
        v.x = p[0];
        if (xn[j] > 1) v.y = p[1];
        if (xn[j] > 2) v.z = p[2];
        if (xn[j] > 3) v.w = p[3];
      }
      xv[j] = v;
    }
  };
  auto store_x = [&](int buf) {
#pragma unroll
    for (int j = 0; j < kMaxX; ++j)
      if (xl[j] >= 0) *reinterpret_cast<float4*>(xs + buf * kRows * XS + xl[j]) = xv[j];
  };
  load_x(0);
  store_x(0);
  __syncthreads();
  for (int t = 0; t < L; ++t) {
    const int cur = t & 1;
    f32x4 acc[4];  // gates i, f, g, o
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = f32x4{bq[q], bq[q], bq[q], bq[q]};
    const float* xr = xs + (cur * kRows + lr) * XS + 4 * lq;
#pragma unroll 4
    for (int ks = 0; ks < KSD; ++ks) {
      const float4 a = *reinterpret_cast<const float4*>(xr + 16 * ks);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 b = Wp[((int64_t)(q * (H / 16) + wave) * KSD + ks) * 64 + lane];
        acc[q] = mfma4(a.x, b.x, acc[q]);
        acc[q] = mfma4(a.y, b.y, acc[q]);
        acc[q] = mfma4(a.z, b.z, acc[q]);
        acc[q] = mfma4(a.w, b.w, acc[q]);
      }
    }
    if (t > 0) {
#pragma unroll 4
      for (int ks = 0; ks < KS; ++ks) {
        const float4 a = *reinterpret_cast<const float4*>(&hs[cur][lr][16 * ks + 4 * lq]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 b = Up[((int64_t)(q * (H / 16) + wave) * KS + ks) * 64 + lane];
          acc[q] = mfma4(a.x, b.x, acc[q]);
          acc[q] = mfma4(a.y, b.y, acc[q]);
          acc[q] = mfma4(a.z, b.z, acc[q]);
          acc[q] = mfma4(a.w, b.w, acc[q]);
        }
      }
    }
    // After the step's last load of W and U (loads complete in order).
    if (t + 1 < L) load_x(t + 1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float i = sigmoidf(acc[0][r]);
      const float f = sigmoidf(acc[1][r]);
      const float g = tanhf(acc[2][r]);
      const float o = sigmoidf(acc[3][r]);
      const float cn = hk[r] * (f * c[r] + i * g);
      const float h = o * tanhf(cn);
      c[r] = cn;
      hs[cur ^ 1][4 * lq + r][u] = ok[r] ? h : 0.f;
      if (ok[r]) {
        const int64_t rt = (r0 + 4 * lq + r) * L + t;
        float* gp = gates + rt * (4 * H) + u;
        gp[0] = i;
        gp[H] = f;
        gp[2 * H] = g;
        gp[3 * H] = o;
        cs[rt * H + u] = cn;
        hout[rt * H + u] = h;
      }
    }
    // x tile buffer cur ^ 1 was last read in step t - 1, before its barrier.
    if (t + 1 < L) store_x(cur ^ 1);
    __syncthreads();
  }
}

// gates [B][L][4H]: on entry (i, f, g, o), on exit dz (the gradient with
// respect to the pre-activations); dh [B][L][H] the loss's gradient with
// respect to each h_t; dhks [B][H] out; dbpart [gridDim.x][4H] out: the
// workgroup's column sums of dz (the bias gradient's share).
template <int H>
__global__ __launch_bounds__(4 * H) void lstm_bwd_kernel(int64_t Bn, int L,
                                                         const float4* __restrict__ UpT,
                                                         const float* __restrict__ hks,
                                                         float* __restrict__ gates,
                                                         const float* __restrict__ cs,
                                                         const float* __restrict__ dh,
                                                         float* __restrict__ dhks,
                                                         float* __restrict__ dbpart) {
  constexpr int KT = 4 * H / 16;  // k-groups over the gate columns
  constexpr int GS = 4 * H + 4;
  __shared__ __attribute__((aligned(16))) float dzs[kRows][GS];  // dz_{t+1}
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lq = lane >> 4;
  const int u = 16 * wave + lr;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  float hk[4], dc[4], dk[4], db[4] = {0.f, 0.f, 0.f, 0.f};
  bool ok[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t row = r0 + 4 * lq + r;
    ok[r] = row < Bn;
    hk[r] = ok[r] ? hks[row * H + u] : 0.f;
    dc[r] = 0.f;
    dk[r] = 0.f;
  }
  // Step t's inputs (gate activations, c_{t-1}, dh_t) are loaded during step
  // t + 1; c_t is the previous step's c_{t-1}.
  float gi[4][4], cpn[4], dhn[4], ctv[4];
  auto load_in = [&](int t) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rt = (r0 + 4 * lq + r) * L + t;
#pragma unroll
      for (int q = 0; q < 4; ++q) gi[q][r] = ok[r] ? gates[rt * (4 * H) + q * H + u] : 0.f;
      cpn[r] = (ok[r] && t > 0) ? cs[(rt - 1) * H + u] : 0.f;
      dhn[r] = ok[r] ? dh[rt * H + u] : 0.f;
    }
  };
#pragma unroll
  for (int r = 0; r < 4; ++r) ctv[r] = ok[r] ? cs[((r0 + 4 * lq + r) * L + L - 1) * H + u] : 0.f;
  load_in(L - 1);
  for (int t = L - 1; t >= 0; --t) {
    float iv[4], fv[4], gv[4], ov[4], cpv[4], dhv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      iv[r] = gi[0][r];
      fv[r] = gi[1][r];
      gv[r] = gi[2][r];
      ov[r] = gi[3][r];
      cpv[r] = cpn[r];
      dhv[r] = dhn[r];
    }
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    if (t < L - 1) {
#pragma unroll 4
      for (int ks = 0; ks < KT; ++ks) {
        const float4 a = *reinterpret_cast<const float4*>(&dzs[lr][16 * ks + 4 * lq]);
        const float4 b = UpT[((int64_t)wave * KT + ks) * 64 + lane];
        acc = mfma4(a.x, b.x, acc);
        acc = mfma4(a.y, b.y, acc);
        acc = mfma4(a.z, b.z, acc);
        acc = mfma4(a.w, b.w, acc);
      }
    }
    if (t > 0) load_in(t - 1);  // after the last load of U, as in the forward kernel
    __syncthreads();  // every read of dz_{t+1} is done
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float dzi = 0.f, dzf = 0.f, dzg = 0.f, dzo = 0.f;
      if (ok[r]) {
        const int64_t rt = (r0 + 4 * lq + r) * L + t;
        float* gp = gates + rt * (4 * H) + u;
        const float i = iv[r], f = fv[r], g = gv[r], o = ov[r];
        const float ct = ctv[r];
        const float cp = cpv[r];
        ctv[r] = cp;  // c_{t-1} is the next step's c_t
        const float dht = dhv[r] + acc[r];
        const float tc = tanhf(ct);
        const float dct = dc[r] + dht * o * (1.f - tc * tc);
        const float s = f * cp + i * g;  // c_t = hks s
        dk[r] += dct * s;
        const float ds = dct * hk[r];
        dzi = ds * g * i * (1.f - i);
        dzf = ds * cp * f * (1.f - f);
        dzg = ds * i * (1.f - g * g);
        dzo = dht * tc * o * (1.f - o);
        dc[r] = ds * f;
        gp[0] = dzi;
        gp[H] = dzf;
        gp[2 * H] = dzg;
        gp[3 * H] = dzo;
        db[0] += dzi;
        db[1] += dzf;
        db[2] += dzg;
        db[3] += dzo;
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
  for (int r = 0; r < 4; ++r)
    if (ok[r]) dhks[(r0 + 4 * lq + r) * H + u] = dk[r];
  // Column sums over the workgroup's 16 sequences: lanes lr, lr + 16,
  // lr + 32 and lr + 48 hold the same unit.
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    float v = db[q];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lq == 0) dbpart[(int64_t)blockIdx.x * (4 * H) + q * H + u] = v;
  }
}

// Phase timing (profiling): HIP events recorded between the phases of the
// last forward and backward calls, on their streams.
struct PhaseTimer {
  bool on = false;
  bool made = false;
  bool used[2] = {false, false};
  hipEvent_t ev[2][MDHP_LSTM_BWD_PHASES + 1];
};
PhaseTimer g_timer;

void mark(int pass, int k, hipStream_t st) {
  if (g_timer.on) (void)hipEventRecord(g_timer.ev[pass][k], st);
}

unsigned ew_blocks(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

struct Shape {
  int64_t B;
  int L, D, H, M, Kb, Kf;
  int Dp;  // padded input width of the fused forward recurrence (0: input GEMM)
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
  s->Dp = d->D <= kFusedMaxD ? (d->D + 15) / 16 * 16 : 0;
  return MDHP_OK;
}

// Saved-state layout (floats): gates [B][L][4H], c [B][L][H], hks [B][H],
// feat [B][Kf].
int64_t saved_floats(const Shape& s) {
  return s.B * s.L * 5 * (int64_t)s.H + s.B * (int64_t)s.H + s.B * (int64_t)s.Kf;
}
// Workspace layout (floats): Up [4H H], UpT [4H H], Wp [4H Dp], GEMM
// partials or the bias gradient's per-workgroup sums, dhks [B][H].
int64_t part_floats(const Shape& s) {
  const int64_t big = std::max<int64_t>(4 * (int64_t)s.H * std::max(s.D, s.H),
                                        (int64_t)s.H * s.Kf);
  return std::max<int64_t>(kMaxSplit * big, ((s.B + kRows - 1) / kRows) * 4 * (int64_t)s.H);
}
int64_t pack_floats(const Shape& s) { return 8 * (int64_t)s.H * s.H + 4 * (int64_t)s.H * s.Dp; }
int64_t work_floats(const Shape& s) {
  return pack_floats(s) + part_floats(s) + s.B * (int64_t)s.H;
}

int64_t recurrent_groups(const Shape& s) { return (s.B + kRows - 1) / kRows; }

template <int H>
void launch_fwd(const Shape& s, const float4* Up, const float* hks, float* gates, float* cs,
                float* h, hipStream_t st) {
  hipLaunchKernelGGL(lstm_fwd_kernel<H>, dim3((unsigned)recurrent_groups(s)), dim3(4 * H), 0, st,
                     s.B, s.L, Up, hks, gates, cs, h);
}
template <int H>
void launch_fwd_fused(const Shape& s, const float* x, const float4* Wp, const float* bias,
                      const float4* Up, const float* hks, float* gates, float* cs, float* h,
                      hipStream_t st) {
  const size_t lds = (size_t)2 * kRows * (s.Dp + 4) * sizeof(float);
  hipLaunchKernelGGL(lstm_fwd_fused_kernel<H>, dim3((unsigned)recurrent_groups(s)), dim3(4 * H),
                     lds, st, s.B, s.L, s.D, s.Dp, x, Wp, bias, Up, hks, gates, cs, h);
}
template <int H>
void launch_bwd(const Shape& s, const float4* UpT, const float* hks, float* gates, const float* cs,
                const float* dh, float* dhks, float* dbpart, hipStream_t st) {
  hipLaunchKernelGGL(lstm_bwd_kernel<H>, dim3((unsigned)recurrent_groups(s)), dim3(4 * H), 0, st,
                     s.B, s.L, UpT, hks, gates, cs, dh, dhks, dbpart);
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
  mark(0, 0, st);
  hipLaunchKernelGGL(lstm_features_kernel, dim3(ew_blocks(s.B * s.Kf)), dim3(256), 0, st, s.B,
                     s.M, s.Kb, alpha, beta, T_span, theta, feat);
  hipLaunchKernelGGL(lstm_pack_kernel, dim3(ew_blocks(H * H)), dim3(256), 0, st, s.H, U, Up, UpT);
  mark(0, 1, st);
  // hks = tanh(feat [B][Kf] Whks^T)
  GemmF32 g1{feat, 0, s.Kf, 1, Whks, 0, 1, s.Kf, 1, s.Kf, s.B, H, hks, H,
             nullptr, nullptr, 1, 0, 1};
  hipError_t he = gemm_f32(g1, nullptr, st);
  mark(0, 2, st);
  if (s.Dp) {
    // the input products run inside the recurrence
    if (he != hipSuccess) return mdhp_hip_fail(he, "lstm_forward");
    float4* Wp = UpT + H * H;
    hipLaunchKernelGGL(lstm_pack_w_kernel, dim3(ew_blocks(H * s.Dp)), dim3(256), 0, st, s.H, s.D,
                       s.Dp, W, Wp);
    mark(0, 3, st);
    switch (s.H) {
      case 64: launch_fwd_fused<64>(s, x, Wp, bias, Up, hks, gates, cs, h, st); break;
      case 128: launch_fwd_fused<128>(s, x, Wp, bias, Up, hks, gates, cs, h, st); break;
      default: launch_fwd_fused<256>(s, x, Wp, bias, Up, hks, gates, cs, h, st); break;
    }
  } else {
    // gates = x [BL][D] W^T + b
    GemmF32 g2{x, 0, s.D, 1, W, 0, 1, s.D, 1, s.D, BL, G, gates, G, nullptr, bias, 0, 0, 1};
    if (he == hipSuccess) he = gemm_f32(g2, nullptr, st);
    if (he != hipSuccess) return mdhp_hip_fail(he, "lstm_forward");
    mark(0, 3, st);
    switch (s.H) {
      case 64: launch_fwd<64>(s, Up, hks, gates, cs, h, st); break;
      case 128: launch_fwd<128>(s, Up, hks, gates, cs, h, st); break;
      default: launch_fwd<256>(s, Up, hks, gates, cs, h, st); break;
    }
  }
  mark(0, 4, st);
  if (g_timer.on) g_timer.used[0] = true;
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
  float* part = work + pack_floats(s);
  float* dpre = part + part_floats(s);
  mark(1, 0, st);
  if (s.B > 0)
    hipLaunchKernelGGL(lstm_pack_kernel, dim3(ew_blocks(H * H)), dim3(256), 0, st, s.H, U, Up,
                       UpT);
  mark(1, 1, st);
  if (s.B > 0) {
    switch (s.H) {
      case 64: launch_bwd<64>(s, UpT, hks, dz, cs, dh, dpre, part, st); break;
      case 128: launch_bwd<128>(s, UpT, hks, dz, cs, dh, dpre, part, st); break;
      default: launch_bwd<256>(s, UpT, hks, dz, cs, dh, dpre, part, st); break;
    }
  }
  // db = sum of the workgroups' column sums, while they are in the workspace
  const int nG = (int)recurrent_groups(s);
  if (nG > 0)
    hipLaunchKernelGGL(colsum_reduce_kernel, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, st,
                       part, (int)G, nG, dbias);
  else
    hipLaunchKernelGGL(lstm_zero_kernel, dim3((unsigned)((G + 255) / 256)), dim3(256), 0, st,
                       dbias, G);
  mark(1, 2, st);
  hipError_t he = hipGetLastError();
  // dx [BL][D] = dZ [BL][4H] W [4H][D]
  if (he == hipSuccess)
    he = gemm_f32(GemmF32{dz, 0, G, 1, W, 0, s.D, 1, 1, G, BL, s.D, dx, s.D, nullptr, nullptr,
                          0, 0, 1},
                  nullptr, st);
  mark(1, 3, st);
  // dW [4H][D] = dZ^T X
  if (he == hipSuccess)
    he = gemm_f32(GemmF32{dz, 0, 1, G, x, 0, s.D, 1, 1, BL, G, s.D, dW, s.D, nullptr, nullptr,
                          0, 0, 1},
                  part, st);
  mark(1, 4, st);
  // dU [4H][H] = sum over sequences b and steps t >= 1 of dz[b][t]^T h[b][t-1]
  if (he == hipSuccess)
    he = gemm_f32(GemmF32{dz + G, (int64_t)s.L * G, 1, G, h, (int64_t)s.L * H, H, 1, s.B,
                          s.L - 1, G, H, dU, H, nullptr, nullptr, 0, 0, 1},
                  part, st);
  mark(1, 5, st);
  if (s.B > 0)
    hipLaunchKernelGGL(lstm_dpre_kernel, dim3(ew_blocks(s.B * H)), dim3(256), 0, st, s.B * H, hks,
                       dpre);
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
  mark(1, 6, st);
  if (g_timer.on) g_timer.used[1] = true;
  he = hipGetLastError();
  return he == hipSuccess ? MDHP_OK : mdhp_hip_fail(he, "lstm_backward");
}

mdhp_status mdhp_lstm_timing(int32_t enable) {
  if (enable && !g_timer.made) {
    for (auto& pass : g_timer.ev)
      for (hipEvent_t& e : pass) {
        const hipError_t he = hipEventCreate(&e);
        if (he != hipSuccess) return mdhp_hip_fail(he, "lstm_timing");
      }
    g_timer.made = true;
  }
  g_timer.on = enable != 0;
  g_timer.used[0] = g_timer.used[1] = false;
  return MDHP_OK;
}

mdhp_status mdhp_lstm_phase_ms(float* fwd_ms, float* bwd_ms) {
  if (!g_timer.made) return mdhp_fail(MDHP_E_INVAL, "lstm_phase_ms: timing was never enabled");
  const int n[2] = {MDHP_LSTM_FWD_PHASES, MDHP_LSTM_BWD_PHASES};
  float* out[2] = {fwd_ms, bwd_ms};
  for (int p = 0; p < 2; ++p) {
    if (!out[p]) continue;
    if (!g_timer.used[p]) {
      for (int k = 0; k < n[p]; ++k) out[p][k] = -1.f;
      continue;
    }
    hipError_t he = hipEventSynchronize(g_timer.ev[p][n[p]]);
    for (int k = 0; he == hipSuccess && k < n[p]; ++k)
      he = hipEventElapsedTime(&out[p][k], g_timer.ev[p][k], g_timer.ev[p][k + 1]);
    if (he != hipSuccess) return mdhp_hip_fail(he, "lstm_phase_ms");
  }
  return MDHP_OK;
}

}  // extern "C"
