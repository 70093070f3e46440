// Shared-decay likelihood, gradient and persistent fits for M <= 16 with one
// chunk of events per lane ("lane per chunk").
//
// Each wavefront owns one window at a time.  The window's N events are cut
// into 64 contiguous chunks of c = ceil(N / 64) events, one per lane, and the
// plan stores them lane-major: event j of lane l's chunk sits at slot
// begin + 64 j + l (padding slots: gap 0, dimension 0xFF), so every step of
// the 64 lanes reads 64 consecutive gaps and dimension bytes.
//
// Every lane keeps the whole decay state of its chunk in registers: R_n, S_n
// and the pending counts P_n for n < MP (MP = M rounded up to 4, 8 or 16),
//   R_n(i) = sum_{k: d_k = n, t_k < t_i} e^{-beta (t_i - t_k)}      (Part1's inner sum, Eq. (5))
//   S_n(i) = sum_{k: d_k = n, t_k < t_i} (t_i - t_k) e^{-beta (t_i - t_k)}   (= -dR/dbeta)
// and applies the exponential-kernel recursion R <- a (R + P), S <- a S + dt R,
// a = e^{-beta dt}, where P holds the events at the previous time (folded in
// only when time moves on, so equal times never excite each other).  No
// lane waits for another.  The chunk carries (zero-start end state, product
// of decays A, summed gaps delta, "has a positive gap" flag) are combined
// across lanes by an inclusive scan (DPP row shifts, then row broadcasts);
// its exclusive form gives every lane the exact start state of its chunk,
// and a second pass over the chunk evaluates
//   lambda_i = mu_m + sum_n alpha_mn R_n(i),   m = d_i           (Eq. (2) at t_i)
//   ll += log lambda_i,  G_R[m][n] += R_n(i) / lambda_i,  Gmu[m] += 1 / lambda_i,
//   Gb += sum_n alpha_mn S_n(i) / lambda_i.
// G_R is a sum of one outer product per event, e_{d_i} (R(i) / lambda_i)^T;
// over a step of 64 events that is a 16 x 64 by 64 x M matrix product, run on
// the matrix cores (v_mfma_f32_16x16x4_f32) from a column-major LDS staging of
// the step (LDS float atomics, one per event and component, are ~6x slower
// than the whole rest of the pass on gfx950).  Gmu and Gb are per-lane sums;
// the per-dimension counts N_m come with the plan.  The compensator (Part2 +
// Part3, Appendix B) comes from the window's end state advanced to T:
//   E_n = sum_{k: d_k = n} e^{-beta (T - t_k)},  F_n = sum (T - t_k) e^{-beta (T - t_k)}.
// The fits run per wave with wave-level reductions: no workgroup barriers.

#include "mdhp_device.h"

namespace mdhp {

namespace {

constexpr int kWaves = kBlock / 64;  // wavefronts per workgroup
constexpr int kPad = 0xFF;           // dimension byte of a padding slot
constexpr int kSpan = 16;            // steps (64 events each) per FP32 accumulation span

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int MP>
struct alignas(16) LpcWave {
  static constexpr int Q = MP + 1;  // row stride of gR64: G_R[m][0..MP-1], Gmu[m]
  float alpha[MP * MP];             // [m * MP + n], zero outside M x M
  float mu[MP];                     // zero outside M
  float colsum[MP];                 // sum_m alpha_mn
  float vst[MP * 64];               // step staging, column-major: w_k R_n(k) at [n * 64 + k]
  float hot[16 * 64];               // one-hot of the step's targets: 1 at [d_k * 64 + k], else 0
  float gmu[64 * Q];                // per-lane sums of w over the lane's events of target m: [lane * Q + m]
  double gR64[MP * Q];              // window sums (FP64 over spans): G_R, Gmu in column MP
  double En[MP], Fn[MP];            // E_n, F_n
  double Cn[MP];                    // (N_n - E_n) / beta
  double scal[2];                   // ll, d ll / d beta
  float beta;
};

template <class F>
__device__ __forceinline__ F wave_sum(F v) {
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) v += __shfl_xor(v, k, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) v = fmax(v, __shfl_xor(v, k, 64));
  return v;
}

// Orders the wave's earlier LDS accesses before its later ones, across lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// v of lane 15 of the previous 16-lane row for the lanes of rows 1 and 3
// (DPP row_bcast:15); the other lanes get 0.
__device__ __forceinline__ float bcast15(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                0x142, 0xA, 0xF, false));
}

// v of lane 31 for the lanes of rows 2 and 3 (DPP row_bcast:31); the other
// lanes get 0.
__device__ __forceinline__ float bcast31(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                0x143, 0xC, 0xF, false));
}

// Chunk carry of one lane: the state a zero start reaches at the end of the
// chunk, the product of its decays A, the sum of its gaps D, and F = 1 if a
// gap is positive (then the pending counts of the start are folded in).
template <int MP>
struct Carry {
  float R[MP], S[MP], P[MP];
  float A, D, F;
};

// One scan step: where `take`, the carry becomes (segment read through
// SHIFT) followed by the lane's own segment.
template <int MP, class SHIFT>
__device__ __forceinline__ void scan_step(Carry<MP>& b, bool take, SHIFT shift) {
  const float aA = shift(b.A), aD = shift(b.D), aF = shift(b.F);
  const bool f = b.F != 0.f;
#pragma unroll
  for (int m = 0; m < MP; ++m) {
    const float aR = shift(b.R[m]), aS = shift(b.S[m]), aP = shift(b.P[m]);
    const float X = aR + aP;
    const float r = f ? fmaf(b.A, X, b.R[m]) : aR;
    const float s = f ? fmaf(b.A, fmaf(b.D, X, aS), b.S[m]) : aS;
    const float p = f ? b.P[m] : aP + b.P[m];
    b.R[m] = take ? r : b.R[m];
    b.S[m] = take ? s : b.S[m];
    b.P[m] = take ? p : b.P[m];
  }
  b.A = take ? b.A * aA : b.A;
  b.D = take ? b.D + aD : b.D;
  b.F = take ? fmaxf(b.F, aF) : b.F;
}

// Inclusive scan of the lanes' carries in lane order.
template <int MP>
__device__ __forceinline__ void scan_carries(Carry<MP>& c, int lane) {
  const int lr = lane & 15;
  scan_step<MP>(c, lr >= 1, [](float v) { return row_shr<1>(v); });
  scan_step<MP>(c, lr >= 2, [](float v) { return row_shr<2>(v); });
  scan_step<MP>(c, lr >= 4, [](float v) { return row_shr<4>(v); });
  scan_step<MP>(c, lr >= 8, [](float v) { return row_shr<8>(v); });
  scan_step<MP>(c, (lane & 16) != 0, [](float v) { return bcast15(v); });
  scan_step<MP>(c, lane >= 32, [](float v) { return bcast31(v); });
}

// G_R over one step: the 64 events' rows w_k R(k) (staged column-major in
// vst) summed by target, G_R[m][n] += sum_k [d_k = m] w_k R_n(k), as the
// product H^T V of the step's one-hot targets H (64 x 16) and V (64 x MP):
// sixteen v_mfma_f32_16x16x4_f32 with K running over the events.  Lane l
// supplies A = H[16q + s][l % 16] and B = V[16q + s][l % 16] (q = l / 16) for
// instruction s, and holds G_R[4q + r][l % 16] in acc[r].
template <int MP>
__device__ __forceinline__ void step_outer(const LpcWave<MP>& sh, f32x4& acc) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, base = (lane >> 4) * 16;
  f32x4 a[4], b[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    a[i] = *reinterpret_cast<const f32x4*>(&sh.hot[col * 64 + base + 4 * i]);
    b[i] = col < MP ? *reinterpret_cast<const f32x4*>(&sh.vst[(col % MP) * 64 + base + 4 * i])
                    : f32x4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][e], b[i][e], acc, 0, 0, 0);
}

// Adds the FP32 span sums of G_R (MFMA accumulators) into the FP64 window
// sums and clears them.
template <int MP>
__device__ __forceinline__ void flush_span(LpcWave<MP>& sh, f32x4& acc) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, row0 = (lane >> 4) * 4;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (row0 + r < MP && col < MP) sh.gR64[(row0 + r) * LpcWave<MP>::Q + col] += (double)acc[r];
    acc[r] = 0.f;
  }
}

// Evaluates the wave's window with the parameters in its LDS slot (alpha,
// mu, colsum, beta; sums cleared; counts = the window's N_m).  On return
// (all lanes): scal[0] = ll; with GRAD also gR64 (G_R and, in column MP,
// Gmu), Cn, Fn and scal[1] = d ll / d beta.
// Per-lane and LDS sums run in FP32 over spans of kSpan steps and are
// accumulated in FP64 across spans.
template <int MP, bool GRAD>
__device__ __forceinline__ void lpc_eval(LpcWave<MP>& sh, const float* __restrict__ dtg,
                                         const uint8_t* __restrict__ dg, int64_t begin, int n,
                                         double T, float end_gap, const int32_t* counts, int M) {
  constexpr int Q = LpcWave<MP>::Q;
  const int lane = threadIdx.x & 63;
  const float beta = sh.beta;
  const int c = (n + 63) / 64;
  const float* __restrict__ dtw = dtg + begin + lane;
  const uint8_t* __restrict__ dw = dg + begin + lane;

  // Pass 1: the chunk's carry from a zero start.  The lane runs the
  // inclusive state Rin = R + P (events at or before the current time):
  //   Rin <- a Rin + e_d,   S <- a (S + dt Rin),
  // which needs no case for equal times because a = 1 exactly when dt = 0.
  Carry<MP> cr;
  float Rin[MP];
#pragma unroll
  for (int m = 0; m < MP; ++m) Rin[m] = cr.S[m] = 0.f;
  cr.A = 1.f;
  cr.D = 0.f;
  {
    float dt_n = c > 0 ? dtw[0] : 0.f;
    int d_n = c > 0 ? (int)dw[0] : kPad;
    for (int j = 0; j < c; ++j) {
      const float dt = dt_n;
      const int d = d_n;
      if (j + 1 < c) {
        dt_n = dtw[(int64_t)(j + 1) * 64];
        d_n = dw[(int64_t)(j + 1) * 64];
      }
      const float a = dt > 0.f ? __expf(-beta * dt) : 1.f;
#pragma unroll
      for (int m = 0; m < MP; ++m) {
        cr.S[m] = a * fmaf(dt, Rin[m], cr.S[m]);
        Rin[m] = fmaf(a, Rin[m], m == d ? 1.f : 0.f);
      }
      cr.A *= a;
      cr.D += dt;
    }
  }
  // Pending counts at the chunk's end: the events after its last positive
  // gap (all of them if it has none); R = Rin - P.
  {
#pragma unroll
    for (int m = 0; m < MP; ++m) cr.P[m] = 0.f;
    const int len = min(max(n - lane * c, 0), c);
    for (int j = len - 1; j >= 0; --j) {
      const int d = dw[(int64_t)j * 64];
#pragma unroll
      for (int m = 0; m < MP; ++m) cr.P[m] += m == d ? 1.f : 0.f;
      if (dtw[(int64_t)j * 64] > 0.f) break;
    }
#pragma unroll
    for (int m = 0; m < MP; ++m) cr.R[m] = Rin[m] - cr.P[m];
  }
  cr.F = cr.D > 0.f ? 1.f : 0.f;
  scan_carries<MP>(cr, lane);
  // Lane 63 now holds the window's end state: E_n and F_n at T.
  if (lane == 63) {
    const double gap = (double)end_gap;
    const double ea = exp(-(double)beta * gap);
#pragma unroll
    for (int m = 0; m < MP; ++m) {
      const double E = ea * ((double)cr.R[m] + (double)cr.P[m]);
      sh.En[m] = E;
      sh.Fn[m] = ea * (double)cr.S[m] + gap * E;
    }
  }
  // Exclusive form: lane l starts from the state after chunks 0 .. l-1
  // (strict R, inclusive Rin = R + P, S).
  float R[MP], S[MP];
#pragma unroll
  for (int m = 0; m < MP; ++m) {
    const float pR = __shfl_up(cr.R[m], 1, 64), pS = __shfl_up(cr.S[m], 1, 64);
    const float pP = __shfl_up(cr.P[m], 1, 64);
    R[m] = lane == 0 ? 0.f : pR;
    S[m] = lane == 0 ? 0.f : pS;
    Rin[m] = lane == 0 ? 0.f : pR + pP;
  }
  // Pass 2: intensities, log-likelihood and gradient sums.  At an event
  // with dt > 0 the strict state is R = a Rin; at an equal time it stays.
  float llp = 0.f, gbp = 0.f;
  double ll64 = 0.0, gb64 = 0.0;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  {
    float dt_n = c > 0 ? dtw[0] : 0.f;
    int d_n = c > 0 ? (int)dw[0] : kPad;
    for (int j = 0; j < c; ++j) {
      const float dt = dt_n;
      const int dr = d_n;
      if (j + 1 < c) {
        dt_n = dtw[(int64_t)(j + 1) * 64];
        d_n = dw[(int64_t)(j + 1) * 64];
      }
      const bool v = dr != kPad;
      const int d = v ? dr : 0;
      const bool f = dt > 0.f;
      const float a = f ? __expf(-beta * dt) : 1.f;
      const float* arow = &sh.alpha[d * MP];
      float lam = sh.mu[d], asum = 0.f;
#pragma unroll
      for (int m = 0; m < MP; ++m) {
        const float t = a * Rin[m];
        S[m] = a * fmaf(dt, Rin[m], S[m]);
        R[m] = f ? t : R[m];
        Rin[m] = t + (m == dr ? 1.f : 0.f);
        const float al = arow[m];
        lam = fmaf(al, R[m], lam);
        asum = fmaf(al, S[m], asum);
      }
      if (v) llp += __logf(lam);
      if constexpr (GRAD) {
        // Padding events stage w = 0 (their one-hot row is 0, target 0).
        const float w = v ? __builtin_amdgcn_rcpf(lam) : 0.f;
        gbp = fmaf(w, asum, gbp);
        sh.gmu[lane * Q + d] += w;  // the lane's own row: no other lane writes it
#pragma unroll
        for (int m = 0; m < MP; ++m) sh.vst[m * 64 + lane] = w * R[m];
        sh.hot[d * 64 + lane] = 1.f;
        wave_sync();
        step_outer(sh, acc);
        wave_sync();
        sh.hot[d * 64 + lane] = 0.f;
      }
      if (j % kSpan == kSpan - 1 || j + 1 == c) {
        ll64 += (double)llp;
        gb64 += (double)gbp;
        llp = gbp = 0.f;
        if constexpr (GRAD) flush_span(sh, acc);
      }
    }
  }
  wave_sync();
  if constexpr (GRAD) {  // Gmu[m]: the lanes' sums, in FP64
    if (lane < MP) {
      double g[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 16
      for (int l = 0; l < 64; ++l) g[l & 3] += (double)sh.gmu[l * Q + lane];
      sh.gR64[lane * Q + MP] = (g[0] + g[1]) + (g[2] + g[3]);
    }
    wave_sync();
  }
  // Compensator: lane m < M finishes source dimension m; one FP64 wave sum
  // each for ll and d ll / d beta.
  const double b = (double)beta;
  double x = ll64, y = gb64;
  if (lane < M) {
    const double C = ((double)counts[lane] - sh.En[lane]) / b;
    const double cs = (double)sh.colsum[lane];
    x -= T * (double)sh.mu[lane] + cs * C;
    y += cs * (sh.Fn[lane] - C) / b;
    sh.Cn[lane] = C;
  } else if (lane < MP) {
    sh.Cn[lane] = 0.0;
  }
  x = wave_sum(x);
  y = wave_sum(y);
  if (lane == 0) {
    sh.scal[0] = x;
    sh.scal[1] = -y;
  }
  wave_sync();
}

template <int MP>
__device__ __forceinline__ void lpc_colsum(LpcWave<MP>& sh, int M) {
  const int lane = threadIdx.x & 63;
  wave_sync();
  if (lane < MP) {
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += sh.alpha[m * MP + lane];
    sh.colsum[lane] = s;
  }
  wave_sync();
}

template <int MP>
__device__ __forceinline__ void lpc_load(LpcWave<MP>& sh, const float* __restrict__ mu,
                                         const float* __restrict__ alpha,
                                         const float* __restrict__ beta, int64_t w, int M) {
  const int lane = threadIdx.x & 63;
  wave_sync();
  for (int e = lane; e < MP * MP; e += 64) {
    const int m = e / MP, n = e % MP;
    sh.alpha[e] = (m < M && n < M) ? alpha[(w * M + m) * M + n] : 0.f;
  }
  if (lane < MP) sh.mu[lane] = lane < M ? mu[w * M + lane] : 0.f;
  if (lane == 0) sh.beta = beta[w];
  lpc_colsum(sh, M);
}

// Clears the gradient sums of the wave's slot.
template <int MP>
__device__ __forceinline__ void lpc_zero(LpcWave<MP>& sh) {
  const int lane = threadIdx.x & 63;
  wave_sync();
  for (int e = lane; e < 64 * LpcWave<MP>::Q; e += 64) sh.gmu[e] = 0.f;
  for (int e = lane; e < MP * LpcWave<MP>::Q; e += 64) sh.gR64[e] = 0.0;
  wave_sync();
}

// Clears the wave's one-hot staging (kept zero between steps).
template <int MP>
__device__ __forceinline__ void lpc_init(LpcWave<MP>& sh) {
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < 16 * 64; e += 64) sh.hot[e] = 0.f;
  wave_sync();
}

// Next queue position of the wave: the first is fixed by the wave's place
// in the grid, the rest come from the atomic queue head.
__device__ __forceinline__ int lpc_next(int* counter, bool first) {
  const int lane = threadIdx.x & 63;
  int q = 0;
  if (lane == 0)
    q = first ? (int)(blockIdx.x * kWaves + (threadIdx.x >> 6))
              : atomicAdd(counter, 1) + (int)(gridDim.x * kWaves);
  return __shfl(q, 0, 64);
}

template <int MP, bool GRAD>
__global__ __launch_bounds__(kBlock) void lpc_eval_kernel(Events ev, int M, const float* mu,
                                                          const float* alpha, const float* beta,
                                                          double* ll, float* g_mu,
                                                          float* g_alpha, float* g_beta,
                                                          int* counter) {
  __shared__ LpcWave<MP> slots[kWaves];
  LpcWave<MP>& sh = slots[threadIdx.x >> 6];
  lpc_init(sh);
  constexpr int Q = LpcWave<MP>::Q;
  const int lane = threadIdx.x & 63;
  for (int q = lpc_next(counter, true); q < ev.W; q = lpc_next(counter, false)) {
    const int64_t w = ev.order[q];
    lpc_zero(sh);
    lpc_load(sh, mu, alpha, beta, w, M);
    const double T = ev.T[w];
    lpc_eval<MP, GRAD>(sh, ev.dt, ev.d, ev.begin[w], ev.n[w], T, ev.end_gap[w],
                       ev.counts + w * M, M);
    if (lane == 0) ll[w] = sh.scal[0];
    if constexpr (GRAD) {
      if (lane == 0) g_beta[w] = (float)sh.scal[1];
      if (lane < M) g_mu[w * M + lane] = (float)(sh.gR64[lane * Q + MP] - T);
      for (int e = lane; e < M * M; e += 64) {
        const int m = e / M, k = e % M;
        g_alpha[w * M * M + e] = (float)(sh.gR64[m * Q + k] - sh.Cn[k]);
      }
    }
  }
}

// Slot layout of the per-wave fits: lane l owns the alpha entries
// e = l + 64 k (k < OWN, e = m * MP + n) and one extra slot k = OWN holding
// mu_l (l < M) or beta (l == M).  Kinds: 0 none, 1 alpha, 2 mu, 3 beta.
template <int MP>
struct Slots {
  static constexpr int OWN = (MP * MP + 63) / 64;
  static constexpr int K = OWN + 1;
  int M, lane, fix_beta;
  __device__ int kind(int k) const {
    if (k < OWN) {
      const int e = lane + k * 64;
      return (e < MP * MP && e / MP < M && e % MP < M) ? 1 : 0;
    }
    if (lane < M) return 2;
    if (lane == M) return fix_beta ? 0 : 3;
    return 0;
  }
  __device__ float get(const LpcWave<MP>& sh, int k) const {
    const int kd = kind(k);
    if (kd == 1) return sh.alpha[lane + k * 64];
    if (kd == 2) return sh.mu[lane];
    if (kd == 3) return sh.beta;
    return 0.f;
  }
  __device__ void set(LpcWave<MP>& sh, int k, float v) const {
    const int kd = kind(k);
    if (kd == 1) sh.alpha[lane + k * 64] = v;
    else if (kd == 2) sh.mu[lane] = v;
    else if (kd == 3) sh.beta = v;
  }
  // d ll / d theta of slot k after an evaluation with gradient.
  __device__ double grad(const LpcWave<MP>& sh, int k, double T) const {
    const int kd = kind(k);
    if (kd == 1) {
      const int e = lane + k * 64;
      return sh.gR64[(e / MP) * LpcWave<MP>::Q + e % MP] - sh.Cn[e % MP];
    }
    if (kd == 2) return sh.gR64[lane * LpcWave<MP>::Q + MP] - T;
    if (kd == 3) return sh.scal[1];
    return 0.0;
  }
};

template <int MP>
__device__ __forceinline__ void lpc_store(const LpcWave<MP>& sh, int64_t w, int M, float* mu,
                                          float* alpha, float* beta) {
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < M * M; e += 64) alpha[w * M * M + e] = sh.alpha[(e / M) * MP + e % M];
  if (lane < M) mu[w * M + lane] = sh.mu[lane];
  if (lane == 0) beta[w] = sh.beta;
}

// Persistent projected gradient ascent / projected Adam, one window per wave
// (the rule of the workgroup kernel: evaluate, stop on a non-finite value,
// on |delta ll| <= ll_tol max(|ll|, 1) or after max_steps updates, else step
// along the gradient divided by N and project).
template <int MP>
__global__ __launch_bounds__(kBlock) void lpc_fit_kernel(Events ev, int M, FitParams o,
                                                         float* mu, float* alpha, float* beta,
                                                         double* ll, int* steps, int* status,
                                                         int* evals_out, int* counter) {
  __shared__ LpcWave<MP> slots[kWaves];
  LpcWave<MP>& sh = slots[threadIdx.x >> 6];
  lpc_init(sh);
  constexpr int K = Slots<MP>::K;
  const int lane = threadIdx.x & 63;
  const Slots<MP> sl{M, lane, o.fix_beta};
  for (int q = lpc_next(counter, true); q < ev.W; q = lpc_next(counter, false)) {
    const int64_t w = ev.order[q];
    lpc_load(sh, mu, alpha, beta, w, M);
    const int n = ev.n[w];
    const double T = ev.T[w];
    const double rate = (double)max(n, 1) / T;
    const double mu_min = o.mu_floor_rel * rate;
    const double beta_min = o.beta_floor_rel * rate;
    const double inv_n = 1.0 / (double)max(n, 1);
    float m1[K], m2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) m1[k] = m2[k] = 0.f;
    double ll_prev = 0.0, b1t = 1.0, b2t = 1.0;
    int s = 0, st = MDHP_FIT_MAX_STEPS;
    for (s = 0;; ++s) {
      lpc_zero(sh);
      lpc_eval<MP, true>(sh, ev.dt, ev.d, ev.begin[w], n, T, ev.end_gap[w], ev.counts + w * M,
                         M);
      const double l = sh.scal[0];
      double g[K];
      bool bad = !isfinite(l) || !isfinite(sh.scal[1]);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        g[k] = sl.grad(sh, k, T);
        if (!isfinite(g[k])) bad = true;
      }
      if (__any(bad)) {
        st = MDHP_FIT_NONFINITE;
        break;
      }
      if (s >= 1 && fabs(l - ll_prev) <= o.ll_tol * fmax(fabs(l), 1.0)) {
        st = MDHP_FIT_CONVERGED;
        break;
      }
      if (s == o.max_steps) {
        st = MDHP_FIT_MAX_STEPS;
        break;
      }
      ll_prev = l;
      b1t *= o.b1;
      b2t *= o.b2;
      const double bc1 = 1.0 - b1t, bc2 = 1.0 - b2t;
      wave_sync();
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int kd = sl.kind(k);
        if (kd == 0) continue;
        const double gn = g[k] * inv_n;
        double step;
        if (o.optimizer == MDHP_OPT_PGD) {
          step = o.lr * gn;
        } else {
          const double nm1 = o.b1 * (double)m1[k] + (1.0 - o.b1) * gn;
          const double nm2 = o.b2 * (double)m2[k] + (1.0 - o.b2) * gn * gn;
          m1[k] = (float)nm1;
          m2[k] = (float)nm2;
          step = o.lr * (nm1 / bc1) / (sqrt(nm2 / bc2) + o.eps);
        }
        const double lo = kd == 2 ? mu_min : (kd == 3 ? beta_min : 0.0);
        sl.set(sh, k, (float)fmax((double)sl.get(sh, k) + step, lo));
      }
      lpc_colsum(sh, M);
    }
    // The parameters of the last evaluation are in LDS.
    lpc_store(sh, w, M, mu, alpha, beta);
    if (lane == 0) {
      ll[w] = sh.scal[0];
      steps[w] = s;
      status[w] = st;
      if (evals_out) evals_out[w] = s + 1;
    }
  }
}

// Workspace floats of one wave of the L-BFGS fit: X, G, D, XN, then the
// S and Y rings; K slots of 64 lanes each.
template <int MP>
constexpr int64_t lpc_ws_per_wave() {
  return (int64_t)(4 + 2 * kMaxHistory) * Slots<MP>::K * 64;
}

// Persistent projected L-BFGS, one window per wave: the rule of the
// workgroup kernel (two-loop recursion on the free set, Armijo backtracking
// on the projected path, curvature-checked history, restart from scaled
// steepest descent) with wave-level reductions.
template <int MP>
__global__ __launch_bounds__(kBlock) void lpc_lbfgs_kernel(Events ev, int M, FitParams o,
                                                           float* mu, float* alpha, float* beta,
                                                           double* ll, int* steps, int* status,
                                                           int* evals_out, float* ws,
                                                           int* counter) {
  __shared__ LpcWave<MP> slots[kWaves];
  __shared__ double rho_s[kWaves][kMaxHistory], a_s[kWaves][kMaxHistory];
  const int wave = threadIdx.x >> 6;
  LpcWave<MP>& sh = slots[wave];
  lpc_init(sh);
  constexpr int K = Slots<MP>::K;
  const int lane = threadIdx.x & 63;
  const int m_hist = o.history;
  const Slots<MP> sl{M, lane, o.fix_beta};
  float* base = ws + (size_t)(blockIdx.x * kWaves + wave) * (size_t)lpc_ws_per_wave<MP>();
  auto X = [&](int k) -> float& { return base[(0 * K + k) * 64 + lane]; };
  auto Gv = [&](int k) -> float& { return base[(1 * K + k) * 64 + lane]; };
  auto Dv = [&](int k) -> float& { return base[(2 * K + k) * 64 + lane]; };
  auto XN = [&](int k) -> float& { return base[(3 * K + k) * 64 + lane]; };
  auto Sv = [&](int j, int k) -> float& { return base[((4 + j) * K + k) * 64 + lane]; };
  auto Yv = [&](int j, int k) -> float& {
    return base[((4 + kMaxHistory + j) * K + k) * 64 + lane];
  };
  for (int q = lpc_next(counter, true); q < ev.W; q = lpc_next(counter, false)) {
    const int64_t w = ev.order[q];
    lpc_load(sh, mu, alpha, beta, w, M);
    const int n = ev.n[w];
    const double T = ev.T[w];
    const double rate = (double)max(n, 1) / T;
    const float mu_min = (float)(o.mu_floor_rel * rate);
    const float beta_min = (float)(o.beta_floor_rel * rate);
    const double inv_n = 1.0 / (double)max(n, 1);
    auto lower = [&](int k) -> float {
      const int kd = sl.kind(k);
      return kd == 2 ? mu_min : (kd == 3 ? beta_min : 0.f);
    };
    // Gradient of f = -ll / N per slot; false if ll or any entry is not finite.
    double gf[K];
    auto evaluate = [&]() -> bool {
      lpc_zero(sh);
      lpc_eval<MP, true>(sh, ev.dt, ev.d, ev.begin[w], n, T, ev.end_gap[w], ev.counts + w * M,
                         M);
      bool bad = !isfinite(sh.scal[0]) || !isfinite(sh.scal[1]);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        gf[k] = -sl.grad(sh, k, T) * inv_n;
        if (!isfinite(gf[k])) bad = true;
      }
      return !__any(bad);
    };
    int nev = 1, st = MDHP_FIT_MAX_STEPS, s = 0, h = 0, head = 0;
    double l = 0.0, sy_new = 0.0, yy_new = 0.0;
    if (!evaluate()) {
      st = MDHP_FIT_NONFINITE;
      l = sh.scal[0];
    } else {
      l = sh.scal[0];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        X(k) = sl.get(sh, k);
        Gv(k) = (float)gf[k];
      }
      double f = -l * inv_n;
      for (s = 0;; ++s) {
        if (s == o.max_steps) {
          st = MDHP_FIT_MAX_STEPS;
          break;
        }
        // Free gradient and its largest entry.
        double qv[K], gmax_l = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float g = Gv(k);
          const bool active = sl.kind(k) == 0 || (X(k) <= lower(k) && g > 0.f);
          qv[k] = active ? 0.0 : (double)g;
          gmax_l = fmax(gmax_l, fabs(qv[k]));
        }
        const double gmax = wave_max(gmax_l);
        if (gmax == 0.0) {
          st = MDHP_FIT_CONVERGED;
          break;
        }
        const double gamma0 = 0.01 / gmax;
        for (int i = 0; i < h; ++i) {
          const int j = (head - 1 - i + kMaxHistory) % kMaxHistory;
          double v = 0.0;
#pragma unroll
          for (int k = 0; k < K; ++k) v += (double)Sv(j, k) * qv[k];
          const double a = rho_s[wave][j] * wave_sum(v);
          a_s[wave][j] = a;  // every lane writes the same value
#pragma unroll
          for (int k = 0; k < K; ++k) qv[k] -= a * (double)Yv(j, k);
        }
        const double gamma = h > 0 ? sy_new / yy_new : gamma0;
#pragma unroll
        for (int k = 0; k < K; ++k) qv[k] *= gamma;
        for (int i = h - 1; i >= 0; --i) {
          const int j = (head - 1 - i + kMaxHistory) % kMaxHistory;
          double v = 0.0;
#pragma unroll
          for (int k = 0; k < K; ++k) v += (double)Yv(j, k) * qv[k];
          const double bcoef = rho_s[wave][j] * wave_sum(v);
          const double a = a_s[wave][j];
#pragma unroll
          for (int k = 0; k < K; ++k) qv[k] += (a - bcoef) * (double)Sv(j, k);
        }
        double dg = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float g = Gv(k);
          const bool active = sl.kind(k) == 0 || (X(k) <= lower(k) && g > 0.f);
          const double dk = active ? 0.0 : -qv[k];
          Dv(k) = (float)dk;
          dg += dk * (double)g;
        }
        dg = wave_sum(dg);
        if (!(dg < 0.0)) {  // restart from scaled steepest descent
          h = 0;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const float g = Gv(k);
            const bool active = sl.kind(k) == 0 || (X(k) <= lower(k) && g > 0.f);
            Dv(k) = active ? 0.f : (float)(-gamma0 * (double)g);
          }
        }
        // Backtracking line search on the projected path.
        double t = 1.0, ln = 0.0, fn = 0.0;
        bool ok = false;
        for (int ls = 0; ls < 20 && !ok; ++ls, t *= 0.5) {
          double dec = 0.0;
          wave_sync();
#pragma unroll
          for (int k = 0; k < K; ++k) {
            if (sl.kind(k) == 0) continue;
            const float x0 = X(k);
            const float xn = fmaxf((float)((double)x0 + t * (double)Dv(k)), lower(k));
            XN(k) = xn;
            sl.set(sh, k, xn);
            dec += (double)Gv(k) * ((double)xn - (double)x0);
          }
          dec = wave_sum(dec);
          lpc_colsum(sh, M);
          const bool fin = evaluate();
          ++nev;
          ln = sh.scal[0];
          fn = -ln * inv_n;
          ok = fin && fn <= f + 1e-4 * dec;
        }
        if (!ok) {
          st = MDHP_FIT_STALLED;
          wave_sync();
#pragma unroll
          for (int k = 0; k < K; ++k) sl.set(sh, k, X(k));
          wave_sync();
          break;
        }
        double sy = 0.0, ss = 0.0, yy = 0.0;
        float sk[K], yk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float gn = (float)gf[k];
          const float xn = sl.kind(k) == 0 ? X(k) : XN(k);
          sk[k] = xn - X(k);
          yk[k] = gn - Gv(k);
          sy += (double)sk[k] * (double)yk[k];
          ss += (double)sk[k] * (double)sk[k];
          yy += (double)yk[k] * (double)yk[k];
          X(k) = xn;
          Gv(k) = gn;
        }
        sy = wave_sum(sy);
        ss = wave_sum(ss);
        yy = wave_sum(yy);
        if (sy > 1e-10 * sqrt(ss * yy)) {
          if (h == m_hist) h -= 1;  // the oldest pair drops out of the ring
#pragma unroll
          for (int k = 0; k < K; ++k) {
            Sv(head, k) = sk[k];
            Yv(head, k) = yk[k];
          }
          rho_s[wave][head] = 1.0 / sy;  // every lane writes the same value
          sy_new = sy;
          yy_new = yy;
          head = (head + 1) % kMaxHistory;
          h += 1;
        }
        const double l_prev = l;
        l = ln;
        f = fn;
        if (fabs(l - l_prev) <= o.ll_tol * fmax(fabs(l), 1.0)) {
          st = MDHP_FIT_CONVERGED;
          s += 1;
          break;
        }
      }
    }
    lpc_store(sh, w, M, mu, alpha, beta);
    if (lane == 0) {
      ll[w] = l;
      steps[w] = s;
      status[w] = st;
      if (evals_out) evals_out[w] = nev;
    }
  }
}

template <int MP>
hipError_t launch_lpc_eval(const Events& ev, int M, const float* mu, const float* alpha,
                           const float* beta, double* ll, float* g_mu, float* g_alpha,
                           float* g_beta, int* counter, hipStream_t s, bool grad) {
  if (ev.W == 0) return hipSuccess;
  reset_counter(counter, s);
  const int64_t groups = (ev.W + kWaves - 1) / kWaves;
  if (grad) {
    auto k = lpc_eval_kernel<MP, true>;
    hipLaunchKernelGGL(k, dim3(occupancy_grid(k, kBlock, groups)), dim3(kBlock), 0, s, ev, M, mu,
                       alpha, beta, ll, g_mu, g_alpha, g_beta, counter);
  } else {
    auto k = lpc_eval_kernel<MP, false>;
    hipLaunchKernelGGL(k, dim3(occupancy_grid(k, kBlock, groups)), dim3(kBlock), 0, s, ev, M, mu,
                       alpha, beta, ll, g_mu, g_alpha, g_beta, counter);
  }
  return hipGetLastError();
}

template <int MP>
hipError_t launch_lpc_fit(const Events& ev, int M, const FitParams& o, float* mu, float* alpha,
                          float* beta, double* ll, int* steps, int* status, int* evals, float* ws,
                          int64_t ws_floats, int* counter, hipStream_t s) {
  if (ev.W == 0) return hipSuccess;
  reset_counter(counter, s);
  const int64_t groups = (ev.W + kWaves - 1) / kWaves;
  if (o.optimizer == MDHP_OPT_LBFGS) {
    auto k = lpc_lbfgs_kernel<MP>;
    const int grid = (int)std::min<int64_t>(occupancy_grid(k, kBlock, groups),
                                            ws_floats / (kWaves * lpc_ws_per_wave<MP>()));
    if (grid < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), 0, s, ev, M, o, mu, alpha, beta, ll, steps,
                       status, evals, ws, counter);
    return hipGetLastError();
  }
  auto k = lpc_fit_kernel<MP>;
  hipLaunchKernelGGL(k, dim3(occupancy_grid(k, kBlock, groups)), dim3(kBlock), 0, s, ev, M, o, mu,
                     alpha, beta, ll, steps, status, evals, counter);
  return hipGetLastError();
}

template <int MP>
int64_t lpc_ws(int64_t W) {
  const int64_t groups = std::max<int64_t>((W + kWaves - 1) / kWaves, 1);
  return kWaves * lpc_ws_per_wave<MP>() * occupancy_grid(lpc_lbfgs_kernel<MP>, kBlock, groups);
}

int mp_for(int M) { return M <= 4 ? 4 : (M <= 8 ? 8 : 16); }

}  // namespace

hipError_t lpc_eval(const Events& ev, int M, const float* mu, const float* alpha,
                    const float* beta, double* ll, float* g_mu, float* g_alpha, float* g_beta,
                    int* counter, hipStream_t s, bool grad) {
  switch (mp_for(M)) {
    case 4: return launch_lpc_eval<4>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
    case 8: return launch_lpc_eval<8>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
    default: return launch_lpc_eval<16>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
  }
}

hipError_t lpc_fit(const Events& ev, int M, const FitParams& o, float* mu, float* alpha,
                   float* beta, double* ll, int* steps, int* status, int* evals, float* ws,
                   int64_t ws_floats, int* counter, hipStream_t s) {
  switch (mp_for(M)) {
    case 4: return launch_lpc_fit<4>(ev, M, o, mu, alpha, beta, ll, steps, status, evals, ws, ws_floats, counter, s);
    case 8: return launch_lpc_fit<8>(ev, M, o, mu, alpha, beta, ll, steps, status, evals, ws, ws_floats, counter, s);
    default: return launch_lpc_fit<16>(ev, M, o, mu, alpha, beta, ll, steps, status, evals, ws, ws_floats, counter, s);
  }
}

int64_t lpc_lbfgs_workspace(int M, int64_t W) {
  switch (mp_for(M)) {
    case 4: return lpc_ws<4>(W);
    case 8: return lpc_ws<8>(W);
    default: return lpc_ws<16>(W);
  }
}

}  // namespace mdhp
