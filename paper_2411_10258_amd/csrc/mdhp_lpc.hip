// Shared-decay likelihood, gradient and persistent fits for M <= 16 with one
// chunk of events per lane ("lane per chunk").
//
// A team of NW wavefronts owns one window at a time: one wavefront for
// ordinary windows, the whole 4-wave workgroup for windows of at least the
// plan's threshold (1,024 events unless tuned).  Those form a prefix of the
// largest-first order; persistent workgroups take them as teams and their
// waves take the rest one each (see for_windows).  The window's N events are cut into T = 64 NW contiguous
// chunks of c = ceil(N / T) events, one per lane of the team, and the plan
// stores them lane-major: event j of chunk t sits at slot begin + T j + t
// (padding slots: gap 0, dimension 0xFF), so every step of a wave reads 64
// consecutive gaps and dimension bytes.
//
// Every lane keeps the whole decay state of its chunk in registers: R_n, S_n
// and the pending counts P_n for n < MP (MP = M rounded up to 4, 8 or 16),
//   R_n(i) = sum_{k: d_k = n, t_k < t_i} e^{-beta (t_i - t_k)}      (Part1's inner sum, Eq. (5))
//   S_n(i) = sum_{k: d_k = n, t_k < t_i} (t_i - t_k) e^{-beta (t_i - t_k)}   (= -dR/dbeta)
// and applies the exponential-kernel recursion to the inclusive state
// Rin = R + P (events at or before the current time):
//   Rin <- a Rin + e_d,  S <- a (S + dt Rin),  R = a Rin if dt > 0 (else R stays),
// a = e^{-beta dt}, exactly 1 at equal times, which therefore never excite
// each other.  No lane waits for another.  The chunk carries (zero-start end
// state, product of decays A, summed gaps delta, "has a positive gap" flag)
// are combined across the team by an inclusive scan (DPP row shifts and row
// broadcasts inside a wave, then the waves' totals in order); its exclusive
// form gives every lane the exact start state of its chunk, and a second
// pass over the chunk evaluates
//   lambda_i = mu_m + sum_n alpha_mn R_n(i),   m = d_i           (Eq. (2) at t_i)
//   ll += log lambda_i,  G_R[m][n] += R_n(i) / lambda_i,  Gmu[m] += 1 / lambda_i,
//   Gb += sum_n alpha_mn S_n(i) / lambda_i.
// G_R is a sum of one outer product per event, e_{d_i} (R(i) / lambda_i)^T;
// over a step of a wave's 64 events that is a 16 x 64 by 64 x M matrix
// product, run on the matrix cores (v_mfma_f32_16x16x4_f32) from a
// column-major LDS staging of the step (LDS float atomics, one per event and
// component, are ~6x slower than the whole rest of the pass on gfx950).
// Gmu and Gb are per-lane sums; the per-dimension counts N_m come with the
// plan.  The compensator (Part2 + Part3, Appendix B) comes from the window's
// end state advanced to T:
//   E_n = sum_{k: d_k = n} e^{-beta (T - t_k)},  F_n = sum (T - t_k) e^{-beta (T - t_k)}.
// Everything that leaves a lane is reduced in FP64 in a fixed order, so a
// window's results do not depend on the rest of the batch or on timing.

#include "mdhp_device.h"

namespace mdhp {

namespace {

constexpr int kWaves = kLpcBlock / 64;  // wavefronts per workgroup
constexpr int kMinBlocksLpc = 8 / kWaves;  // workgroups per CU: 2 waves per SIMD
constexpr int kPad = 0xFF;           // dimension byte of a padding slot
constexpr int kSpan = 16;            // steps per FP32 span of the MFMA sums

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- wave level

// A value every lane of the wave holds, moved to a scalar register (the
// compiler then treats it, and what is derived from it, as uniform).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uni(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double uni(double x) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
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

// Chunk carry: the state a zero start reaches at the end of a run of
// events, the product of its decays A, the sum of its gaps D, and F = 1 if a
// gap is positive (then the pending counts of the start are folded in).
template <int MP>
struct Carry {
  float R[MP], S[MP], P[MP];
  float A, D, F;
};

// One step of the in-wave scan: where `take`, the lane's run b becomes the
// run ending at the lane chosen by SHIFT (a DPP lane map) followed by b.
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

// Inclusive scan of the wave's carries in lane order.
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

// ---------------------------------------------------------------- team level

// LDS of one team (NW wavefronts sharing a window).
template <int MP, int NW>
struct alignas(16) Team {
  static constexpr int Q = MP + 1;   // row stride of gR64: G_R[m][0..MP-1], Gmu[m]
  static constexpr int T = 64 * NW;  // lanes (= chunks) of the team
  static constexpr int XC = 3 * MP + 4;
  // LDS strides chosen against bank conflicts (32 banks of 4 bytes): rows of
  // alpha start in distinct bank quads for 8 consecutive targets, so that
  // 16-byte row gathers by 8 lanes with different targets do not collide;
  // staging columns are 68 floats apart, so that 8 lanes reading 16 bytes
  // each from 8 columns cover all 32 banks once.
  static constexpr int AS = MP == 4 ? 4 : MP + 4;  // alpha row stride
  static constexpr int VS = 68;                    // staging column stride
  static constexpr int GS = 65;                    // per-lane Gmu row stride
  float alpha[MP * AS];              // [m * AS + n], zero outside M x M
  float mu[MP];                      // zero outside M
  float colsum[MP];                  // sum_m alpha_mn
  float vst[NW][MP * VS];            // per wave: step staging, w_k R_n(k) at [n * VS + k]
  float hot[NW][16 * VS];            // per wave: 1 at [d_k * VS + k] during a step, else 0
  float gmu[NW][MP * GS];            // per lane k: sum of w over its events of target m, [m * GS + k]
  double gpart[NW][MP * MP + MP];    // per wave: FP64 G_R (MFMA spans) and Gmu partials
  float xc[NW][XC];                  // per wave: its inclusive total (R, S, P, A, D, F), then
                                     // the carry of the team's earlier waves
  double gR64[MP * Q];               // window sums: G_R, Gmu in column MP
  double En[MP], Fn[MP];             // E_n, F_n
  double Cn[MP];                     // (N_n - E_n) / beta
  double scal[2];                    // ll, d ll / d beta
  double red[NW][2];                 // cross-wave reduction slots
  double rho[kMaxHistory], alf[kMaxHistory];  // L-BFGS two-loop scalars
  int q;                             // queue position broadcast to the team
  float beta;
};

// One-hot rows e_m (m < MP) and a zero row MP for the recursion's newly
// pending event: the add of [d = m] to R_m + P_m becomes one 16-byte row read
// per four components instead of a compare and select per component.  Rows
// are kOhStride floats apart (distinct bank groups for neighbouring rows).
constexpr int kOhStride = 20;
__shared__ float4 g_onehot[(16 + 1) * kOhStride / 4];

template <int MP>
__device__ __forceinline__ void onehot_init() {
  float* oh = reinterpret_cast<float*>(g_onehot);
  for (int e = threadIdx.x; e < (MP + 1) * kOhStride; e += blockDim.x) {
    const int r = e / kOhStride, m = e % kOhStride;
    oh[e] = (r < MP && m == r) ? 1.f : 0.f;
  }
}

// Row d of the table (the zero row for d >= MP, e.g. a padding slot).
template <int MP>
__device__ __forceinline__ void onehot_row(int d, float (&oh)[MP]) {
  const float4* row = &g_onehot[(d < MP ? d : MP) * (kOhStride / 4)];
#pragma unroll
  for (int q = 0; q < MP / 4; ++q) {
    const float4 v = row[q];
    oh[4 * q] = v.x;
    oh[4 * q + 1] = v.y;
    oh[4 * q + 2] = v.z;
    oh[4 * q + 3] = v.w;
  }
}

template <int NW>
__device__ __forceinline__ int team_tid() {
  return threadIdx.x & (64 * NW - 1);
}

template <int NW>
__device__ __forceinline__ void team_sync() {
  if constexpr (NW == 1) wave_sync();
  else __syncthreads();
}

// Sums of x and y over the team (every lane gets them; fixed order).
template <int MP, int NW>
__device__ __forceinline__ void team_sum2(Team<MP, NW>& sh, double& x, double& y) {
  x = wave_sum(x);
  y = wave_sum(y);
  if constexpr (NW > 1) {
    const int t = team_tid<NW>();
    __syncthreads();
    if ((t & 63) == 0) {
      sh.red[t >> 6][0] = x;
      sh.red[t >> 6][1] = y;
    }
    __syncthreads();
    x = y = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      x += sh.red[k][0];
      y += sh.red[k][1];
    }
  }
  x = uni(x);
  y = uni(y);
}

template <int MP, int NW>
__device__ __forceinline__ double team_sum(Team<MP, NW>& sh, double x) {
  double y = 0.0;
  team_sum2(sh, x, y);
  return x;
}

template <int MP, int NW>
__device__ __forceinline__ double team_max(Team<MP, NW>& sh, double x) {
  x = wave_max(x);
  if constexpr (NW > 1) {
    const int t = team_tid<NW>();
    __syncthreads();
    if ((t & 63) == 0) sh.red[t >> 6][0] = x;
    __syncthreads();
    x = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) x = fmax(x, sh.red[k][0]);
  }
  return uni(x);
}

// True on every lane if `bad` is true on any lane of the team.
template <int MP, int NW>
__device__ __forceinline__ bool team_any(Team<MP, NW>& sh, bool bad) {
  return team_max(sh, __any(bad) ? 1.0 : 0.0) != 0.0;
}

// G_R over one step of a wave: the 64 events' rows w_k R(k) (staged
// column-major in vst) summed by target, G_R[m][n] += sum_k [d_k = m] w_k R_n(k),
// as the product H^T V of the step's one-hot targets H (64 x 16) and V
// (64 x MP): sixteen v_mfma_f32_16x16x4_f32 with K running over the events,
// in two independent accumulator chains.  Lane l supplies A = H[16q + s][l % 16]
// and B = V[16q + s][l % 16] (q = l / 16) to instruction s, and holds
// G_R[4q + r][l % 16] in acc0[r] + acc1[r].
template <int MP, int VS>
__device__ __forceinline__ void step_outer(const float* vst, const float* hot, f32x4& acc0,
                                           f32x4& acc1) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, base = (lane >> 4) * 16;
  f32x4 a[4], b[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    a[i] = *reinterpret_cast<const f32x4*>(&hot[col * VS + base + 4 * i]);
    b[i] = col < MP ? *reinterpret_cast<const f32x4*>(&vst[(col % MP) * VS + base + 4 * i])
                    : f32x4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][0], b[i][0], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][1], b[i][1], acc1, 0, 0, 0);
    acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][2], b[i][2], acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][3], b[i][3], acc1, 0, 0, 0);
  }
}

// Runs body(j, dt_j, d_j) for the steps j = 0 .. c-1 of a lane's chunk
// (slot stride T), with the loads of the next kAhead steps in flight.
constexpr int kAhead = 4;
template <int T, class BODY>
__device__ __forceinline__ void for_steps(const float* __restrict__ dtw,
                                          const uint8_t* __restrict__ dw, int c, BODY&& body) {
  float dt_c[kAhead];
  int d_c[kAhead];
  auto load = [&](int j0, float (&dtq)[kAhead], int (&dq)[kAhead]) {
    static_for<kAhead>([&](auto Q) {
      constexpr int q = decltype(Q)::value;
      const bool in = j0 + q < c;  // uniform
      dtq[q] = in ? dtw[(int64_t)(j0 + q) * T] : 0.f;
      dq[q] = in ? (int)dw[(int64_t)(j0 + q) * T] : kPad;
    });
  };
  load(0, dt_c, d_c);
  for (int jb = 0; jb < c; jb += kAhead) {
    float dt_n[kAhead];
    int d_n[kAhead];
    load(jb + kAhead, dt_n, d_n);
    static_for<kAhead>([&](auto Q) {
      constexpr int q = decltype(Q)::value;
      if (jb + q < c) body(jb + q, dt_c[q], d_c[q]);
    });
    static_for<kAhead>([&](auto Q) {
      constexpr int q = decltype(Q)::value;
      dt_c[q] = dt_n[q];
      d_c[q] = d_n[q];
    });
  }
}

// Compensator sums of a slowly decaying window from its events (the lane's
// chunk: c slots, T apart; padding slots have tau 0 and no dimension): lane
// m < MP gets qs = sum over source-m events of -expm1(-beta tau) and hs = the
// sum of h(beta tau).  One component per sweep over the events, so that
// the few registers it needs leave the fit kernels' allocation alone.
template <int MP, int NW>
__device__ __forceinline__ void slow_decay_sums(Team<MP, NW>& sh, const float* __restrict__ tw,
                                                const uint8_t* __restrict__ dw, int c, float beta,
                                                double& qs, double& hs) {
  constexpr int T = Team<MP, NW>::T;
  const int t = team_tid<NW>();
  const int lane = t & 63, wv = t >> 6;
#pragma unroll 1
  for (int m = 0; m < MP; ++m) {
    float q = 0.f, h = 0.f;
#pragma unroll 1
    for (int j = 0; j < c; ++j) {
      if (dw[(int64_t)j * T] != m) continue;
      const float xk = beta * tw[(int64_t)j * T];
      q += comp_q(xk);
      h += comp_h(xk);
    }
    // gpart is free here (its G_R partials were summed before the last sync).
    const double qt = wave_sum((double)q), ht = wave_sum((double)h);
    if (lane == 0) {
      sh.gpart[wv][m] = qt;
      sh.gpart[wv][MP + m] = ht;
    }
  }
  team_sync<NW>();
  qs = hs = 0.0;
  if (t < MP) {
#pragma unroll
    for (int wk = 0; wk < NW; ++wk) {
      qs += sh.gpart[wk][t];
      hs += sh.gpart[wk][MP + t];
    }
  }
}

// Evaluates the team's window with the parameters in its LDS (alpha, mu,
// colsum, beta; gmu cleared; counts = the window's N_m).  On return (all
// lanes, after a team sync): scal[0] = ll; with GRAD also gR64 (G_R and, in
// column MP, Gmu), Cn, Fn and scal[1] = d ll / d beta.  FP32 sums run over
// spans of kSpan steps (MFMA) or over the lane's chunk, then FP64.
template <int MP, int NW, bool GRAD>
__device__ __forceinline__ void team_eval(Team<MP, NW>& sh, const float* __restrict__ dtg,
                                          const uint8_t* __restrict__ dg,
                                          const float* __restrict__ taug, int64_t begin, int n,
                                          double Tw, float end_gap,
                                          const int32_t* __restrict__ counts, int M) {
  constexpr int Q = Team<MP, NW>::Q;
  constexpr int T = Team<MP, NW>::T;
  const int t = team_tid<NW>();
  const int lane = t & 63, wv = t >> 6;
  const float beta = uni(sh.beta);
  const int c = (n + T - 1) / T;
  const float* __restrict__ dtw = dtg + begin + t;
  const uint8_t* __restrict__ dw = dg + begin + t;

  // Pass 1: the chunk's carry from a zero start.
  Carry<MP> cr;
  float Rin[MP];
#pragma unroll
  for (int m = 0; m < MP; ++m) Rin[m] = cr.S[m] = 0.f;
  cr.A = 1.f;
  cr.D = 0.f;
  for_steps<T>(dtw, dw, c, [&](int, float dt, int d) {
    const float a = dt > 0.f ? __expf(-beta * dt) : 1.f;
    float oh[MP];
    onehot_row<MP>(d, oh);
#pragma unroll
    for (int m = 0; m < MP; ++m) {
      cr.S[m] = a * fmaf(dt, Rin[m], cr.S[m]);
      Rin[m] = fmaf(a, Rin[m], oh[m]);
    }
    cr.A *= a;
    cr.D += dt;
  });
  // Pending counts at the chunk's end: the events after its last positive
  // gap (all of them if it has none); R = Rin - P.
  {
#pragma unroll
    for (int m = 0; m < MP; ++m) cr.P[m] = 0.f;
    const int len = (int)min<int64_t>(max<int64_t>((int64_t)n - (int64_t)t * c, 0), c);
    for (int j = len - 1; j >= 0; --j) {
      const int d = dw[(int64_t)j * T];
#pragma unroll
      for (int m = 0; m < MP; ++m) cr.P[m] += m == d ? 1.f : 0.f;
      if (dtw[(int64_t)j * T] > 0.f) break;
    }
#pragma unroll
    for (int m = 0; m < MP; ++m) cr.R[m] = Rin[m] - cr.P[m];
  }
  cr.F = cr.D > 0.f ? 1.f : 0.f;
  scan_carries<MP>(cr, lane);
  // Cross-wave: xc[w] first receives wave w's total, then (lanes m <= MP of
  // wave 0, one component each, in wave order) the carry X of waves 0..w-1;
  // every lane's inclusive carry becomes X followed by its in-wave prefix.
  if constexpr (NW > 1) {
    if (lane == 63) {
#pragma unroll
      for (int m = 0; m < MP; ++m) {
        sh.xc[wv][m] = cr.R[m];
        sh.xc[wv][MP + m] = cr.S[m];
        sh.xc[wv][2 * MP + m] = cr.P[m];
      }
      sh.xc[wv][3 * MP] = cr.A;
      sh.xc[wv][3 * MP + 1] = cr.D;
      sh.xc[wv][3 * MP + 2] = cr.F;
    }
    __syncthreads();
    if (wv == 0) {
      // Lane m < MP: component m; lane MP: the shared A, D, F.
      const int m = lane < MP ? lane : 0;
      float xr = 0.f, xs = 0.f, xp = 0.f, xa = 1.f, xd = 0.f, xf = 0.f;
      float out[NW][3];
#pragma unroll
      for (int k = 0; k + 1 < NW; ++k) {
        const float br = sh.xc[k][m], bs = sh.xc[k][MP + m], bp = sh.xc[k][2 * MP + m];
        const float ba = sh.xc[k][3 * MP], bd = sh.xc[k][3 * MP + 1], bf = sh.xc[k][3 * MP + 2];
        const float Xs = xr + xp;
        const bool f = bf != 0.f;
        const float nr = f ? fmaf(ba, Xs, br) : xr;
        const float ns = f ? fmaf(ba, fmaf(bd, Xs, xs), bs) : xs;
        const float np = f ? bp : xp + bp;
        xr = nr;
        xs = ns;
        xp = np;
        xa *= ba;
        xd += bd;
        xf = fmaxf(xf, bf);
        out[k + 1][0] = lane < MP ? xr : xa;
        out[k + 1][1] = lane < MP ? xs : xd;
        out[k + 1][2] = lane < MP ? xp : xf;
      }
      wave_sync();  // every lane of wave 0 has read the totals
#pragma unroll
      for (int k = 1; k < NW; ++k) {
        if (lane < MP) {
          sh.xc[k][m] = out[k][0];
          sh.xc[k][MP + m] = out[k][1];
          sh.xc[k][2 * MP + m] = out[k][2];
        } else if (lane == MP) {
          sh.xc[k][3 * MP] = out[k][0];
          sh.xc[k][3 * MP + 1] = out[k][1];
          sh.xc[k][3 * MP + 2] = out[k][2];
        }
      }
    }
    __syncthreads();
    if (wv > 0) {  // cr <- X followed by cr
      const float* x = sh.xc[wv];
      const bool f = cr.F != 0.f;
#pragma unroll
      for (int m = 0; m < MP; ++m) {
        const float aR = x[m], aS = x[MP + m], aP = x[2 * MP + m];
        const float Xs = aR + aP;
        const float r = f ? fmaf(cr.A, Xs, cr.R[m]) : aR;
        const float sv = f ? fmaf(cr.A, fmaf(cr.D, Xs, aS), cr.S[m]) : aS;
        const float p = f ? cr.P[m] : aP + cr.P[m];
        cr.R[m] = r;
        cr.S[m] = sv;
        cr.P[m] = p;
      }
      cr.A *= x[3 * MP];
      cr.D += x[3 * MP + 1];
      cr.F = fmaxf(cr.F, x[3 * MP + 2]);
    }
  }
  // The team's last lane now holds the window's end state: E_n, F_n at T.
  if (t == T - 1) {
    const double gap = (double)end_gap;
    const double ea = exp(-(double)beta * gap);
#pragma unroll
    for (int m = 0; m < MP; ++m) {
      const double E = ea * ((double)cr.R[m] + (double)cr.P[m]);
      sh.En[m] = E;
      sh.Fn[m] = ea * (double)cr.S[m] + gap * E;
    }
  }
  // Exclusive form: lane t starts from the state after chunks 0 .. t-1
  // (strict R, inclusive Rin = R + P, S); lane 0 of a later wave from the
  // carry of the earlier waves.
  float R[MP], S[MP];
  const bool from_x = NW > 1 && lane == 0 && wv > 0;
  const float* xw = sh.xc[wv];
#pragma unroll
  for (int m = 0; m < MP; ++m) {
    float pR = __shfl_up(cr.R[m], 1, 64), pS = __shfl_up(cr.S[m], 1, 64);
    float pP = __shfl_up(cr.P[m], 1, 64);
    if (lane == 0) {
      pR = from_x ? xw[m] : 0.f;
      pS = from_x ? xw[MP + m] : 0.f;
      pP = from_x ? xw[2 * MP + m] : 0.f;
    }
    R[m] = pR;
    S[m] = pS;
    Rin[m] = pR + pP;
  }
  // Pass 2: intensities, log-likelihood and gradient sums.
  float llp = 0.f, gbp = 0.f;
  double ll64 = 0.0, gb64 = 0.0;
  f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  double* gpart = sh.gpart[wv];
  const int gcol = lane & 15, grow0 = (lane >> 4) * 4;  // this lane's G_R[grow0 + r][gcol]
  constexpr int AS = Team<MP, NW>::AS, VS = Team<MP, NW>::VS, GS = Team<MP, NW>::GS;
  float* vst = sh.vst[wv];
  float* hot = sh.hot[wv];
  float* gmu = &sh.gmu[wv][lane];
  for_steps<T>(dtw, dw, c, [&](int j, float dt, int dr) {
    const bool v = dr != kPad;
    const int d = v ? dr : 0;
    const bool f = dt > 0.f;
    const float a = f ? __expf(-beta * dt) : 1.f;
    const float* arow = &sh.alpha[d * AS];
    float lam = sh.mu[d], asum = 0.f;
    float g_old = 0.f;
    if constexpr (GRAD) g_old = gmu[d * GS];
    float oh[MP];
    onehot_row<MP>(dr, oh);
#pragma unroll
    for (int m = 0; m < MP; ++m) {
      const float tm = a * Rin[m];
      S[m] = a * fmaf(dt, Rin[m], S[m]);
      R[m] = f ? tm : R[m];
      Rin[m] = tm + oh[m];
      const float al = arow[m];
      lam = fmaf(al, R[m], lam);
      asum = fmaf(al, S[m], asum);
    }
    if (v) llp += __logf(lam);
    if constexpr (GRAD) {
      // Padding events stage w = 0 (target 0, so their one-hot entry adds 0).
      const float w = v ? __builtin_amdgcn_rcpf(lam) : 0.f;
      gbp = fmaf(w, asum, gbp);
      gmu[d * GS] = g_old + w;  // the lane's own entry: no other lane touches it
#pragma unroll
      for (int m = 0; m < MP; ++m) vst[m * VS + lane] = w * R[m];
      hot[d * VS + lane] = 1.f;
      wave_sync();
      step_outer<MP, VS>(vst, hot, acc0, acc1);
      wave_sync();
      hot[d * VS + lane] = 0.f;
      if (j % kSpan == kSpan - 1 || j + 1 == c) {
#pragma unroll
        for (int r = 0; r < 4; ++r)  // the lane's own entries: no other lane touches them
          if (grow0 + r < MP && gcol < MP)
            gpart[(grow0 + r) * MP + gcol] += (double)acc0[r] + (double)acc1[r];
        acc0 = f32x4{0.f, 0.f, 0.f, 0.f};
        acc1 = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
    if (j % kSpan == kSpan - 1 || j + 1 == c) {
      ll64 += (double)llp;
      gb64 += (double)gbp;
      llp = gbp = 0.f;
    }
  });
  if constexpr (GRAD) {
    // Each wave's Gmu partials (FP64) next to its G_R partials, then the
    // team's sums over waves in order.
    wave_sync();
    if (lane < MP) {
      const float* gw = sh.gmu[wv];
      double g[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 16
      for (int l = 0; l < 64; ++l) g[l & 3] += (double)gw[lane * GS + l];
      gpart[MP * MP + lane] = (g[0] + g[1]) + (g[2] + g[3]);
    }
    team_sync<NW>();
    for (int e = t; e < MP * Q; e += T) {
      const int m = e / Q, k = e % Q;
      const int src = k < MP ? m * MP + k : MP * MP + m;
      double s = 0.0;
#pragma unroll
      for (int wk = 0; wk < NW; ++wk) s += sh.gpart[wk][src];
      sh.gR64[e] = s;
    }
  }
  team_sync<NW>();
  // Compensator: lane m < M finishes source dimension m, from the end state
  // (C = (N - E) / beta, F - C) or, for a slow decay, from the events.
  const double b = (double)beta;
  const bool slow = b * Tw < kSlowDecayLane;  // uniform
  double qs = 0.0, hs = 0.0;  // lane m: sum over source-m events of -expm1(-beta tau), h(beta tau)
  if (__builtin_expect(slow, 0)) slow_decay_sums<MP, NW>(sh, taug + begin + t, dw, c, beta, qs, hs);
  double x = ll64, y = gb64;
  if (t < M) {
    const double C = slow ? qs / b : ((double)counts[t] - sh.En[t]) / b;
    const double FmC = slow ? hs / b : sh.Fn[t] - C;  // F_n - C_n
    const double cs = (double)sh.colsum[t];
    x -= Tw * (double)sh.mu[t] + cs * C;
    y += cs * FmC / b;
    sh.Cn[t] = C;
  } else if (t < MP) {
    sh.Cn[t] = 0.0;
  }
  team_sum2(sh, x, y);
  if (t == 0) {
    sh.scal[0] = x;
    sh.scal[1] = -y;
  }
  team_sync<NW>();
}

template <int MP, int NW>
__device__ __forceinline__ void team_colsum(Team<MP, NW>& sh, int M) {
  const int t = team_tid<NW>();
  team_sync<NW>();
  if (t < MP) {
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += sh.alpha[m * Team<MP, NW>::AS + t];
    sh.colsum[t] = s;
  }
  team_sync<NW>();
}

template <int MP, int NW>
__device__ __forceinline__ void team_load(Team<MP, NW>& sh, const float* __restrict__ mu,
                                          const float* __restrict__ alpha,
                                          const float* __restrict__ beta, int64_t w, int M) {
  const int t = team_tid<NW>();
  team_sync<NW>();
  for (int e = t; e < MP * MP; e += Team<MP, NW>::T) {
    const int m = e / MP, n = e % MP;
    sh.alpha[m * Team<MP, NW>::AS + n] = (m < M && n < M) ? alpha[(w * M + m) * M + n] : 0.f;
  }
  if (t < MP) sh.mu[t] = t < M ? mu[w * M + t] : 0.f;
  if (t == 0) sh.beta = beta[w];
  team_colsum(sh, M);
}

// Clears the Gmu and G_R partial sums (before every evaluation with gradient).
template <int MP, int NW>
__device__ __forceinline__ void team_zero(Team<MP, NW>& sh) {
  const int t = team_tid<NW>();
  team_sync<NW>();
  float* g = &sh.gmu[0][0];
  for (int e = t; e < NW * MP * Team<MP, NW>::GS; e += Team<MP, NW>::T) g[e] = 0.f;
  double* gp = &sh.gpart[0][0];
  for (int e = t; e < NW * (MP * MP + MP); e += Team<MP, NW>::T) gp[e] = 0.0;
  team_sync<NW>();
}

// Clears the one-hot staging (kept zero between steps).
template <int MP, int NW>
__device__ __forceinline__ void team_init(Team<MP, NW>& sh) {
  const int t = team_tid<NW>();
  float* h = &sh.hot[0][0];
  for (int e = t; e < NW * 16 * Team<MP, NW>::VS; e += Team<MP, NW>::T) h[e] = 0.f;
  team_sync<NW>();
}

// Next window of the team: queue position `first_q` the first time, then
// from the atomic head `head` (offset by the positions handed out at start).
template <int MP, int NW>
__device__ __forceinline__ int team_next(Team<MP, NW>& sh, int* head, bool first, int first_q,
                                         int started) {
  const int t = team_tid<NW>();
  int q = 0;
  if (t == 0) q = first ? first_q : atomicAdd(head, 1) + started;
  if constexpr (NW == 1) {
    return uni(q);  // lane 0 of the wave holds it
  } else {
    __syncthreads();
    if (t == 0) sh.q = q;
    __syncthreads();
    return uni(sh.q);
  }
}

// Both team shapes share the workgroup's LDS.
template <int MP>
union BlockLds {
  Team<MP, kWaves> big;
  Team<MP, 1> small[kWaves];
};

// Runs every window once: the first n_big of the largest-first order as
// workgroup teams (queue head counter[0], largest first), the rest one per
// wavefront (counter[1], smallest first).  One workgroup in kSmallFirst
// starts with the one-wave windows, the others with the workgroup windows;
// each turns to the other queue when its first is empty.  Small windows are
// cheap per evaluation but some need many evaluations, so they start from
// the beginning instead of after every large window, and the longest of
// them no longer ends the batch.
constexpr int kSmallFirst = 4;
template <int MP, class BIG, class SMALL>
__device__ __forceinline__ void for_windows(BlockLds<MP>& lds, const Events& ev, int* counter,
                                            BIG&& big_body, SMALL&& small_body) {
  const int nb = (int)ev.n_big;
  const int W = (int)ev.W;
  auto big_phase = [&]() {
    Team<MP, kWaves>& sh = lds.big;
    team_init(sh);
    for (int q = team_next(sh, &counter[0], false, 0, 0); q < nb;
         q = team_next(sh, &counter[0], false, 0, 0))
      big_body(sh, (int64_t)ev.order[q]);
    __syncthreads();
  };
  auto small_phase = [&]() {
    Team<MP, 1>& sh = lds.small[threadIdx.x >> 6];
    team_init(sh);
    for (int k = team_next(sh, &counter[1], false, 0, 0); nb + k < W;
         k = team_next(sh, &counter[1], false, 0, 0))
      small_body(sh, (int64_t)ev.order[W - 1 - k]);
    __syncthreads();
  };
  if ((int)blockIdx.x % kSmallFirst == kSmallFirst - 1) {
    small_phase();
    big_phase();
  } else {
    big_phase();
    small_phase();
  }
}

// ---------------------------------------------------------------- kernels

template <int MP, int NW, bool GRAD>
__device__ __forceinline__ void eval_one(Team<MP, NW>& sh, const Events& ev, int64_t w, int M,
                                         const float* mu, const float* alpha, const float* beta,
                                         double* ll, float* g_mu, float* g_alpha,
                                         float* g_beta) {
  constexpr int Q = Team<MP, NW>::Q;
  const int t = team_tid<NW>();
  if constexpr (GRAD) team_zero(sh);
  team_load(sh, mu, alpha, beta, w, M);
  const double Tw = ev.T[w];
  team_eval<MP, NW, GRAD>(sh, ev.dt, ev.d, ev.tau, ev.begin[w], ev.n[w], Tw, ev.end_gap[w],
                          ev.counts + w * M, M);
  if (t == 0) ll[w] = sh.scal[0];
  if constexpr (GRAD) {
    if (t == 0) g_beta[w] = (float)sh.scal[1];
    if (t < M) g_mu[w * M + t] = (float)(sh.gR64[t * Q + MP] - Tw);
    for (int e = t; e < M * M; e += Team<MP, NW>::T) {
      const int m = e / M, k = e % M;
      g_alpha[w * M * M + e] = (float)(sh.gR64[m * Q + k] - sh.Cn[k]);
    }
  }
}

template <int MP, bool GRAD>
__global__ __launch_bounds__(kLpcBlock, kMinBlocksLpc) void lpc_eval_kernel(Events ev, int M, const float* mu,
                                                          const float* alpha, const float* beta,
                                                          double* ll, float* g_mu,
                                                          float* g_alpha, float* g_beta,
                                                          int* counter) {
  __shared__ BlockLds<MP> lds;
  onehot_init<MP>();
  __syncthreads();
  for_windows<MP>(
      lds, ev, counter,
      [&](Team<MP, kWaves>& sh, int64_t w) {
        eval_one<MP, kWaves, GRAD>(sh, ev, w, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta);
      },
      [&](Team<MP, 1>& sh, int64_t w) {
        eval_one<MP, 1, GRAD>(sh, ev, w, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta);
      });
}

// Parameter slots of a team's fit: lane t owns the alpha entries
// e = t + T k (k < OWN, e = m * MP + n) and one extra slot k = OWN holding
// mu_t (t < M) or beta (t == M).  Kinds: 0 none, 1 alpha, 2 mu, 3 beta.
template <int MP, int NW>
struct Slots {
  static constexpr int T = 64 * NW;
  static constexpr int OWN = (MP * MP + T - 1) / T;
  static constexpr int K = OWN + 1;
  int M, t, fix_beta;
  // LDS index of alpha entry e = m * MP + n.
  __device__ static int at(int e) { return (e / MP) * Team<MP, NW>::AS + e % MP; }
  __device__ int kind(int k) const {
    if (k < OWN) {
      const int e = t + k * T;
      return (e < MP * MP && e / MP < M && e % MP < M) ? 1 : 0;
    }
    if (t < M) return 2;
    if (t == M) return fix_beta ? 0 : 3;
    return 0;
  }
  __device__ float get(const Team<MP, NW>& sh, int k) const {
    const int kd = kind(k);
    if (kd == 1) return sh.alpha[at(t + k * T)];
    if (kd == 2) return sh.mu[t];
    if (kd == 3) return sh.beta;
    return 0.f;
  }
  __device__ void set(Team<MP, NW>& sh, int k, float v) const {
    const int kd = kind(k);
    if (kd == 1) sh.alpha[at(t + k * T)] = v;
    else if (kd == 2) sh.mu[t] = v;
    else if (kd == 3) sh.beta = v;
  }
  // d ll / d theta of slot k after an evaluation with gradient.
  __device__ double grad(const Team<MP, NW>& sh, int k, double Tw) const {
    constexpr int Q = Team<MP, NW>::Q;
    const int kd = kind(k);
    if (kd == 1) {
      const int e = t + k * T;
      return sh.gR64[(e / MP) * Q + e % MP] - sh.Cn[e % MP];
    }
    if (kd == 2) return sh.gR64[t * Q + MP] - Tw;
    if (kd == 3) return uni(sh.scal[1]);
    return 0.0;
  }
};

template <int MP, int NW>
__device__ __forceinline__ void team_store(Team<MP, NW>& sh, int64_t w, int M, float* mu,
                                           float* alpha, float* beta) {
  const int t = team_tid<NW>();
  team_sync<NW>();
  for (int e = t; e < M * M; e += Team<MP, NW>::T)
    alpha[w * M * M + e] = sh.alpha[(e / M) * Team<MP, NW>::AS + e % M];
  if (t < M) mu[w * M + t] = sh.mu[t];
  if (t == 0) beta[w] = sh.beta;
}

// Projected gradient ascent / projected Adam on one window (the rule of the
// workgroup kernel: evaluate, stop on a non-finite value, on
// |delta ll| <= ll_tol max(|ll|, N, 1) or after max_steps updates, else step
// along the gradient divided by N and project).
template <int MP, int NW>
__device__ __forceinline__ void fit_one(Team<MP, NW>& sh, const Events& ev, int64_t w, int M,
                                        const FitParams& o, float* mu, float* alpha, float* beta,
                                        double* ll, int* steps, int* status, int* evals_out) {
  constexpr int K = Slots<MP, NW>::K;
  const int t = team_tid<NW>();
  const Slots<MP, NW> sl{M, t, o.fix_beta};
  team_load(sh, mu, alpha, beta, w, M);
  const int n = ev.n[w];
  const double Tw = ev.T[w];
  const double rate = (double)max(n, 1) / Tw;
  const double mu_min = o.mu_floor_rel * rate;
  const double beta_min = o.beta_floor_rel * rate;
  const double inv_n = 1.0 / (double)max(n, 1);
  float m1[K], m2[K];
#pragma unroll
  for (int k = 0; k < K; ++k) m1[k] = m2[k] = 0.f;
  double ll_prev = 0.0, b1t = 1.0, b2t = 1.0;
  int s = 0, st = MDHP_FIT_MAX_STEPS;
  for (s = 0;; ++s) {
    team_zero(sh);
    team_eval<MP, NW, true>(sh, ev.dt, ev.d, ev.tau, ev.begin[w], n, Tw, ev.end_gap[w],
                            ev.counts + w * M, M);
    const double l = uni(sh.scal[0]);
    double g[K];
    bool bad = !isfinite(l) || !isfinite(uni(sh.scal[1]));
#pragma unroll
    for (int k = 0; k < K; ++k) {
      g[k] = sl.grad(sh, k, Tw);
      if (!isfinite(g[k])) bad = true;
    }
    if (team_any(sh, bad)) {
      st = MDHP_FIT_NONFINITE;
      break;
    }
    if (s >= 1 && fabs(l - ll_prev) <= o.ll_tol * fmax(fabs(l), (double)max(n, 1))) {
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
    team_sync<NW>();
    if (o.optimizer == MDHP_OPT_EM) {
      // Expected background and offspring counts over their exposures
      // (the decays are fixed: kind 3 does not occur).
      constexpr int Q = Team<MP, NW>::Q, TT = Team<MP, NW>::T;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int kd = sl.kind(k);
        const double x = (double)sl.get(sh, k);
        if (kd == 1) {
          const int e = t + k * TT, nn = e % MP;
          const double C = sh.Cn[nn];
          if (C > 0.0) sl.set(sh, k, (float)(x * (sh.gR64[(e / MP) * Q + nn] / C)));
        } else if (kd == 2) {
          sl.set(sh, k, (float)fmax(x * (sh.gR64[t * Q + MP] / Tw), mu_min));
        }
      }
      team_colsum(sh, M);
      continue;
    }
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
    team_colsum(sh, M);
  }
  // The parameters of the last evaluation are in LDS.
  team_store(sh, w, M, mu, alpha, beta);
  if (t == 0) {
    ll[w] = sh.scal[0];
    steps[w] = s;
    status[w] = st;
    if (evals_out) evals_out[w] = s + 1;
  }
}

template <int MP>
__global__ __launch_bounds__(kLpcBlock, kMinBlocksLpc) void lpc_fit_kernel(Events ev, int M, FitParams o,
                                                         float* mu, float* alpha, float* beta,
                                                         double* ll, int* steps, int* status,
                                                         int* evals_out, int* counter) {
  __shared__ BlockLds<MP> lds;
  onehot_init<MP>();
  __syncthreads();
  for_windows<MP>(
      lds, ev, counter,
      [&](Team<MP, kWaves>& sh, int64_t w) {
        fit_one<MP, kWaves>(sh, ev, w, M, o, mu, alpha, beta, ll, steps, status, evals_out);
      },
      [&](Team<MP, 1>& sh, int64_t w) {
        fit_one<MP, 1>(sh, ev, w, M, o, mu, alpha, beta, ll, steps, status, evals_out);
      });
}

// Workspace floats of one team's L-BFGS fit: x, g, d, then the s and y
// rings; K slots of T lanes each.
template <int MP, int NW>
constexpr int64_t team_ws() {
  return (int64_t)kLbfgsVectors * Slots<MP, NW>::K * 64 * NW;
}

// Per workgroup: the larger of one big team and kWaves small teams.
template <int MP>
constexpr int64_t block_ws() {
  return team_ws<MP, kWaves>() > kWaves * team_ws<MP, 1>() ? team_ws<MP, kWaves>()
                                                            : kWaves * team_ws<MP, 1>();
}

// Projected L-BFGS on one window: the rule of the workgroup kernel (two-loop
// recursion on the free set, Armijo backtracking on the projected path,
// curvature-checked history, restart from scaled steepest descent) with
// team-level reductions.  Between evaluations the lane's slices of x, g and
// the direction are in registers; x, g and d go to the team's workspace
// (base: the same for the whole team) for the line search, whose
// evaluations need every register.
template <int MP, int NW>
__device__ __forceinline__ void lbfgs_one(Team<MP, NW>& sh, const Events& ev, int64_t w, int M,
                                          const FitParams& o, float* mu, float* alpha,
                                          float* beta, double* ll, int* steps, int* status,
                                          int* evals_out, float* base) {
  constexpr int K = Slots<MP, NW>::K;
  constexpr int T = Team<MP, NW>::T;
  using Ws = LbfgsWs<K, T>;
  const int t = team_tid<NW>();
  const int m_hist = o.history;
  const Slots<MP, NW> sl{M, t, o.fix_beta};
  const Ws wsp(base, t);
  team_load(sh, mu, alpha, beta, w, M);
  const int n = ev.n[w];
  const double Tw = ev.T[w];
  const double rate = (double)max(n, 1) / Tw;
  const float mu_min = (float)(o.mu_floor_rel * rate);
  const float beta_min = (float)(o.beta_floor_rel * rate);
  const double inv_n = 1.0 / (double)max(n, 1);
  auto lower = [&](int k) -> float {
    const int kd = sl.kind(k);
    return kd == 2 ? mu_min : (kd == 3 ? beta_min : 0.f);
  };
  // Gradient of f = -ll / N for slot k, from the last evaluation in LDS.
  auto gf = [&](int k) -> double { return -sl.grad(sh, k, Tw) * inv_n; };
  // Evaluates at the LDS parameters; false if ll or any gradient entry is
  // not finite.
  auto evaluate = [&]() -> bool {
    team_zero(sh);
    team_eval<MP, NW, true>(sh, ev.dt, ev.d, ev.tau, ev.begin[w], n, Tw, ev.end_gap[w],
                            ev.counts + w * M, M);
    bool bad = !isfinite(uni(sh.scal[0])) || !isfinite(uni(sh.scal[1]));
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (!isfinite(gf(k))) bad = true;
    return !team_any(sh, bad);
  };
  int nev = 1, st = MDHP_FIT_MAX_STEPS, s = 0, h = 0, head = 0;
  double l = 0.0, sy_new = 0.0, yy_new = 0.0;
  if (!evaluate()) {
    st = MDHP_FIT_NONFINITE;
    l = uni(sh.scal[0]);
  } else {
    l = uni(sh.scal[0]);
    float gk[K];  // gradient at the current point
#pragma unroll
    for (int k = 0; k < K; ++k) gk[k] = (float)gf(k);
    double f = -l * inv_n;
    for (s = 0;; ++s) {
      if (s == o.max_steps) {
        st = MDHP_FIT_MAX_STEPS;
        break;
      }
      // Current point (the LDS parameters) and active set: a slot is held
      // when it holds no parameter or sits at its bound with the gradient
      // pushing out.  Free gradient and its largest entry.
      float xk[K];
      unsigned act = 0;
      double qv[K], gmax_l = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        xk[k] = sl.get(sh, k);
        if (sl.kind(k) == 0 || (xk[k] <= lower(k) && gk[k] > 0.f)) act |= 1u << k;
        qv[k] = (act >> k) & 1 ? 0.0 : (double)gk[k];
        gmax_l = fmax(gmax_l, fabs(qv[k]));
      }
      const double gmax = team_max(sh, gmax_l);
      if (gmax == 0.0) {
        st = MDHP_FIT_CONVERGED;
        break;
      }
      const double gamma0 = 0.01 / gmax;
      const double gamma = h > 0 ? sy_new / yy_new : gamma0;
      for (int i = 0; i < h; ++i) {
        const int j = (head - 1 - i + m_hist) % m_hist;
        float sj[K], yj[K];  // both loads in flight together
#pragma unroll
        for (int k = 0; k < K; ++k) {
          sj[k] = wsp.ld(Ws::S(j), k);
          yj[k] = wsp.ld(Ws::Y(j), k);
        }
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) v += (double)sj[k] * qv[k];
        const double a = uni(sh.rho[j]) * team_sum(sh, v);
        if (t == 0) sh.alf[j] = a;
#pragma unroll
        for (int k = 0; k < K; ++k) qv[k] -= a * (double)yj[k];
      }
#pragma unroll
      for (int k = 0; k < K; ++k) qv[k] *= gamma;
      team_sync<NW>();
      for (int i = h - 1; i >= 0; --i) {
        const int j = (head - 1 - i + m_hist) % m_hist;
        float sj[K], yj[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          sj[k] = wsp.ld(Ws::S(j), k);
          yj[k] = wsp.ld(Ws::Y(j), k);
        }
        double v = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) v += (double)yj[k] * qv[k];
        const double bcoef = uni(sh.rho[j]) * team_sum(sh, v);
        const double a = uni(sh.alf[j]);
#pragma unroll
        for (int k = 0; k < K; ++k) qv[k] += (a - bcoef) * (double)sj[k];
      }
      float dk[K];
      double dg = 0.0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const double dd = (act >> k) & 1 ? 0.0 : -qv[k];
        dk[k] = (float)dd;
        dg += dd * (double)gk[k];
      }
      dg = team_sum(sh, dg);
      if (!(dg < 0.0)) {  // restart from scaled steepest descent
        h = 0;
#pragma unroll
        for (int k = 0; k < K; ++k)
          dk[k] = (act >> k) & 1 ? 0.f : (float)(-gamma0 * (double)gk[k]);
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        wsp.st(Ws::X, k, xk[k]);
        wsp.st(Ws::G, k, gk[k]);
        wsp.st(Ws::D, k, dk[k]);
      }
      // Backtracking line search on the projected path; every trial reads
      // x, g and d back from the workspace.
      double step = 1.0, ln = 0.0, fn = 0.0;
      bool ok = false;
      for (int ls = 0; ls < 20 && !ok; ++ls, step *= 0.5) {
        double dec = 0.0;
        team_sync<NW>();
#pragma unroll
        for (int k = 0; k < K; ++k) {
          if (sl.kind(k) == 0) continue;
          const float x0 = wsp.ld(Ws::X, k);
          const float xn = fmaxf((float)((double)x0 + step * (double)wsp.ld(Ws::D, k)), lower(k));
          sl.set(sh, k, xn);
          dec += (double)wsp.ld(Ws::G, k) * ((double)xn - (double)x0);
        }
        dec = team_sum(sh, dec);
        team_colsum(sh, M);
        const bool fin = evaluate();
        ++nev;
        ln = uni(sh.scal[0]);
        fn = -ln * inv_n;
        ok = fin && fn <= f + 1e-4 * dec;
      }
      if (!ok) {
        st = MDHP_FIT_STALLED;
        team_sync<NW>();
#pragma unroll
        for (int k = 0; k < K; ++k) sl.set(sh, k, wsp.ld(Ws::X, k));
        team_sync<NW>();
        break;
      }
      // New pair s = x' - x, y = g' - g; x' is the accepted point in LDS.
      double sy = 0.0, ss = 0.0, yy = 0.0;
      float sk[K], yk[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float gn = (float)gf(k);
        const float x0 = wsp.ld(Ws::X, k);
        const float xn = sl.kind(k) == 0 ? x0 : sl.get(sh, k);
        sk[k] = xn - x0;
        yk[k] = gn - wsp.ld(Ws::G, k);
        sy += (double)sk[k] * (double)yk[k];
        ss += (double)sk[k] * (double)sk[k];
        yy += (double)yk[k] * (double)yk[k];
        gk[k] = gn;
      }
      team_sum2(sh, sy, ss);
      yy = team_sum(sh, yy);
      if (sy > 1e-10 * sqrt(ss * yy)) {
        if (h == m_hist) h -= 1;  // the oldest pair drops out of the ring
#pragma unroll
        for (int k = 0; k < K; ++k) {
          wsp.st(Ws::S(head), k, sk[k]);
          wsp.st(Ws::Y(head), k, yk[k]);
        }
        if (t == 0) sh.rho[head] = 1.0 / sy;
        sy_new = sy;
        yy_new = yy;
        head = (head + 1) % m_hist;
        h += 1;
        team_sync<NW>();
      }
      const double l_prev = l;
      l = ln;
      f = fn;
      if (fabs(l - l_prev) <= o.ll_tol * fmax(fabs(l), (double)max(n, 1))) {
        st = MDHP_FIT_CONVERGED;
        s += 1;
        break;
      }
    }
  }
  team_store(sh, w, M, mu, alpha, beta);
  if (t == 0) {
    ll[w] = l;
    steps[w] = s;
    status[w] = st;
    if (evals_out) evals_out[w] = nev;
  }
}

template <int MP>
__global__ __launch_bounds__(kLpcBlock, kMinBlocksLpc) void lpc_lbfgs_kernel(Events ev, int M, FitParams o,
                                                           float* mu, float* alpha, float* beta,
                                                           double* ll, int* steps, int* status,
                                                           int* evals_out, float* ws,
                                                           int* counter) {
  __shared__ BlockLds<MP> lds;
  onehot_init<MP>();
  __syncthreads();
  float* blk = ws + (size_t)blockIdx.x * (size_t)block_ws<MP>();
  for_windows<MP>(
      lds, ev, counter,
      [&](Team<MP, kWaves>& sh, int64_t w) {
        lbfgs_one<MP, kWaves>(sh, ev, w, M, o, mu, alpha, beta, ll, steps, status, evals_out,
                              blk);
      },
      [&](Team<MP, 1>& sh, int64_t w) {
        lbfgs_one<MP, 1>(sh, ev, w, M, o, mu, alpha, beta, ll, steps, status, evals_out,
                         blk + (size_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) *
                                   (size_t)team_ws<MP, 1>());
      });
}

// Grid: enough workgroups for the big windows and the waves for the rest,
// at most what fits on the device at once.
template <class KERN>
int lpc_grid(KERN k, int64_t W, int64_t n_big) {
  const int64_t want = std::max<int64_t>(n_big, (W - n_big + kWaves - 1) / kWaves);
  return occupancy_grid(k, kLpcBlock, std::max<int64_t>(want, 1));
}

template <int MP>
hipError_t launch_lpc_eval(const Events& ev, int M, const float* mu, const float* alpha,
                           const float* beta, double* ll, float* g_mu, float* g_alpha,
                           float* g_beta, int* counter, hipStream_t s, bool grad) {
  if (ev.W == 0) return hipSuccess;
  reset_counter(counter, s);
  if (grad) {
    auto k = lpc_eval_kernel<MP, true>;
    hipLaunchKernelGGL(k, dim3(lpc_grid(k, ev.W, ev.n_big)), dim3(kLpcBlock), 0, s, ev, M, mu, alpha, beta, ll,
                       g_mu, g_alpha, g_beta, counter);
  } else {
    auto k = lpc_eval_kernel<MP, false>;
    hipLaunchKernelGGL(k, dim3(lpc_grid(k, ev.W, ev.n_big)), dim3(kLpcBlock), 0, s, ev, M, mu, alpha, beta, ll,
                       g_mu, g_alpha, g_beta, counter);
  }
  return hipGetLastError();
}

template <int MP>
hipError_t launch_lpc_fit(const Events& ev, int M, const FitParams& o, float* mu, float* alpha,
                          float* beta, double* ll, int* steps, int* status, int* evals, float* ws,
                          int64_t ws_floats, int* counter, hipStream_t s) {
  if (ev.W == 0) return hipSuccess;
  reset_counter(counter, s);
  if (o.optimizer == MDHP_OPT_LBFGS) {
    auto k = lpc_lbfgs_kernel<MP>;
    const int grid = (int)std::min<int64_t>(lpc_grid(k, ev.W, ev.n_big), ws_floats / block_ws<MP>());
    if (grid < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(grid), dim3(kLpcBlock), 0, s, ev, M, o, mu, alpha, beta, ll, steps,
                       status, evals, ws, counter);
    return hipGetLastError();
  }
  auto k = lpc_fit_kernel<MP>;
  hipLaunchKernelGGL(k, dim3(lpc_grid(k, ev.W, ev.n_big)), dim3(kLpcBlock), 0, s, ev, M, o, mu, alpha, beta, ll,
                     steps, status, evals, counter);
  return hipGetLastError();
}

template <int MP>
int64_t lpc_ws(int64_t W, int64_t n_big) {
  return block_ws<MP>() * lpc_grid(lpc_lbfgs_kernel<MP>, W, n_big);
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

int64_t lpc_lbfgs_workspace(int M, int64_t W, int64_t n_big) {
  switch (mp_for(M)) {
    case 4: return lpc_ws<4>(W, n_big);
    case 8: return lpc_ws<8>(W, n_big);
    default: return lpc_ws<16>(W, n_big);
  }
}

}  // namespace mdhp
