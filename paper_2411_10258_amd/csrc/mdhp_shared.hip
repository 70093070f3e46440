// Shared-decay (one beta per window) evaluation of the MDHP log-likelihood
// of Eq. (5) and its gradient, and the persistent projected-gradient fit.
//
// One workgroup (256 threads) owns one window at a time; windows are taken
// largest first from an atomic queue.  Lanes are grouped in groups of P
// lanes (P = M rounded up to a power of two, 4..64); lane n of a group holds
// component n of the decay state of its chunk of events:
//   R_n(i) = sum_{k: d_k = n, t_k < t_i} e^{-beta (t_i - t_k)}        (Part1's inner sum)
//   S_n(i) = sum_{k: d_k = n, t_k < t_i} (t_i - t_k) e^{-beta (t_i - t_k)}  (= -dR/dbeta)
// with the recursion R <- a (R + P), S <- a S + dt R, a = e^{-beta dt}, where
// P counts the events that share the previous time (they are folded in only
// when time moves on, so equal times never excite each other).
//
// Each group owns one contiguous chunk of the window (N / G events).  Pass 1
// computes every chunk's affine carry from a zero start, one event per lane
// (suffix sums of the gaps, one exponential per event, LDS atomics into the
// chunk's state); one group combines the carries in order (the scan of the
// (a, delta, b_R, b_S) monoid); pass 2 re-runs every chunk from its exact
// start state in batches of B events and accumulates, per event i with
// target m = d_i:
//   lambda_i = mu_m + sum_n alpha_mn R_n(i)          (Eq. (2) at t_i)
//   ll      += log lambda_i                          (Part1)
//   G_R[m][n] += R_n(i) / lambda_i                   (d ll / d alpha, Part1 share)
//   Gmu[m]  += 1 / lambda_i
//   Gb      += sum_n alpha_mn S_n(i) / lambda_i      (d ll / d beta, Part1 share)
// The compensator (Part2 + Part3, Appendix B) needs
//   E_n = sum_{k: d_k = n} e^{-beta (T - t_k)},  F_n = sum (T - t_k) e^{-beta (T - t_k)},
// which are the scan state advanced from the last event to T.
// Per-lane FP32 partial sums are reduced in FP64 at the end of the window.

#include <utility>

#include "mdhp_internal.h"

namespace mdhp {

namespace {

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// Sum over the P consecutive lanes of a group; every lane gets the sum.
template <int P>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (P >= 2) v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  if constexpr (P >= 4) v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  if constexpr (P >= 8) v += dpp<0x141>(v);  // row_half_mirror: the other quad of the 8
  if constexpr (P >= 16) v += dpp<0x140>(v); // row_mirror: the other 8 of the 16-lane row
  if constexpr (P >= 32) v += __shfl_xor(v, 16);
  if constexpr (P >= 64) v += __shfl_xor(v, 32);
  return v;
}

// Lane J of the caller's group, broadcast to the whole group (J < P).
template <int P, int J>
__device__ __forceinline__ float group_bcast(float x) {
  const int v = __builtin_bit_cast(int, x);
  int r;
  if constexpr (P == 4) r = __builtin_amdgcn_mov_dpp(v, J * 0x55, 0xF, 0xF, false);  // quad_perm [J,J,J,J]
  else if constexpr (P == 8) r = __builtin_amdgcn_ds_swizzle(v, 0x18 | (J << 5));      // (lane & 24) | J
  else if constexpr (P == 16) r = __builtin_amdgcn_mov_dpp(v, 0x150 + J, 0xF, 0xF, false);  // row_newbcast
  else if constexpr (P == 32) r = __builtin_amdgcn_ds_swizzle(v, J << 5);              // lane J of the 32
  else r = __builtin_amdgcn_readlane(v, J);
  return __builtin_bit_cast(float, r);
}

template <class F, int... Is>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}

// f(std::integral_constant<int, j>) for j = 0 .. N-1, fully unrolled.
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Inclusive prefix sum over the P lanes of a group (lane order).
template <int P>
__device__ __forceinline__ float group_scan(float v, int lane) {
#pragma unroll
  for (int k = 1; k < P; k <<= 1) {
    const float y = __shfl_up(v, k, P);
    if (lane >= k) v += y;
  }
  return v;
}

#ifndef MDHP_BATCH
#define MDHP_BATCH 16
#endif
// Events per pass-2 batch (at most the group size).
constexpr int kBatch = MDHP_BATCH;

template <int P>
struct SharedLds {
  static constexpr int G = kBlock / P;                 // groups (chunks) per tile
  static constexpr int NCOPY = P <= 32 ? kBlock / 64 : 1;  // G_R copies (one per wave if small)
  float alpha[P * P];  // alpha[m * P + n], zero outside M x M
  float mu[P];         // zero outside M
  float colsum[P];     // sum_m alpha_mn
  float cR[G][P], cS[G][P], cP[G][P];  // chunk carries, then chunk start states
  float cA[G], cD[G];
  int cF[G];
  float tR[P], tS[P], tP[P];  // state after the last event of the tiles done so far
  float gR[NCOPY][P * P];     // FP32 tile partials of G_R
  double red[4][kBlock];      // end-of-window reductions
  double Cn[P];               // (N_n - E_n) / beta
  double Fn[P];               // F_n
  double gmu[P];              // Gmu_m - T
  double scal[4];             // ll, g_beta, |sum| helpers
  float beta;
  int next_window;
  int stop;
};

// Evaluates one window with the parameters already in LDS (alpha, mu,
// colsum, beta).  Results: sh.scal[0] = ll, and if GRAD: gR64[k] holds
// G_R[e] for e = tid + k * kBlock (FP64), sh.Cn, sh.Fn, sh.gmu (= d ll/d mu),
// sh.scal[1] = d ll / d beta.
template <int P, bool GRAD>
__device__ void eval_window(SharedLds<P>& sh, const float* __restrict__ dtg,
                            const uint8_t* __restrict__ dg, int64_t begin, int n, double T,
                            float end_gap, int M, double (&gR64)[own_count(P)]) {
  constexpr int G = SharedLds<P>::G;
  constexpr int OWN = own_count(P);
  constexpr int B = kBatch < P ? kBatch : P;
  const int tid = threadIdx.x;
  const int lane = tid & (P - 1);
  const int grp = tid / P;
  float* gRc = sh.gR[SharedLds<P>::NCOPY > 1 ? (tid >> 6) : 0];
  const float beta = sh.beta;
  const float* __restrict__ dtw = dtg + begin;
  const uint8_t* __restrict__ dw = dg + begin;

  double ll64 = 0.0, gmu64 = 0.0, gb64 = 0.0;
  int cnt = 0;
  // Group g owns the contiguous chunk [j0, j1) of the window.
  const int c = (n + G - 1) / G;
  const int j0 = min(grp * c, n);
  const int len = min(j0 + c, n) - j0;

  // Pass 1: carry of this group's chunk from a zero start, one event per
  // lane.  An event at suffix time tau (sum of the later gaps of the chunk)
  // adds e^{-beta tau} to R and tau e^{-beta tau} to S of its dimension, or
  // counts as pending if no positive gap follows it (tau == 0); the chunk
  // decays everything before it by e^{-beta delta}, delta = sum of its gaps.
  {
    sh.cR[grp][lane] = 0.f;
    sh.cS[grp][lane] = 0.f;
    sh.cP[grp][lane] = 0.f;
    float later = 0.f;
    const int nsub = (c + P - 1) / P;
    int jr = (nsub - 1) * P + (P - 1 - lane);  // lanes run backwards through a sub-batch
    float dt_n = jr < len ? dtw[j0 + jr] : 0.f;
    int d_n = jr < len ? (int)dw[j0 + jr] : 0;
    for (int bb = nsub - 1; bb >= 0; --bb) {
      const bool valid = jr < len;
      const float dt = dt_n;
      const int d = d_n;
      jr -= P;
      if (bb > 0) {  // prefetch the previous sub-batch
        dt_n = jr < len ? dtw[j0 + jr] : 0.f;
        d_n = jr < len ? (int)dw[j0 + jr] : 0;
      }
      float prev = __shfl_up(dt, 1, P);  // gap of the next event (exclusive scan input)
      prev = lane == 0 ? 0.f : prev;
      const float tau = later + group_scan<P>(prev, lane);
      if (valid) {
        if (tau > 0.f) {
          const float e = __expf(-beta * tau);
          atomicAdd(&sh.cR[grp][d], e);
          atomicAdd(&sh.cS[grp][d], tau * e);
        } else {
          atomicAdd(&sh.cP[grp][d], 1.f);
        }
      }
      later += group_sum<P>(dt);
    }
    if (lane == 0) {
      sh.cA[grp] = __expf(-beta * later);
      sh.cD[grp] = later;
      sh.cF[grp] = later > 0.f ? 1 : 0;
    }
  }
  __syncthreads();
  // Ordered combine of the chunk carries: chunk g starts from the state
  // after chunks 0..g-1; the final state is the window's end state.
  if (grp == 0) {
    float R = 0.f, S = 0.f, Pn = 0.f;
    for (int g = 0; g < G; ++g) {
      const float Rg = sh.cR[g][lane], Sg = sh.cS[g][lane], Pg = sh.cP[g][lane];
      const float Ag = sh.cA[g], Dg = sh.cD[g];
      const int Fg = sh.cF[g];
      sh.cR[g][lane] = R;
      sh.cS[g][lane] = S;
      sh.cP[g][lane] = Pn;
      if (Fg) {
        const float X = R + Pn;
        R = fmaf(Ag, X, Rg);
        S = fmaf(Ag, fmaf(Dg, X, S), Sg);
        Pn = Pg;
      } else {
        Pn += Pg;
      }
    }
    sh.tR[lane] = R;
    sh.tS[lane] = S;
    sh.tP[lane] = Pn;
  }
  __syncthreads();
  // Pass 2: exact states, intensities and gradient sums, B events per
  // batch: the recurrence runs over the batch with the gaps, decays and
  // dims broadcast from the lane that loaded them, the B intensity sums are
  // independent group reductions, and lane j takes log and reciprocal of
  // lambda_j for the whole group.
  {
    float R = sh.cR[grp][lane], S = sh.cS[grp][lane], Pn = sh.cP[grp][lane];
    float llp = 0.f, gmup = 0.f, gbp = 0.f;
    const int nb = (c + B - 1) / B;
    int jl = lane & (B - 1);
    float dt_n = jl < len ? dtw[j0 + jl] : 0.f;
    int d_n = jl < len ? (int)dw[j0 + jl] : 0;
    for (int bb = 0; bb < nb; ++bb) {
      const bool vl = jl < len;
      const float dt_l = dt_n;
      const float d_l = __builtin_bit_cast(float, d_n);
      const int nvalid = min(B, len - bb * B);  // valid events of this batch (may be <= 0)
      jl += B;
      if (bb + 1 < nb) {  // prefetch the next batch
        dt_n = jl < len ? dtw[j0 + jl] : 0.f;
        d_n = jl < len ? (int)dw[j0 + jl] : 0;
      }
      const float a_l = __expf(-beta * dt_l);
      float Rj[B], Sj[B], Lj[B];
      int Dj[B];
      static_for<B>([&](auto J) {
        constexpr int j = decltype(J)::value;
        const float dt = group_bcast<P, j>(dt_l);
        const float a = group_bcast<P, j>(a_l);
        const int d = __builtin_bit_cast(int, group_bcast<P, j>(d_l));
        const bool f = dt > 0.f;
        const float X = f ? R + Pn : R;
        R = a * X;
        S = fmaf(a, S, dt * R);
        Pn = f ? 0.f : Pn;
        Rj[j] = R;
        Sj[j] = S;
        Dj[j] = d;
        Lj[j] = sh.alpha[d * P + lane] * R;
        const bool mine = j < nvalid && d == lane;
        Pn += mine ? 1.f : 0.f;
        cnt += mine ? 1 : 0;
      });
      static_for<B>([&](auto J) {
        constexpr int j = decltype(J)::value;
        Lj[j] = group_sum<P>(Lj[j]);
      });
      float lk = Lj[0];
      static_for<B>([&](auto J) {
        constexpr int j = decltype(J)::value;
        if (j > 0) lk = (lane & (B - 1)) == j ? Lj[j] : lk;
      });
      lk += sh.mu[__builtin_bit_cast(int, d_l)];
      const float lg = __logf(lk);
      llp += (vl && lane < B) ? lg : 0.f;
      if constexpr (GRAD) {
        const float wk = vl ? __builtin_amdgcn_rcpf(lk) : 0.f;
        static_for<B>([&](auto J) {
          constexpr int j = decltype(J)::value;
          const float w = group_bcast<P, j>(wk);  // zero for events past the chunk end
          atomicAdd(&gRc[Dj[j] * P + lane], w * Rj[j]);
          gbp = fmaf(w * sh.alpha[Dj[j] * P + lane], Sj[j], gbp);
          gmup += Dj[j] == lane ? w : 0.f;
        });
      }
    }
    ll64 += (double)llp;
    gmu64 += (double)gmup;
    gb64 += (double)gbp;
  }
#pragma unroll
  for (int k = 0; k < OWN; ++k) gR64[k] = 0.0;
  if constexpr (GRAD) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
      const int e = tid + k * kBlock;
      if (e < P * P) {
        float sum = 0.f;
#pragma unroll
        for (int cpy = 0; cpy < SharedLds<P>::NCOPY; ++cpy) {
          sum += sh.gR[cpy][e];
          sh.gR[cpy][e] = 0.f;
        }
        gR64[k] = (double)sum;
      }
    }
  }

  // End of window: reduce the per-lane partials over groups.
  __syncthreads();
  sh.red[0][tid] = ll64;
  sh.red[1][tid] = gmu64;
  sh.red[2][tid] = gb64;
  sh.red[3][tid] = (double)cnt;
  __syncthreads();
  if (tid < P) {
    double l = 0.0, gm = 0.0, gb = 0.0, nn = 0.0;
    for (int g = 0; g < G; ++g) {
      l += sh.red[0][g * P + tid];
      gm += sh.red[1][g * P + tid];
      gb += sh.red[2][g * P + tid];
      nn += sh.red[3][g * P + tid];
    }
    // Advance the end state to T: E_n and F_n of the compensator.
    const double gap = (double)end_gap;
    const double b = (double)beta;
    const double a = exp(-b * gap);
    const double E = a * ((double)sh.tR[tid] + (double)sh.tP[tid]);
    const double F = a * (double)sh.tS[tid] + gap * E;
    const double C = (nn - E) / b;
    const bool in = tid < M;
    sh.Cn[tid] = in ? C : 0.0;
    sh.Fn[tid] = in ? F : 0.0;
    sh.gmu[tid] = in ? gm - T : 0.0;
    // Per-lane pieces of the window sums, reduced below.
    sh.red[0][tid] = l;                                                     // Part1
    sh.red[1][tid] = in ? (double)sh.mu[tid] : 0.0;                         // sum mu
    sh.red[2][tid] = in ? (double)sh.colsum[tid] * C : 0.0;                 // Part3 (sign below)
    sh.red[3][tid] = in ? gb + (double)sh.colsum[tid] * (F - C) / b : 0.0;  // -d ll / d beta
  }
  __syncthreads();
  if (tid == 0) {
    double p1 = 0.0, smu = 0.0, p3 = 0.0, gbeta = 0.0;
    for (int k = 0; k < P; ++k) {
      p1 += sh.red[0][k];
      smu += sh.red[1][k];
      p3 += sh.red[2][k];
      gbeta += sh.red[3][k];
    }
    sh.scal[0] = p1 - T * smu - p3;
    sh.scal[1] = -gbeta;
  }
  __syncthreads();
}

template <int P>
__device__ void load_params(SharedLds<P>& sh, const float* __restrict__ mu,
                            const float* __restrict__ alpha, const float* __restrict__ beta,
                            int64_t w, int M) {
  const int tid = threadIdx.x;
  for (int e = tid; e < P * P; e += kBlock) {
    const int m = e / P, n = e % P;
    sh.alpha[e] = (m < M && n < M) ? alpha[(w * M + m) * M + n] : 0.f;
  }
  if (tid < P) sh.mu[tid] = tid < M ? mu[w * M + tid] : 0.f;
  if (tid == 0) sh.beta = beta[w];
  __syncthreads();
  if (tid < P) {
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += sh.alpha[m * P + tid];
    sh.colsum[tid] = s;
  }
  __syncthreads();
}

// LDS is not initialised at launch; the G_R tile accumulators must start at
// zero (eval_window leaves them zero after every tile).
template <int P>
__device__ void zero_accumulators(SharedLds<P>& sh) {
  for (int e = threadIdx.x; e < SharedLds<P>::NCOPY * P * P; e += kBlock) (&sh.gR[0][0])[e] = 0.f;
}

template <int P>
__device__ int next_window(SharedLds<P>& sh, int* counter, int first) {
  __syncthreads();
  if (threadIdx.x == 0) sh.next_window = first ? (int)blockIdx.x : atomicAdd(counter, 1) + (int)gridDim.x;
  __syncthreads();
  return sh.next_window;
}

template <int P, bool GRAD>
__global__ __launch_bounds__(kBlock) void shared_eval_kernel(Events ev, int M, const float* mu,
                                                             const float* alpha,
                                                             const float* beta, double* ll,
                                                             float* g_mu, float* g_alpha,
                                                             float* g_beta, int* counter) {
  __shared__ SharedLds<P> sh;
  constexpr int OWN = own_count(P);
  double gR64[OWN];
  const int tid = threadIdx.x;
  if constexpr (GRAD) zero_accumulators(sh);
  for (int q = next_window(sh, counter, 1); q < ev.W; q = next_window(sh, counter, 0)) {
    const int64_t w = ev.order[q];
    load_params(sh, mu, alpha, beta, w, M);
    const double T = ev.T[w];
    eval_window<P, GRAD>(sh, ev.dt, ev.d, ev.begin[w], ev.n[w], T, ev.end_gap[w], M, gR64);
    if (tid == 0) ll[w] = sh.scal[0];
    if constexpr (GRAD) {
      if (tid == 0) g_beta[w] = (float)sh.scal[1];
      if (tid < M) g_mu[w * M + tid] = (float)sh.gmu[tid];
#pragma unroll
      for (int k = 0; k < OWN; ++k) {
        const int e = tid + k * kBlock;
        const int m = e / P, n = e % P;
        if (e < P * P && m < M && n < M)
          g_alpha[(w * M + m) * M + n] = (float)(gR64[k] - sh.Cn[n]);
      }
    }
  }
}

// Persistent projected-gradient fit (see mdhp_fit_opts for the rule).
template <int P>
__global__ __launch_bounds__(kBlock) void shared_fit_kernel(Events ev, int M, FitParams o,
                                                            float* mu, float* alpha, float* beta,
                                                            double* ll, int* steps, int* status,
                                                            int* counter) {
  __shared__ SharedLds<P> sh;
  constexpr int OWN = own_count(P);
  double gR64[OWN];
  float m1a[OWN], m2a[OWN];
  const int tid = threadIdx.x;
  zero_accumulators(sh);
  for (int q = next_window(sh, counter, 1); q < ev.W; q = next_window(sh, counter, 0)) {
    const int64_t w = ev.order[q];
    load_params(sh, mu, alpha, beta, w, M);
    const int n = ev.n[w];
    const double T = ev.T[w];
    const double rate = (double)max(n, 1) / T;
    const double mu_min = o.mu_floor_rel * rate;
    const double beta_min = o.beta_floor_rel * rate;
    const double inv_n = 1.0 / (double)max(n, 1);
#pragma unroll
    for (int k = 0; k < OWN; ++k) m1a[k] = m2a[k] = 0.f;
    float m1mu = 0.f, m2mu = 0.f, m1b = 0.f, m2b = 0.f;
    double ll_prev = 0.0, b1t = 1.0, b2t = 1.0;
    int s = 0, st = MDHP_FIT_MAX_STEPS;
    for (s = 0;; ++s) {
      eval_window<P, true>(sh, ev.dt, ev.d, ev.begin[w], n, T, ev.end_gap[w], M, gR64);
      const double l = sh.scal[0];
      // Finiteness of ll and of the whole gradient (one flag per block).
      if (tid == 0) sh.stop = isfinite(l) && isfinite(sh.scal[1]) ? 0 : 1;
      __syncthreads();
      bool bad = false;
#pragma unroll
      for (int k = 0; k < OWN; ++k) {
        const int e = tid + k * kBlock;
        if (e < P * P && !isfinite(gR64[k])) bad = true;
      }
      if (tid < P && !isfinite(sh.gmu[tid])) bad = true;
      if (bad) atomicOr(&sh.stop, 1);
      __syncthreads();
      if (sh.stop) {
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
      auto step = [&](double g, float& m1, float& m2) -> double {
        const double gn = g * inv_n;
        if (o.optimizer == MDHP_OPT_PGD) return o.lr * gn;
        const double nm1 = o.b1 * (double)m1 + (1.0 - o.b1) * gn;
        const double nm2 = o.b2 * (double)m2 + (1.0 - o.b2) * gn * gn;
        m1 = (float)nm1;
        m2 = (float)nm2;
        return o.lr * (nm1 / bc1) / (sqrt(nm2 / bc2) + o.eps);
      };
#pragma unroll
      for (int k = 0; k < OWN; ++k) {
        const int e = tid + k * kBlock;
        const int m = e / P, nn = e % P;
        if (e < P * P && m < M && nn < M) {
          const double g = gR64[k] - sh.Cn[nn];
          const double v = (double)sh.alpha[e] + step(g, m1a[k], m2a[k]);
          sh.alpha[e] = (float)fmax(v, 0.0);
        }
      }
      if (tid < M) {
        const double v = (double)sh.mu[tid] + step(sh.gmu[tid], m1mu, m2mu);
        sh.mu[tid] = (float)fmax(v, mu_min);
      }
      if (tid == 0 && !o.fix_beta) {
        const double v = (double)sh.beta + step(sh.scal[1], m1b, m2b);
        sh.beta = (float)fmax(v, beta_min);
      }
      __syncthreads();
      if (tid < P) {
        float cs = 0.f;
        for (int m = 0; m < M; ++m) cs += sh.alpha[m * P + tid];
        sh.colsum[tid] = cs;
      }
      __syncthreads();
    }
    // theta_s of the last evaluation is in LDS.
    for (int e = tid; e < M * M; e += kBlock) alpha[w * M * M + e] = sh.alpha[(e / M) * P + e % M];
    if (tid < M) mu[w * M + tid] = sh.mu[tid];
    if (tid == 0) {
      beta[w] = sh.beta;
      ll[w] = sh.scal[0];
      steps[w] = s;
      status[w] = st;
    }
  }
}

template <class K>
int occupancy_grid(K kernel, int64_t W) {
  int dev = 0, cus = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0);
  int64_t g = (int64_t)std::max(cus, 1) * std::max(per_cu, 1);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, W));
}

template <int P>
hipError_t launch_shared_eval(const Events& ev, int M, const float* mu, const float* alpha,
                              const float* beta, double* ll, float* g_mu, float* g_alpha,
                              float* g_beta, int* counter, hipStream_t s, bool grad) {
  if (ev.W == 0) return hipSuccess;
  reset_counter(counter, s);
  if (grad) {
    auto k = shared_eval_kernel<P, true>;
    hipLaunchKernelGGL(k, dim3(occupancy_grid(k, ev.W)), dim3(kBlock), 0, s, ev, M, mu, alpha,
                       beta, ll, g_mu, g_alpha, g_beta, counter);
  } else {
    auto k = shared_eval_kernel<P, false>;
    hipLaunchKernelGGL(k, dim3(occupancy_grid(k, ev.W)), dim3(kBlock), 0, s, ev, M, mu, alpha,
                       beta, ll, g_mu, g_alpha, g_beta, counter);
  }
  return hipGetLastError();
}

template <int P>
hipError_t launch_shared_fit(const Events& ev, int M, const FitParams& o, float* mu,
                             float* alpha, float* beta, double* ll, int* steps, int* status,
                             int* counter, hipStream_t s) {
  if (ev.W == 0) return hipSuccess;
  reset_counter(counter, s);
  auto k = shared_fit_kernel<P>;
  hipLaunchKernelGGL(k, dim3(occupancy_grid(k, ev.W)), dim3(kBlock), 0, s, ev, M, o, mu, alpha,
                     beta, ll, steps, status, counter);
  return hipGetLastError();
}

}  // namespace

hipError_t shared_eval(const Events& ev, int M, const float* mu, const float* alpha,
                       const float* beta, double* ll, float* g_mu, float* g_alpha, float* g_beta,
                       int* counter, hipStream_t s, bool grad) {
  switch (lanes_for(M)) {
    case 4: return launch_shared_eval<4>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
    case 8: return launch_shared_eval<8>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
    case 16: return launch_shared_eval<16>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
    case 32: return launch_shared_eval<32>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
    default: return launch_shared_eval<64>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
  }
}

hipError_t shared_fit(const Events& ev, int M, const FitParams& o, float* mu, float* alpha,
                      float* beta, double* ll, int* steps, int* status, int* counter,
                      hipStream_t s) {
  switch (lanes_for(M)) {
    case 4: return launch_shared_fit<4>(ev, M, o, mu, alpha, beta, ll, steps, status, counter, s);
    case 8: return launch_shared_fit<8>(ev, M, o, mu, alpha, beta, ll, steps, status, counter, s);
    case 16: return launch_shared_fit<16>(ev, M, o, mu, alpha, beta, ll, steps, status, counter, s);
    case 32: return launch_shared_fit<32>(ev, M, o, mu, alpha, beta, ll, steps, status, counter, s);
    default: return launch_shared_fit<64>(ev, M, o, mu, alpha, beta, ll, steps, status, counter, s);
  }
}

}  // namespace mdhp
