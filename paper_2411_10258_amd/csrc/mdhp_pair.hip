// Per-pair decays (beta_mn for every target m and source n; the (D, D) beta
// of Sec. IV-B): evaluation of the log-likelihood of Eq. (5), its gradient
// with respect to mu, alpha and every beta_mn, and the persistent fit.
//
// With a decay per pair, R_mn(i) = sum_{k: d_k = n, t_k < t_i}
// e^{-beta_mn (t_i - t_k)} no longer shares one decay across a row, so the
// full M x M state would need M^2 exponentials per event.  Instead each
// chunk keeps the state column by column, decayed lazily: column n is held
// as of the last source-n event (Rt[n][m], St[n][m]) together with the time
// z_n elapsed since then and the number c_n of source-n events at that time.
// An event with dimension d costs two exponentials per lane:
//   * row read for target m = d (lane = source n):
//       R_mn = e^{-beta_mn z_n} Rt[n][m] - (z_n == 0 ? c_n : 0)
//       S_mn = e^{-beta_mn z_n} (St[n][m] + z_n Rt[n][m])
//     (events at the current time are excluded: the sums of Eq. (2) run over
//     strictly earlier times);
//   * column update for source n = d (lane = target m):
//       Rt[d][m] <- e^{-beta_md z_d} Rt[d][m] + 1,
//       St[d][m] <- e^{-beta_md z_d} (St[d][m] + z_d Rt[d][m]),  z_d <- 0.
// The state lives in LDS with a padded stride (P + 1) so that both the row
// read (lanes across n) and the column update (lanes across m) are free of
// bank conflicts.
//
// Chunks, carries and the ordered combine follow the shared-decay kernel,
// with the carry's decay taken per pair: A_mn = e^{-beta_mn delta}.

#include "mdhp_device.h"

namespace mdhp {

namespace {

template <int P>
struct PairCfg {
  static constexpr int Q = P + 1;                      // padded stride
  static constexpr int THREADS = P <= 16 ? 256 : 128;  // workgroup size
  static constexpr int G = THREADS / P;                // chunks per window
  static constexpr int OWN = (P * P + THREADS - 1) / THREADS;
  static constexpr int B = P < 16 ? P : 16;            // events per loaded batch
};

template <int P>
struct PairLds {
  using C = PairCfg<P>;
  static constexpr int Q = C::Q, G = C::G;
  float alpha[P * Q];  // [m * Q + n], zero outside M x M
  float beta[P * Q];   // [m * Q + n], one outside M x M
  float mu[P];
  float Rs[G][P * Q];  // chunk state, column-major [n * Q + m]
  float Ss[G][P * Q];
  float Pl[G][P];      // pending events per source column at the chunk end
  float Ps[G][P];      // pending events per source column at the chunk start
  float cnt[G][P];     // events per source dimension in the chunk
  float cD[G];
  int cF[G];
  float gR[P * Q];  // FP32 sums of R_mn / lambda over target-m events, [m * Q + n]
  float gS[P * Q];  // same for S_mn
  double Cmn[P * P];  // (N_n - E_mn) / beta_mn, [m * P + n]
  double Fmn[P * P];  // F_mn = sum_{k: d_k = n} (T - t_k) e^{-beta_mn (T - t_k)}
  double red[2][C::THREADS];
  double gmu[P];
  double scal[2];
  int next_window;
  int stop;
};

template <int P>
__device__ __forceinline__ void column_update(PairLds<P>& sh, float* Rs, float* Ss, int lane,
                                              int d, float& z, float& cn) {
  constexpr int Q = PairCfg<P>::Q;
  const float zd = __shfl(z, d, P);
  const int a = d * Q + lane;
  const float Rt = Rs[a];
  const float St = Ss[a];
  if (zd > 0.f) {
    const float e = __expf(-sh.beta[lane * Q + d] * zd);
    Rs[a] = fmaf(e, Rt, 1.f);
    Ss[a] = e * fmaf(zd, Rt, St);
  } else {
    Rs[a] = Rt + 1.f;
  }
  if (lane == d) {
    cn = zd > 0.f ? 1.f : cn + 1.f;
    z = 0.f;
  }
}

// Evaluates one window with parameters in LDS.  Results: sh.scal[0] = ll;
// if GRAD also sh.gR / sh.gS (FP32 sums), sh.Cmn, sh.Fmn, sh.gmu.
template <int P, bool GRAD>
__device__ __forceinline__ void eval_window_pair(PairLds<P>& sh, const float* __restrict__ dtg,
                                 const uint8_t* __restrict__ dg, int64_t begin, int n, double T,
                                 float end_gap, int M) {
  using C = PairCfg<P>;
  constexpr int Q = C::Q, G = C::G, B = C::B;
  const int tid = threadIdx.x;
  const int lane = tid & (P - 1);
  const int grp = tid / P;
  const float* __restrict__ dtw = dtg + begin;
  const uint8_t* __restrict__ dw = dg + begin;
  float* Rs = sh.Rs[grp];
  float* Ss = sh.Ss[grp];
  const int c = (n + G - 1) / G;
  const int j0 = min(grp * c, n);
  const int len = min(j0 + c, n) - j0;
  const int nb = (len + B - 1) / B;  // uniform within a group

  // Pass 1: zero-start state of this chunk, column updates only.
  for (int e = lane; e < P * Q; e += P) {
    Rs[e] = 0.f;
    Ss[e] = 0.f;
  }
  float z = 0.f, cn = 0.f, count = 0.f, delta = 0.f;
  for (int bb = 0; bb < nb; ++bb) {
    const int jl = bb * B + (lane & (B - 1));
    const float dt_l = jl < len ? dtw[j0 + jl] : 0.f;
    const float d_l = __builtin_bit_cast(float, jl < len ? (int)dw[j0 + jl] : 0);
    const int nv = min(B, len - bb * B);
    static_for<B>([&](auto J) {
      constexpr int j = decltype(J)::value;
      if (j < nv) {
        const float dt = group_bcast<P, j>(dt_l);
        const int d = __builtin_bit_cast(int, group_bcast<P, j>(d_l));
        z += dt;
        delta += dt;
        count += lane == d ? 1.f : 0.f;
        column_update<P>(sh, Rs, Ss, lane, d, z, cn);
      }
    });
  }
  // Lazy columns -> full state at the chunk's last event (lane = column n).
  for (int m = 0; m < P; ++m) {
    const int a = lane * Q + m;
    const float e = __expf(-sh.beta[m * Q + lane] * z);
    const float Rt = Rs[a];
    Rs[a] = e * Rt - (z == 0.f ? cn : 0.f);
    Ss[a] = e * fmaf(z, Rt, Ss[a]);
  }
  sh.Pl[grp][lane] = z == 0.f ? cn : 0.f;
  sh.cnt[grp][lane] = count;
  if (lane == 0) {
    sh.cD[grp] = delta;
    sh.cF[grp] = delta > 0.f ? 1 : 0;
  }
  __syncthreads();
  // Ordered combine over chunks, one pair (m, n) per thread slot; chunk g's
  // slot is overwritten with its start state.  The end state gives the
  // compensator sums E_mn, F_mn.
  for (int e = tid; e < P * P; e += C::THREADS) {
    const int m = e / P, nn = e % P;
    const int a = nn * Q + m;
    const float b = sh.beta[m * Q + nn];
    float R = 0.f, S = 0.f, Pc = 0.f, Ntot = 0.f;
    for (int g = 0; g < G; ++g) {
      const float Rl = sh.Rs[g][a], Sl = sh.Ss[g][a], Pg = sh.Pl[g][nn];
      const float D = sh.cD[g];
      sh.Rs[g][a] = R;
      sh.Ss[g][a] = S;
      if (m == 0) sh.Ps[g][nn] = Pc;
      Ntot += sh.cnt[g][nn];
      if (sh.cF[g]) {
        const float A = __expf(-b * D);
        const float X = R + Pc;
        R = fmaf(A, X, Rl);
        S = fmaf(A, fmaf(D, X, S), Sl);
        Pc = Pg;
      } else {
        Pc += Pg;
      }
    }
    const double gap = (double)end_gap, bd = (double)b;
    const double ad = exp(-bd * gap);
    const double E = ad * ((double)R + (double)Pc);
    const double F = ad * (double)S + gap * E;
    const bool in = m < M && nn < M;
    sh.Cmn[m * P + nn] = in ? ((double)Ntot - E) / bd : 0.0;
    sh.Fmn[m * P + nn] = in ? F : 0.0;
  }
  __syncthreads();
  // Pass 2: from the exact chunk start, row reads (intensity, gradient
  // sums) and column updates.
  {
    const float pend = sh.Ps[grp][lane];
    for (int m = 0; m < P; ++m) Rs[lane * Q + m] += pend;  // pending events enter at weight 1
    z = 0.f;
    cn = pend;
    float llp = 0.f, gmup = 0.f;
    for (int bb = 0; bb < nb; ++bb) {
      const int jl = bb * B + (lane & (B - 1));
      const float dt_l = jl < len ? dtw[j0 + jl] : 0.f;
      const float d_l = __builtin_bit_cast(float, jl < len ? (int)dw[j0 + jl] : 0);
      const int nv = min(B, len - bb * B);
      static_for<B>([&](auto J) {
        constexpr int j = decltype(J)::value;
        if (j < nv) {
          const float dt = group_bcast<P, j>(dt_l);
          const int d = __builtin_bit_cast(int, group_bcast<P, j>(d_l));
          z += dt;
          // Row read for target d (lane = source n).
          const int a = lane * Q + d;
          const float Rt = Rs[a];
          const float St = Ss[a];
          const float e = __expf(-sh.beta[d * Q + lane] * z);
          const float R = e * Rt - (z == 0.f ? cn : 0.f);
          const float S = e * fmaf(z, Rt, St);
          const float al = sh.alpha[d * Q + lane];
          const float lam = group_sum<P>(al * R) + sh.mu[d];
          llp += lane == 0 ? __logf(lam) : 0.f;
          if constexpr (GRAD) {
            const float w = __builtin_amdgcn_rcpf(lam);
            atomicAdd(&sh.gR[d * Q + lane], w * R);
            atomicAdd(&sh.gS[d * Q + lane], w * S);
            gmup += lane == d ? w : 0.f;
          }
          column_update<P>(sh, Rs, Ss, lane, d, z, cn);
        }
      });
    }
    sh.red[0][tid] = (double)llp;
    sh.red[1][tid] = (double)gmup;
  }
  __syncthreads();
  if (tid < P) {
    double l = 0.0, gm = 0.0;
    for (int g = 0; g < G; ++g) {
      l += sh.red[0][g * P + tid];
      gm += sh.red[1][g * P + tid];
    }
    sh.gmu[tid] = tid < M ? gm - T : 0.0;
    sh.red[0][tid] = l;
    sh.red[1][tid] = tid < M ? (double)sh.mu[tid] : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    double p1 = 0.0, smu = 0.0, p3 = 0.0;
    for (int k = 0; k < P; ++k) {
      p1 += sh.red[0][k];
      smu += sh.red[1][k];
    }
    for (int e = 0; e < P * P; ++e) p3 += (double)sh.alpha[(e / P) * Q + e % P] * sh.Cmn[e];
    sh.scal[0] = p1 - T * smu - p3;
  }
  __syncthreads();
}

template <int P>
__device__ void load_params_pair(PairLds<P>& sh, const float* __restrict__ mu,
                                 const float* __restrict__ alpha, const float* __restrict__ beta,
                                 int64_t w, int M) {
  constexpr int Q = PairCfg<P>::Q;
  for (int e = threadIdx.x; e < P * P; e += PairCfg<P>::THREADS) {
    const int m = e / P, n = e % P;
    const bool in = m < M && n < M;
    sh.alpha[m * Q + n] = in ? alpha[(w * M + m) * M + n] : 0.f;
    sh.beta[m * Q + n] = in ? beta[(w * M + m) * M + n] : 1.f;
  }
  if (threadIdx.x < P) sh.mu[threadIdx.x] = threadIdx.x < M ? mu[w * M + threadIdx.x] : 0.f;
  __syncthreads();
}

template <int P>
__device__ int next_window_pair(PairLds<P>& sh, int* counter, int first) {
  __syncthreads();
  if (threadIdx.x == 0)
    sh.next_window = first ? (int)blockIdx.x : atomicAdd(counter, 1) + (int)gridDim.x;
  __syncthreads();
  return sh.next_window;
}

template <int P>
__device__ void zero_pair_accumulators(PairLds<P>& sh) {
  for (int e = threadIdx.x; e < P * PairCfg<P>::Q; e += PairCfg<P>::THREADS) {
    sh.gR[e] = 0.f;
    sh.gS[e] = 0.f;
  }
}

template <int P, bool GRAD>
__global__ __launch_bounds__(PairCfg<P>::THREADS) void pair_eval_kernel(
    Events ev, int M, const float* mu, const float* alpha, const float* beta, double* ll,
    float* g_mu, float* g_alpha, float* g_beta, int* counter) {
  __shared__ PairLds<P> sh;
  constexpr int Q = PairCfg<P>::Q;
  const int tid = threadIdx.x;
  zero_pair_accumulators(sh);
  for (int q = next_window_pair(sh, counter, 1); q < ev.W; q = next_window_pair(sh, counter, 0)) {
    const int64_t w = ev.order[q];
    load_params_pair(sh, mu, alpha, beta, w, M);
    const double T = ev.T[w];
    eval_window_pair<P, GRAD>(sh, ev.dt, ev.d, ev.begin[w], ev.n[w], T, ev.end_gap[w], M);
    if (tid == 0) ll[w] = sh.scal[0];
    if constexpr (GRAD) {
      if (tid < M) g_mu[w * M + tid] = (float)sh.gmu[tid];
      for (int e = tid; e < P * P; e += PairCfg<P>::THREADS) {
        const int m = e / P, n = e % P;
        const double C = sh.Cmn[e], F = sh.Fmn[e];
        const double gR = (double)sh.gR[m * Q + n], gS = (double)sh.gS[m * Q + n];
        sh.gR[m * Q + n] = 0.f;
        sh.gS[m * Q + n] = 0.f;
        if (m < M && n < M) {
          const double a = (double)sh.alpha[m * Q + n], b = (double)sh.beta[m * Q + n];
          g_alpha[(w * M + m) * M + n] = (float)(gR - C);
          g_beta[(w * M + m) * M + n] = (float)(-a * (gS + (F - C) / b));
        }
      }
    }
  }
}

// Persistent projected-gradient fit with per-pair decays.
template <int P>
__global__ __launch_bounds__(PairCfg<P>::THREADS) void pair_fit_kernel(
    Events ev, int M, FitParams o, float* mu, float* alpha, float* beta, double* ll, int* steps,
    int* status, int* evals_out, int* counter) {
  __shared__ PairLds<P> sh;
  using C = PairCfg<P>;
  constexpr int Q = C::Q, OWN = C::OWN;
  const int tid = threadIdx.x;
  float m1a[OWN], m2a[OWN], m1b[OWN], m2b[OWN];
  zero_pair_accumulators(sh);
  for (int q = next_window_pair(sh, counter, 1); q < ev.W; q = next_window_pair(sh, counter, 0)) {
    const int64_t w = ev.order[q];
    load_params_pair(sh, mu, alpha, beta, w, M);
    const int n = ev.n[w];
    const double T = ev.T[w];
    const double rate = (double)max(n, 1) / T;
    const double mu_min = o.mu_floor_rel * rate;
    const double beta_min = o.beta_floor_rel * rate;
    const double inv_n = 1.0 / (double)max(n, 1);
#pragma unroll
    for (int k = 0; k < OWN; ++k) m1a[k] = m2a[k] = m1b[k] = m2b[k] = 0.f;
    float m1mu = 0.f, m2mu = 0.f;
    double ll_prev = 0.0, b1t = 1.0, b2t = 1.0;
    int s = 0, st = MDHP_FIT_MAX_STEPS;
    for (s = 0;; ++s) {
      eval_window_pair<P, true>(sh, ev.dt, ev.d, ev.begin[w], n, T, ev.end_gap[w], M);
      const double l = sh.scal[0];
      // Gradient of the owned pairs (and reset of the FP32 sums).
      double ga[OWN], gb[OWN];
      bool bad = false;
#pragma unroll
      for (int k = 0; k < OWN; ++k) {
        const int e = tid + k * C::THREADS;
        ga[k] = gb[k] = 0.0;
        if (e < P * P) {
          const int m = e / P, nn = e % P;
          const double Cv = sh.Cmn[e], F = sh.Fmn[e];
          const double gR = (double)sh.gR[m * Q + nn], gS = (double)sh.gS[m * Q + nn];
          sh.gR[m * Q + nn] = 0.f;
          sh.gS[m * Q + nn] = 0.f;
          const double a = (double)sh.alpha[m * Q + nn], b = (double)sh.beta[m * Q + nn];
          ga[k] = gR - Cv;
          gb[k] = -a * (gS + (F - Cv) / b);
          if (!isfinite(ga[k]) || !isfinite(gb[k])) bad = true;
        }
      }
      if (tid < P && !isfinite(sh.gmu[tid])) bad = true;
      if (tid == 0) sh.stop = isfinite(l) ? 0 : 1;
      __syncthreads();
      if (bad) atomicOr(&sh.stop, 1);
      __syncthreads();
      if (sh.stop) {
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
      auto step = [&](double g, float& m1, float& m2) -> double {
        const double gn = g * inv_n;
        if (o.optimizer == MDHP_OPT_PGD) return o.lr * gn;
        const double nm1 = o.b1 * (double)m1 + (1.0 - o.b1) * gn;
        const double nm2 = o.b2 * (double)m2 + (1.0 - o.b2) * gn * gn;
        m1 = (float)nm1;
        m2 = (float)nm2;
        return o.lr * (nm1 / bc1) / (sqrt(nm2 / bc2) + o.eps);
      };
      // alpha, beta of the owned pairs and mu; the new values are written
      // after everyone has read the old ones for the gradient above.
      float na[OWN], nbv[OWN];
#pragma unroll
      for (int k = 0; k < OWN; ++k) {
        const int e = tid + k * C::THREADS;
        na[k] = nbv[k] = 0.f;
        if (e < P * P) {
          const int m = e / P, nn = e % P;
          if (m < M && nn < M) {
            na[k] = (float)fmax((double)sh.alpha[m * Q + nn] + step(ga[k], m1a[k], m2a[k]), 0.0);
            nbv[k] = o.fix_beta ? sh.beta[m * Q + nn]
                                : (float)fmax((double)sh.beta[m * Q + nn] +
                                                  step(gb[k], m1b[k], m2b[k]),
                                              beta_min);
          }
        }
      }
      float nmu = 0.f;
      if (tid < M) nmu = (float)fmax((double)sh.mu[tid] + step(sh.gmu[tid], m1mu, m2mu), mu_min);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < OWN; ++k) {
        const int e = tid + k * C::THREADS;
        if (e < P * P) {
          const int m = e / P, nn = e % P;
          if (m < M && nn < M) {
            sh.alpha[m * Q + nn] = na[k];
            sh.beta[m * Q + nn] = nbv[k];
          }
        }
      }
      if (tid < M) sh.mu[tid] = nmu;
      __syncthreads();
    }
    // The FP32 sums of the last evaluation are still in LDS when the loop
    // stops before reading them; clear them for the next window.
    __syncthreads();
    for (int e = tid; e < P * Q; e += C::THREADS) {
      sh.gR[e] = 0.f;
      sh.gS[e] = 0.f;
    }
    for (int e = tid; e < M * M; e += C::THREADS) {
      const int m = e / M, nn = e % M;
      alpha[w * M * M + e] = sh.alpha[m * Q + nn];
      beta[w * M * M + e] = sh.beta[m * Q + nn];
    }
    if (tid < M) mu[w * M + tid] = sh.mu[tid];
    if (tid == 0) {
      ll[w] = sh.scal[0];
      steps[w] = s;
      status[w] = st;
      if (evals_out) evals_out[w] = s + 1;
    }
  }
}

template <int P>
hipError_t launch_pair_eval(const Events& ev, int M, const float* mu, const float* alpha,
                            const float* beta, double* ll, float* g_mu, float* g_alpha,
                            float* g_beta, int* counter, hipStream_t s, bool grad) {
  if (ev.W == 0) return hipSuccess;
  constexpr int TH = PairCfg<P>::THREADS;
  reset_counter(counter, s);
  if (grad) {
    auto k = pair_eval_kernel<P, true>;
    hipLaunchKernelGGL(k, dim3(occupancy_grid(k, TH, ev.W)), dim3(TH), 0, s, ev, M, mu, alpha,
                       beta, ll, g_mu, g_alpha, g_beta, counter);
  } else {
    auto k = pair_eval_kernel<P, false>;
    hipLaunchKernelGGL(k, dim3(occupancy_grid(k, TH, ev.W)), dim3(TH), 0, s, ev, M, mu, alpha,
                       beta, ll, g_mu, g_alpha, g_beta, counter);
  }
  return hipGetLastError();
}

template <int P>
hipError_t launch_pair_fit(const Events& ev, int M, const FitParams& o, float* mu, float* alpha,
                           float* beta, double* ll, int* steps, int* status, int* evals,
                           int* counter, hipStream_t s) {
  if (ev.W == 0) return hipSuccess;
  constexpr int TH = PairCfg<P>::THREADS;
  reset_counter(counter, s);
  auto k = pair_fit_kernel<P>;
  hipLaunchKernelGGL(k, dim3(occupancy_grid(k, TH, ev.W)), dim3(TH), 0, s, ev, M, o, mu, alpha,
                     beta, ll, steps, status, evals, counter);
  return hipGetLastError();
}

}  // namespace

hipError_t pair_eval(const Events& ev, int M, const float* mu, const float* alpha,
                     const float* beta, double* ll, float* g_mu, float* g_alpha, float* g_beta,
                     int* counter, hipStream_t s, bool grad) {
  switch (lanes_for(M)) {
    case 4: return launch_pair_eval<4>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
    case 8: return launch_pair_eval<8>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
    case 16: return launch_pair_eval<16>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
    case 32: return launch_pair_eval<32>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
    default: return hipErrorInvalidValue;
  }
}

hipError_t pair_fit(const Events& ev, int M, const FitParams& o, float* mu, float* alpha,
                    float* beta, double* ll, int* steps, int* status, int* evals, int* counter,
                    hipStream_t s) {
  switch (lanes_for(M)) {
    case 4: return launch_pair_fit<4>(ev, M, o, mu, alpha, beta, ll, steps, status, evals, counter, s);
    case 8: return launch_pair_fit<8>(ev, M, o, mu, alpha, beta, ll, steps, status, evals, counter, s);
    case 16: return launch_pair_fit<16>(ev, M, o, mu, alpha, beta, ll, steps, status, evals, counter, s);
    case 32: return launch_pair_fit<32>(ev, M, o, mu, alpha, beta, ll, steps, status, evals, counter, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mdhp
