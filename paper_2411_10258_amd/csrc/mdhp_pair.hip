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

constexpr float kLog2e = 1.44269504088896340736f;

template <int P>
struct PairCfg {
  static constexpr int Q = P + 1;                      // padded stride
  static constexpr int THREADS = 256;                  // workgroup size
  static constexpr int G = THREADS / P;                // chunks per window
  static constexpr int OWN = (P * P + THREADS - 1) / THREADS;
  static constexpr int B = P < 16 ? P : 16;            // events per loaded batch
  static constexpr int WAVES = THREADS / 64;
};

// LDS of one workgroup.  At P = 32 the eight chunks' states and gradient
// sums take 132 KB; the rest is kept small enough for the whole to fit in
// one CU's 160 KB.
template <int P>
struct PairLds {
  using C = PairCfg<P>;
  static constexpr int Q = C::Q, G = C::G;
  float alpha[P * Q];  // [m * Q + n], zero outside M x M
  float nbeta[P * Q];  // -beta_mn log2(e), the exponent scale of exp2 (beta one outside M x M)
  float mu[P];
  float Rs[G][P * Q];  // chunk state, column-major [n * Q + m]
  float Ss[G][P * Q];
  float Pl[G][P];      // pending events per source column at the chunk end
  float Ps[G][P];      // pending events per source column at the chunk start
  float cnt[G][P];     // events per source dimension in the chunk
  float cD[G];
  int cF[G];
  float gR[G][P * Q];  // per chunk, FP32 sums of R_mn / lambda over target-m events, [m * Q + n]
  float gS[G][P * Q];  // same for S_mn
  float red[2][C::THREADS];  // per-lane sums of a chunk: log2 lambda, 1/lambda
  double gmu[P];
  double wsum[C::WAVES];
  double scal[2];
  int next_window;
  int stop;
};

// The pairs a thread owns, e = tid + k THREADS < P^2 (m = e / P, n = e % P),
// with their exact decay and compensator sums in registers.
template <int P>
struct PairOwn {
  static constexpr int OWN = PairCfg<P>::OWN;
  float beta[OWN];   // beta_mn (one outside M x M)
  double C[OWN];     // (N_n - E_mn) / beta_mn
  double F[OWN];     // F_mn = sum_{k: d_k = n} (T - t_k) e^{-beta_mn (T - t_k)}
};

// Event J of the loaded batch, to every lane of the group.  At P = 32 the
// batch is held once per 16-lane row of the group, so a row broadcast does.
template <int P, int J>
__device__ __forceinline__ float batch_bcast(float x) {
  if constexpr (P == 32)
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x),
                                                              0x150 + J, 0xF, 0xF, false));
  else
    return group_bcast<P, J>(x);
}

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// One event of a chunk as a lane sees it: the dimension d, the lane's
// elapsed time z and pending count c before the event (row read), the
// elapsed time zd of column d (column update) and the LDS values both read.
struct PairEvent {
  int d, ac;        // ac = d * Q + lane: column d's entry for target lane, also (d, lane) of alpha/beta
  float z, c, zd, inc, ok;
  float Rrow, Srow, brow, arow, mud;  // row read: column lane, target d
  float Rcol, Scol, bcol;             // column update: column d, target lane
};

// Advances the lane's lazy clock to event J of the batch and issues every
// LDS read the event needs.  Events past the chunk's end (J >= nv) are null:
// no elapsed time, no count, no contribution.  FULL: the whole batch is
// inside every chunk of the wavefront (no null events; the checks fold).
template <int P, int J, bool FULL>
__device__ __forceinline__ PairEvent pair_issue(PairLds<P>& sh, const float* Rs, const float* Ss,
                                                int lane, float dt_l, int d_l, float g_l, int nv,
                                                float& z, float& cn, float& dl) {
  constexpr int Q = PairCfg<P>::Q;
  PairEvent e;
  const int d = __builtin_bit_cast(int, batch_bcast<P, J>(__builtin_bit_cast(float, d_l)));
  const int ar = lane * Q + d;
  e.d = d;
  e.ac = d * Q + lane;
  e.Rcol = Rs[e.ac];
  e.Scol = Ss[e.ac];
  e.bcol = sh.nbeta[ar];
  e.Rrow = Rs[ar];
  e.Srow = Ss[ar];
  e.brow = sh.nbeta[e.ac];
  e.arow = sh.alpha[e.ac];
  e.mud = sh.mu[d];
  // The reads above stay ahead of the previous event's remaining work.
  __builtin_amdgcn_sched_barrier(0);
  const float dt = batch_bcast<P, J>(dt_l);
  const bool ok = FULL || J < nv;
  z += dt;
  dl += dt;
  // Column d's elapsed time: since the previous source-d event, or since the
  // chunk's start if that event lies before it.
  const float zd = fminf(batch_bcast<P, J>(g_l), dl);
  e.z = z;
  e.c = cn;
  e.zd = ok ? zd : 0.f;
  e.inc = ok ? 1.f : 0.f;
  e.ok = e.inc;
  // The lane's own column restarts its clock (arithmetic, not a branch).
  const float own = (ok && lane == d) ? 1.f : 0.f;
  const float ncn = zd > 0.f ? 1.f : cn + 1.f;
  cn = fmaf(own, ncn - cn, cn);
  z = fmaf(-own, z, z);
  return e;
}

// Column update of source d for target lane: the column decays to the
// event's time and gains the event (a null event writes the same values).
__device__ __forceinline__ void pair_column(float* Rs, float* Ss, const PairEvent& e) {
  const float ec = exp2_fast(e.bcol * e.zd);
  Rs[e.ac] = fmaf(ec, e.Rcol, e.inc);
  Ss[e.ac] = ec * fmaf(e.zd, e.Rcol, e.Scol);
}

// Row read for target d (lane = source n): the lane's term of the intensity,
// log2 lambda on lane 0, and with GRAD the gradient sums R/lambda, S/lambda.
template <int P, bool GRAD>
__device__ __forceinline__ void pair_row(PairLds<P>& sh, const PairEvent& e, int lane, int grp,
                                         float& llp, float& gmup) {
  // The chunk's own gradient sums: a plain read-modify-write (LDS float
  // atomics are several times slower), read early, written last.
  float oR = 0.f, oS = 0.f;
  if constexpr (GRAD) {
    oR = sh.gR[grp][e.ac];
    oS = sh.gS[grp][e.ac];
  }
  const float ex = exp2_fast(e.brow * e.z);
  const float R = ex * e.Rrow - (e.z == 0.f ? e.c : 0.f);
  const float S = ex * fmaf(e.z, e.Rrow, e.Srow);
  const float lam = group_sum<P>(e.arow * R) + e.mud;
  const bool ok = e.ok != 0.f;
  llp += (ok && lane == 0) ? __builtin_amdgcn_logf(lam) : 0.f;
  if constexpr (GRAD) {
    const float w = ok ? __builtin_amdgcn_rcpf(lam) : 0.f;
    sh.gR[grp][e.ac] = fmaf(w, R, oR);
    sh.gS[grp][e.ac] = fmaf(w, S, oS);
    gmup += lane == e.d ? w : 0.f;
  }
}

// Whether some pair of the window decays slowly against its length (beta_mn
// T below the threshold); uniform over the workgroup.  Uses sh.wsum.
template <int P>
__device__ __forceinline__ bool slow_decay_pair(PairLds<P>& sh, const PairOwn<P>& own, double T,
                                                int M) {
  using C = PairCfg<P>;
  float bmin = 3.0e38f;
#pragma unroll
  for (int k = 0; k < C::OWN; ++k) {
    const int e = threadIdx.x + k * C::THREADS;
    if (e < P * P && e / P < M && e % P < M) bmin = fminf(bmin, own.beta[k]);
  }
  const double wmin = -wave_max(-(double)bmin);
  __syncthreads();  // wsum: the previous window's readers are done
  if ((threadIdx.x & 63) == 0) sh.wsum[threadIdx.x >> 6] = wmin;
  __syncthreads();
  double m = sh.wsum[0];
  for (int v = 1; v < C::WAVES; ++v) m = fmin(m, sh.wsum[v]);
  return m * T < kSlowDecayPair;
}

// Compensator sums of a slowly decaying window from its events.  Each chunk
// adds, per event with source n = d and per target m (lane), -expm1(-x) and
// h(x), x = beta_mn tau, into column n of its LDS state arrays (cleared
// first, and by pass 1 after); the owner of pair (m, n) then sums the chunks
// in FP64: C_mn = Q / beta_mn, F_mn = C_mn + H / beta_mn.
template <int P>
__device__ __noinline__ void slow_decay_sums_pair(PairLds<P>& sh, PairOwn<P>& own,
                                                  const float* __restrict__ tw,
                                                  const uint8_t* __restrict__ dw, int len,
                                                  int nb, int lane, int grp, int M) {
  using C = PairCfg<P>;
  constexpr int Q = C::Q, B = C::B;
  float* Qs = sh.Rs[grp];
  float* Hs = sh.Ss[grp];
  for (int e = lane; e < P * Q; e += P) {
    Qs[e] = 0.f;
    Hs[e] = 0.f;
  }
  for (int bb = 0; bb < nb; ++bb) {
    const int jl = bb * B + (lane & (B - 1));
    const float tau_l = jl < len ? tw[jl] : 0.f;  // null events: tau 0 adds nothing
    const int d_l = jl < len ? (int)dw[jl] : 0;
    static_for<B>([&](auto J) {
      constexpr int j = decltype(J)::value;
      const float tau = batch_bcast<P, j>(tau_l);
      const int d = __builtin_bit_cast(int, batch_bcast<P, j>(__builtin_bit_cast(float, d_l)));
      const float x = tau * (sh.nbeta[lane * Q + d] * (-1.f / kLog2e));
      const int a = d * Q + lane;
      Qs[a] += comp_q(x);
      Hs[a] += comp_h(x);
    });
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < C::OWN; ++k) {
    const int e = threadIdx.x + k * C::THREADS;
    if (e >= P * P) break;
    const int m = e / P, n = e % P;
    double q = 0.0, h = 0.0;
    for (int g = 0; g < C::G; ++g) {
      q += (double)sh.Rs[g][n * Q + m];
      h += (double)sh.Ss[g][n * Q + m];
    }
    const bool in = m < M && n < M;
    const double b = (double)own.beta[k];
    own.C[k] = in ? q / b : 0.0;
    own.F[k] = in ? q / b + h / b : 0.0;
  }
  __syncthreads();  // pass 1 clears the arrays next
}

// Evaluates one window with parameters in LDS (and the owned decays in
// own.beta).  Results: sh.scal[0] = ll, own.C and own.F; if GRAD also sh.gR /
// sh.gS (FP32 sums) and sh.gmu.
//
// Within a chunk the events are a chain through LDS (an event's row read
// sees every earlier column update), so per event the reads go out together
// and the column update is written before the next event's reads; the
// event's intensity, logarithm and gradient sums follow the next event's
// reads, off the chain.  The gradient sums are kept per chunk, so that the
// chunks never write the same LDS word.
template <int P, bool GRAD>
__device__ __forceinline__ void eval_window_pair(PairLds<P>& sh, PairOwn<P>& own,
                                                 const float* __restrict__ dtg,
                                                 const uint8_t* __restrict__ dg,
                                                 const float* __restrict__ taug,
                                                 const float* __restrict__ gsdg, int64_t begin,
                                                 int n, double T, float end_gap, int M) {
  using C = PairCfg<P>;
  constexpr int Q = C::Q, G = C::G, B = C::B;
  const int tid = threadIdx.x;
  const int lane = tid & (P - 1);
  const int grp = tid / P;
  const float* __restrict__ dtw = dtg + begin;
  const uint8_t* __restrict__ dw = dg + begin;
  const float* __restrict__ gw = gsdg + begin;
  float* Rs = sh.Rs[grp];
  float* Ss = sh.Ss[grp];
  const int c = (n + G - 1) / G;
  const int j0 = min(grp * c, n);
  const int len = min(j0 + c, n) - j0;
  const int nb = (c + B - 1) / B;  // uniform over the workgroup; short chunks run null events
  auto load = [&](int bb, float& dt_l, int& d_l, float& g_l) {
    const int jl = bb * B + (lane & (B - 1));
    dt_l = jl < len ? dtw[j0 + jl] : 0.f;
    d_l = jl < len ? (int)dw[j0 + jl] : 0;
    g_l = jl < len ? gw[j0 + jl] : 0.f;
  };

  const bool slow = slow_decay_pair<P>(sh, own, T, M);
  if (slow) slow_decay_sums_pair<P>(sh, own, taug + begin + j0, dw + j0, len, nb, lane, grp, M);

  // Pass 1: zero-start state of this chunk, column updates only.
  for (int e = lane; e < P * Q; e += P) {
    Rs[e] = 0.f;
    Ss[e] = 0.f;
  }
  float z = 0.f, cn = 0.f, count = 0.f, delta = 0.f;
  {
    float dt_l, dt_n = 0.f, g_l, g_n = 0.f;
    int d_l, d_n = 0;
    load(0, dt_l, d_l, g_l);
    for (int bb = 0; bb < nb; ++bb) {
      if (bb + 1 < nb) load(bb + 1, dt_n, d_n, g_n);
      const int nv = len - bb * B;
      auto batch = [&](auto F) {
        constexpr bool FULL = decltype(F)::value;
        static_for<B>([&](auto J) {
          constexpr int j = decltype(J)::value;
          const int d = __builtin_bit_cast(int, batch_bcast<P, j>(__builtin_bit_cast(float, d_l)));
          const int a = d * Q + lane;
          const float Rt = Rs[a], St = Ss[a], bc = sh.nbeta[lane * Q + d];
          __builtin_amdgcn_sched_barrier(0);  // reads first, the clock work under their latency
          const float dt = batch_bcast<P, j>(dt_l);
          const bool ok = FULL || j < nv;
          z += dt;
          delta += dt;
          const float zd0 = fminf(batch_bcast<P, j>(g_l), delta);  // column d's elapsed time
          const float zd = ok ? zd0 : 0.f;
          const float own = (ok && lane == d) ? 1.f : 0.f;
          count += own;
          const float ncn = zd > 0.f ? 1.f : cn + 1.f;
          cn = fmaf(own, ncn - cn, cn);
          z = fmaf(-own, z, z);
          const float ec = exp2_fast(bc * zd);
          Rs[a] = fmaf(ec, Rt, ok ? 1.f : 0.f);
          Ss[a] = ec * fmaf(zd, Rt, St);
        });
      };
      if (__ballot(nv < B) == 0)  // uniform over the wavefront
        batch(std::true_type{});
      else
        batch(std::false_type{});
      dt_l = dt_n;
      d_l = d_n;
      g_l = g_n;
    }
  }
  // Lazy columns -> full state at the chunk's last event (lane = column n).
  for (int m = 0; m < P; ++m) {
    const int a = lane * Q + m;
    const float e = exp2_fast(sh.nbeta[m * Q + lane] * z);
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
#pragma unroll
  for (int k = 0; k < C::OWN; ++k) {
    const int e = tid + k * C::THREADS;
    if (e >= P * P) break;
    const int m = e / P, nn = e % P;
    const int a = nn * Q + m;
    const float b = own.beta[k];
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
    if (!slow) {
      own.C[k] = in ? ((double)Ntot - E) / bd : 0.0;
      own.F[k] = in ? F : 0.0;
    }
  }
  __syncthreads();
  // Pass 2: from the exact chunk start, row reads (intensity, gradient
  // sums) and column updates.
  {
    const float pend = sh.Ps[grp][lane];
    for (int m = 0; m < P; ++m) Rs[lane * Q + m] += pend;  // pending events enter at weight 1
    z = 0.f;
    cn = pend;
    float llp = 0.f, gmup = 0.f;  // llp: sum of log2 lambda
    float dt_l, dt_n = 0.f, g_l, g_n = 0.f, dl = 0.f;  // dl: time since the chunk's start
    int d_l, d_n = 0;
    load(0, dt_l, d_l, g_l);
    for (int bb = 0; bb < nb; ++bb) {
      if (bb + 1 < nb) load(bb + 1, dt_n, d_n, g_n);
      const int nv = len - bb * B;
      auto batch = [&](auto F) {
        constexpr bool FULL = decltype(F)::value;
        PairEvent cur = pair_issue<P, 0, FULL>(sh, Rs, Ss, lane, dt_l, d_l, g_l, nv, z, cn, dl);
        static_for<B>([&](auto J) {
          constexpr int j = decltype(J)::value;
          pair_column(Rs, Ss, cur);
          if constexpr (j + 1 < B) {
            const PairEvent nxt =
                pair_issue<P, j + 1, FULL>(sh, Rs, Ss, lane, dt_l, d_l, g_l, nv, z, cn, dl);
            pair_row<P, GRAD>(sh, cur, lane, grp, llp, gmup);
            cur = nxt;
          } else {
            pair_row<P, GRAD>(sh, cur, lane, grp, llp, gmup);
          }
        });
      };
      if (__ballot(nv < B) == 0)  // uniform over the wavefront
        batch(std::true_type{});
      else
        batch(std::false_type{});
      dt_l = dt_n;
      d_l = d_n;
      g_l = g_n;
    }
    sh.red[0][tid] = llp;
    sh.red[1][tid] = gmup;
  }
  // ll = sum log lambda - T sum mu - sum alpha_mn C_mn: the last sum over the
  // owned pairs and the waves, the others over the chunks, then the lanes.
  double p3 = 0.0;
#pragma unroll
  for (int k = 0; k < C::OWN; ++k) {
    const int e = tid + k * C::THREADS;
    if (e < P * P) p3 += (double)sh.alpha[(e / P) * Q + e % P] * own.C[k];
  }
  p3 = wave_sum(p3);
  if ((tid & 63) == 0) sh.wsum[tid >> 6] = p3;
  __syncthreads();
  double l2 = 0.0, smu = 0.0;
  if (tid < 64) {  // the first wavefront, whole
    if (tid < P) {
      double gm = 0.0;
      for (int g = 0; g < G; ++g) {
        l2 += (double)sh.red[0][g * P + tid];
        gm += (double)sh.red[1][g * P + tid];
      }
      sh.gmu[tid] = tid < M ? gm - T : 0.0;
      smu = tid < M ? (double)sh.mu[tid] : 0.0;
    }
    l2 = wave_sum(l2);
    smu = wave_sum(smu);
  }
  if (tid == 0) {
    double s3 = 0.0;
    for (int v = 0; v < C::WAVES; ++v) s3 += sh.wsum[v];
    sh.scal[0] = l2 * 0.69314718055994530942 - T * smu - s3;  // log2 -> natural log
  }
  __syncthreads();
}

template <int P>
__device__ void load_params_pair(PairLds<P>& sh, PairOwn<P>& own, const float* __restrict__ mu,
                                 const float* __restrict__ alpha, const float* __restrict__ beta,
                                 int64_t w, int M) {
  using C = PairCfg<P>;
  constexpr int Q = C::Q;
#pragma unroll
  for (int k = 0; k < C::OWN; ++k) {
    const int e = threadIdx.x + k * C::THREADS;
    if (e >= P * P) break;
    const int m = e / P, n = e % P;
    const bool in = m < M && n < M;
    sh.alpha[m * Q + n] = in ? alpha[(w * M + m) * M + n] : 0.f;
    const float b = in ? beta[(w * M + m) * M + n] : 1.f;
    own.beta[k] = b;
    sh.nbeta[m * Q + n] = -b * kLog2e;
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
  for (int e = threadIdx.x; e < PairCfg<P>::G * P * PairCfg<P>::Q; e += PairCfg<P>::THREADS) {
    sh.gR[0][e] = 0.f;
    sh.gS[0][e] = 0.f;
  }
}

// Sum over the chunks of the gradient sums of pair (m, n), which it clears
// for the next evaluation.
template <int P>
__device__ __forceinline__ void take_pair_sums(PairLds<P>& sh, int a, double& gR, double& gS) {
  gR = 0.0;
  gS = 0.0;
  for (int g = 0; g < PairCfg<P>::G; ++g) {
    gR += (double)sh.gR[g][a];
    gS += (double)sh.gS[g][a];
    sh.gR[g][a] = 0.f;
    sh.gS[g][a] = 0.f;
  }
}

template <int P, bool GRAD>
__global__ __launch_bounds__(PairCfg<P>::THREADS) void pair_eval_kernel(
    Events ev, int M, const float* mu, const float* alpha, const float* beta, double* ll,
    float* g_mu, float* g_alpha, float* g_beta, int* counter) {
  __shared__ PairLds<P> sh;
  using C = PairCfg<P>;
  constexpr int Q = C::Q;
  const int tid = threadIdx.x;
  PairOwn<P> own;
  zero_pair_accumulators(sh);
  for (int q = next_window_pair(sh, counter, 1); q < ev.W; q = next_window_pair(sh, counter, 0)) {
    const int64_t w = ev.order[q];
    load_params_pair(sh, own, mu, alpha, beta, w, M);
    const double T = ev.T[w];
    eval_window_pair<P, GRAD>(sh, own, ev.dt, ev.d, ev.tau, ev.gsd, ev.begin[w], ev.n[w], T, ev.end_gap[w], M);
    if (tid == 0) ll[w] = sh.scal[0];
    if constexpr (GRAD) {
      if (tid < M) g_mu[w * M + tid] = (float)sh.gmu[tid];
#pragma unroll
      for (int k = 0; k < C::OWN; ++k) {
        const int e = tid + k * C::THREADS;
        if (e >= P * P) break;
        const int m = e / P, n = e % P;
        double gR, gS;
        take_pair_sums(sh, m * Q + n, gR, gS);
        if (m < M && n < M) {
          const double a = (double)sh.alpha[m * Q + n], b = (double)own.beta[k];
          g_alpha[(w * M + m) * M + n] = (float)(gR - own.C[k]);
          g_beta[(w * M + m) * M + n] = (float)(-a * (gS + (own.F[k] - own.C[k]) / b));
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
  PairOwn<P> own;
  float m1a[OWN], m2a[OWN], m1b[OWN], m2b[OWN];
  zero_pair_accumulators(sh);
  for (int q = next_window_pair(sh, counter, 1); q < ev.W; q = next_window_pair(sh, counter, 0)) {
    const int64_t w = ev.order[q];
    load_params_pair(sh, own, mu, alpha, beta, w, M);
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
      eval_window_pair<P, true>(sh, own, ev.dt, ev.d, ev.tau, ev.gsd, ev.begin[w], n, T, ev.end_gap[w], M);
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
          double gR, gS;
          take_pair_sums(sh, m * Q + nn, gR, gS);
          const double a = (double)sh.alpha[m * Q + nn], b = (double)own.beta[k];
          ga[k] = gR - own.C[k];
          gb[k] = -a * (gS + (own.F[k] - own.C[k]) / b);
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
      const bool em = o.optimizer == MDHP_OPT_EM;
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
      float na[OWN];
#pragma unroll
      for (int k = 0; k < OWN; ++k) {
        const int e = tid + k * C::THREADS;
        na[k] = 0.f;
        if (e < P * P) {
          const int m = e / P, nn = e % P;
          if (m < M && nn < M && em) {
            // Expected offspring count over its exposure (ga = G_mn - C_mn).
            const double a = (double)sh.alpha[m * Q + nn], Cmn = (double)own.C[k];
            na[k] = Cmn > 0.0 ? (float)(a * ((ga[k] + Cmn) / Cmn)) : (float)a;
          } else if (m < M && nn < M) {
            na[k] = (float)fmax((double)sh.alpha[m * Q + nn] + step(ga[k], m1a[k], m2a[k]), 0.0);
            if (!o.fix_beta)
              own.beta[k] = (float)fmax((double)own.beta[k] + step(gb[k], m1b[k], m2b[k]),
                                        beta_min);
          }
        }
      }
      float nmu = 0.f;
      if (tid < M)
        nmu = em ? (float)fmax((double)sh.mu[tid] * ((sh.gmu[tid] + T) / T), mu_min)
                 : (float)fmax((double)sh.mu[tid] + step(sh.gmu[tid], m1mu, m2mu), mu_min);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < OWN; ++k) {
        const int e = tid + k * C::THREADS;
        if (e < P * P) {
          const int m = e / P, nn = e % P;
          if (m < M && nn < M) {
            sh.alpha[m * Q + nn] = na[k];
            sh.nbeta[m * Q + nn] = -own.beta[k] * kLog2e;
          }
        }
      }
      if (tid < M) sh.mu[tid] = nmu;
      __syncthreads();
    }
    // The FP32 sums of the last evaluation are still in LDS when the loop
    // stops before reading them; clear them for the next window.
    __syncthreads();
    for (int e = tid; e < C::G * P * Q; e += C::THREADS) {
      sh.gR[0][e] = 0.f;
      sh.gS[0][e] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
      const int e = tid + k * C::THREADS;
      if (e < P * P) {
        const int m = e / P, nn = e % P;
        if (m < M && nn < M) {
          alpha[(w * M + m) * M + nn] = sh.alpha[m * Q + nn];
          beta[(w * M + m) * M + nn] = own.beta[k];
        }
      }
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
