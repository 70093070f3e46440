// Batched simulation of exponential-kernel MDHP windows on the GPU by
// Ogata's thinning method (the model of Eq. (2)).
//
// One wavefront simulates one window; lane m holds dimension m's state:
// X_m = sum_n alpha_mn sum_{k: d_k = n, t_k < s} e^{-beta (s - t_k)} for one
// decay per window, or the row X_m[n] of pair states for one decay per
// pair.  At the current time s the total intensity can only decay until the
// next event, so lbar = sum_m lambda_m(s+) bounds it: a candidate
// s' = s + Exp(lbar) is drawn, accepted with probability
// sum_m lambda_m(s') / lbar, and on acceptance its dimension is the first m
// whose cumulative intensity reaches a uniform fraction of the total.
// Everything runs in FP64, like the host generator the library's tests take
// their windows from; sums over lanes are butterfly reductions and scans.
//
// Random numbers: SplitMix64 (Steele, Lea and Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014), one stream per window
// derived from (seed, window index): the same streams as the host generator,
// so a window's events do not depend on the batch it is simulated in.

#include <cfloat>

#include "mdhp_device.h"

namespace mdhp {

namespace {

struct SplitMix64 {
  uint64_t s;
  __device__ uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  // Uniform on (0, 1): the top 53 bits plus half an ulp (0 never appears).
  __device__ double uniform() { return ((double)(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
};

// The stream of window w: a generator seeded from `seed` gives one word,
// which keyed with w seeds the window's generator (one draw discarded).
__device__ SplitMix64 window_stream(uint64_t seed, int64_t w) {
  SplitMix64 g{seed ^ 0x6A09E667F3BCC909ull};
  const uint64_t a = g.next();
  SplitMix64 h{a ^ ((uint64_t)w * 0xD1B54A32D192ED03ull + 0x243F6A8885A308D3ull)};
  h.next();
  return h;
}

__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) v += __shfl_xor(v, k, 64);
  return v;
}

__device__ __forceinline__ double wave_inclusive_scan(double v, int lane) {
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    const double u = __shfl_up(v, k, 64);
    if (lane >= k) v += u;
  }
  return v;
}

constexpr int kSimBlock = 256;  // four windows per workgroup
// n_out values of a window or attack that could not be drawn.
constexpr int64_t kSimNoRoom = -1;    // more events than its room
constexpr int64_t kSimBadInput = -2;  // parameters or range that cannot be sampled
// Most candidate times one attack window may expect, r (t_max - t_min).
constexpr double kAttackMaxCandidates = 16777216.0;

// NP: pair states per lane (1: one decay per window; MDHP_SIM_PAIR_MAX_M:
// one per pair, M <= MDHP_SIM_PAIR_MAX_M).
template <int NP>
__global__ __launch_bounds__(kSimBlock) void ogata_kernel(
    int64_t W, int M, const double* __restrict__ mu, const double* __restrict__ alpha,
    const double* __restrict__ beta, int mode, const double* __restrict__ T_in,
    const int64_t* __restrict__ offsets, uint64_t seed, int64_t first_window,
    double* __restrict__ t_out, int32_t* __restrict__ dim_out, int64_t* __restrict__ n_out,
    double* __restrict__ T_out) {
  const int64_t w = (int64_t)blockIdx.x * (kSimBlock / 64) +
                    __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (w >= W) return;  // the whole wavefront
  const int lane = threadIdx.x & 63;
  const bool in = lane < M;
  const double mu_l = in ? mu[w * M + lane] : 0.0;
  // Decays of this lane's pairs (target lane, source n) and their states.
  double b[NP], X[NP];
#pragma unroll
  for (int n = 0; n < NP; ++n) {
    X[n] = 0.0;
    if constexpr (NP == 1) b[n] = beta[w];
    else b[n] = (in && n < M) ? beta[(w * M + lane) * M + n] : 0.0;
  }
  const int64_t base = offsets[w], cap = offsets[w + 1] - offsets[w];
  const double T_fix = mode == MDHP_SIM_UNTIL_T ? T_in[w] : 0.0;
  if (mode == MDHP_SIM_UNTIL_T && !(T_fix >= 0.0 && T_fix <= DBL_MAX)) {
    if (lane == 0) n_out[w] = kSimBadInput;
    return;
  }
  SplitMix64 rng = window_stream(seed, first_window + w);
  double s = 0.0;
  double lbar = wave_total(mu_l);
  int64_t n = 0;
  for (;;) {
    // The bound is the same on every lane (butterfly sums are symmetric).
    // A zero bound ends a window of fixed length (no event can follow); a
    // negative, infinite or NaN one (invalid parameters), or a zero one
    // where events are still owed, would never end the loop.
    if (!(lbar > 0.0 && lbar <= DBL_MAX)) {
      if (mode == MDHP_SIM_UNTIL_T && lbar == 0.0) break;
      if (lane == 0) n_out[w] = kSimBadInput;
      return;
    }
    const double s_new = s - log(rng.uniform()) / lbar;
    if (mode == MDHP_SIM_UNTIL_T && s_new > T_fix) break;
    const double dt = s_new - s;
    double lam = mu_l;
    if constexpr (NP == 1) {
      X[0] *= exp(-b[0] * dt);
      lam += X[0];
    } else {
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        X[k] *= exp(-b[k] * dt);
        lam += X[k];
      }
    }
    lam = in ? lam : 0.0;
    const double total = wave_total(lam);
    s = s_new;
    if (rng.uniform() * lbar <= total) {
      const double pick = rng.uniform() * total;
      const double c = wave_inclusive_scan(lam, lane);
      const uint64_t hit = __ballot(in && c >= pick);
      const int m = hit ? (int)__builtin_ctzll(hit) : M - 1;
      if (mode == MDHP_SIM_COUNT && n == cap) {
        if (lane == 0) T_out[w] = s;
        break;
      }
      if (n == cap) {  // until T: the window holds more events than its capacity
        if (lane == 0) n_out[w] = kSimNoRoom;
        return;
      }
      if (lane == 0) {
        t_out[base + n] = s;
        dim_out[base + n] = m;
      }
      ++n;
      const double a = in ? alpha[(w * M + lane) * M + m] : 0.0;
      if constexpr (NP == 1) {
        X[0] += a;
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k) X[k] += k == m ? a : 0.0;
      }
      lbar = total + wave_total(a);
    } else {
      lbar = total;
    }
  }
  if (lane == 0) {
    n_out[w] = n;
    if (mode == MDHP_SIM_UNTIL_T) T_out[w] = T_fix;
  }
}

// ---------------------------------------------------------------- attacks
// Injection times of the paper's attack strategies (Sec. III, the attack
// rates g(t) of its strategy table) drawn by its three samplers (appendix,
// "Sampling algorithm"), one attack window per thread:
//   PLA  g = a t^b                                      p = (a, b)
//   DEA  g = W1 a1 t^(a1-1) (t < t1), W2 a2 e^(c (t - t1)) (t >= t1)
//                                                       p = (W1, a1, W2, a2, c, t1)
//   ASA  g = C e^(c t) / (1 + e^(c (t - t0)))^2         p = (C, c, t0)
//   DAM  g = w a1 t^(a1-1) + (1 - w) a2 e^(a2 t)        p = (w, a1, a2)
// NPP: candidate gaps Exp with mean 1 / r, a candidate t kept when a
// Uniform(0, g_max) draw is below g(t); ND: candidate gaps |Normal(1 / r,
// 1 / (2 r))|, kept with probability g(t) / g_max; DRP: DAM with its weight
// w drawn per third of the range from U(0, 1/3), U(1/3, 2/3), U(2/3, 1)
// (a1, a2 from p[1], p[2]), then NPP's thinning.  r = p[7] (512 when 0).
// g_max is the largest value of g on a grid of kAttackGrid + 1 points of the
// range, as the paper takes it from evaluations of g.
constexpr int kAttackGrid = 4096;

__device__ double attack_rate(int strategy, const double* p, double t, const double* wseg,
                              double b1, double b2) {
  switch (strategy) {
    case MDHP_ATTACK_PLA:
      return p[0] * pow(t, p[1]);
    case MDHP_ATTACK_DEA:
      return t < p[5] ? p[0] * p[1] * pow(t, p[1] - 1.0) : p[2] * p[3] * exp(p[4] * (t - p[5]));
    case MDHP_ATTACK_ASA: {
      const double e = exp(p[1] * (t - p[2]));
      return p[0] * exp(p[1] * t) / ((1.0 + e) * (1.0 + e));
    }
    default: {  // DAM, with the weight of t's third when wseg is given (DRP)
      const double w = wseg ? (t < b1 ? wseg[0] : (t < b2 ? wseg[1] : wseg[2])) : p[0];
      return w * p[1] * pow(t, p[1] - 1.0) + (1.0 - w) * p[2] * exp(p[2] * t);
    }
  }
}

__global__ __launch_bounds__(256) void attack_kernel(
    int64_t A, const int32_t* __restrict__ strategy, const int32_t* __restrict__ sampler,
    const double* __restrict__ params, const double* __restrict__ range,
    const int64_t* __restrict__ offsets, uint64_t seed, int64_t first, double* __restrict__ t_out,
    int64_t* __restrict__ n_out) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= A) return;
  double p[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) p[k] = params[a * 8 + k];
  const int smp = sampler[a];
  const int strat = smp == MDHP_SAMPLER_DRP ? MDHP_ATTACK_DAM : strategy[a];
  const double lo = range[2 * a], hi = range[2 * a + 1];
  const double r = p[7] > 0.0 ? p[7] : 512.0;
  // Also false for NaN or infinite ends: the candidate loop runs until t
  // passes t_max, about r (t_max - t_min) times.
  if (!(hi >= lo && r * (hi - lo) <= kAttackMaxCandidates)) {
    n_out[a] = kSimBadInput;
    return;
  }
  SplitMix64 rng = window_stream(seed, first + a);
  double wseg[3];
  const double b1 = lo + (hi - lo) / 3.0, b2 = lo + 2.0 * (hi - lo) / 3.0;
  if (smp == MDHP_SAMPLER_DRP) {
    wseg[0] = rng.uniform() / 3.0;
    wseg[1] = (1.0 + rng.uniform()) / 3.0;
    wseg[2] = (2.0 + rng.uniform()) / 3.0;
  }
  const double* ws = smp == MDHP_SAMPLER_DRP ? wseg : nullptr;
  double gmax = 0.0;
  for (int i = 0; i <= kAttackGrid; ++i)
    gmax = fmax(gmax, attack_rate(strat, p, lo + (hi - lo) * i / kAttackGrid, ws, b1, b2));
  const int64_t base = offsets[a], cap = offsets[a + 1] - offsets[a];
  int64_t n = 0;
  double t = lo;
  for (;;) {
    double dt;
    if (smp == MDHP_SAMPLER_ND) {
      const double u1 = rng.uniform(), u2 = rng.uniform();  // Box-Muller
      dt = fabs(1.0 / r + 0.5 / r * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
    } else {
      dt = -log(rng.uniform()) / r;
    }
    t += dt;
    if (t > hi) break;
    const double u = rng.uniform();
    const bool keep = smp == MDHP_SAMPLER_ND ? u < attack_rate(strat, p, t, ws, b1, b2) / gmax
                                             : u * gmax < attack_rate(strat, p, t, ws, b1, b2);
    if (keep) {
      if (n == cap) {
        n_out[a] = kSimNoRoom;
        return;
      }
      t_out[base + n] = t;
      ++n;
    }
  }
  n_out[a] = n;
}

}  // namespace

}  // namespace mdhp

using namespace mdhp;

extern "C" {

mdhp_status mdhp_simulate(int64_t W, int32_t M, int32_t beta_mode, const double* mu,
                          const double* alpha, const double* beta, int32_t mode,
                          const double* T_in, const int64_t* offsets, uint64_t seed,
                          int64_t first_window, double* t_out, int32_t* dim_out, int64_t* n_out,
                          double* T_out, void* stream) {
  if (W < 0 || M < 1 || M > 64 || (beta_mode != MDHP_BETA_SHARED && beta_mode != MDHP_BETA_PAIR) ||
      (beta_mode == MDHP_BETA_PAIR && M > MDHP_SIM_PAIR_MAX_M) ||
      (mode != MDHP_SIM_UNTIL_T && mode != MDHP_SIM_COUNT) || first_window < 0)
    return mdhp_fail(MDHP_E_INVAL, "simulate: bad sizes, decay mode or simulation mode");
  if (W == 0) return MDHP_OK;
  if (!mu || !alpha || !beta || !offsets || !t_out || !dim_out || !n_out || !T_out ||
      (mode == MDHP_SIM_UNTIL_T && !T_in))
    return mdhp_fail(MDHP_E_INVAL, "simulate: null pointer");
  hipStream_t s = (hipStream_t)stream;
  const int grid = (int)((W + kSimBlock / 64 - 1) / (kSimBlock / 64));
  if (beta_mode == MDHP_BETA_SHARED)
    hipLaunchKernelGGL(ogata_kernel<1>, dim3(grid), dim3(kSimBlock), 0, s, W, M, mu, alpha, beta,
                       mode, T_in, offsets, seed, first_window, t_out, dim_out, n_out, T_out);
  else
    hipLaunchKernelGGL(ogata_kernel<MDHP_SIM_PAIR_MAX_M>, dim3(grid), dim3(kSimBlock), 0, s, W, M,
                       mu, alpha, beta, mode, T_in, offsets, seed, first_window, t_out, dim_out,
                       n_out, T_out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MDHP_OK : mdhp_hip_fail(e, "simulate");
}

mdhp_status mdhp_attack_times(int64_t A, const int32_t* strategy, const int32_t* sampler,
                              const double* params, const double* range, const int64_t* offsets,
                              uint64_t seed, int64_t first, double* t_out, int64_t* n_out,
                              void* stream) {
  if (A < 0 || first < 0) return mdhp_fail(MDHP_E_INVAL, "attack_times: bad sizes");
  if (A == 0) return MDHP_OK;
  if (!strategy || !sampler || !params || !range || !offsets || !t_out || !n_out)
    return mdhp_fail(MDHP_E_INVAL, "attack_times: null pointer");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(attack_kernel, dim3((unsigned)((A + 255) / 256)), dim3(256), 0, s, A,
                     strategy, sampler, params, range, offsets, seed, first, t_out, n_out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MDHP_OK : mdhp_hip_fail(e, "attack_times");
}

}  // extern "C"
