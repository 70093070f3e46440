// Seeded synthetic event windows: multivariate exponential-kernel Hawkes
// processes simulated by Ogata's thinning method.
//
// This is input generation only.  The GPU library and the CPU oracle both
// consume its output; it evaluates no likelihood, gradient or update.
//
// Model (paper "MDHP-Net", Eq. (2)): lambda_m(s) = mu_m + sum_n X_mn(s) with
// X_mn(s) = alpha_mn sum_{k: d_k = n, t_k < s} e^{-beta_mn (s - t_k)}.
// Thinning (Ogata 1981): at the current time s the total intensity can only
// decay until the next event, so lbar = sum_m lambda_m(s+) bounds it; draw a
// candidate s' = s + Exp(lbar), accept it with probability
// sum_m lambda_m(s') / lbar, and on acceptance pick the dimension m with
// probability lambda_m(s') / sum lambda(s').
//
// Random numbers: SplitMix64 (Steele, Lea and Flood, 2014), one stream per
// window keyed by (seed, window index), so the output does not depend on the
// number of threads.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <thread>
#include <vector>

namespace {

struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  // Uniform on (0, 1): 53 random bits, offset by half an ulp so 0 never appears.
  double uniform() { return ((double)(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
};

SplitMix64 stream_for(uint64_t seed, int64_t w) {
  SplitMix64 g{seed ^ 0x6A09E667F3BCC909ull};
  const uint64_t a = g.next();
  SplitMix64 h{a ^ ((uint64_t)w * 0xD1B54A32D192ED03ull + 0x243F6A8885A308D3ull)};
  h.next();
  return h;
}

// Simulates one window.  mode 0: until time T_fix (at most cap events, more
// is an error).  mode 1: until n_fix + 1 events are accepted; the window keeps
// the first n_fix and ends at the time of the last one.
int simulate(int M, int beta_mode, const double* mu, const double* alpha, const double* beta,
             int mode, double T_fix, int64_t n_fix, int64_t cap, SplitMix64& rng, double* t_out,
             int32_t* d_out, int64_t* n_out, double* T_out) {
  const int MM = M * M;
  std::vector<double> X(MM, 0.0), lam(M, 0.0);
  double s = 0.0;
  double mu_sum = 0.0;
  for (int m = 0; m < M; ++m) mu_sum += mu[m];
  double lbar = mu_sum;
  int64_t n = 0;
  const int64_t limit = mode == 0 ? cap : n_fix + 1;
  for (;;) {
    const double e = -std::log(rng.uniform());
    const double s_new = s + e / lbar;
    if (mode == 0 && s_new > T_fix) break;
    const double dt = s_new - s;
    double total = 0.0;
    if (beta_mode == 0) {
      // One decay for every pair: only the row sums Y_m = sum_n X_mn matter,
      // and they decay by the same factor (kept in X[m]).
      const double a = std::exp(-beta[0] * dt);
      for (int m = 0; m < M; ++m) {
        X[m] *= a;
        lam[m] = mu[m] + X[m];
        total += lam[m];
      }
    } else {
      for (int i = 0; i < MM; ++i) X[i] *= std::exp(-beta[i] * dt);
      for (int m = 0; m < M; ++m) {
        double l = mu[m];
        for (int nn = 0; nn < M; ++nn) l += X[m * M + nn];
        lam[m] = l;
        total += l;
      }
    }
    s = s_new;
    const double u = rng.uniform();
    if (u * lbar <= total) {
      const double pick = rng.uniform() * total;
      int m = 0;
      double c = lam[0];
      while (m < M - 1 && c < pick) c += lam[++m];
      if (n >= limit) return -5;
      if (mode == 1 && n == n_fix) {
        *T_out = s;
        *n_out = n;
        return 0;
      }
      t_out[n] = s;
      d_out[n] = m;
      ++n;
      double add = 0.0;
      for (int tgt = 0; tgt < M; ++tgt) {
        X[beta_mode == 0 ? tgt : tgt * M + m] += alpha[tgt * M + m];
        add += alpha[tgt * M + m];
      }
      lbar = total + add;
    } else {
      lbar = total;
    }
  }
  *T_out = T_fix;
  *n_out = n;
  return 0;
}

}  // namespace

extern "C" {

// W windows; per-window parameters mu[W*M], alpha[W*M*M], beta[W] or [W*M*M].
// mode 0: T_in[w] is the window end and offsets[w+1]-offsets[w] the capacity;
// mode 1: offsets[w+1]-offsets[w] is the exact event count.
// Window w of the call draws the random stream of global window first_window + w.
// Outputs: t_out/dim_out at offsets[w], n_out[w] events written, T_out[w].
// Returns 0, -1 on bad arguments, -5 if a window exceeded its capacity.
int synth_ogata(int64_t W, int32_t M, int32_t beta_mode, const double* mu, const double* alpha,
                const double* beta, int32_t mode, const double* T_in, const int64_t* offsets,
                uint64_t seed, int64_t first_window, double* t_out, int32_t* dim_out,
                int64_t* n_out, double* T_out, int32_t nthreads) {
  if (W < 0 || M < 1 || (beta_mode != 0 && beta_mode != 1) || (mode != 0 && mode != 1))
    return -1;
  if (mode == 0 && !T_in) return -1;
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  nthreads = (int)std::min<int64_t>(nthreads, std::max<int64_t>(W, 1));
  std::atomic<int64_t> next{0};
  std::atomic<int> err{0};
  auto worker = [&]() {
    for (;;) {
      const int64_t w = next.fetch_add(1);
      if (w >= W) break;
      SplitMix64 rng = stream_for(seed, first_window + w);
      const int64_t cap = offsets[w + 1] - offsets[w];
      const double* b = beta_mode == 0 ? beta + w : beta + w * M * M;
      const int rc = simulate(M, beta_mode, mu + w * M, alpha + w * M * M, b, mode,
                              mode == 0 ? T_in[w] : 0.0, cap, cap, rng, t_out + offsets[w],
                              dim_out + offsets[w], n_out + w, T_out + w);
      if (rc) err.store(rc);
    }
  };
  std::vector<std::thread> pool;
  for (int i = 0; i < nthreads; ++i) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
  return err.load();
}

}  // extern "C"
