// FP64 CPU oracle for the exponential-kernel multi-dimensional Hawkes
// process (MDHP) log-likelihood, its gradient and the projected gradient
// fit.  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the
// bench's cpu_baseline leg call it; the product path never does.  It shares
// no source with the GPU library.
//
// What it computes (paper: "MDHP-Net", Sec. II-B and Sec. IV-B):
//   intensity, Eq. (2):
//     lambda_m(t) = mu_m + sum_n sum_{k: d_k = n, t_k < t} alpha_mn e^{-beta_mn (t - t_k)}
//   closed-form log-likelihood, Eq. (5) (Part1 + Part2 + Part3, Appendix B):
//     ll = sum_i log lambda_{d_i}(t_i) - T sum_m mu_m
//          + sum_{m,n} (alpha_mn / beta_mn) sum_{k: d_k = n} (e^{-beta_mn (T - t_k)} - 1)
//   Notation: the paper's theta is mu, its D is M, its T_span is T.  alpha_mn
//   is the excitation of target m by source n (the direction the formula of
//   Eq. (2) gives; the prose under Eq. (2) states the opposite, and the
//   formula is taken).  Events at equal times never excite each other: the
//   inner sum of Eq. (2) and Eq. (5) is over strictly earlier times.
//
// Three independent evaluations:
//   * brute:     Eq. (5) written out, O(N^2) per window (tiny inputs).
//   * recursion: the same sums with Part1's inner double sum replaced by the
//                standard exponential-kernel recursion (Ozaki, cited by the
//                paper for Eq. (1)), O(N M^2) per window; exact up to rounding.
//                With one decay for every pair the recursion depends on the
//                source only: O(N M) per window (recursion_window_shared).
//   * fit:       projected gradient ascent on ll / max(N, 1) (plain step or
//                Adam step), projection mu >= mu_min, alpha >= 0,
//                beta >= beta_min; the paper uses "a PyTorch optimizer" on
//                -ll without naming it (Sec. IV-B), so the update rule is a
//                stated reading, not the paper's; projected L-BFGS; and EM on
//                the branching structure with the decays fixed (the paper
//                names EM among the estimators of related work).
//
// Layouts (host memory, caller-owned):
//   offsets int64[W+1]; window w owns events [offsets[w], offsets[w+1])
//   t f64[sum N]  non-decreasing within a window, 0 <= t <= T[w]
//   dim i32[sum N] in [0, M)
//   T f64[W] > 0
//   mu f64[W*M]; alpha f64[W*M*M] row-major, alpha[w][m][n] = source n -> target m
//   beta f64[W] (beta_mode 0, one decay per window) or f64[W*M*M] (beta_mode 1)
// Return codes: 0 ok, -1 invalid argument, -2 unsorted times, -3 t/dim/T out
// of domain, -4 bad parameter (mu <= 0, alpha < 0, beta <= 0 or non-finite).

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>

namespace {

struct Window {
  const double* t;
  const int32_t* d;
  int64_t n;
  double T;
};

// One window's parameters expanded to M x M decays (a shared decay is copied
// into every pair; nothing else differs between the two modes).
struct Params {
  int M;
  std::vector<double> mu, alpha, beta;  // M, M*M, M*M
  bool shared = false;                  // one decay for every pair (beta_mode 0)
};

Params load_params(int M, int beta_mode, const double* mu, const double* alpha,
                   const double* beta, int64_t w) {
  Params p;
  p.M = M;
  p.mu.assign(mu + w * M, mu + (w + 1) * M);
  p.alpha.assign(alpha + w * M * M, alpha + (w + 1) * M * M);
  p.beta.resize((size_t)M * M);
  for (int i = 0; i < M * M; ++i)
    p.beta[i] = beta_mode == 0 ? beta[w] : beta[w * M * M + i];
  p.shared = beta_mode == 0;
  return p;
}

int check_params(const Params& p) {
  const int M = p.M;
  for (int m = 0; m < M; ++m)
    if (!(p.mu[m] > 0.0) || !std::isfinite(p.mu[m])) return -4;
  for (int i = 0; i < M * M; ++i) {
    if (!(p.alpha[i] >= 0.0) || !std::isfinite(p.alpha[i])) return -4;
    if (!(p.beta[i] > 0.0) || !std::isfinite(p.beta[i])) return -4;
  }
  return 0;
}

int check_batch(const int64_t* offsets, const double* t, const int32_t* dim,
                const double* T, int64_t W, int M) {
  if (W < 0 || M < 1 || !offsets || !T) return -1;
  if (offsets[0] != 0) return -1;
  for (int64_t w = 0; w < W; ++w) {
    if (offsets[w + 1] < offsets[w]) return -1;
    if (!(T[w] > 0.0) || !std::isfinite(T[w])) return -3;
    for (int64_t i = offsets[w]; i < offsets[w + 1]; ++i) {
      if (!(t[i] >= 0.0) || !(t[i] <= T[w])) return -3;
      if (dim[i] < 0 || dim[i] >= M) return -3;
      if (i > offsets[w] && t[i] < t[i - 1]) return -2;
    }
  }
  return 0;
}

// Runs f(w) for every window on a pool of host threads; windows are handed
// out dynamically so that uneven window sizes balance.
template <class F>
void for_windows(int64_t W, int nthreads, F f) {
  if (nthreads <= 0) nthreads = (int)std::max(1u, std::thread::hardware_concurrency());
  nthreads = (int)std::min<int64_t>(nthreads, std::max<int64_t>(W, 1));
  std::atomic<int64_t> next{0};
  auto worker = [&]() {
    for (;;) {
      int64_t w = next.fetch_add(1);
      if (w >= W) break;
      f(w);
    }
  };
  if (nthreads == 1) {
    worker();
    return;
  }
  std::vector<std::thread> pool;
  for (int i = 0; i < nthreads; ++i) pool.emplace_back(worker);
  for (auto& th : pool) th.join();
}

// Gradient container (same layout as the parameters, per-pair decays).
struct Grad {
  std::vector<double> mu, alpha, beta;
};

// Magnitudes that set parity tolerances: sum_i |log lambda_i| + Gamma for
// ll, and for every gradient component the sum of the absolute values of the
// terms whose signed sum it is.
struct Scale {
  double ll = 0.0;
  std::vector<double> mu, alpha, beta;
};

// ---------------------------------------------------------------------------
// Brute force: Eq. (5) term by term.  Part1 = sum over events of the log of
// Eq. (2) at the event, with the inner sum over every strictly earlier event;
// Part2 = -T sum mu; Part3 = sum_{m,n} alpha_mn/beta_mn sum_{k: d_k=n}
// (e^{-beta_mn (T - t_k)} - 1) (with the "-1" of Eq. (5) and Appendix B).
// The gradient is the term-by-term derivative of the same expression.
// ---------------------------------------------------------------------------
double brute_window(const Window& win, const Params& p, Grad* g) {
  const int M = p.M;
  if (g) {
    g->mu.assign(M, 0.0);
    g->alpha.assign((size_t)M * M, 0.0);
    g->beta.assign((size_t)M * M, 0.0);
  }
  double part1 = 0.0;
  for (int64_t i = 0; i < win.n; ++i) {
    const int m = win.d[i];
    double lam = p.mu[m];
    for (int64_t k = 0; k < win.n; ++k) {
      if (!(win.t[k] < win.t[i])) continue;
      const int n = win.d[k];
      lam += p.alpha[m * M + n] * std::exp(-p.beta[m * M + n] * (win.t[i] - win.t[k]));
    }
    part1 += std::log(lam);
    if (g) {
      const double w = 1.0 / lam;
      g->mu[m] += w;
      for (int64_t k = 0; k < win.n; ++k) {
        if (!(win.t[k] < win.t[i])) continue;
        const int n = win.d[k];
        const double u = win.t[i] - win.t[k];
        const double e = std::exp(-p.beta[m * M + n] * u);
        g->alpha[m * M + n] += w * e;
        g->beta[m * M + n] += -w * p.alpha[m * M + n] * u * e;
      }
    }
  }
  double sum_mu = 0.0;
  for (int m = 0; m < M; ++m) sum_mu += p.mu[m];
  const double part2 = -win.T * sum_mu;
  double part3 = 0.0;
  for (int m = 0; m < M; ++m) {
    for (int n = 0; n < M; ++n) {
      const double a = p.alpha[m * M + n], b = p.beta[m * M + n];
      double s = 0.0, s_tau = 0.0;  // sum (e^{-b tau} - 1), sum tau e^{-b tau}
      for (int64_t k = 0; k < win.n; ++k) {
        if (win.d[k] != n) continue;
        const double tau = win.T - win.t[k];
        s += std::expm1(-b * tau);
        s_tau += tau * std::exp(-b * tau);
      }
      part3 += a / b * s;
      if (g) {
        g->alpha[m * M + n] += s / b;
        // d/db [a/b * s(b)] = -a/b^2 s + a/b * ds/db, ds/db = -sum tau e^{-b tau}
        g->beta[m * M + n] += -a / (b * b) * s - a / b * s_tau;
      }
    }
  }
  if (g)
    for (int m = 0; m < M; ++m) g->mu[m] -= win.T;
  return part1 + part2 + part3;
}

// ---------------------------------------------------------------------------
// Recursion: Part1's inner sum R_mn(i) = sum_{k: d_k=n, t_k<t_i}
// e^{-beta_mn (t_i - t_k)} follows R(i) = e^{-beta Dt} (R(i') + P) where i'
// is the last event strictly before t_i and P counts the events at t_{i'}
// (events that share a time stay "pending" until time moves on, so they
// never excite each other).  S_mn(i) = sum (t_i - t_k) e^{-beta_mn (t_i -
// t_k)} = -dR/dbeta follows S(i) = e^{-beta Dt} S(i') + Dt R(i).  Part2 and
// Part3 are summed per event exactly as in the brute form.
// ---------------------------------------------------------------------------
double recursion_window(const Window& win, const Params& p, Grad* g, Scale* sc = nullptr) {
  const int M = p.M;
  const int MM = M * M;
  std::vector<double> R(MM, 0.0), S(MM, 0.0), pend(M, 0.0);
  std::vector<double> gR(MM, 0.0), gS(MM, 0.0), gmu(M, 0.0);
  double t_prev = 0.0;
  double part1 = 0.0, abs1 = 0.0;
  for (int64_t i = 0; i < win.n; ++i) {
    const double dt = win.t[i] - t_prev;
    if (dt > 0.0) {
      for (int m = 0; m < M; ++m)
        for (int n = 0; n < M; ++n) {
          const double a = std::exp(-p.beta[m * M + n] * dt);
          const double r = a * (R[m * M + n] + pend[n]);
          S[m * M + n] = a * S[m * M + n] + dt * r;
          R[m * M + n] = r;
        }
      std::fill(pend.begin(), pend.end(), 0.0);
      t_prev = win.t[i];
    }
    const int m = win.d[i];
    double lam = p.mu[m];
    for (int n = 0; n < M; ++n) lam += p.alpha[m * M + n] * R[m * M + n];
    part1 += std::log(lam);
    abs1 += std::fabs(std::log(lam));
    if (g || sc) {
      const double w = 1.0 / lam;
      gmu[m] += w;
      for (int n = 0; n < M; ++n) {
        gR[m * M + n] += w * R[m * M + n];
        gS[m * M + n] += w * S[m * M + n];
      }
    }
    pend[m] += 1.0;
  }
  double sum_mu = 0.0;
  for (int m = 0; m < M; ++m) sum_mu += p.mu[m];
  const double part2 = -win.T * sum_mu;
  // Part3, one event at a time: for every source event k and every target m.
  std::vector<double> s(MM, 0.0), s_tau(MM, 0.0);
  for (int64_t k = 0; k < win.n; ++k) {
    const int n = win.d[k];
    const double tau = win.T - win.t[k];
    for (int m = 0; m < M; ++m) {
      const double b = p.beta[m * M + n];
      s[m * M + n] += std::expm1(-b * tau);
      s_tau[m * M + n] += tau * std::exp(-b * tau);
    }
  }
  double part3 = 0.0;
  for (int i = 0; i < MM; ++i) part3 += p.alpha[i] / p.beta[i] * s[i];
  if (sc) {
    // Gamma = T sum mu + sum alpha/beta sum (1 - e^{-beta tau}) >= 0.
    sc->ll = abs1 + win.T * sum_mu - part3;
    sc->mu.resize(M);
    sc->alpha.resize(MM);
    sc->beta.resize(MM);
    for (int m = 0; m < M; ++m) sc->mu[m] = gmu[m] + win.T;
    for (int i = 0; i < MM; ++i) {
      const double a = p.alpha[i], b = p.beta[i];
      sc->alpha[i] = gR[i] + std::fabs(s[i]) / b;
      sc->beta[i] = a * gS[i] + a / (b * b) * std::fabs(s[i]) + a / b * s_tau[i];
    }
  }
  if (g) {
    g->mu.resize(M);
    g->alpha.resize(MM);
    g->beta.resize(MM);
    for (int m = 0; m < M; ++m) g->mu[m] = gmu[m] - win.T;
    for (int i = 0; i < MM; ++i) {
      const double a = p.alpha[i], b = p.beta[i];
      g->alpha[i] = gR[i] + s[i] / b;
      g->beta[i] = -a * gS[i] - a / (b * b) * s[i] - a / b * s_tau[i];
    }
  }
  return part1 + part2 + part3;
}

// Recursion with one decay for every pair (beta_mn = beta, the shared mode):
// R_mn(i) = R_n(i) and S_mn(i) = S_n(i) depend on the source only, and so
// do the compensator's sums, so a time step costs one exponential and O(M)
// work instead of M^2 exponentials.  Same sums, same outputs as
// recursion_window (which the shared mode can be forced back to, for the
// cross-check of the two).
bool g_pairwise_shared = false;

double recursion_window_shared(const Window& win, const Params& p, Grad* g, Scale* sc) {
  const int M = p.M;
  const int MM = M * M;
  const double b = p.beta[0];
  std::vector<double> R(M, 0.0), S(M, 0.0), pend(M, 0.0);
  std::vector<double> gR(MM, 0.0), gS(MM, 0.0), gmu(M, 0.0);
  double t_prev = 0.0;
  double part1 = 0.0, abs1 = 0.0;
  for (int64_t i = 0; i < win.n; ++i) {
    const double dt = win.t[i] - t_prev;
    if (dt > 0.0) {
      const double a = std::exp(-b * dt);
      for (int n = 0; n < M; ++n) {
        const double r = a * (R[n] + pend[n]);
        S[n] = a * S[n] + dt * r;
        R[n] = r;
      }
      std::fill(pend.begin(), pend.end(), 0.0);
      t_prev = win.t[i];
    }
    const int m = win.d[i];
    double lam = p.mu[m];
    for (int n = 0; n < M; ++n) lam += p.alpha[m * M + n] * R[n];
    part1 += std::log(lam);
    abs1 += std::fabs(std::log(lam));
    if (g || sc) {
      const double w = 1.0 / lam;
      gmu[m] += w;
      for (int n = 0; n < M; ++n) {
        gR[m * M + n] += w * R[n];
        gS[m * M + n] += w * S[n];
      }
    }
    pend[m] += 1.0;
  }
  double sum_mu = 0.0;
  for (int m = 0; m < M; ++m) sum_mu += p.mu[m];
  const double part2 = -win.T * sum_mu;
  // Part3: sums over the source-n events, the same for every target.
  std::vector<double> s(M, 0.0), s_tau(M, 0.0);
  for (int64_t k = 0; k < win.n; ++k) {
    const int n = win.d[k];
    const double tau = win.T - win.t[k];
    s[n] += std::expm1(-b * tau);
    s_tau[n] += tau * std::exp(-b * tau);
  }
  double part3 = 0.0;
  for (int i = 0; i < MM; ++i) part3 += p.alpha[i] / b * s[i % M];
  if (sc) {
    sc->ll = abs1 + win.T * sum_mu - part3;
    sc->mu.resize(M);
    sc->alpha.resize(MM);
    sc->beta.resize(MM);
    for (int m = 0; m < M; ++m) sc->mu[m] = gmu[m] + win.T;
    for (int i = 0; i < MM; ++i) {
      const double a = p.alpha[i], sn = s[i % M];
      sc->alpha[i] = gR[i] + std::fabs(sn) / b;
      sc->beta[i] = a * gS[i] + a / (b * b) * std::fabs(sn) + a / b * s_tau[i % M];
    }
  }
  if (g) {
    g->mu.resize(M);
    g->alpha.resize(MM);
    g->beta.resize(MM);
    for (int m = 0; m < M; ++m) g->mu[m] = gmu[m] - win.T;
    for (int i = 0; i < MM; ++i) {
      const double a = p.alpha[i], sn = s[i % M];
      g->alpha[i] = gR[i] + sn / b;
      g->beta[i] = -a * gS[i] - a / (b * b) * sn - a / b * s_tau[i % M];
    }
  }
  return part1 + part2 + part3;
}

// The recursion form for a window: shared or per-pair decays.
double recursion_eval(const Window& win, const Params& p, Grad* g, Scale* sc = nullptr) {
  if (p.shared && !g_pairwise_shared) return recursion_window_shared(win, p, g, sc);
  return recursion_window(win, p, g, sc);
}

void store_grad(const Grad& g, int M, int beta_mode, int64_t w, double* g_mu,
                double* g_alpha, double* g_beta) {
  const int MM = M * M;
  if (g_mu) std::copy(g.mu.begin(), g.mu.end(), g_mu + w * M);
  if (g_alpha) std::copy(g.alpha.begin(), g.alpha.end(), g_alpha + w * MM);
  if (g_beta) {
    if (beta_mode == 0) {
      // One shared decay: the chain rule sums the per-pair derivatives.
      double sb = 0.0;
      for (int i = 0; i < MM; ++i) sb += g.beta[i];
      g_beta[w] = sb;
    } else {
      std::copy(g.beta.begin(), g.beta.end(), g_beta + w * MM);
    }
  }
}

template <bool kBrute>
int eval_batch(const int64_t* offsets, const double* t, const int32_t* dim,
               const double* T, int64_t W, int32_t M, int32_t beta_mode,
               const double* mu, const double* alpha, const double* beta,
               double* ll, double* g_mu, double* g_alpha, double* g_beta,
               int32_t nthreads) {
  if (beta_mode != 0 && beta_mode != 1) return -1;
  if (!mu || !alpha || !beta || !ll) return -1;
  int rc = check_batch(offsets, t, dim, T, W, M);
  if (rc) return rc;
  for (int64_t w = 0; w < W; ++w) {
    rc = check_params(load_params(M, beta_mode, mu, alpha, beta, w));
    if (rc) return rc;
  }
  const bool want_grad = g_mu || g_alpha || g_beta;
  for_windows(W, nthreads, [&](int64_t w) {
    Window win{t + offsets[w], dim + offsets[w], offsets[w + 1] - offsets[w], T[w]};
    Params p = load_params(M, beta_mode, mu, alpha, beta, w);
    Grad g;
    ll[w] = kBrute ? brute_window(win, p, want_grad ? &g : nullptr)
                   : recursion_eval(win, p, want_grad ? &g : nullptr);
    if (want_grad) store_grad(g, M, beta_mode, w, g_mu, g_alpha, g_beta);
  });
  return 0;
}

// Part3's coefficient of alpha_mn (Appendix B), the exposure of dimension m
// to the events of dimension n: C_mn = sum_{k: d_k = n} (1 - e^{-beta_mn
// (T - t_k)}) / beta_mn, straight from its definition.
std::vector<double> exposure(const Window& win, const Params& p) {
  const int M = p.M;
  std::vector<double> C((size_t)M * M, 0.0);
  for (int64_t k = 0; k < win.n; ++k) {
    const int n = win.d[k];
    const double tau = win.T - win.t[k];
    for (int m = 0; m < M; ++m) {
      const double b = p.beta[(size_t)m * M + n];
      C[(size_t)m * M + n] += -std::expm1(-b * tau) / b;
    }
  }
  return C;
}

// Options of the projected gradient fit; same field order as the library's
// public struct so that one Python packing serves both (declared separately:
// the two share no source).
struct FitOpts {
  int32_t max_steps;
  int32_t optimizer;  // 0 projected gradient step, 1 projected Adam step, 2 projected L-BFGS,
                      // 3 EM (decays fixed)
  int32_t fix_beta;
  int32_t history;    // L-BFGS memory (0: 8)
  double lr;
  double ll_tol;
  double mu_floor_rel;
  double beta_floor_rel;
  double adam_b1, adam_b2, adam_eps;
};

// Projected L-BFGS on f = -ll / max(N, 1) with bounds x >= lb (a
// quasi-Newton variant of the projected update; the paper leaves the
// optimizer open).  One iteration: variables at their bound whose gradient
// pushes outward are held fixed; the direction is the two-loop recursion
// over the last `history` (s, y) pairs applied to the free gradient (scale
// gamma = s.y / y.y of the newest pair, or 0.01 / max|g| without history),
// restarted as scaled steepest descent if it is not a descent direction;
// the step t = 1, 1/2, 1/4, ... (at most 20 trials, each a full likelihood
// + gradient evaluation) is the first whose projected point satisfies
// f(x') <= f(x) + 1e-4 g.(x' - x); the pair (x' - x, g' - g) enters the
// history if its curvature s.y exceeds 1e-10 |s| |y|.  Stops as converged
// when |ll' - ll| <= ll_tol max(|ll'|, N, 1) after an accepted step (or when
// the free gradient vanishes), as MAX_STEPS after max_steps accepted steps,
// and as STALLED (3) when no trial step is accepted.
struct LbfgsResult {
  int steps, status, evals;
  double ll;
};

template <class Eval>
LbfgsResult lbfgs_fit(std::vector<double>& x, const std::vector<double>& lb,
                      const std::vector<char>& frozen, double inv_n, const FitOpts& o,
                      Eval eval) {
  const int P = (int)x.size();
  const int m = o.history > 0 ? o.history : 8;
  std::vector<std::vector<double>> S, Y;
  std::vector<double> rho;
  std::vector<double> gl(P), g(P), q(P), d(P), xn(P), gn(P);
  double l = eval(x, gl);
  int evals = 1;
  auto finite_all = [&](double v, const std::vector<double>& gv) {
    if (!std::isfinite(v)) return false;
    for (double e : gv)
      if (!std::isfinite(e)) return false;
    return true;
  };
  if (!finite_all(l, gl)) return {0, 2, evals, l};
  for (int i = 0; i < P; ++i) g[i] = frozen[i] ? 0.0 : -gl[i] * inv_n;
  double f = -l * inv_n;
  for (int s = 0;; ++s) {
    if (s == o.max_steps) return {s, 1, evals, l};
    double gmax = 0.0;
    for (int i = 0; i < P; ++i) {
      const bool active = frozen[i] || (x[i] <= lb[i] && g[i] > 0.0);
      q[i] = active ? 0.0 : g[i];
      gmax = std::max(gmax, std::fabs(q[i]));
    }
    if (gmax == 0.0) return {s, 0, evals, l};
    const double gamma0 = 0.01 / gmax;
    const int h = (int)S.size();
    std::vector<double> a(h);
    for (int k = h - 1; k >= 0; --k) {
      double sq = 0.0;
      for (int i = 0; i < P; ++i) sq += S[k][i] * q[i];
      a[k] = rho[k] * sq;
      for (int i = 0; i < P; ++i) q[i] -= a[k] * Y[k][i];
    }
    double gamma = gamma0;
    if (h > 0) {
      double sy = 0.0, yy = 0.0;
      for (int i = 0; i < P; ++i) {
        sy += S[h - 1][i] * Y[h - 1][i];
        yy += Y[h - 1][i] * Y[h - 1][i];
      }
      gamma = sy / yy;
    }
    for (int i = 0; i < P; ++i) q[i] *= gamma;
    for (int k = 0; k < h; ++k) {
      double yr = 0.0;
      for (int i = 0; i < P; ++i) yr += Y[k][i] * q[i];
      const double b = rho[k] * yr;
      for (int i = 0; i < P; ++i) q[i] += S[k][i] * (a[k] - b);
    }
    double dg = 0.0;
    for (int i = 0; i < P; ++i) {
      const bool active = frozen[i] || (x[i] <= lb[i] && g[i] > 0.0);
      d[i] = active ? 0.0 : -q[i];
      dg += d[i] * g[i];
    }
    if (!(dg < 0.0)) {  // not a descent direction: restart from steepest descent
      S.clear();
      Y.clear();
      rho.clear();
      for (int i = 0; i < P; ++i) {
        const bool active = frozen[i] || (x[i] <= lb[i] && g[i] > 0.0);
        d[i] = active ? 0.0 : -gamma0 * g[i];
      }
    }
    double t = 1.0, ln = 0.0, fn = 0.0;
    bool ok = false;
    for (int ls = 0; ls < 20 && !ok; ++ls, t *= 0.5) {
      double decrease = 0.0;
      for (int i = 0; i < P; ++i) {
        xn[i] = std::max(x[i] + t * d[i], lb[i]);
        decrease += g[i] * (xn[i] - x[i]);
      }
      ln = eval(xn, gn);
      ++evals;
      fn = -ln * inv_n;
      ok = finite_all(ln, gn) && fn <= f + 1e-4 * decrease;
    }
    if (!ok) return {s, 3, evals, l};
    std::vector<double> sv(P), yv(P);
    double sy = 0.0, ss = 0.0, yy = 0.0;
    for (int i = 0; i < P; ++i) {
      const double gi = frozen[i] ? 0.0 : -gn[i] * inv_n;
      sv[i] = xn[i] - x[i];
      yv[i] = gi - g[i];
      sy += sv[i] * yv[i];
      ss += sv[i] * sv[i];
      yy += yv[i] * yv[i];
      g[i] = gi;
      x[i] = xn[i];
    }
    if (sy > 1e-10 * std::sqrt(ss * yy)) {
      if ((int)S.size() == m) {
        S.erase(S.begin());
        Y.erase(Y.begin());
        rho.erase(rho.begin());
      }
      S.push_back(sv);
      Y.push_back(yv);
      rho.push_back(1.0 / sy);
    }
    const double l_prev = l;
    l = ln;
    f = fn;
    if (std::fabs(l - l_prev) <= o.ll_tol * std::max(std::fabs(l), 1.0 / inv_n))
      return {s + 1, 0, evals, l};
  }
}

}  // namespace

extern "C" {

int mdhp_oracle_loglik(const int64_t* offsets, const double* t, const int32_t* dim,
                       const double* T, int64_t W, int32_t M, int32_t beta_mode,
                       const double* mu, const double* alpha, const double* beta,
                       double* ll, int32_t nthreads) {
  return eval_batch<false>(offsets, t, dim, T, W, M, beta_mode, mu, alpha, beta, ll,
                           nullptr, nullptr, nullptr, nthreads);
}

int mdhp_oracle_grad(const int64_t* offsets, const double* t, const int32_t* dim,
                     const double* T, int64_t W, int32_t M, int32_t beta_mode,
                     const double* mu, const double* alpha, const double* beta,
                     double* ll, double* g_mu, double* g_alpha, double* g_beta,
                     int32_t nthreads) {
  if (!g_mu || !g_alpha || !g_beta) return -1;
  return eval_batch<false>(offsets, t, dim, T, W, M, beta_mode, mu, alpha, beta, ll,
                           g_mu, g_alpha, g_beta, nthreads);
}

int mdhp_oracle_loglik_brute(const int64_t* offsets, const double* t, const int32_t* dim,
                             const double* T, int64_t W, int32_t M, int32_t beta_mode,
                             const double* mu, const double* alpha, const double* beta,
                             double* ll, int32_t nthreads) {
  return eval_batch<true>(offsets, t, dim, T, W, M, beta_mode, mu, alpha, beta, ll,
                          nullptr, nullptr, nullptr, nthreads);
}

int mdhp_oracle_grad_brute(const int64_t* offsets, const double* t, const int32_t* dim,
                           const double* T, int64_t W, int32_t M, int32_t beta_mode,
                           const double* mu, const double* alpha, const double* beta,
                           double* ll, double* g_mu, double* g_alpha, double* g_beta,
                           int32_t nthreads) {
  if (!g_mu || !g_alpha || !g_beta) return -1;
  return eval_batch<true>(offsets, t, dim, T, W, M, beta_mode, mu, alpha, beta, ll,
                          g_mu, g_alpha, g_beta, nthreads);
}

// Projected gradient ascent per window.  Step s = 0, 1, ...: evaluate ll_s
// and the gradient g_s at theta_s (recursion form); stop as converged when
// s >= 1 and |ll_s - ll_{s-1}| <= ll_tol * max(|ll_s|, N, 1); stop as not
// converged when s == max_steps; otherwise theta_{s+1} = Proj(theta_s +
// step(g_s / max(N, 1))).  The returned theta is theta_s with ll_s, and
// steps[w] = s (the number of updates applied), evals[w] (optional) the
// number of likelihood evaluations.  Optimizer 2 is the projected L-BFGS
// described at lbfgs_fit.  status: 0 converged,
// 1 step budget exhausted, 2 non-finite likelihood or gradient (theta_s,
// the parameters of that evaluation, is returned with its ll), 3 (L-BFGS)
// no step of the line search was accepted.
int mdhp_oracle_fit(const int64_t* offsets, const double* t, const int32_t* dim,
                    const double* T, int64_t W, int32_t M, int32_t beta_mode,
                    const void* opts_ptr, double* mu, double* alpha, double* beta,
                    double* ll, int32_t* steps, int32_t* status, int32_t* evals_out,
                    int32_t nthreads) {
  if (beta_mode != 0 && beta_mode != 1) return -1;
  if (!opts_ptr || !mu || !alpha || !beta || !ll || !steps || !status) return -1;
  FitOpts o;
  std::memcpy(&o, opts_ptr, sizeof(o));
  if (o.max_steps < 0 || o.optimizer < 0 || o.optimizer > 3) return -1;
  if (o.optimizer <= 1 && !(o.lr > 0.0)) return -1;
  if (o.optimizer == 3 && !o.fix_beta) return -1;  // EM keeps the decays
  int rc = check_batch(offsets, t, dim, T, W, M);
  if (rc) return rc;
  for (int64_t w = 0; w < W; ++w) {
    rc = check_params(load_params(M, beta_mode, mu, alpha, beta, w));
    if (rc) return rc;
  }
  const int MM = M * M;
  const int nb = beta_mode == 0 ? 1 : MM;
  for_windows(W, nthreads, [&](int64_t w) {
    Window win{t + offsets[w], dim + offsets[w], offsets[w + 1] - offsets[w], T[w]};
    const double rate = (double)std::max<int64_t>(win.n, 1) / win.T;
    const double mu_min = o.mu_floor_rel * rate;
    const double beta_min = o.beta_floor_rel * rate;
    const double inv_n = 1.0 / (double)std::max<int64_t>(win.n, 1);
    // theta as one vector: [mu (M) | alpha (MM) | beta (nb)]
    const int P = M + MM + nb;
    std::vector<double> th(P), m1(P, 0.0), m2(P, 0.0), gv(P);
    std::copy(mu + w * M, mu + (w + 1) * M, th.begin());
    std::copy(alpha + w * MM, alpha + (w + 1) * MM, th.begin() + M);
    if (beta_mode == 0) th[M + MM] = beta[w];
    else std::copy(beta + w * MM, beta + (w + 1) * MM, th.begin() + M + MM);
    if (o.optimizer == 2) {
      std::vector<double> lb(P, 0.0);
      std::vector<char> frozen(P, 0);
      for (int i = 0; i < M; ++i) lb[i] = mu_min;
      for (int i = M + MM; i < P; ++i) {
        lb[i] = beta_min;
        frozen[i] = o.fix_beta ? 1 : 0;
      }
      auto eval = [&](const std::vector<double>& x, std::vector<double>& gout) {
        Params p;
        p.M = M;
        p.mu.assign(x.begin(), x.begin() + M);
        p.alpha.assign(x.begin() + M, x.begin() + M + MM);
        p.beta.resize(MM);
        for (int i = 0; i < MM; ++i) p.beta[i] = beta_mode == 0 ? x[M + MM] : x[M + MM + i];
        p.shared = beta_mode == 0;
        Grad g;
        const double l = recursion_eval(win, p, &g);
        std::copy(g.mu.begin(), g.mu.end(), gout.begin());
        std::copy(g.alpha.begin(), g.alpha.end(), gout.begin() + M);
        if (beta_mode == 0) {
          double sb = 0.0;
          for (int i = 0; i < MM; ++i) sb += g.beta[i];
          gout[M + MM] = sb;
        } else {
          std::copy(g.beta.begin(), g.beta.end(), gout.begin() + M + MM);
        }
        return l;
      };
      const LbfgsResult r = lbfgs_fit(th, lb, frozen, inv_n, o, eval);
      std::copy(th.begin(), th.begin() + M, mu + w * M);
      std::copy(th.begin() + M, th.begin() + M + MM, alpha + w * MM);
      if (beta_mode == 0) beta[w] = th[M + MM];
      else std::copy(th.begin() + M + MM, th.end(), beta + w * MM);
      ll[w] = r.ll;
      steps[w] = r.steps;
      status[w] = r.status;
      if (evals_out) evals_out[w] = r.evals;
      return;
    }
    double ll_prev = 0.0;
    int st = 1, s = 0;
    std::vector<double> th_eval = th;
    double ll_eval = 0.0;
    for (s = 0;; ++s) {
      Params p;
      p.M = M;
      p.mu.assign(th.begin(), th.begin() + M);
      p.alpha.assign(th.begin() + M, th.begin() + M + MM);
      p.beta.resize(MM);
      for (int i = 0; i < MM; ++i) p.beta[i] = beta_mode == 0 ? th[M + MM] : th[M + MM + i];
      p.shared = beta_mode == 0;
      Grad g;
      const double l = recursion_eval(win, p, &g);
      bool finite = std::isfinite(l);
      std::copy(g.mu.begin(), g.mu.end(), gv.begin());
      std::copy(g.alpha.begin(), g.alpha.end(), gv.begin() + M);
      if (beta_mode == 0) {
        double sb = 0.0;
        for (int i = 0; i < MM; ++i) sb += g.beta[i];
        gv[M + MM] = sb;
      } else {
        std::copy(g.beta.begin(), g.beta.end(), gv.begin() + M + MM);
      }
      for (int i = 0; i < P; ++i) finite = finite && std::isfinite(gv[i]);
      if (!finite) {
        st = 2;  // returns the parameters whose evaluation was not finite
        th_eval = th;
        ll_eval = l;
        break;
      }
      th_eval = th;
      ll_eval = l;
      if (s >= 1 && std::fabs(l - ll_prev) <= o.ll_tol * std::max(std::fabs(l), 1.0 / inv_n)) {
        st = 0;
        break;
      }
      if (s == o.max_steps) {
        st = 1;
        break;
      }
      ll_prev = l;
      if (o.optimizer == 3) {
        // EM on the branching structure (decays fixed): mu_m takes the
        // expected number of background events of dimension m over T,
        // alpha_mn the expected number of dimension-m offspring of
        // dimension-n events over their exposure C_mn.  With G_m =
        // sum_{i: d_i = m} 1 / lambda_i and G_mn = sum_{i: d_i = m} R_mn(i) /
        // lambda_i these counts are mu_m G_m and alpha_mn G_mn, and the
        // gradient gives G_m = dll/dmu_m + T, G_mn = dll/dalpha_mn + C_mn.
        const std::vector<double> C = exposure(win, p);
        for (int m = 0; m < M; ++m) th[m] = std::max(th[m] * (gv[m] + win.T) / win.T, mu_min);
        for (int i = 0; i < MM; ++i)
          if (C[i] > 0.0) th[M + i] = th[M + i] * (gv[M + i] + C[i]) / C[i];
        continue;
      }
      const double bc1 = 1.0 - std::pow(o.adam_b1, (double)(s + 1));
      const double bc2 = 1.0 - std::pow(o.adam_b2, (double)(s + 1));
      for (int i = 0; i < P; ++i) {
        const bool is_beta = i >= M + MM;
        if (is_beta && o.fix_beta) continue;
        const double gn = gv[i] * inv_n;
        double step;
        if (o.optimizer == 0) {
          step = o.lr * gn;
        } else {
          m1[i] = o.adam_b1 * m1[i] + (1.0 - o.adam_b1) * gn;
          m2[i] = o.adam_b2 * m2[i] + (1.0 - o.adam_b2) * gn * gn;
          step = o.lr * (m1[i] / bc1) / (std::sqrt(m2[i] / bc2) + o.adam_eps);
        }
        double v = th[i] + step;
        if (i < M) v = std::max(v, mu_min);
        else if (!is_beta) v = std::max(v, 0.0);
        else v = std::max(v, beta_min);
        th[i] = v;
      }
    }
    std::copy(th_eval.begin(), th_eval.begin() + M, mu + w * M);
    std::copy(th_eval.begin() + M, th_eval.begin() + M + MM, alpha + w * MM);
    if (beta_mode == 0) beta[w] = th_eval[M + MM];
    else std::copy(th_eval.begin() + M + MM, th_eval.end(), beta + w * MM);
    ll[w] = ll_eval;
    steps[w] = s;
    status[w] = st;
    if (evals_out) evals_out[w] = s + 1;
  });
  return 0;
}

// Tolerance scales (see Scale): ll_scale[W], s_mu[W*M], s_alpha[W*M*M],
// s_beta[W] (shared mode: summed over pairs) or [W*M*M].
int mdhp_oracle_scales(const int64_t* offsets, const double* t, const int32_t* dim,
                       const double* T, int64_t W, int32_t M, int32_t beta_mode,
                       const double* mu, const double* alpha, const double* beta,
                       double* ll_scale, double* s_mu, double* s_alpha, double* s_beta,
                       int32_t nthreads) {
  if (beta_mode != 0 && beta_mode != 1) return -1;
  if (!mu || !alpha || !beta || !ll_scale || !s_mu || !s_alpha || !s_beta) return -1;
  int rc = check_batch(offsets, t, dim, T, W, M);
  if (rc) return rc;
  for_windows(W, nthreads, [&](int64_t w) {
    Window win{t + offsets[w], dim + offsets[w], offsets[w + 1] - offsets[w], T[w]};
    Params p = load_params(M, beta_mode, mu, alpha, beta, w);
    Scale sc;
    recursion_eval(win, p, nullptr, &sc);
    ll_scale[w] = sc.ll;
    Grad g{sc.mu, sc.alpha, sc.beta};
    store_grad(g, M, beta_mode, w, s_mu, s_alpha, s_beta);
  });
  return 0;
}

// Non-zero: the shared mode runs the per-pair recursion with the decay
// copied into every pair (the cross-check of the two forms).
void mdhp_oracle_set_pairwise_shared(int32_t on) { g_pairwise_shared = on != 0; }

// Threads the pool uses when nthreads <= 0 is passed.
int mdhp_oracle_default_threads(void) {
  return (int)std::max(1u, std::thread::hardware_concurrency());
}

}  // extern "C"
