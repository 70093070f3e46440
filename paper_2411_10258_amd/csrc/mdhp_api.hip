// C ABI of libmdhp: plan creation (validation + compact preparation of the
// events), the compute entry points and error reporting.

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "mdhp_internal.h"

struct mdhp_plan {
  int64_t W = 0, N = 0;
  int32_t M = 0, beta_mode = 0;
  bool lane_major = false;  // events stored lane-major per window (M <= 16, one decay)
  int64_t slots = 0;        // length of dt / d
  float* dt = nullptr;
  float* tau = nullptr;    // per event T - t (FP64 difference, stored FP32), same slots as dt
  float* gsd = nullptr;    // per-pair plans: per event the gap to the previous event of its
                           // dimension in the window (FP64 difference, FP32; +inf if none)
  uint8_t* d = nullptr;
  int64_t* begin = nullptr;
  int32_t* n = nullptr;
  double* T = nullptr;
  float* end_gap = nullptr;
  int32_t* order = nullptr;
  int32_t* counts = nullptr;  // [W][M] events per dimension
  int* counter = nullptr;  // window queue heads [2]
  int64_t n_big = 0;       // lane-major: windows run by a whole workgroup
  int64_t big_min = 0;     // lane-major: events from which a window is run by a workgroup
  int32_t scatter = 0;     // M > 16: events per reduce-scatter
  int* flags = nullptr;    // [0] error bits of prepare / check_params
  double* ll_ws = nullptr; // [2 W] likelihoods of the warm and cold starts
  float* fit_ws = nullptr; // L-BFGS per-workgroup vectors
  int64_t fit_ws_floats = 0;
  uint32_t magic = 0;
};

namespace mdhp {

__global__ void reset_counter_kernel(int* counter) {
  counter[0] = 0;
  counter[1] = 0;
}

namespace {
thread_local std::string g_last_msg;
thread_local mdhp_status g_last_status = MDHP_OK;
}  // namespace

mdhp_status mdhp_fail(mdhp_status s, const std::string& msg) {
  g_last_status = s;
  g_last_msg = msg;
  return s;
}

mdhp_status mdhp_hip_fail(hipError_t e, const char* where) {
  return mdhp_fail(e == hipErrorOutOfMemory ? MDHP_E_NOMEM : MDHP_E_HIP,
                   std::string(where) + ": " + hipGetErrorString(e));
}

namespace {

constexpr uint32_t kMagic = 0x4d444850u;  // "MDHP"
constexpr int kErrUnsorted = 1, kErrDomain = 2, kErrParam = 4;

mdhp_status fail(mdhp_status s, const std::string& msg) { return mdhp_fail(s, msg); }
mdhp_status hip_fail(hipError_t e, const char* where) { return mdhp_hip_fail(e, where); }

// Events [b, e) of window w, clamped to [0, n_events] with e >= b; true if
// the offsets needed clamping (or offsets[0] != 0, offsets[W] != n_events).
__device__ __forceinline__ bool window_bounds(const int64_t* __restrict__ offsets, int64_t w,
                                             int64_t W, int64_t n_events, int64_t& b,
                                             int64_t& e) {
  const int64_t ob = offsets[w], oe = offsets[w + 1];
  b = ob < 0 ? 0 : (ob > n_events ? n_events : ob);
  e = oe < b ? b : (oe > n_events ? n_events : oe);
  return b != ob || e != oe || (w == 0 && ob != 0) || (w == W - 1 && oe != n_events) ||
         e - b > INT32_MAX;
}

// Sec. IV-B "Stage 1" counterpart: per event, the gap to the previous event
// of the same window in FP64 (stored FP32; a positive gap never rounds to 0),
// the distance T - t to the window's end (FP64, stored FP32; the compensator
// of windows with a slow decay is summed from it), for per-pair plans (gsd)
// the gap to the previous event of the same dimension, the u8 dimension id,
// and validation of order and domain.  With slot_begin
// the window's events go lane-major: event k of a window of n events lands
// in slot slot_begin[w] + L (k mod c) + k / c, with L = lane_team(n, big_min) chunks
// and c = ceil(n / L), so that chunk l (events l c .. l c + c - 1) is read
// a wave at a time.
__global__ void prepare_kernel(const int64_t* __restrict__ offsets, const double* __restrict__ t,
                               const int32_t* __restrict__ dim, const double* __restrict__ T,
                               const int64_t* __restrict__ slot_begin, int64_t big_min,
                               int64_t W, int M,
                               float* __restrict__ dt, float* __restrict__ tau,
                               float* __restrict__ gsd, uint8_t* __restrict__ d8,
                               float* __restrict__ end_gap, double* __restrict__ Tc,
                               int32_t* __restrict__ counts, int* flags, int64_t n_events,
                               int* __restrict__ wflags) {
  __shared__ int cnt[MDHP_MAX_M];
  for (int64_t w = blockIdx.x; w < W; w += gridDim.x) {
    if (counts) {
      for (int m = threadIdx.x; m < M; m += blockDim.x) cnt[m] = 0;
      __syncthreads();
    }
    // Offsets checked on the host are in range already; the allocation-free
    // path cannot check them before launch and relies on this clamp (see
    // window_bounds) to stay inside the event arrays.
    int64_t b, e;
    const bool bad_off = window_bounds(offsets, w, W, n_events, b, e);
    const int64_t L = lane_team(e - b, big_min);
    const int64_t c = (e - b + L - 1) / L;
    const double Tw = T[w];
    int err = bad_off ? kErrDomain : 0;
    if (!(Tw > 0.0) || !isfinite(Tw)) err |= kErrDomain;
    for (int64_t i = b + threadIdx.x; i < e; i += blockDim.x) {
      const double ti = t[i];
      const double prev = i > b ? t[i - 1] : 0.0;
      if (!(ti >= 0.0) || !(ti <= Tw)) err |= kErrDomain;
      if (i > b && ti < prev) err |= kErrUnsorted;
      const int di = dim[i];
      if (di < 0 || di >= M) err |= kErrDomain;
      float g = (float)(ti - prev);
      if (ti > prev && !(g > 0.f)) g = 1.17549435e-38f;
      const int64_t k = i - b;
      const int64_t dst = slot_begin ? slot_begin[w] + L * (k % c) + k / c : i;
      dt[dst] = g > 0.f ? g : 0.f;
      tau[dst] = (float)fmax(Tw - ti, 0.0);
      if (gsd && di >= 0 && di < M) {
        // Time since the previous event of the same dimension (+inf if
        // none), FP64 difference stored FP32; a positive gap never rounds
        // to 0 (0 means "same time", a tie).  Per dimension the searches
        // telescope to at most n steps, plus at most n for its first
        // event: about 2 M n steps per window, one thread per event.
        int64_t j = i - 1;
        while (j >= b && dim[j] != di) --j;
        float gs = __builtin_inff();
        if (j >= b) {
          gs = (float)(ti - t[j]);
          if (ti > t[j] && !(gs > 0.f)) gs = 1.17549435e-38f;
        }
        gsd[dst] = gs;
      }
      d8[dst] = (uint8_t)(di < 0 ? 0 : (di >= M ? 0 : di));
      if (counts && di >= 0 && di < M) atomicAdd(&cnt[di], 1);
    }
    if (counts) {
      __syncthreads();
      for (int m = threadIdx.x; m < M; m += blockDim.x) counts[w * M + m] = cnt[m];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double last = e > b ? t[e - 1] : 0.0;
      float g = (float)(Tw - last);
      end_gap[w] = g > 0.f ? g : 0.f;
      Tc[w] = Tw;
    }
    if (err) atomicOr(flags, err);
    if (wflags) {  // per window: every thread's bits
      if (threadIdx.x == 0) wflags[w] = 0;
      __syncthreads();
      if (err) atomicOr(&wflags[w], err);
    }
  }
}

// Cold start (see mdhp_cold_start): one thread per parameter entry.
__global__ void cold_start_kernel(const int32_t* __restrict__ counts, const double* __restrict__ T,
                                  int64_t W, int M, int pair, float* mu, float* alpha,
                                  float* beta) {
  const int64_t MM = (int64_t)M * M;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < W * MM; i += stride) {
    const int64_t w = i / MM, e = i % MM;
    alpha[i] = (float)(0.5 / M);
    if (pair) beta[i] = 1.f;
    else if (e == 0) beta[w] = 1.f;
    if (e < M) mu[w * M + e] = (float)(0.5 * fmax((double)counts[w * M + e], 0.5) / T[w]);
  }
}

// mu > 0, alpha >= 0, beta > 0, all finite.
__global__ void check_params_kernel(const float* mu, const float* alpha, const float* beta,
                                    int64_t n_mu, int64_t n_alpha, int64_t n_beta, int* flags) {
  int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_alpha; i += stride) {
    if (i < n_mu && !(mu[i] > 0.f && isfinite(mu[i]))) bad = 1;
    if (!(alpha[i] >= 0.f && isfinite(alpha[i]))) bad = 1;
    if (i < n_beta && !(beta[i] > 0.f && isfinite(beta[i]))) bad = 1;
  }
  if (bad) atomicOr(flags, kErrParam);
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

bool plan_ok(const mdhp_plan* p) { return p && p->magic == kMagic; }

Events events_of(const mdhp_plan* p);

// Likelihood (and gradient if g_mu) of every window: per-pair, lane-major
// (M <= 16) or workgroup (M > 16) kernels, as the plan was laid out.
hipError_t eval_plan(const mdhp_plan* p, const float* mu, const float* alpha, const float* beta,
                     double* ll, float* g_mu, float* g_alpha, float* g_beta, hipStream_t s) {
  const Events ev = events_of(p);
  const bool grad = g_mu != nullptr;
  if (p->beta_mode == MDHP_BETA_PAIR)
    return pair_eval(ev, p->M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, p->counter, s, grad);
  if (p->lane_major)
    return lpc_eval(ev, p->M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, p->counter, s, grad);
  return shared_eval(ev, p->M, p->scatter, mu, alpha, beta, ll, g_mu, g_alpha, g_beta,
                     p->counter, s, grad);
}

Events events_of(const mdhp_plan* p) {
  return Events{p->W,     p->dt,      p->d,     p->begin,  p->n,
                p->T,     p->end_gap, p->order, p->counts, p->n_big, p->tau, p->gsd};
}

template <class T>
hipError_t dev_alloc(T** ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)ptr, count * sizeof(T));
}

void free_plan(mdhp_plan* p) {
  if (!p) return;
  (void)hipFree(p->dt);
  (void)hipFree(p->tau);
  (void)hipFree(p->gsd);
  (void)hipFree(p->d);
  (void)hipFree(p->begin);
  (void)hipFree(p->n);
  (void)hipFree(p->T);
  (void)hipFree(p->end_gap);
  (void)hipFree(p->order);
  (void)hipFree(p->counts);
  (void)hipFree(p->counter);
  (void)hipFree(p->flags);
  (void)hipFree(p->ll_ws);
  (void)hipFree(p->fit_ws);
  p->magic = 0;
  delete p;
}

}  // namespace
}  // namespace mdhp

using namespace mdhp;

extern "C" {

const char* mdhp_status_string(mdhp_status s) {
  switch (s) {
    case MDHP_OK: return "ok";
    case MDHP_E_INVAL: return "invalid argument";
    case MDHP_E_UNSORTED: return "event times decrease inside a window";
    case MDHP_E_DOMAIN: return "event time, dimension or window length out of range";
    case MDHP_E_PARAM: return "invalid parameter value";
    case MDHP_E_NOMEM: return "device allocation failed";
    case MDHP_E_HIP: return "HIP runtime error";
    case MDHP_E_IO: return "checkpoint file error";
    default: return "unknown status";
  }
}

mdhp_status mdhp_last_error(char* buf, size_t n) {
  if (buf && n) {
    std::snprintf(buf, n, "%s", g_last_msg.c_str());
  }
  return g_last_status;
}

}  // extern "C"

namespace {

// Validates and prepares a batch with lane-major team threshold big_min.
mdhp_status build_plan(const mdhp_batch* b, int32_t M, int32_t beta_mode, int64_t big_min,
                       hipStream_t s, mdhp_plan** out) {
  if (!out) return fail(MDHP_E_INVAL, "plan_create: out is NULL");
  *out = nullptr;
  if (!b) return fail(MDHP_E_INVAL, "plan_create: batch is NULL");
  if (M < 1 || M > MDHP_MAX_M) return fail(MDHP_E_INVAL, "plan_create: M must be in [1, 64]");
  if (beta_mode != MDHP_BETA_SHARED && beta_mode != MDHP_BETA_PAIR)
    return fail(MDHP_E_INVAL, "plan_create: unknown beta_mode");
  if (beta_mode == MDHP_BETA_PAIR && M > MDHP_MAX_M_PAIR)
    return fail(MDHP_E_INVAL, "plan_create: per-pair decays support M <= 32");
  if (b->W < 0 || b->n_events < 0) return fail(MDHP_E_INVAL, "plan_create: negative sizes");
  if (b->W > INT32_MAX) return fail(MDHP_E_INVAL, "plan_create: too many windows");
  if (!b->offsets || (b->W > 0 && !b->T) || (b->n_events > 0 && (!b->t || !b->dim)))
    return fail(MDHP_E_INVAL, "plan_create: null array");
  const int64_t W = b->W;
  std::vector<int64_t> off(W + 1);
  hipError_t e = hipMemcpyAsync(off.data(), b->offsets, (W + 1) * sizeof(int64_t),
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "plan_create: reading offsets");
  if (off[0] != 0) return fail(MDHP_E_INVAL, "plan_create: offsets[0] != 0");
  for (int64_t w = 0; w < W; ++w) {
    if (off[w + 1] < off[w]) return fail(MDHP_E_INVAL, "plan_create: offsets decrease");
    if (off[w + 1] - off[w] > INT32_MAX)
      return fail(MDHP_E_INVAL, "plan_create: window has more than 2^31-1 events");
  }
  if (off[W] != b->n_events) return fail(MDHP_E_INVAL, "plan_create: offsets[W] != n_events");

  mdhp_plan* p = new mdhp_plan();
  p->W = W;
  p->N = b->n_events;
  p->M = M;
  p->beta_mode = beta_mode;
  p->magic = kMagic;
  p->big_min = big_min;
  p->scatter = kDefaultScatter;
  const int64_t N = b->n_events;
  // Lane-major slots: L ceil(n_w / L) per window, L = lane_team(n_w, big_min).
  p->lane_major = beta_mode == MDHP_BETA_SHARED && M <= kLaneMajorMaxM;
  std::vector<int64_t> sbeg;
  if (p->lane_major) {
    sbeg.resize(W);
    int64_t acc = 0;
    for (int64_t w = 0; w < W; ++w) {
      const int64_t n = off[w + 1] - off[w], L = lane_team(n, big_min);
      sbeg[w] = acc;
      acc += L * ((n + L - 1) / L);
      if (n >= big_min) ++p->n_big;
    }
    p->slots = acc;
  } else {
    p->slots = N;
  }
  const int64_t fit_ws = beta_mode != MDHP_BETA_SHARED ? 0
                         : p->lane_major             ? lpc_lbfgs_workspace(M, W, p->n_big)
                                                     : shared_lbfgs_workspace(M, W);
  if ((e = dev_alloc(&p->dt, p->slots)) != hipSuccess ||
      (e = dev_alloc(&p->tau, p->slots)) != hipSuccess ||
      (beta_mode == MDHP_BETA_PAIR && (e = dev_alloc(&p->gsd, p->slots)) != hipSuccess) ||
      (e = dev_alloc(&p->d, p->slots)) != hipSuccess ||
      (e = dev_alloc(&p->begin, W)) != hipSuccess || (e = dev_alloc(&p->n, W)) != hipSuccess ||
      (e = dev_alloc(&p->T, W)) != hipSuccess || (e = dev_alloc(&p->end_gap, W)) != hipSuccess ||
      (e = dev_alloc(&p->order, W)) != hipSuccess ||
      (e = dev_alloc(&p->counts, W * M)) != hipSuccess ||
      (e = dev_alloc(&p->counter, 2)) != hipSuccess ||
      (e = dev_alloc(&p->flags, 1)) != hipSuccess ||
      (e = dev_alloc(&p->ll_ws, 2 * W)) != hipSuccess ||
      (fit_ws > 0 && (e = dev_alloc(&p->fit_ws, (size_t)(p->fit_ws_floats = fit_ws))) !=
                         hipSuccess)) {
    free_plan(p);
    return hip_fail(e, "plan_create: allocation");
  }
  // Window sizes and the largest-first order, on the host.
  std::vector<int32_t> cnt(W), order(W);
  for (int64_t w = 0; w < W; ++w) cnt[w] = (int32_t)(off[w + 1] - off[w]);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t c) { return cnt[a] > cnt[c]; });
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, p->flags);
  e = hipGetLastError();
  if (e == hipSuccess && p->lane_major && p->slots > 0) {  // padding slots: gap 0, no dimension
    e = hipMemsetAsync(p->dt, 0, p->slots * sizeof(float), s);
    if (e == hipSuccess) e = hipMemsetAsync(p->tau, 0, p->slots * sizeof(float), s);
    if (e == hipSuccess) e = hipMemsetAsync(p->d, 0xFF, p->slots, s);
  }
  if (e == hipSuccess && W > 0) {
    e = hipMemcpyAsync(p->begin, p->lane_major ? sbeg.data() : off.data(), W * sizeof(int64_t),
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(p->n, cnt.data(), W * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(p->order, order.data(), W * sizeof(int32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) {
      const int grid = (int)std::min<int64_t>(W, 65536);
      hipLaunchKernelGGL(prepare_kernel, dim3(grid), dim3(256), 0, s, b->offsets, b->t, b->dim,
                         b->T, p->lane_major ? p->begin : nullptr, p->big_min, W, M, p->dt,
                         p->tau, p->gsd, p->d, p->end_gap, p->T, p->counts, p->flags,
                         b->n_events, nullptr);
      e = hipGetLastError();
    }
  }
  int flags = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&flags, p->flags, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "plan_create: prepare");
  }
  if (flags & kErrUnsorted) {
    free_plan(p);
    return fail(MDHP_E_UNSORTED, "plan_create: event times decrease inside a window");
  }
  if (flags & kErrDomain) {
    free_plan(p);
    return fail(MDHP_E_DOMAIN, "plan_create: t outside [0, T], dim outside [0, M) or bad T");
  }
  *out = p;
  return MDHP_OK;
}

}  // namespace

extern "C" {

mdhp_status mdhp_plan_create(const mdhp_batch* b, int32_t M, int32_t beta_mode, void* stream,
                             mdhp_plan** out) {
  return build_plan(b, M, beta_mode, kBigWindow, (hipStream_t)stream, out);
}

mdhp_status mdhp_plan_create_scheduled(const mdhp_batch* b, int32_t M, int32_t beta_mode,
                                       int32_t schedule, void* stream, mdhp_plan** out) {
  if (schedule == 0) return mdhp_plan_create(b, M, beta_mode, stream, out);
  if (out) *out = nullptr;
  const bool lane_major = beta_mode == MDHP_BETA_SHARED && M >= 1 && M <= kLaneMajorMaxM;
  if (lane_major) {
    const int32_t c[] = {512, 1024, 2048, 4096, MDHP_TEAM_NEVER};
    bool known = false;
    for (int32_t v : c) known = known || v == schedule;
    if (!known) return fail(MDHP_E_INVAL, "plan_create: schedule is not a candidate");
    return build_plan(b, M, beta_mode, schedule, (hipStream_t)stream, out);
  }
  if (beta_mode != MDHP_BETA_SHARED || !shared_scatter_ok(M, schedule))
    return fail(MDHP_E_INVAL, "plan_create: schedule is not a candidate");
  const mdhp_status st = build_plan(b, M, beta_mode, kBigWindow, (hipStream_t)stream, out);
  if (st == MDHP_OK) (*out)->scatter = schedule;
  return st;
}

void mdhp_plan_destroy(mdhp_plan* p) {
  if (!plan_ok(p)) return;
  (void)hipDeviceSynchronize();
  free_plan(p);
}

int64_t mdhp_plan_windows(const mdhp_plan* p) { return plan_ok(p) ? p->W : 0; }
int64_t mdhp_plan_events(const mdhp_plan* p) { return plan_ok(p) ? p->N : 0; }
int32_t mdhp_plan_dims(const mdhp_plan* p) { return plan_ok(p) ? p->M : 0; }

mdhp_status mdhp_loglik(mdhp_plan* p, const float* mu, const float* alpha, const float* beta,
                        double* ll, void* stream) {
  if (!plan_ok(p)) return fail(MDHP_E_INVAL, "loglik: invalid plan");
  if (p->W > 0 && (!mu || !alpha || !beta || !ll))
    return fail(MDHP_E_INVAL, "loglik: null pointer");
  const hipError_t e = eval_plan(p, mu, alpha, beta, ll, nullptr, nullptr, nullptr,
                                 (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "loglik: launch");
  return MDHP_OK;
}

mdhp_status mdhp_grad(mdhp_plan* p, const float* mu, const float* alpha, const float* beta,
                      double* ll, float* g_mu, float* g_alpha, float* g_beta, void* stream) {
  if (!plan_ok(p)) return fail(MDHP_E_INVAL, "grad: invalid plan");
  if (p->W > 0 && (!mu || !alpha || !beta || !ll || !g_mu || !g_alpha || !g_beta))
    return fail(MDHP_E_INVAL, "grad: null pointer");
  const hipError_t e = eval_plan(p, mu, alpha, beta, ll, g_mu, g_alpha, g_beta,
                                 (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "grad: launch");
  return MDHP_OK;
}

mdhp_status mdhp_fit_batch(mdhp_plan* p, const mdhp_fit_opts* o, float* mu, float* alpha,
                           float* beta, double* ll, int32_t* steps, int32_t* status,
                           int32_t* evals, void* stream) {
  if (!plan_ok(p)) return fail(MDHP_E_INVAL, "fit_batch: invalid plan");
  if (!o) return fail(MDHP_E_INVAL, "fit_batch: opts is NULL");
  if (p->W > 0 && (!mu || !alpha || !beta || !ll || !steps || !status))
    return fail(MDHP_E_INVAL, "fit_batch: null pointer");
  if (o->max_steps < 0 || !(o->ll_tol >= 0.0) ||
      ((o->optimizer == MDHP_OPT_PGD || o->optimizer == MDHP_OPT_PADAM) &&
       (!(o->lr > 0.0) || !std::isfinite(o->lr))) ||
      (o->optimizer != MDHP_OPT_PGD && o->optimizer != MDHP_OPT_PADAM &&
       o->optimizer != MDHP_OPT_LBFGS && o->optimizer != MDHP_OPT_EM) ||
      o->history < 0 || o->history > MDHP_MAX_HISTORY ||
      !(o->mu_floor_rel >= 0.0) || !(o->beta_floor_rel >= 0.0) ||
      (o->optimizer == MDHP_OPT_PADAM &&
       !(o->adam_b1 >= 0.0 && o->adam_b1 < 1.0 && o->adam_b2 >= 0.0 && o->adam_b2 < 1.0 &&
         o->adam_eps >= 0.0)))
    return fail(MDHP_E_INVAL, "fit_batch: invalid options");
  if (o->optimizer == MDHP_OPT_LBFGS && p->beta_mode != MDHP_BETA_SHARED)
    return fail(MDHP_E_INVAL, "fit_batch: L-BFGS needs one decay per window");
  if (o->optimizer == MDHP_OPT_EM && !o->fix_beta)
    return fail(MDHP_E_INVAL, "fit_batch: EM holds the decays; set fix_beta");
  if (o->check_params && p->W > 0) {
    const mdhp_status st = mdhp_check_params(p, mu, alpha, beta, stream);
    if (st != MDHP_OK)
      return st == MDHP_E_PARAM
                 ? fail(MDHP_E_PARAM, "fit_batch: initial mu <= 0, alpha < 0, beta <= 0 or "
                                      "non-finite")
                 : st;
  }
  FitParams fp{o->max_steps,  o->optimizer,      o->fix_beta, o->history > 0 ? o->history : 8,
               o->lr,         o->ll_tol,         o->mu_floor_rel, o->beta_floor_rel,
               o->adam_b1,    o->adam_b2,        o->adam_eps};
  hipStream_t s = (hipStream_t)stream;
  const Events ev = events_of(p);
  hipError_t e =
      p->beta_mode == MDHP_BETA_PAIR
          ? pair_fit(ev, p->M, fp, mu, alpha, beta, ll, steps, status, evals, p->counter, s)
      : p->lane_major ? lpc_fit(ev, p->M, fp, mu, alpha, beta, ll, steps, status, evals,
                                p->fit_ws, p->fit_ws_floats, p->counter, s)
                      : shared_fit(ev, p->M, p->scatter, fp, mu, alpha, beta, ll, steps,
                                   status, evals, p->fit_ws, p->fit_ws_floats, p->counter, s);
  if (e != hipSuccess) return hip_fail(e, "fit_batch: launch");
  return MDHP_OK;
}

mdhp_status mdhp_warm_start(mdhp_plan* p, const float* pred, const float* mean,
                            const float* stdv, const mdhp_fit_opts* o, const float* mu_cold,
                            const float* alpha_cold, const float* beta_cold, float* mu,
                            float* alpha, float* beta, int32_t* used_warm, void* stream) {
  if (!plan_ok(p)) return fail(MDHP_E_INVAL, "warm_start: invalid plan");
  if (p->beta_mode != MDHP_BETA_SHARED)
    return fail(MDHP_E_INVAL, "warm_start: needs one decay per window");
  if (!o) return fail(MDHP_E_INVAL, "warm_start: opts is NULL");
  if (p->W == 0) return MDHP_OK;
  if (!pred || !mean || !stdv || !mu_cold || !alpha_cold || !beta_cold || !mu || !alpha ||
      !beta || !used_warm)
    return fail(MDHP_E_INVAL, "warm_start: null pointer");
  hipStream_t s = (hipStream_t)stream;
  double* ll_w = p->ll_ws;
  double* ll_c = p->ll_ws + p->W;
  hipError_t e = warm_params(pred, mean, stdv, p->counts, p->n, p->T, p->W, p->M,
                             (float)o->mu_floor_rel, (float)o->beta_floor_rel, mu, alpha, beta,
                             s);
  if (e == hipSuccess) e = eval_plan(p, mu, alpha, beta, ll_w, nullptr, nullptr, nullptr, s);
  if (e == hipSuccess)
    e = eval_plan(p, mu_cold, alpha_cold, beta_cold, ll_c, nullptr, nullptr, nullptr, s);
  if (e == hipSuccess)
    e = choose_init(ll_w, ll_c, p->W, p->M, mu_cold, alpha_cold, beta_cold, mu, alpha, beta,
                    used_warm, s);
  if (e != hipSuccess) return hip_fail(e, "warm_start");
  return MDHP_OK;
}

mdhp_status mdhp_cold_start(mdhp_plan* p, float* mu, float* alpha, float* beta, void* stream) {
  if (!plan_ok(p)) return fail(MDHP_E_INVAL, "cold_start: invalid plan");
  if (p->W == 0) return MDHP_OK;
  if (!mu || !alpha || !beta) return fail(MDHP_E_INVAL, "cold_start: null pointer");
  const int64_t n = p->W * p->M * p->M;
  const int grid = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(cold_start_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, p->counts,
                     p->T, p->W, p->M, p->beta_mode == MDHP_BETA_PAIR ? 1 : 0, mu, alpha, beta);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "cold_start: launch");
  return MDHP_OK;
}

mdhp_status mdhp_check_params(mdhp_plan* p, const float* mu, const float* alpha,
                              const float* beta, void* stream) {
  if (!plan_ok(p)) return fail(MDHP_E_INVAL, "check_params: invalid plan");
  if (p->W == 0) return MDHP_OK;
  if (!mu || !alpha || !beta) return fail(MDHP_E_INVAL, "check_params: null pointer");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nm = p->W * p->M, na = p->W * p->M * p->M;
  const int64_t nb = p->beta_mode == MDHP_BETA_SHARED ? p->W : na;
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, p->flags);
  const int grid = (int)std::min<int64_t>((na + 255) / 256, 4096);
  hipLaunchKernelGGL(check_params_kernel, dim3(grid), dim3(256), 0, s, mu, alpha, beta, nm, na,
                     nb, p->flags);
  int flags = 0;
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&flags, p->flags, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "check_params");
  if (flags & kErrParam)
    return fail(MDHP_E_PARAM, "check_params: mu <= 0, alpha < 0, beta <= 0 or non-finite");
  return MDHP_OK;
}

}  // extern "C"

namespace {

// Schedules a plan can be tuned to: kind 1, the events from which a
// lane-major window is run by a whole workgroup; kind 2, the events per
// reduce-scatter of the M > 16 kernels; kind 0, nothing (per-pair decays).
int tune_candidates(const mdhp_plan* p, int32_t* kind, int32_t (&v)[MDHP_TUNE_MAX]) {
  if (p->beta_mode != MDHP_BETA_SHARED) {
    *kind = 0;
    return 0;
  }
  if (p->lane_major) {
    *kind = 1;
    const int32_t c[] = {512, 1024, 2048, 4096, MDHP_TEAM_NEVER};
    for (int i = 0; i < 5; ++i) v[i] = c[i];
    return 5;
  }
  *kind = 2;
  int n = 0;
  for (int32_t b : {4, 8, 16, (int32_t)MDHP_SCATTER_MFMA})
    if (shared_scatter_ok(p->M, b)) v[n++] = b;
  return n;
}

// Switches the plan to schedule `value` of its kind; a new team threshold
// re-prepares the batch (which must be the one the plan was made from).
mdhp_status apply_schedule(mdhp_plan* p, const mdhp_batch* b, int32_t value, hipStream_t s) {
  int32_t kind = 0, v[MDHP_TUNE_MAX];
  const int n = tune_candidates(p, &kind, v);
  bool known = false;
  for (int i = 0; i < n; ++i) known = known || v[i] == value;
  if (!known) return fail(MDHP_E_INVAL, "schedule: value is not a candidate of this plan");
  if (kind == 2) {
    p->scatter = value;
    return MDHP_OK;
  }
  if ((int64_t)value == p->big_min) return MDHP_OK;
  if (!b || b->W != p->W || b->n_events != p->N)
    return fail(MDHP_E_INVAL, "schedule: the batch is not the plan's");
  mdhp_plan* np = nullptr;
  const mdhp_status st = build_plan(b, p->M, p->beta_mode, value, s, &np);
  if (st != MDHP_OK) return st;
  (void)hipStreamSynchronize(s);
  std::swap(*p, *np);  // p takes the new layout; np holds the old buffers
  free_plan(np);
  return MDHP_OK;
}

}  // namespace

extern "C" {

mdhp_status mdhp_plan_set_schedule(mdhp_plan* p, const mdhp_batch* b, int32_t value,
                                   void* stream) {
  if (!plan_ok(p)) return fail(MDHP_E_INVAL, "set_schedule: invalid plan");
  return apply_schedule(p, b, value, (hipStream_t)stream);
}

mdhp_status mdhp_plan_dim_counts(const mdhp_plan* p, int32_t* counts, void* stream) {
  if (!plan_ok(p)) return fail(MDHP_E_INVAL, "dim_counts: invalid plan");
  const int64_t n = p->W * (int64_t)p->M;
  if (n == 0) return MDHP_OK;
  if (!counts) return fail(MDHP_E_INVAL, "dim_counts: null pointer");
  const hipError_t e = hipMemcpyAsync(counts, p->counts, n * sizeof(int32_t),
                                      hipMemcpyDeviceToDevice, (hipStream_t)stream);
  return e == hipSuccess ? MDHP_OK : hip_fail(e, "dim_counts");
}

int32_t mdhp_plan_schedule(const mdhp_plan* p) {
  if (!plan_ok(p) || p->beta_mode != MDHP_BETA_SHARED) return 0;
  return p->lane_major ? (int32_t)std::min<int64_t>(p->big_min, MDHP_TEAM_NEVER) : p->scatter;
}

mdhp_status mdhp_plan_autotune(mdhp_plan* p, const mdhp_batch* b, const mdhp_fit_opts* o,
                               int32_t reps, mdhp_tune_result* r, void* stream) {
  if (!plan_ok(p)) return fail(MDHP_E_INVAL, "autotune: invalid plan");
  if (!r || reps < 1) return fail(MDHP_E_INVAL, "autotune: bad result pointer or reps");
  hipStream_t s = (hipStream_t)stream;
  std::memset(r, 0, sizeof(*r));
  int32_t kind = 0, v[MDHP_TUNE_MAX];
  const int n = tune_candidates(p, &kind, v);
  r->kind = kind;
  if (n == 0 || p->W == 0) return MDHP_OK;
  if (kind == 1 && (!b || b->W != p->W || b->n_events != p->N))
    return fail(MDHP_E_INVAL, "autotune: the batch is not the plan's");
  const int64_t W = p->W, M = p->M;
  float *mu0 = nullptr, *al0 = nullptr, *be0 = nullptr, *mu = nullptr, *al = nullptr,
        *be = nullptr, *gmu = nullptr, *gal = nullptr, *gbe = nullptr;
  double* ll = nullptr;
  int32_t *steps = nullptr, *status = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipSuccess;
  auto cleanup = [&]() {
    for (void* q : {(void*)mu0, (void*)al0, (void*)be0, (void*)mu, (void*)al, (void*)be,
                    (void*)gmu, (void*)gal, (void*)gbe, (void*)ll, (void*)steps, (void*)status})
      (void)hipFree(q);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if ((e = dev_alloc(&mu0, W * M)) != hipSuccess || (e = dev_alloc(&al0, W * M * M)) != hipSuccess ||
      (e = dev_alloc(&be0, W)) != hipSuccess || (e = dev_alloc(&mu, W * M)) != hipSuccess ||
      (e = dev_alloc(&al, W * M * M)) != hipSuccess || (e = dev_alloc(&be, W)) != hipSuccess ||
      (e = dev_alloc(&gmu, W * M)) != hipSuccess || (e = dev_alloc(&gal, W * M * M)) != hipSuccess ||
      (e = dev_alloc(&gbe, W)) != hipSuccess || (e = dev_alloc(&ll, W)) != hipSuccess ||
      (e = dev_alloc(&steps, W)) != hipSuccess || (e = dev_alloc(&status, W)) != hipSuccess ||
      (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    cleanup();
    return hip_fail(e, "autotune: allocation");
  }
  mdhp_status st = MDHP_OK;
  int best = -1;
  for (int i = 0; i < n && st == MDHP_OK; ++i) {
    st = apply_schedule(p, b, v[i], s);
    if (st != MDHP_OK) break;
    st = mdhp_cold_start(p, mu0, al0, be0, s);
    float fastest = 0.f;
    for (int rep = 0; rep <= reps && st == MDHP_OK; ++rep) {  // rep 0 warms up
      if (o) {
        e = hipMemcpyAsync(mu, mu0, W * M * sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
          e = hipMemcpyAsync(al, al0, W * M * M * sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
          e = hipMemcpyAsync(be, be0, W * sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) break;
      }
      if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
      st = o ? mdhp_fit_batch(p, o, mu, al, be, ll, steps, status, nullptr, s)
             : mdhp_grad(p, mu0, al0, be0, ll, gmu, gal, gbe, s);
      if (st != MDHP_OK) break;
      if ((e = hipEventRecord(e1, s)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess)
        break;
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      if (rep > 0) fastest = rep == 1 ? ms : std::min(fastest, ms);
    }
    if (e != hipSuccess && st == MDHP_OK) st = hip_fail(e, "autotune: timing");
    r->value[i] = v[i];
    r->ms[i] = fastest;  // the least disturbed repetition
    r->n = i + 1;
    if (st == MDHP_OK && (best < 0 || r->ms[i] < r->ms[best])) best = i;
  }
  cleanup();
  if (st != MDHP_OK) return st;
  r->chosen = best;
  return apply_schedule(p, b, v[best], s);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free likelihood and gradient (mdhp_grad_static).  The compact
// events and per-window arrays of the call live in `scratch`, a fixed device
// array of this library: one copy per GPU, held until the process ends,
// shared by every call on that GPU (calls that overlap on one GPU race).
namespace mdhp {
namespace {

constexpr int64_t kStaticEvents = MDHP_STATIC_MAX_EVENTS;
constexpr int64_t kStaticWindows = MDHP_STATIC_MAX_WINDOWS;

constexpr size_t up256(size_t x) { return (x + 255) & ~size_t(255); }
// Byte offsets of the arrays in scratch, sized for the largest call.
constexpr size_t kOffDt = 0;
constexpr size_t kOffTau = kOffDt + up256(kStaticEvents * sizeof(float));
constexpr size_t kOffD = kOffTau + up256(kStaticEvents * sizeof(float));
constexpr size_t kOffBegin = kOffD + up256(kStaticEvents);
constexpr size_t kOffN = kOffBegin + up256(kStaticWindows * sizeof(int64_t));
constexpr size_t kOffT = kOffN + up256(kStaticWindows * sizeof(int32_t));
constexpr size_t kOffEnd = kOffT + up256(kStaticWindows * sizeof(double));
constexpr size_t kOffOrder = kOffEnd + up256(kStaticWindows * sizeof(float));
constexpr size_t kOffCounts = kOffOrder + up256(kStaticWindows * sizeof(int32_t));
constexpr size_t kOffWflags = kOffCounts + up256(kStaticWindows * MDHP_MAX_M * sizeof(int32_t));
constexpr size_t kOffCounter = kOffWflags + up256(kStaticWindows * sizeof(int32_t));
constexpr size_t kOffFlags = kOffCounter + 256;
constexpr size_t kStaticBytes = kOffFlags + 256;
static_assert(kStaticBytes == MDHP_STATIC_BYTES, "scratch layout and header disagree");

__device__ __align__(256) unsigned char scratch[kStaticBytes];

// Per device: the address of that device's copy of scratch.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Window table of the call (natural order) and the cleared queue head.
__global__ void static_windows_kernel(const int64_t* __restrict__ offsets, int64_t W,
                                      int64_t n_events, int64_t* __restrict__ begin,
                                      int32_t* __restrict__ n, int32_t* __restrict__ order,
                                      int* counter) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < W; w += stride) {
    int64_t b, e;
    (void)window_bounds(offsets, w, W, n_events, b, e);
    begin[w] = b;
    n[w] = (int32_t)(e - b > INT32_MAX ? 0 : e - b);
    order[w] = (int32_t)w;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    counter[0] = 0;
    counter[1] = 0;
  }
}

// Windows whose events failed validation: ll and the gradient are NaN.
__global__ void static_flag_kernel(const int* __restrict__ wflags, int64_t W, int M,
                                   double* ll, float* g_mu, float* g_alpha, float* g_beta) {
  const int64_t MM = (int64_t)M * M;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < W * MM; i += stride) {
    const int64_t w = i / MM, e = i % MM;
    if (!wflags[w]) continue;
    if (g_alpha) g_alpha[i] = __builtin_nanf("");
    if (e < M && g_mu) g_mu[w * M + e] = __builtin_nanf("");
    if (e == 0) {
      ll[w] = __builtin_nan("");
      if (g_beta) g_beta[w] = __builtin_nanf("");
    }
  }
}

}  // namespace
}  // namespace mdhp

extern "C" {

mdhp_status mdhp_grad_static(const mdhp_batch* b, int32_t M, const float* mu, const float* alpha,
                             const float* beta, double* ll, float* g_mu, float* g_alpha,
                             float* g_beta, void* stream) {
  if (!b) return fail(MDHP_E_INVAL, "grad_static: batch is NULL");
  if (M < 1 || M > MDHP_MAX_M) return fail(MDHP_E_INVAL, "grad_static: M must be in [1, 64]");
  if (b->W < 0 || b->n_events < 0) return fail(MDHP_E_INVAL, "grad_static: negative sizes");
  if (b->W > kStaticWindows || b->n_events > kStaticEvents)
    return fail(MDHP_E_INVAL, "grad_static: batch larger than the static workspace (at most " +
                                  std::to_string(kStaticWindows) + " windows and " +
                                  std::to_string(kStaticEvents) + " events)");
  const bool grad = g_mu || g_alpha || g_beta;
  if (grad && !(g_mu && g_alpha && g_beta))
    return fail(MDHP_E_INVAL, "grad_static: give all three gradient arrays or none");
  if (b->W == 0) return MDHP_OK;
  if (!b->offsets || !b->T || (b->n_events > 0 && (!b->t || !b->dim)) || !mu || !alpha ||
      !beta || !ll)
    return fail(MDHP_E_INVAL, "grad_static: null pointer");
  void* base = nullptr;
  hipError_t e = scratch_address(&base);
  if (e != hipSuccess) return hip_fail(e, "grad_static: scratch address");
  unsigned char* sc = static_cast<unsigned char*>(base);
  float* dt = reinterpret_cast<float*>(sc + kOffDt);
  float* tau = reinterpret_cast<float*>(sc + kOffTau);
  uint8_t* d8 = sc + kOffD;
  int64_t* begin = reinterpret_cast<int64_t*>(sc + kOffBegin);
  int32_t* n = reinterpret_cast<int32_t*>(sc + kOffN);
  double* Tc = reinterpret_cast<double*>(sc + kOffT);
  float* end_gap = reinterpret_cast<float*>(sc + kOffEnd);
  int32_t* order = reinterpret_cast<int32_t*>(sc + kOffOrder);
  int32_t* counts = reinterpret_cast<int32_t*>(sc + kOffCounts);
  int* wflags = reinterpret_cast<int*>(sc + kOffWflags);
  int* counter = reinterpret_cast<int*>(sc + kOffCounter);
  int* flags = reinterpret_cast<int*>(sc + kOffFlags);

  hipStream_t s = (hipStream_t)stream;
  const int64_t W = b->W;
  const int grid = (int)std::min<int64_t>(W, 65536);
  hipLaunchKernelGGL(static_windows_kernel, dim3((unsigned)((W + 255) / 256)), dim3(256), 0, s,
                     b->offsets, W, b->n_events, begin, n, order, counter);
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, s, flags);
  hipLaunchKernelGGL(prepare_kernel, dim3(grid), dim3(256), 0, s, b->offsets, b->t, b->dim, b->T,
                     nullptr, (int64_t)0, W, M, dt, tau, nullptr, d8, end_gap, Tc, counts, flags,
                     b->n_events, wflags);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "grad_static: prepare");
  const Events ev{W, dt, d8, begin, n, Tc, end_gap, order, counts, 0, tau, nullptr};
  e = shared_eval_wide(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta, counter, s, grad);
  if (e != hipSuccess) return hip_fail(e, "grad_static: launch");
  const int64_t work = W * (int64_t)M * M;
  hipLaunchKernelGGL(static_flag_kernel, dim3((unsigned)std::min<int64_t>((work + 255) / 256, 65536)),
                     dim3(256), 0, s, wflags, W, M, ll, g_mu, g_alpha, g_beta);
  e = hipGetLastError();
  return e == hipSuccess ? MDHP_OK : hip_fail(e, "grad_static: launch");
}

}  // extern "C"
