// Internal declarations shared by the library's HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "mdhp.h"

namespace mdhp {

constexpr int kBlock = 256;  // threads per workgroup (4 waves of 64)
#ifndef MDHP_MIN_BLOCKS
#define MDHP_MIN_BLOCKS 1
#endif
// Workgroups per CU the fit kernels are compiled for (register budget).
constexpr int kMinBlocks = MDHP_MIN_BLOCKS;
constexpr int kMaxHistory = 16;  // largest L-BFGS memory

// FP64 G_R accumulators each thread owns for a P x P matrix.
constexpr int own_count(int P) { return P * P >= kBlock ? P * P / kBlock : 1; }

// Lanes per group: M rounded up to a power of two, at least 4.
inline int lanes_for(int M) {
  int p = 4;
  while (p < M) p <<= 1;
  return p;
}

// Compact events of a prepared batch (device pointers).
struct Events {
  int64_t W;
  const float* dt;       // gap to the previous event of the window (the first: t_0), FP64-computed
  const uint8_t* d;      // dimension ids
  const int64_t* begin;  // [W] first event (compact) or first slot (lane-major) of each window
  const int32_t* n;      // [W] events per window
  const double* T;       // [W] window lengths
  const float* end_gap;  // [W] T - t_last (T for an empty window), FP64-computed
  const int32_t* order;  // [W] window ids, largest first
  const int32_t* counts; // [W][M] events per dimension
  int64_t n_big;         // lane-major plans: windows of >= kBigWindow events (a prefix of order)
  const float* tau;      // T - t per event (same slots as dt), FP64-computed
  const float* gsd;      // per-pair plans: gap to the previous event of the same dimension
};

// Windows whose decay is slow against their length (beta T below the
// kernel's threshold) take the compensator sums from the events' distances
// to T: sum_k -expm1(-beta tau_k) / beta and sum_k h(beta tau_k) / beta,
// h(x) = x e^{-x} + expm1(-x), every term of one sign.  The end-state form
// N - E subtracts two nearly equal numbers there.
// beta T below which the lane-major kernels (M <= 16) take the event form.
constexpr double kSlowDecayLane = 8.0;
// beta T below which the lane-per-dimension kernels (16 < M <= 64) take it.
constexpr double kSlowDecayDim = 2.0;
// min over pairs of beta_mn T below which the per-pair kernels take it.
constexpr double kSlowDecayPair = 4.0;
// Both by their Taylor series below x = 0.5 (to x^12, relative error below
// 1e-9 there), above it from one exponential (cancellation at most ~4x).
__device__ __forceinline__ float comp_q(float x) {  // 1 - e^{-x}
  if (x < 0.5f) {
    // sum_{j >= 1} (-1)^{j+1} x^j / j!
    float p = -1.f / 479001600.f;
    p = fmaf(p, x, 1.f / 39916800.f);
    p = fmaf(p, x, -1.f / 3628800.f);
    p = fmaf(p, x, 1.f / 362880.f);
    p = fmaf(p, x, -1.f / 40320.f);
    p = fmaf(p, x, 1.f / 5040.f);
    p = fmaf(p, x, -1.f / 720.f);
    p = fmaf(p, x, 1.f / 120.f);
    p = fmaf(p, x, -1.f / 24.f);
    p = fmaf(p, x, 1.f / 6.f);
    p = fmaf(p, x, -1.f / 2.f);
    p = fmaf(p, x, 1.f);
    return x * p;
  }
  return 1.f - __expf(-x);
}
__device__ __forceinline__ float comp_h(float x) {  // x e^{-x} - (1 - e^{-x})
  if (x < 0.5f) {
    // -sum_{j >= 2} (-1)^j (j - 1) x^j / j!
    float p = 11.f / 479001600.f;
    p = fmaf(p, x, -10.f / 39916800.f);
    p = fmaf(p, x, 9.f / 3628800.f);
    p = fmaf(p, x, -8.f / 362880.f);
    p = fmaf(p, x, 7.f / 40320.f);
    p = fmaf(p, x, -6.f / 5040.f);
    p = fmaf(p, x, 5.f / 720.f);
    p = fmaf(p, x, -4.f / 120.f);
    p = fmaf(p, x, 3.f / 24.f);
    p = fmaf(p, x, -2.f / 6.f);
    p = fmaf(p, x, 1.f / 2.f);
    return -(x * x) * p;
  }
  const float e = __expf(-x);
  return fmaf(x, e, e - 1.f);
}

// Fit options as the kernels read them.
struct FitParams {
  int max_steps;
  int optimizer;
  int fix_beta;
  int history;
  double lr, ll_tol, mu_floor_rel, beta_floor_rel, b1, b2, eps;
};

__global__ void reset_counter_kernel(int* counter);

// Records the calling thread's last error and returns its status.
mdhp_status mdhp_fail(mdhp_status s, const std::string& msg);
mdhp_status mdhp_hip_fail(hipError_t e, const char* where);

hipError_t warm_params(const float* pred, const float* mean, const float* stdv,
                       const int32_t* counts, const int32_t* n, const double* T, int64_t W,
                       int M, float mu_floor_rel, float beta_floor_rel, float* mu, float* alpha,
                       float* beta, hipStream_t s);
hipError_t choose_init(const double* ll_warm, const double* ll_cold, int64_t W, int M,
                       const float* mu_c, const float* al_c, const float* be_c, float* mu,
                       float* alpha, float* beta, int32_t* used_warm, hipStream_t s);

// Zeroes the two queue heads counter[0..1].
inline void reset_counter(int* counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
}

#ifndef MDHP_LANE_MAJOR_MAX_M
#define MDHP_LANE_MAJOR_MAX_M 16
#endif
// Largest M whose shared-decay plans use the lane-major layout and kernels.
constexpr int kLaneMajorMaxM = MDHP_LANE_MAJOR_MAX_M;
// Lane-major windows of at least big_min events are laid out for, and run
// by, a whole workgroup (256 chunks); shorter ones by one wavefront (64).
// The default threshold; a plan can be tuned to another.
constexpr int64_t kBigWindow = 1024;
#ifndef MDHP_LPC_WAVES
#define MDHP_LPC_WAVES 4
#endif
// Workgroup of the lane-major kernels: MDHP_LPC_WAVES wavefronts, the team
// that runs a window of at least big_min events.
constexpr int kLpcBlock = 64 * MDHP_LPC_WAVES;
// Default events per reduce-scatter of the M > 16 kernels.
constexpr int kDefaultScatter = 8;
// The scatter value of the M > 32 schedule that sums the intensities of
// 16-event blocks on the matrix cores instead of a reduce-scatter.
constexpr int kScatterMfma = MDHP_SCATTER_MFMA;
__host__ __device__ inline int64_t lane_team(int64_t n, int64_t big_min) {
  return n >= big_min ? kLpcBlock : 64;
}

// Lane-major (one chunk per lane, one window per wave) kernels, M <= 16.
hipError_t lpc_eval(const Events& ev, int M, const float* mu, const float* alpha,
                    const float* beta, double* ll, float* g_mu, float* g_alpha, float* g_beta,
                    int* counter, hipStream_t s, bool grad);
hipError_t lpc_fit(const Events& ev, int M, const FitParams& o, float* mu, float* alpha,
                   float* beta, double* ll, int* steps, int* status, int* evals, float* ws,
                   int64_t ws_floats, int* counter, hipStream_t s);
int64_t lpc_lbfgs_workspace(int M, int64_t W, int64_t n_big);

// Workgroup-per-window kernels for the compact layout, 16 < M <= 64.
// scatter: events per reduce-scatter (M > 16; see shared_scatter_ok).
hipError_t shared_eval(const Events& ev, int M, int scatter, const float* mu, const float* alpha,
                       const float* beta, double* ll, float* g_mu, float* g_alpha, float* g_beta,
                       int* counter, hipStream_t s, bool grad);
hipError_t shared_fit(const Events& ev, int M, int scatter, const FitParams& o, float* mu,
                      float* alpha, float* beta, double* ll, int* steps, int* status, int* evals,
                      float* ws, int64_t ws_floats, int* counter, hipStream_t s);
bool shared_scatter_ok(int M, int scatter);
// The lane-per-dimension kernels for any M <= 64 (groups of 32 lanes up to
// M = 32, 64 above), default scatter; compact (not lane-major) events.
hipError_t shared_eval_wide(const Events& ev, int M, const float* mu, const float* alpha,
                            const float* beta, double* ll, float* g_mu, float* g_alpha,
                            float* g_beta, int* counter, hipStream_t s, bool grad);
// Floats of workspace the L-BFGS fit needs for a plan of W windows.
int64_t shared_lbfgs_workspace(int M, int64_t W);
hipError_t pair_eval(const Events& ev, int M, const float* mu, const float* alpha,
                     const float* beta, double* ll, float* g_mu, float* g_alpha, float* g_beta,
                     int* counter, hipStream_t s, bool grad);
hipError_t pair_fit(const Events& ev, int M, const FitParams& o, float* mu, float* alpha,
                    float* beta, double* ll, int* steps, int* status, int* evals, int* counter,
                    hipStream_t s);

}  // namespace mdhp
