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
};

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
                       const int32_t* n, const double* T, int64_t W, int M, float mu_floor_rel,
                       float beta_floor_rel, float* mu, float* alpha, float* beta, hipStream_t s);
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
// Floats of workspace the L-BFGS fit needs for a plan of W windows.
int64_t shared_lbfgs_workspace(int M, int64_t W);
hipError_t pair_eval(const Events& ev, int M, const float* mu, const float* alpha,
                     const float* beta, double* ll, float* g_mu, float* g_alpha, float* g_beta,
                     int* counter, hipStream_t s, bool grad);
hipError_t pair_fit(const Events& ev, int M, const FitParams& o, float* mu, float* alpha,
                    float* beta, double* ll, int* steps, int* status, int* evals, int* counter,
                    hipStream_t s);

}  // namespace mdhp
