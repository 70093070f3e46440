// Internal declarations shared by the library's HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "mdhp.h"

namespace mdhp {

constexpr int kBlock = 256;  // threads per workgroup (4 waves of 64)

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
  const int64_t* begin;  // [W] first event of each window
  const int32_t* n;      // [W] events per window
  const double* T;       // [W] window lengths
  const float* end_gap;  // [W] T - t_last (T for an empty window), FP64-computed
  const int32_t* order;  // [W] window ids, largest first
};

// Fit options as the kernels read them.
struct FitParams {
  int max_steps;
  int optimizer;
  int fix_beta;
  double lr, ll_tol, mu_floor_rel, beta_floor_rel, b1, b2, eps;
};

__global__ void reset_counter_kernel(int* counter);

inline void reset_counter(int* counter, hipStream_t s) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, counter);
}

hipError_t shared_eval(const Events& ev, int M, const float* mu, const float* alpha,
                       const float* beta, double* ll, float* g_mu, float* g_alpha, float* g_beta,
                       int* counter, hipStream_t s, bool grad);
hipError_t shared_fit(const Events& ev, int M, const FitParams& o, float* mu, float* alpha,
                      float* beta, double* ll, int* steps, int* status, int* counter,
                      hipStream_t s);
hipError_t pair_eval(const Events& ev, int M, const float* mu, const float* alpha,
                     const float* beta, double* ll, float* g_mu, float* g_alpha, float* g_beta,
                     int* counter, hipStream_t s, bool grad);
hipError_t pair_fit(const Events& ev, int M, const FitParams& o, float* mu, float* alpha,
                    float* beta, double* ll, int* steps, int* status, int* counter,
                    hipStream_t s);

}  // namespace mdhp
