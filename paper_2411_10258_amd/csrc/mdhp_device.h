// Device helpers shared by the library's kernels: cross-lane operations
// within groups of P consecutive lanes of a 64-wide wavefront.
#pragma once

#include <utility>

#include "mdhp_internal.h"

namespace mdhp {

// Orders the calling wavefront's LDS accesses before and after this point
// (lanes of one wavefront exchanging data through LDS).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// v of another lane of the same 16-lane row by a DPP lane map (both halves
// of the double moved).
template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double,
                            ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double lane64(double v, int l) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum (or max) over the wave in a fixed order: butterflies inside each
// 16-lane row by DPP (xor 1, xor 2, then the row's half and full mirrors),
// then the four row totals read as scalars.  The result is uniform.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp64<0x141>(v);  // row_half_mirror
  v += dpp64<0x140>(v);  // row_mirror
  return (lane64(v, 0) + lane64(v, 16)) + (lane64(v, 32) + lane64(v, 48));
}

__device__ __forceinline__ double wave_max(double v) {
  v = fmax(v, dpp64<0xB1>(v));
  v = fmax(v, dpp64<0x4E>(v));
  v = fmax(v, dpp64<0x141>(v));
  v = fmax(v, dpp64<0x140>(v));
  return fmax(fmax(lane64(v, 0), lane64(v, 16)), fmax(lane64(v, 32), lane64(v, 48)));
}

// v of rows 2k and 2k+1 (16 lanes each) added, in every lane of both rows
// (a lane swap between the two rows).
__device__ __forceinline__ float rows_pair_sum(float v) {
  const unsigned u = __builtin_bit_cast(unsigned, v);
  const auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  const unsigned x = r[0], y = r[1];  // (a bit cast of r[i] itself reads element 0)
  return __uint_as_float(x) + __uint_as_float(y);
}

// v of the two 32-lane halves of the wavefront added, in every lane.
__device__ __forceinline__ float halves_sum(float v) {
  const unsigned u = __builtin_bit_cast(unsigned, v);
  const auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
  const unsigned x = r[0], y = r[1];
  return __uint_as_float(x) + __uint_as_float(y);
}

// Sum over the P consecutive lanes of a group; every lane gets the sum.
// Lane swaps across rows and halves: no LDS traffic.
template <int P>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (P >= 2) v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]: lane ^ 1
  if constexpr (P >= 4) v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]: lane ^ 2
  if constexpr (P >= 8) v += dpp<0x141>(v);  // row_half_mirror: the other quad of the 8
  if constexpr (P >= 16) v += dpp<0x140>(v); // row_mirror: the other 8 of the 16-lane row
  if constexpr (P >= 32) v = rows_pair_sum(v);
  if constexpr (P >= 64) v = halves_sum(v);
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

// v from lane - K of the same 16-lane row, 0 where that lane is outside the
// row (DPP row_shr with bound_ctrl).
template <int K>
__device__ __forceinline__ float row_shr(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                0x110 + K, 0xF, 0xF, true));
}

// v from lane - 1 of the wavefront, 0 in lane 0 (DPP wave_shr:1 with
// bound_ctrl).
__device__ __forceinline__ float wave_shr1(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                0x138, 0xF, 0xF, true));
}

// Inclusive prefix sum over the P lanes of a group (lane order).  Within
// 16-lane rows by DPP shifts; groups wider than a row add the earlier rows'
// totals, read from the rows' last lanes as scalars.
template <int P>
__device__ __forceinline__ float group_scan(float v, int lane) {
  constexpr int R = P < 16 ? P : 16;
  const int lr = lane & (R - 1);
  float y;
  y = row_shr<1>(v);
  if (R > 1 && lr >= 1) v += y;
  if constexpr (R > 2) {
    y = row_shr<2>(v);
    if (lr >= 2) v += y;
  }
  if constexpr (R > 4) {
    y = row_shr<4>(v);
    if (lr >= 4) v += y;
  }
  if constexpr (R > 8) {
    y = row_shr<8>(v);
    if (lr >= 8) v += y;
  }
  if constexpr (P > 16) {
    // Add the totals of the earlier 16-lane rows of the group.
    static_assert(P == 32 || P == 64, "");
    const int row = lane >> 4;
    const int vi = __builtin_bit_cast(int, v);
    const float r15 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(vi, 15));
    const float r47 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(vi, 47));
    float add;
    if constexpr (P == 32) {
      add = row >= 1 ? ((threadIdx.x & 32) ? r47 : r15) : 0.f;
    } else {
      const float r31 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(vi, 31));
      add = row >= 1 ? r15 : 0.f;
      add += (row >= 2 ? r31 : 0.f) + (row >= 3 ? r47 : 0.f);
    }
    v += add;
  }
  return v;
}

// L-BFGS vectors of one team (T threads, K parameter slots per thread) in
// the global workspace: vector v, slot k of team thread t at float
// (v * K + k) * T + t, so that one wavefront's access to a slot is 256
// contiguous bytes.  Vectors 0..2 are x, g and d of the current iteration,
// then the history pairs s_j (3 + j) and y_j (3 + kMaxHistory + j).  Buffer
// loads and stores with the thread's byte offset in one register and the
// slot's in a scalar: no per-slot address registers.  `base` must be the
// same for every thread of the team.
constexpr int kLbfgsVectors = 3 + 2 * kMaxHistory;

template <int K, int T>
struct LbfgsWs {
  __amdgpu_buffer_rsrc_t r;
  int voff;
  __device__ LbfgsWs(float* base, int t) {
    r = __builtin_amdgcn_make_buffer_rsrc(base, 0, kLbfgsVectors * K * T * 4, 0x00020000);
    voff = t * 4;
  }
  __device__ float ld(int v, int k) const {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, (v * K + k) * T * 4, 0));
  }
  __device__ void st(int v, int k, float x) const {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, voff, (v * K + k) * T * 4, 0);
  }
  static constexpr int X = 0, G = 1, D = 2;
  static constexpr int S(int j) { return 3 + j; }
  static constexpr int Y(int j) { return 3 + kMaxHistory + j; }
};

template <class K>
int occupancy_grid(K kernel, int threads, int64_t W) {
  int dev = 0, cus = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0);
  int64_t g = (int64_t)std::max(cus, 1) * std::max(per_cu, 1);
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, W));
}

}  // namespace mdhp
