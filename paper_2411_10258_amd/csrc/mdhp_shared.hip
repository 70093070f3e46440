// Shared-decay (one beta per window) evaluation of the MDHP log-likelihood
// of Eq. (5) and its gradient, and the persistent projected-gradient fit.
//
// One workgroup (256 threads) owns one window at a time; windows are taken
// largest first from an atomic queue.  Lanes are grouped in groups of P
// lanes (P = M rounded up to a power of two, 4..64); lane n of a group holds
// component n of the decay state of its chunk of events:
//   R_n(i) = sum_{k: d_k = n, t_k < t_i} e^{-beta (t_i - t_k)}        (Part1's inner sum)
//   S_n(i) = sum_{k: d_k = n, t_k < t_i} (t_i - t_k) e^{-beta (t_i - t_k)}  (= -dR/dbeta)
// with the recursion R <- a (R + P), S <- a S + dt R, a = e^{-beta dt}, where
// P counts the events that share the previous time (they are folded in only
// when time moves on, so equal times never excite each other).
//
// Each group owns one contiguous chunk of the window (N / G events).  Pass 1
// computes every chunk's affine carry from a zero start, one event per lane
// (suffix sums of the gaps, one exponential per event, LDS atomics into the
// chunk's state); one group combines the carries in order (the scan of the
// (a, delta, b_R, b_S) monoid); pass 2 re-runs every chunk from its exact
// start state and accumulates, per event i with target m = d_i:
//   lambda_i = mu_m + sum_n alpha_mn R_n(i)          (Eq. (2) at t_i)
//   ll      += log lambda_i                          (Part1)
//   G_R[m][n] += R_n(i) / lambda_i                   (d ll / d alpha, Part1 share)
//   Gmu[m]  += 1 / lambda_i
//   Gb      += sum_n alpha_mn S_n(i) / lambda_i      (d ll / d beta, Part1 share)
// For P >= 32 a group runs its chunk P events at a time: the block's gaps,
// decays and dimensions are staged in LDS and read back as broadcasts; the
// recursion runs B = 8 events, then one reduce-scatter across the group's
// lanes (lane swaps 32 and 16 apart, DPP within rows) turns the B partial
// dot products alpha_{d_i n} R_n(i) into intensities, P / B lanes per
// event.  At P = 64 each wave keeps its chunk's G_R in registers (lane n:
// column n) and G_R[d_i][n] += R_n(i) / lambda_i is one FMA on the register
// of row d_i, with 1 / lambda_i read from its lane as a scalar; at P = 32
// the reciprocals return through LDS and the row update is one LDS add per
// event and lane (lane n owns column n, so the adds of one event never
// collide).  A block of events without equal times skips the
// pending-count select of the recursion.  The pending one-hot row [d_i = n] is
// read from LDS next to alpha_{d_i n}.  LDS sums that several lanes add to
// (chunk carries, G_R at P = 32, Gmu) have one copy per group or wavefront:
// adds from different wavefronts never meet, and the copies are summed in a
// fixed order, so that a window's results do not depend on timing.
// The compensator (Part2 + Part3, Appendix B) needs
//   E_n = sum_{k: d_k = n} e^{-beta (T - t_k)},  F_n = sum (T - t_k) e^{-beta (T - t_k)},
// which are the scan state advanced from the last event to T.
// Per-lane FP32 partial sums are reduced in FP64 at the end of the window.

#include "mdhp_device.h"

namespace mdhp {

namespace {

#ifndef MDHP_BATCH
#define MDHP_BATCH 16
#endif
// Events per pass-2 batch (at most the group size).
constexpr int kBatch = MDHP_BATCH;
// Events per reduce-scatter for groups of 32 or 64 lanes: the default, and
// the choices a plan can be tuned to.
constexpr int kScatter = kDefaultScatter;

typedef float f32x32 __attribute__((ext_vector_type(32)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int P>
struct SharedLds {
  static constexpr bool kLaneDim = P >= 32;            // pass 2 by reduce-scatter
  static constexpr int G = kBlock / P;                 // groups (chunks) per tile
  // G_R copies: one per wavefront wherever its lanes add into LDS (only the
  // register form at P = 64 needs a single transfer buffer), so that adds
  // from different wavefronts never meet and the sums do not depend on
  // timing.
  static constexpr int NCOPY = P == 64 ? 1 : kBlock / 64;
  static constexpr int AR = kLaneDim ? P + 1 : P;      // rows of ao and gR (row P: padding events)
  static constexpr int NG = kLaneDim ? G : 1;
  // .x: alpha[m * P + n], zero outside M x M and in row P; .y: [m == n].
  float2 ao[AR * P];
  float mu[P];         // zero outside M
  float colsum[P];     // sum_m alpha_mn
  float cR[G][P], cS[G][P], cP[G][P];  // chunk carries, then chunk start states
  float cA[G], cD[G];
  int cF[G];
  float tR[P], tS[P], tP[P];  // state after the last event of the tiles done so far
  float gR[NCOPY][AR * P];    // FP32 tile partials of G_R
  float4 meta[NG][P];         // per group: a, dt, d (bits), mu_d (-1: padding) of a block
  float wb[NG][16];           // per group: 1 / lambda of a reduce-scatter's events
  float gmuL[NG][P + 1];      // per group: FP32 Gmu partials (entry P: padding)
  double red[4][kBlock];      // end-of-window reductions
  double Cn[P];               // (N_n - E_n) / beta
  double Fn[P];               // F_n
  double gmu[P];              // Gmu_m - T
  double scal[4];             // ll, g_beta, |sum| helpers
  float beta;
  int next_window;
  int stop;
  __device__ float& A(int e) { return ao[e].x; }
};

// Sums B values (B = 4, 8 or 16) over each group of P lanes (P = 32 or 64)
// at once: on return every lane holds the group total of value
// (lane mod P) / (P / B).  Each halving exchange, from the group's top lane
// bit down, keeps half of the values and adds the partner lane's copy of
// them: lanes 32 apart (P = 64) and 16 apart by lane swaps, 8 apart by a DPP
// rotation of the row, then mirrored within 8; plain DPP sums over the lane
// bits left below end it.
__device__ __forceinline__ void swap_add32(float& a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a),
                                                  __builtin_bit_cast(unsigned, b), false, false);
  const unsigned x = r[0], y = r[1];  // (a bit cast of r[i] itself reads element 0)
  a = __uint_as_float(x) + __uint_as_float(y);
}
__device__ __forceinline__ void swap_add16(float& a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a),
                                                  __builtin_bit_cast(unsigned, b), false, false);
  const unsigned x = r[0], y = r[1];  // (a bit cast of r[i] itself reads element 0)
  a = __uint_as_float(x) + __uint_as_float(y);
}
// G_R row `row` += w * r for the wave's 64 x 64 register accumulator:
// lane n holds column n, rows 0..31 in v40..v71 and 32..63 in v72..v103
// (fixed registers, so that one indexed FMA reaches any row: the row is
// uniform, one event's target).  The index mode applies to the FMA's
// accumulator operand and destination only.
__device__ __forceinline__ void gr_row_fma(f32x32& lo, f32x32& hi, int row, float w, float r) {
  int m0;  // the index mode writes M0
  asm volatile(
      "s_set_gpr_idx_on %3, gpr_idx(SRC2,DST)\n\t"
      "v_fma_f32 v40, %4, %5, v40\n\t"
      "s_set_gpr_idx_off"
      : "+{v[40:71]}"(lo), "+{v[72:103]}"(hi), "={m0}"(m0)
      : "s"(row), "s"(w), "v"(r));
}
// Keeps v[e + h] where the lane bit is set (else v[e]) and adds the partner's.
template <int CTRL, int H>
__device__ __forceinline__ void dpp_halve(float* v, bool bit) {
#pragma unroll
  for (int e = 0; e < H; ++e) {
    const float keep = bit ? v[e + H] : v[e], send = bit ? v[e] : v[e + H];
    v[e] = keep + dpp<CTRL>(send);
  }
}
template <int P, int B>
__device__ __forceinline__ float group_reduce_scatter(float (&v)[B]) {
  static_assert((P == 32 || P == 64) && (B == 4 || B == 8 || B == 16) && B <= P / 4, "");
  const int lane = threadIdx.x & 63;
  constexpr int B1 = P == 64 ? B / 2 : B;  // values left after the 32-apart stage
  if constexpr (P == 64) {
#pragma unroll
    for (int e = 0; e < B1; ++e) swap_add32(v[e], v[e + B1]);  // lanes >= 32 keep e + B1
  }
  constexpr int B2 = B1 / 2;
#pragma unroll
  for (int e = 0; e < B2; ++e) swap_add16(v[e], v[e + B2]);    // odd rows keep e + B2
  constexpr int B3 = B2 / 2;
  if constexpr (B3 >= 1) dpp_halve<0x128, B3>(v, lane & 8);    // row_ror:8
  constexpr int B4 = B3 / 2;
  if constexpr (B4 >= 1) dpp_halve<0x141, B4>(v, lane & 4);    // row_half_mirror
  float z = v[0];
  if constexpr (B3 == 0) z += dpp<0x128>(z);                   // bit 3 left: row_ror:8
  if constexpr (B4 == 0) z += dpp<0x141>(z);                   // bit 2 left: row_half_mirror
  z += dpp<0xB1>(z);                                           // quad_perm [1,0,3,2]
  z += dpp<0x4E>(z);                                           // quad_perm [2,3,0,1]
  return z;
}

// Compensator sums of a slowly decaying window from its events: group g
// takes chunk g of the window P events at a time, computing -expm1(-beta tau)
// and h(beta tau) with a lane per event, then adding them event by event
// with a lane per dimension.  On return lane n < P of the first group holds
// the window's sums over source-n events in qs, hs.  Kept out of line (the
// fit kernels' registers are full).
template <int P>
__device__ __noinline__ void slow_decay_sums(SharedLds<P>& sh, const float* __restrict__ tw,
                                             const uint8_t* __restrict__ dw, int n, float beta,
                                             double& qs, double& hs) {
  constexpr int G = SharedLds<P>::G;
  const int tid = threadIdx.x;
  const int lane = tid & (P - 1);
  const int grp = tid / P;
  const int c = (n + G - 1) / G;
  const int j0 = min(grp * c, n);
  const int len = min(j0 + c, n) - j0;
  const int nsub = (c + P - 1) / P;  // uniform
  double q64 = 0.0, h64 = 0.0;
  for (int sb = 0; sb < nsub; ++sb) {
    const int j = sb * P + lane;
    const bool ok = j < len;
    const float x = ok ? beta * tw[j0 + j] : 0.f;
    const float q = comp_q(x), h = comp_h(x);
    const int d = ok ? (int)dw[j0 + j] : -1;
    float qa = 0.f, ha = 0.f;
    for (int k = 0; k < P; ++k) {
      float qk, hk;
      int dk;
      if constexpr (P == 64) {
        qk = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, q), k));
        hk = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, h), k));
        dk = __builtin_amdgcn_readlane(d, k);
      } else if constexpr (P == 32) {  // two groups per wavefront
        const bool hi = (tid & 32) != 0;
        const int qi = __builtin_bit_cast(int, q), hi_ = __builtin_bit_cast(int, h);
        qk = __builtin_bit_cast(float, hi ? __builtin_amdgcn_readlane(qi, 32 + k)
                                          : __builtin_amdgcn_readlane(qi, k));
        hk = __builtin_bit_cast(float, hi ? __builtin_amdgcn_readlane(hi_, 32 + k)
                                          : __builtin_amdgcn_readlane(hi_, k));
        dk = hi ? __builtin_amdgcn_readlane(d, 32 + k) : __builtin_amdgcn_readlane(d, k);
      } else {
        qk = __shfl(q, k, P);
        hk = __shfl(h, k, P);
        dk = __shfl(d, k, P);
      }
      qa += dk == lane ? qk : 0.f;
      ha += dk == lane ? hk : 0.f;
    }
    q64 += (double)qa;
    h64 += (double)ha;
  }
  sh.red[0][tid] = q64;
  sh.red[1][tid] = h64;
  __syncthreads();
  qs = hs = 0.0;
  if (tid < P) {
    for (int g = 0; g < G; ++g) {
      qs += sh.red[0][g * P + tid];
      hs += sh.red[1][g * P + tid];
    }
  }
  __syncthreads();  // red is reused by the caller
}

// Evaluates one window with the parameters already in LDS (alpha, mu,
// colsum, beta).  ASM_GR (P = 64, the evaluation kernel): 1 / lambda read
// from its lane as a scalar, the G_R row update as the fixed-register
// indexed FMA of gr_row_fma, and tie-free blocks without the pending-count
// select.  Without it (the fit kernels): 1 / lambda through LDS and the
// compiler's indexed access to the register rows.  Built into the fit
// kernels at their register budget (two workgroups per CU), the former gave
// wrong likelihoods from the second window a workgroup ran on (see
// tests/test_gpu_multiwindow.py), with no cause found in the generated code,
// so it stays in the evaluation kernel only, where every window is checked.
// Results: sh.scal[0] = ll, and if GRAD: gR64[k] holds
// G_R[e] for e = tid + k * kBlock (FP64), sh.Cn, sh.Fn, sh.gmu (= d ll/d mu),
// sh.scal[1] = d ll / d beta.  cnt_w: the window's events per dimension.
template <int P, bool GRAD, int SB, bool ASM_GR = false>
__device__ __forceinline__ void eval_window(SharedLds<P>& sh, const float* __restrict__ dtg,
                            const uint8_t* __restrict__ dg, const float* __restrict__ taug,
                            int64_t begin, int n, double T,
                            float end_gap, int M, const int32_t* __restrict__ cnt_w,
                            double (&gR64)[own_count(P)]) {
  constexpr int G = SharedLds<P>::G;
  constexpr int OWN = own_count(P);
  constexpr int B = kBatch < P ? kBatch : P;
  const int tid = threadIdx.x;
  const int lane = tid & (P - 1);
  const int grp = tid / P;
  float* gRc = sh.gR[SharedLds<P>::NCOPY > 1 ? (tid >> 6) : 0];
  const float beta = sh.beta;
  const float* __restrict__ dtw = dtg + begin;
  const uint8_t* __restrict__ dw = dg + begin;

  double ll64 = 0.0, gmu64 = 0.0, gb64 = 0.0;
  if constexpr (SharedLds<P>::kLaneDim) {
    // Ordered before pass 2 by the barriers below.
    for (int e = tid; e < SharedLds<P>::NG * (P + 1); e += kBlock) (&sh.gmuL[0][0])[e] = 0.f;
  }
  // Group g owns the contiguous chunk [j0, j1) of the window.
  const int c = (n + G - 1) / G;
  const int j0 = min(grp * c, n);
  const int len = min(j0 + c, n) - j0;

  // Pass 1: carry of this group's chunk from a zero start, one event per
  // lane.  An event at suffix time tau (sum of the later gaps of the chunk)
  // adds e^{-beta tau} to R and tau e^{-beta tau} to S of its dimension, or
  // counts as pending if no positive gap follows it (tau == 0); the chunk
  // decays everything before it by e^{-beta delta}, delta = sum of its gaps.
  {
    sh.cR[grp][lane] = 0.f;
    sh.cS[grp][lane] = 0.f;
    sh.cP[grp][lane] = 0.f;
    float later = 0.f;
    const int nsub = (c + P - 1) / P;
    // Lanes run backwards through a sub-batch.  An empty window has no
    // sub-batch (nsub = 0) and jr < 0: nothing may be read there, the window
    // may start at the first event of the plan's arrays.
    int jr = (nsub - 1) * P + (P - 1 - lane);
    float dt_n = (jr >= 0 && jr < len) ? dtw[j0 + jr] : 0.f;
    int d_n = (jr >= 0 && jr < len) ? (int)dw[j0 + jr] : 0;
    for (int bb = nsub - 1; bb >= 0; --bb) {
      const bool valid = jr < len;
      const float dt = dt_n;
      const int d = d_n;
      jr -= P;
      if (bb > 0) {  // prefetch the previous sub-batch
        dt_n = jr < len ? dtw[j0 + jr] : 0.f;
        d_n = jr < len ? (int)dw[j0 + jr] : 0;
      }
      // Gap of the next event (the exclusive scan's input).
      float prev = P <= 16 ? row_shr<1>(dt) : wave_shr1(dt);  // lane 0 of each group: below
      prev = lane == 0 ? 0.f : prev;
      const float tau = later + group_scan<P>(prev, lane);
      if (valid) {
        if (tau > 0.f) {
          const float e = __expf(-beta * tau);
          atomicAdd(&sh.cR[grp][d], e);
          atomicAdd(&sh.cS[grp][d], tau * e);
        } else {
          atomicAdd(&sh.cP[grp][d], 1.f);
        }
      }
      later += group_sum<P>(dt);
    }
    if (lane == 0) {
      sh.cA[grp] = __expf(-beta * later);
      sh.cD[grp] = later;
      sh.cF[grp] = later > 0.f ? 1 : 0;
    }
  }
  __syncthreads();
  // Ordered combine of the chunk carries: chunk g starts from the state
  // after chunks 0..g-1; the final state is the window's end state.
  if (grp == 0) {
    float R = 0.f, S = 0.f, Pn = 0.f;
    for (int g = 0; g < G; ++g) {
      const float Rg = sh.cR[g][lane], Sg = sh.cS[g][lane], Pg = sh.cP[g][lane];
      const float Ag = sh.cA[g], Dg = sh.cD[g];
      const int Fg = sh.cF[g];
      sh.cR[g][lane] = R;
      sh.cS[g][lane] = S;
      sh.cP[g][lane] = Pn;
      if (Fg) {
        const float X = R + Pn;
        R = fmaf(Ag, X, Rg);
        S = fmaf(Ag, fmaf(Dg, X, S), Sg);
        Pn = Pg;
      } else {
        Pn += Pg;
      }
    }
    sh.tR[lane] = R;
    sh.tS[lane] = S;
    sh.tP[lane] = Pn;
  }
  __syncthreads();
  // Pass 2: exact states, intensities and gradient sums.  With P = 64 each
  // wave keeps its chunk's G_R in registers (lane n: column n, rows 0..31 in
  // gacc0 and 32..63 in gacc1, indexed by the event's uniform target).
  constexpr bool kRegGR = GRAD && P == 64;
  f32x32 gacc0, gacc1;
  if constexpr (SharedLds<P>::kLaneDim) {
    // P events per block: lane j of the group stages event j (decay, gap,
    // dimension, mu of its target; padding events have dimension P, whose
    // alpha and one-hot rows are zero, and mu -1).  Then B events at a time:
    // the recursion with broadcast reads of the staged values, one
    // reduce-scatter for their intensities, log and reciprocal there, and
    // the G_R row adds.
    // SB = kScatterMfma: 16-event blocks whose intensity sums come from the
    // matrix cores (P = 64 only).
    constexpr bool kMfma = SB == kScatterMfma;
    static_assert(!kMfma || P == 64, "the matrix-core intensity tile is built for 64 lanes");
    constexpr int B = kMfma ? 16 : SB;
    constexpr int SH = P == 64 ? (B == 16 ? 2 : B == 8 ? 3 : 4) : (B == 16 ? 1 : B == 8 ? 2 : 3);
    const int ev_l = lane >> SH;                 // the event whose intensity this lane gets
    const bool lead = (lane & ((1 << SH) - 1)) == 0;
    float4* meta = sh.meta[SharedLds<P>::NG > 1 ? grp : 0];
    float* wb = sh.wb[SharedLds<P>::NG > 1 ? grp : 0];
    float* gmuL = sh.gmuL[SharedLds<P>::NG > 1 ? grp : 0];
    float R = sh.cR[grp][lane], S = sh.cS[grp][lane];
    float Rin = R + sh.cP[grp][lane];  // R plus the events pending at the current time
    float llp = 0.f, gbp = 0.f;
    for (int m = 0; m < 32; ++m) gacc0[m] = gacc1[m] = 0.f;
    const int nblk = (len + P - 1) / P;
    int jl = lane;
    float dt_n = jl < len ? dtw[j0 + jl] : 0.f;
    int d_n = jl < len ? (int)dw[j0 + jl] : P;
    for (int blk = 0; blk < nblk; ++blk) {
      const float dt_l = dt_n;
      const int d_l = d_n;
      jl += P;
      if (blk + 1 < nblk) {  // prefetch the next block
        dt_n = jl < len ? dtw[j0 + jl] : 0.f;
        d_n = jl < len ? (int)dw[j0 + jl] : P;
      }
      wave_sync();  // the previous block's reads are done
      meta[lane] = make_float4(__expf(-beta * dt_l), dt_l, __builtin_bit_cast(float, d_l),
                               d_l < P ? sh.mu[d_l] : -1.f);
      // A block without equal times (the usual case for continuous times)
      // needs no pending-count select: R(j) is the decayed inclusive state.
      const bool tie_free = __builtin_amdgcn_ballot_w64(d_l < P && !(dt_l > 0.f)) == 0;
      wave_sync();
#pragma unroll 1
      for (int sb = 0; sb < P; sb += B) {
        float L[B], AS[B], Rj[B];
        int Dj[B];
        auto recur = [&](auto tf) {
          constexpr bool kTieFree = decltype(tf)::value;
          static_for<B>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const float4 m = meta[sb + j];
            const float a = m.x, dt = m.y;
            const int d = __builtin_bit_cast(int, m.z);
            const float x = a * Rin;  // decayed over the gap; R moves only when time does
            S = fmaf(a, S, dt * x);
            if constexpr (kTieFree) R = x;
            else R = dt > 0.f ? x : R;
            const float2 ao = sh.ao[d * P + lane];
            L[j] = ao.x * R;
            AS[j] = ao.x * S;
            Rj[j] = R;
            Dj[j] = d;
            Rin = x + ao.y;  // the event itself is pending until time moves on
          });
        };
        if (ASM_GR && tie_free) recur(std::true_type{});
        else recur(std::false_type{});
        float lam;
        if constexpr (kMfma) {
          // Lam[j][m] = sum_n R_n(j) alpha_mn for the block's 16 events and
          // all 64 targets (one column per event is used): R staged in the
          // wave's part of the G_R transfer buffer (free until the end of
          // the window; rows padded to 65 floats), 16 steps of 4 sources x
          // 4 tiles of 16 targets on v_mfma_f32_16x16x4_f32 (A: event
          // lane % 16, source lane / 16; B: source lane / 16, target
          // lane % 16; D: lane holds events 4 (lane / 16) + r, target
          // lane % 16), then each event's own target read back.
          constexpr int RS = P + 1;
          float* Rt = sh.gR[0] + (tid >> 6) * (16 * RS);
          static_for<B>([&](auto J) {
            constexpr int j = decltype(J)::value;
            Rt[j * RS + lane] = Rj[j];
          });
          wave_sync();
          const int i16 = lane & 15, k4 = lane >> 4;
          f32x4 acc[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s4 = 0; s4 < P / 4; ++s4) {
            const float a = Rt[i16 * RS + 4 * s4 + k4];
#pragma unroll
            for (int q = 0; q < 4; ++q)
              acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                  a, sh.ao[(16 * q + i16) * P + 4 * s4 + k4].x, acc[q], 0, 0, 0);
          }
          wave_sync();  // every lane has read its A operands
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) Rt[(4 * k4 + r) * RS + 16 * q + i16] = acc[q][r];
          wave_sync();
          const int dj = __builtin_bit_cast(int, meta[sb + ev_l].z);
          lam = dj < P ? Rt[ev_l * RS + dj] : 0.f;
          wave_sync();  // read before the next block's R overwrites the tile
        } else {
          lam = group_reduce_scatter<P, B>(L);
        }
        const float4 me = meta[sb + ev_l];
        const bool valid = me.w >= 0.f;
        lam += me.w;
        llp += (lead && valid) ? __logf(lam) : 0.f;
        if constexpr (kRegGR && ASM_GR) {
          // 1 / lambda of event j is in lane j << SH; read as a scalar, it
          // scales R(j) into row d_j of the wave's G_R registers (one
          // indexed FMA) and S into the decay gradient.
          const float w = valid ? __builtin_amdgcn_rcpf(lam) : 0.f;
          if (lead && valid) atomicAdd(&gmuL[__builtin_bit_cast(int, me.z)], w);
          static_for<B>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const float wj = __builtin_bit_cast(
                float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, w), j << SH));
            const int dj = __builtin_amdgcn_readfirstlane(Dj[j]) & (P - 1);
            gr_row_fma(gacc0, gacc1, dj, wj, Rj[j]);
            gbp = fmaf(wj, AS[j], gbp);
          });
        } else if constexpr (GRAD) {
          const float w = valid ? __builtin_amdgcn_rcpf(lam) : 0.f;
          if (lead) {
            wb[ev_l] = w;
            if (valid) atomicAdd(&gmuL[__builtin_bit_cast(int, me.z)], w);
          }
          wave_sync();
          float wv[B];
#pragma unroll
          for (int q = 0; q < B / 4; ++q) {
            const float4 w4 = reinterpret_cast<const float4*>(wb)[q];
            wv[4 * q] = w4.x;
            wv[4 * q + 1] = w4.y;
            wv[4 * q + 2] = w4.z;
            wv[4 * q + 3] = w4.w;
          }
#pragma unroll
          for (int j = 0; j < B; ++j) {
            const float x = wv[j] * Rj[j];
            if constexpr (kRegGR) {
              // Row d of the wave's G_R registers (d is uniform: one event).
              const int d = __builtin_amdgcn_readfirstlane(Dj[j]);
              const int dl = d & 31;
              const bool hi = d >= 32;
              gacc0[dl] += hi ? 0.f : x;
              gacc1[dl] += hi ? x : 0.f;
            } else {
              atomicAdd(&gRc[Dj[j] * P + lane], x);
            }
            gbp = fmaf(wv[j], AS[j], gbp);
          }
          wave_sync();  // wb is rewritten by the next events
        }
      }
    }
    ll64 += (double)llp;
    gb64 += (double)gbp;
  } else {
    // B events per batch: the recurrence runs over the batch with the gaps,
    // decays and dims broadcast from the lane that loaded them, the B intensity sums are
    // independent group reductions, and lane j takes log and reciprocal of
    // lambda_j for the whole group.
    {
      float R = sh.cR[grp][lane], S = sh.cS[grp][lane], Pn = sh.cP[grp][lane];
      float llp = 0.f, gmup = 0.f, gbp = 0.f;
      const int nb = (c + B - 1) / B;
      int jl = lane & (B - 1);
      float dt_n = jl < len ? dtw[j0 + jl] : 0.f;
      int d_n = jl < len ? (int)dw[j0 + jl] : 0;
      for (int bb = 0; bb < nb; ++bb) {
        const bool vl = jl < len;
        const float dt_l = dt_n;
        const float d_l = __builtin_bit_cast(float, d_n);
        const int nvalid = min(B, len - bb * B);  // valid events of this batch (may be <= 0)
        jl += B;
        if (bb + 1 < nb) {  // prefetch the next batch
          dt_n = jl < len ? dtw[j0 + jl] : 0.f;
          d_n = jl < len ? (int)dw[j0 + jl] : 0;
        }
        const float a_l = __expf(-beta * dt_l);
        float Rj[B], ASj[B], Lj[B];  // R(j), alpha_{d_j n} S_n(j), alpha_{d_j n} R_n(j)
        int Dj[B];
        static_for<B>([&](auto J) {
          constexpr int j = decltype(J)::value;
          const float dt = group_bcast<P, j>(dt_l);
          const float a = group_bcast<P, j>(a_l);
          const int d = __builtin_bit_cast(int, group_bcast<P, j>(d_l));
          const bool f = dt > 0.f;
          const float X = f ? R + Pn : R;
          R = a * X;
          S = fmaf(a, S, dt * R);
          Pn = f ? 0.f : Pn;
          const float al = sh.A(d * P + lane);
          Rj[j] = R;
          ASj[j] = al * S;
          Dj[j] = d;
          Lj[j] = al * R;
          Pn += (j < nvalid && d == lane) ? 1.f : 0.f;
        });
        static_for<B>([&](auto J) {
          constexpr int j = decltype(J)::value;
          Lj[j] = group_sum<P>(Lj[j]);
        });
        float lk = Lj[0];
        static_for<B>([&](auto J) {
          constexpr int j = decltype(J)::value;
          if (j > 0) lk = (lane & (B - 1)) == j ? Lj[j] : lk;
        });
        lk += sh.mu[__builtin_bit_cast(int, d_l)];
        const float lg = __logf(lk);
        llp += (vl && lane < B) ? lg : 0.f;
        if constexpr (GRAD) {
          const float wk = vl ? __builtin_amdgcn_rcpf(lk) : 0.f;
          static_for<B>([&](auto J) {
            constexpr int j = decltype(J)::value;
            const float w = group_bcast<P, j>(wk);  // zero for events past the chunk end
            atomicAdd(&gRc[Dj[j] * P + lane], w * Rj[j]);
            gbp = fmaf(w, ASj[j], gbp);
            gmup += Dj[j] == lane ? w : 0.f;
          });
        }
      }
      ll64 += (double)llp;
      gmu64 += (double)gmup;
      gb64 += (double)gbp;
    }
  }
#pragma unroll
  for (int k = 0; k < OWN; ++k) gR64[k] = 0.0;
  if constexpr (kRegGR) {
    // The waves' register G_R, one wave at a time through LDS.
#pragma unroll 1
    for (int r = 0; r < kBlock / 64; ++r) {
      __syncthreads();
      if ((tid >> 6) == r) {
#pragma unroll
        for (int m = 0; m < 32; ++m) {
          sh.gR[0][m * P + lane] = gacc0[m];
          sh.gR[0][(m + 32) * P + lane] = gacc1[m];
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < OWN; ++k) gR64[k] += (double)sh.gR[0][tid + k * kBlock];
    }
  } else if constexpr (GRAD) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
      const int e = tid + k * kBlock;
      if (e < P * P) {
        float sum = 0.f;
#pragma unroll
        for (int cpy = 0; cpy < SharedLds<P>::NCOPY; ++cpy) {
          sum += sh.gR[cpy][e];
          sh.gR[cpy][e] = 0.f;
        }
        gR64[k] = (double)sum;
      }
    }
  }

  // End of window: reduce the per-lane partials over groups (lane n of
  // wave 0 takes component n), then the window sums over the wave.  A
  // slowly decaying window takes its compensator sums from the events.
  const bool slow = (double)beta * T < kSlowDecayDim;  // uniform
  double qs = 0.0, hs = 0.0;
  __syncthreads();
  if (slow) slow_decay_sums<P>(sh, taug + begin, dw, n, beta, qs, hs);
  sh.red[0][tid] = ll64;
  sh.red[1][tid] = gmu64;
  sh.red[2][tid] = gb64;
  __syncthreads();
  if (tid < 64) {
    double p1 = 0.0, smu = 0.0, p3 = 0.0, gbeta = 0.0;
    if (tid < P) {
      double l = 0.0, gm = 0.0, gb = 0.0;
#pragma unroll 1
      for (int g = 0; g < G; ++g) {
        l += sh.red[0][g * P + tid];
        gm += sh.red[1][g * P + tid];
        gb += sh.red[2][g * P + tid];
      }
      if constexpr (SharedLds<P>::kLaneDim) {
        gm = 0.0;
#pragma unroll 1
        for (int g = 0; g < SharedLds<P>::NG; ++g) gm += (double)sh.gmuL[g][tid];
      }
      const bool in = tid < M;
      const double nn = in ? (double)cnt_w[tid] : 0.0;
      // Advance the end state to T: E_n and F_n of the compensator.
      const double gap = (double)end_gap;
      const double b = (double)beta;
      const double a = exp(-b * gap);
      const double E = a * ((double)sh.tR[tid] + (double)sh.tP[tid]);
      const double F = a * (double)sh.tS[tid] + gap * E;
      const double C = slow ? qs / b : (nn - E) / b;
      const double FmC = slow ? hs / b : F - C;  // F_n - C_n
      sh.Cn[tid] = in ? C : 0.0;
      sh.Fn[tid] = in ? C + FmC : 0.0;
      sh.gmu[tid] = in ? gm - T : 0.0;
      p1 = l;                                                     // Part1
      smu = in ? (double)sh.mu[tid] : 0.0;                        // sum mu
      p3 = in ? (double)sh.colsum[tid] * C : 0.0;                 // Part3 (sign below)
      gbeta = in ? gb + (double)sh.colsum[tid] * FmC / b : 0.0;  // -d ll / d beta
    }
    p1 = wave_sum(p1);
    smu = wave_sum(smu);
    p3 = wave_sum(p3);
    gbeta = wave_sum(gbeta);
    if (tid == 0) {
      sh.scal[0] = p1 - T * smu - p3;
      sh.scal[1] = -gbeta;
    }
  }
  __syncthreads();
}

template <int P>
__device__ void load_params(SharedLds<P>& sh, const float* __restrict__ mu,
                            const float* __restrict__ alpha, const float* __restrict__ beta,
                            int64_t w, int M) {
  const int tid = threadIdx.x;
  for (int e = tid; e < P * P; e += kBlock) {
    const int m = e / P, n = e % P;
    sh.A(e) = (m < M && n < M) ? alpha[(w * M + m) * M + n] : 0.f;
  }
  if (tid < P) sh.mu[tid] = tid < M ? mu[w * M + tid] : 0.f;
  if (tid == 0) sh.beta = beta[w];
  __syncthreads();
  if (tid < P) {
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += sh.A(m * P + tid);
    sh.colsum[tid] = s;
  }
  __syncthreads();
}

// LDS is not initialised at launch: the G_R tile accumulators must start at
// zero (eval_window leaves them zero after every tile), the one-hot column
// of ao is the identity and ao's padding row P is zero.
template <int P>
__device__ void init_lds(SharedLds<P>& sh) {
  constexpr int AR = SharedLds<P>::AR;
  for (int e = threadIdx.x; e < SharedLds<P>::NCOPY * AR * P; e += kBlock) (&sh.gR[0][0])[e] = 0.f;
  for (int e = threadIdx.x; e < AR * P; e += kBlock) {
    const int m = e / P, n = e % P;
    sh.ao[e] = make_float2(0.f, m == n ? 1.f : 0.f);
  }
}

template <int P>
__device__ int next_window(SharedLds<P>& sh, int* counter, int first) {
  __syncthreads();
  if (threadIdx.x == 0) sh.next_window = first ? (int)blockIdx.x : atomicAdd(counter, 1) + (int)gridDim.x;
  __syncthreads();
  return sh.next_window;
}

template <int P, bool GRAD, int SB>
__global__ __launch_bounds__(kBlock, (P >= 32 ? 2 : kMinBlocks)) void shared_eval_kernel(Events ev, int M, const float* mu,
                                                             const float* alpha,
                                                             const float* beta, double* ll,
                                                             float* g_mu, float* g_alpha,
                                                             float* g_beta, int* counter) {
  __shared__ SharedLds<P> sh;
  constexpr int OWN = own_count(P);
  double gR64[OWN];
  const int tid = threadIdx.x;
  init_lds(sh);
  for (int q = next_window(sh, counter, 1); q < ev.W; q = next_window(sh, counter, 0)) {
    const int64_t w = ev.order[q];
    load_params(sh, mu, alpha, beta, w, M);
    const double T = ev.T[w];
    eval_window<P, GRAD, SB, true>(sh, ev.dt, ev.d, ev.tau, ev.begin[w], ev.n[w], T,
                                   ev.end_gap[w], M, ev.counts + w * M, gR64);
    if (tid == 0) ll[w] = sh.scal[0];
    if constexpr (GRAD) {
      if (tid == 0) g_beta[w] = (float)sh.scal[1];
      if (tid < M) g_mu[w * M + tid] = (float)sh.gmu[tid];
#pragma unroll
      for (int k = 0; k < OWN; ++k) {
        const int e = tid + k * kBlock;
        const int m = e / P, n = e % P;
        if (e < P * P && m < M && n < M)
          g_alpha[(w * M + m) * M + n] = (float)(gR64[k] - sh.Cn[n]);
      }
    }
  }
}

// Persistent projected-gradient fit (see mdhp_fit_opts for the rule).
template <int P, int SB>
__global__ __launch_bounds__(kBlock, (P >= 32 ? 2 : kMinBlocks)) void shared_fit_kernel(Events ev, int M, FitParams o,
                                                            float* mu, float* alpha, float* beta,
                                                            double* ll, int* steps, int* status,
                                                            int* evals_out, int* counter) {
  __shared__ SharedLds<P> sh;
  constexpr int OWN = own_count(P);
  double gR64[OWN];
  float m1a[OWN], m2a[OWN];
  const int tid = threadIdx.x;
  init_lds(sh);
  for (int q = next_window(sh, counter, 1); q < ev.W; q = next_window(sh, counter, 0)) {
    const int64_t w = ev.order[q];
    load_params(sh, mu, alpha, beta, w, M);
    const int n = ev.n[w];
    const double T = ev.T[w];
    const double rate = (double)max(n, 1) / T;
    const double mu_min = o.mu_floor_rel * rate;
    const double beta_min = o.beta_floor_rel * rate;
    const double inv_n = 1.0 / (double)max(n, 1);
#pragma unroll
    for (int k = 0; k < OWN; ++k) m1a[k] = m2a[k] = 0.f;
    float m1mu = 0.f, m2mu = 0.f, m1b = 0.f, m2b = 0.f;
    double ll_prev = 0.0, b1t = 1.0, b2t = 1.0;
    int s = 0, st = MDHP_FIT_MAX_STEPS;
    for (s = 0;; ++s) {
      eval_window<P, true, SB>(sh, ev.dt, ev.d, ev.tau, ev.begin[w], n, T, ev.end_gap[w], M, ev.counts + w * M, gR64);
      const double l = sh.scal[0];
      // Finiteness of ll and of the whole gradient (one flag per block).
      if (tid == 0) sh.stop = isfinite(l) && isfinite(sh.scal[1]) ? 0 : 1;
      __syncthreads();
      bool bad = false;
#pragma unroll
      for (int k = 0; k < OWN; ++k) {
        const int e = tid + k * kBlock;
        if (e < P * P && !isfinite(gR64[k])) bad = true;
      }
      if (tid < P && !isfinite(sh.gmu[tid])) bad = true;
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
      if (o.optimizer == MDHP_OPT_EM) {
        // Expected background and offspring counts over their exposures
        // (the decay is fixed).
#pragma unroll
        for (int k = 0; k < OWN; ++k) {
          const int e = tid + k * kBlock;
          const int m = e / P, nn = e % P;
          const double C = sh.Cn[nn];
          if (e < P * P && m < M && nn < M && C > 0.0)
            sh.A(e) = (float)((double)sh.A(e) * (gR64[k] / C));
        }
        if (tid < M)
          sh.mu[tid] = (float)fmax((double)sh.mu[tid] * ((sh.gmu[tid] + T) / T), mu_min);
      } else {
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
#pragma unroll
        for (int k = 0; k < OWN; ++k) {
          const int e = tid + k * kBlock;
          const int m = e / P, nn = e % P;
          if (e < P * P && m < M && nn < M) {
            const double g = gR64[k] - sh.Cn[nn];
            const double v = (double)sh.A(e) + step(g, m1a[k], m2a[k]);
            sh.A(e) = (float)fmax(v, 0.0);
          }
        }
        if (tid < M) {
          const double v = (double)sh.mu[tid] + step(sh.gmu[tid], m1mu, m2mu);
          sh.mu[tid] = (float)fmax(v, mu_min);
        }
        if (tid == 0 && !o.fix_beta) {
          const double v = (double)sh.beta + step(sh.scal[1], m1b, m2b);
          sh.beta = (float)fmax(v, beta_min);
        }
      }
      __syncthreads();
      if (tid < P) {
        float cs = 0.f;
        for (int m = 0; m < M; ++m) cs += sh.A(m * P + tid);
        sh.colsum[tid] = cs;
      }
      __syncthreads();
    }
    // theta_s of the last evaluation is in LDS.
    for (int e = tid; e < M * M; e += kBlock) alpha[w * M * M + e] = sh.A((e / M) * P + e % M);
    if (tid < M) mu[w * M + tid] = sh.mu[tid];
    if (tid == 0) {
      beta[w] = sh.beta;
      ll[w] = sh.scal[0];
      steps[w] = s;
      status[w] = st;
      if (evals_out) evals_out[w] = s + 1;
    }
  }
}

// Block-wide sums of NV doubles (every thread gets the sums).
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double* scratch) {
#pragma unroll
  for (int j = 0; j < NV; ++j)
#pragma unroll
    for (int k = 32; k > 0; k >>= 1) v[j] += __shfl_xor(v[j], k, 64);
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) scratch[j * 4 + wave] = v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NV; ++j)
    v[j] = scratch[j * 4 + 0] + scratch[j * 4 + 1] + scratch[j * 4 + 2] + scratch[j * 4 + 3];
}

__device__ __forceinline__ double block_max_abs(double v, double* scratch) {
  v = fabs(v);
#pragma unroll
  for (int k = 32; k > 0; k >>= 1) v = fmax(v, __shfl_xor(v, k, 64));
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) scratch[wave] = v;
  __syncthreads();
  return fmax(fmax(scratch[0], scratch[1]), fmax(scratch[2], scratch[3]));
}

// Projected L-BFGS fit (the update rule is described with the options in
// the public header).  Thread tid owns parameter slots k < OWN: alpha
// entry e = tid + k * kBlock (row e / P, column e % P), and slot OWN: mu_tid
// (tid < M) or beta (tid == M).  Between evaluations its slices of x, g and
// of the direction are in registers; x, g and d go to the workspace before
// the line search (whose evaluations need every register) and are read back
// by each trial and by the update; the history pairs live there.  The scalars of the two-loop
// recursion come from block reductions.
template <int P, int SB>
__global__ __launch_bounds__(kBlock, (P >= 32 ? 2 : kMinBlocks)) void shared_lbfgs_kernel(Events ev, int M, FitParams o,
                                                              float* mu, float* alpha,
                                                              float* beta, double* ll,
                                                              int* steps, int* status,
                                                              int* evals_out, float* ws,
                                                              int* counter) {
  __shared__ SharedLds<P> sh;
  __shared__ double scratch[16];
  __shared__ double a_s[kMaxHistory], rho_s[kMaxHistory];
  __shared__ int flag;
  constexpr int OWN = own_count(P);
  constexpr int K = OWN + 1;
  constexpr int VX = 0, VG = 1, VD = 2;
  double gR64[OWN];
  const int tid = threadIdx.x;
  const int m_hist = o.history;
  const LbfgsWs<K, kBlock> wsp(ws + (size_t)blockIdx.x * ((size_t)kLbfgsVectors * K * kBlock),
                               tid);
  auto VS = [](int j) { return LbfgsWs<K, kBlock>::S(j); };
  auto VY = [](int j) { return LbfgsWs<K, kBlock>::Y(j); };
  init_lds(sh);
  for (int q = next_window(sh, counter, 1); q < ev.W; q = next_window(sh, counter, 0)) {
    const int64_t w = ev.order[q];
    load_params(sh, mu, alpha, beta, w, M);
    const int n = ev.n[w];
    const double T = ev.T[w];
    const double rate = (double)max(n, 1) / T;
    const float mu_min = (float)(o.mu_floor_rel * rate);
    const float beta_min = (float)(o.beta_floor_rel * rate);
    const double inv_n = 1.0 / (double)max(n, 1);
    // Slot kinds: 0 none, 1 alpha, 2 mu, 3 beta (frozen when fix_beta).
    auto kind = [&](int k) -> int {
      if (k < OWN) {
        const int e = tid + k * kBlock;
        return (e < P * P && e / P < M && e % P < M) ? 1 : 0;
      }
      if (tid < M) return 2;
      if (tid == M) return o.fix_beta ? 0 : 3;
      return 0;
    };
    auto lower = [&](int k) -> float {
      const int kd = kind(k);
      return kd == 2 ? mu_min : (kd == 3 ? beta_min : 0.f);
    };
    // Current parameter of slot k (zero for slots that hold none).
    auto get_param = [&](int k) -> float {
      const int kd = kind(k);
      if (kd == 1) return sh.A(tid + k * kBlock);
      if (kd == 2) return sh.mu[tid];
      if (kd == 3) return sh.beta;
      return 0.f;
    };
    auto set_param = [&](int k, float v) {
      const int kd = kind(k);
      if (kd == 1) sh.A(tid + k * kBlock) = v;
      else if (kd == 2) sh.mu[tid] = v;
      else if (kd == 3) sh.beta = v;
    };
    // Gradient of f = -ll / N for slot k after eval_window.
    auto grad_f = [&](int k) -> double {
      const int kd = kind(k);
      if (kd == 1) return -(gR64[k] - sh.Cn[(tid + k * kBlock) % P]) * inv_n;
      if (kd == 2) return -sh.gmu[tid] * inv_n;
      if (kd == 3) return -sh.scal[1] * inv_n;
      return 0.0;
    };
    auto refresh_colsum = [&]() {
      __syncthreads();
      if (tid < P) {
        float cs = 0.f;
        for (int m = 0; m < M; ++m) cs += sh.A(m * P + tid);
        sh.colsum[tid] = cs;
      }
      __syncthreads();
    };
    // Evaluates at the LDS parameters; true if ll and the gradient are finite.
    auto evaluate = [&]() -> bool {
      eval_window<P, true, SB>(sh, ev.dt, ev.d, ev.tau, ev.begin[w], n, T, ev.end_gap[w], M, ev.counts + w * M, gR64);
      if (tid == 0) flag = isfinite(sh.scal[0]) && isfinite(sh.scal[1]) ? 0 : 1;
      __syncthreads();
      bool bad = false;
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (!isfinite(grad_f(k))) bad = true;
      if (bad) atomicOr(&flag, 1);
      __syncthreads();
      return flag == 0;
    };
    int nev = 1, st = MDHP_FIT_MAX_STEPS, s = 0, h = 0, head = 0;
    double l = 0.0, sy_new = 0.0, yy_new = 0.0;
    if (!evaluate()) {
      st = MDHP_FIT_NONFINITE;
      l = sh.scal[0];
    } else {
      l = sh.scal[0];
#pragma unroll
      for (int k = 0; k < K; ++k) wsp.st(VG, k, (float)grad_f(k));
      double f = -l * inv_n;
      for (s = 0;; ++s) {
        if (s == o.max_steps) {
          st = MDHP_FIT_MAX_STEPS;
          break;
        }
        // Current point and active set: a slot is held when it holds no
        // parameter or sits at its bound with the gradient pushing out.
        float xk[K], gk[K];
        unsigned act = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          xk[k] = get_param(k);
          gk[k] = wsp.ld(VG, k);
          if (kind(k) == 0 || (xk[k] <= lower(k) && gk[k] > 0.f)) act |= 1u << k;
        }
        // Free gradient and its largest entry.
        double qv[K], gmax_local = 0.0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          qv[k] = (act >> k) & 1 ? 0.0 : (double)gk[k];
          gmax_local = fmax(gmax_local, fabs(qv[k]));
        }
        const double gmax = block_max_abs(gmax_local, scratch);
        if (gmax == 0.0) {
          st = MDHP_FIT_CONVERGED;
          break;
        }
        const double gamma0 = 0.01 / gmax;
        for (int i = 0; i < h; ++i) {
          const int j = (head - 1 - i + m_hist) % m_hist;
          float sj[K], yj[K];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            sj[k] = wsp.ld(VS(j), k);
            yj[k] = wsp.ld(VY(j), k);
          }
          double v[1] = {0.0};
#pragma unroll
          for (int k = 0; k < K; ++k) v[0] += (double)sj[k] * qv[k];
          block_sums<1>(v, scratch);
          const double a = rho_s[j] * v[0];
          if (tid == 0) a_s[j] = a;
#pragma unroll
          for (int k = 0; k < K; ++k) qv[k] -= a * (double)yj[k];
        }
        const double gamma = h > 0 ? sy_new / yy_new : gamma0;
#pragma unroll
        for (int k = 0; k < K; ++k) qv[k] *= gamma;
        for (int i = h - 1; i >= 0; --i) {
          const int j = (head - 1 - i + m_hist) % m_hist;
          float sj[K], yj[K];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            yj[k] = wsp.ld(VY(j), k);
            sj[k] = wsp.ld(VS(j), k);
          }
          double v[1] = {0.0};
#pragma unroll
          for (int k = 0; k < K; ++k) v[0] += (double)yj[k] * qv[k];
          block_sums<1>(v, scratch);
          const double b = rho_s[j] * v[0];
          const double a = a_s[j];
#pragma unroll
          for (int k = 0; k < K; ++k) qv[k] += (a - b) * (double)sj[k];
        }
        float dk[K];
        double dg[1] = {0.0};
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const double dd = (act >> k) & 1 ? 0.0 : -qv[k];
          dk[k] = (float)dd;
          dg[0] += dd * (double)gk[k];
        }
        block_sums<1>(dg, scratch);
        if (!(dg[0] < 0.0)) {  // restart from scaled steepest descent
          h = 0;
#pragma unroll
          for (int k = 0; k < K; ++k)
            dk[k] = (act >> k) & 1 ? 0.f : (float)(-gamma0 * (double)gk[k]);
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
          wsp.st(VX, k, xk[k]);
          wsp.st(VD, k, dk[k]);
        }
        // Backtracking line search on the projected path.  Every trial reads
        // x, g and d back from the workspace, so that none of them is held in
        // registers across an evaluation.
        double t = 1.0, ln = 0.0, fn = 0.0;
        bool ok = false;
        for (int ls = 0; ls < 20 && !ok; ++ls, t *= 0.5) {
          double dec[1] = {0.0};
#pragma unroll
          for (int k = 0; k < K; ++k) {
            if (kind(k) == 0) continue;
            const float x0 = wsp.ld(VX, k);
            const float xn = fmaxf((float)((double)x0 + t * (double)wsp.ld(VD, k)), lower(k));
            set_param(k, xn);
            dec[0] += (double)wsp.ld(VG, k) * ((double)xn - (double)x0);
          }
          block_sums<1>(dec, scratch);
          refresh_colsum();
          const bool fin = evaluate();
          ++nev;
          ln = sh.scal[0];
          fn = -ln * inv_n;
          ok = fin && fn <= f + 1e-4 * dec[0];
        }
        if (!ok) {
          st = MDHP_FIT_STALLED;
#pragma unroll
          for (int k = 0; k < K; ++k) set_param(k, wsp.ld(VX, k));
          __syncthreads();
          break;
        }
        // New pair s = x' - x, y = g' - g; x' is the accepted point in LDS.
        double sums[3] = {0.0, 0.0, 0.0};  // s.y, s.s, y.y
        float sk[K], yk[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const float gn = (float)grad_f(k);
          const float x0 = wsp.ld(VX, k);
          const float xn = kind(k) == 0 ? x0 : get_param(k);
          sk[k] = xn - x0;
          yk[k] = gn - wsp.ld(VG, k);
          wsp.st(VG, k, gn);  // g' replaces g (read by the next iteration)
          sums[0] += (double)sk[k] * (double)yk[k];
          sums[1] += (double)sk[k] * (double)sk[k];
          sums[2] += (double)yk[k] * (double)yk[k];
        }
        block_sums<3>(sums, scratch);
        if (sums[0] > 1e-10 * sqrt(sums[1] * sums[2])) {
          if (h == m_hist) h -= 1;  // the oldest pair drops out of the ring
#pragma unroll
          for (int k = 0; k < K; ++k) {
            wsp.st(VS(head), k, sk[k]);
            wsp.st(VY(head), k, yk[k]);
          }
          if (tid == 0) rho_s[head] = 1.0 / sums[0];
          sy_new = sums[0];
          yy_new = sums[2];
          head = (head + 1) % m_hist;
          h += 1;
          __syncthreads();
        }
        const double l_prev = l;
        l = ln;
        f = fn;
        if (fabs(l - l_prev) <= o.ll_tol * fmax(fabs(l), (double)max(n, 1))) {
          st = MDHP_FIT_CONVERGED;
          s += 1;
          break;
        }
      }
    }
    __syncthreads();
    for (int e = tid; e < M * M; e += kBlock) alpha[w * M * M + e] = sh.A((e / M) * P + e % M);
    if (tid < M) mu[w * M + tid] = sh.mu[tid];
    if (tid == 0) {
      beta[w] = sh.beta;
      ll[w] = l;
      steps[w] = s;
      status[w] = st;
      if (evals_out) evals_out[w] = nev;
    }
  }
}

template <int P, int SB>
hipError_t launch_shared_eval(const Events& ev, int M, const float* mu, const float* alpha,
                              const float* beta, double* ll, float* g_mu, float* g_alpha,
                              float* g_beta, int* counter, hipStream_t s, bool grad) {
  if (ev.W == 0) return hipSuccess;
  reset_counter(counter, s);
  if (grad) {
    auto k = shared_eval_kernel<P, true, SB>;
    hipLaunchKernelGGL(k, dim3(occupancy_grid(k, kBlock, ev.W)), dim3(kBlock), 0, s, ev, M, mu, alpha,
                       beta, ll, g_mu, g_alpha, g_beta, counter);
  } else {
    auto k = shared_eval_kernel<P, false, SB>;
    hipLaunchKernelGGL(k, dim3(occupancy_grid(k, kBlock, ev.W)), dim3(kBlock), 0, s, ev, M, mu, alpha,
                       beta, ll, g_mu, g_alpha, g_beta, counter);
  }
  return hipGetLastError();
}

template <int P, int SB>
hipError_t launch_shared_fit(const Events& ev, int M, const FitParams& o, float* mu,
                             float* alpha, float* beta, double* ll, int* steps, int* status,
                             int* evals, float* ws, int64_t ws_floats, int* counter,
                             hipStream_t s) {
  if (ev.W == 0) return hipSuccess;
  reset_counter(counter, s);
  if (o.optimizer == MDHP_OPT_LBFGS) {
    auto k = shared_lbfgs_kernel<P, SB>;
    const int64_t per_block = (int64_t)kLbfgsVectors * (own_count(P) + 1) * kBlock;
    const int grid = (int)std::min<int64_t>(occupancy_grid(k, kBlock, ev.W), ws_floats / per_block);
    if (grid < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), 0, s, ev, M, o, mu, alpha, beta, ll, steps,
                       status, evals, ws, counter);
    return hipGetLastError();
  }
  auto k = shared_fit_kernel<P, SB>;
  hipLaunchKernelGGL(k, dim3(occupancy_grid(k, kBlock, ev.W)), dim3(kBlock), 0, s, ev, M, o, mu,
                     alpha, beta, ll, steps, status, evals, counter);
  return hipGetLastError();
}

template <int P, int SB>
int64_t shared_lbfgs_ws(int64_t W) {
  const int64_t per_block = (int64_t)kLbfgsVectors * (own_count(P) + 1) * kBlock;
  return per_block * occupancy_grid(shared_lbfgs_kernel<P, SB>, kBlock, std::max<int64_t>(W, 1));
}

// Calls f(std::integral_constant<int, P>, std::integral_constant<int, B>) for
// the plan's group width P and reduce-scatter width B (B matters for P >= 32
// only; other widths fall back to the default).
template <class F>
auto with_shape(int M, int scatter, F&& f) {
  using std::integral_constant;
  switch (lanes_for(M)) {
    case 4: return f(integral_constant<int, 4>{}, integral_constant<int, kScatter>{});
    case 8: return f(integral_constant<int, 8>{}, integral_constant<int, kScatter>{});
    case 16: return f(integral_constant<int, 16>{}, integral_constant<int, kScatter>{});
    case 32:
      if (scatter == 4) return f(integral_constant<int, 32>{}, integral_constant<int, 4>{});
      return f(integral_constant<int, 32>{}, integral_constant<int, 8>{});
    default:
      if (scatter == 4) return f(integral_constant<int, 64>{}, integral_constant<int, 4>{});
      if (scatter == 16) return f(integral_constant<int, 64>{}, integral_constant<int, 16>{});
      if (scatter == kScatterMfma)
        return f(integral_constant<int, 64>{}, integral_constant<int, kScatterMfma>{});
      return f(integral_constant<int, 64>{}, integral_constant<int, 8>{});
  }
}

}  // namespace

hipError_t shared_eval(const Events& ev, int M, int scatter, const float* mu, const float* alpha,
                       const float* beta, double* ll, float* g_mu, float* g_alpha, float* g_beta,
                       int* counter, hipStream_t s, bool grad) {
  return with_shape(M, scatter, [&](auto P, auto B) {
    return launch_shared_eval<P(), B()>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta,
                                        counter, s, grad);
  });
}

hipError_t shared_eval_wide(const Events& ev, int M, const float* mu, const float* alpha,
                            const float* beta, double* ll, float* g_mu, float* g_alpha,
                            float* g_beta, int* counter, hipStream_t s, bool grad) {
  if (M <= 32)
    return launch_shared_eval<32, kScatter>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta,
                                            counter, s, grad);
  return launch_shared_eval<64, kScatter>(ev, M, mu, alpha, beta, ll, g_mu, g_alpha, g_beta,
                                          counter, s, grad);
}

hipError_t shared_fit(const Events& ev, int M, int scatter, const FitParams& o, float* mu,
                      float* alpha, float* beta, double* ll, int* steps, int* status, int* evals,
                      float* ws, int64_t ws_floats, int* counter, hipStream_t s) {
  return with_shape(M, scatter, [&](auto P, auto B) {
    return launch_shared_fit<P(), B()>(ev, M, o, mu, alpha, beta, ll, steps, status, evals, ws,
                                       ws_floats, counter, s);
  });
}

int64_t shared_lbfgs_workspace(int M, int64_t W) {
  // Enough for every reduce-scatter width the plan may be tuned to.
  int64_t most = 0;
  for (int b : {4, 8, 16})
    most = std::max(most, with_shape(M, b, [&](auto P, auto B) {
      return shared_lbfgs_ws<P(), B()>(W);
    }));
  return most;
}

bool shared_scatter_ok(int M, int scatter) {
  const int p = lanes_for(M);
  if (p == 64) return scatter == 4 || scatter == 8 || scatter == 16 || scatter == kScatterMfma;
  if (p == 32) return scatter == 4 || scatter == 8;
  return scatter == kScatter;
}

}  // namespace mdhp
