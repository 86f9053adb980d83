// pamc_device.hpp -- device-side building blocks of the gfx950 PAMC library:
// the counter-based generator, the exponential used for every probability
// that decides an integer, and the device-resident run state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pamc {

// Stream tags carried in the fourth Philox counter word.
enum : uint32_t { kTagInit = 0, kTagSweep = 1, kTagResample = 2, kTagCluster = 3,
                  kTagOrder = 4, kTagDense = 5, kTagPotts = 6 };

// Pointers in the global address space.  Device pointers read from a
// descriptor table are generic to the compiler; casting them back lets it
// emit global (and, for uniform read-only data, scalar) loads instead of
// flat ones.
#define PAMC_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ PAMC_GLOBAL T* gmem(T* p) {
  return (PAMC_GLOBAL T*)p;
}

constexpr int kLanes = 64;      // replicas per tile = wavefront width
constexpr int kMaxHubs = 2;     // hub vertices with incrementally kept fields in the gathered-field mode
constexpr int kHistCap = 64;    // controller history capacity (>= win_long)

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products on counter words 0 and 2, whose high halves are xored with the
// other two words and the round key; the key is bumped by the Weyl
// increments (golden ratio and sqrt(3)-1 in 32-bit fixed point).
// ---------------------------------------------------------------------------
struct u32x4 { uint32_t a, b, c, d; };

// a ^ b ^ c in one three-input bitwise instruction (truth table 0x96).  Only
// worth it when at most one operand is wave-uniform: two scalar operands
// would need a copy to a vector register first.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// The counters used here always hold some uniform words (quad, sweep, tag
// or the like), so the first rounds mix uniform and per-lane values: those
// keep plain xors (uniform pairs are combined on the scalar unit); from the
// fourth round on every word is per-lane and the three-input form halves
// the xor count.
__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t m0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t m1 = (uint64_t)c2 * 0xCD9E8D57u;
    const uint32_t h0 = (uint32_t)(m0 >> 32), h1 = (uint32_t)(m1 >> 32);
    const uint32_t n0 = i < 3 ? (h1 ^ (c1 ^ k0)) : xor3(h1, c1, k0);
    const uint32_t n2 = i < 2 ? (h0 ^ (c3 ^ k1)) : xor3(h0, c3, k1);
    c1 = (uint32_t)m1;
    c3 = (uint32_t)m0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return u32x4{c0, c1, c2, c3};
}

__host__ __device__ __forceinline__ uint32_t pick(const u32x4& w, int i) {
  return i == 0 ? w.a : (i == 1 ? w.b : (i == 2 ? w.c : w.d));
}

// ---------------------------------------------------------------------------
// e^x in binary64 from basic operations only, so that host and device agree
// bit for bit: Cody-Waite reduction x = k ln2 + r with a two-part ln2 whose
// leading part times k is exact, e^r from the degree-13 Taylor polynomial in
// fused Horner form, and 2^k applied in exact power-of-two factors so that a
// subnormal result is rounded only once.  Must be compiled without
// floating-point contraction.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double two_to(int k) {  // -1022 <= k <= 1023
  return __longlong_as_double((long long)(k + 1023) << 52);
}

__device__ inline double exp_cw(double x) {
  if (!(x == x)) return x;
  if (x > 709.8) return __longlong_as_double(0x7FF0000000000000LL);
  if (x < -745.5) return 0.0;
  const double k = rint(x * 1.4426950408889634);
  const double r = (x - k * 0.6931471803691238) - k * 1.9082149292705877e-10;
  // coefficients 1/13!, 1/12!, ..., 1/2!, 1, 1
  double p = 1.6059043836821613e-10;
  p = fma(p, r, 2.08767569878681e-09);
  p = fma(p, r, 2.505210838544172e-08);
  p = fma(p, r, 2.755731922398589e-07);
  p = fma(p, r, 2.7557319223985893e-06);
  p = fma(p, r, 2.48015873015873e-05);
  p = fma(p, r, 0.0001984126984126984);
  p = fma(p, r, 0.001388888888888889);
  p = fma(p, r, 0.008333333333333333);
  p = fma(p, r, 0.041666666666666664);
  p = fma(p, r, 0.16666666666666666);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  p = fma(p, r, 1.0);
  const int ki = (int)k;
  if (ki > 1000) return (p * two_to(ki - 200)) * two_to(200);
  if (ki < -1000) return (p * two_to(ki + 200)) * two_to(-200);
  return p * two_to(ki);
}

// Flip threshold for x = s*h: a flip happens iff a uniform 32-bit word is
// below it.  Heat bath (Eq. 4): p = 1/(1 + e^{2 beta x}); Metropolis:
// p = e^{-2 beta x} for x > 0 (x <= 0 is accepted before the table is read).
// T = min(floor(p * 2^32), 2^32 - 1).
__device__ inline uint32_t flip_threshold(double beta, int rule, long long x) {
  const double tb = 2.0 * beta;
  double p;
  if (rule == 1) {
    if (x <= 0) return 0xFFFFFFFFu;
    p = exp_cw(-(tb * (double)x));
  } else {
    p = 1.0 / (1.0 + exp_cw(tb * (double)x));
  }
  const double f = floor(p * 4294967296.0);
  return f >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)f;
}

// Half-width of the threshold table: beyond |x| = ceil(12.5/|beta|) + 1 the
// heat-bath and Metropolis thresholds are saturated (e^{25} > 2^32), so
// clamping x into the table is exact.
// Potts labels: entries d = 0..D of the table e^{-beta d} (d = max syn -
// syn_k, at most 2X).  Beyond D (only when D < 2X) the value is exactly 0:
// beta d >= 746 + beta exceeds the point below which the exponential
// returns 0.
__host__ __device__ inline int64_t potts_table_last(double beta, int64_t X) {
  if (!(beta > 0)) return 2 * X;
  const double lim = 746.0 / beta;
  return lim >= (double)(2 * X) ? 2 * X : (int64_t)lim + 1;
}

__host__ __device__ inline int64_t table_halfwidth(double beta, int64_t X) {
  const double b = beta < 0 ? -beta : beta;
  if (b < 1e-300) return X < 1 ? X : 1;
  const double c = ceil(12.5 / b) + 1.0;
  if (c >= (double)X) return X;
  return (int64_t)c;
}

// ---------------------------------------------------------------------------
// Device-resident run state: Algorithm 1's controller variables, counters,
// per-step decisions and statistics.  Written by single-thread kernels
// between the data-parallel ones, read by all.
// ---------------------------------------------------------------------------
struct RunState {
  // schedule
  double beta0, dbeta, reheat;
  int64_t target;
  int32_t steps, sweeps, z_rst, augmented, resample;
  int32_t win_short, win_long, max_ds, max_dl, tau, n_top, mis_trials;
  int32_t stop_at_target, literal_break;
  // controller (Algorithm 1)
  double beta, delta;
  int32_t z, cycle, cooldown, enable, hist_len, stopped;
  int64_t hist[kHistCap];
  // per-step decisions
  int32_t step, active, do_resample, do_cluster, cur, best_slot;
  double rs_delta, sweep_beta;
  int32_t cl_n_top, cl_trials;
  int32_t nsweeps_now, pad1;  // sweeps of the current step / primitive call
  int64_t table_x;   // half-width of the current threshold table
  // counters of the random streams
  uint32_t gs, g_rs, g_cl, pad0;
  // best so far
  int64_t mstar;
  int32_t step_reached, steps_run;
  // statistics
  double sum_lnq, last_lnq;
  int32_t n_cluster_moves, n_reheats, n_reversals, n_restarts;
  int64_t flips, attempts, cl_flipped;
  uint64_t t_start, t_reached, t_last;  // device wall clock (100 MHz)
  // population diversity: mean pair distance every dh_every steps (0: off)
  int32_t dh_every, pad3;
  int64_t dh_sum;  // sum over pairs of min(d, n - d) for the step being measured
};

}  // namespace pamc
