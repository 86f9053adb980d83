// dense.hip -- fully connected instances (Sec. "Scalability on a Large-Scale
// Ising Problem"): int8 couplings J[n][n] in HBM, spins visited in the fixed
// order 0..n-1.
//
// A sweep runs over super-blocks of kSB = 1024 consecutive spins.  For each,
// one matrix-core launch computes the local fields of Eq. 3 of all its rows
// against the spins as they stand, G = J[sb, :] . S (int8 x int8 -> int32,
// exact since |h| <= 127 n < 2^31; split over the K dimension and summed
// atomically).  A sequential pass (one work-group per 64 replicas) then
// walks the super-block in blocks of kDB = 64 spins: the couplings to spins
// already flipped in earlier blocks of the super-block are added with a
// small matrix-core product over the recorded changes dS, and the block's
// spins are decided in order with h_k = G_k + C_k + sum_{k' < k in block}
// J_kk' d_k' (d = 2 s_new for flipped spins; packed int8 with dot4, or four
// bits with dot8 when every coupling fits), by the same threshold test as
// the sparse path in the form x < c (each visit's critical field c, computed
// for the whole sweep beforehand).  The pass and the next super-block's
// product share one launch.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/pamc.h"
#include "instance.hpp"
#include "pamc_device.hpp"

namespace pamc {

namespace {

constexpr int kDB = 64;          // spins per sequential block
static_assert(kDB / 4 == 6 + 6 + 4, "the helper waves' share of the critical-field groups assumes 16 groups");
constexpr int kSB = 1024;        // rows per super-block: one field product, one sequential launch
constexpr int kGM = 128, kGN = 128, kGK = 64;  // field-product tile: rows x replicas x K stage
constexpr int kLdsRow = kGK + 16;              // bytes per staged row (padded)
constexpr int kGStages = 3;                    // field-product K stages in flight per thread
constexpr int kThrL = 2047;      // half-width of the LDS copy of the threshold table
constexpr int32_t kCritInf = 1 << 30;  // critical field of a visit that flips (or not) at every x
typedef int v4i __attribute__((ext_vector_type(4)));

// J_ij = J_ji = +-1 from the low bit of Philox(key = seed; (i, j, 0, DENSE))
// word 0 for i < j; zero diagonal and zero padding.  Also accumulates
// W = sum_{i<j} (-J_ij).
__global__ void __launch_bounds__(256) k_dense_generate(int8_t* J, int32_t n, int32_t np, uint32_t k0,
                                                        uint32_t k1, int64_t* W) {
  const int64_t total = (int64_t)np * np;
  int64_t wsum = 0;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(idx / np), j = (int)(idx % np);
    int8_t v = 0;
    if (i < n && j < n && i != j) {
      const int a = i < j ? i : j, b = i < j ? j : i;
      v = (philox10((uint32_t)a, (uint32_t)b, 0u, kTagDense, k0, k1).a & 1u) ? 1 : -1;
      if (i < j) wsum -= v;
    }
    J[idx] = v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o, 64);
  if ((threadIdx.x & 63) == 0 && wsum)
    __hip_atomic_fetch_add((unsigned long long*)W, (unsigned long long)wsum, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Spins: +1 iff word (v & 3) of Philox(v >> 2, 0, r, INIT) < 2^31 (the same
// stream as sparse instances); padding columns are 0.
__global__ void __launch_bounds__(256) k_dense_init_spins(int8_t* S, int32_t* fam, int32_t n,
                                                          int32_t np, int32_t R, uint32_t k0,
                                                          uint32_t k1) {
  const int64_t total = (int64_t)R * (np / 4);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(i / (np / 4));
    const int q = (int)(i % (np / 4));
    const u32x4 w = philox10((uint32_t)q, 0u, (uint32_t)r, kTagInit, k0, k1);
    uint32_t word = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int v = 4 * q + k;
      const int8_t s = v < n ? (pick(w, k) < 0x80000000u ? (int8_t)1 : (int8_t)-1) : (int8_t)0;
      word |= (uint32_t)(uint8_t)s << (8 * k);
    }
    reinterpret_cast<uint32_t*>(S)[i] = word;
    if (q == 0) fam[r] = r;
  }
}

// G[m][r] += sum_{k in slice p} J[row0 + m][k] S[r][k] for the super-block's
// rows m < rows and every replica r (the K slices meet by atomic addition in
// G, which its reader clears).  Work-group = (128-row tile, 128-replica
// tile, K slice); each 64-column K stage of both operands is staged through
// LDS (double-buffered, rows padded by 16 bytes against bank conflicts) and
// the four waves (2 x 2) each compute a 64 x 64 block as 4 x 4
// v_mfma_i32_16x16x64_i8 tiles.  Operand fragments: lane l supplies 16
// consecutive K bytes at 16*(l/16) of row (A) / replica (B) l % 16; the
// result holds rows 4*(l/16)..+3 of column l % 16.
// The product runs over a K domain given as columns kbase .. kbase + kcount
// + xlen with the xlen columns from kbase + x0 left out (x0, xlen, kbase and
// kcount multiples of 64): compacted column k maps to kbase + k, plus xlen
// once k >= x0.
struct GemmArgs {
  const int8_t* J;
  const int8_t* S0;
  const int8_t* S1;
  int32_t* G;
  const RunState* st;
  int32_t row0, rows, np, R, use_state, kslice;
  int32_t kbase, kcount, x0, xlen;
};

struct GemmLds {
  __attribute__((aligned(16))) int8_t As[2][kGM * kLdsRow];
  __attribute__((aligned(16))) int8_t Bs[2][kGN * kLdsRow];
};

__device__ __forceinline__ void gemm_body(const GemmArgs g, int bid, GemmLds& L) {
  auto& As = L.As;
  auto& Bs = L.Bs;
  const int8_t* __restrict__ J = g.J;
  int32_t* __restrict__ G = g.G;
  const int32_t row0 = g.row0, rows = g.rows, np = g.np, R = g.R, kslice = g.kslice;
  if (g.use_state == 1 && !g.st->active) return;
  const int8_t* __restrict__ S = (g.use_state ? g.st->cur : 0) ? g.S1 : g.S0;
  // XCD-aware order: work-groups are dealt to the 8 XCDs round-robin, so
  // every output tile of K slice p lands on XCD p % 8 and the slice's J
  // columns and spins are fetched into that XCD's L2 once, not once per
  // tile row / column
  const int MT = (rows + kGM - 1) / kGM, NT = (R + kGN - 1) / kGN;
  const int xcd = bid & 7, q = bid >> 3;
  const int tile = q % (MT * NT);
  const int p = (q / (MT * NT)) * 8 + xcd;
  const int mt = tile % MT, ntile = tile / MT;
  const int k_beg = p * kslice, k_end = min(g.kcount, k_beg + kslice);
  if (k_beg >= k_end) return;
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  // staging: 512 chunks of 16 bytes per operand tile, chunks t and t + 256
  // per thread; chunk c = (row c / 4, bytes 16 (c % 4) ..).  Rows past the
  // super-block or replicas past R re-read the last valid one; their results
  // are dropped below.
  const v4i zero = {0, 0, 0, 0};
  const int8_t* ag[2];
  const int8_t* bg[2];
  int lofs[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int c = t + 256 * i, row = c >> 2, col = (c & 3) * 16;
    const int m = min(mt * kGM + row, rows - 1), n = min(ntile * kGN + row, R - 1);
    ag[i] = J + (size_t)(row0 + m) * np + col;
    bg[i] = S + (size_t)n * np + col;
    lofs[i] = row * kLdsRow + col;
  }
  // kGStages K stages in flight in registers: the loads of stage s + D are
  // issued while stage s is multiplied, so each load has D - 1 stages of
  // matrix-core work to arrive in; stage s + 1 goes to the other LDS buffer
  // at the end of stage s.  In the main loop every load and store is
  // unconditional (a prefetch past the last stage re-reads the last stage
  // and is never used), so the compiler waits for exactly the stage it
  // stores, not for everything in flight.
  constexpr int D = kGStages;
  const int nst = (k_end - k_beg) / kGK;
  v4i ra[D][2], rb[D][2];
  auto load_stage = [&](int slot, int stage) {
    const int kc = k_beg + stage * kGK;  // compacted column of the stage
    const int k = g.kbase + kc + (kc >= g.x0 ? g.xlen : 0);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ra[slot][i] = *reinterpret_cast<const v4i*>(ag[i] + k);
      rb[slot][i] = *reinterpret_cast<const v4i*>(bg[i] + k);
    }
  };
  auto store_stage = [&](int slot, int buf) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      *reinterpret_cast<v4i*>(As[buf] + lofs[i]) = ra[slot][i];
      *reinterpret_cast<v4i*>(Bs[buf] + lofs[i]) = rb[slot][i];
    }
  };
  v4i acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = zero;
  const int frag = (lane & 15) * kLdsRow + 16 * (lane >> 4);
  auto multiply = [&](int buf) {
    v4i af[4], bf[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      af[i] = *reinterpret_cast<const v4i*>(As[buf] + (wm * 64 + 16 * i) * kLdsRow + frag);
      bf[i] = *reinterpret_cast<const v4i*>(Bs[buf] + (wn * 64 + 16 * i) * kLdsRow + frag);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
        acc[i][jj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[i], bf[jj], acc[i][jj], 0, 0, 0);
  };
#pragma unroll
  for (int d = 0; d < D; ++d) load_stage(d, min(d, nst - 1));
  store_stage(0, 0);
  __syncthreads();
  int s0 = 0;
  for (; s0 + D <= nst; s0 += D) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const int st_ = s0 + j;  // in LDS buffer st_ & 1; register slot j is free
      load_stage(j, min(st_ + D, nst - 1));
      multiply(st_ & 1);
      store_stage((j + 1) % D, (st_ + 1) & 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int j = 0; j < D; ++j) {  // the last nst % D stages
    const int st_ = s0 + j;
    if (st_ < nst) {
      multiply(st_ & 1);
      if (st_ + 1 < nst) store_stage((j + 1) % D, (st_ + 1) & 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = mt * kGM + wm * 64 + 16 * i + 4 * (lane >> 4) + e;
        const int n = ntile * kGN + wn * 64 + 16 * j + (lane & 15);
        const int32_t v = acc[i][j][e];
        if (v != 0 && m < rows && n < R)
          __hip_atomic_fetch_add(&G[(size_t)m * R + n], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
}

__global__ void __launch_bounds__(256) k_dense_gemm(GemmArgs g) {
  __shared__ GemmLds L;
  gemm_body(g, blockIdx.x, L);
}

// Sequential visit of one super-block's spins for one 64-replica tile.
struct SeqArgs {
  const int8_t* J;
  int8_t* S0;
  int8_t* S1;
  int64_t* E0;
  int64_t* E1;
  int32_t* G;   // [kSB][R] fields of the super-block rows against its starting spins
  const uint32_t* thr;
  const v4i* C;  // [n_pad / 4][R] critical fields of the sweep (k_dense_crit)
  RunState* st;
  int32_t n, np, R;
  int32_t j4;  // every coupling in [-8, 7]: the sequential pass uses four-bit dot products
  uint32_t k0, k1;
  int64_t* flip_ctr;
};


// Critical fields of one sweep's visits.  The thresholds T[x + Xl] (|x| <=
// Xl) do not increase with x, so the test u < T[x + Xl] holds exactly for
// x < c - Xl, c = the number of leading entries of T[0 .. 2Xl] above u.  The
// stored value is c - Xl, with c = 0 stored as -2^30 and c = 2Xl + 1 as
// +2^30, so that a field beyond the table (|x| > Xl, when the table is
// saturated) meets the decision of the clamped lookup (|x| < 2^30 - 2^12);
// Metropolis then raises it to 1 (x <= 0 always flips).  C[q][r] holds the
// four spins of quad q for replica r, from the same Philox words (q, sweep,
// r, SWEEP) as the visits.  The table lives in LDS; the search is a
// fixed-step binary lifting over it.
template <int RULE>
__global__ void __launch_bounds__(256) k_dense_crit(const uint32_t* thr, const RunState* st, v4i* C,
                                                    int32_t sweep_idx, int32_t nq, int32_t R, uint32_t k0,
                                                    uint32_t k1) {
  __shared__ uint32_t thr_s[2 * kThrL + 1];
  if (!st->active) return;
  const int32_t Xt = (int32_t)st->table_x, Xl = min(Xt, kThrL), L = 2 * Xl + 1;
  const uint32_t gs = st->gs + (uint32_t)sweep_idx;
  for (int i = threadIdx.x; i < L; i += blockDim.x) thr_s[i] = thr[Xt - Xl + i];
  __syncthreads();
  const int64_t total = (int64_t)nq * R, stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t q = (int32_t)(first / R), r = (int32_t)(first % R);
  const int32_t dq = (int32_t)(stride / R), dr = (int32_t)(stride % R);
  for (int64_t it = first; it < total; it += stride) {
    const u32x4 w = philox10((uint32_t)q, gs, (uint32_t)r, kTagSweep, k0, k1);
    int32_t pos[4] = {0, 0, 0, 0};
    // pos + step <= 4096 - step before each step, so every read is inside
    // the table's 2 kThrL + 1 entries (entries at or past L are never taken)
#pragma unroll
    for (int step = 2048; step > 0; step >>= 1)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int32_t p = pos[kk] + step;
        const uint32_t tv = thr_s[p - 1];
        pos[kk] = (p <= L && tv > pick(w, kk)) ? p : pos[kk];
      }
    v4i c;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      int32_t v = pos[kk] == 0 ? -kCritInf : pos[kk] == L ? kCritInf : pos[kk] - Xl;
      if (RULE == 1) v = max(v, 1);
      c[kk] = v;
    }
    C[it] = c;
    q += dq;
    r += dr;
    if (r >= R) {
      r -= R;
      q += 1;
    }
  }
}

// One pass over the 64 spins of one block for one replica per lane (wave 0):
// h_k = gsum_k + sum_{k' < k in block} J_kk' d_k' (d = 2 s_new of flipped
// spins, packed int8, dot4), x = s h, flip iff x < cc (the visit's critical
// field, from LDS); every spin of the block is below n.  sw: the block's 16
// starting spin words; d: the block's d words.  With WIDE the pass also
// returns whether any lane met |x| > Xl (needed only when the LDS table is
// narrower than the full one).  The sign is applied as a mask, m = 0 or -1:
// x < cc is (h ^ m) < cc + m, since h ^ -1 = -h - 1.  The pass has no
// branches, so the compiler can move the independent work (the couplings to
// earlier groups, LDS reads) into the latency of the decision chain, which
// per spin is dot4, xor, compare, select.
template <int RULE, bool WIDE>
__device__ __forceinline__ bool decide_pass(const uint32_t (*jd)[kDB / 4], const int32_t (*gsum)[64],
                                            const v4i (*crit)[64], int32_t Xl, const uint32_t (&sw)[kDB / 4],
                                            int lane, uint32_t (&d)[kDB / 4], int32_t& dE32, int32_t& nflip) {
  uint32_t wide = 0;
  int32_t xsum = 0, nf = 0;
#pragma unroll
  for (int g = 0; g < kDB / 4; ++g) d[g] = 0;
#pragma unroll
  for (int g = 0; g < kDB / 4; ++g) {
    const v4i cc = crit[g][lane];
    // couplings to the flips of the earlier groups of the block: four
    // independent accumulations, in group order, so only the last one
    // (the previous group's flips) waits for the decision chain
    int32_t base[4];
    uint32_t jg[4];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * g + kk;
      int32_t p = gsum[k][lane];
#pragma unroll
      for (int g2 = 0; g2 < g; ++g2) p = __builtin_amdgcn_sdot4((int)jd[k][g2], (int)d[g2], p, false);
      base[kk] = p;
      jg[kk] = jd[k][g];
    }
    const uint32_t w = sw[g];
    // the d byte of a flip, -2 s: 0xFE for s = +1 (0x01), 0x02 for s = -1 (0xFF)
    const uint32_t bw = 0xFEFEFEFEu ^ (((w >> 7) & 0x01010101u) * 0xFCu);
    uint32_t dg = 0;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      // m = -1 for s = -1 (its own spin has not changed yet), else 0
      const int32_t m = (int32_t)(w << (24 - 8 * kk)) >> 31;
      const int32_t h = __builtin_amdgcn_sdot4((int)jg[kk], (int)dg, base[kk], false);
      const int32_t y = h ^ m;  // x = y - m
      if (WIDE) wide |= (uint32_t)(h + Xl) > (uint32_t)(2 * Xl);
      const bool flip = y < cc[kk] + m;
      dg = flip ? dg | (bw & (0xFFu << (8 * kk))) : dg;
      xsum += flip ? y : 0;
    }
    d[g] = dg;
  }
  // a flipped byte is 0xFE (s = +1) or 0x02 (s = -1): bit 1 counts the
  // flips, bit 2 those of s = +1; sum x = sum y + the flips of s = -1
  int32_t npos = 0;
#pragma unroll
  for (int g = 0; g < kDB / 4; ++g) {
    nf += __builtin_popcount(d[g] & 0x02020202u);
    npos += __builtin_popcount(d[g] & 0x04040404u);
  }
  dE32 += xsum + (nf - npos);
  nflip += nf;
  return wide != 0;
}

// The same pass for couplings in [-8, 7], four bits each.  jd8 packs a
// row's couplings to eight spins of the block per word and the flips are
// kept in the same layout -- of the eight spins 8G + j, nibble 2j holds
// spin j < 4 and nibble 2 (j - 4) + 1 spin j >= 4 -- so that one dot8 covers
// eight couplings; a flip is the nibble 0xE (s = +1) or 0x2 (s = -1).  The
// d words go out as bytes, unpacked at the end.
template <int RULE, bool WIDE>
__device__ __forceinline__ bool decide_pass8(const uint32_t (*jd8)[kDB / 8], const int32_t (*gsum)[64],
                                             const v4i (*crit)[64], int32_t Xl, const uint32_t (&sw)[kDB / 4],
                                             int lane, uint32_t (&d)[kDB / 4], int32_t& dE32, int32_t& nflip) {
  uint32_t wide = 0, d8[kDB / 8];
  int32_t xsum = 0, nf = 0, npos = 0;
#pragma unroll
  for (int G = 0; G < kDB / 8; ++G) d8[G] = 0;
#pragma unroll
  for (int G = 0; G < kDB / 8; ++G) {
    const v4i cc0 = crit[2 * G][lane], cc1 = crit[2 * G + 1][lane];
    int32_t base[8];
    uint32_t jg[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * G + j;
      int32_t p = gsum[k][lane];
#pragma unroll
      for (int G2 = 0; G2 < G; ++G2) p = __builtin_amdgcn_sdot8((int)jd8[k][G2], (int)d8[G2], p, false);
      base[j] = p;
      jg[j] = jd8[k][G];
    }
    const uint32_t w0 = sw[2 * G], w1 = sw[2 * G + 1];
    // the flip nibbles, 0xE, or 0x2 where the spin is -1
    const uint32_t negn = ((w0 >> 7) & 0x01010101u) | ((w1 >> 3) & 0x10101010u);
    const uint32_t bw = 0xEEEEEEEEu ^ (negn * 0xCu);
    uint32_t dg = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int jb = j & 3, sh = j < 4 ? 8 * jb : 8 * jb + 4;
      const int32_t m = (int32_t)((j < 4 ? w0 : w1) << (24 - 8 * jb)) >> 31;
      const int32_t h = __builtin_amdgcn_sdot8((int)jg[j], (int)dg, base[j], false);
      const int32_t y = h ^ m;  // x = y - m
      if (WIDE) wide |= (uint32_t)(h + Xl) > (uint32_t)(2 * Xl);
      const bool flip = y < (j < 4 ? cc0[jb] : cc1[jb]) + m;
      dg = flip ? dg | (bw & (0xFu << sh)) : dg;
      xsum += flip ? y : 0;
    }
    d8[G] = dg;
  }
#pragma unroll
  for (int G = 0; G < kDB / 8; ++G) {
    // bit 1 of a flip nibble counts the flips, bit 2 those of s = +1
    nf += __builtin_popcount(d8[G] & 0x22222222u);
    npos += __builtin_popcount(d8[G] & 0x44444444u);
    // nibbles 0, 2, 4, 6 are spins 0..3, nibbles 1, 3, 5, 7 spins 4..7;
    // 0x0E becomes the byte 0xFE
    const uint32_t lo = d8[G] & 0x0F0F0F0Fu, hi = (d8[G] >> 4) & 0x0F0F0F0Fu;
    d[2 * G] = lo | ((lo & 0x08080808u) * 0x1Eu);
    d[2 * G + 1] = hi | ((hi & 0x08080808u) * 0x1Eu);
  }
  dE32 += xsum + (nf - npos);
  nflip += nf;
  return wide != 0;
}

struct BlockTally {
  int32_t dE32, nflip;
};

// The same decisions with every threshold exact (fields beyond the LDS
// table recomputed by the function that fills it), from the block's
// starting spin words sw0 (LDS); the d words go to dout (LDS).  Out of line
// and unoptimised for speed: only reached when a lane met |x| > Xl.
template <int RULE>
__device__ __noinline__ BlockTally decide_block_exact(const uint32_t (*jd)[kDB / 4], const int32_t (*gsum)[64],
                                                      const uint32_t* thr_s, double beta, int32_t Xl, int32_t Xt,
                                                      const uint32_t* sw0, uint32_t* dout, int rb0, int n,
                                                      uint32_t gs, uint32_t r, uint32_t k0, uint32_t k1, int lane) {
  BlockTally t = {0, 0};
  for (int g = 0; g < kDB / 4; ++g) {
    const int vq = rb0 + 4 * g;
    const u32x4 rnd = philox10((uint32_t)(vq >> 2), gs, r, kTagSweep, k0, k1);
    uint32_t w = sw0[g], dg = 0;
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 4 * g + kk;
      int32_t h = gsum[k][lane];
      for (int g2 = 0; g2 < g; ++g2) h = __builtin_amdgcn_sdot4((int)jd[k][g2], (int)dout[g2], h, false);
      h = __builtin_amdgcn_sdot4((int)jd[k][g], (int)dg, h, false);
      const int32_t sm = -(int32_t)((w >> (8 * kk + 7)) & 1u);
      const int32_t x = (h ^ sm) - sm;
      const int32_t xl = min(max(x, -Xl), Xl);
      const uint32_t thr = x == xl ? thr_s[xl + Xl] : flip_threshold(beta, RULE, min(max(x, -Xt), Xt));
      const uint32_t u = kk == 0 ? rnd.a : kk == 1 ? rnd.b : kk == 2 ? rnd.c : rnd.d;
      bool flip = u < thr;
      if (RULE == 1) flip = flip || x <= 0;
      flip = flip && vq + kk < n;
      if (flip) {
        t.dE32 += x;
        w ^= 0xFEu << (8 * kk);
        dg |= (uint32_t)(uint8_t)(int8_t)(sm == 0 ? -2 : 2) << (8 * kk);
        t.nflip += 1;
      }
    }
    dout[g] = dg;
  }
  return t;
}

// Decides the 64 spins of one block; d words into dout (LDS).  The critical
// fields cover |x| <= Xl; when the LDS table is narrower than the full one
// (Xl < Xt) and some lane met a field beyond it, the block is decided
// again, exactly, from its starting spins (one uniform branch per block
// keeps the common pass free of control flow).  The last block of the
// matrix, which holds spins at or beyond n, takes the exact path directly,
// and so does every block when the table is not monotone (all_exact).
template <int RULE, bool WIDE, bool J4>
__device__ __forceinline__ void decide_block(const uint32_t (*jd)[kDB / 4], const uint32_t (*jd8)[kDB / 8],
                                             const int32_t (*gsum)[64],
                                             const v4i (*crit)[64], const uint32_t* thr_s, double beta,
                                             int32_t Xl, int32_t Xt, bool all_exact, const uint32_t* sw0,
                                             uint32_t* dout, int rb0, int n, uint32_t gs, uint32_t r, uint32_t k0,
                                             uint32_t k1, int lane, int64_t& dE, int32_t& nflip) {
  int32_t dE32 = 0, nf = 0;  // |dE32| <= 64 X < 2^31 (X < 2^25)
  bool exact = all_exact || rb0 + kDB > n;
  if (!exact) {
    uint32_t sw[kDB / 4], d[kDB / 4];
#pragma unroll
    for (int g = 0; g < kDB / 4; ++g) sw[g] = sw0[g];
    const bool wide = J4 ? decide_pass8<RULE, WIDE>(jd8, gsum, crit, Xl, sw, lane, d, dE32, nf)
                         : decide_pass<RULE, WIDE>(jd, gsum, crit, Xl, sw, lane, d, dE32, nf);
    exact = WIDE && __builtin_amdgcn_ballot_w64(wide) != 0;
    if (!exact) {
#pragma unroll
      for (int g = 0; g < kDB / 4; ++g) dout[g] = d[g];
    }
  }
  if (exact) {
    const BlockTally t = decide_block_exact<RULE>(jd, gsum, thr_s, beta, Xl, Xt, sw0, dout, rb0, n, gs, r, k0, k1,
                                                  lane);
    dE32 = t.dE32;
    nf = t.nflip;
  }
  dE += 2 * (int64_t)dE32;
  nflip += nf;
}

// One work-group per tile walks the super-block's 64-spin blocks in order,
// pipelined: while wave 0 decides block b (and writes its replica's new spin
// words back), waves 1-3 prepare block b + 1 -- its fields G (taken from the
// field product, which is cleared for the next super-block), plus the
// couplings to the spins flipped in blocks 0..b-1 of the super-block, C =
// J[blk b+1, blocks 0..b-1] . dS (matrix cores; the spin changes dS of the
// super-block are kept in LDS, replica-major), its diagonal block of J and
// its critical fields.  After wave 0 is done, the four waves add block b's
// own contribution to block b + 1 (one 64-column matrix-core step, its J
// fragments loaded before the decisions).
struct SeqLds {
  uint32_t jd[2][kDB][kDB / 4];   // J[rb0 + k][rb0 + 4g .. 4g+3], packed int8
  uint32_t jd8[2][kDB][kDB / 8];  // the same, eight four-bit couplings per word (order of decide_pass8)
  int32_t gsum[2][kDB][64];       // fields of this tile before the block's own flips
  uint32_t thr_s[2 * kThrL + 1];  // thresholds for |x| <= Xl
  __attribute__((aligned(16))) int8_t dsl[64][kSB + 16];  // spin changes d, [replica][row - row0]
  uint32_t swl[2][64][kDB / 4 + 1];                       // the block's spin words, [replica][word]
  int32_t part[16][64];  // wave 2's part of strip 3, fragment rows x replicas
  __attribute__((aligned(16))) v4i crit[kDB / 4][64];     // the block's critical fields, [group][replica]
};

// Barrier for work-groups whose waves exchange data through LDS only: the
// waves' LDS writes complete before it, and their global loads and stores
// in flight stay in flight (a full __syncthreads would wait for those too,
// e.g. for the deciding wave's spin write-back).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int RULE, bool WIDE, bool J4>
__device__ __forceinline__ void seq_body(const SeqArgs a, int tile, int32_t sweep_idx, int32_t row0, int32_t rows,
                                         SeqLds& L) {
  auto& jd = L.jd;
  auto& jd8 = L.jd8;
  auto& gsum = L.gsum;
  auto& thr_s = L.thr_s;
  auto& dsl = L.dsl;
  auto& swl = L.swl;
  auto& crit = L.crit;
  auto& part = L.part;
  RunState* st = a.st;
  if (!st->active) return;
  const int cur = st->cur;
  int8_t* S = cur ? a.S1 : a.S0;
  int64_t* E = cur ? a.E1 : a.E0;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = tile * 64 + lane;
  const uint32_t gs = st->gs + (uint32_t)sweep_idx;
  const int32_t Xt = (int32_t)st->table_x;
  const double beta = st->sweep_beta;
  // The central part of the table lives in LDS, for the exact path (which
  // recomputes it for |x| > Xl) and the monotonicity check below.
  const int32_t Xl = min(Xt, kThrL);
  for (int i = threadIdx.x; i <= 2 * Xl; i += blockDim.x) thr_s[i] = a.thr[Xt - Xl + i];
  const int nb = min(rows, a.n - row0 + kDB - 1) / kDB;  // blocks holding real spins
  // fields of block bb (rows row0 + 64 bb ..) from G, cleared behind for
  // the next super-block's product; the diagonal J block
  auto load_fields = [&](int bb, int buf) {
    for (int i = threadIdx.x; i < kDB * 64; i += blockDim.x) {
      const int k = i >> 6, c = i & 63;
      int32_t* gp = a.G + (size_t)(bb * kDB + k) * a.R + tile * 64 + c;
      gsum[buf][k][c] = *gp;
      *gp = 0;
    }
  };
  // words 2 gp and 2 gp + 1 of row k of the diagonal J block, in bytes and
  // in four-bit couplings (nibble 2 b from the first word's byte b, nibble
  // 2 b + 1 from the second's)
  auto put_jd = [&](int buf, int k, int gp, uint32_t lo, uint32_t hi) {
    jd[buf][k][2 * gp] = lo;
    jd[buf][k][2 * gp + 1] = hi;
    jd8[buf][k][gp] = (lo & 0x0F0F0F0Fu) | ((hi & 0x0F0F0F0Fu) << 4);
  };
  auto load_diag = [&](int bb, int buf, int t, int nt) {
    const int rb0 = row0 + bb * kDB;
    for (int i = t; i < kDB * kDB / 8; i += nt) {
      const int k = i / (kDB / 8), gp = i % (kDB / 8);
      const uint2 w = *reinterpret_cast<const uint2*>(a.J + (size_t)(rb0 + k) * a.np + rb0 + 8 * gp);
      put_jd(buf, k, gp, w.x, w.y);
    }
    for (int i = t; i < kDB * kDB / 4; i += nt) {
      const int k = i / (kDB / 4), g = i % (kDB / 4);
      // the block's spin words of the tile (replica k, word g)
      swl[buf][k][g] = *reinterpret_cast<const uint32_t*>(S + (size_t)(tile * 64 + k) * a.np + rb0 + 4 * g);
    }
  };
  // the diagonal block of bb into registers (lane t of wave 3) and from
  // there into LDS
  constexpr int kDiagPer = kDB * kDB / 4 / 64;  // spin words per thread of wave 3
  constexpr int kPairPer = kDB * kDB / 8 / 64;  // J word pairs per thread of wave 3
  auto fetch_diag = [&](int bb, int t, uint2 (&dj)[kPairPer], uint32_t (&dsw)[kDiagPer]) {
    const int rb0 = row0 + bb * kDB;
#pragma unroll
    for (int it = 0; it < kPairPer; ++it) {
      const int i = t + 64 * it, k = i / (kDB / 8), gp = i % (kDB / 8);
      dj[it] = *reinterpret_cast<const uint2*>(a.J + (size_t)(rb0 + k) * a.np + rb0 + 8 * gp);
    }
#pragma unroll
    for (int it = 0; it < kDiagPer; ++it) {
      const int i = t + 64 * it, k = i / (kDB / 4), g = i % (kDB / 4);
      dsw[it] = *reinterpret_cast<const uint32_t*>(S + (size_t)(tile * 64 + k) * a.np + rb0 + 4 * g);
    }
  };
  auto put_diag = [&](int buf, int t, const uint2 (&dj)[kPairPer], const uint32_t (&dsw)[kDiagPer]) {
#pragma unroll
    for (int it = 0; it < kPairPer; ++it) {
      const int i = t + 64 * it;
      put_jd(buf, i / (kDB / 8), i % (kDB / 8), dj[it].x, dj[it].y);
    }
#pragma unroll
    for (int it = 0; it < kDiagPer; ++it) {
      const int i = t + 64 * it, k = i / (kDB / 4), g = i % (kDB / 4);
      swl[buf][k][g] = dsw[it];
    }
  };
  // the 16-row strip sr of block bb against the column steps kbeg .. kend
  // of the super-block (64 columns each): its J fragments (step kbeg + i in
  // av[i]), and its fields from G (fragment layout: row 4 (lane / 16) + j
  // of the strip, replica 16 nt + lane % 16)
  auto load_frags = [&](int bb, int sr, int kbeg, int kend, auto& av) {
    constexpr int N = sizeof(av) / sizeof(av[0]);
    const int8_t* arow = a.J + (size_t)(row0 + bb * kDB + 16 * sr + (lane & 15)) * a.np + row0 + 16 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < N; ++i)
      av[i] = kbeg + i < kend ? *reinterpret_cast<const v4i*>(arow + 64 * (kbeg + i)) : v4i{0, 0, 0, 0};
  };
  auto load_g = [&](int bb, int sr, int32_t (&gv)[16]) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        gv[4 * nt + j] = a.G[(size_t)(bb * kDB + 16 * sr + 4 * (lane >> 4) + j) * a.R + tile * 64 + nt * 16 +
                             (lane & 15)];
  };
  // acc += J[strip rows][steps kbeg .. kend) . dsl[:, those columns] on
  // the matrix cores
  auto strip_product = [&](int kbeg, int kend, const auto& av, v4i (&acc)[4]) {
    constexpr int N = sizeof(av) / sizeof(av[0]);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (kbeg + i < kend) {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
          const v4i bv =
              *reinterpret_cast<const v4i*>(&dsl[nt * 16 + (lane & 15)][64 * (kbeg + i) + 16 * (lane >> 4)]);
          acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[i], bv, acc[nt], 0, 0, 0);
        }
      }
    }
  };
  // result fragment of strip sr into gsum[buf]: with G, the fields gv
  // taken from the field product plus the product (G is cleared behind for
  // the next super-block's product), else added to gsum
  auto add_strip = [&](int bb, int buf, int sr, const v4i (&acc)[4], const int32_t* gv) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = 16 * sr + 4 * (lane >> 4) + j, c = nt * 16 + (lane & 15);
        if (gv) {
          gsum[buf][k][c] = gv[4 * nt + j] + acc[nt][j];
          a.G[(size_t)(bb * kDB + k) * a.R + tile * 64 + c] = 0;
        } else {
          gsum[buf][k][c] += acc[nt][j];
        }
      }
  };
  // critical fields of block bb, group g (four spins), this lane's replica
  auto crit_group = [&](int bb, int g) { return a.C[(size_t)(((row0 + bb * kDB) >> 2) + g) * a.R + r]; };
  if (nb > 0) {
    load_fields(0, 0);
    load_diag(0, 0, threadIdx.x, blockDim.x);
    for (int g = wave; g < kDB / 4; g += 4) crit[g][lane] = crit_group(0, g);
  }
  __syncthreads();
  // the critical fields assume thresholds that do not increase with x;
  // should the table ever break that, every block takes the exact path
  bool mono = true;
  for (int i = threadIdx.x; i < 2 * Xl; i += blockDim.x) mono = mono && thr_s[i] >= thr_s[i + 1];
  const bool all_exact = !__syncthreads_and(mono);
  int64_t dE = 0;
  int32_t nflip = 0;
  const v4i zero = {0, 0, 0, 0};
  for (int b = 0; b < nb; ++b) {
    const int cb = b & 1;
    const int rb0 = row0 + b * kDB;
    const bool next = b + 1 < nb;
    // J fragment of block b+1, strip `wave`, against block b's columns
    v4i a_next = zero;
    if (next)
      a_next = *reinterpret_cast<const v4i*>(a.J + (size_t)(rb0 + kDB + 16 * wave + (lane & 15)) * a.np + rb0 +
                                             16 * (lane >> 4));
    // waves 1..3: the critical fields of block b+1 (held in registers
    // until wave 0 is done with block b's); wave 3, which also takes the
    // diagonal block, loads 4 of the 16 groups, waves 1 and 2 six each
    constexpr int kCritPerHelper = 6;
    const int crit_g0 = wave == 1 ? 0 : wave == 2 ? 6 : 12;
    const int crit_cnt = wave == 3 ? 4 : 6;
    v4i crit_next[kCritPerHelper];
    if (wave == 0) {
      // the d words go to the super-block's spin changes (dsl)
      decide_block<RULE, WIDE, J4>(jd[cb], jd8[cb], gsum[cb], crit, thr_s, beta, Xl, Xt, all_exact, swl[cb][lane],
                                   reinterpret_cast<uint32_t*>(&dsl[lane][b * kDB]), rb0, a.n, gs, (uint32_t)r,
                                   a.k0, a.k1, lane, dE, nflip);
      // the lane's new spin words of the block go straight back: a byte of
      // d is 0 (no flip), 2 or -2, and a flip turns 0x01 <-> 0xFF, i.e. xor
      // 0xFE
      {
        const uint32_t* dw = reinterpret_cast<const uint32_t*>(&dsl[lane][b * kDB]);
        const uint32_t* sw = swl[cb][lane];
        uint4* dst = reinterpret_cast<uint4*>(S + (size_t)r * a.np + rb0);
#pragma unroll
        for (int q = 0; q < kDB / 16; ++q) {
          uint4 v;
          v.x = sw[4 * q] ^ ((dw[4 * q] & 0x02020202u) * 0x7Fu);
          v.y = sw[4 * q + 1] ^ ((dw[4 * q + 1] & 0x02020202u) * 0x7Fu);
          v.z = sw[4 * q + 2] ^ ((dw[4 * q + 2] & 0x02020202u) * 0x7Fu);
          v.w = sw[4 * q + 3] ^ ((dw[4 * q + 3] & 0x02020202u) * 0x7Fu);
          dst[q] = v;
        }
      }
    } else {
      // Helper wave w takes strip w - 1 of block b+1 over all b column
      // steps; strip 3 is split at step h = b / 2, steps [0, h) to wave 1
      // (with its fields G) and [h, b) to wave 2 (into an LDS partial that
      // wave 3 adds after the barrier); wave 3 also takes the diagonal
      // block.  The global reads of a part are issued before any of them
      // is used, so that their latencies overlap.
      const int h = b / 2;
      if (next) {
#pragma unroll
        for (int i = 0; i < kCritPerHelper; ++i)
          if (i < crit_cnt) crit_next[i] = crit_group(b + 1, crit_g0 + i);
        v4i acc[4] = {zero, zero, zero, zero};
        v4i av[kSB / kDB - 2];  // b <= kSB / kDB - 2 when there is a next block
        int32_t gv[16];
        if (wave == 3) {
          // every read of the wave for block b+1 (diagonal block, strip,
          // fields) in flight together
          uint2 dj[kPairPer];
          uint32_t dsw[kDiagPer];
          fetch_diag(b + 1, lane, dj, dsw);
          load_frags(b + 1, 2, 0, b, av);
          load_g(b + 1, 2, gv);
          put_diag(cb ^ 1, lane, dj, dsw);
          strip_product(0, b, av, acc);
          add_strip(b + 1, cb ^ 1, 2, acc, gv);
        } else {
          // the wave's strip and its part of strip 3, read together
          v4i a3[(kSB / kDB - 1) / 2];
          int32_t gv3[16];
          const int kb = wave == 1 ? 0 : h, ke = wave == 1 ? h : b;
          load_frags(b + 1, wave - 1, 0, b, av);
          load_g(b + 1, wave - 1, gv);
          load_frags(b + 1, 3, kb, ke, a3);
          if (wave == 1) load_g(b + 1, 3, gv3);
          strip_product(0, b, av, acc);
          add_strip(b + 1, cb ^ 1, wave - 1, acc, gv);
          v4i acc3[4] = {zero, zero, zero, zero};
          strip_product(kb, ke, a3, acc3);
          if (wave == 1) {
            add_strip(b + 1, cb ^ 1, 3, acc3, gv3);
          } else {
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
              for (int j = 0; j < 4; ++j) part[4 * (lane >> 4) + j][nt * 16 + (lane & 15)] = acc3[nt][j];
          }
        }
      }
    }
    lds_barrier();
    if (next) {
      if (wave != 0) {
#pragma unroll
        for (int i = 0; i < kCritPerHelper; ++i)
          if (i < crit_cnt) crit[crit_g0 + i][lane] = crit_next[i];
      }
      // block b's own flips, strip `wave` of block b+1
      v4i acc[4] = {zero, zero, zero, zero};
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const v4i bv = *reinterpret_cast<const v4i*>(&dsl[nt * 16 + (lane & 15)][b * kDB + 16 * (lane >> 4)]);
        acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a_next, bv, acc[nt], 0, 0, 0);
      }
      if (wave == 3) {
        // wave 2's part of strip 3
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[nt][j] += part[4 * (lane >> 4) + j][nt * 16 + (lane & 15)];
      }
      add_strip(b + 1, cb ^ 1, wave, acc, nullptr);
    }
    lds_barrier();
  }
  if (wave != 0) return;
  if (dE != 0)
    __hip_atomic_fetch_add((unsigned long long*)&E[r], (unsigned long long)dE, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  if (a.flip_ctr) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nflip += __shfl_xor(nflip, o, 64);
    if (lane == 0)
      __hip_atomic_fetch_add((unsigned long long*)&a.flip_ctr[tile & 255],
                             (unsigned long long)nflip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One super-block step: work-groups 0..T-1 run the sequential pass of this
// super-block (one per replica tile); with gemm_on the others compute the
// field product of the next super-block over every column except this
// super-block's own (which the pass is changing), into the other field
// buffer.  The two parts share no data, so the product runs on the compute
// units the pass leaves idle; the missing columns are added by a small
// product once the pass is done.
template <int RULE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_dense_step(SeqArgs a, GemmArgs g, int32_t sweep_idx, int32_t row0, int32_t rows, int32_t T, int32_t gemm_on) {
  __shared__ union {
    SeqLds seq;
    GemmLds gemm;
  } L;
  if ((int)blockIdx.x < T) {
    // fields beyond the LDS table need checking only when it is narrower
    // than the full one
    const int32_t Xt = (int32_t)a.st->table_x;
    if (a.j4) {
      if (Xt > kThrL)
        seq_body<RULE, true, true>(a, blockIdx.x, sweep_idx, row0, rows, L.seq);
      else
        seq_body<RULE, false, true>(a, blockIdx.x, sweep_idx, row0, rows, L.seq);
    } else {
      if (Xt > kThrL)
        seq_body<RULE, true, false>(a, blockIdx.x, sweep_idx, row0, rows, L.seq);
      else
        seq_body<RULE, false, false>(a, blockIdx.x, sweep_idx, row0, rows, L.seq);
    }
  }
  else if (gemm_on)
    gemm_body(g, blockIdx.x - T, L.gemm);
}

// Energy of the population from super-block fields: E_r += sum_k s_rk G_kr
// (the caller negates and halves at the end); clears G.  Work-group =
// (tile, 64-row block), wave 0 lanes = replicas.
__global__ void __launch_bounds__(64) k_dense_energy_sb(const int8_t* S, int32_t* G, int64_t* E, int32_t row0,
                                                        int32_t rows, int32_t n, int32_t np, int32_t R) {
  const int T = R / 64;
  const int tile = blockIdx.x % T, rb = blockIdx.x / T;
  const int r = tile * 64 + threadIdx.x;
  int64_t acc = 0;
  for (int k = 64 * rb; k < 64 * rb + 64 && row0 + k < n; ++k) {
    int32_t* gp = G + (size_t)k * R + r;
    acc += (int64_t)*gp * S[(size_t)r * np + row0 + k];
    *gp = 0;
  }
  if (acc)
    __hip_atomic_fetch_add((unsigned long long*)&E[r], (unsigned long long)acc, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_dense_init_finish(int64_t* E, int32_t R, RunState* st, int8_t* best, int32_t np) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < R) E[i] = -(E[i] / 2);
  for (int v = i; v < np; v += gridDim.x * blockDim.x) best[v] = 1;
  if (i == 0) {
    st->mstar = 0;
    st->cur = 0;
    st->gs = st->g_rs = st->g_cl = 0;
    st->stopped = 0;
    st->active = 0;
    st->steps_run = 0;
  }
}

// Energies of a population the host loaded into buffer 0: E = -E / 2 and
// buffer 0 becomes the current one.
__global__ void k_dense_load_finish(int64_t* E, int32_t R, RunState* st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < R) E[i] = -(E[i] / 2);
  if (i == 0) st->cur = 0;
}

// Resampling gather for the replica-major layout.
__global__ void __launch_bounds__(256) k_dense_gather(const RunState* st, int8_t* S0, int8_t* S1,
                                                      int64_t* E0, int64_t* E1, int32_t* F0, int32_t* F1,
                                                      const int32_t* parent, int32_t np, int32_t R) {
  if (!st->active || !st->do_resample) return;
  const int cur = st->cur;
  const uint32_t* Ss = reinterpret_cast<const uint32_t*>(cur ? S1 : S0);
  uint32_t* Sd = reinterpret_cast<uint32_t*>(cur ? S0 : S1);
  const int c = blockIdx.y;
  const int p = parent[c];
  const int words = np / 4;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x)
    Sd[(size_t)c * words + i] = Ss[(size_t)p * words + i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    (cur ? E0 : E1)[c] = (cur ? E1 : E0)[p];
    (cur ? F0 : F1)[c] = (cur ? F1 : F0)[p];
  }
}



// H[r][row0 + k] = G[k][r] for the super-block's rows (snapshots); clears G.
__global__ void __launch_bounds__(256) k_dense_collect_sb(int32_t* G, int32_t* H, int32_t row0, int32_t rows,
                                                          int32_t n, int32_t np, int32_t R) {
  const int64_t total = (int64_t)rows * R;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(i / R), r = (int)(i % R);
    if (row0 + k < n) H[(size_t)r * np + row0 + k] = G[i];
    G[i] = 0;
  }
}

}  // namespace


// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline uint32_t key0(const pamc_instance* I) { return (uint32_t)I->seed; }
static inline uint32_t key1(const pamc_instance* I) { return (uint32_t)(I->seed >> 32); }

hipError_t launch_dense_generate(pamc_instance* I, uint64_t graph_seed) {
  int64_t* W = I->flip_ctr + 400;
  hipMemsetAsync(W, 0, sizeof(int64_t), I->stream);
  const int64_t total = (int64_t)I->dn_pad * I->dn_pad;
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 1 << 16);
  k_dense_generate<<<grid, 256, 0, I->stream>>>(I->Jd, I->n, I->dn_pad, (uint32_t)graph_seed,
                                                (uint32_t)(graph_seed >> 32), W);
  return hipGetLastError();
}

// rows of the super-block starting at row0 (a multiple of 64)
static inline int sb_rows(const pamc_instance* I, int row0) { return std::min(kSB, I->dn_pad - row0); }

// K slices of the field product, each a multiple of the 64-column stage.
struct GemmShape {
  int grid, kslice;
};
// About 192 working work-groups: the K range is cut into P slices of whole
// stages; the grid covers the slices in groups of 8 (one per XCD;
// work-groups of slices past the end return at once).  The product shares
// the device with the sequential pass, and fewer, longer work-groups leave
// it more of the memory system: C3 sweeps timed at 128, 192, 256, 384, 512,
// 768 and 1,024 were fastest at 192.
static inline GemmShape gemm_shape(const pamc_instance* I, int rows, int kcount) {
  const int tiles = ((rows + kGM - 1) / kGM) * ((I->R + kGN - 1) / kGN);
  const int stages = std::max(1, kcount / kGK);
  // at least 4 stages per work-group: a short K range (the previous
  // super-block's columns, 16 stages) splits in 4 slices (timed against
  // 1, 2, 8 and 16 stages per work-group)
  const int P = std::max(1, std::min(stages / 4, (192 + tiles - 1) / tiles));
  const int kslice = ((stages + P - 1) / P) * kGK;
  const int slices = (kcount + kslice - 1) / kslice;
  return {tiles * ((slices + 7) / 8) * 8, kslice};
}

// Field product G = J[row0 .. row0 + rows) . S over the K domain (kbase,
// kcount, x0, xlen; see GemmArgs), and its grid.
struct GemmLaunch {
  GemmArgs g;
  int grid;
};
static GemmLaunch gemm_launch(const pamc_instance* I, int32_t row0, int32_t rows, int32_t use_state, int32_t* G,
                              int32_t kbase, int32_t kcount, int32_t x0, int32_t xlen) {
  const GemmShape gsh = gemm_shape(I, rows, kcount);
  GemmArgs g;
  g.J = I->Jd;
  g.S0 = I->Sd;
  g.S1 = I->Sd2;
  g.G = G;
  g.st = I->st;
  g.row0 = row0;
  g.rows = rows;
  g.np = I->dn_pad;
  g.R = I->R;
  g.use_state = use_state;
  g.kslice = gsh.kslice;
  g.kbase = kbase;
  g.kcount = kcount;
  g.x0 = x0;
  g.xlen = xlen;
  return {g, gsh.grid};
}
static GemmLaunch gemm_full(const pamc_instance* I, int32_t row0, int32_t rows, int32_t use_state, int32_t* G) {
  return gemm_launch(I, row0, rows, use_state, G, 0, I->dn_pad, I->dn_pad, 0);
}

static hipError_t dense_full_energy(pamc_instance* I, int buf) {
  const int T = I->R / 64;
  hipMemsetAsync(I->pop.E[buf], 0, sizeof(int64_t) * I->R, I->stream);
  for (int row0 = 0; row0 < I->n; row0 += kSB) {
    const int rows = sb_rows(I, row0);
    const GemmLaunch gl = gemm_full(I, row0, rows, 0, I->Gd);
    k_dense_gemm<<<gl.grid, 256, 0, I->stream>>>(gl.g);
    k_dense_energy_sb<<<T * (rows / 64), 64, 0, I->stream>>>(buf ? I->Sd2 : I->Sd, I->Gd, I->pop.E[buf], row0,
                                                             rows, I->n, I->dn_pad, I->R);
  }
  return hipGetLastError();
}

hipError_t launch_init_dense(pamc_instance* I) {
  const int64_t total = (int64_t)I->R * (I->dn_pad / 4);
  const int grid = (int)std::min<int64_t>((total + 255) / 256, 65535);
  k_dense_init_spins<<<grid, 256, 0, I->stream>>>(I->Sd, I->pop.fam[0], I->n, I->dn_pad, I->R, key0(I),
                                                  key1(I));
  dense_full_energy(I, 0);
  k_dense_init_finish<<<(std::max(I->R, I->dn_pad) + 255) / 256, 256, 0, I->stream>>>(
      I->pop.E[0], I->R, I->st, I->best, I->dn_pad);
  return hipGetLastError();
}

hipError_t launch_dense_load(pamc_instance* I) {
  dense_full_energy(I, 0);
  k_dense_load_finish<<<(I->R + 255) / 256, 256, 0, I->stream>>>(I->pop.E[0], I->R, I->st);
  return hipGetLastError();
}

// Sweeps of the dense path, super-block by super-block (rows row0_i ..).
// The field buffer alternates between two halves of Gd.  Each sweep starts
// with its critical fields (every visit's, one launch); super-block 0 of a
// sweep gets its full product first; then, for each super-block i, the
// launch that runs its sequential pass also computes the product of i+1
// over every column except i's, and a small product adds i's (now final)
// columns to i+1 before its pass.  With profiling, one event pair brackets
// each super-block step (the completing product and the pass with the
// overlapped product).
static hipError_t dense_sweeps(Batch& b, int32_t nsweeps) {
  pamc_instance* I = b.I[0];
  const int T = I->R / 64;
  SeqArgs a;
  a.J = I->Jd;
  a.S0 = I->Sd;
  a.S1 = I->Sd2;
  a.E0 = I->pop.E[0];
  a.E1 = I->pop.E[1];
  a.thr = I->thr;
  a.C = reinterpret_cast<const v4i*>(I->Cd);
  a.st = I->st;
  a.n = I->n;
  a.np = I->dn_pad;
  a.R = I->R;
  a.j4 = I->dense_j4;
  a.k0 = key0(I);
  a.k1 = key1(I);
  a.flip_ctr = I->prof ? I->flip_ctr : nullptr;
  auto gbuf = [&](int i) { return I->Gd + (size_t)(i & 1) * kSB * I->R; };
  const int nsb = (I->n + kSB - 1) / kSB;
  ctl_thresholds(b);
  for (int s = 0; s < nsweeps; ++s) {
    for (int i = 0; i < nsb; ++i) {
      const int row0 = i * kSB, rows = sb_rows(I, row0);
      hipEvent_t e0 = nullptr;
      if (I->prof) {
        e0 = ctl_event(I);
        hipEventRecord(e0, I->stream);
      }
      if (i == 0) {
        // the sweep's critical fields, then super-block 0's full product
        const int64_t items = (int64_t)(I->dn_pad / 4) * I->R;
        const int cgrid = (int)std::min<int64_t>((items + 255) / 256, 2048);
        v4i* C = reinterpret_cast<v4i*>(I->Cd);
        if (I->rule == 1)
          k_dense_crit<1><<<cgrid, 256, 0, I->stream>>>(I->thr, I->st, C, s, I->dn_pad / 4, I->R, a.k0, a.k1);
        else
          k_dense_crit<0><<<cgrid, 256, 0, I->stream>>>(I->thr, I->st, C, s, I->dn_pad / 4, I->R, a.k0, a.k1);
        const GemmLaunch gl = gemm_full(I, row0, rows, 1, gbuf(0));
        k_dense_gemm<<<gl.grid, 256, 0, I->stream>>>(gl.g);
      } else {
        // the previous super-block's columns, final now
        const int p0 = row0 - kSB;
        const GemmLaunch gl = gemm_launch(I, row0, rows, 1, gbuf(i), p0, sb_rows(I, p0), 0, 0);
        k_dense_gemm<<<gl.grid, 256, 0, I->stream>>>(gl.g);
      }
      a.G = gbuf(i);
      const bool next = i + 1 < nsb;
      GemmLaunch nx{};
      if (next) {
        const int n0 = row0 + kSB;
        nx = gemm_launch(I, n0, sb_rows(I, n0), 1, gbuf(i + 1), 0, I->dn_pad - rows, row0, rows);
      }
      const int grid = T + (next ? nx.grid : 0);
      if (I->rule == 1)
        k_dense_step<1><<<grid, 256, 0, I->stream>>>(a, nx.g, s, row0, rows, T, next ? 1 : 0);
      else
        k_dense_step<0><<<grid, 256, 0, I->stream>>>(a, nx.g, s, row0, rows, T, next ? 1 : 0);
      if (I->prof) {
        hipEvent_t e1 = ctl_event(I);
        hipEventRecord(e1, I->stream);
        I->prof_launches += 1;
      }
    }
    if (I->prof) I->prof_attempts += (int64_t)I->n * I->R;
  }
  return hipGetLastError();
}

static void dense_gather(pamc_instance* I) {
  k_dense_gather<<<dim3(std::max(1, std::min(64, I->dn_pad / 1024)), I->R), 256, 0, I->stream>>>(
      I->st, I->Sd, I->Sd2, I->pop.E[0], I->pop.E[1], I->pop.fam[0], I->pop.fam[1], I->rs_parent,
      I->dn_pad, I->R);
}

hipError_t launch_dense_step(Batch& b, int32_t sweeps, int32_t resample) {
  pamc_instance* I = b.I[0];
  ctl_step_begin(b);
  if (resample) {
    ctl_resample_select(b);
    dense_gather(I);
  }
  ctl_commit(b, 1);
  hipError_t e = dense_sweeps(b, sweeps);
  if (e != hipSuccess) return e;
  ctl_step_end(b, 1);
  return hipGetLastError();
}

hipError_t launch_dense_prim_sweep(Batch& b, double beta, int32_t nsweeps) {
  ctl_prim_set(b, 0, beta, nsweeps);
  hipError_t e = dense_sweeps(b, nsweeps);
  if (e != hipSuccess) return e;
  ctl_advance(b, nsweeps);
  return hipGetLastError();
}

hipError_t launch_dense_prim_resample(Batch& b, double delta) {
  ctl_prim_set(b, 1, delta, 0);
  ctl_resample_select(b);
  dense_gather(b.I[0]);
  ctl_commit(b, 0);
  ctl_deactivate(b);
  return hipGetLastError();
}

hipError_t launch_dense_prim_update_best(Batch& b) {
  ctl_prim_set(b, 0, 0.0, 0);
  ctl_step_end(b, 0);
  ctl_deactivate(b);
  return hipGetLastError();
}

hipError_t launch_dense_fields(pamc_instance* I, int32_t* H_rmajor) {
  // fields H[r][v] (replica-major) of the current population, for snapshots
  for (int row0 = 0; row0 < I->n; row0 += kSB) {
    const int rows = sb_rows(I, row0);
    const GemmLaunch gl = gemm_full(I, row0, rows, 2, I->Gd);
    k_dense_gemm<<<gl.grid, 256, 0, I->stream>>>(gl.g);
    k_dense_collect_sb<<<std::min(1024, (rows * I->R + 255) / 256), 256, 0, I->stream>>>(
        I->Gd, H_rmajor, row0, rows, I->n, I->dn_pad, I->R);
  }
  return hipGetLastError();
}

int32_t dense_superblock_rows() { return kSB; }
int32_t dense_field_buffers() { return 2; }

}  // namespace pamc
