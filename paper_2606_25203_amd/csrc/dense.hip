// dense.hip -- fully connected instances (Sec. "Scalability on a Large-Scale
// Ising Problem"): int8 couplings J[n][n] in HBM, spins visited in the fixed
// order 0..n-1.
//
// A sweep runs over super-blocks of kSB = 1024 consecutive spins.  For each,
// one matrix-core launch computes the local fields of Eq. 3 of all its rows
// against the spins as they stand, G = J[sb, :] . S (int8 x int8 -> int32,
// exact since |h| <= 127 n < 2^31; split over the K dimension and summed
// atomically).  A sequential launch (one work-group per 64 replicas) then
// walks the super-block in blocks of kDB = 64 spins: the couplings to spins
// already flipped in earlier blocks of the super-block are added with a
// small matrix-core product over the recorded changes dS, and the block's
// spins are decided in order with h_k = G_k + C_k + sum_{k' < k in block}
// J_kk' d_k' (d = 2 s_new for flipped spins, packed int8, dot4), the same
// threshold test as the sparse path.
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
constexpr int kSB = 2048;        // rows per super-block: one field product, one sequential launch
constexpr int kGM = 128, kGN = 128, kGK = 64;  // field-product tile: rows x replicas x K stage
constexpr int kLdsRow = kGK + 16;              // bytes per staged row (padded)
constexpr int kThrL = 4095;      // half-width of the LDS copy of the threshold table
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
__global__ void __launch_bounds__(256) k_dense_gemm(const int8_t* __restrict__ J,
                                                    const int8_t* __restrict__ S0,
                                                    const int8_t* __restrict__ S1,
                                                    int32_t* __restrict__ G, const RunState* st,
                                                    int32_t row0, int32_t rows, int32_t np, int32_t R,
                                                    int32_t use_state, int32_t kslice) {
  __shared__ __attribute__((aligned(16))) int8_t As[2][kGM * kLdsRow];
  __shared__ __attribute__((aligned(16))) int8_t Bs[2][kGN * kLdsRow];
  if (use_state == 1 && !st->active) return;
  const int8_t* __restrict__ S = (use_state ? st->cur : 0) ? S1 : S0;
  const int MT = (rows + kGM - 1) / kGM, NT = (R + kGN - 1) / kGN;
  int g = blockIdx.x;
  const int mt = g % MT;
  g /= MT;
  const int ntile = g % NT;
  const int p = g / NT;
  const int k_beg = p * kslice, k_end = min(np, k_beg + kslice);
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
  v4i ra[2], rb[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    ra[i] = *reinterpret_cast<const v4i*>(ag[i] + k_beg);
    rb[i] = *reinterpret_cast<const v4i*>(bg[i] + k_beg);
    *reinterpret_cast<v4i*>(As[0] + lofs[i]) = ra[i];
    *reinterpret_cast<v4i*>(Bs[0] + lofs[i]) = rb[i];
  }
  __syncthreads();
  v4i acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = zero;
  const int frag = (lane & 15) * kLdsRow + 16 * (lane >> 4);
  int buf = 0;
  for (int k0 = k_beg; k0 < k_end; k0 += kGK) {
    const bool more = k0 + kGK < k_end;
    if (more) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ra[i] = *reinterpret_cast<const v4i*>(ag[i] + k0 + kGK);
        rb[i] = *reinterpret_cast<const v4i*>(bg[i] + k0 + kGK);
      }
    }
    v4i af[4], bf[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      af[i] = *reinterpret_cast<const v4i*>(As[buf] + (wm * 64 + 16 * i) * kLdsRow + frag);
      bf[i] = *reinterpret_cast<const v4i*>(Bs[buf] + (wn * 64 + 16 * i) * kLdsRow + frag);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(af[i], bf[j], acc[i][j], 0, 0, 0);
    if (more) {
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        *reinterpret_cast<v4i*>(As[buf ^ 1] + lofs[i]) = ra[i];
        *reinterpret_cast<v4i*>(Bs[buf ^ 1] + lofs[i]) = rb[i];
      }
    }
    __syncthreads();
    buf ^= 1;
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

// Sequential visit of one super-block's spins for one 64-replica tile.
struct SeqArgs {
  const int8_t* J;
  int8_t* S0;
  int8_t* S1;
  int8_t* dS;   // [R][np]: 2 s_new where a spin flipped in this super-block, else 0
  int64_t* E0;
  int64_t* E1;
  int32_t* G;   // [kSB][R] fields of the super-block rows against its starting spins
  const uint32_t* thr;
  RunState* st;
  int32_t n, np, R;
  uint32_t k0, k1;
  int64_t* flip_ctr;
};

// One work-group per tile walks the super-block's 64-spin blocks in order.
// For block b, the four waves first add to G the couplings to the spins that
// flipped in the earlier blocks of the super-block, C = J[blk, row0 ..
// row0 + 64b) . dS (matrix cores; dS read past the L1 with coherent buffer
// loads, since this work-group wrote it), then wave 0 (lane = replica)
// decides the block's spins in order with the in-block corrections
// h_k = G_k + C_k + sum_{k' < k in block} J_kk' d_k' (d packed int8, dot4),
// and records d in dS.
template <int RULE>
__global__ void __launch_bounds__(256) k_dense_seq(SeqArgs a, int32_t sweep_idx, int32_t row0, int32_t rows) {
  __shared__ uint32_t jd[kDB][kDB / 4];  // J[rb0 + k][rb0 + 4g .. 4g+3], packed int8
  __shared__ int32_t gsum[kDB][64];      // fields of this tile before the block's own flips
  __shared__ uint32_t thr_s[2 * kThrL + 1];  // thresholds for |x| <= Xl
  RunState* st = a.st;
  if (!st->active) return;
  const int cur = st->cur;
  int8_t* S = cur ? a.S1 : a.S0;
  int64_t* E = cur ? a.E1 : a.E0;
  const int tile = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int r = tile * 64 + lane;
  const uint32_t gs = st->gs + (uint32_t)sweep_idx;
  const int32_t Xt = (int32_t)st->table_x;
  // The decision chain waits for every threshold read, so the central part
  // of the table lives in LDS; |x| > Xl (beyond about 13 standard deviations
  // of the field at n = 100,000) reads global memory.
  const int32_t Xl = min(Xt, kThrL);
  for (int i = threadIdx.x; i <= 2 * Xl; i += blockDim.x) thr_s[i] = a.thr[Xt - Xl + i];
  const __amdgpu_buffer_rsrc_t dsr =
      __builtin_amdgcn_make_buffer_rsrc((void*)(a.dS + (size_t)tile * 64 * a.np), (short)0, 64 * a.np, 0x00020000);
  int64_t dE = 0;
  int32_t nflip = 0;
  for (int b = 0; b * kDB < rows; ++b) {
    const int rb0 = row0 + b * kDB;
    if (rb0 >= a.n) break;
    // corrections from the earlier blocks of the super-block
    v4i acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    const int8_t* arow = a.J + (size_t)(rb0 + 16 * wave + (lane & 15)) * a.np + row0 + 16 * (lane >> 4);
    const int boff = (lane & 15) * a.np + row0 + 16 * (lane >> 4);
    for (int k0 = 0; k0 < b * kDB; k0 += 64) {
      const v4i av = *reinterpret_cast<const v4i*>(arow + k0);
      v4i bv[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        bv[nt] = __builtin_bit_cast(v4i, __builtin_amdgcn_raw_buffer_load_b128(dsr, boff + nt * 16 * a.np + k0, 0, 1));
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) acc[nt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(av, bv[nt], acc[nt], 0, 0, 0);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = 16 * wave + 4 * (lane >> 4) + j, c = nt * 16 + (lane & 15);
        int32_t* gp = a.G + (size_t)(b * kDB + m) * a.R + tile * 64 + c;
        gsum[m][c] = acc[nt][j] + *gp;
        *gp = 0;  // cleared for the next super-block's accumulation
      }
    for (int i = threadIdx.x; i < kDB * kDB / 4; i += blockDim.x) {
      const int k = i / (kDB / 4), g = i % (kDB / 4);
      jd[k][g] = *reinterpret_cast<const uint32_t*>(a.J + (size_t)(rb0 + k) * a.np + rb0 + 4 * g);
    }
    __syncthreads();
    if (wave == 0) {
      uint32_t d[kDB / 4];  // packed int8 d_k' of this lane's replica
#pragma unroll
      for (int g = 0; g < kDB / 4; ++g) d[g] = 0;
      uint32_t* srow = reinterpret_cast<uint32_t*>(S + (size_t)r * a.np + rb0);
#pragma unroll
      for (int g = 0; g < kDB / 4; ++g) {
        const int vq = rb0 + 4 * g;
        if (vq >= a.n) break;
        const u32x4 rnd = philox10((uint32_t)(vq >> 2), gs, (uint32_t)r, kTagSweep, a.k0, a.k1);
        uint32_t sw = srow[g];
        uint32_t dg = 0;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 4 * g + kk;
          if (rb0 + k >= a.n) break;
          int32_t h = gsum[k][lane];
#pragma unroll
          for (int g2 = 0; g2 < g; ++g2) h = __builtin_amdgcn_sdot4((int)jd[k][g2], (int)d[g2], h, false);
          h = __builtin_amdgcn_sdot4((int)jd[k][g], (int)dg, h, false);
          const int32_t s = (int32_t)(int8_t)(sw >> (8 * kk));
          const int32_t x = s * h;
          const int32_t xl = min(max(x, -Xl), Xl);
          uint32_t T = thr_s[xl + Xl];
          if (x != xl && Xl < Xt) T = a.thr[min(max(x, -Xt), Xt) + Xt];
          const bool flip = (RULE == 1 && x <= 0) || (pick(rnd, kk) < T);
          if (flip) {
            dE += 2 * (int64_t)x;
            sw ^= (0xFEu << (8 * kk));
            dg |= (uint32_t)(uint8_t)(int8_t)(-2 * s) << (8 * kk);
            ++nflip;
          }
        }
        d[g] = dg;
        srow[g] = sw;
      }
      uint32_t* drow = reinterpret_cast<uint32_t*>(a.dS + (size_t)r * a.np + rb0);
#pragma unroll
      for (int g = 0; g < kDB / 4; ++g) drow[g] = d[g];
    }
    __syncthreads();  // dS of this block is read by the next block's corrections
  }
  if (wave != 0) return;
  if (dE != 0)
    __hip_atomic_fetch_add((unsigned long long*)&E[r], (unsigned long long)dE, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  if (a.flip_ctr) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nflip += __shfl_xor(nflip, o, 64);
    if (lane == 0)
      __hip_atomic_fetch_add((unsigned long long*)&a.flip_ctr[blockIdx.x & 255],
                             (unsigned long long)nflip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
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

// K slices of the field product: enough work-groups for two per compute
// unit, each slice a multiple of the 64-column stage.
struct GemmShape {
  int grid, kslice;
};
static inline GemmShape gemm_shape(const pamc_instance* I, int rows) {
  const int tiles = ((rows + kGM - 1) / kGM) * ((I->R + kGN - 1) / kGN);
  const int stages = I->dn_pad / kGK;
  const int P = std::max(1, std::min(stages, (512 + tiles - 1) / tiles));
  const int kslice = ((stages + P - 1) / P) * kGK;
  return {tiles * ((I->dn_pad + kslice - 1) / kslice), kslice};
}

static hipError_t dense_full_energy(pamc_instance* I, int buf) {
  const int T = I->R / 64;
  hipMemsetAsync(I->pop.E[buf], 0, sizeof(int64_t) * I->R, I->stream);
  for (int row0 = 0; row0 < I->n; row0 += kSB) {
    const int rows = sb_rows(I, row0);
    const GemmShape gsh = gemm_shape(I, rows);
    k_dense_gemm<<<gsh.grid, 256, 0, I->stream>>>(I->Jd, I->Sd, I->Sd2, I->Gd, I->st, row0, rows, I->dn_pad, I->R,
                                                  0, gsh.kslice);
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

static hipError_t dense_sweeps(Batch& b, int32_t nsweeps) {
  pamc_instance* I = b.I[0];
  const int T = I->R / 64;
  SeqArgs a;
  a.J = I->Jd;
  a.S0 = I->Sd;
  a.S1 = I->Sd2;
  a.dS = I->Dd;
  a.E0 = I->pop.E[0];
  a.E1 = I->pop.E[1];
  a.G = I->Gd;
  a.thr = I->thr;
  a.st = I->st;
  a.n = I->n;
  a.np = I->dn_pad;
  a.R = I->R;
  a.k0 = key0(I);
  a.k1 = key1(I);
  a.flip_ctr = I->prof ? I->flip_ctr : nullptr;
  ctl_thresholds(b);
  for (int s = 0; s < nsweeps; ++s) {
    for (int row0 = 0; row0 < I->n; row0 += kSB) {
      const int rows = sb_rows(I, row0);
      hipEvent_t e0 = nullptr;
      if (I->prof) {
        e0 = ctl_event(I);
        hipEventRecord(e0, I->stream);
      }
      const GemmShape gsh = gemm_shape(I, rows);
      k_dense_gemm<<<gsh.grid, 256, 0, I->stream>>>(I->Jd, I->Sd, I->Sd2, I->Gd, I->st, row0, rows, I->dn_pad,
                                                    I->R, 1, gsh.kslice);
      if (I->prof) {
        hipEvent_t e1 = ctl_event(I);
        hipEventRecord(e1, I->stream);
        I->prof_launches += 1;
      }
      if (I->rule == 1)
        k_dense_seq<1><<<T, 256, 0, I->stream>>>(a, s, row0, rows);
      else
        k_dense_seq<0><<<T, 256, 0, I->stream>>>(a, s, row0, rows);
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
    const GemmShape gsh = gemm_shape(I, rows);
    k_dense_gemm<<<gsh.grid, 256, 0, I->stream>>>(I->Jd, I->Sd, I->Sd2, I->Gd, I->st, row0, rows, I->dn_pad, I->R,
                                                  2, gsh.kslice);
    k_dense_collect_sb<<<std::min(1024, (rows * I->R + 255) / 256), 256, 0, I->stream>>>(
        I->Gd, H_rmajor, row0, rows, I->n, I->dn_pad, I->R);
  }
  return hipGetLastError();
}

int32_t dense_superblock_rows() { return kSB; }

}  // namespace pamc
