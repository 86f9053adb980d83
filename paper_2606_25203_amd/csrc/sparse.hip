// sparse.hip -- gfx950 kernels of the sparse PAMC path and of the
// device-side controller (Algorithm 1), with their host launchers.
//
// One β step of Algorithm 1 is a fixed sequence of launches whose behaviour
// is decided on the device from RunState, so the host never waits inside a
// run:
//   step_begin -> rs_select -> rs_gather -> cl_select -> cl_mis -> cl_apply
//   -> commit -> thresholds -> S x K sweep phases -> step_end
// Kernels that have nothing to do in a step return at once.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "instance.hpp"
#include "pamc_device.hpp"

namespace pamc {

namespace {

constexpr int kSweepWaves = 4;             // waves per sweep workgroup
constexpr int kQuadsPerWave = 4;           // quads per wave per workgroup
constexpr int kQuadsPerBlock = kSweepWaves * kQuadsPerWave;
constexpr int kGatherQuadsPerBlock = 64;
constexpr int kClusterMaxN = 26000;        // LDS: 5 bytes per vertex
constexpr int kRsMaxR = 16384;

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int32_t spin_at(const uint32_t* S, int nq, int tile, int v, int lane) {
  const uint32_t w = S[((size_t)tile * nq + (v >> 2)) * kLanes + lane];
  return (int32_t)(int8_t)(w >> (8 * (v & 3)));
}

// blockIdx -> (tile, chunk).  Work-groups are dealt round-robin to the eight
// XCDs, so tile t is kept on XCD t % 8 when T is a multiple of 8: all field
// atomics of a tile then meet in one L2.
__device__ __forceinline__ void tile_chunk(int T, int& tile, int& chunk) {
  const int b = blockIdx.x;
  if ((T & 7) == 0) {
    const int xcd = b & 7, j = b >> 3, tp = T >> 3;
    tile = (j % tp) * 8 + xcd;
    chunk = j / tp;
  } else {
    tile = b % T;
    chunk = b / T;
  }
}


// Field of Eq. 3 for vertex v of replica lane `lane` of a tile, gathered
// from the neighbours' spin words.  Neighbours are taken four at a time with
// unconditional loads (the CSR arrays carry kCsrPad trailing entries, and an
// entry past the row is a valid vertex id), and the couplings of entries past
// the row are masked to zero, so the loop body has no per-entry branches.
// Srow points at the tile's spin words + lane.
constexpr int kCsrPad = 8;
template <bool SMALLJ>
__device__ __forceinline__ int32_t gather_field(const int32_t* __restrict__ col,
                                                const int32_t* __restrict__ J, int e0, int e1,
                                                const uint32_t* __restrict__ Srow) {
  int32_t h = 0;
  for (int e = e0; e < e1; e += 4) {
    const int cnt = e1 - e;
    int j[4];
    int32_t c[4];
    uint32_t w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      j[u] = col[e + u];
      c[u] = J[e + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = Srow[(uint32_t)(j[u] >> 2) * (uint32_t)kLanes];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t cu = u < cnt ? c[u] : 0;
      const int32_t sv = __builtin_amdgcn_sbfe((int32_t)w[u], 8u * (uint32_t)(j[u] & 3), 8u);
      // couplings below 2^23 in magnitude use the full-rate 24-bit multiply
      h += SMALLJ ? __mul24(cu, sv) : cu * sv;
    }
  }
  return h;
}

constexpr int kThrLds = 2048;  // threshold entries staged in LDS when they fit

struct SweepArgs {
  const int32_t* row_ptr;
  const int32_t* col;
  const int32_t* J;
  const int32_t* class_ptr;
  const int32_t* order;
  uint32_t* S0;
  uint32_t* S1;
  int32_t* H0;
  int32_t* H1;
  int64_t* E0;
  int64_t* E1;
  const uint32_t* thr;
  RunState* st;
  int64_t* flip_ctr;
  int32_t nq, np, T, ncls;
  uint32_t k0, k1;
};

// ---------------------------------------------------------------------------
// One colour class of one sweep (Eqs. 3-4).  Work-group = (replica tile,
// chunk of the class's vertex quads); wave = up to 4 quads; lane = replica.
// For each vertex: x = s*h, u = Philox word (quad, sweep, replica), flip iff
// u < T[x] (Metropolis also for x <= 0); on a flip E += 2x and every
// neighbour field gets 2 J s_new by a coalesced no-return atomic.  Vertices of
// a class are mutually uncoupled, so no field read here is written here.
// ---------------------------------------------------------------------------
template <int RULE>
__global__ void __launch_bounds__(256) k_sweep(const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ Jc,
                                                  const int32_t* __restrict__ class_ptr,
                                                  const int32_t* __restrict__ order,
                                                  const uint32_t* __restrict__ thr_g, SweepArgs a,
                                                  int sweep_idx, int phase) {
  __shared__ int64_t red[kSweepWaves][kLanes];
  __shared__ int32_t fred[kSweepWaves];
  __shared__ uint32_t thr_s[kThrLds];
  RunState* st = a.st;
  if (!st->active) return;
  const int cur = st->cur;
  uint32_t* __restrict__ S = cur ? a.S1 : a.S0;
  int32_t* __restrict__ H = cur ? a.H1 : a.H0;
  int64_t* __restrict__ E = cur ? a.E1 : a.E0;
  const int cls = order[sweep_idx * a.ncls + phase];
  const int v0 = class_ptr[cls], v1 = class_ptr[cls + 1];
  const int q0 = v0 >> 2;
  const int nqc = ((v1 + 3) >> 2) - q0;
  int tile, chunk;
  tile_chunk(a.T, tile, chunk);
  if (chunk * kQuadsPerBlock >= nqc) return;
  const uint32_t gs = st->gs + (uint32_t)sweep_idx;
  const int32_t Xt = (int32_t)st->table_x;
  const bool thr_lds = 2 * Xt + 1 <= kThrLds;
  if (thr_lds)
    for (int i = threadIdx.x; i <= 2 * Xt; i += blockDim.x) thr_s[i] = thr_g[i];
  __syncthreads();
  const uint32_t* __restrict__ thr = thr_lds ? thr_s : a.thr;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t r = (uint32_t)(tile * kLanes + lane);
  const size_t hbase = (size_t)tile * a.np;
  int64_t dE = 0;
  int32_t nflip = 0;
  for (int i = 0; i < kQuadsPerWave; ++i) {
    const int qi = chunk * kQuadsPerBlock + i * kSweepWaves + wave;
    if (qi >= nqc) break;
    const int q = q0 + qi;
    const size_t sidx = ((size_t)tile * a.nq + q) * kLanes + lane;
    uint32_t sw = S[sidx];
    const u32x4 rnd = philox10((uint32_t)q, gs, r, kTagSweep, a.k0, a.k1);
    bool dirty = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int v = 4 * q + k;
      if (v < v0 || v >= v1) continue;
      const int32_t h = H[(hbase + v) * kLanes + lane];
      const int32_t s = (int32_t)(int8_t)(sw >> (8 * k));
      const int32_t x = s * h;
      const int32_t xi = x < -Xt ? -Xt : (x > Xt ? Xt : x);
      const uint32_t T = thr[xi + Xt];
      const bool flip = (RULE == 1 && x <= 0) || (pick(rnd, k) < T);
      const int32_t snew = -s;
      if (flip) {
        dE += 2 * (int64_t)x;
        sw = (sw & ~(0xFFu << (8 * k))) | ((uint32_t)(uint8_t)(int8_t)snew << (8 * k));
        dirty = true;
        ++nflip;
      }
      if (__ballot(flip)) {
        const int e0 = row_ptr[v], e1 = row_ptr[v + 1];
        const int32_t d = 2 * snew;
        for (int e = e0; e < e1; ++e) {
          const int j = col[e];
          const int32_t add = Jc[e] * d;
          if (flip)
            __hip_atomic_fetch_add(&H[(hbase + j) * kLanes + lane], add, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    if (dirty) S[sidx] = sw;
  }
  red[wave][lane] = dE;
  int32_t wf = 0;
  if (a.flip_ctr) {
    wf = nflip;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wf += __shfl_xor(wf, o, 64);
    if (lane == 0) fred[wave] = wf;
  }
  __syncthreads();
  if (wave == 0) {
    int64_t t = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
    if (t != 0)
      __hip_atomic_fetch_add((unsigned long long*)&E[r], (unsigned long long)t, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    if (a.flip_ctr && lane == 0) {
      int64_t f = (int64_t)fred[0] + fred[1] + fred[2] + fred[3];
      __hip_atomic_fetch_add((unsigned long long*)&a.flip_ctr[blockIdx.x & 255],
                             (unsigned long long)f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// Same class phase with the local field of Eq. 3 gathered at visit time from
// the neighbours' spins instead of being kept in a field array.  The integer
// h and hence every decision are identical to the incremental form; what
// changes is the memory traffic: no field array and no atomics, only spin
// words (one byte per replica and vertex), which suits low-degree graphs.
// ---------------------------------------------------------------------------
// Fields of one vertex for TPW tiles at once: the scalar work (CSR entries,
// neighbour offsets, coupling masks) is shared by the tiles, the spin loads
// and arithmetic are per tile.  Srow0 points at the first tile's spin words
// + lane; tiles are tstride words apart.
template <bool SMALLJ, int TPW>
__device__ __forceinline__ void gather_fields(const int32_t* __restrict__ col,
                                              const int32_t* __restrict__ J, int e0, int e1,
                                              const uint32_t* __restrict__ Srow0, uint32_t tstride,
                                              int32_t (&h)[TPW]) {
#pragma unroll
  for (int t = 0; t < TPW; ++t) h[t] = 0;
  for (int e = e0; e < e1; e += 4) {
    const int cnt = e1 - e;
    int j[4];
    int32_t c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      j[u] = col[e + u];
      c[u] = u < cnt ? J[e + u] : 0;
    }
    uint32_t w[TPW][4];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        w[t][u] = Srow0[(uint32_t)t * tstride + (uint32_t)(j[u] >> 2) * (uint32_t)kLanes];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int32_t sv = __builtin_amdgcn_sbfe((int32_t)w[t][u], 8u * (uint32_t)(j[u] & 3), 8u);
        h[t] += SMALLJ ? __mul24(c[u], sv) : c[u] * sv;
      }
  }
}

template <int RULE, bool SMALLJ, int TPW>
__global__ void __launch_bounds__(256) k_sweep_pull(const int32_t* __restrict__ row_ptr,
                                                  const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ Jc,
                                                  const int32_t* __restrict__ class_ptr,
                                                  const int32_t* __restrict__ order,
                                                  const uint32_t* __restrict__ thr_g, SweepArgs a,
                                                  int sweep_idx, int phase) {
  __shared__ int64_t red[kSweepWaves][TPW][kLanes];
  __shared__ int32_t fred[kSweepWaves];
  __shared__ uint32_t thr_s[kThrLds];
  RunState* st = a.st;
  if (!st->active) return;
  const int cur = st->cur;
  uint32_t* __restrict__ S = cur ? a.S1 : a.S0;
  int64_t* __restrict__ E = cur ? a.E1 : a.E0;
  const int cls = order[sweep_idx * a.ncls + phase];
  const int v0 = class_ptr[cls], v1 = class_ptr[cls + 1];
  const int q0 = v0 >> 2;
  const int nqc = ((v1 + 3) >> 2) - q0;
  int group, chunk;
  tile_chunk(a.T / TPW, group, chunk);
  if (chunk * kQuadsPerBlock >= nqc) return;
  const uint32_t gs = st->gs + (uint32_t)sweep_idx;
  const int32_t Xt = (int32_t)st->table_x;
  const bool thr_lds = 2 * Xt + 1 <= kThrLds;
  if (thr_lds)
    for (int i = threadIdx.x; i <= 2 * Xt; i += blockDim.x) thr_s[i] = thr_g[i];
  __syncthreads();
  const uint32_t* __restrict__ thr = thr_lds ? thr_s : thr_g;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile0 = group * TPW;
  const uint32_t tstride = (uint32_t)a.nq * kLanes;
  uint32_t* __restrict__ Srow0 = S + (size_t)tile0 * tstride + lane;
  int64_t dE[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) dE[t] = 0;
  int32_t nflip = 0;
  for (int i = 0; i < kQuadsPerWave; ++i) {
    const int qi = chunk * kQuadsPerBlock + i * kSweepWaves + wave;
    if (qi >= nqc) break;
    const int q = q0 + qi;
    uint32_t sw[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) sw[t] = Srow0[(uint32_t)t * tstride + (uint32_t)q * kLanes];
    int32_t h[4][TPW];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int v = 4 * q + k;
      if (v >= v0 && v < v1) {
        gather_fields<SMALLJ, TPW>(col, Jc, row_ptr[v], row_ptr[v + 1], Srow0, tstride, h[k]);
      } else {
#pragma unroll
        for (int t = 0; t < TPW; ++t) h[k][t] = 0;
      }
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const uint32_t r = (uint32_t)((tile0 + t) * kLanes + lane);
      const u32x4 rnd = philox10((uint32_t)q, gs, r, kTagSweep, a.k0, a.k1);
      bool dirty = false;
      uint32_t swt = sw[t];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int v = 4 * q + k;
        if (v < v0 || v >= v1) continue;
        const int32_t s = (int32_t)(int8_t)(swt >> (8 * k));
        const int32_t x = s * h[k][t];
        const int32_t xi = x < -Xt ? -Xt : (x > Xt ? Xt : x);
        const uint32_t T = thr[xi + Xt];
        const bool flip = (RULE == 1 && x <= 0) || (pick(rnd, k) < T);
        if (flip) {
          dE[t] += 2 * (int64_t)x;
          swt ^= (0xFEu << (8 * k));  // +1 (0x01) <-> -1 (0xFF)
          dirty = true;
          ++nflip;
        }
      }
      if (dirty) Srow0[(uint32_t)t * tstride + (uint32_t)q * kLanes] = swt;
    }
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) red[wave][t][lane] = dE[t];
  if (a.flip_ctr) {
    int32_t wf = nflip;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wf += __shfl_xor(wf, o, 64);
    if (lane == 0) fred[wave] = wf;
  }
  __syncthreads();
  if (wave < TPW) {
    const int t = wave;
    const int64_t sum = red[0][t][lane] + red[1][t][lane] + red[2][t][lane] + red[3][t][lane];
    if (sum != 0)
      __hip_atomic_fetch_add((unsigned long long*)&E[(tile0 + t) * kLanes + lane],
                             (unsigned long long)sum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (a.flip_ctr && threadIdx.x == 0) {
    const int64_t f = (int64_t)fred[0] + fred[1] + fred[2] + fred[3];
    __hip_atomic_fetch_add((unsigned long long*)&a.flip_ctr[blockIdx.x & 255], (unsigned long long)f,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// Population initialisation (Algorithm 1, initialization): spins uniform from
// Philox(quad, 0, replica, INIT) (spin +1 iff the word < 2^31); then local
// fields by Eq. 3 and energies H = -1/2 sum s h.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_init_spins(uint32_t* S, int32_t* fam, int32_t n, int32_t nq,
                                                    int32_t T, uint32_t k0, uint32_t k1) {
  const size_t total = (size_t)T * nq * kLanes;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const int lane = (int)(i & 63);
    const size_t tq = i >> 6;
    const int q = (int)(tq % nq);
    const int tile = (int)(tq / nq);
    const uint32_t r = (uint32_t)(tile * kLanes + lane);
    const u32x4 w = philox10((uint32_t)q, 0u, r, kTagInit, k0, k1);
    uint32_t sw = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int v = 4 * q + k;
      int8_t s = 0;
      if (v < n) s = pick(w, k) < 0x80000000u ? (int8_t)1 : (int8_t)-1;
      sw |= (uint32_t)(uint8_t)s << (8 * k);
    }
    S[i] = sw;
    if (q == 0) fam[r] = (int32_t)r;
  }
}

// h = J s per (tile, vertex) row; accumulates -s h / 2 into E.
__global__ void __launch_bounds__(256) k_init_fields(const int32_t* row_ptr, const int32_t* col,
                                                     const int32_t* J, const uint32_t* S, int32_t* H,
                                                     int64_t* E, int32_t n, int32_t np, int32_t nq,
                                                     int32_t T) {
  __shared__ int64_t red[4][kLanes];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tile = blockIdx.x % T;
  const int vchunk = blockIdx.x / T;
  int64_t acc = 0;
  for (int v = vchunk * 64 + wave; v < n && v < (vchunk + 1) * 64; v += 4) {
    int64_t h = 0;
    for (int e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
      h += (int64_t)J[e] * spin_at(S, nq, tile, col[e], lane);
    if (H) H[((size_t)tile * np + v) * kLanes + lane] = (int32_t)h;
    acc += h * spin_at(S, nq, tile, v, lane);
  }
  red[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && E) {
    const int64_t t = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
    if (t != 0)
      __hip_atomic_fetch_add((unsigned long long*)&E[tile * kLanes + lane],
                             (unsigned long long)t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// E currently holds sum_v s_v h_v (= 2 sum_{i<j} J s s); H = -that / 2.
__global__ void k_init_finish(int64_t* E, int32_t R, RunState* st, int8_t* best, int32_t np) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < R) E[i] = -(E[i] / 2);
  for (int v = i; v < np; v += gridDim.x * blockDim.x) best[v] = 1;
  if (i == 0) {
    st->mstar = 0;
    st->cur = 0;
    st->gs = st->g_rs = st->g_cl = 0;
    st->stopped = 0;
    st->active = 0;
  }
}

// ---------------------------------------------------------------------------
// Controller kernels (single thread): Algorithm 1's per-step decisions.
// ---------------------------------------------------------------------------
__global__ void k_anneal_setup(RunState* st, Schedule s) {
  st->beta0 = s.beta0;
  st->dbeta = s.dbeta;
  st->reheat = s.reheat;
  st->target = s.target;
  st->steps = s.steps;
  st->sweeps = s.sweeps;
  st->z_rst = s.z_rst;
  st->augmented = s.augmented;
  st->resample = s.resample;
  st->win_short = s.win_short;
  st->win_long = s.win_long;
  st->max_ds = s.max_ds;
  st->max_dl = s.max_dl;
  st->tau = s.tau;
  st->n_top = s.n_top;
  st->mis_trials = s.mis_trials;
  st->stop_at_target = s.stop_at_target;
  st->literal_break = s.literal_break;
  st->z = 1;
  st->cycle = 0;
  st->beta = s.beta0;
  st->delta = s.dbeta;
  st->enable = 0;
  st->cooldown = 0;
  st->hist_len = 0;
  st->stopped = 0;
  st->active = 0;
  st->step_reached = -1;
  st->steps_run = 0;
  st->sum_lnq = 0.0;
  st->last_lnq = 0.0;
  st->n_cluster_moves = st->n_reheats = st->n_reversals = st->n_restarts = 0;
  st->t_start = wall_clock64();
  st->t_reached = 0;
}

__global__ void k_step_begin(RunState* st, int32_t step, int64_t X) {
  if (st->stopped || (st->stop_at_target && st->mstar >= st->target)) {
    st->stopped = 1;
    st->active = 0;
    return;
  }
  st->active = 1;
  st->step = step;
  st->do_resample = (st->z > 1 && st->resample) ? 1 : 0;
  st->do_cluster = (st->do_resample && st->augmented && st->enable && st->cooldown == 0) ? 1 : 0;
  st->rs_delta = st->delta;
  st->sweep_beta = st->beta;
  st->cl_n_top = st->n_top;
  st->cl_trials = st->mis_trials;
  st->table_x = table_halfwidth(st->beta, X);
  st->last_lnq = 0.0;
}

// Primitive calls: one data-parallel action outside a run.
__global__ void k_prim_set(RunState* st, int32_t kind, double value, int32_t n_top, int32_t trials,
                           int64_t X) {
  st->active = 1;
  st->do_resample = kind == 1;
  st->do_cluster = kind == 2;
  st->rs_delta = value;
  st->sweep_beta = value;
  st->cl_n_top = n_top;
  st->cl_trials = trials;
  st->table_x = table_halfwidth(value, X);
  st->last_lnq = 0.0;
}

// After resampling / cluster move: switch population buffers and advance the
// stream counters; in a run also apply Algorithm 1's "enable <- false;
// cooldown <- tau" after a cluster move.
__global__ void k_commit(RunState* st, int32_t in_run, double* tr_lnq, int32_t tr_cap) {
  if (!st->active) return;
  if (st->do_resample) {
    st->cur ^= 1;
    st->g_rs += 1;
    if (in_run) {
      st->sum_lnq += st->last_lnq;
      if (st->step < tr_cap) tr_lnq[st->step] = st->last_lnq;
    }
  } else if (in_run && st->step < tr_cap) {
    tr_lnq[st->step] = 0.0;
  }
  if (st->do_cluster) {
    st->g_cl += 1;
    if (in_run) {
      st->enable = 0;
      st->cooldown = st->tau;
      st->n_cluster_moves += 1;
    }
  }
}

// Threshold table for the step's beta (entries x = -Xt..Xt) and the class
// order of each of the step's sweeps: a Fisher-Yates shuffle driven by
// Philox(i, sweep, 0, ORDER), j = floor(u (i+1) / 2^32).
__global__ void __launch_bounds__(256) k_thresholds(RunState* st, uint32_t* thr, int32_t rule,
                                                    int32_t* order, int32_t ncls, int32_t nsweeps,
                                                    int32_t shuffle, uint32_t k0, uint32_t k1) {
  if (!st->active) return;
  const int64_t Xt = st->table_x;
  const double beta = st->sweep_beta;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= 2 * Xt;
       i += (int64_t)gridDim.x * blockDim.x)
    thr[i] = flip_threshold(beta, rule, i - Xt);
  if (blockIdx.x == 0) {
    for (int s = threadIdx.x; s < nsweeps; s += blockDim.x) {
      int32_t* o = order + (size_t)s * ncls;
      for (int k = 0; k < ncls; ++k) o[k] = k;
      if (shuffle) {
        const uint32_t gs = st->gs + (uint32_t)s;
        for (int i = ncls - 1; i >= 1; --i) {
          const u32x4 w = philox10((uint32_t)i, gs, 0u, kTagOrder, k0, k1);
          const int j = (int)(((uint64_t)w.a * (uint64_t)(i + 1)) >> 32);
          const int32_t t = o[i];
          o[i] = o[j];
          o[j] = t;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Best cut (Algorithm 1: M* <- max(M*, max Cut(P)), lowest slot on ties),
// then, in a run, the recent-progress history, the adaptive temperature rule
// and the schedule advance.
// ---------------------------------------------------------------------------
struct StepEndArgs {
  RunState* st;
  int64_t* E0;
  int64_t* E1;
  const uint32_t* S0;
  const uint32_t* S1;
  int8_t* best;
  int64_t W;
  int32_t R, nq, np;
  int64_t* tr_mstar;
  double* tr_beta;
  int32_t* tr_events;
  uint64_t* tr_time;
  int32_t tr_cap;
  int32_t ev_bits_extra;
  const int8_t* D0;  // dense instances: replica-major spins [R][np]
  const int8_t* D1;
  int32_t dense;
};

__device__ int32_t distinct_tail(const int64_t* h, int len, int w) {
  int d = 0;
  for (int i = len - w; i < len; ++i) {
    bool dup = false;
    for (int j = len - w; j < i; ++j)
      if (h[j] == h[i]) { dup = true; break; }
    if (!dup) ++d;
  }
  return d;
}

__global__ void __launch_bounds__(1024) k_step_end(StepEndArgs a, int32_t in_run) {
  __shared__ int64_t bc[1024];
  __shared__ int32_t bs[1024];
  __shared__ int improved;
  RunState* st = a.st;
  if (!st->active) return;
  const int cur = st->cur;
  const int64_t* E = cur ? a.E1 : a.E0;
  const uint32_t* S = cur ? a.S1 : a.S0;
  int64_t c = INT64_MIN;
  int32_t cs = 0x7FFFFFFF;
  for (int r = threadIdx.x; r < a.R; r += blockDim.x) {
    const int64_t cut = (a.W - E[r]) / 2;
    if (cut > c) { c = cut; cs = r; }
  }
  bc[threadIdx.x] = c;
  bs[threadIdx.x] = cs;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      const int64_t c2 = bc[threadIdx.x + o];
      const int32_t s2 = bs[threadIdx.x + o];
      if (c2 > bc[threadIdx.x] || (c2 == bc[threadIdx.x] && s2 < bs[threadIdx.x])) {
        bc[threadIdx.x] = c2;
        bs[threadIdx.x] = s2;
      }
    }
    __syncthreads();
  }
  const int64_t m = bc[0];
  const int32_t slot = bs[0];
  if (threadIdx.x == 0) improved = m > st->mstar;
  __syncthreads();
  if (improved) {
    if (a.dense) {
      const int8_t* D = (cur ? a.D1 : a.D0) + (size_t)slot * a.np;
      for (int v = threadIdx.x; v < a.np; v += blockDim.x) a.best[v] = D[v];
    } else {
      const int tile = slot >> 6, lane = slot & 63;
      for (int v = threadIdx.x; v < a.np; v += blockDim.x) {
        const uint32_t w = S[((size_t)tile * a.nq + (v >> 2)) * kLanes + lane];
        a.best[v] = (int8_t)(w >> (8 * (v & 3)));
      }
    }
  }
  if (threadIdx.x != 0) return;
  if (improved) {
    st->mstar = m;
    st->best_slot = slot;
  }
  if (!in_run) return;
  const int64_t ms = st->mstar;
  int32_t ev = (st->do_resample ? 1 : 0) | (st->do_cluster ? 2 : 0);
  const uint64_t now = wall_clock64();
  if (st->step_reached < 0 && ms >= st->target) {
    st->step_reached = st->step;
    st->t_reached = now;
  }
  // recent-progress history (only the last win_long values are needed)
  if (st->hist_len >= st->win_long) {
    for (int i = 1; i < st->hist_len; ++i) st->hist[i - 1] = st->hist[i];
    st->hist_len -= 1;
  }
  st->hist[st->hist_len++] = ms;
  if (st->augmented && st->cooldown == 0 && st->hist_len >= st->win_long) {
    const int ds = distinct_tail(st->hist, st->hist_len, st->win_short);
    const int dl = distinct_tail(st->hist, st->hist_len, st->win_long);
    if (ds <= st->max_ds && dl <= st->max_dl) {          // strong stagnation
      st->beta = st->reheat * st->beta;
      st->delta = st->dbeta;
      st->enable = 1;
      ev |= 4;
      st->n_reheats += 1;
    } else if (ds <= st->max_ds) {                       // mild stagnation
      if (st->beta > st->beta0) {
        st->delta = -st->dbeta;
        ev |= 8;
        st->n_reversals += 1;
      } else if (st->literal_break) {
        st->stopped = 1;
      } else {
        st->delta = st->dbeta;
      }
    } else {                                             // progress: cool
      st->delta = st->dbeta;
    }
  }
  if (st->z_rst > 0 && st->z >= st->z_rst) {             // restart
    st->cycle += 1;
    st->z = 1;
    st->beta = st->beta0;
    st->delta = st->dbeta;
    st->enable = 0;
    st->cooldown = 0;
    st->hist_len = 0;
    ev |= 16;
    st->n_restarts += 1;
  } else {
    st->z += 1;
    st->beta = st->beta + st->delta;
    if (st->cooldown > 0) st->cooldown -= 1;
  }
  st->gs += (uint32_t)st->sweeps;
  st->steps_run = st->step + 1;
  if (st->step < a.tr_cap) {
    a.tr_mstar[st->step] = ms;
    a.tr_beta[st->step] = st->sweep_beta;
    a.tr_events[st->step] = ev;
    a.tr_time[st->step] = now;
  }
  if (st->stop_at_target && ms >= st->target) st->stopped = 1;
}

__global__ void k_advance_sweeps(RunState* st, int32_t nsweeps) {
  st->gs += (uint32_t)nsweeps;
  st->active = 0;
}

__global__ void k_deactivate(RunState* st) { st->active = 0; }

// ---------------------------------------------------------------------------
// Resampling (Eqs. 1-2), one work-group.  Weights relative to the extreme
// energy, w_r = e^{-Delta (E_r - E_ref)} in binary64; ln Q = -Delta E_ref +
// ln sum w - ln R.  Selection is exact integer arithmetic: q_r =
// floor(w_r 2^48), inclusive prefix P, child k draws a 64-bit Philox word u,
// y = floor(u Q / 2^64), parent = least j with P_j > y; children are then
// laid out by parent (counting sort).
// ---------------------------------------------------------------------------
template <typename V>
__device__ V block_scan_incl(V x, V* tmp) {  // 1024 threads, Hillis-Steele
  tmp[threadIdx.x] = x;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    V y = (int)threadIdx.x >= o ? tmp[threadIdx.x - o] : (V)0;
    __syncthreads();
    tmp[threadIdx.x] += y;
    __syncthreads();
  }
  V r = tmp[threadIdx.x];
  __syncthreads();
  return r;
}

struct RsArgs {
  RunState* st;
  int64_t* E0;
  int64_t* E1;
  uint64_t* P;
  int32_t* parent;
  int32_t R;
  uint32_t k0, k1;
};

__global__ void __launch_bounds__(1024) k_rs_select(RsArgs a) {
  __shared__ int32_t cnt[kRsMaxR];
  __shared__ uint64_t tmp64[1024];
  __shared__ double tmpd[1024];
  __shared__ int64_t eref_s;
  RunState* st = a.st;
  if (!st->active || !st->do_resample) return;
  const int64_t* E = st->cur ? a.E1 : a.E0;
  const double delta = st->rs_delta;
  const int R = a.R;
  const int tid = threadIdx.x;
  // extreme energy: min for delta >= 0, max otherwise
  {
    int64_t m = E[0];
    for (int r = tid; r < R; r += 1024) {
      const int64_t e = E[r];
      if (delta >= 0 ? e < m : e > m) m = e;
    }
    tmp64[tid] = (uint64_t)m;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
      if (tid < o) {
        const int64_t x = (int64_t)tmp64[tid], y = (int64_t)tmp64[tid + o];
        tmp64[tid] = (uint64_t)(delta >= 0 ? (y < x ? y : x) : (y > x ? y : x));
      }
      __syncthreads();
    }
    if (tid == 0) eref_s = (int64_t)tmp64[0];
    __syncthreads();
  }
  const int64_t eref = eref_s;
  // contiguous chunk per thread
  const int per = (R + 1023) / 1024;
  const int r0 = tid * per, r1 = min(R, r0 + per);
  double wsum = 0.0;
  uint64_t run = 0;
  for (int r = r0; r < r1; ++r) {
    const double w = exp_cw(-(delta * (double)(E[r] - eref)));
    wsum += w;
    run += (uint64_t)floor(w * 281474976710656.0);
    a.P[r] = run;  // local inclusive prefix
  }
  const uint64_t off = block_scan_incl<uint64_t>(run, tmp64) - run;
  for (int r = r0; r < r1; ++r) a.P[r] += off;
  tmpd[tid] = wsum;
  for (int r = tid; r < R; r += 1024) cnt[r] = 0;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (tid < o) tmpd[tid] += tmpd[tid + o];
    __syncthreads();
  }
  const double wtot = tmpd[0];
  __threadfence_block();
  __syncthreads();
  const uint64_t Q = a.P[R - 1];
  const uint32_t g = st->g_rs;
  for (int k = tid; k < R; k += 1024) {
    const u32x4 w = philox10((uint32_t)(k >> 1), g, 0u, kTagResample, a.k0, a.k1);
    const uint64_t u = (k & 1) ? ((uint64_t)w.c | ((uint64_t)w.d << 32))
                               : ((uint64_t)w.a | ((uint64_t)w.b << 32));
    const uint64_t y = __umul64hi(u, Q);
    int lo = 0, hi = R - 1;  // least j with P[j] > y; P[R-1] = Q > y
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (a.P[mid] > y) hi = mid; else lo = mid + 1;
    }
    atomicAdd(&cnt[lo], 1);
  }
  __syncthreads();
  // children ordered by parent
  int local = 0;
  for (int r = r0; r < r1; ++r) local += cnt[r];
  const int start = (int)block_scan_incl<uint64_t>((uint64_t)local, tmp64) - local;
  int pos = start;
  for (int r = r0; r < r1; ++r)
    for (int c = 0; c < cnt[r]; ++c) a.parent[pos++] = r;
  if (tid == 0) st->last_lnq = -delta * (double)eref + log(wtot) - log((double)R);
}

struct GatherArgs {
  RunState* st;
  uint32_t* S0;
  uint32_t* S1;
  int32_t* H0;
  int32_t* H1;
  int64_t* E0;
  int64_t* E1;
  int32_t* F0;
  int32_t* F1;
  const int32_t* parent;
  int32_t nq, np, T;
};

// Copies every child's spins, fields, energy and lineage from its parent into
// the other population buffer.
__global__ void __launch_bounds__(256) k_rs_gather(GatherArgs a) {
  RunState* st = a.st;
  if (!st->active || !st->do_resample) return;
  const int cur = st->cur;
  const uint32_t* Ss = cur ? a.S1 : a.S0;
  uint32_t* Sd = cur ? a.S0 : a.S1;
  const int32_t* Hs = cur ? a.H1 : a.H0;
  int32_t* Hd = cur ? a.H0 : a.H1;
  int tile, chunk;
  tile_chunk(a.T, tile, chunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = tile * kLanes + lane;
  const int p = a.parent[c];
  const int pt = p >> 6, pl = p & 63;
  if (chunk == 0 && wave == 0) {
    (cur ? a.E0 : a.E1)[c] = (cur ? a.E1 : a.E0)[p];
    (cur ? a.F0 : a.F1)[c] = (cur ? a.F1 : a.F0)[p];
  }
  const int qb = chunk * kGatherQuadsPerBlock;
  for (int qi = wave; qi < kGatherQuadsPerBlock; qi += 4) {
    const int q = qb + qi;
    if (q >= a.nq) break;
    Sd[((size_t)tile * a.nq + q) * kLanes + lane] = Ss[((size_t)pt * a.nq + q) * kLanes + pl];
    if (!Hs) continue;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int v = 4 * q + k;
      Hd[((size_t)tile * a.np + v) * kLanes + lane] = Hs[((size_t)pt * a.np + v) * kLanes + pl];
    }
  }
}

// ---------------------------------------------------------------------------
// Non-local cluster move (Algorithm 1; Sec. "Augmented PAMC").
// cl_select: the n_top slots with the lowest (E, slot), by rank counting.
// cl_mis: per (target, trial), the greedy independent set of iso-sites
//   (h = 0) in the order of Philox keys (v, g_cl, r, CL | t<<8), ties by id.
//   The sequential greedy is computed with parallel rounds: an undecided
//   vertex joins once no undecided neighbour precedes it, and leaves once a
//   neighbour has joined; this selects exactly the sequential greedy set.
// cl_apply: flips the largest set (earliest trial on ties); fields of the
//   neighbours change, the energy does not (every flipped spin has h = 0 and
//   no two are coupled).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_cl_select(RunState* st, int64_t* E0, int64_t* E1,
                                                    int32_t R, int32_t* targets) {
  __shared__ int64_t es[4096];
  if (!st->active || !st->do_cluster) return;
  const int buf = st->cur ^ st->do_resample;
  const int64_t* E = buf ? E1 : E0;
  const int n_top = min(st->cl_n_top, R);
  constexpr int kPer = kRsMaxR / 1024;
  int64_t mine[kPer];
  int rank[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int r = threadIdx.x + i * 1024;
    mine[i] = r < R ? E[r] : 0;
    rank[i] = 0;
  }
  for (int base = 0; base < R; base += 4096) {
    const int len = min(4096, R - base);
    __syncthreads();
    for (int q = threadIdx.x; q < len; q += 1024) es[q] = E[base + q];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int r = threadIdx.x + i * 1024;
      if (r >= R) continue;
      int c = 0;
      for (int q = 0; q < len; ++q) {
        const int64_t f = es[q];
        c += (f < mine[i]) || (f == mine[i] && base + q < r);
      }
      rank[i] += c;
    }
  }
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int r = threadIdx.x + i * 1024;
    if (r < R && rank[i] < n_top) targets[rank[i]] = r;
  }
}

struct ClArgs {
  RunState* st;
  const int32_t* row_ptr;
  const int32_t* col;
  const int32_t* J;
  uint32_t* S0;
  uint32_t* S1;
  int32_t* H0;
  int32_t* H1;
  const int32_t* targets;
  uint8_t* sel;
  int32_t* sizes;
  int32_t n, np, nq, trials;
  uint32_t k0, k1;
};

enum : uint8_t { kOut = 0, kUnd = 1, kCand = 2, kIn = 3 };

__global__ void __launch_bounds__(1024) k_cl_mis(ClArgs a) {
  extern __shared__ uint8_t lds[];
  __shared__ int32_t cnt_s;
  RunState* st = a.st;
  if (!st->active || !st->do_cluster) return;
  const int i = blockIdx.x / a.trials, t = blockIdx.x % a.trials;
  if (i >= min(st->cl_n_top, (int)(gridDim.x / a.trials))) return;
  const int buf = st->cur ^ st->do_resample;
  const int32_t* H = buf ? a.H1 : a.H0;
  const uint32_t* S = buf ? a.S1 : a.S0;
  uint32_t* key = (uint32_t*)lds;
  uint8_t* state = lds + sizeof(uint32_t) * (size_t)a.np;
  const int r = a.targets[i];
  const int tile = r >> 6, lane = r & 63;
  const uint32_t g = st->g_cl;
  for (int v = threadIdx.x; v < a.np; v += blockDim.x) {
    uint8_t s = kOut;
    int32_t h = 1;
    if (v < a.n) {
      if (H) {
        h = H[((size_t)tile * a.np + v) * kLanes + lane];
      } else {
        h = 0;
        for (int e = a.row_ptr[v]; e < a.row_ptr[v + 1]; ++e) h += a.J[e] * spin_at(S, a.nq, tile, a.col[e], lane);
      }
    }
    if (v < a.n && h == 0) {
      s = kUnd;
      key[v] = philox10((uint32_t)v, g, (uint32_t)r, kTagCluster | ((uint32_t)t << 8), a.k0, a.k1).a;
    }
    state[v] = s;
  }
  __syncthreads();
  while (true) {
    for (int v = threadIdx.x; v < a.n; v += blockDim.x) {
      if (state[v] != kUnd) continue;
      const uint32_t kv = key[v];
      bool root = true;
      for (int e = a.row_ptr[v]; e < a.row_ptr[v + 1]; ++e) {
        const int u = a.col[e];
        const uint8_t su = state[u];
        if ((su == kUnd || su == kCand) && (key[u] < kv || (key[u] == kv && u < v))) {
          root = false;
          break;
        }
      }
      if (root) state[v] = kCand;
    }
    __syncthreads();
    for (int v = threadIdx.x; v < a.n; v += blockDim.x)
      if (state[v] == kCand) state[v] = kIn;
    __syncthreads();
    int und = 0;
    for (int v = threadIdx.x; v < a.n; v += blockDim.x) {
      if (state[v] != kUnd) continue;
      bool out = false;
      for (int e = a.row_ptr[v]; e < a.row_ptr[v + 1]; ++e)
        if (state[a.col[e]] == kIn) { out = true; break; }
      if (out) state[v] = kOut; else und = 1;
    }
    if (!__syncthreads_or(und)) break;
  }
  if (threadIdx.x == 0) cnt_s = 0;
  __syncthreads();
  int mine = 0;
  uint8_t* out = a.sel + (size_t)blockIdx.x * a.np;
  for (int v = threadIdx.x; v < a.np; v += blockDim.x) {
    const uint8_t in = state[v] == kIn;
    out[v] = in;
    mine += in;
  }
  atomicAdd(&cnt_s, mine);
  __syncthreads();
  if (threadIdx.x == 0) a.sizes[blockIdx.x] = cnt_s;
}

__global__ void __launch_bounds__(256) k_cl_apply(ClArgs a, int64_t* flipped) {
  RunState* st = a.st;
  if (!st->active || !st->do_cluster) return;
  const int i = blockIdx.y;
  if (i >= st->cl_n_top) return;
  const int buf = st->cur ^ st->do_resample;
  uint32_t* S = buf ? a.S1 : a.S0;
  int32_t* H = buf ? a.H1 : a.H0;
  int tb = 0, best = -1;
  for (int t = 0; t < a.trials; ++t) {
    const int s = a.sizes[i * a.trials + t];
    if (s > best) { best = s; tb = t; }
  }
  const uint8_t* sel = a.sel + (size_t)(i * a.trials + tb) * a.np;
  const int r = a.targets[i];
  const int tile = r >> 6, lane = r & 63;
  int mine = 0;
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < a.n; v += gridDim.x * blockDim.x) {
    if (!sel[v]) continue;
    int8_t* sb = (int8_t*)&S[((size_t)tile * a.nq + (v >> 2)) * kLanes + lane] + (v & 3);
    const int32_t snew = -(int32_t)*sb;
    *sb = (int8_t)snew;
    if (H)
      for (int e = a.row_ptr[v]; e < a.row_ptr[v + 1]; ++e)
      __hip_atomic_fetch_add(&H[((size_t)tile * a.np + a.col[e]) * kLanes + lane], 2 * a.J[e] * snew,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ++mine;
  }
  if (mine)
    __hip_atomic_fetch_add((unsigned long long*)flipped, (unsigned long long)mine, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Max-3-Cut decode (see pamc.h) and the pairwise Hamming diagnostic.
// ---------------------------------------------------------------------------
__global__ void k_m3_decode(const int8_t* spins_internal, const int32_t* to_internal_emb,
                            int32_t n3, const int32_t* row_ptr, const int32_t* col, const int32_t* w,
                            int32_t* labels, int64_t* cut) {
  // pass 1 (all threads): labels
  const int anc = to_internal_emb[3 * n3];
  const int g = spins_internal[anc] < 0 ? -1 : 1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += gridDim.x * blockDim.x) {
    int lab = 0;
    for (int aa = 2; aa >= 0; --aa)
      if (g * spins_internal[to_internal_emb[3 * i + aa]] > 0) lab = aa;
    labels[i] = lab;
  }
}

__global__ void k_m3_cut(const int32_t* labels, int32_t n3, const int32_t* row_ptr, const int32_t* col,
                         const int32_t* w, int64_t* cut) {
  int64_t c = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += gridDim.x * blockDim.x)
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int j = col[e];
      if (j > i && labels[i] != labels[j]) c += w[e];
    }
  c = wave_sum_i64(c);
  if ((threadIdx.x & 63) == 0 && c)
    __hip_atomic_fetch_add((unsigned long long*)cut, (unsigned long long)c, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(256) k_pair_distance(const uint32_t* S0, const uint32_t* S1,
                                                       const RunState* st, int32_t n, int32_t nq,
                                                       int32_t R, double* out) {
  const uint32_t* S = st->cur ? S1 : S0;
  const int a = blockIdx.x;
  double acc = 0.0;
  for (int b = a + 1 + threadIdx.x; b < R; b += blockDim.x) {
    int d = 0;
    for (int q = 0; q < nq; ++q) {
      const uint32_t x = S[((size_t)(a >> 6) * nq + q) * kLanes + (a & 63)];
      const uint32_t y = S[((size_t)(b >> 6) * nq + q) * kLanes + (b & 63)];
      uint32_t diff = x ^ y;  // spins are 0x01 / 0xFF bytes: a byte differs iff nonzero
      diff = (diff | (diff >> 1) | (diff >> 2) | (diff >> 3) | (diff >> 4) | (diff >> 5) |
              (diff >> 6) | (diff >> 7)) & 0x01010101u;
      d += __popc(diff);
    }
    const double f = (double)d / n;
    acc += f < 1.0 - f ? f : 1.0 - f;
  }
  atomicAdd(out, acc);
}

}  // namespace

// ===========================================================================
// Host launchers
// ===========================================================================
static inline uint32_t key0(const pamc_instance* I) { return (uint32_t)I->seed; }
static inline uint32_t key1(const pamc_instance* I) { return (uint32_t)(I->seed >> 32); }

int32_t cluster_max_n() { return kClusterMaxN; }

static SweepArgs sweep_args(pamc_instance* I) {
  SweepArgs a;
  a.row_ptr = I->g.row_ptr;
  a.col = I->g.col;
  a.J = I->g.J;
  a.class_ptr = I->g.class_ptr;
  a.order = I->order;
  a.S0 = I->pop.S[0];
  a.S1 = I->pop.S[1];
  a.H0 = I->pop.H[0];
  a.H1 = I->pop.H[1];
  a.E0 = I->pop.E[0];
  a.E1 = I->pop.E[1];
  a.thr = I->thr;
  a.st = I->st;
  a.flip_ctr = I->prof ? I->flip_ctr : nullptr;
  a.nq = I->nq;
  a.np = I->np;
  a.T = I->T;
  a.ncls = I->ncls;
  a.k0 = key0(I);
  a.k1 = key1(I);
  return a;
}

static hipEvent_t next_event(pamc_instance* I) {
  if (I->ev_used == I->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    I->ev_pool.push_back(e);
  }
  return I->ev_pool[I->ev_used++];
}

using PullKernel = void (*)(const int32_t*, const int32_t*, const int32_t*, const int32_t*,
                           const int32_t*, const uint32_t*, SweepArgs, int, int);

template <int RULE, bool SMALLJ>
static PullKernel pull_kernel_t(int tpw) {
  return tpw == 4 ? k_sweep_pull<RULE, SMALLJ, 4>
                  : (tpw == 2 ? k_sweep_pull<RULE, SMALLJ, 2> : k_sweep_pull<RULE, SMALLJ, 1>);
}

static PullKernel pull_kernel(const pamc_instance* I) {
  if (I->rule == 1) return I->small_j ? pull_kernel_t<1, true>(I->tpw) : pull_kernel_t<1, false>(I->tpw);
  return I->small_j ? pull_kernel_t<0, true>(I->tpw) : pull_kernel_t<0, false>(I->tpw);
}

// Sweeps of one step (or primitive): thresholds + class orders, then
// nsweeps x ncls phase launches.
static hipError_t launch_sweeps(pamc_instance* I, int32_t nsweeps) {
  const int shuffle = (I->flags & 1u) ? 0 : 1;
  int done = 0;
  while (done < nsweeps) {
    const int batch = std::min(nsweeps - done, I->order_cap);
    // thresholds are recomputed per batch; class orders use gs + done + s
    k_thresholds<<<64, 256, 0, I->stream>>>(I->st, I->thr, I->rule, I->order, I->ncls, batch,
                                            shuffle, key0(I), key1(I));
    SweepArgs a = sweep_args(I);
    const int chunks = (I->max_class_quads + kQuadsPerBlock - 1) / kQuadsPerBlock;
    const int grid = I->T * chunks;
    for (int s = 0; s < batch; ++s) {
      for (int p = 0; p < I->ncls; ++p) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (I->prof) {
          e0 = next_event(I);
          hipEventRecord(e0, I->stream);
        }
        if (I->pull) {
          pull_kernel(I)<<<grid / I->tpw, 256, 0, I->stream>>>(I->g.row_ptr, I->g.col, I->g.J,
                                                               I->g.class_ptr, I->order, I->thr, a,
                                                               s, p);
        } else if (I->rule == 1) {
          k_sweep<1><<<grid, 256, 0, I->stream>>>(I->g.row_ptr, I->g.col, I->g.J, I->g.class_ptr, I->order, I->thr, a, s, p);
        } else {
          k_sweep<0><<<grid, 256, 0, I->stream>>>(I->g.row_ptr, I->g.col, I->g.J, I->g.class_ptr, I->order, I->thr, a, s, p);
        }
        if (I->prof) {
          e1 = next_event(I);
          hipEventRecord(e1, I->stream);
          I->prof_launches += 1;
        }
      }
    }
    if (I->prof) I->prof_attempts += (int64_t)batch * I->n * I->R;
    done += batch;
    if (done < nsweeps) {
      // advance the sweep counter between batches (only the primitive path
      // can exceed order_cap; a run's step has sweeps <= order_cap)
      k_advance_sweeps<<<1, 1, 0, I->stream>>>(I->st, batch);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

hipError_t launch_init_sparse(pamc_instance* I) {
  const size_t words = (size_t)I->T * I->nq * kLanes;
  int grid = (int)std::min<size_t>((words + 255) / 256, 65535);
  k_init_spins<<<grid, 256, 0, I->stream>>>(I->pop.S[0], I->pop.fam[0], I->n, I->nq, I->T, key0(I),
                                            key1(I));
  hipMemsetAsync(I->pop.E[0], 0, sizeof(int64_t) * I->R, I->stream);
  const int vchunks = (I->n + 63) / 64;
  k_init_fields<<<I->T * vchunks, 256, 0, I->stream>>>(I->g.row_ptr, I->g.col, I->g.J, I->pop.S[0],
                                                       I->pop.H[0], I->pop.E[0], I->n, I->np, I->nq,
                                                       I->T);
  k_init_finish<<<(std::max(I->R, I->np) + 255) / 256, 256, 0, I->stream>>>(I->pop.E[0], I->R,
                                                                             I->st, I->best, I->np);
  return hipGetLastError();
}

hipError_t launch_fields(pamc_instance* I, int32_t* H) {
  const int vchunks = (I->n + 63) / 64;
  // current buffer index is read by the host before this call
  k_init_fields<<<I->T * vchunks, 256, 0, I->stream>>>(I->g.row_ptr, I->g.col, I->g.J,
                                                       I->pop.S[I->host_cur], H, nullptr, I->n,
                                                       I->np, I->nq, I->T);
  return hipGetLastError();
}

hipError_t launch_anneal_setup(pamc_instance* I, const Schedule& s) {
  k_anneal_setup<<<1, 1, 0, I->stream>>>(I->st, s);
  return hipGetLastError();
}

static hipError_t launch_resample_kernels(pamc_instance* I) {
  RsArgs r;
  r.st = I->st;
  r.E0 = I->pop.E[0];
  r.E1 = I->pop.E[1];
  r.P = I->rs_P;
  r.parent = I->rs_parent;
  r.R = I->R;
  r.k0 = key0(I);
  r.k1 = key1(I);
  k_rs_select<<<1, 1024, 0, I->stream>>>(r);
  GatherArgs g;
  g.st = I->st;
  g.S0 = I->pop.S[0];
  g.S1 = I->pop.S[1];
  g.H0 = I->pop.H[0];
  g.H1 = I->pop.H[1];
  g.E0 = I->pop.E[0];
  g.E1 = I->pop.E[1];
  g.F0 = I->pop.fam[0];
  g.F1 = I->pop.fam[1];
  g.parent = I->rs_parent;
  g.nq = I->nq;
  g.np = I->np;
  g.T = I->T;
  const int chunks = (I->nq + kGatherQuadsPerBlock - 1) / kGatherQuadsPerBlock;
  k_rs_gather<<<I->T * chunks, 256, 0, I->stream>>>(g);
  return hipGetLastError();
}

static hipError_t launch_cluster_kernels(pamc_instance* I, int32_t n_top, int32_t trials) {
  if (n_top <= 0 || trials <= 0) return hipSuccess;
  n_top = std::min(n_top, I->R);
  k_cl_select<<<1, 1024, 0, I->stream>>>(I->st, I->pop.E[0], I->pop.E[1], I->R, I->cl_targets);
  ClArgs c;
  c.st = I->st;
  c.row_ptr = I->g.row_ptr;
  c.col = I->g.col;
  c.J = I->g.J;
  c.S0 = I->pop.S[0];
  c.S1 = I->pop.S[1];
  c.H0 = I->pop.H[0];
  c.H1 = I->pop.H[1];
  c.targets = I->cl_targets;
  c.sel = I->cl_sel;
  c.sizes = I->cl_sizes;
  c.n = I->n;
  c.np = I->np;
  c.nq = I->nq;
  c.trials = trials;
  c.k0 = key0(I);
  c.k1 = key1(I);
  const size_t lds = (size_t)I->np * 5;
  k_cl_mis<<<n_top * trials, 1024, lds, I->stream>>>(c);
  const int chunks = std::max(1, std::min(64, (I->n + 255) / 256));
  k_cl_apply<<<dim3(chunks, n_top), 256, 0, I->stream>>>(c, &((int64_t*)I->flip_ctr)[256]);
  return hipGetLastError();
}

static StepEndArgs step_end_args(pamc_instance* I) {
  StepEndArgs e;
  e.st = I->st;
  e.E0 = I->pop.E[0];
  e.E1 = I->pop.E[1];
  e.S0 = I->pop.S[0];
  e.S1 = I->pop.S[1];
  e.best = I->best;
  e.W = I->W;
  e.R = I->R;
  e.nq = I->nq;
  e.np = I->np;
  e.tr_mstar = I->tr_mstar;
  e.tr_beta = I->tr_beta;
  e.tr_events = I->tr_events;
  e.tr_time = I->tr_time;
  e.tr_cap = I->tr_cap;
  e.ev_bits_extra = 0;
  e.D0 = I->Sd;
  e.D1 = I->Sd2;
  e.dense = I->dense;
  return e;
}

hipError_t launch_step(pamc_instance* I, const Schedule& s, int32_t step) {
  k_step_begin<<<1, 1, 0, I->stream>>>(I->st, step, I->X);
  if (s.resample) launch_resample_kernels(I);
  if (s.augmented && s.resample) launch_cluster_kernels(I, std::min(s.n_top, I->R), s.mis_trials);
  k_commit<<<1, 1, 0, I->stream>>>(I->st, 1, I->tr_lnq, I->tr_cap);
  hipError_t e = launch_sweeps(I, s.sweeps);
  if (e != hipSuccess) return e;
  k_step_end<<<1, 1024, 0, I->stream>>>(step_end_args(I), 1);
  return hipGetLastError();
}

hipError_t launch_prim_sweep(pamc_instance* I, double beta, int32_t nsweeps) {
  k_prim_set<<<1, 1, 0, I->stream>>>(I->st, 0, beta, 0, 0, I->X);
  hipError_t e = launch_sweeps(I, nsweeps);
  if (e != hipSuccess) return e;
  const int last = nsweeps - ((nsweeps - 1) / I->order_cap) * I->order_cap;
  k_advance_sweeps<<<1, 1, 0, I->stream>>>(I->st, last);
  return hipGetLastError();
}

hipError_t launch_prim_resample(pamc_instance* I, double delta) {
  k_prim_set<<<1, 1, 0, I->stream>>>(I->st, 1, delta, 0, 0, I->X);
  launch_resample_kernels(I);
  k_commit<<<1, 1, 0, I->stream>>>(I->st, 0, I->tr_lnq, 0);
  k_deactivate<<<1, 1, 0, I->stream>>>(I->st);
  return hipGetLastError();
}

hipError_t launch_prim_cluster(pamc_instance* I, int32_t n_top, int32_t trials) {
  k_prim_set<<<1, 1, 0, I->stream>>>(I->st, 2, 0.0, n_top, trials, I->X);
  launch_cluster_kernels(I, n_top, trials);
  k_commit<<<1, 1, 0, I->stream>>>(I->st, 0, I->tr_lnq, 0);
  k_deactivate<<<1, 1, 0, I->stream>>>(I->st);
  return hipGetLastError();
}

hipError_t launch_prim_update_best(pamc_instance* I) {
  k_prim_set<<<1, 1, 0, I->stream>>>(I->st, 0, 0.0, 0, 0, I->X);
  k_step_end<<<1, 1024, 0, I->stream>>>(step_end_args(I), 0);
  k_deactivate<<<1, 1, 0, I->stream>>>(I->st);
  return hipGetLastError();
}

hipError_t launch_m3_decode(pamc_instance* I, const int8_t* spins_internal_dev) {
  hipMemsetAsync(I->m3_cut, 0, sizeof(int64_t), I->stream);
  const int grid = (I->m3_n + 255) / 256;
  k_m3_decode<<<grid, 256, 0, I->stream>>>(spins_internal_dev, I->to_internal_dev, I->m3_n,
                                           I->m3_row_ptr, I->m3_col, I->m3_w, I->m3_labels,
                                           I->m3_cut);
  k_m3_cut<<<grid, 256, 0, I->stream>>>(I->m3_labels, I->m3_n, I->m3_row_ptr, I->m3_col, I->m3_w,
                                        I->m3_cut);
  return hipGetLastError();
}

hipError_t launch_pair_distance(pamc_instance* I, double* out_dev) {
  hipMemsetAsync(out_dev, 0, sizeof(double), I->stream);
  k_pair_distance<<<I->R, 256, 0, I->stream>>>(I->pop.S[0], I->pop.S[1], I->st, I->n, I->nq, I->R,
                                               out_dev);
  return hipGetLastError();
}

// Controller pieces shared with the dense path.
hipError_t ctl_step_begin(pamc_instance* I, int32_t step) {
  k_step_begin<<<1, 1, 0, I->stream>>>(I->st, step, I->X);
  return hipGetLastError();
}
hipError_t ctl_resample_select(pamc_instance* I) {
  RsArgs r;
  r.st = I->st;
  r.E0 = I->pop.E[0];
  r.E1 = I->pop.E[1];
  r.P = I->rs_P;
  r.parent = I->rs_parent;
  r.R = I->R;
  r.k0 = key0(I);
  r.k1 = key1(I);
  k_rs_select<<<1, 1024, 0, I->stream>>>(r);
  return hipGetLastError();
}
hipError_t ctl_commit(pamc_instance* I, int32_t in_run) {
  k_commit<<<1, 1, 0, I->stream>>>(I->st, in_run, I->tr_lnq, in_run ? I->tr_cap : 0);
  return hipGetLastError();
}
hipError_t ctl_thresholds(pamc_instance* I) {
  k_thresholds<<<64, 256, 0, I->stream>>>(I->st, I->thr, I->rule, I->order, 0, 0, 0, key0(I), key1(I));
  return hipGetLastError();
}
hipError_t ctl_step_end(pamc_instance* I, int32_t in_run) {
  k_step_end<<<1, 1024, 0, I->stream>>>(step_end_args(I), in_run);
  return hipGetLastError();
}
hipError_t ctl_prim_set(pamc_instance* I, int32_t kind, double value) {
  k_prim_set<<<1, 1, 0, I->stream>>>(I->st, kind, value, 0, 0, I->X);
  return hipGetLastError();
}
hipError_t ctl_advance(pamc_instance* I, int32_t nsweeps) {
  k_advance_sweeps<<<1, 1, 0, I->stream>>>(I->st, nsweeps);
  return hipGetLastError();
}
hipError_t ctl_deactivate(pamc_instance* I) {
  k_deactivate<<<1, 1, 0, I->stream>>>(I->st);
  return hipGetLastError();
}
hipEvent_t ctl_event(pamc_instance* I) { return next_event(I); }

hipError_t prepare_cluster_lds() {
  return hipFuncSetAttribute((const void*)k_cl_mis, hipFuncAttributeMaxDynamicSharedMemorySize,
                             kClusterMaxN * 5 + 64);
}

}  // namespace pamc
