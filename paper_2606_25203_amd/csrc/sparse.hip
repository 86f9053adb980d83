// sparse.hip -- gfx950 kernels of the sparse PAMC path and of the
// device-side controller (Algorithm 1), with their batch launchers.
//
// Every kernel works on a batch of instances: it reads the instance's
// descriptor (Desc) and its device-resident run state, and grid kernels map
// blockIdx through a per-batch table to (instance, local block).  A single
// instance is a batch of one, so one code path serves the plain, batched and
// served modes.  One beta step of Algorithm 1 is a fixed launch sequence
// whose behaviour is decided on the device from RunState, so the host never
// waits inside a run:
//   step_begin -> rs_select -> rs_gather -> cl_select -> cl_mis -> cl_apply
//   -> commit -> thresholds -> S x K sweep phases -> step_end
// Kernels with nothing to do for an instance return at once.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

#include "instance.hpp"
#include "pamc_device.hpp"

namespace pamc {

namespace {

constexpr int kSweepWaves = 4;             // waves per sweep workgroup
constexpr int kMaxQuadsPerWave = 4;        // quads per wave per sweep work-group: 1, 2 or 4 (Desc::qpw)
constexpr int kPushWorkGroups = 2048;      // incremental-field sweep work-groups of a lone instance (8 per CU)
constexpr int kPushMinWorkGroups = 512;    // ... and the least per instance of a batch
constexpr int kGatherQuadsPerBlock = 64;
constexpr int kClusterMaxN = 26000;        // LDS: 5 bytes per vertex
constexpr int kRsMaxR = 16384;
constexpr int kThrLds = 2048;              // threshold entries staged in LDS when they fit
constexpr int kThrBlocks = 16;             // threshold work-groups per instance
constexpr int kInitBlocks = 64;            // spin-init work-groups per instance
constexpr int kApplyChunks = 16;           // cluster-apply work-groups per target
constexpr int kFieldBlocks = 1024;         // max field-init work-groups per instance
constexpr uint32_t kIdle = 0xFFFFFFFFu;    // padding block: returns at once
typedef int i32x4 __attribute__((ext_vector_type(4)));
constexpr int kBufferWord3 = 0x00020000;   // buffer resource word 3: 32-bit raw data

// Map word: instance index in the high half, local block in the low half.
__device__ __forceinline__ bool resolve(const uint64_t* __restrict__ map, int& inst, int& lb) {
  const uint64_t m = map[blockIdx.x];
  inst = (int)(m >> 32);
  lb = (int)(uint32_t)m;
  return (uint32_t)m != kIdle;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int32_t spin_at(const uint32_t* S, int nq, int tile, int v, int lane) {
  const uint32_t w = S[((size_t)tile * nq + (v >> 2)) * kLanes + lane];
  return (int32_t)(int8_t)(w >> (8 * (v & 3)));
}

// local block -> (tile group, chunk).  Work-groups are dealt round-robin to
// the eight XCDs in launch order; an instance's blocks start at a multiple of
// 8 in its map, so keeping a group's blocks 8 apart keeps group g on one XCD
// when the group count is a multiple of 8.  Otherwise a plain split.
__device__ __forceinline__ void group_chunk(int G, int lb, int& group, int& chunk) {
  if ((G & 7) == 0) {
    const int xcd = lb & 7, j = lb >> 3, gp = G >> 3;
    group = (j % gp) * 8 + xcd;
    chunk = j / gp;
  } else {
    group = lb % G;
    chunk = lb / G;
  }
}

// ---------------------------------------------------------------------------
// Field of Eq. 3 for TPW tiles at once, gathered from the neighbours' spin
// words.  The scalar work (CSR entries, neighbour offsets, coupling masks) is
// shared by the tiles; the spin loads and arithmetic are per tile.
// Neighbours are taken four at a time from a copy of the CSR whose rows are
// padded to multiples of 4 entries (padding: vertex 0, coupling 0), so the
// loop body has no per-entry branches or masks.  Its column entries hold the
// byte offset of the neighbour's spin word within a tile, 256 (v >> 2), plus
// (v & 3) in coupling modes 0 and 1.  Spin words are read with
// buffer loads: the neighbour quad as the scalar offset, tile and lane as the
// vector offset, so address arithmetic stays on the scalar unit.  Coupling modes (JM): 0 full 32-bit products, 1 24-bit
// products (|J| < 2^23), 2 int8 couplings pre-shifted to the neighbour's byte
// of its spin word, so one 4 x int8 dot product adds J s_j.
// ---------------------------------------------------------------------------
template <int JM, int TPW>
__device__ __forceinline__ void gather_fields(const PAMC_GLOBAL int32_t* __restrict__ gcol,
                                              const PAMC_GLOBAL int32_t* __restrict__ gJ, int e0, int e1,
                                              __amdgpu_buffer_rsrc_t Sr, const int (&voff)[TPW],
                                              int32_t (&h)[TPW]) {
#pragma unroll
  for (int t = 0; t < TPW; ++t) h[t] = 0;
  for (int e = e0; e < e1; e += 4) {
    // rows start at multiples of 4 entries: one 16-byte scalar load each
    const i32x4 cj = *reinterpret_cast<const PAMC_GLOBAL i32x4*>(gcol + e);
    const i32x4 cJ = *reinterpret_cast<const PAMC_GLOBAL i32x4*>(gJ + e);
    // uniform by construction; stated so that a vector load of them can
    // never turn the buffer offsets below into per-lane values
    const int j[4] = {__builtin_amdgcn_readfirstlane(cj.x), __builtin_amdgcn_readfirstlane(cj.y),
                      __builtin_amdgcn_readfirstlane(cj.z), __builtin_amdgcn_readfirstlane(cj.w)};
    const int32_t c[4] = {__builtin_amdgcn_readfirstlane(cJ.x), __builtin_amdgcn_readfirstlane(cJ.y),
                          __builtin_amdgcn_readfirstlane(cJ.z), __builtin_amdgcn_readfirstlane(cJ.w)};
    uint32_t w[TPW][4];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        w[t][u] = __builtin_amdgcn_raw_buffer_load_b32(Sr, voff[t], JM == 2 ? j[u] : (j[u] & ~3), 0);
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (JM == 2) {
          h[t] = __builtin_amdgcn_sdot4((int)w[t][u], c[u], h[t], false);
        } else {
          const int32_t sv = __builtin_amdgcn_sbfe((int32_t)w[t][u], 8u * (uint32_t)(j[u] & 3), 8u);  // byte of the spin
          h[t] += JM == 1 ? __mul24(c[u], sv) : c[u] * sv;
        }
      }
  }
}

// Hub fields of the current population buffer (null without hubs).
__device__ __forceinline__ int32_t* st_cur_hub(const Desc& d) {
  return d.nhub ? (gmem((const RunState*)d.st)->cur ? d.HF1 : d.HF0) : nullptr;
}

// Work-group totals: energy changes per replica (red[wave * ntiles + t][lane])
// into E, flip counts per wave (fred, filled by lane 0 of each wave) into
// the profiling counters.
__device__ __forceinline__ void reduce_energy_and_flips(int64_t (*red)[kLanes], int32_t* fred, int wave,
                                                        int lane, int ntiles, int tile0,
                                                        PAMC_GLOBAL int64_t* E,
                                                        PAMC_GLOBAL int64_t* flip_ctr) {
  __syncthreads();
  if (wave < ntiles) {
    const int t = wave;
    int64_t sum = 0;
#pragma unroll
    for (int w = 0; w < kSweepWaves; ++w) sum += red[w * ntiles + t][lane];
    if (sum != 0)
      __hip_atomic_fetch_add((unsigned long long*)&E[(tile0 + t) * kLanes + lane], (unsigned long long)sum,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (flip_ctr && threadIdx.x == 0) {
    const int64_t f = (int64_t)fred[0] + fred[1] + fred[2] + fred[3];
    __hip_atomic_fetch_add((unsigned long long*)&flip_ctr[blockIdx.x & 255], (unsigned long long)f,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// One colour class of one sweep with fields gathered at visit time (Eqs.
// 3-4).  Work-group = (group of TPW replica tiles, chunk of the class's
// vertex quads); wave = up to 4 quads; lane = replica.  For each vertex:
// x = s*h, u = Philox word (quad, sweep, replica), flip iff u < T[x]
// (Metropolis also for x <= 0).  Vertices of a class are mutually
// uncoupled, so no spin read here as a neighbour is written here.
// The threshold table is read from LDS (THR_LDS) or from global memory.
// With int8 couplings (JM 2) the energy change of a lane over one
// work-group stays below 2^31 (|x| <= X < 2^26, at most 4 kMaxQuadsPerWave
// vertices), so it is summed in 32 bits.
// ---------------------------------------------------------------------------
template <int JM, int TPW, bool THR_LDS, bool HUB>
__device__ __forceinline__ void sweep_pull_body(const PAMC_GLOBAL int32_t* __restrict__ row_ptr,
                                                const PAMC_GLOBAL int32_t* __restrict__ col,
                                                const PAMC_GLOBAL int32_t* __restrict__ Jc,
                                                const PAMC_GLOBAL uint32_t* __restrict__ thr_g,
                                                uint32_t* thr_s, PAMC_GLOBAL uint32_t* __restrict__ S,
                                                PAMC_GLOBAL int64_t* __restrict__ E, const Desc& d,
                                                int group, int chunk, int v0, int v1, uint32_t gs,
                                                int32_t Xt) {
  using acc_t = typename std::conditional<JM == 2, int32_t, int64_t>::type;
  __shared__ int64_t red[kSweepWaves * TPW][kLanes];
  __shared__ int32_t fred[kSweepWaves];
  const int q0 = v0 >> 2;
  const int nqc = ((v1 + 3) >> 2) - q0;
  const bool metropolis = d.rule == 1;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile0 = group * TPW;
  const uint32_t tstride = (uint32_t)d.nq * kLanes;
  const __amdgpu_buffer_rsrc_t Sr = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(S + (size_t)tile0 * tstride), (short)0, (int)(TPW * tstride * 4), kBufferWord3);
  int voff[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) voff[t] = (int)(t * tstride * 4) + lane * 4;
  acc_t dE[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) dE[t] = 0;
  int32_t nflip = 0;
  // hubs (rows too long to gather): their fields come from HF, and each
  // flip's change to them (2 J s_new) is summed per lane in registers, then
  // over the work-group's waves, before one atomic per lane and hub
  const int nhub = HUB ? d.nhub : 0;
  PAMC_GLOBAL int32_t* HF = gmem(HUB ? st_cur_hub(d) : nullptr);
  int32_t hacc[kMaxHubs][TPW];
#pragma unroll
  for (int hk = 0; hk < kMaxHubs; ++hk)
#pragma unroll
    for (int t = 0; t < TPW; ++t) hacc[hk][t] = 0;
  for (int i = 0; i < d.qpw; ++i) {
    const int qi = chunk * (kSweepWaves * d.qpw) + i * kSweepWaves + wave;
    if (qi >= nqc) break;
    const int q = q0 + qi;
    uint32_t sw[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) sw[t] = __builtin_amdgcn_raw_buffer_load_b32(Sr, voff[t], q * (kLanes * 4), 0);
    int32_t h[4][TPW];
    int32_t hj[4][kMaxHubs];  // couplings of the quad's vertices to the hubs (uniform)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int v = 4 * q + k;
      const bool in = v >= v0 && v < v1;
#pragma unroll
      for (int hk = 0; hk < kMaxHubs; ++hk) hj[k][hk] = (HUB && in) ? gmem(d.hubJ)[v * kMaxHubs + hk] : 0;
      if (HUB && in && (v == d.hub_v0 || v == d.hub_v1)) {
        const int hk = v == d.hub_v0 ? 0 : 1;
#pragma unroll
        for (int t = 0; t < TPW; ++t) h[k][t] = HF[hk * d.R + (tile0 + t) * kLanes + lane];
      } else if (in) {
        gather_fields<JM, TPW>(col, Jc, row_ptr[v], row_ptr[v + 1], Sr, voff, h[k]);
      } else {
#pragma unroll
        for (int t = 0; t < TPW; ++t) h[k][t] = 0;
      }
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const uint32_t r = (uint32_t)((tile0 + t) * kLanes + lane);
      const u32x4 rnd = philox10((uint32_t)q, gs, r, kTagSweep, d.k0, d.k1);
      const uint32_t swt = sw[t];
      uint32_t flipmask = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int v = 4 * q + k;
        if (v < v0 || v >= v1) continue;
        const int32_t s = __builtin_amdgcn_sbfe((int32_t)swt, 8u * k, 8u);
        const int32_t x = __mul24(s, h[k][t]);
        const int32_t xi = min(max(x, -Xt), Xt) + Xt;
        const uint32_t T = THR_LDS ? thr_s[xi] : thr_g[xi];
        const bool flip = (pick(rnd, k) < T) || (metropolis && x <= 0);
        dE[t] += flip ? (acc_t)x : (acc_t)0;
        flipmask |= flip ? (0xFEu << (8 * k)) : 0u;  // +1 (0x01) <-> -1 (0xFF)
        nflip += __popcll(__ballot(flip));
        if constexpr (HUB) {
#pragma unroll
          for (int hk = 0; hk < kMaxHubs; ++hk) hacc[hk][t] += flip ? -2 * s * hj[k][hk] : 0;
        }
      }
      if (flipmask) __builtin_amdgcn_raw_buffer_store_b32(swt ^ flipmask, Sr, voff[t], q * (kLanes * 4), 0);
    }
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t) red[wave * TPW + t][lane] = 2 * (int64_t)dE[t];
  if (lane == 0) fred[wave] = nflip;
  reduce_energy_and_flips(red, fred, wave, lane, TPW, tile0, E, gmem(d.flip_ctr));
  if constexpr (HUB) {
    // the energy sums are done with red: it now holds the waves' hub sums
    // (kSweepWaves x kMaxHubs x TPW x 64 int32, the same 2048 TPW bytes)
    int32_t* hred = reinterpret_cast<int32_t*>(&red[0][0]);
    __syncthreads();
#pragma unroll
    for (int hk = 0; hk < kMaxHubs; ++hk)
#pragma unroll
      for (int t = 0; t < TPW; ++t) hred[((wave * kMaxHubs + hk) * TPW + t) * kLanes + lane] = hacc[hk][t];
    __syncthreads();
    if (wave < TPW) {
      const int t = wave;
      for (int hk = 0; hk < nhub; ++hk) {
        int32_t sum = 0;
#pragma unroll
        for (int w = 0; w < kSweepWaves; ++w) sum += hred[((w * kMaxHubs + hk) * TPW + t) * kLanes + lane];
        if (sum != 0)
          __hip_atomic_fetch_add(&HF[hk * d.R + (tile0 + t) * kLanes + lane], sum, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// WIDE: the instance's threshold table (2X + 1 entries) may exceed the LDS
// copy; a step whose table does not fit reads it from global memory.  The
// host picks the variant from X, so instances whose table always fits get
// one loop body.  HUB: the instance keeps the fields of its hub vertices.
template <int JM, int TPW, bool WIDE, bool HUB>
__global__ void __launch_bounds__(256) k_sweep_pull(const Desc* __restrict__ D,
                                                  const uint64_t* __restrict__ map, int sweep_idx,
                                                  int phase) {
  __shared__ uint32_t thr_s[kThrLds];
  int inst, lb;
  if (!resolve(map, inst, lb)) return;
  const Desc& d = D[inst];
  const PAMC_GLOBAL RunState* __restrict__ st = gmem((const RunState*)d.st);
  if (!st->active || sweep_idx >= st->nsweeps_now || phase >= d.ncls) return;
  const int cur = st->cur;
  const PAMC_GLOBAL int32_t* __restrict__ order = gmem((const int32_t*)d.order);
  const PAMC_GLOBAL int32_t* __restrict__ class_ptr = gmem(d.class_ptr);
  const int cls = order[sweep_idx * d.ncls + phase];
  const int v0 = class_ptr[cls], v1 = class_ptr[cls + 1];
  const int nqc = ((v1 + 3) >> 2) - (v0 >> 2);
  int group, chunk;
  group_chunk(d.T / TPW, lb, group, chunk);
  if (chunk * (kSweepWaves * d.qpw) >= nqc) return;
  const uint32_t gs = st->gs + (uint32_t)sweep_idx;
  const int32_t Xt = (int32_t)st->table_x;
  const PAMC_GLOBAL uint32_t* __restrict__ thr_g = gmem((const uint32_t*)d.thr);
  PAMC_GLOBAL uint32_t* __restrict__ S = gmem(cur ? d.S1 : d.S0);
  PAMC_GLOBAL int64_t* __restrict__ E = gmem(cur ? d.E1 : d.E0);
  const PAMC_GLOBAL int32_t* __restrict__ Jc = gmem(d.gJ);
  // the step's table (2 Xt + 1 entries) goes to LDS whenever it fits, also
  // for instances whose full range (WIDE: 2X + 1) would not
  if (!WIDE || 2 * Xt + 1 <= kThrLds) {
    for (int i = threadIdx.x; i <= 2 * Xt; i += blockDim.x) thr_s[i] = thr_g[i];
    __syncthreads();
    sweep_pull_body<JM, TPW, true, HUB>(gmem(d.grow), gmem(d.gcol), Jc, thr_g, thr_s, S, E, d, group, chunk, v0,
                                        v1, gs, Xt);
  } else {
    sweep_pull_body<JM, TPW, false, HUB>(gmem(d.grow), gmem(d.gcol), Jc, thr_g, thr_s, S, E, d, group, chunk, v0,
                                         v1, gs, Xt);
  }
}

// ---------------------------------------------------------------------------
// All of a step's sweeps of one replica tile in one work-group, for small
// instances (gathered fields, at most kTileMaxQuads vertex quads): the
// tile's spin words live in LDS for the whole launch, and the work-group
// walks the sweeps and, in each, the colour classes in the sweep's order,
// its four waves sharing a class's quads, with a barrier between classes.
// Replica tiles never interact within a step, so no other synchronisation
// is needed; the decisions are those of k_sweep_pull (same fields, same
// Philox words, same thresholds), so the trajectory is the same, while a
// step is one launch instead of sweeps x classes.
// ---------------------------------------------------------------------------
constexpr int kTileMaxQuads = 512;      // 128 KB of LDS spin words: n <= 2048
constexpr int kTileWaves = 16;          // waves of a tile-resident work-group
constexpr int kTileLdsBytes = 150 * 1024;  // dynamic LDS: spins, table, one class's rows (8 KB static beside)

template <int JM>
__global__ void __launch_bounds__(kTileWaves * 64) k_sweep_tile(const Desc* __restrict__ D,
                                                                const uint64_t* __restrict__ map) {
  // LDS: [nq][64] spin words, the threshold table (kThrLds words), then the
  // current class's gathered rows (columns, then couplings; d.tile_rows
  // entries each at most)
  extern __shared__ uint32_t tl[];
  __shared__ int64_t red[kTileWaves][kLanes];
  __shared__ int32_t fred[kTileWaves];
  int inst, tile;
  if (!resolve(map, inst, tile)) return;
  const Desc& d = D[inst];
  const PAMC_GLOBAL RunState* __restrict__ st = gmem((const RunState*)d.st);
  const int nsw = st->nsweeps_now;
  if (!st->active || nsw <= 0) return;
  const int cur = st->cur;
  const int nq = d.nq;
  const int32_t Xt = (int32_t)st->table_x;
  PAMC_GLOBAL uint32_t* __restrict__ S = gmem(cur ? d.S1 : d.S0) + (size_t)tile * nq * kLanes;
  PAMC_GLOBAL int64_t* __restrict__ E = gmem(cur ? d.E1 : d.E0);
  const PAMC_GLOBAL uint32_t* __restrict__ thr_g = gmem((const uint32_t*)d.thr);
  const PAMC_GLOBAL int32_t* __restrict__ order = gmem((const int32_t*)d.order);
  const PAMC_GLOBAL int32_t* __restrict__ class_ptr = gmem(d.class_ptr);
  const PAMC_GLOBAL int32_t* __restrict__ grow = gmem(d.grow);
  const PAMC_GLOBAL int32_t* __restrict__ gcol = gmem(d.gcol);
  const PAMC_GLOBAL int32_t* __restrict__ gJ = gmem(d.gJ);
  uint32_t* Sl = tl;
  uint32_t* thr_s = tl + (size_t)nq * kLanes;
  int32_t* rc = reinterpret_cast<int32_t*>(thr_s + kThrLds);
  int32_t* rj = rc + d.tile_rows;
  for (int i = threadIdx.x; i < nq * kLanes; i += blockDim.x) Sl[i] = S[i];
  for (int i = threadIdx.x; i <= 2 * Xt; i += blockDim.x) thr_s[i] = thr_g[i];
  const int lane = threadIdx.x & 63;
  const int lane4 = 4 * lane;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t r = (uint32_t)(tile * kLanes + lane);
  const bool metropolis = d.rule == 1;
  int64_t dE = 0;
  int32_t nflip = 0;
  for (int sw_i = 0; sw_i < nsw; ++sw_i) {
    const uint32_t gs = st->gs + (uint32_t)sw_i;
    for (int p = 0; p < d.ncls; ++p) {
      const int cls = order[sw_i * d.ncls + p];
      const int v0 = class_ptr[cls], v1 = class_ptr[cls + 1];
      const int g0 = grow[v0], ng = grow[v1] - g0;
      __syncthreads();  // the previous class is done with the row buffer (and its spins are in)
      for (int i = threadIdx.x; i < ng; i += blockDim.x) {
        rc[i] = gcol[g0 + i];
        rj[i] = gJ[g0 + i];
      }
      __syncthreads();
      const int q0 = v0 >> 2, nqc = ((v1 + 3) >> 2) - q0;
      for (int qi = wave; qi < nqc; qi += kTileWaves) {
        const int q = q0 + qi;
        uint32_t sw = Sl[q * kLanes + lane];
        int32_t h[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int v = 4 * q + k;
          h[k] = 0;
          if (v < v0 || v >= v1) continue;
          const int e1 = grow[v + 1] - g0;
          for (int e = grow[v] - g0; e < e1; e += 4) {
            const i32x4 cj = *reinterpret_cast<const i32x4*>(rc + e);  // uniform: broadcast reads
            const i32x4 cJ = *reinterpret_cast<const i32x4*>(rj + e);
            const int j[4] = {cj.x, cj.y, cj.z, cj.w};
            const int32_t c[4] = {cJ.x, cJ.y, cJ.z, cJ.w};
            // the neighbour's word: j is its byte offset in the tile (plus
            // its byte index in modes 0 and 1), so one add per neighbour
            // addresses it
            uint32_t w[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
              w[u] = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(Sl) +
                                                        (JM == 2 ? j[u] : (j[u] & ~3)) + lane4);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (JM == 2) {
                h[k] = __builtin_amdgcn_sdot4((int)w[u], c[u], h[k], false);
              } else {
                const int32_t sv = __builtin_amdgcn_sbfe((int32_t)w[u], 8u * (uint32_t)(j[u] & 3), 8u);
                h[k] += JM == 1 ? __mul24(c[u], sv) : c[u] * sv;
              }
            }
          }
        }
        const u32x4 rnd = philox10((uint32_t)q, gs, r, kTagSweep, d.k0, d.k1);
        uint32_t flipmask = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int v = 4 * q + k;
          if (v < v0 || v >= v1) continue;
          const int32_t s = __builtin_amdgcn_sbfe((int32_t)sw, 8u * k, 8u);
          const int32_t x = __mul24(s, h[k]);
          const int32_t xi = min(max(x, -Xt), Xt) + Xt;
          const bool flip = (pick(rnd, k) < thr_s[xi]) || (metropolis && x <= 0);
          dE += flip ? (int64_t)x : 0;
          flipmask |= flip ? (0xFEu << (8 * k)) : 0u;
          nflip += __popcll(__ballot(flip));
        }
        if (flipmask) Sl[q * kLanes + lane] = sw ^ flipmask;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nq * kLanes; i += blockDim.x) S[i] = Sl[i];
  red[wave][lane] = 2 * dE;
  if (lane == 0) fred[wave] = nflip;
  __syncthreads();
  if (wave == 0) {  // the work-group owns its tile's replicas: no atomics
    int64_t sum = 0;
#pragma unroll
    for (int w = 0; w < kTileWaves; ++w) sum += red[w][lane];
    E[tile * kLanes + lane] += sum;
    if (d.flip_ctr && lane == 0) {
      int64_t f = 0;
      for (int w = 0; w < kTileWaves; ++w) f += fred[w];
      __hip_atomic_fetch_add((unsigned long long*)&d.flip_ctr[blockIdx.x & 255], (unsigned long long)f,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// The tile-resident step with the fields of a colour class computed on the
// matrix cores, for small instances with int8 couplings (at most
// kTmmaMaxN vertices): the class's fields for the tile's 64 replicas are
// h = J[class rows, :] . S, an int8 x int8 -> int32 product (exact: |h| <=
// 127 n), so a dense-ish graph costs one v_mfma_i32_16x16x64_i8 per 16
// rows, 16 replicas and 64 vertices instead of a gather per neighbour.
// The spins sit in LDS replica-major (int8 [64][npk + 16], the B operand);
// J sits in HBM as 16-row x 64-column fragments in the order the A operand
// wants them (1 KB per fragment: lane l holds bytes 16 (l / 16) .. + 15 of
// row l % 16).  Vertices of one class share no edge (J = 0 between them),
// so the product may read the class's spins while they change.  Each wave
// keeps one group of 16 replicas (wave % 4) and takes 16-row tiles of the
// class in turn; the product leaves in each lane the four fields of one
// vertex quad for one replica, exactly the unit of one Philox block, and
// the decisions are those of the other sweep kernels (same fields, words
// and thresholds), so the trajectory is the same.
// ---------------------------------------------------------------------------
constexpr int kComputeUnits = 256;      // MI355X
constexpr int64_t kCuLdsBytes = 160 * 1024;
constexpr int kTmmaMaxN = 1024;  // vertices (padded): 64 x 1040 B of LDS spins
constexpr int kTmmaMaxKs = kTmmaMaxN / 64;

// NW waves per work-group (16, or 8 so that two work-groups share a
// compute unit when a batch has enough of them).
template <int NW>
__global__ void __launch_bounds__(NW * 64) k_sweep_tmma(const Desc* __restrict__ D, const uint64_t* __restrict__ map) {
  extern __shared__ uint32_t tl[];  // int8 spins [64][rowb], then the threshold table
  __shared__ int64_t red[NW][kLanes];
  __shared__ int32_t fred[NW];
  int inst, tile;
  if (!resolve(map, inst, tile)) return;
  const Desc& d = D[inst];
  const PAMC_GLOBAL RunState* __restrict__ st = gmem((const RunState*)d.st);
  const int nsw = st->nsweeps_now;
  if (!st->active || nsw <= 0) return;
  const int cur = st->cur;
  const int nq = d.nq, nks = d.nks;
  const int rowb = 64 * nks + 16;  // bytes per replica row (padded against bank conflicts)
  const int32_t Xt = (int32_t)st->table_x;
  PAMC_GLOBAL uint32_t* __restrict__ S = gmem(cur ? d.S1 : d.S0) + (size_t)tile * nq * kLanes;
  PAMC_GLOBAL int64_t* __restrict__ E = gmem(cur ? d.E1 : d.E0);
  const PAMC_GLOBAL uint32_t* __restrict__ thr_g = gmem((const uint32_t*)d.thr);
  const PAMC_GLOBAL int32_t* __restrict__ order = gmem((const int32_t*)d.order);
  const PAMC_GLOBAL int32_t* __restrict__ class_ptr = gmem(d.class_ptr);
  const PAMC_GLOBAL int8_t* __restrict__ Jt = gmem(d.Jt);
  int8_t* Sb = reinterpret_cast<int8_t*>(tl);
  uint32_t* thr_s = tl + 16 * rowb;  // 64 rowb bytes
  // the tile's spin words into replica-major rows: word (q, l) holds the
  // bytes of vertices 4q .. 4q + 3 of replica l
  for (int i = threadIdx.x; i < nq * kLanes; i += blockDim.x)
    *reinterpret_cast<uint32_t*>(Sb + (i & 63) * rowb + 4 * (i >> 6)) = S[i];
  for (int i = threadIdx.x; i <= 2 * Xt; i += blockDim.x) thr_s[i] = thr_g[i];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int grp = wave & 3;                 // the wave's 16 replicas
  const int rl = 16 * grp + (lane & 15);    // the lane's replica in the tile
  const uint32_t r = (uint32_t)(tile * kLanes + rl);
  const int kq = lane >> 4;                 // the lane's quad within a 16-row tile
  const int8_t* brow = Sb + rl * rowb + 16 * kq;  // B operand: replica rl, bytes 16 kq ..
  const bool metropolis = d.rule == 1;
  int64_t dE = 0;
  int32_t nflip = 0;
  for (int sw_i = 0; sw_i < nsw; ++sw_i) {
    const uint32_t gs = st->gs + (uint32_t)sw_i;
    for (int p = 0; p < d.ncls; ++p) {
      const int cls = order[sw_i * d.ncls + p];
      const int v0 = class_ptr[cls], v1 = class_ptr[cls + 1];
      const int q0 = v0 >> 2, q1 = (v1 + 3) >> 2;  // the class's quads
      const int t0 = q0 >> 2, t1 = (q1 + 3) >> 2;  // its 16-row tiles
      __syncthreads();  // the previous class's spins are in
      for (int t = t0 + (wave >> 2); t < t1; t += NW / 4) {
        // every A fragment of the row tile first; the lane's random words
        // (they do not depend on the fields) while the fragments arrive;
        // then the products
        const PAMC_GLOBAL int8_t* arow = Jt + ((size_t)t * nks * 64 + lane) * 16;
        i32x4 av[kTmmaMaxKs];
#pragma unroll
        for (int ks = 0; ks < kTmmaMaxKs; ++ks)
          if (ks < nks) av[ks] = *reinterpret_cast<const PAMC_GLOBAL i32x4*>(arow + (size_t)ks * 1024);
        // the lane's quad: vertices 4q .. 4q + 3 of the tile, replica rl
        const int q = 4 * t + kq;
        const u32x4 rnd = philox10((uint32_t)q, gs, r, kTagSweep, d.k0, d.k1);
        __builtin_amdgcn_sched_barrier(0);
        i32x4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < kTmmaMaxKs; ++ks)
          if (ks < nks)
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[ks], *reinterpret_cast<const i32x4*>(brow + 64 * ks),
                                                        acc, 0, 0, 0);
        if (q < q0 || q >= q1) continue;
        uint32_t* wp = reinterpret_cast<uint32_t*>(Sb + rl * rowb + 4 * q);
        const uint32_t sw = *wp;
        uint32_t flipmask = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int v = 4 * q + k;
          if (v < v0 || v >= v1) continue;
          const int32_t s = __builtin_amdgcn_sbfe((int32_t)sw, 8u * k, 8u);
          const int32_t x = __mul24(s, acc[k]);
          const int32_t xi = min(max(x, -Xt), Xt) + Xt;
          const bool flip = (pick(rnd, k) < thr_s[xi]) || (metropolis && x <= 0);
          dE += flip ? (int64_t)x : 0;
          flipmask |= flip ? (0xFEu << (8 * k)) : 0u;
          nflip += flip ? 1 : 0;
        }
        if (flipmask) *wp = sw ^ flipmask;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nq * kLanes; i += blockDim.x)
    S[i] = *reinterpret_cast<const uint32_t*>(Sb + (i & 63) * rowb + 4 * (i >> 6));
  red[wave][lane] = 2 * dE;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nflip += __shfl_xor(nflip, o, 64);
  if (lane == 0) fred[wave] = nflip;
  __syncthreads();
  if (wave == 0) {  // replica rl = 16 (w % 4) + (l % 16): the waves w and lanes l holding it
    const int g = lane >> 4, c = lane & 15;
    int64_t sum = 0;
#pragma unroll
    for (int w = g; w < NW; w += 4)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) sum += red[w][16 * kk + c];
    E[tile * kLanes + lane] += sum;
    if (d.flip_ctr && lane == 0) {
      int64_t f = 0;
      for (int w = 0; w < NW; ++w) f += fred[w];
      __hip_atomic_fetch_add((unsigned long long*)&d.flip_ctr[blockIdx.x & 255], (unsigned long long)f,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// The same step with one work-group per 16-replica group of a tile (four
// per tile): a single instance spreads over four times the compute units,
// each holding a quarter of the tile's spins.  Wave w takes the class's
// 16-row tiles w, w + NW, ...; lane l's replica is 16 g + l % 16 and its
// quad 4 t + l / 16, as above.
template <int NW>
__global__ void __launch_bounds__(NW * 64) k_sweep_tmma_g(const Desc* __restrict__ D,
                                                          const uint64_t* __restrict__ map) {
  extern __shared__ uint32_t tl[];  // int8 spins [16][rowb], then the threshold table
  __shared__ int64_t red[NW][kLanes];
  __shared__ int32_t fred[NW];
  int inst, lb;
  if (!resolve(map, inst, lb)) return;
  const Desc& d = D[inst];
  const PAMC_GLOBAL RunState* __restrict__ st = gmem((const RunState*)d.st);
  const int nsw = st->nsweeps_now;
  if (!st->active || nsw <= 0) return;
  const int tile = lb >> 2, grp = lb & 3;
  const int cur = st->cur;
  const int nq = d.nq, nks = d.nks;
  const int rowb = 64 * nks + 16;  // bytes per replica row (padded against bank conflicts)
  const int32_t Xt = (int32_t)st->table_x;
  PAMC_GLOBAL uint32_t* __restrict__ S = gmem(cur ? d.S1 : d.S0) + (size_t)tile * nq * kLanes + 16 * grp;
  PAMC_GLOBAL int64_t* __restrict__ E = gmem(cur ? d.E1 : d.E0);
  const PAMC_GLOBAL uint32_t* __restrict__ thr_g = gmem((const uint32_t*)d.thr);
  const PAMC_GLOBAL int32_t* __restrict__ order = gmem((const int32_t*)d.order);
  const PAMC_GLOBAL int32_t* __restrict__ class_ptr = gmem(d.class_ptr);
  const PAMC_GLOBAL int8_t* __restrict__ Jt = gmem(d.Jt);
  int8_t* Sb = reinterpret_cast<int8_t*>(tl);
  uint32_t* thr_s = tl + 4 * rowb;  // 16 rowb bytes
  // the group's spin words (q, 16 grp + c) into replica-major rows
  for (int i = threadIdx.x; i < nq * 16; i += blockDim.x)
    *reinterpret_cast<uint32_t*>(Sb + (i & 15) * rowb + 4 * (i >> 4)) = S[(i >> 4) * kLanes + (i & 15)];
  for (int i = threadIdx.x; i <= 2 * Xt; i += blockDim.x) thr_s[i] = thr_g[i];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = lane & 15;                  // the lane's replica in the group
  const uint32_t r = (uint32_t)(tile * kLanes + 16 * grp + c);
  const int kq = lane >> 4;                 // the lane's quad within a 16-row tile
  const int8_t* brow = Sb + c * rowb + 16 * kq;  // B operand: replica c, bytes 16 kq ..
  const bool metropolis = d.rule == 1;
  int64_t dE = 0;
  int32_t nflip = 0;
  for (int sw_i = 0; sw_i < nsw; ++sw_i) {
    const uint32_t gs = st->gs + (uint32_t)sw_i;
    for (int p = 0; p < d.ncls; ++p) {
      const int cls = order[sw_i * d.ncls + p];
      const int v0 = class_ptr[cls], v1 = class_ptr[cls + 1];
      const int q0 = v0 >> 2, q1 = (v1 + 3) >> 2;  // the class's quads
      const int t0 = q0 >> 2, t1 = (q1 + 3) >> 2;  // its 16-row tiles
      __syncthreads();  // the previous class's spins are in
      for (int t = t0 + wave; t < t1; t += NW) {
        const PAMC_GLOBAL int8_t* arow = Jt + ((size_t)t * nks * 64 + lane) * 16;
        i32x4 av[kTmmaMaxKs];
#pragma unroll
        for (int ks = 0; ks < kTmmaMaxKs; ++ks)
          if (ks < nks) av[ks] = *reinterpret_cast<const PAMC_GLOBAL i32x4*>(arow + (size_t)ks * 1024);
        const int q = 4 * t + kq;
        const u32x4 rnd = philox10((uint32_t)q, gs, r, kTagSweep, d.k0, d.k1);
        __builtin_amdgcn_sched_barrier(0);
        i32x4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < kTmmaMaxKs; ++ks)
          if (ks < nks)
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(av[ks], *reinterpret_cast<const i32x4*>(brow + 64 * ks),
                                                        acc, 0, 0, 0);
        if (q < q0 || q >= q1) continue;
        uint32_t* wp = reinterpret_cast<uint32_t*>(Sb + c * rowb + 4 * q);
        const uint32_t sw = *wp;
        uint32_t flipmask = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int v = 4 * q + k;
          if (v < v0 || v >= v1) continue;
          const int32_t s = __builtin_amdgcn_sbfe((int32_t)sw, 8u * k, 8u);
          const int32_t x = __mul24(s, acc[k]);
          const int32_t xi = min(max(x, -Xt), Xt) + Xt;
          const bool flip = (pick(rnd, k) < thr_s[xi]) || (metropolis && x <= 0);
          dE += flip ? (int64_t)x : 0;
          flipmask |= flip ? (0xFEu << (8 * k)) : 0u;
          nflip += flip ? 1 : 0;
        }
        if (flipmask) *wp = sw ^ flipmask;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nq * 16; i += blockDim.x)
    S[(i >> 4) * kLanes + (i & 15)] = *reinterpret_cast<const uint32_t*>(Sb + (i & 15) * rowb + 4 * (i >> 4));
  red[wave][lane] = dE;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nflip += __shfl_xor(nflip, o, 64);
  if (lane == 0) fred[wave] = nflip;
  __syncthreads();
  if (wave == 0 && lane < 16) {  // replica 16 grp + lane: lanes lane, 16 + lane, ... of every wave
    int64_t sum = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w)
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) sum += red[w][16 * kk + lane];
    E[tile * kLanes + 16 * grp + lane] += 2 * sum;
    if (d.flip_ctr && lane == 0) {
      int64_t f = 0;
      for (int w = 0; w < NW; ++w) f += fred[w];
      __hip_atomic_fetch_add((unsigned long long*)&d.flip_ctr[blockIdx.x & 255], (unsigned long long)f,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// The same class phase with incremental fields: x = s*h from the field
// array; on a flip E += 2x and every neighbour field gets 2 J s_new by a
// coalesced no-return atomic.  Used where gathering is dearer (high degree,
// hub vertices).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sweep_push_body(const PAMC_GLOBAL int32_t* __restrict__ row_ptr,
                                                const PAMC_GLOBAL int32_t* __restrict__ col,
                                                const PAMC_GLOBAL int32_t* __restrict__ Jc,
                                                const PAMC_GLOBAL int32_t* __restrict__ class_ptr,
                                                const PAMC_GLOBAL int32_t* __restrict__ order,
                                                const PAMC_GLOBAL uint32_t* __restrict__ thr_g, const Desc& d,
                                                int lb, int sweep_idx, int phase) {
  __shared__ int64_t red[kSweepWaves][kLanes];
  __shared__ int32_t fred[kSweepWaves];
  __shared__ uint32_t thr_s[kThrLds];
  const PAMC_GLOBAL RunState* __restrict__ st = gmem((const RunState*)d.st);
  const int cur = st->cur;
  PAMC_GLOBAL uint32_t* __restrict__ S = gmem(cur ? d.S1 : d.S0);
  PAMC_GLOBAL int32_t* H = gmem(cur ? d.H1 : d.H0);
  PAMC_GLOBAL int64_t* __restrict__ E = gmem(cur ? d.E1 : d.E0);
  const int cls = order[sweep_idx * d.ncls + phase];
  const int v0 = class_ptr[cls], v1 = class_ptr[cls + 1];
  const int q0 = v0 >> 2;
  const int nqc = ((v1 + 3) >> 2) - q0;
  int tile, chunk0;
  group_chunk(d.T, lb, tile, chunk0);
  // a class whose quads fit one pass of the tile's work-groups at one quad
  // per wave takes one (a shorter chain per wave); larger ones the
  // instance's quads per wave
  const int qpw = (nqc + kSweepWaves - 1) / kSweepWaves <= d.sweep_stride ? 1 : d.qpw;
  if (chunk0 * (kSweepWaves * qpw) >= nqc) return;
  const uint32_t gs = st->gs + (uint32_t)sweep_idx;
  const int rule = d.rule;
  const int32_t Xt = (int32_t)st->table_x;
  const bool thr_lds = 2 * Xt + 1 <= kThrLds;
  if (thr_lds)
    for (int i = threadIdx.x; i <= 2 * Xt; i += blockDim.x) thr_s[i] = thr_g[i];
  __syncthreads();
  const uint32_t* __restrict__ thr = thr_lds ? thr_s : (const uint32_t*)thr_g;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t r = (uint32_t)(tile * kLanes + lane);
  const size_t hbase = (size_t)tile * d.np;
  int64_t dE = 0;
  int32_t nflip = 0;
  // the work-group's chunks of the class: chunk0, chunk0 + stride, ... (the
  // tile stays the same, so the energy sums stay per tile)
  for (int chunk = chunk0; chunk * (kSweepWaves * qpw) < nqc; chunk += d.sweep_stride) {
    // the spin words and fields of all of the wave's quads up front: the
    // vertices of one class are not neighbours, so no flip of this phase
    // changes them (v < np always)
    constexpr int kMaxQpw = 4;
    uint32_t swq[kMaxQpw];
    int32_t hqq[kMaxQpw][4];
#pragma unroll
    for (int i = 0; i < kMaxQpw; ++i) {
      const int qi = chunk * (kSweepWaves * qpw) + i * kSweepWaves + wave;
      if (i < qpw && qi < nqc) {
        const int q = q0 + qi;
        swq[i] = S[((size_t)tile * d.nq + q) * kLanes + lane];
#pragma unroll
        for (int k = 0; k < 4; ++k) hqq[i][k] = H[(hbase + 4 * q + k) * kLanes + lane];
      }
    }
#pragma unroll
    for (int i = 0; i < kMaxQpw; ++i) {
      if (i >= qpw) break;
      const int qi = chunk * (kSweepWaves * qpw) + i * kSweepWaves + wave;
      if (qi >= nqc) break;
      const int q = q0 + qi;
      const size_t sidx = ((size_t)tile * d.nq + q) * kLanes + lane;
      uint32_t sw = swq[i];
      const u32x4 rnd = philox10((uint32_t)q, gs, r, kTagSweep, d.k0, d.k1);
      const int32_t (&hq)[4] = hqq[i];
      bool dirty = false;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int v = 4 * q + k;
        if (v < v0 || v >= v1) continue;
        const int32_t h = hq[k];
        const int32_t s = (int32_t)(int8_t)(sw >> (8 * k));
        const int32_t x = s * h;
        const int32_t xi = x < -Xt ? -Xt : (x > Xt ? Xt : x);
        const uint32_t T = thr[xi + Xt];
        const bool flip = (rule == 1 && x <= 0) || (pick(rnd, k) < T);
        const int32_t snew = -s;
        if (flip) {
          dE += 2 * (int64_t)x;
          sw ^= (0xFEu << (8 * k));
          dirty = true;
          ++nflip;
        }
        if (__ballot(flip)) {
          const int e0 = row_ptr[v], e1 = row_ptr[v + 1];
          const int32_t dd = 2 * snew;
          for (int e = e0; e < e1; ++e) {
            const int j = col[e];
            const int32_t add = Jc[e] * dd;
            if (flip)
              __hip_atomic_fetch_add(&H[(hbase + j) * kLanes + lane], add, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      if (dirty) S[sidx] = sw;
    }
  }
  red[wave][lane] = dE;
  if (d.flip_ctr) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nflip += __shfl_xor(nflip, o, 64);
    if (lane == 0) fred[wave] = nflip;
  }
  reduce_energy_and_flips(red, fred, wave, lane, 1, tile, E, gmem(d.flip_ctr));
}

__global__ void __launch_bounds__(256) k_sweep_push(const Desc* __restrict__ D,
                                                  const uint64_t* __restrict__ map, int sweep_idx,
                                                  int phase) {
  int inst, lb;
  if (!resolve(map, inst, lb)) return;
  const Desc& d = D[inst];
  const PAMC_GLOBAL RunState* __restrict__ st = gmem((const RunState*)d.st);
  if (!st->active || sweep_idx >= st->nsweeps_now || phase >= d.ncls) return;
  sweep_push_body(gmem(d.row_ptr), gmem(d.col), gmem(d.J), gmem(d.class_ptr), gmem((const int32_t*)d.order),
                  gmem((const uint32_t*)d.thr), d, lb, sweep_idx, phase);
}

// ---------------------------------------------------------------------------
// Potts labels (Sec. "Max-3-Cut"; Eqs. 6-9; the cascaded K = 3 sampler of the
// Supplement).  A label word holds the labels (bytes 0..K-1) of the four
// vertices of a quad, like a spin word.  Visiting vertex v of replica r:
// the K-label field syn_k = sum_j J_vj [s_j = k] over the CSR row (Eq. 7),
// omega_k = e^{beta (syn_k - max syn)} from the step's table, then the
// comparisons of the paper's formulas multiplied through by their positive
// denominators (no division):
//   softmax: the k with the largest omega_k - (gamma u_k 2^-32) S, S = sum
//     omega (Eqs. 8-9: P_k - gamma U_k times S; lowest k on ties);
//   cascade: label 0 iff w0 - s12 > eta_1 (w0 + s12), s12 = w1 + w2 (the
//     p-bit tanh(Delta_1) > eta_1), else label 1 iff w1 - w2 > eta_2 s12,
//     else 2; eta = u 2^-31 - 1;
// u: the visit's words of its quad's Philox blocks (below).  Every operation
// is a correctly rounded binary64 operation in a fixed order (no
// contraction), so the choice is the same wherever it is computed.  The
// energy (Eq. 6) changes by -2 (syn_new - syn_old).
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ int32_t syn_of(const int32_t (&syn)[K], int k) {
  int32_t x = syn[0];
#pragma unroll
  for (int i = 1; i < K; ++i) x = k == i ? syn[i] : x;
  return x;
}

template <int K>
__device__ __forceinline__ int potts_choose(const int32_t (&syn)[K], const uint32_t (&u)[K],
                                            const double* __restrict__ tab, int32_t last, int rule, double gamma) {
  int32_t m = syn[0];
#pragma unroll
  for (int k = 1; k < K; ++k) m = max(m, syn[k]);
  double om[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int32_t dd = m - syn[k];
    om[k] = dd <= last ? tab[dd] : 0.0;
  }
  if constexpr (K == 3) {
    if (rule == 1) {
      const double s12 = om[1] + om[2];
      const double eta1 = (double)u[0] * (1.0 / 2147483648.0) - 1.0;
      if (om[0] - s12 > eta1 * (om[0] + s12)) return 0;
      const double eta2 = (double)u[1] * (1.0 / 2147483648.0) - 1.0;
      return om[1] - om[2] > eta2 * s12 ? 1 : 2;
    }
  }
  double S = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) S += om[k];
  int best = 0;
  double bs = om[0] - (gamma * ((double)u[0] * (1.0 / 4294967296.0))) * S;
#pragma unroll
  for (int k = 1; k < K; ++k) {
    const double sc = om[k] - (gamma * ((double)u[k] * (1.0 / 4294967296.0))) * S;
    if (sc > bs) {
      bs = sc;
      best = k;
    }
  }
  return best;
}

constexpr int kPottsTabLds = 1024;  // doubles of the weight table kept in LDS (8 KB: occupancy)

// K-label field of one vertex from the gathered CSR (rows padded to
// multiples of 4 entries with coupling 0; columns as the byte offset of the
// neighbour's label word in a tile plus its byte index), four neighbours per
// step: two 16-byte scalar loads and four buffer loads.
template <int K>
__device__ __forceinline__ void gather_labels(const PAMC_GLOBAL int32_t* __restrict__ gcol,
                                              const PAMC_GLOBAL int32_t* __restrict__ gJ, int e0, int e1,
                                              __amdgpu_buffer_rsrc_t Sr, int voff, int32_t (&syn)[K]) {
#pragma unroll
  for (int c = 0; c < K; ++c) syn[c] = 0;
  for (int e = e0; e < e1; e += 4) {
    const i32x4 cj = *reinterpret_cast<const PAMC_GLOBAL i32x4*>(gcol + e);
    const i32x4 cJ = *reinterpret_cast<const PAMC_GLOBAL i32x4*>(gJ + e);
    const int j[4] = {__builtin_amdgcn_readfirstlane(cj.x), __builtin_amdgcn_readfirstlane(cj.y),
                      __builtin_amdgcn_readfirstlane(cj.z), __builtin_amdgcn_readfirstlane(cj.w)};
    const int32_t c4[4] = {__builtin_amdgcn_readfirstlane(cJ.x), __builtin_amdgcn_readfirstlane(cJ.y),
                           __builtin_amdgcn_readfirstlane(cJ.z), __builtin_amdgcn_readfirstlane(cJ.w)};
    uint32_t w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = __builtin_amdgcn_raw_buffer_load_b32(Sr, voff, j[u] & ~3, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t lab = __builtin_amdgcn_ubfe(w[u], 8u * (uint32_t)(j[u] & 3), 8u);
#pragma unroll
      for (int c = 0; c < K; ++c) syn[c] += lab == (uint32_t)c ? c4[u] : 0;
    }
  }
}

// The same field when every |syn_k| fits W = 32 / K bits less one (X <
// 2^(W-1)): the K sums are kept as W-bit fields of one 32-bit integer, sum_j
// J_vj 2^(W label_j), so a neighbour costs a shift and an add instead of K
// compare-select-adds; the fields are taken apart at the end, each as the
// sign-extended low W bits of what remains (exact: the integer is
// sum_k syn_k 2^(W k) with every |syn_k| < 2^(W-1), which fits 32 bits).
template <int K>
__device__ __forceinline__ void gather_labels_packed(const PAMC_GLOBAL int32_t* __restrict__ gcol,
                                                     const PAMC_GLOBAL int32_t* __restrict__ gJ, int e0, int e1,
                                                     __amdgpu_buffer_rsrc_t Sr, int voff, int32_t (&syn)[K]) {
  constexpr int W = 32 / K;
  uint32_t acc = 0;
  for (int e = e0; e < e1; e += 4) {
    const i32x4 cj = *reinterpret_cast<const PAMC_GLOBAL i32x4*>(gcol + e);
    const i32x4 cJ = *reinterpret_cast<const PAMC_GLOBAL i32x4*>(gJ + e);
    const int j[4] = {__builtin_amdgcn_readfirstlane(cj.x), __builtin_amdgcn_readfirstlane(cj.y),
                      __builtin_amdgcn_readfirstlane(cj.z), __builtin_amdgcn_readfirstlane(cj.w)};
    const uint32_t c4[4] = {(uint32_t)__builtin_amdgcn_readfirstlane(cJ.x),
                            (uint32_t)__builtin_amdgcn_readfirstlane(cJ.y),
                            (uint32_t)__builtin_amdgcn_readfirstlane(cJ.z),
                            (uint32_t)__builtin_amdgcn_readfirstlane(cJ.w)};
    uint32_t w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = __builtin_amdgcn_raw_buffer_load_b32(Sr, voff, j[u] & ~3, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const uint32_t lab = __builtin_amdgcn_ubfe(w[u], 8u * (uint32_t)(j[u] & 3), 8u);
      acc += c4[u] << (W * lab);
    }
  }
  int32_t rest = (int32_t)acc;
#pragma unroll
  for (int k = 0; k < K - 1; ++k) {
    const int32_t f = (int32_t)((uint32_t)rest << (32 - W)) >> (32 - W);
    syn[k] = f;
    rest = (rest - f) >> W;
  }
  syn[K - 1] = rest;
}

template <int K>
__global__ void __launch_bounds__(256) k_sweep_potts(const Desc* __restrict__ D,
                                                   const uint64_t* __restrict__ map, int sweep_idx,
                                                   int phase) {
  __shared__ int64_t red[kSweepWaves][kLanes];
  __shared__ int32_t fred[kSweepWaves];
  __shared__ double tab_s[kPottsTabLds];
  int inst, lb;
  if (!resolve(map, inst, lb)) return;
  const Desc& d = D[inst];
  const PAMC_GLOBAL RunState* __restrict__ st = gmem((const RunState*)d.st);
  if (!st->active || sweep_idx >= st->nsweeps_now || phase >= d.ncls) return;
  const PAMC_GLOBAL int32_t* __restrict__ grow = gmem(d.grow);
  const PAMC_GLOBAL int32_t* __restrict__ gcol = gmem(d.gcol);
  const PAMC_GLOBAL int32_t* __restrict__ gJ = gmem(d.gJ);
  const PAMC_GLOBAL int32_t* __restrict__ class_ptr = gmem(d.class_ptr);
  const int cur = st->cur;
  PAMC_GLOBAL uint32_t* __restrict__ S = gmem(cur ? d.S1 : d.S0);
  PAMC_GLOBAL int64_t* __restrict__ E = gmem(cur ? d.E1 : d.E0);
  const int cls = gmem((const int32_t*)d.order)[sweep_idx * d.ncls + phase];
  const int v0 = class_ptr[cls], v1 = class_ptr[cls + 1];
  const int q0 = v0 >> 2;
  const int nqc = ((v1 + 3) >> 2) - q0;
  int tile, chunk;
  group_chunk(d.T, lb, tile, chunk);
  if (chunk * (kSweepWaves * d.qpw) >= nqc) return;
  const uint32_t gs = st->gs + (uint32_t)sweep_idx;
  const int32_t last = (int32_t)st->table_x;
  const bool lds = last < kPottsTabLds;
  if (lds)
    for (int i = threadIdx.x; i <= last; i += blockDim.x) tab_s[i] = d.ptab[i];
  __syncthreads();
  const double* __restrict__ tab = lds ? tab_s : (const double*)d.ptab;
  const int rule = d.potts_rule;
  const double gamma = d.potts_gamma;
  const bool packed = d.X < (1 << (32 / K - 1));
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t r = (uint32_t)(tile * kLanes + lane);
  const uint32_t tstride = (uint32_t)d.nq * kLanes;
  const __amdgpu_buffer_rsrc_t Sr = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(S + (size_t)tile * tstride), (short)0, (int)(tstride * 4), kBufferWord3);
  const int voff = lane * 4;
  int64_t dE = 0;
  int32_t nflip = 0;
  for (int i = 0; i < d.qpw; ++i) {
    const int qi = chunk * (kSweepWaves * d.qpw) + i * kSweepWaves + wave;
    if (qi >= nqc) break;
    const int q = q0 + qi;
    uint32_t sw = __builtin_amdgcn_raw_buffer_load_b32(Sr, voff, q * (kLanes * 4), 0);
    const uint32_t sw0 = sw;
    // the four fields first (the class's vertices do not see each other)
    int32_t synq[4][K];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int v = 4 * q + k;
      const bool in = v >= v0 && v < v1;
      if (packed)
        gather_labels_packed<K>(gcol, gJ, in ? grow[v] : 0, in ? grow[v + 1] : 0, Sr, voff, synq[k]);
      else
        gather_labels<K>(gcol, gJ, in ? grow[v] : 0, in ? grow[v + 1] : 0, Sr, voff, synq[k]);
    }
    // uniform words: W per visit (K, or 2 for the cascade); the quad's
    // visits share W Philox blocks (quad, sweep, replica, POTTS | b << 8),
    // read as one sequence, vertex k of the quad taking words k W .. k W + W-1
    uint32_t uw[4 * K];
    const bool cascade = K == 3 && rule == 1;
#pragma unroll
    for (int b = 0; b < K; ++b) {
      if (b < 2 || !cascade) {
        const u32x4 w = philox10((uint32_t)q, gs, r, kTagPotts | ((uint32_t)b << 8), d.k0, d.k1);
        uw[4 * b] = w.a;
        uw[4 * b + 1] = w.b;
        uw[4 * b + 2] = w.c;
        uw[4 * b + 3] = w.d;
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int v = 4 * q + k;
      if (v >= v0 && v < v1) {
        int32_t syn[K];
#pragma unroll
        for (int c = 0; c < K; ++c) syn[c] = synq[k][c];
        uint32_t u[K];
#pragma unroll
        for (int c = 0; c < K; ++c) u[c] = cascade ? (c < 2 ? uw[2 * k + c] : 0u) : uw[K * k + c];
        const int old = (int)((sw >> (8 * k)) & 0xFFu);
        const int nw = potts_choose<K>(syn, u, tab, last, rule, gamma);
        if (nw != old) {
          dE += -2 * (int64_t)(syn_of<K>(syn, nw) - syn_of<K>(syn, old));
          sw = (sw & ~(0xFFu << (8 * k))) | ((uint32_t)nw << (8 * k));
          ++nflip;
        }
      }
    }
    if (sw != sw0) __builtin_amdgcn_raw_buffer_store_b32(sw, Sr, voff, q * (kLanes * 4), 0);
  }
  red[wave][lane] = dE;
  if (d.flip_ctr) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) nflip += __shfl_xor(nflip, o, 64);
    if (lane == 0) fred[wave] = nflip;
  }
  reduce_energy_and_flips(red, fred, wave, lane, 1, tile, E, gmem(d.flip_ctr));
}

// ---------------------------------------------------------------------------
// Population initialisation (Algorithm 1, initialization): spins uniform from
// Philox(quad, 0, replica, INIT) (spin +1 iff the word < 2^31); then local
// fields by Eq. 3 and energies H = -1/2 sum s h.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_init_spins(const Desc* __restrict__ D,
                                                    const uint64_t* __restrict__ map) {
  int inst, lb;
  if (!resolve(map, inst, lb)) return;
  const Desc& d = D[inst];
  const size_t total = (size_t)d.T * d.nq * kLanes;
  for (size_t i = (size_t)lb * blockDim.x + threadIdx.x; i < total; i += (size_t)kInitBlocks * blockDim.x) {
    const int lane = (int)(i & 63);
    const size_t tq = i >> 6;
    const int q = (int)(tq % d.nq);
    const int tile = (int)(tq / d.nq);
    const uint32_t r = (uint32_t)(tile * kLanes + lane);
    const u32x4 w = philox10((uint32_t)q, 0u, r, kTagInit, d.k0, d.k1);
    uint32_t sw = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int v = 4 * q + k;
      int8_t s = 0;
      if (d.potts_K)  // label floor(u K / 2^32)
        s = v < d.n ? (int8_t)(((uint64_t)pick(w, k) * (uint64_t)d.potts_K) >> 32) : (int8_t)0;
      else if (v < d.n)
        s = pick(w, k) < 0x80000000u ? (int8_t)1 : (int8_t)-1;
      sw |= (uint32_t)(uint8_t)s << (8 * k);
    }
    d.S0[i] = sw;
    if (q == 0) d.F0[r] = (int32_t)r;
  }
}

// h = J s per (tile, vertex) row of buffer `buf` (-1: the current one);
// writes H (Hout if given, else the instance's field array if it has one)
// and, if asked, accumulates sum s h into E.  Work item = (64-vertex chunk,
// tile), dealt to the instance's min(items, kFieldBlocks) work-groups.
__global__ void __launch_bounds__(256) k_init_fields(const Desc* __restrict__ D,
                                                     const uint64_t* __restrict__ map, int32_t buf,
                                                     int32_t* Hout, int32_t accumulate_energy) {
  __shared__ int64_t red[4][kLanes];
  int inst, lb;
  if (!resolve(map, inst, lb)) return;
  const Desc& d = D[inst];
  const int b = buf < 0 ? d.st->cur : buf;
  const uint32_t* S = b ? d.S1 : d.S0;
  int32_t* H = Hout ? Hout : (b ? d.H1 : d.H0);
  int64_t* E = accumulate_energy ? (b ? d.E1 : d.E0) : nullptr;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t items = (int64_t)d.T * ((d.n + 63) / 64);
  const int64_t nblocks = items < kFieldBlocks ? items : kFieldBlocks;
  for (int64_t it = lb; it < items; it += nblocks) {
    const int tile = (int)(it % d.T);
    const int vchunk = (int)(it / d.T);
    int64_t acc = 0;
    for (int v = vchunk * 64 + wave; v < d.n && v < (vchunk + 1) * 64; v += 4) {
      if (d.potts_K) {
        // Potts labels (Eq. 6): sum_j J_vj (2 delta(s_v, s_j) - 1); no fields
        const int32_t lv = spin_at(S, d.nq, tile, v, lane);
        for (int e = d.row_ptr[v]; e < d.row_ptr[v + 1]; ++e)
          acc += spin_at(S, d.nq, tile, d.col[e], lane) == lv ? d.J[e] : -d.J[e];
        if (H) H[((size_t)tile * d.np + v) * kLanes + lane] = 0;
        continue;
      }
      // four independent sums, so that a long (hub) row has several spin
      // reads in flight rather than one at a time
      const int e0 = d.row_ptr[v], e1 = d.row_ptr[v + 1];
      int64_t hp[4] = {0, 0, 0, 0};
      int e = e0;
      for (; e + 4 <= e1; e += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) hp[u] += (int64_t)d.J[e + u] * spin_at(S, d.nq, tile, d.col[e + u], lane);
      }
      for (; e < e1; ++e) hp[0] += (int64_t)d.J[e] * spin_at(S, d.nq, tile, d.col[e], lane);
      const int64_t h = (hp[0] + hp[1]) + (hp[2] + hp[3]);
      if (H) H[((size_t)tile * d.np + v) * kLanes + lane] = (int32_t)h;
      if (!Hout && d.nhub && (v == d.hub_v0 || v == d.hub_v1))  // the kept hub fields
        (b ? d.HF1 : d.HF0)[(v == d.hub_v0 ? 0 : 1) * d.R + tile * kLanes + lane] = (int32_t)h;
      acc += h * spin_at(S, d.nq, tile, v, lane);
    }
    __syncthreads();
    red[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && E) {
      const int64_t t = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
      if (t != 0)
        __hip_atomic_fetch_add((unsigned long long*)&E[tile * kLanes + lane], (unsigned long long)t,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// E currently holds sum_v s_v h_v (= 2 sum_{i<j} J s s; Potts labels: 2
// sum_{i<j} J (2 delta - 1)); H = -that / 2.  The best configuration starts
// with cut 0: all spins +1, or all labels 0.  One work-group per instance.
__global__ void __launch_bounds__(256) k_init_finish(const Desc* __restrict__ D) {
  const Desc& d = D[blockIdx.x];
  for (int i = threadIdx.x; i < d.R; i += blockDim.x) d.E0[i] = -(d.E0[i] / 2);
  for (int v = threadIdx.x; v < d.np; v += blockDim.x) d.best[v] = d.potts_K ? 0 : 1;
  if (threadIdx.x == 0) {
    RunState* st = d.st;
    st->mstar = 0;
    st->cur = 0;
    st->gs = st->g_rs = st->g_cl = 0;
    st->stopped = 0;
    st->active = 0;
    st->steps_run = 0;
  }
}

// Population loaded by the host into buffer 0: E holds sum_v s_v h_v (Potts
// labels: 2 sum_{i<j} J (2 delta - 1)); H = -that / 2, and buffer 0 becomes
// the current one.  One work-group per instance.
__global__ void __launch_bounds__(256) k_load_finish(const Desc* __restrict__ D) {
  const Desc& d = D[blockIdx.x];
  for (int i = threadIdx.x; i < d.R; i += blockDim.x) d.E0[i] = -(d.E0[i] / 2);
  if (threadIdx.x == 0) d.st->cur = 0;
}

// ---------------------------------------------------------------------------
// Controller kernels (one thread per instance): Algorithm 1's decisions.
// ---------------------------------------------------------------------------
__global__ void k_anneal_setup(const Desc* __restrict__ D, const Schedule* __restrict__ sched,
                               const int32_t* __restrict__ idx, int32_t count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  RunState* st = D[idx ? idx[i] : i].st;
  const Schedule s = sched[i];
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
  st->stopped = 0;
  st->active = 0;
  st->dh_every = s.dh_every;
  st->dh_sum = 0;
  st->t_start = wall_clock64();
  st->t_last = st->t_start;
  if (s.resume) {  // the run goes on from the controller it holds
    st->t_reached = st->step_reached >= 0 ? st->t_start : 0;
    return;
  }
  st->z = 1;
  st->cycle = 0;
  st->beta = s.beta0;
  st->delta = s.dbeta;
  st->enable = 0;
  st->cooldown = 0;
  st->hist_len = 0;
  st->step_reached = -1;
  st->steps_run = 0;
  st->sum_lnq = 0.0;
  st->last_lnq = 0.0;
  st->n_cluster_moves = st->n_reheats = st->n_reversals = st->n_restarts = 0;
  st->t_reached = 0;
}

// Decisions of a run's beta step (Algorithm 1), by one thread per instance.
__device__ __forceinline__ void begin_step(const Desc& d) {
  RunState* st = d.st;
  if (st->stopped || st->steps_run >= st->steps || (st->stop_at_target && st->mstar >= st->target)) {
    st->stopped = 1;
    st->active = 0;
    return;
  }
  st->active = 1;
  st->step = st->steps_run;
  st->do_resample = (st->z > 1 && st->resample) ? 1 : 0;
  // cluster moves are defined for Ising spins only
  st->do_cluster = (st->do_resample && st->augmented && st->enable && st->cooldown == 0 && !d.potts_K) ? 1 : 0;
  st->rs_delta = st->delta;
  st->sweep_beta = st->beta;
  st->nsweeps_now = st->sweeps;
  st->cl_n_top = st->n_top;
  st->cl_trials = st->mis_trials;
  st->table_x = d.potts_K ? potts_table_last(st->beta, d.X) : table_halfwidth(st->beta, d.X);
  st->last_lnq = 0.0;
}

__global__ void k_step_begin(const Desc* __restrict__ D, int32_t ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) begin_step(D[i]);
}

// Primitive calls: one data-parallel action outside a run.
__global__ void k_prim_set(const Desc* __restrict__ D, int32_t ninst, int32_t kind, double value,
                           int32_t n_top, int32_t trials, int32_t nsweeps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  RunState* st = D[i].st;
  st->active = 1;
  st->do_resample = kind == 1;
  st->do_cluster = kind == 2;
  st->rs_delta = value;
  st->sweep_beta = value;
  st->nsweeps_now = nsweeps;
  st->cl_n_top = n_top;
  st->cl_trials = trials;
  st->table_x = D[i].potts_K ? potts_table_last(value, D[i].X) : table_halfwidth(value, D[i].X);
  st->last_lnq = 0.0;
}

// After resampling / cluster move: switch population buffers and advance the
// stream counters; in a run also apply Algorithm 1's "enable <- false;
// cooldown <- tau" after a cluster move.
__device__ __forceinline__ void commit_step(const Desc& d, int32_t in_run) {
  RunState* st = d.st;
  if (!st->active) return;
  if (st->do_resample) {
    st->cur ^= 1;
    st->g_rs += 1;
    if (in_run) {
      st->sum_lnq += st->last_lnq;
      if (st->step < d.tr_cap) d.tr_lnq[st->step] = st->last_lnq;
    }
  } else if (in_run && st->step < d.tr_cap) {
    d.tr_lnq[st->step] = 0.0;
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

__global__ void k_commit(const Desc* __restrict__ D, int32_t ninst, int32_t in_run) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) commit_step(D[i], in_run);
}

// Threshold table for the step's beta (entries x = -Xt..Xt) and the class
// order of each of the step's sweeps: a Fisher-Yates shuffle driven by
// Philox(i, sweep, 0, ORDER), j = floor(u (i+1) / 2^32).  With commit >= 0
// the instance's first block also commits the step's resampling / cluster
// move (commit = in_run); no field read here is changed by that.
__global__ void __launch_bounds__(256) k_thresholds(const Desc* __restrict__ D,
                                                    const uint64_t* __restrict__ map, int32_t commit) {
  int inst, lb;
  if (!resolve(map, inst, lb)) return;
  const Desc& d = D[inst];
  const RunState* st = d.st;
  if (!st->active) return;
  if (commit >= 0 && lb == 0 && threadIdx.x == 0) commit_step(d, commit);
  const int64_t Xt = st->table_x;
  const double beta = st->sweep_beta;
  if (d.potts_K) {  // e^{beta (syn_k - max syn)} for max syn - syn_k = i
    for (int64_t i = (int64_t)lb * blockDim.x + threadIdx.x; i <= Xt; i += (int64_t)kThrBlocks * blockDim.x)
      d.ptab[i] = exp_cw(beta * (double)(-i));
  } else {
    for (int64_t i = (int64_t)lb * blockDim.x + threadIdx.x; i <= 2 * Xt; i += (int64_t)kThrBlocks * blockDim.x)
      d.thr[i] = flip_threshold(beta, d.rule, i - Xt);
  }
  if (lb == 0 && d.ncls > 0) {
    const int nsw = min(st->nsweeps_now, d.order_cap);
    for (int s = threadIdx.x; s < nsw; s += blockDim.x) {
      int32_t* o = d.order + (size_t)s * d.ncls;
      for (int k = 0; k < d.ncls; ++k) o[k] = k;
      if (d.shuffle) {
        const uint32_t gs = st->gs + (uint32_t)s;
        for (int i = d.ncls - 1; i >= 1; --i) {
          const u32x4 w = philox10((uint32_t)i, gs, 0u, kTagOrder, d.k0, d.k1);
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
// Block-wide helpers for the 1024-thread per-instance kernels: shuffles
// within each wave, then the 16 wave results through LDS.
// ---------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ V block_excl_scan(V x, V* part16) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  V inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const V y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) part16[wv] = inc;
  __syncthreads();
  V off = 0;
  for (int i = 0; i < wv; ++i) off += part16[i];
  __syncthreads();
  return off + inc - x;
}

// Stagnation classes of the recent-progress history (Sec. "Augmented PAMC"),
// from the distinct M* values in its short (ds) and long (dl) tails: few
// distinct values in both tails is a strong stall, in the short tail only a
// mild one, otherwise the search still progresses.
enum : int { kStagNone = 0, kStagProgress = 1, kStagMild = 2, kStagStrong = 3 };
__device__ __forceinline__ int stagnation_class(int ds, int dl, int max_ds, int max_dl) {
  if (ds > max_ds) return kStagProgress;
  return dl <= max_dl ? kStagStrong : kStagMild;
}

// ---------------------------------------------------------------------------
// Best cut (Algorithm 1: M* <- max(M*, max Cut(P)), lowest slot on ties),
// then, in a run, the recent-progress history, the adaptive temperature rule
// and the schedule advance.  One work-group per instance; the distinct
// counts over the two history windows are taken by one thread per entry.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_step_end(const Desc* __restrict__ D, int32_t in_run) {
  __shared__ int64_t bc[16];
  __shared__ int32_t bs[16];
  __shared__ int64_t hs[kHistCap];
  const Desc& a = D[blockIdx.x];
  RunState* st = a.st;
  if (!st->active) return;
  // every thread reads the state it needs before the first barrier; thread
  // 0 writes it only after the last one
  const int cur = st->cur;
  const int64_t mstar_old = st->mstar;
  const int L0 = st->hist_len, wl = st->win_long, ws = st->win_short;
  const bool eval_ok = st->augmented && st->cooldown == 0;
  const int64_t* E = cur ? a.E1 : a.E0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int64_t c = INT64_MIN;
  int32_t cs = 0x7FFFFFFF;
  for (int r = tid; r < a.R; r += blockDim.x) {
    const int64_t cut = (a.W - E[r]) / 2;
    if (cut > c) { c = cut; cs = r; }  // r increases: ties keep the lower slot
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t c2 = __shfl_xor(c, o, 64);
    const int32_t s2 = __shfl_xor(cs, o, 64);
    if (c2 > c || (c2 == c && s2 < cs)) { c = c2; cs = s2; }
  }
  if (lane == 0) { bc[wv] = c; bs[wv] = cs; }
  __syncthreads();
  int64_t m = bc[0];
  int32_t slot = bs[0];
  for (int i = 1; i < 16; ++i)
    if (bc[i] > m || (bc[i] == m && bs[i] < slot)) { m = bc[i]; slot = bs[i]; }
  const bool improved = m > mstar_old;
  if (improved) {
    if (a.dense) {
      const int8_t* Dsp = (cur ? a.D1 : a.D0) + (size_t)slot * a.np;
      for (int v = tid; v < a.np; v += blockDim.x) a.best[v] = Dsp[v];
    } else {
      // one spin word (4 spins) per thread and step
      const uint32_t* S = cur ? a.S1 : a.S0;
      const int tile = slot >> 6, sl = slot & 63;
      for (int q = tid; q < a.nq; q += blockDim.x)
        reinterpret_cast<uint32_t*>(a.best)[q] = S[((size_t)tile * a.nq + q) * kLanes + sl];
    }
  }
  if (!in_run) {
    if (tid == 0 && improved) {
      st->mstar = m;
      st->best_slot = slot;
    }
    return;
  }
  const int64_t ms = improved ? m : mstar_old;
  // recent-progress history: the oldest value leaves once win_long are
  // held, then M* is appended
  const int drop = L0 >= wl ? 1 : 0;
  const int L = L0 - drop + 1;
  if (tid < L - 1) hs[tid] = st->hist[tid + drop];
  if (tid == L - 1) hs[tid] = ms;
  __syncthreads();
  if (tid < L) st->hist[tid] = hs[tid];
  int ds = 0, dl = 0;
  if (eval_ok && L >= wl) {  // uniform
    // entry tid counts for a window when no earlier entry of that window
    // holds the same value
    bool first_s = tid >= L - ws && tid < L, first_l = tid >= L - wl && tid < L;
    if (first_l) {
      const int64_t v = hs[tid];
      for (int j = L - wl; j < tid; ++j)
        if (hs[j] == v) {
          first_l = false;
          if (j >= L - ws) first_s = false;
        }
    }
    ds = __syncthreads_count(first_s);
    dl = __syncthreads_count(first_l);
  }
  if (tid != 0) return;
  if (improved) {
    st->mstar = m;
    st->best_slot = slot;
  }
  st->hist_len = L;
  int32_t ev = (st->do_resample ? 1 : 0) | (st->do_cluster ? 2 : 0);
  const uint64_t now = wall_clock64();
  if (st->step_reached < 0 && ms >= st->target) {
    st->step_reached = st->step;
    st->t_reached = now;
  }
  // the history's stagnation class picks the temperature action (see
  // stagnation_class), then the schedule moves on
  switch (eval_ok && L >= wl ? stagnation_class(ds, dl, st->max_ds, st->max_dl) : kStagNone) {
    case kStagStrong:  // reheat and arm the cluster move
      st->beta = st->reheat * st->beta;
      st->delta = st->dbeta;
      st->enable = 1;
      ev |= 4;
      st->n_reheats += 1;
      break;
    case kStagMild:  // run the schedule backwards while above beta0
      if (st->beta > st->beta0) {
        st->delta = -st->dbeta;
        ev |= 8;
        st->n_reversals += 1;
      } else if (st->literal_break) {
        st->stopped = 1;
      } else {
        st->delta = st->dbeta;
      }
      break;
    case kStagProgress:
      st->delta = st->dbeta;
      break;
    default:
      break;
  }
  const bool restart = st->z_rst > 0 && st->z >= st->z_rst;
  if (restart) {  // schedule, arming, cooldown and history start over
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
  st->t_last = now;
  if (st->step < a.tr_cap) {
    a.tr_mstar[st->step] = ms;
    a.tr_beta[st->step] = st->sweep_beta;
    a.tr_events[st->step] = ev;
    a.tr_time[st->step] = now;
  }
  if (st->stop_at_target && ms >= st->target) st->stopped = 1;
  if (st->steps_run >= st->steps) st->stopped = 1;
}

__global__ void k_advance_sweeps(const Desc* __restrict__ D, int32_t ninst, int32_t nsweeps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  D[i].st->gs += (uint32_t)nsweeps;
  D[i].st->active = 0;
}

__global__ void k_deactivate(const Desc* __restrict__ D, int32_t ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) D[i].st->active = 0;
}

// Per-instance status words for the host: bit 0 stopped, bits 1.. steps run.
__global__ void k_status(const Desc* __restrict__ D, int32_t ninst, int32_t* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) out[i] = (D[i].st->steps_run << 1) | (D[i].st->stopped ? 1 : 0);
}

// ---------------------------------------------------------------------------
// Targets of the non-local cluster move: the n_top slots with the lowest
// (E, slot), by a radix select on E - min E; they are listed in slot order
// (each target's move depends on its slot only).
// ---------------------------------------------------------------------------
// LDS of the target selection (declared by the calling kernel).
struct SelectLds {
  uint32_t hist[256];
  uint64_t part_u[16];
  int32_t part_i[16];
  uint64_t pick_prefix;
  int32_t pick_want;
};

// Energy of slot r of the population the cluster move acts on: E[r], or,
// right after the resampling draw, the energy of r's parent.
__device__ __forceinline__ int64_t target_energy(const int64_t* E, const int32_t* parent, int r) {
  return E[parent ? parent[r] : r];
}

// Called by all 1024 threads of the work-group.
__device__ __forceinline__ void select_cluster_targets(const Desc& d, const RunState* st, const int64_t* E,
                                       const int32_t* parent, SelectLds& L) {
  uint32_t* hist = L.hist;
  uint64_t* part_u = L.part_u;
  int32_t* part_i = L.part_i;
  const int R = d.R;
  // no targets without scratch (a move with no trials flips nothing)
  const int n_top = (d.cl_targets && st->cl_trials > 0) ? min(st->cl_n_top, R) : 0;
  if (n_top <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // a contiguous chunk of slots per thread, keys E - min E as unsigned
  constexpr int kPer = kRsMaxR / 1024;
  const int per = (R + 1023) >> 10;
  const int r0 = min(R, tid * per), r1 = min(R, r0 + per);
  int64_t e[kPer];
  int64_t emin = INT64_MAX;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    e[i] = r0 + i < r1 ? target_energy(E, parent, r0 + i) : INT64_MAX;
    emin = e[i] < emin ? e[i] : emin;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t y = __shfl_xor(emin, o, 64);
    emin = y < emin ? y : emin;
  }
  if (lane == 0) part_u[wv] = (uint64_t)emin;
  __syncthreads();
  emin = (int64_t)part_u[0];
  for (int i = 1; i < 16; ++i) emin = (int64_t)part_u[i] < emin ? (int64_t)part_u[i] : emin;
  __syncthreads();
  uint64_t key[kPer], kmax = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    key[i] = (uint64_t)e[i] - (uint64_t)emin;
    if (r0 + i < r1 && key[i] > kmax) kmax = key[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t y = __shfl_xor(kmax, o, 64);
    kmax = y > kmax ? y : kmax;
  }
  if (lane == 0) part_u[wv] = kmax;
  __syncthreads();
  kmax = part_u[0];
  for (int i = 1; i < 16; ++i) kmax = part_u[i] > kmax ? part_u[i] : kmax;
  // radix select, 8 bits a pass from the highest used bit: t = the key of
  // the n_top-th smallest (E, slot); want = how many slots with key t are
  // taken (the lowest ones)
  const int nbits = kmax ? 64 - __clzll((long long)kmax) : 0;
  uint64_t t = 0;
  int want = n_top;
  for (int s = ((nbits + 7) / 8) * 8 - 8; s >= 0; s -= 8) {
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kPer; ++i)
      if (r0 + i < r1 && (s + 8 >= 64 || ((key[i] ^ t) >> (s + 8)) == 0))
        atomicAdd(&hist[(key[i] >> s) & 255u], 1u);
    __syncthreads();
    if (wv == 0) {
      uint32_t h[4], tot = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) { h[j] = hist[4 * lane + j]; tot += h[j]; }
      uint32_t inc = tot;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
      }
      uint32_t cum = inc - tot;
      if (cum < (uint32_t)want && (uint32_t)want <= inc) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (cum + h[j] >= (uint32_t)want) {
            L.pick_prefix = t | ((uint64_t)(4 * lane + j) << s);
            L.pick_want = want - (int)cum;
            break;
          }
          cum += h[j];
        }
      }
    }
    __syncthreads();
    t = L.pick_prefix;
    want = L.pick_want;
  }
  // selected: key < t, or key == t among the first `want` such slots
  int neq = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) neq += (r0 + i < r1 && key[i] == t) ? 1 : 0;
  int eq_before = block_excl_scan<int32_t>(neq, part_i);
  bool sel[kPer];
  int nsel = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    sel[i] = false;
    if (r0 + i < r1) {
      if (key[i] < t) sel[i] = true;
      else if (key[i] == t) sel[i] = eq_before++ < want;
    }
    nsel += sel[i] ? 1 : 0;
  }
  int pos = block_excl_scan<int32_t>(nsel, part_i);
#pragma unroll
  for (int i = 0; i < kPer; ++i)
    if (sel[i]) d.cl_targets[pos++] = r0 + i;
}

// ---------------------------------------------------------------------------
// Resampling (Eqs. 1-2), one work-group per instance.  Weights relative to
// the extreme energy, w_r = e^{-Delta (E_r - E_ref)} in binary64; ln Q =
// -Delta E_ref + ln sum w - ln R.  Selection is exact integer arithmetic:
// q_r = floor(w_r 2^48), inclusive prefix P, child k draws a 64-bit Philox
// word u, y = floor(u Q / 2^64), parent = least j with P_j > y; children are
// then laid out by parent (counting sort).
// ---------------------------------------------------------------------------
// In a run (fused = 1) the kernel first takes the step's decisions and,
// when the step makes a cluster move, ends by selecting its targets from the
// children's energies.
__global__ void __launch_bounds__(1024) k_rs_select(const Desc* __restrict__ D, int32_t fused) {
  // the prefix P in LDS for the children's searches, then the same space
  // holds the number of children of each slot
  extern __shared__ uint64_t P[];
  __shared__ int64_t part_m[16];
  __shared__ uint64_t part_u[16];
  __shared__ double part_d[16];
  __shared__ int32_t part_i[16];
  __shared__ SelectLds L;
  const Desc& a = D[blockIdx.x];
  RunState* st = a.st;
  if (fused) {
    if (threadIdx.x == 0) begin_step(a);
    __syncthreads();
  }
  if (!st->active || !st->do_resample) return;
  const int64_t* E = st->cur ? a.E1 : a.E0;
  // Potts labels: the update of Eq. 8 at beta leaves e^{-(beta/2) E}
  // invariant for the Eq. 6 energy, so the weights use Delta/2
  const double delta = a.potts_K ? 0.5 * st->rs_delta : st->rs_delta;
  const bool lowest = delta >= 0;  // reference energy: min for delta >= 0, max otherwise
  const int R = a.R;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  int64_t m = E[0];
  for (int r = tid; r < R; r += 1024) {
    const int64_t e = E[r];
    if (lowest ? e < m : e > m) m = e;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int64_t y = __shfl_xor(m, o, 64);
    if (lowest ? y < m : y > m) m = y;
  }
  if (lane == 0) part_m[wv] = m;
  __syncthreads();
  int64_t eref = part_m[0];
  for (int i = 1; i < 16; ++i)
    if (lowest ? part_m[i] < eref : part_m[i] > eref) eref = part_m[i];
  // weights and their integer prefix, a contiguous chunk of slots per thread
  const int per = (R + 1023) >> 10;
  const int r0 = min(R, tid * per), r1 = min(R, r0 + per);
  double wsum = 0.0;
  uint64_t run = 0;
  for (int r = r0; r < r1; ++r) {
    const double w = exp_cw(-(delta * (double)(E[r] - eref)));
    wsum += w;
    run += (uint64_t)floor(w * 281474976710656.0);
    P[r] = run;  // local inclusive prefix
  }
  const uint64_t off = block_excl_scan<uint64_t>(run, part_u);
  for (int r = r0; r < r1; ++r) P[r] += off;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o, 64);
  if (lane == 0) part_d[wv] = wsum;
  __syncthreads();
  double wtot = 0.0;
  for (int i = 0; i < 16; ++i) wtot += part_d[i];
  const uint64_t Q = P[R - 1];
  const uint32_t g = st->g_rs;
  // searches with a fixed number of steps (no divergence; the LDS reads of a
  // thread's searches overlap): least j with P[j] > y, as the count of
  // entries <= y; P[R-1] = Q > y
  const int top = 1 << (31 - __clz(R));  // largest power of two <= R
  int par[kRsMaxR / 1024];
#pragma unroll
  for (int i0 = 0; i0 < kRsMaxR / 1024; i0 += 4) {  // four searches at a time
    uint64_t yv[4];
#pragma unroll
    for (int i = i0; i < i0 + 4; ++i) {
      const int k = tid + 1024 * i;
      par[i] = -1;
      yv[i - i0] = 0;
      if (k < R) {
        const u32x4 w = philox10((uint32_t)(k >> 1), g, 0u, kTagResample, a.k0, a.k1);
        const uint64_t u = (k & 1) ? ((uint64_t)w.c | ((uint64_t)w.d << 32))
                                   : ((uint64_t)w.a | ((uint64_t)w.b << 32));
        yv[i - i0] = __umul64hi(u, Q);
        par[i] = 0;
      }
    }
    if (tid + 1024 * i0 >= R) continue;
    for (int step = top; step > 0; step >>= 1) {
#pragma unroll
      for (int i = i0; i < i0 + 4; ++i) {
        const int nx = par[i] + step;  // candidate count: P[nx - 1] <= y
        if (par[i] >= 0 && nx <= R && P[nx - 1] <= yv[i - i0]) par[i] = nx;
      }
    }
  }
  __syncthreads();
  int32_t* cnt = reinterpret_cast<int32_t*>(P);
  for (int r = tid; r < R; r += 1024) cnt[r] = 0;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kRsMaxR / 1024; ++i)
    if (par[i] >= 0) atomicAdd(&cnt[par[i]], 1);
  __syncthreads();
  // children ordered by parent: cnt becomes the inclusive prefix C, and
  // child j's parent is the least r with C_r > j
  int local = 0;
  for (int r = r0; r < r1; ++r) {
    local += cnt[r];
    cnt[r] = local;
  }
  const int coff = block_excl_scan<int32_t>(local, part_i);
  for (int r = r0; r < r1; ++r) cnt[r] += coff;
  __syncthreads();
#pragma unroll
  for (int i0 = 0; i0 < kRsMaxR / 1024; i0 += 4) {
    if (tid + 1024 * i0 >= R) break;
    int pj[4] = {0, 0, 0, 0};
    for (int step = top; step > 0; step >>= 1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = tid + 1024 * (i0 + i), nx = pj[i] + step;
        if (j < R && nx <= R && cnt[nx - 1] <= j) pj[i] = nx;
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (tid + 1024 * (i0 + i) < R) a.rs_parent[tid + 1024 * (i0 + i)] = pj[i];
  }
  if (tid == 0) st->last_lnq = -delta * (double)eref + log(wtot) - log((double)R);
  if (fused && st->do_cluster) {
    __syncthreads();
    select_cluster_targets(a, st, E, a.rs_parent, L);
  }
}

// Copies every child's spins, fields, energy and lineage from its parent into
// the other population buffer.  Local block = (tile, quad chunk).
__global__ void __launch_bounds__(256) k_rs_gather(const Desc* __restrict__ D,
                                                   const uint64_t* __restrict__ map) {
  int inst, lb;
  if (!resolve(map, inst, lb)) return;
  const Desc& a = D[inst];
  RunState* st = a.st;
  if (!st->active || !st->do_resample) return;
  const int cur = st->cur;
  const PAMC_GLOBAL uint32_t* __restrict__ Ss = gmem((const uint32_t*)(cur ? a.S1 : a.S0));
  PAMC_GLOBAL uint32_t* __restrict__ Sd = gmem(cur ? a.S0 : a.S1);
  const PAMC_GLOBAL int32_t* __restrict__ Hs = gmem((const int32_t*)(cur ? a.H1 : a.H0));
  PAMC_GLOBAL int32_t* __restrict__ Hd = gmem(cur ? a.H0 : a.H1);
  int tile, chunk;
  group_chunk(a.T, lb, tile, chunk);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = tile * kLanes + lane;
  const int p = gmem(a.rs_parent)[c];
  const int pt = p >> 6, pl = p & 63;
  if (chunk == 0 && wave == 0) {
    (cur ? a.E0 : a.E1)[c] = (cur ? a.E1 : a.E0)[p];
    (cur ? a.F0 : a.F1)[c] = (cur ? a.F1 : a.F0)[p];
    for (int hk = 0; hk < a.nhub; ++hk) (cur ? a.HF0 : a.HF1)[hk * a.R + c] = (cur ? a.HF1 : a.HF0)[hk * a.R + p];
  }
  const int qb = chunk * kGatherQuadsPerBlock;
  // the wave's spin words: every read issued before the first write, so
  // that they are in flight together
  constexpr int kPer = kGatherQuadsPerBlock / 4;
  uint32_t w[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int q = qb + wave + 4 * i;
    if (q < a.nq) w[i] = Ss[((size_t)pt * a.nq + q) * kLanes + pl];
  }
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int q = qb + wave + 4 * i;
    if (q < a.nq) Sd[((size_t)tile * a.nq + q) * kLanes + lane] = w[i];
  }
  if (!Hs) return;
  // the fields (incremental mode), four quads (16 words) in flight at a time
  for (int i0 = 0; i0 < kPer; i0 += 4) {
    int32_t hv[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = qb + wave + 4 * (i0 + i);
      if (q < a.nq) {
#pragma unroll
        for (int k = 0; k < 4; ++k) hv[i][k] = Hs[((size_t)pt * a.np + 4 * q + k) * kLanes + pl];
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = qb + wave + 4 * (i0 + i);
      if (q < a.nq) {
#pragma unroll
        for (int k = 0; k < 4; ++k) Hd[((size_t)tile * a.np + 4 * q + k) * kLanes + lane] = hv[i][k];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Non-local cluster move (Algorithm 1; Sec. "Augmented PAMC").
// cl_select: the targets (see select_cluster_targets; in a run this is done
//   at the end of the resampling selection).
// cl_mis: per (target, trial), the greedy independent set of iso-sites
//   (h = 0) in the order of Philox keys (v, g_cl, r, CL | t<<8), ties by id.
//   The sequential greedy is computed with parallel rounds: an undecided
//   vertex joins once no undecided neighbour precedes it, and leaves once a
//   neighbour has joined; this selects exactly the sequential greedy set.
// cl_apply: flips the largest set (earliest trial on ties); fields of the
//   neighbours change, the energy does not (every flipped spin has h = 0 and
//   no two are coupled).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) k_cl_select(const Desc* __restrict__ D) {
  __shared__ SelectLds L;
  const Desc& d = D[blockIdx.x];
  RunState* st = d.st;
  if (!st->active || !st->do_cluster) return;
  const int buf = st->cur ^ st->do_resample;
  select_cluster_targets(d, st, buf ? d.E1 : d.E0, nullptr, L);
}

enum : uint8_t { kOut = 0, kUnd = 1, kCand = 2, kIn = 3 };

// Local block = target * trials + trial.
__global__ void __launch_bounds__(1024) k_cl_mis(const Desc* __restrict__ D, const uint64_t* __restrict__ map) {
  extern __shared__ uint8_t lds[];
  __shared__ int32_t cnt_s;
  int inst, lb;
  if (!resolve(map, inst, lb)) return;
  const Desc& a = D[inst];
  RunState* st = a.st;
  if (!st->active || !st->do_cluster) return;
  const int trials = st->cl_trials;
  if (trials <= 0) return;
  const int i = lb / trials, t = lb % trials;
  if (i >= min(st->cl_n_top, a.R)) return;
  const int buf = st->cur ^ st->do_resample;
  const int32_t* H = buf ? a.H1 : a.H0;
  const uint32_t* S = buf ? a.S1 : a.S0;
  uint32_t* key = (uint32_t*)lds;
  uint8_t* state = lds + sizeof(uint32_t) * (size_t)a.np;
  const int r = a.cl_targets[i];
  const int tile = r >> 6, lane = r & 63;
  const uint32_t g = st->g_cl;
  for (int v = threadIdx.x; v < a.np; v += blockDim.x) {
    uint8_t s = kOut;
    int32_t h = 1;
    if (v < a.n) {
      if (H) {
        h = H[((size_t)tile * a.np + v) * kLanes + lane];
      } else if (a.nhub && (v == a.hub_v0 || v == a.hub_v1)) {
        h = (buf ? a.HF1 : a.HF0)[(v == a.hub_v0 ? 0 : 1) * a.R + r];
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
  uint8_t* out = a.cl_sel + (size_t)lb * a.np;
  for (int v = threadIdx.x; v < a.np; v += blockDim.x) {
    const uint8_t in = state[v] == kIn;
    out[v] = in;
    mine += in;
  }
  atomicAdd(&cnt_s, mine);
  __syncthreads();
  if (threadIdx.x == 0) a.cl_sizes[lb] = cnt_s;
}

// Local block = target * kApplyChunks + chunk.
__global__ void __launch_bounds__(256) k_cl_apply(const Desc* __restrict__ D, const uint64_t* __restrict__ map) {
  int inst, lb;
  if (!resolve(map, inst, lb)) return;
  const Desc& a = D[inst];
  RunState* st = a.st;
  if (!st->active || !st->do_cluster) return;
  const int i = lb / kApplyChunks, chunk = lb % kApplyChunks;
  if (i >= min(st->cl_n_top, a.R)) return;
  const int trials = st->cl_trials;
  if (trials <= 0) return;
  const int buf = st->cur ^ st->do_resample;
  uint32_t* S = buf ? a.S1 : a.S0;
  int32_t* H = buf ? a.H1 : a.H0;
  int tb = 0, best = -1;
  for (int t = 0; t < trials; ++t) {
    const int s = a.cl_sizes[i * trials + t];
    if (s > best) { best = s; tb = t; }
  }
  const uint8_t* sel = a.cl_sel + (size_t)(i * trials + tb) * a.np;
  const int r = a.cl_targets[i];
  const int tile = r >> 6, lane = r & 63;
  int mine = 0;
  for (int v = chunk * blockDim.x + threadIdx.x; v < a.n; v += kApplyChunks * blockDim.x) {
    if (!sel[v]) continue;
    int8_t* sb = (int8_t*)&S[((size_t)tile * a.nq + (v >> 2)) * kLanes + lane] + (v & 3);
    const int32_t snew = -(int32_t)*sb;
    *sb = (int8_t)snew;
    if (H)
      for (int e = a.row_ptr[v]; e < a.row_ptr[v + 1]; ++e)
        __hip_atomic_fetch_add(&H[((size_t)tile * a.np + a.col[e]) * kLanes + lane], 2 * a.J[e] * snew,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      for (int hk = 0; hk < a.nhub; ++hk) {  // gathered fields: only the kept hub fields change
        const int32_t hj = a.hubJ[v * kMaxHubs + hk];
        if (hj)
          __hip_atomic_fetch_add(&(buf ? a.HF1 : a.HF0)[hk * a.R + r], 2 * hj * snew, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
      }
    ++mine;
  }
  // one counter update per work-group
  __shared__ int32_t part[4];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mine += __shfl_xor(mine, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = mine;
  __syncthreads();
  const int total = part[0] + part[1] + part[2] + part[3];
  if (threadIdx.x == 0 && total)
    __hip_atomic_fetch_add((unsigned long long*)a.cl_flipped, (unsigned long long)total, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Max-3-Cut decode (see pamc.h) and the pairwise Hamming diagnostic.
// ---------------------------------------------------------------------------
__global__ void k_m3_decode(const int8_t* spins_internal, const int32_t* to_internal_emb, int32_t n3,
                            int32_t* labels) {
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
    int dd = 0;
    for (int q = 0; q < nq; ++q) {
      const uint32_t x = S[((size_t)(a >> 6) * nq + q) * kLanes + (a & 63)];
      const uint32_t y = S[((size_t)(b >> 6) * nq + q) * kLanes + (b & 63)];
      uint32_t diff = x ^ y;  // spins are 0x01 / 0xFF bytes: a byte differs iff nonzero
      diff = (diff | (diff >> 1) | (diff >> 2) | (diff >> 3) | (diff >> 4) | (diff >> 5) |
              (diff >> 6) | (diff >> 7)) & 0x01010101u;
      dd += __popc(diff);
    }
    const double f = (double)dd / n;
    acc += f < 1.0 - f ? f : 1.0 - f;
  }
  atomicAdd(out, acc);
}

// Number of spins in which replicas a and b differ, folded by the global flip:
// min(d, n - d).  Spins are 0x01 / 0xFF bytes, so a byte of the xor is
// nonzero iff the spins differ.
__device__ __forceinline__ int32_t pair_dist(const uint32_t* S, int nq, int n, int a, int b) {
  int dd = 0;
  for (int q = 0; q < nq; ++q) {
    const uint32_t x = S[((size_t)(a >> 6) * nq + q) * kLanes + (a & 63)];
    const uint32_t y = S[((size_t)(b >> 6) * nq + q) * kLanes + (b & 63)];
    uint32_t diff = x ^ y;
    diff = (diff | (diff >> 1) | (diff >> 2) | (diff >> 3) | (diff >> 4) | (diff >> 5) | (diff >> 6) |
            (diff >> 7)) & 0x01010101u;
    dd += __popc(diff);
  }
  return dd < n - dd ? dd : n - dd;
}

// Work-group a: the pairs (a, b > a); histogram in LDS, then to memory.
__global__ void __launch_bounds__(256) k_pair_hist(const uint32_t* S0, const uint32_t* S1, const RunState* st,
                                                   int32_t n, int32_t nq, int32_t R, int32_t nbins,
                                                   int64_t* hist, int64_t* sum) {
  extern __shared__ int32_t hl[];
  const uint32_t* S = st->cur ? S1 : S0;
  for (int i = threadIdx.x; i < nbins; i += blockDim.x) hl[i] = 0;
  __syncthreads();
  const int a = blockIdx.x;
  int64_t acc = 0;
  for (int b = a + 1 + threadIdx.x; b < R; b += blockDim.x) {
    const int32_t dh = pair_dist(S, nq, n, a, b);
    acc += dh;
    const int bin = (int)min((int64_t)nbins - 1, (2 * (int64_t)nbins * dh) / n);
    atomicAdd(&hl[bin], 1);
  }
  acc = wave_sum_i64(acc);
  if ((threadIdx.x & 63) == 0 && acc)
    __hip_atomic_fetch_add((unsigned long long*)sum, (unsigned long long)acc, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  for (int i = threadIdx.x; i < nbins; i += blockDim.x)
    if (hl[i])
      __hip_atomic_fetch_add((unsigned long long*)&hist[i], (unsigned long long)hl[i], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

// In a run with a diversity trace: local block a of an instance sums
// min(d, n - d) over the pairs (a, b > a) of the population just swept, on
// the steps the trace samples.
__global__ void __launch_bounds__(256) k_step_dh(const Desc* __restrict__ D, const uint64_t* __restrict__ map) {
  int inst, a;
  if (!resolve(map, inst, a)) return;
  const Desc& d = D[inst];
  RunState* st = d.st;
  if (!st->active || st->dh_every <= 0 || st->step % st->dh_every != 0) return;
  const uint32_t* S = st->cur ? d.S1 : d.S0;
  int64_t acc = 0;
  for (int b = a + 1 + threadIdx.x; b < d.R; b += blockDim.x) acc += pair_dist(S, d.nq, d.n, a, b);
  acc = wave_sum_i64(acc);
  if ((threadIdx.x & 63) == 0 && acc)
    __hip_atomic_fetch_add((unsigned long long*)&st->dh_sum, (unsigned long long)acc, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// The sampled step's mean d_H into the trace (-1 on steps not sampled).
__global__ void k_step_dh_finish(const Desc* __restrict__ D, int32_t ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  const Desc& d = D[i];
  RunState* st = d.st;
  if (!st->active || st->dh_every <= 0) return;
  const int step = st->step;
  if (step < d.tr_cap && d.tr_dh) {
    const double pairs = 0.5 * (double)d.R * (double)(d.R - 1);
    d.tr_dh[step] = (step % st->dh_every == 0 && d.R > 1) ? (double)st->dh_sum / ((double)d.n * pairs) : -1.0;
  }
  st->dh_sum = 0;
}

}  // namespace

// ===========================================================================
// Batches and their launchers
// ===========================================================================
int32_t cluster_max_n() { return kClusterMaxN; }
int32_t sweep_waves() { return kSweepWaves; }
int32_t tile_max_quads() { return kTileMaxQuads; }
int64_t tile_lds_bytes(int32_t nq, int32_t rows) { return (int64_t)nq * kLanes * 4 + kThrLds * 4 + 8 * (int64_t)rows; }
int64_t tile_lds_limit() { return kTileLdsBytes; }
int32_t tmma_max_n() { return kTmmaMaxN; }
int64_t tmma_lds_bytes(int32_t nks, int32_t rows) { return rows * (64 * (int64_t)nks + 16) + kThrLds * 4; }

// Kernels whose dynamic LDS may exceed the default limit.
hipError_t prepare_kernel_lds() {
  hipError_t e = hipFuncSetAttribute((const void*)k_cl_mis, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     kClusterMaxN * 5 + 64);
  if (e != hipSuccess) return e;
  for (const void* k : {(const void*)k_sweep_tile<0>, (const void*)k_sweep_tile<1>, (const void*)k_sweep_tile<2>,
                        (const void*)k_sweep_tmma<16>, (const void*)k_sweep_tmma<8>, (const void*)k_sweep_tmma_g<8>})
    if ((e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kTileLdsBytes)) != hipSuccess)
      return e;
  return hipFuncSetAttribute((const void*)k_rs_select, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)sizeof(uint64_t) * kRsMaxR);
}

static int64_t sweep_chunks(const pamc_instance* I) {
  const int qpb = kSweepWaves * I->qpw;
  return (I->max_class_quads + qpb - 1) / qpb;
}

// Work-groups per replica tile of a sweep launch.  Incremental-field sweeps
// keep about `budget` per instance that loop over the class's chunks (a
// launch sized for the largest class then costs a small class little: its
// idle work-groups are few), the others one per chunk (capping those was
// measured too: C2's gathered-field phase took 50.1 us with 4,096
// work-groups and 60.2 with 1,024 against 49.4 uncapped; C4's Potts sweep
// 28.0 us with 2,048 against 28.3).
static int64_t sweep_slots(const pamc_instance* I, int64_t budget) {
  const int64_t chunks = sweep_chunks(I);
  if (I->pull || I->potts_K) return chunks;
  return std::min<int64_t>(chunks, std::max<int64_t>(1, budget / I->T));
}

// The budget: kPushWorkGroups for a lone instance, shared by the batch's
// incremental-field instances down to kPushMinWorkGroups each (C4: 2,048
// work-groups alone 3.21e11 attempts/s against 3.04e11 with 1,024 and
// 3.11e11 with 4,096; 16 instances 5.14e11 with 512 each against 4.83e11
// with 2,048).  PAMC_PUSH_WGS overrides.
static int64_t push_budget(const std::vector<pamc_instance*>& insts) {
  if (const char* e = getenv("PAMC_PUSH_WGS")) return std::max(1, atoi(e));
  int64_t n_push = 0;
  for (const pamc_instance* I : insts)
    if (!I->dense && !I->potts_K && !I->pull && !I->tile) ++n_push;
  return std::max<int64_t>(kPushMinWorkGroups, kPushWorkGroups / std::max<int64_t>(1, n_push));
}

Desc make_desc(const pamc_instance* I) {
  Desc d;
  memset(&d, 0, sizeof d);
  d.row_ptr = I->g.row_ptr;
  d.col = I->g.col;
  d.J = I->g.J;
  d.grow = I->g.grow;
  d.gcol = I->g.gcol;
  d.gJ = I->g.gJ;
  d.class_ptr = I->g.class_ptr;
  d.hubJ = I->g.hubJ;
  d.HF0 = I->pop.HF[0];
  d.HF1 = I->pop.HF[1];
  d.nhub = I->nhub;
  d.hub_v0 = I->hub_v[0];
  d.hub_v1 = I->hub_v[1];
  d.order = I->order;
  d.thr = I->thr;
  d.S0 = I->pop.S[0];
  d.S1 = I->pop.S[1];
  // incremental fields only in push mode (an instance keeping both forms
  // has them allocated in pull mode too, stale there)
  d.H0 = I->pull ? nullptr : I->pop.H[0];
  d.H1 = I->pull ? nullptr : I->pop.H[1];
  d.E0 = I->pop.E[0];
  d.E1 = I->pop.E[1];
  d.F0 = I->pop.fam[0];
  d.F1 = I->pop.fam[1];
  d.best = I->best;
  d.st = I->st;
  d.rs_parent = I->rs_parent;
  d.cl_targets = I->cl_targets;
  d.cl_sel = I->cl_sel;
  d.cl_sizes = I->cl_sizes;
  d.cl_flipped = I->flip_ctr ? I->flip_ctr + 256 : nullptr;
  d.tr_mstar = I->tr_mstar;
  d.tr_beta = I->tr_beta;
  d.tr_lnq = I->tr_lnq;
  d.tr_events = I->tr_events;
  d.tr_time = I->tr_time;
  d.tr_dh = I->tr_dh;
  d.flip_ctr = I->prof ? I->flip_ctr : nullptr;
  d.D0 = I->Sd;
  d.D1 = I->Sd2;
  d.W = I->W;
  d.X = I->X;
  d.n = I->n;
  d.np = I->np;
  d.nq = I->nq;
  d.R = I->R;
  d.T = I->T;
  d.ncls = I->ncls;
  d.rule = I->rule;
  d.pull = I->pull;
  d.dense = I->dense;
  d.ptab = I->ptab;
  d.potts_gamma = I->potts_gamma;
  d.potts_K = I->potts_K;
  d.potts_rule = I->potts_rule;
  d.shuffle = (I->flags & 1u) ? 0 : 1;
  d.tr_cap = I->tr_cap;
  d.qpw = I->qpw;
  d.sweep_stride = (int32_t)sweep_slots(I, kPushWorkGroups);  // batch_build sets the batch's
  d.tile_rows = I->tile_rows;
  d.Jt = I->g.Jt;
  d.nks = I->nks;
  d.order_cap = I->order_cap;
  d.k0 = (uint32_t)I->seed;
  d.k1 = (uint32_t)(I->seed >> 32);
  return d;
}

int Batch::group_of(const pamc_instance* I) {
  if (I->potts_K) return 37 + (I->potts_K - 2);
  if (!I->pull) return 0;
  const int ti = I->tpw == 4 ? 2 : (I->tpw == 2 ? 1 : 0);
  const int wide = 2 * I->X + 1 > kThrLds ? 1 : 0;
  return 1 + 18 * (I->nhub ? 1 : 0) + 9 * wide + 3 * I->jmode + ti;
}

void Batch::free_device() {
  const bool own = arena == nullptr;  // arena pieces are not the batch's to free
  auto release = [&](void* p) {
    if (!p || !own) return;
    if (al)
      al->free(al->ctx, p, (void*)stream);
    else
      hipFree(p);
  };
  release(d_desc);
  d_desc = nullptr;
  Launch* all[] = {&init_spins, &init_fields, &thr, &thr_dense, &gather, &cl_mis, &cl_apply, &dh};
  for (Launch* l : all) {
    release(l->map);
    l->map = nullptr;
    l->grid = 0;
  }
  for (Launch& l : sweep) {
    release(l.map);
    l.map = nullptr;
    l.grid = 0;
  }
  for (Launch& l : tile) {
    release(l.map);
    l.map = nullptr;
    l.grid = 0;
  }
  for (int64_t& x : tile_lds) x = 0;
  tmma_waves = 16;
  arena_used = 0;
  if (step_graph) hipGraphExecDestroy(step_graph);
  step_graph = nullptr;
  graph_key = -1;
}

hipError_t batch_alloc(Batch& b, void** p, size_t bytes) {
  if (!b.arena && b.al) {
    *p = b.al->alloc(b.al->ctx, bytes, (void*)b.stream);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  if (!b.arena) return hipMalloc(p, bytes);
  const size_t at = (b.arena_used + 255) & ~(size_t)255;
  b.arena_need = at + bytes;
  if (bytes > b.arena_cap || at > b.arena_cap - bytes) return hipErrorOutOfMemory;
  *p = b.arena + at;
  b.arena_used = at + bytes;
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Fixed device scratch for callers that cannot allocate device memory
// (pamc_anneal_batch_noalloc).  Every GPU the library runs on holds its own
// copy of this array until the process ends.  Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
// ---------------------------------------------------------------------------
constexpr size_t kFixedScratchBytes = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

hipError_t fixed_scratch(void** ptr, size_t* bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex m;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(m);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kFixedScratchBytes;
  return hipSuccess;
}


// Appends an instance's local blocks to a map.  With align8 the instance's
// first block is placed at a multiple of 8 (idle blocks fill the gap), so
// that its XCD placement does not depend on the instances before it.
static void add_blocks(std::vector<uint64_t>& map, int inst, int64_t count, bool align8) {
  if (count <= 0) return;
  const uint64_t hi = (uint64_t)(uint32_t)inst << 32;
  if (align8)
    while (map.size() % 8) map.push_back(hi | kIdle);
  for (int64_t b = 0; b < count; ++b) map.push_back(hi | (uint64_t)b);
}

static int64_t field_blocks(const pamc_instance* I) {
  return std::min<int64_t>((int64_t)I->T * ((I->n + 63) / 64), kFieldBlocks);
}

hipError_t batch_build(Batch& b, const std::vector<pamc_instance*>& insts, const std::vector<Schedule>* scheds) {
  // the old maps may still be read by queued kernels
  if (b.stream && b.n > 0) {
    const hipError_t e = hipStreamSynchronize(b.stream);
    if (e != hipSuccess) return e;
  }
  b.free_device();
  b.I = insts;
  b.n = (int32_t)insts.size();
  if (b.n == 0) return hipSuccess;
  b.stream = insts[0]->stream;
  std::vector<Desc> desc(b.n);
  const int64_t push_wgs = push_budget(insts);
  for (int i = 0; i < b.n; ++i) {
    desc[i] = make_desc(insts[i]);
    desc[i].sweep_stride = (int32_t)sweep_slots(insts[i], push_wgs);
  }
  // arena mode: per-run scratch sized for each instance's schedule
  std::vector<int32_t> cl_top(b.n), cl_trials(b.n);
  for (int i = 0; i < b.n; ++i) {
    cl_top[i] = std::min(insts[i]->cl_cap_top, insts[i]->R);
    cl_trials[i] = insts[i]->cl_cap_trials;
  }
  if (b.arena) {
    if (!scheds) return hipErrorInvalidValue;
    for (int i = 0; i < b.n; ++i) {
      const pamc_instance* I = insts[i];
      const Schedule& s = (*scheds)[i];
      Desc& d = desc[i];
      d.flip_ctr = nullptr;
      d.tr_cap = 0;
      d.order_cap = std::max(s.sweeps, 1);
      hipError_t e = batch_alloc(b, (void**)&d.order, sizeof(int32_t) * (size_t)d.order_cap * std::max(I->ncls, 1));
      if (e != hipSuccess) return e;
      const bool cl = s.augmented && s.resample && s.n_top > 0 && s.mis_trials > 0 && !I->potts_K && !I->dense;
      cl_top[i] = cl ? std::min(s.n_top, I->R) : 0;
      cl_trials[i] = cl ? s.mis_trials : 0;
      d.cl_targets = nullptr;
      d.cl_sel = nullptr;
      d.cl_sizes = nullptr;
      if (cl) {
        if ((e = batch_alloc(b, (void**)&d.cl_targets, sizeof(int32_t) * cl_top[i])) != hipSuccess) return e;
        if ((e = batch_alloc(b, (void**)&d.cl_sizes, sizeof(int32_t) * (size_t)cl_top[i] * cl_trials[i])) != hipSuccess)
          return e;
        if ((e = batch_alloc(b, (void**)&d.cl_sel, (size_t)cl_top[i] * cl_trials[i] * I->np)) != hipSuccess) return e;
      }
    }
  }
  std::vector<uint64_t> m_init, m_fields, m_thr, m_gather, m_mis, m_apply, m_dh;
  std::vector<std::vector<uint64_t>> m_sweep(Batch::kGroups), m_tile(4);
  b.max_ncls = 0;
  for (int g = 0; g < Batch::kGroups; ++g) b.group_ncls[g] = 0;
  b.max_sweeps = 1;
  b.any_cluster = 0;
  b.max_lds = 0;
  b.max_R = 0;
  // Matrix-core tiles: while the batch has at most 128 of them, one
  // work-group per 16-replica group spreads them over four times the
  // compute units (a single instance's step is 1.4x faster); beyond, one
  // work-group per tile shares each coupling block between its four groups
  // in the unit's L1 (1.7x the throughput of group work-groups with 1,024
  // tiles).  PAMC_TMMA_GROUPS = 0 or 1 forces one.
  {
    int64_t mt = 0;
    for (int i = 0; i < b.n; ++i)
      if (!insts[i]->dense && insts[i]->tile == 2) mt += insts[i]->T;
    b.tmma_groups = mt <= 128;
    if (const char* g = getenv("PAMC_TMMA_GROUPS")) b.tmma_groups = atoi(g) != 0;
  }
  for (int i = 0; i < b.n; ++i) {
    pamc_instance* I = insts[i];
    b.max_R = std::max(b.max_R, I->R);
    if (I->dense) continue;
    add_blocks(m_init, i, kInitBlocks, false);
    add_blocks(m_fields, i, field_blocks(I), false);
    add_blocks(m_thr, i, kThrBlocks, false);
    add_blocks(m_gather, i, (int64_t)I->T * ((I->nq + kGatherQuadsPerBlock - 1) / kGatherQuadsPerBlock), true);
    if (I->tile == 2) {  // the same with matrix-core fields
      add_blocks(m_tile[3], i, (int64_t)I->T * (b.tmma_groups ? 4 : 1), false);
      b.tile_lds[3] = std::max<int64_t>(b.tile_lds[3], tmma_lds_bytes(I->nks, b.tmma_groups ? 16 : 64));
    } else if (I->tile) {  // one work-group per replica tile walks the whole step
      add_blocks(m_tile[I->jmode], i, I->T, false);
      b.tile_lds[I->jmode] = std::max<int64_t>(b.tile_lds[I->jmode], tile_lds_bytes(I->nq, I->tile_rows));
    } else {
      const int grp = Batch::group_of(I);
      add_blocks(m_sweep[grp], i, (int64_t)(I->T / (I->pull ? I->tpw : 1)) * sweep_slots(I, push_wgs), true);
      b.max_ncls = std::max(b.max_ncls, I->ncls);
      b.group_ncls[grp] = std::max(b.group_ncls[grp], I->ncls);
    }
    const int nt = cl_top[i];
    if (nt > 0 && cl_trials[i] > 0) {
      add_blocks(m_mis, i, (int64_t)nt * cl_trials[i], false);
      add_blocks(m_apply, i, (int64_t)nt * kApplyChunks, false);
      b.max_lds = std::max<int64_t>(b.max_lds, (int64_t)I->np * 5);
    }
  }
  // diversity samples: one work-group per replica.  A batch without
  // schedules (an instance's own) keeps the map; its runs switch it on.
  b.any_dh = 0;
  for (int i = 0; i < b.n; ++i) {
    if (scheds) {
      const Schedule& s = (*scheds)[i];
      b.max_sweeps = std::max(b.max_sweeps, s.sweeps);
      if (s.augmented && s.resample && s.n_top > 0 && s.mis_trials > 0) b.any_cluster = 1;
      if (s.dh_every <= 0) continue;
    }
    if (insts[i]->dense || insts[i]->potts_K) continue;
    add_blocks(m_dh, i, insts[i]->R, false);
    if (scheds) b.any_dh = 1;
  }
  hipError_t e = batch_alloc(b, (void**)&b.d_desc, sizeof(Desc) * b.n);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(b.d_desc, desc.data(), sizeof(Desc) * b.n, hipMemcpyHostToDevice, b.stream);
  if (e != hipSuccess) return e;
  auto up = [&](std::vector<uint64_t>& m, Batch::Launch& l) -> hipError_t {
    if (m.size() > (size_t)INT32_MAX) return hipErrorInvalidValue;
    l.grid = (int32_t)m.size();
    if (m.empty()) return hipSuccess;
    hipError_t err = batch_alloc(b, (void**)&l.map, sizeof(uint64_t) * m.size());
    if (err != hipSuccess) return err;
    return hipMemcpyAsync(l.map, m.data(), sizeof(uint64_t) * m.size(), hipMemcpyHostToDevice, b.stream);
  };
  if ((e = up(m_init, b.init_spins)) != hipSuccess) return e;
  if ((e = up(m_fields, b.init_fields)) != hipSuccess) return e;
  if ((e = up(m_thr, b.thr)) != hipSuccess) return e;
  if ((e = up(m_gather, b.gather)) != hipSuccess) return e;
  if ((e = up(m_mis, b.cl_mis)) != hipSuccess) return e;
  if ((e = up(m_apply, b.cl_apply)) != hipSuccess) return e;
  if ((e = up(m_dh, b.dh)) != hipSuccess) return e;
  for (int g = 0; g < Batch::kGroups; ++g)
    if ((e = up(m_sweep[g], b.sweep[g])) != hipSuccess) return e;
  for (int g = 0; g < 4; ++g)
    if ((e = up(m_tile[g], b.tile[g])) != hipSuccess) return e;
  // matrix-core tiles: 8-wave work-groups, two per compute unit, once the
  // launch has at least two per unit and two fit the unit's LDS
  // (PAMC_TMMA_WAVES = 8 or 16 forces a size)
  b.tmma_waves = ((int64_t)m_tile[3].size() >= 2 * kComputeUnits &&
                  2 * (b.tile_lds[3] + (int64_t)sizeof(int64_t) * 8 * kLanes + 64) <= kCuLdsBytes)
                     ? 8
                     : 16;
  if (const char* w = getenv("PAMC_TMMA_WAVES")) b.tmma_waves = atoi(w) == 8 ? 8 : 16;
  // the staging vectors are local: wait for the copies before they go
  return hipStreamSynchronize(b.stream);
}

using SweepKernel = void (*)(const Desc*, const uint64_t*, int, int);
using SweepTileKernel = void (*)(const Desc*, const uint64_t*);

template <bool WIDE, bool HUB>
static SweepKernel pull_kernel(int jm, int ti) {
  static const SweepKernel k[3][3] = {
      {k_sweep_pull<0, 1, WIDE, HUB>, k_sweep_pull<0, 2, WIDE, HUB>, k_sweep_pull<0, 4, WIDE, HUB>},
      {k_sweep_pull<1, 1, WIDE, HUB>, k_sweep_pull<1, 2, WIDE, HUB>, k_sweep_pull<1, 4, WIDE, HUB>},
      {k_sweep_pull<2, 1, WIDE, HUB>, k_sweep_pull<2, 2, WIDE, HUB>, k_sweep_pull<2, 4, WIDE, HUB>}};
  return k[jm][ti];
}

static SweepKernel sweep_kernel_of_group(int g) {
  // group = 0 (incremental fields), 1 + 18 * hubs + 9 * wide table + 3 * coupling mode +
  // tiles-per-wave index (gathered fields), 37 + K - 2 (Potts labels)
  if (g == 0) return k_sweep_push;
  if (g >= 37) return g == 37 ? k_sweep_potts<2> : (g == 38 ? k_sweep_potts<3> : k_sweep_potts<4>);
  int x = g - 1;
  const bool hub = x >= 18;
  x %= 18;
  const bool wide = x >= 9;
  x %= 9;
  if (hub) return wide ? pull_kernel<true, true>(x / 3, x % 3) : pull_kernel<false, true>(x / 3, x % 3);
  return wide ? pull_kernel<true, false>(x / 3, x % 3) : pull_kernel<false, false>(x / 3, x % 3);
}

static hipEvent_t next_event(pamc_instance* I) {
  if (I->ev_used == I->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    I->ev_pool.push_back(e);
  }
  return I->ev_pool[I->ev_used++];
}

static inline int tgrid(int n) { return (n + 63) / 64; }

// thresholds + class orders (and, with commit >= 0, the step's commit), then
// nsweeps x max_ncls phase launches.  When
// profiling, one event pair brackets the step's back-to-back sweep launches
// (nothing else runs between them), so the mean launch time includes the
// launch boundaries and the events cost two markers per step, not two per
// launch.
static hipError_t batch_sweeps(Batch& b, int32_t nsweeps, int32_t commit = -1) {
  pamc_instance* P = b.I[0];
  const bool prof = P->prof && !b.arena;
  if (b.thr.grid) k_thresholds<<<b.thr.grid, 256, 0, b.stream>>>(b.d_desc, b.thr.map, commit);
  int64_t launches = 0;
  if (prof) hipEventRecord(next_event(P), b.stream);
  static const SweepTileKernel tile_kernels[3] = {k_sweep_tile<0>, k_sweep_tile<1>, k_sweep_tile<2>};
  for (int g = 0; g < 3; ++g)
    if (b.tile[g].grid) {  // every sweep of the step, in one launch
      tile_kernels[g]<<<b.tile[g].grid, kTileWaves * 64, b.tile_lds[g], b.stream>>>(b.d_desc, b.tile[g].map);
      ++launches;
    }
  if (b.tile[3].grid) {
    if (b.tmma_groups)
      k_sweep_tmma_g<8><<<b.tile[3].grid, 8 * 64, b.tile_lds[3], b.stream>>>(b.d_desc, b.tile[3].map);
    else if (b.tmma_waves == 8)
      k_sweep_tmma<8><<<b.tile[3].grid, 8 * 64, b.tile_lds[3], b.stream>>>(b.d_desc, b.tile[3].map);
    else
      k_sweep_tmma<16><<<b.tile[3].grid, 16 * 64, b.tile_lds[3], b.stream>>>(b.d_desc, b.tile[3].map);
    ++launches;
  }
  for (int s = 0; s < nsweeps; ++s) {
    for (int p = 0; p < b.max_ncls; ++p) {
      for (int g = 0; g < Batch::kGroups; ++g) {
        if (!b.sweep[g].grid || p >= b.group_ncls[g]) continue;  // no instance of the group has class p
        sweep_kernel_of_group(g)<<<b.sweep[g].grid, 256, 0, b.stream>>>(b.d_desc, b.sweep[g].map, s, p);
        ++launches;
      }
    }
  }
  if (prof) {
    hipEventRecord(next_event(P), b.stream);
    P->prof_launches += launches;
    for (pamc_instance* I : b.I) P->prof_attempts += (int64_t)nsweeps * I->n * I->R;
  }
  return hipGetLastError();
}

hipError_t batch_init(Batch& b) {
  if (b.init_spins.grid) k_init_spins<<<b.init_spins.grid, 256, 0, b.stream>>>(b.d_desc, b.init_spins.map);
  for (pamc_instance* I : b.I) hipMemsetAsync(I->pop.E[0], 0, sizeof(int64_t) * I->R, b.stream);
  if (b.init_fields.grid)
    k_init_fields<<<b.init_fields.grid, 256, 0, b.stream>>>(b.d_desc, b.init_fields.map, 0, nullptr, 1);
  k_init_finish<<<b.n, 256, 0, b.stream>>>(b.d_desc);
  return hipGetLastError();
}

hipError_t batch_anneal_setup(Batch& b, const Schedule* d_sched, const int32_t* d_idx, int32_t count) {
  if (count <= 0) return hipSuccess;
  k_anneal_setup<<<tgrid(count), 64, 0, b.stream>>>(b.d_desc, d_sched, d_idx, count);
  return hipGetLastError();
}

// fused: the run step's decisions before, the cluster targets after the draw
static hipError_t batch_resample(Batch& b, int32_t fused) {
  k_rs_select<<<b.n, 1024, sizeof(uint64_t) * b.max_R, b.stream>>>(b.d_desc, fused);
  if (b.gather.grid) k_rs_gather<<<b.gather.grid, 256, 0, b.stream>>>(b.d_desc, b.gather.map);
  return hipGetLastError();
}

// select: false when the targets were chosen with the resampling draw
static hipError_t batch_cluster(Batch& b, bool select) {
  if (select) k_cl_select<<<b.n, 1024, 0, b.stream>>>(b.d_desc);
  if (b.cl_mis.grid) k_cl_mis<<<b.cl_mis.grid, 1024, b.max_lds, b.stream>>>(b.d_desc, b.cl_mis.map);
  if (b.cl_apply.grid) k_cl_apply<<<b.cl_apply.grid, 256, 0, b.stream>>>(b.d_desc, b.cl_apply.map);
  return hipGetLastError();
}

hipError_t batch_step(Batch& b) {
  // step decisions + resampling draw (+ cluster targets), gather, cluster
  // move, thresholds + commit, sweeps, step end
  batch_resample(b, 1);
  if (b.any_cluster) batch_cluster(b, false);
  hipError_t e = batch_sweeps(b, b.max_sweeps, 1);
  if (e != hipSuccess) return e;
  if (b.any_dh && b.dh.grid) {  // diversity of the swept population, on sampled steps
    k_step_dh<<<b.dh.grid, 256, 0, b.stream>>>(b.d_desc, b.dh.map);
    k_step_dh_finish<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n);
  }
  k_step_end<<<b.n, 1024, 0, b.stream>>>(b.d_desc, 1);
  return hipGetLastError();
}

// k beta steps.  Without profiling, one step is captured once as a HIP graph
// (kernels only: the launch sequence of a step is fixed and every decision
// is read from device state) and replayed; if the stream cannot be captured
// the steps are launched one by one.  PAMC_NO_GRAPH=1 forces the latter.
hipError_t batch_run_steps(Batch& b, int32_t k) {
  const char* ng = getenv("PAMC_NO_GRAPH");
  const bool no_graph = ng && atoi(ng) != 0;
  const int64_t key = ((int64_t)b.max_sweeps << 2) | (b.any_dh ? 2 : 0) | (b.any_cluster ? 1 : 0);
  bool use_graph = !no_graph && !b.arena && !b.I[0]->prof && !b.graph_failed && k > 1;
  if (use_graph && (!b.step_graph || b.graph_key != key)) {
    if (b.step_graph) hipGraphExecDestroy(b.step_graph);
    b.step_graph = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      const hipError_t es = batch_step(b);
      e = hipStreamEndCapture(b.stream, &g);
      if (es != hipSuccess) e = es;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b.step_graph, g, nullptr, nullptr, 0);
    if (g) hipGraphDestroy(g);
    if (e != hipSuccess) {
      (void)hipGetLastError();  // clear the capture error; launch eagerly from now on
      b.step_graph = nullptr;
      b.graph_failed = true;
      use_graph = false;
    } else {
      b.graph_key = key;
    }
  }
  for (int32_t i = 0; i < k; ++i) {
    const hipError_t e = use_graph ? hipGraphLaunch(b.step_graph, b.stream) : batch_step(b);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

hipError_t batch_status(Batch& b, int32_t* d_out) {
  k_status<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n, d_out);
  return hipGetLastError();
}

hipError_t prim_sweep(Batch& b, double beta, int32_t nsweeps) {
  pamc_instance* I = b.I[0];
  int done = 0;
  while (done < nsweeps) {
    const int chunk = std::min(nsweeps - done, I->order_cap);
    k_prim_set<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n, 0, beta, 0, 0, chunk);
    hipError_t e = batch_sweeps(b, chunk);
    if (e != hipSuccess) return e;
    k_advance_sweeps<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n, chunk);
    done += chunk;
  }
  return hipGetLastError();
}

hipError_t prim_resample(Batch& b, double delta) {
  k_prim_set<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n, 1, delta, 0, 0, 0);
  batch_resample(b, 0);
  k_commit<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n, 0);
  k_deactivate<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n);
  return hipGetLastError();
}

hipError_t prim_cluster(Batch& b, int32_t n_top, int32_t trials) {
  k_prim_set<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n, 2, 0.0, n_top, trials, 0);
  batch_cluster(b, true);
  k_commit<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n, 0);
  k_deactivate<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n);
  return hipGetLastError();
}

hipError_t prim_update_best(Batch& b) {
  k_prim_set<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n, 0, 0.0, 0, 0, 0);
  k_step_end<<<b.n, 1024, 0, b.stream>>>(b.d_desc, 0);
  k_deactivate<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n);
  return hipGetLastError();
}

hipError_t launch_fields(Batch& b, int32_t buf, int32_t* H) {
  k_init_fields<<<b.init_fields.grid, 256, 0, b.stream>>>(b.d_desc, b.init_fields.map, buf, H, 0);
  return hipGetLastError();
}

hipError_t launch_load_population(Batch& b) {
  for (pamc_instance* I : b.I) hipMemsetAsync(I->pop.E[0], 0, sizeof(int64_t) * I->R, b.stream);
  if (b.init_fields.grid)
    k_init_fields<<<b.init_fields.grid, 256, 0, b.stream>>>(b.d_desc, b.init_fields.map, 0, nullptr, 1);
  k_load_finish<<<b.n, 256, 0, b.stream>>>(b.d_desc);
  return hipGetLastError();
}

hipError_t launch_m3_decode(pamc_instance* I, const int8_t* spins_internal_dev) {
  hipMemsetAsync(I->m3_cut, 0, sizeof(int64_t), I->stream);
  const int grid = (I->m3_n + 255) / 256;
  k_m3_decode<<<grid, 256, 0, I->stream>>>(spins_internal_dev, I->to_internal_dev, I->m3_n, I->m3_labels);
  k_m3_cut<<<grid, 256, 0, I->stream>>>(I->m3_labels, I->m3_n, I->m3_row_ptr, I->m3_col, I->m3_w,
                                        I->m3_cut);
  return hipGetLastError();
}

// The fields the instance's current form keeps, recomputed from the current
// population (no energy change): the incremental fields in push mode, the
// kept hub fields.
hipError_t launch_refresh_fields(Batch& b) {
  if (b.init_fields.grid)
    k_init_fields<<<b.init_fields.grid, 256, 0, b.stream>>>(b.d_desc, b.init_fields.map, -1, nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_pair_hist(pamc_instance* I, int32_t nbins, int64_t* hist_dev, int64_t* sum_dev) {
  hipMemsetAsync(hist_dev, 0, sizeof(int64_t) * nbins, I->stream);
  hipMemsetAsync(sum_dev, 0, sizeof(int64_t), I->stream);
  k_pair_hist<<<I->R, 256, sizeof(int32_t) * nbins, I->stream>>>(I->pop.S[0], I->pop.S[1], I->st, I->n, I->nq, I->R,
                                                                 nbins, hist_dev, sum_dev);
  return hipGetLastError();
}

hipError_t launch_pair_distance(pamc_instance* I, double* out_dev) {
  hipMemsetAsync(out_dev, 0, sizeof(double), I->stream);
  k_pair_distance<<<I->R, 256, 0, I->stream>>>(I->pop.S[0], I->pop.S[1], I->st, I->n, I->nq, I->R,
                                               out_dev);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Controller pieces used by the dense path (single instance via its batch).
// ---------------------------------------------------------------------------
hipError_t ctl_step_begin(Batch& b) {
  k_step_begin<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n);
  return hipGetLastError();
}
hipError_t ctl_resample_select(Batch& b) {
  k_rs_select<<<b.n, 1024, sizeof(uint64_t) * b.max_R, b.stream>>>(b.d_desc, 0);
  return hipGetLastError();
}
hipError_t ctl_commit(Batch& b, int32_t in_run) {
  k_commit<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n, in_run);
  return hipGetLastError();
}
hipError_t ctl_thresholds(Batch& b) {
  // dense instances have no classes: only the table is computed
  if (!b.thr_dense.grid) {
    std::vector<uint64_t> m;
    for (int i = 0; i < b.n; ++i) add_blocks(m, i, kThrBlocks, false);
    b.thr_dense.grid = (int32_t)m.size();
    hipError_t e = batch_alloc(b, (void**)&b.thr_dense.map, sizeof(uint64_t) * m.size());
    if (e != hipSuccess) return e;
    e = hipMemcpy(b.thr_dense.map, m.data(), sizeof(uint64_t) * m.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
  }
  k_thresholds<<<b.thr_dense.grid, 256, 0, b.stream>>>(b.d_desc, b.thr_dense.map, -1);
  return hipGetLastError();
}
hipError_t ctl_step_end(Batch& b, int32_t in_run) {
  k_step_end<<<b.n, 1024, 0, b.stream>>>(b.d_desc, in_run);
  return hipGetLastError();
}
hipError_t ctl_prim_set(Batch& b, int32_t kind, double value, int32_t nsweeps) {
  k_prim_set<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n, kind, value, 0, 0, nsweeps);
  return hipGetLastError();
}
hipError_t ctl_advance(Batch& b, int32_t nsweeps) {
  k_advance_sweeps<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n, nsweeps);
  return hipGetLastError();
}
hipError_t ctl_deactivate(Batch& b) {
  k_deactivate<<<tgrid(b.n), 64, 0, b.stream>>>(b.d_desc, b.n);
  return hipGetLastError();
}
hipEvent_t ctl_event(pamc_instance* I) { return next_event(I); }

}  // namespace pamc
