// capi.hip -- the C ABI (include/pamc.h): instance construction on the host
// (validation, DSATUR colouring, class-major relabelling, Max-3-Cut
// embedding), device memory, and the host code that enqueues the kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pamc.h"
#include "instance.hpp"

using pamc::Schedule;

namespace {

thread_local std::string g_err;

pamc_status fail(pamc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

pamc_status dev_fail(hipError_t e, const char* where) {
  g_err = std::string(where) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? PAMC_ERR_OUT_OF_MEMORY : PAMC_ERR_DEVICE;
}

#define HIP_TRY(expr, where)                 \
  do {                                       \
    hipError_t _e = (expr);                  \
    if (_e != hipSuccess) return dev_fail(_e, where); \
  } while (0)

// Device memory of an instance: from its allocator when it has one, else
// hipMalloc.
hipError_t dev_alloc(pamc_instance* I, void** p, size_t bytes) {
  if (I->use_al) {
    *p = I->al.alloc(I->al.ctx, bytes, (void*)I->stream);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

void dev_free(pamc_instance* I, void* p) {
  if (!p) return;
  if (I->use_al)
    I->al.free(I->al.ctx, p, (void*)I->stream);
  else
    hipFree(p);
}

template <typename T>
hipError_t dalloc(pamc_instance* I, T** p, size_t count) {
  const size_t bytes = std::max<size_t>(sizeof(T) * count, 16);
  void* q = nullptr;
  hipError_t e = dev_alloc(I, &q, bytes);
  if (e == hipSuccess) {
    *p = (T*)q;
    I->device_bytes += (int64_t)bytes;
  }
  return e;
}

// Frees a buffer that dalloc made for count elements of T and takes it off
// the instance's byte count.
template <typename T>
void dfree(pamc_instance* I, T*& p, size_t count) {
  if (!p) return;
  dev_free(I, p);
  I->device_bytes -= (int64_t)std::max<size_t>(sizeof(T) * count, 16);
  p = nullptr;
}

void free_instance(pamc_instance* I) {
  if (!I) return;
  if (I->device >= 0) hipSetDevice(I->device);
  if (I->stream) hipStreamSynchronize(I->stream);
  delete I->self;
  I->self = nullptr;
  dev_free(I, I->d_sched);
  void* ptrs[] = {I->g.row_ptr, I->g.col, I->g.J, I->g.grow, I->g.gcol, I->g.gJ, I->g.class_ptr, I->pop.S[0], I->pop.S[1],
                  I->pop.H[0], I->pop.H[1], I->pop.E[0], I->pop.E[1], I->pop.fam[0],
                  I->pop.fam[1], I->best, I->to_internal_dev, I->st, I->thr, I->order,
                  I->rs_parent, I->cl_targets, I->cl_sel, I->cl_sizes, I->tr_mstar, I->tr_beta,
                  I->tr_lnq, I->tr_events, I->tr_time, I->tr_dh, I->m3_row_ptr, I->m3_col, I->m3_w,
                  I->m3_labels, I->m3_cut, I->Jd, I->Sd, I->Sd2, I->Gd, I->Cd, I->Ed[0], I->Ed[1],
                  I->flip_ctr, I->H_scratch, I->ptab, I->g.hubJ, I->pop.HF[0], I->pop.HF[1], I->g.Jt};
  for (void* p : ptrs) dev_free(I, p);
  if (I->pinned) hipHostFree(I->pinned);
  for (hipEvent_t e : I->ev_pool) hipEventDestroy(e);
  if (I->own_stream && I->stream) hipStreamDestroy(I->stream);
  delete I;
}

// Structural checks of a symmetric CSR graph (both directions stored).
pamc_status validate_csr(int32_t n, const int32_t* rp, const int32_t* col, const int32_t* w,
                         bool positive_only) {
  if (n <= 0) return fail(PAMC_ERR_INVALID_ARG, "n must be positive");
  if (!rp || (!col && rp[n] > 0) || (!w && rp[n] > 0))
    return fail(PAMC_ERR_INVALID_ARG, "NULL CSR array");
  if (rp[0] != 0) return fail(PAMC_ERR_INVALID_ARG, "row_ptr[0] must be 0");
  for (int32_t v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v]) return fail(PAMC_ERR_INVALID_ARG, "row_ptr must be non-decreasing");
  const int64_t nnz = rp[n];
  std::vector<std::tuple<int32_t, int32_t, int32_t>> fwd, bwd;
  fwd.reserve(nnz);
  bwd.reserve(nnz);
  for (int32_t v = 0; v < n; ++v) {
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
      const int32_t u = col[e];
      if (u < 0 || u >= n) return fail(PAMC_ERR_INVALID_ARG, "column index out of range");
      if (u == v) return fail(PAMC_ERR_INVALID_ARG, "self loop");
      if (w[e] == 0) return fail(PAMC_ERR_INVALID_ARG, "zero weight entry");
      if (positive_only && w[e] < 0) return fail(PAMC_ERR_INVALID_ARG, "weights must be positive");
      fwd.emplace_back(v, u, w[e]);
      bwd.emplace_back(u, v, w[e]);
    }
  }
  std::sort(fwd.begin(), fwd.end());
  for (size_t i = 1; i < fwd.size(); ++i)
    if (std::get<0>(fwd[i]) == std::get<0>(fwd[i - 1]) && std::get<1>(fwd[i]) == std::get<1>(fwd[i - 1]))
      return fail(PAMC_ERR_INVALID_ARG, "duplicate edge");
  std::sort(bwd.begin(), bwd.end());
  if (fwd != bwd) return fail(PAMC_ERR_INVALID_ARG, "graph is not symmetric");
  return PAMC_OK;
}

pamc_status check_cfg(const pamc_config* cfg) {
  if (!cfg) return fail(PAMC_ERR_INVALID_ARG, "NULL config");
  if (cfg->replicas <= 0 || cfg->replicas % 64 != 0)
    return fail(PAMC_ERR_INVALID_ARG, "replicas must be a positive multiple of 64");
  if (cfg->replicas > 16384) return fail(PAMC_ERR_UNSUPPORTED, "replicas > 16384");
  if (cfg->rule != 0 && cfg->rule != 1) return fail(PAMC_ERR_INVALID_ARG, "unknown rule");
  return PAMC_OK;
}

pamc_status open_device(pamc_instance* I, const pamc_config* cfg) {
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count), "hipGetDeviceCount");
  if (cfg->device < 0 || cfg->device >= count) return fail(PAMC_ERR_INVALID_ARG, "bad device");
  I->device = cfg->device;
  if (cfg->alloc) {
    if (!cfg->alloc->alloc || !cfg->alloc->free) return fail(PAMC_ERR_INVALID_ARG, "allocator without functions");
    I->al = *cfg->alloc;
    I->use_al = true;
  }
  HIP_TRY(hipSetDevice(I->device), "hipSetDevice");
  if (cfg->stream) {
    I->stream = (hipStream_t)cfg->stream;
  } else {
    HIP_TRY(hipStreamCreateWithFlags(&I->stream, hipStreamNonBlocking), "hipStreamCreate");
    I->own_stream = true;
  }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, I->device) == hipSuccess && khz > 0)
    I->clock_hz = khz * 1000.0;
  HIP_TRY(hipHostMalloc(&I->pinned, 4096, hipHostMallocDefault), "hipHostMalloc");
  I->seed = cfg->seed;
  I->R = cfg->replicas;
  I->T = cfg->replicas / 64;
  I->rule = cfg->rule;
  I->flags = cfg->flags;
  return PAMC_OK;
}

// The instance as a batch of one, rebuilt after any change of the buffers or
// keys its descriptor names.
pamc::Batch* self_batch(pamc_instance* I, hipError_t* err) {
  *err = hipSuccess;
  if (!I->self) {
    I->self = new (std::nothrow) pamc::Batch();
    if (I->self && I->use_al) I->self->al = &I->al;
  }
  if (!I->self) {
    *err = hipErrorOutOfMemory;
    return nullptr;
  }
  if (I->self_dirty) {
    *err = pamc::batch_build(*I->self, std::vector<pamc_instance*>{I}, nullptr);
    if (*err != hipSuccess) return nullptr;
    I->self_dirty = false;
  }
  return I->self;
}

#define SELF_BATCH(I, var)                                  \
  hipError_t var##_err;                                     \
  pamc::Batch* var = self_batch(I, &var##_err);             \
  if (!var) return dev_fail(var##_err, "batch descriptors")

// Host half of building a sparse instance (no device calls, safe on any
// thread): colouring, class-major relabelling, the relabelled and
// padded CSR, W, X and the choice of sweep kernel.  Jin: couplings J in
// caller ids (already validated).  T: replica tiles.
struct HostSparse {
  int32_t potts_K = 0;  // set by the caller for Potts labels (no fields, plain CSR only)
  int32_t n = 0, np = 0, nq = 0, ncls = 0, max_class_quads = 0;
  int32_t small_j = 0, jmode = 0, pull = 0, tpw = 1, qpw = 1;
  int32_t nhub = 0, hub_v[pamc::kMaxHubs] = {-1, -1};  // internal ids of the hubs (pull mode)
  int32_t tile = 0;  // a step's sweeps of a replica tile in one work-group
  int32_t tile_ok = 0;  // tile-resident sweeps possible (the autotuner may switch them)
  int32_t tile_rows = 0;  // gathered-CSR entries of the largest colour class
  int32_t dual = 0;  // both field forms kept (hub graphs; see dual_field_step)
  int32_t tmma_ok = 0, nks = 0;  // the matrix-core tile form possible; its 64-column steps
  std::vector<int8_t> Jt;        // J as matrix-core A fragments
  int32_t hub_tpw = 1, hub_qpw = 1, push_tpw = 1, push_qpw = 1;  // the two forms' wave shapes
  int64_t nnz = 0, W = 0, X = 0;
  std::vector<int32_t> class_ptr, to_internal, to_input, rp2, col2, J2, grow, gcol, gJ, hubJ;
};

// Field storage of a sparse graph: gathered at visit time (pull) or kept
// incrementally (push); both give the same integer fields and trajectory.
// Gathering a vertex's field costs its degree at every visit; keeping it
// costs one device-scope atomic per neighbour of every flip.  Pull is the
// default when every row is short: at most 16 entries per vertex on average
// and 64 at most.  With PAMC_FLAG_FIELDS_PULL, up to kMaxHubs hub rows
// (more than 64 entries) are allowed too: their fields are kept (the
// updates of a work-group summed in LDS before one atomic per replica),
// since gathering a hub serialises one wavefront per tile over all of its
// neighbours.  On the Max-3-Cut embedding of G(7000, 21000) that mode takes
// about 25 us per class phase at any temperature, incremental fields 17 us
// at a flip rate of 0.16% but 170 us at 10%; the benchmark's runs average
// 1%, where incremental fields are faster, so graphs with hubs default to
// them.  Returns pull; hubs receives the hubs' caller ids.
// Small instances (at most tile_max_quads vertex quads, a threshold table
// that fits LDS) sweep tile-resident: one work-group per replica tile holds
// the tile's spins in LDS and makes all of a step's sweeps in one launch,
// where per-class launches would each carry microseconds of launch latency
// for a few dozen vertices.
bool tile_fits(int64_t nq, int64_t X) { return nq <= pamc::tile_max_quads() && 2 * X + 1 <= 2048; }

bool choose_fields(int32_t n, const int32_t* rp, uint32_t flags, bool potts, std::vector<int32_t>* hubs) {
  hubs->clear();
  if (potts) return true;  // Potts labels: K-label fields gathered at visit time
  if (flags & PAMC_FLAG_FIELDS_PUSH) return false;
  std::vector<int32_t> h;
  for (int32_t v = 0; v < n; ++v)
    if (rp[v + 1] - rp[v] > 64) h.push_back(v);
  if (flags & PAMC_FLAG_FIELDS_PULL) {
    if ((int)h.size() <= pamc::kMaxHubs) *hubs = h;  // more hubs than that: gathered like any row
    return true;
  }
  return h.empty() && (int64_t)rp[n] <= 16 * (int64_t)n;
}

// Saturation-degree (DSATUR) colouring: the next vertex is the uncoloured
// one with the most distinct colours among its coloured neighbours (ties:
// the longer row, then the lower id); it takes the least colour none of its
// neighbours has.  Vertices are ranked once by (row length descending, id);
// each saturation level keeps a min-heap of ranks, a vertex being pushed
// again at its new level when its saturation grows (entries for coloured
// vertices or for an older level are skipped when they come up); each
// vertex keeps the sorted colours its neighbours have taken.  Returns the
// number of colours.
int32_t dsatur_colour(int32_t n, const int32_t* rp, const int32_t* col, std::vector<int32_t>& colour) {
  colour.assign(n, -1);
  std::vector<int32_t> order(n), rank(n), sat(n, 0);
  for (int32_t v = 0; v < n; ++v) order[v] = v;
  std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    const int32_t da = rp[a + 1] - rp[a], db = rp[b + 1] - rp[b];
    return da != db ? da > db : a < b;
  });
  for (int32_t i = 0; i < n; ++i) rank[order[i]] = i;
  std::vector<std::vector<int32_t>> level(1);  // level[s]: min-heap of ranks at saturation s
  auto push = [&](int32_t s, int32_t r) {
    if ((int32_t)level.size() <= s) level.resize(s + 1);
    level[s].push_back(r);
    std::push_heap(level[s].begin(), level[s].end(), std::greater<int32_t>());
  };
  level[0] = order.empty() ? std::vector<int32_t>() : std::vector<int32_t>(n);
  for (int32_t i = 0; i < n; ++i) level[0][i] = i;  // ascending: already a min-heap
  std::vector<std::vector<int32_t>> seen(n);        // per vertex: its neighbours' colours, sorted
  std::vector<int32_t> stamp(n + 1, -1);
  int32_t ncls = 0, top = 0;
  for (int32_t done = 0; done < n;) {
    while (level[top].empty()) --top;
    std::pop_heap(level[top].begin(), level[top].end(), std::greater<int32_t>());
    const int32_t v = order[level[top].back()];
    level[top].pop_back();
    if (colour[v] >= 0 || sat[v] != top) continue;  // coloured, or now at a higher level
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
      if (colour[col[e]] >= 0) stamp[colour[col[e]]] = v;
    int32_t c = 0;
    while (stamp[c] == v) ++c;
    colour[v] = c;
    ncls = std::max(ncls, c + 1);
    ++done;
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
      const int32_t u = col[e];
      if (colour[u] >= 0) continue;
      std::vector<int32_t>& su = seen[u];
      const auto it = std::lower_bound(su.begin(), su.end(), c);
      if (it != su.end() && *it == c) continue;  // u has a neighbour of colour c already
      su.insert(it, c);
      push(++sat[u], rank[u]);
      top = std::max(top, sat[u]);
    }
  }
  return ncls;
}

pamc_status prepare_sparse(HostSparse& h, int32_t n, const int32_t* rp, const int32_t* col,
                           const std::vector<int32_t>& Jin, uint32_t flags, int32_t T, bool allow_dual = true,
                           const std::vector<int32_t>* colour_in = nullptr) {
  h.n = n;
  h.np = (n + 3) & ~3;
  h.nq = h.np / 4;
  h.nnz = rp[n];
  // the visit order's colour classes: the given colouring (the Max-3-Cut
  // embedding's) or the DSATUR one
  std::vector<int32_t> colour;
  int32_t ncls = 0;
  if (colour_in) {
    colour = *colour_in;
    for (int32_t v = 0; v < n; ++v) ncls = std::max(ncls, colour[v] + 1);
  } else {
    ncls = dsatur_colour(n, rp, col, colour);
  }
  h.ncls = ncls;
  h.class_ptr.assign(ncls + 1, 0);
  for (int32_t v = 0; v < n; ++v) h.class_ptr[colour[v] + 1]++;
  for (int32_t c = 0; c < ncls; ++c) h.class_ptr[c + 1] += h.class_ptr[c];
  h.to_internal.resize(n);
  h.to_input.resize(n);
  {
    std::vector<int32_t> next(h.class_ptr.begin(), h.class_ptr.end() - 1);
    for (int32_t v = 0; v < n; ++v) {
      const int32_t iv = next[colour[v]]++;
      h.to_internal[v] = iv;
      h.to_input[iv] = v;
    }
  }
  h.max_class_quads = 0;
  for (int32_t c = 0; c < ncls; ++c) {
    const int32_t a = h.class_ptr[c], b = h.class_ptr[c + 1];
    h.max_class_quads = std::max(h.max_class_quads, ((b + 3) >> 2) - (a >> 2));
  }
  // relabelled CSR; the arrays carry trailing padding (vertex 0, coupling
  // 0) so that the sweep kernels may read a few entries past the last row
  const size_t nnzp = (size_t)h.nnz + 16;
  h.rp2.assign(n + 1, 0);
  h.col2.assign(nnzp, 0);
  h.J2.assign(nnzp, 0);
  int64_t W = 0, X = 0, maxdeg = 0;
  for (int32_t iv = 0; iv < n; ++iv) {
    const int32_t v = h.to_input[iv];
    int32_t p = h.rp2[iv];
    int64_t ab = 0;
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e, ++p) {
      h.col2[p] = h.to_internal[col[e]];
      h.J2[p] = Jin[e];
      ab += std::llabs((long long)Jin[e]);
      if (col[e] > v) W -= Jin[e];
    }
    h.rp2[iv + 1] = p;
    X = std::max(X, ab);
    maxdeg = std::max<int64_t>(maxdeg, rp[v + 1] - rp[v]);
  }
  if (2 * X >= INT32_MAX) return fail(PAMC_ERR_INVALID_ARG, "local field range exceeds int32");
  h.W = W;
  h.X = X;
  h.small_j = 1;
  bool int8_j = true;
  for (int32_t e = 0; e < rp[n]; ++e) {
    const long long a = std::llabs((long long)Jin[e]);
    if (a >= (1 << 23)) h.small_j = 0;
    if (a > 127) int8_j = false;
  }
  // packed int8 couplings when they fit a byte and a work-group's energy
  // change per replica fits 32 bits
  h.jmode = (int8_j && X < (1 << 26)) ? 2 : (h.small_j ? 1 : 0);
  if (const char* e = getenv("PAMC_JMODE")) {
    const int m = atoi(e);
    if (m == 0 || (m == 1 && h.small_j) || (m == 2 && h.jmode == 2)) h.jmode = m;
  }
  std::vector<int32_t> hubs;
  h.pull = choose_fields(n, rp, flags, h.potts_K != 0, &hubs) ? 1 : 0;
  // Small instances sweep tile-resident (see below): the spins sit in LDS,
  // so gathering is cheap whatever the degree, and no field array is kept.
  h.tile = (!h.potts_K && !(flags & PAMC_FLAG_FIELDS_PUSH) && tile_fits(h.nq, X)) ? 1 : 0;
  if (const char* e = getenv("PAMC_TILE")) h.tile = h.tile && atoi(e) != 0 ? 1 : 0;
  if (h.tile) {
    h.pull = 1;
    hubs.clear();
  }
  // Graphs whose only long rows are a few hubs (at most kMaxHubs rows of
  // more than 64 entries) keep both field forms when no form is forced: a
  // run takes gathered fields with the hubs' fields kept while its
  // schedule's beta is low, where incremental fields would walk a hub's
  // whole row from one wavefront at each of its frequent flips, and
  // incremental fields afterwards (dual_field_step).
  if (allow_dual && !h.pull && !h.tile && !h.potts_K &&
      !(flags & (PAMC_FLAG_FIELDS_PUSH | PAMC_FLAG_FIELDS_PULL))) {
    std::vector<int32_t> hh;
    choose_fields(n, rp, PAMC_FLAG_FIELDS_PULL, false, &hh);
    if (!hh.empty()) {
      h.dual = 1;
      hubs = hh;
    }
  }
  h.nhub = (h.pull || h.dual) ? (int32_t)hubs.size() : 0;
  for (int32_t k = 0; k < h.nhub; ++k) h.hub_v[k] = h.to_internal[hubs[k]];
  if (h.nhub) {  // couplings of every vertex to each hub
    h.hubJ.assign((size_t)h.np * pamc::kMaxHubs, 0);
    for (int32_t iv = 0; iv < n; ++iv)
      for (int32_t e = h.rp2[iv]; e < h.rp2[iv + 1]; ++e)
        for (int32_t k = 0; k < h.nhub; ++k)
          if (h.col2[e] == h.hub_v[k]) h.hubJ[(size_t)iv * pamc::kMaxHubs + k] = h.J2[e];
  }
  // Gathered-field CSR: rows padded to multiples of 4 entries; columns as
  // byte offsets of the neighbour's spin word in a tile (plus its byte index
  // in modes 0 and 1), couplings in the kernel's mode (mode 2: the int8
  // coupling in the neighbour's byte).
  // Potts labels are read with a byte index: coupling mode 0 or 1 layout
  if (h.potts_K && h.jmode == 2) h.jmode = h.small_j ? 1 : 0;
  if (h.pull || h.dual) {
    // a hub's row is not gathered (its field is kept), so it stays empty here
    auto is_hub = [&](int32_t iv) { return h.nhub && (iv == h.hub_v[0] || iv == h.hub_v[1]); };
    h.grow.assign(n + 1, 0);
    for (int32_t iv = 0; iv < n; ++iv)
      h.grow[iv + 1] = h.grow[iv] + (is_hub(iv) ? 0 : ((h.rp2[iv + 1] - h.rp2[iv] + 3) & ~3));
    h.gcol.assign(std::max(h.grow[n], 4), 0);
    h.gJ.assign(std::max(h.grow[n], 4), 0);
    for (int32_t iv = 0; iv < n; ++iv) {
      if (is_hub(iv)) continue;
      int32_t p = h.grow[iv];
      for (int32_t e = h.rp2[iv]; e < h.rp2[iv + 1]; ++e, ++p) {
        h.gcol[p] = (h.col2[e] >> 2) * 256 + (h.jmode == 2 ? 0 : (h.col2[e] & 3));
        h.gJ[p] = h.jmode == 2 ? (int32_t)((uint32_t)(uint8_t)(int8_t)h.J2[e] << (8 * (h.col2[e] & 3))) : h.J2[e];
      }
    }
  }
  const bool tile_candidate = h.pull && !h.nhub && !h.potts_K && tile_fits(h.nq, X);
  if (tile_candidate) {  // a class's gathered rows are staged in LDS next to the spins
    for (int32_t c = 0; c < h.ncls; ++c)
      h.tile_rows = std::max(h.tile_rows, h.grow[h.class_ptr[c + 1]] - h.grow[h.class_ptr[c]]);
    h.tile_rows = (h.tile_rows + 3) & ~3;
    h.tile_ok = pamc::tile_lds_bytes(h.nq, h.tile_rows) <= pamc::tile_lds_limit() ? 1 : 0;
    if (!h.tile_ok) h.tile_rows = 0;
  }
  // Small instances with int8 couplings can also compute a class's fields
  // on the matrix cores (k_sweep_tmma): J as 16-row x 64-column A fragments
  // in the order the kernel reads them (lane l: row 16 t + l % 16, columns
  // 64 ks + 16 (l / 16) .. + 15).  Per attempt the gathered form reads 4
  // bytes of LDS per neighbour and this one 4 bytes of fragments per 64
  // columns through the vector L1, which moves half as many bytes per
  // cycle: so graphs whose average degree is at least n_pad / 32 (and 8)
  // take this form, and so do those whose gathered rows do not fit LDS.
  // PAMC_TILE = 0, 1 or 2 forces none, the gathered form or this one where
  // it applies.
  if (allow_dual && h.tile && h.jmode == 2 && h.np <= pamc::tmma_max_n() && 2 * X + 1 <= 2048) {
    h.tmma_ok = 1;
    h.nks = (h.np + 63) / 64;
    const int32_t nrt = (h.np + 15) / 16;
    h.Jt.assign((size_t)nrt * h.nks * 1024, 0);
    for (int32_t iv = 0; iv < n; ++iv)
      for (int32_t e = h.rp2[iv]; e < h.rp2[iv + 1]; ++e) {
        const int32_t c = h.col2[e], t = iv >> 4, ks = c >> 6, lane = (iv & 15) + 16 * ((c & 63) >> 4);
        h.Jt[(((size_t)t * h.nks + ks) * 64 + lane) * 16 + (c & 15)] = (int8_t)h.J2[e];
      }
    const char* te = getenv("PAMC_TILE");
    const bool dense_ish = (int64_t)h.nnz >= 8 * (int64_t)n && 32 * (int64_t)h.nnz >= (int64_t)n * h.np;
    if (te ? atoi(te) == 2 || !h.tile_ok : dense_ish || !h.tile_ok) h.tile = 2;
  }
  if (h.tile == 1 && !h.tile_ok) {  // the rows do not fit: per-class launches
    h.tile = 0;
    if (!choose_fields(n, rp, flags, false, &hubs)) {  // back to the field storage it would have had
      h.pull = 0;
      h.grow.clear();
      h.gcol.clear();
      h.gJ.clear();
    }
  }
  // Tiles per wavefront: share the per-vertex scalar work among up to 4
  // tiles while keeping enough work-groups (one quad per wave) to fill the
  // chip.  Then quads per wave: the most (fewer partial energy sums) that
  // still leave about 16 work-groups per compute unit.
  const int64_t W4 = pamc::sweep_waves();
  const int64_t q1 = (h.max_class_quads + W4 - 1) / W4;
  h.tpw = 1;
  if (h.pull && !h.potts_K)
    for (int t : {4, 2})
      if (T % t == 0 && (T / t) * q1 >= 1024) {
        h.tpw = t;
        break;
      }
  if (h.nhub && !h.dual)  // the measured best shape of the kept-hub mode on the Max-3-Cut embedding: 4 x 1
    h.tpw = (T % 4 == 0) ? 4 : ((T % 2 == 0) ? 2 : 1);
  if (const char* e = getenv("PAMC_TPW")) {
    const int t = atoi(e);
    if ((t == 1 || t == 2 || t == 4) && T % t == 0 && !h.potts_K) h.tpw = t;
  }
  h.qpw = 1;
  for (int q : {4, 2})
    if ((!h.nhub || h.dual) && (T / h.tpw) * ((h.max_class_quads + W4 * q - 1) / (W4 * q)) >= 4096) {
      h.qpw = q;
      break;
    }
  if (h.dual) {  // starts with incremental fields; the kept-hub shape as measured (4 x 1)
    h.hub_tpw = (T % 4 == 0) ? 4 : ((T % 2 == 0) ? 2 : 1);
    h.hub_qpw = 1;
  }
  if (const char* e = getenv("PAMC_QPW")) {
    const int q = atoi(e);
    if (q == 1 || q == 2 || q == 4) h.qpw = q;
  }
  h.push_tpw = h.tpw;
  h.push_qpw = h.qpw;
  return PAMC_OK;
}

// Sweep shapes chosen by pamc_autotune, per instance shape (this process).
struct TuneShape {
  int32_t tile, tpw, qpw;
};

std::mutex g_tune_mutex;
std::unordered_map<std::string, TuneShape> g_tune_cache;

std::string tune_key(const pamc_instance* I) {
  return std::to_string(I->n) + "/" + std::to_string(I->nnz) + "/" + std::to_string(I->R) + "/" +
         std::to_string(I->ncls) + "/" + std::to_string(I->max_class_quads) + "/" + std::to_string(I->pull) + "/" +
         std::to_string(I->jmode) + "/" + std::to_string(I->potts_K) + "/" + std::to_string(I->nhub) + "/" +
         std::to_string(I->tile_ok) + "/" + std::to_string(I->tmma_ok) + "/" + std::to_string(I->rule);
}

void apply_shape(pamc_instance* I, const TuneShape& t) {
  I->tile = t.tile;
  I->tpw = t.tpw;
  I->qpw = t.qpw;
  if (I->dual && !I->pull) {  // the incremental-field form's shape
    I->push_tpw = t.tpw;
    I->push_qpw = t.qpw;
  }
  I->self_dirty = true;
}

// A new instance of a shape the autotuner has seen takes its choice (unless
// a shape is forced from the environment).
void apply_cached_shape(pamc_instance* I) {
  if (getenv("PAMC_TPW") || getenv("PAMC_QPW") || getenv("PAMC_TILE")) return;
  std::lock_guard<std::mutex> g(g_tune_mutex);
  auto it = g_tune_cache.find(tune_key(I));
  if (it != g_tune_cache.end()) apply_shape(I, it->second);
}

// Device half: buffers, upload and the initial population (waits).
pamc_status upload_sparse(pamc_instance* I, HostSparse& h) {
  const int32_t n = h.n, ncls = h.ncls;
  I->n = n;
  I->np = h.np;
  I->nq = h.nq;
  I->nnz = h.nnz;
  I->ncls = ncls;
  I->W = h.W;
  I->X = h.X;
  I->small_j = h.small_j;
  I->jmode = h.jmode;
  I->pull = h.pull;
  I->tile = h.tile;
  I->tile_ok = h.tile_ok;
  I->tmma_ok = h.tmma_ok;
  I->nks = h.nks;
  I->tile_rows = h.tile_rows;
  I->nhub = h.nhub;
  for (int k = 0; k < pamc::kMaxHubs; ++k) I->hub_v[k] = h.hub_v[k];
  I->tpw = h.tpw;
  I->qpw = h.qpw;
  I->dual = h.dual;
  I->hub_tpw = h.hub_tpw;
  I->hub_qpw = h.hub_qpw;
  I->push_tpw = h.push_tpw;
  I->push_qpw = h.push_qpw;
  I->max_class_quads = h.max_class_quads;
  I->class_ptr = std::move(h.class_ptr);
  I->to_internal = std::move(h.to_internal);
  I->to_input = std::move(h.to_input);
  const size_t nnz = (size_t)I->nnz + 16;
  const size_t words = (size_t)I->T * I->nq * 64, hs = (size_t)I->T * I->np * 64;
  HIP_TRY(dalloc(I, &I->g.row_ptr, n + 1), "alloc");
  HIP_TRY(dalloc(I, &I->g.col, nnz), "alloc");
  HIP_TRY(dalloc(I, &I->g.J, nnz), "alloc");
  const bool gathered = I->pull || I->dual;
  if (gathered) {
    HIP_TRY(dalloc(I, &I->g.grow, n + 1), "alloc");
    HIP_TRY(dalloc(I, &I->g.gcol, h.gcol.size()), "alloc");
    HIP_TRY(dalloc(I, &I->g.gJ, h.gJ.size()), "alloc");
  }
  HIP_TRY(dalloc(I, &I->g.class_ptr, ncls + 1), "alloc");
  if (I->nhub) HIP_TRY(dalloc(I, &I->g.hubJ, h.hubJ.size()), "alloc");
  if (I->tmma_ok) HIP_TRY(dalloc(I, &I->g.Jt, h.Jt.size()), "alloc");
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(dalloc(I, &I->pop.S[b], words), "alloc population");
    if (!I->pull) HIP_TRY(dalloc(I, &I->pop.H[b], hs), "alloc population");
    if (I->nhub) HIP_TRY(dalloc(I, &I->pop.HF[b], (size_t)pamc::kMaxHubs * I->R), "alloc population");
    HIP_TRY(dalloc(I, &I->pop.E[b], I->R), "alloc population");
    HIP_TRY(dalloc(I, &I->pop.fam[b], I->R), "alloc population");
  }
  HIP_TRY(dalloc(I, &I->best, I->np), "alloc");
  HIP_TRY(dalloc(I, &I->to_internal_dev, n), "alloc");
  HIP_TRY(dalloc(I, &I->st, 1), "alloc");
  if (I->potts_K)
    HIP_TRY(dalloc(I, &I->ptab, 2 * I->X + 1), "alloc");
  HIP_TRY(dalloc(I, &I->thr, I->potts_K ? 1 : 2 * I->X + 1), "alloc");
  I->order_cap = 64;
  HIP_TRY(dalloc(I, &I->order, (size_t)I->order_cap * ncls), "alloc");
  HIP_TRY(dalloc(I, &I->rs_parent, I->R), "alloc");
  HIP_TRY(dalloc(I, &I->flip_ctr, 512), "alloc");
  HIP_TRY(hipMemsetAsync(I->flip_ctr, 0, sizeof(int64_t) * 512, I->stream), "memset");
  HIP_TRY(hipMemsetAsync(I->st, 0, sizeof(pamc::RunState), I->stream), "memset");
  if (!I->pull) {
    HIP_TRY(hipMemsetAsync(I->pop.H[0], 0, sizeof(int32_t) * hs, I->stream), "memset");
    HIP_TRY(hipMemsetAsync(I->pop.H[1], 0, sizeof(int32_t) * hs, I->stream), "memset");
  }
  HIP_TRY(hipMemcpyAsync(I->g.row_ptr, h.rp2.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, I->stream), "upload");
  HIP_TRY(hipMemcpyAsync(I->g.col, h.col2.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, I->stream), "upload");
  HIP_TRY(hipMemcpyAsync(I->g.J, h.J2.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, I->stream), "upload");
  if (gathered) {
    HIP_TRY(hipMemcpyAsync(I->g.grow, h.grow.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, I->stream), "upload");
    HIP_TRY(hipMemcpyAsync(I->g.gcol, h.gcol.data(), sizeof(int32_t) * h.gcol.size(), hipMemcpyHostToDevice, I->stream), "upload");
    HIP_TRY(hipMemcpyAsync(I->g.gJ, h.gJ.data(), sizeof(int32_t) * h.gJ.size(), hipMemcpyHostToDevice, I->stream), "upload");
  }
  HIP_TRY(hipMemcpyAsync(I->g.class_ptr, I->class_ptr.data(), sizeof(int32_t) * (ncls + 1), hipMemcpyHostToDevice, I->stream), "upload");
  if (I->nhub)
    HIP_TRY(hipMemcpyAsync(I->g.hubJ, h.hubJ.data(), sizeof(int32_t) * h.hubJ.size(), hipMemcpyHostToDevice, I->stream), "upload");
  if (I->tmma_ok)
    HIP_TRY(hipMemcpyAsync(I->g.Jt, h.Jt.data(), h.Jt.size(), hipMemcpyHostToDevice, I->stream), "upload");
  HIP_TRY(hipMemcpyAsync(I->to_internal_dev, I->to_internal.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, I->stream), "upload");
  HIP_TRY(pamc::prepare_kernel_lds(), "hipFuncSetAttribute");
  apply_cached_shape(I);
  SELF_BATCH(I, b);
  HIP_TRY(pamc::batch_init(*b), "init kernels");
  // the host arrays are read by the queued copies: wait before they go
  HIP_TRY(hipStreamSynchronize(I->stream), "init");
  return PAMC_OK;
}

pamc_status build_sparse(pamc_instance* I, int32_t n, const int32_t* rp, const int32_t* col,
                         const std::vector<int32_t>& Jin, const std::vector<int32_t>* colour = nullptr) {
  HostSparse h;
  h.potts_K = I->potts_K;
  pamc_status st = prepare_sparse(h, n, rp, col, Jin, I->flags, I->T, true, colour);
  if (st) return st;
  return upload_sparse(I, h);
}

Schedule to_sched(const pamc_schedule* s) {
  Schedule d;
  d.beta0 = s->beta0;
  d.dbeta = s->dbeta;
  d.reheat = s->reheat;
  d.target = s->target;
  d.steps = s->steps;
  d.sweeps = s->sweeps;
  d.z_rst = s->z_rst;
  d.augmented = s->augmented;
  d.resample = s->resample;
  d.win_short = s->win_short;
  d.win_long = s->win_long;
  d.max_ds = s->max_distinct_short;
  d.max_dl = s->max_distinct_long;
  d.tau = s->tau;
  d.n_top = s->n_top;
  d.mis_trials = s->mis_trials;
  d.stop_at_target = s->stop_at_target;
  d.literal_break = s->literal_break;
  d.resume = s->resume ? 1 : 0;
  d.dh_every = s->dh_every > 0 ? s->dh_every : 0;
  return d;
}

// The ensure_* helpers grow per-run buffers.  The old buffers go first (the
// stream is drained), and a size is recorded only once all of its buffers
// exist: after a failed allocation the instance holds none of that kind and
// a size of 0, so no kernel is ever handed a missing buffer.
pamc_status ensure_cluster_scratch(pamc_instance* I, int32_t n_top, int32_t trials) {
  n_top = std::min(n_top, I->R);
  if (n_top <= 0 || trials <= 0) return PAMC_OK;
  if (I->n > pamc::cluster_max_n())
    return fail(PAMC_ERR_UNSUPPORTED, "cluster moves need n <= 26000");
  if (trials > 64) return fail(PAMC_ERR_UNSUPPORTED, "mis_trials > 64");
  if (n_top <= I->cl_cap_top && trials <= I->cl_cap_trials) return PAMC_OK;
  HIP_TRY(hipStreamSynchronize(I->stream), "sync");
  const int32_t top = std::max(n_top, I->cl_cap_top), tr = std::max(trials, I->cl_cap_trials);
  dfree(I, I->cl_targets, I->cl_cap_top);
  dfree(I, I->cl_sel, (size_t)I->cl_cap_top * I->cl_cap_trials * I->np);
  dfree(I, I->cl_sizes, (size_t)I->cl_cap_top * I->cl_cap_trials);
  I->cl_cap_top = I->cl_cap_trials = 0;
  I->self_dirty = true;
  hipError_t e = dalloc(I, &I->cl_targets, top);
  if (e == hipSuccess) e = dalloc(I, &I->cl_sel, (size_t)top * tr * I->np);
  if (e == hipSuccess) e = dalloc(I, &I->cl_sizes, (size_t)top * tr);
  if (e != hipSuccess) {
    dfree(I, I->cl_targets, top);
    dfree(I, I->cl_sel, (size_t)top * tr * I->np);
    dfree(I, I->cl_sizes, (size_t)top * tr);
    return dev_fail(e, "alloc cluster");
  }
  I->cl_cap_top = top;
  I->cl_cap_trials = tr;
  return PAMC_OK;
}

pamc_status ensure_trace(pamc_instance* I, int32_t steps) {
  if (steps <= I->tr_cap) return PAMC_OK;
  HIP_TRY(hipStreamSynchronize(I->stream), "sync");
  dfree(I, I->tr_mstar, I->tr_cap);
  dfree(I, I->tr_beta, I->tr_cap);
  dfree(I, I->tr_lnq, I->tr_cap);
  dfree(I, I->tr_events, I->tr_cap);
  dfree(I, I->tr_time, I->tr_cap);
  dfree(I, I->tr_dh, I->tr_cap);
  I->tr_cap = 0;
  I->self_dirty = true;
  hipError_t e = dalloc(I, &I->tr_mstar, steps);
  if (e == hipSuccess) e = dalloc(I, &I->tr_beta, steps);
  if (e == hipSuccess) e = dalloc(I, &I->tr_lnq, steps);
  if (e == hipSuccess) e = dalloc(I, &I->tr_events, steps);
  if (e == hipSuccess) e = dalloc(I, &I->tr_time, steps);
  if (e == hipSuccess) e = dalloc(I, &I->tr_dh, steps);
  if (e != hipSuccess) {
    dfree(I, I->tr_mstar, steps);
    dfree(I, I->tr_beta, steps);
    dfree(I, I->tr_lnq, steps);
    dfree(I, I->tr_events, steps);
    dfree(I, I->tr_time, steps);
    dfree(I, I->tr_dh, steps);
    return dev_fail(e, "alloc trace");
  }
  I->tr_cap = steps;
  return PAMC_OK;
}

pamc_status ensure_order(pamc_instance* I, int32_t sweeps) {
  if (sweeps <= I->order_cap) return PAMC_OK;
  HIP_TRY(hipStreamSynchronize(I->stream), "sync");
  int32_t* fresh = nullptr;
  HIP_TRY(dalloc(I, &fresh, (size_t)sweeps * I->ncls), "alloc order");  // the old orders stay on failure
  dfree(I, I->order, (size_t)I->order_cap * I->ncls);
  I->order = fresh;
  I->order_cap = sweeps;
  I->self_dirty = true;
  return PAMC_OK;
}

// Folds the recorded sweep-launch event pairs into the running total.
pamc_status resolve_events(pamc_instance* I) {
  for (size_t i = 0; i + 1 < I->ev_used; i += 2) {
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, I->ev_pool[i], I->ev_pool[i + 1]), "hipEventElapsedTime");
    I->prof_ms += t;
  }
  I->ev_used = 0;
  return PAMC_OK;
}

pamc_status read_state(pamc_instance* I, pamc::RunState* out) {
  HIP_TRY(hipStreamSynchronize(I->stream), "kernel execution");
  HIP_TRY(hipMemcpy(out, I->st, sizeof(pamc::RunState), hipMemcpyDeviceToHost), "readback");
  return PAMC_OK;
}

// Dense instance buffers (couplings uploaded or generated by the caller of
// this helper), then the initial population.
pamc_status build_dense_common(pamc_instance* I, int32_t n) {
  I->dense = 1;
  I->n = n;
  I->dn_pad = (n + 63) & ~63;
  I->np = I->dn_pad;
  I->nq = I->dn_pad / 4;
  I->ncls = 0;
  I->to_internal.resize(n);
  I->to_input.resize(n);
  for (int32_t v = 0; v < n; ++v) I->to_internal[v] = I->to_input[v] = v;
  const size_t np = (size_t)I->dn_pad;
  HIP_TRY(dalloc(I, &I->Jd, np * np), "alloc couplings");
  HIP_TRY(dalloc(I, &I->Sd, (size_t)I->R * np), "alloc population");
  HIP_TRY(dalloc(I, &I->Sd2, (size_t)I->R * np), "alloc population");
  for (int b = 0; b < 2; ++b) {
    HIP_TRY(dalloc(I, &I->pop.E[b], I->R), "alloc population");
    HIP_TRY(dalloc(I, &I->pop.fam[b], I->R), "alloc population");
  }
  HIP_TRY(dalloc(I, &I->best, np), "alloc");
  HIP_TRY(dalloc(I, &I->st, 1), "alloc");
  HIP_TRY(dalloc(I, &I->rs_parent, I->R), "alloc");
  HIP_TRY(dalloc(I, &I->flip_ctr, 512), "alloc");
  HIP_TRY(pamc::prepare_kernel_lds(), "hipFuncSetAttribute");
  const size_t gsz = (size_t)pamc::dense_field_buffers() * pamc::dense_superblock_rows() * I->R;
  HIP_TRY(dalloc(I, &I->Gd, gsz), "alloc fields");
  HIP_TRY(hipMemsetAsync(I->Gd, 0, sizeof(int32_t) * gsz, I->stream), "memset");
  HIP_TRY(dalloc(I, &I->Cd, np * (size_t)I->R), "alloc critical fields");
  I->order_cap = 1;
  HIP_TRY(dalloc(I, &I->order, 1), "alloc");
  HIP_TRY(hipMemsetAsync(I->flip_ctr, 0, sizeof(int64_t) * 512, I->stream), "memset");
  HIP_TRY(hipMemsetAsync(I->st, 0, sizeof(pamc::RunState), I->stream), "memset");
  HIP_TRY(hipMemsetAsync(I->Sd2, 0, (size_t)I->R * np, I->stream), "memset");
  return PAMC_OK;
}

pamc_status finish_dense(pamc_instance* I) {
  HIP_TRY(dalloc(I, &I->thr, 2 * I->X + 1), "alloc");
  I->self_dirty = true;
  HIP_TRY(pamc::launch_init_dense(I), "init kernels");
  HIP_TRY(hipStreamSynchronize(I->stream), "init");
  return PAMC_OK;
}

pamc_status check_schedule(const pamc_instance* I, const pamc_schedule* sched) {
  if (sched->steps < 0 || sched->sweeps < 0 || !std::isfinite(sched->beta0) || !std::isfinite(sched->dbeta))
    return fail(PAMC_ERR_INVALID_ARG, "bad schedule");
  if (sched->augmented &&
      (sched->win_long > pamc::kHistCap || sched->win_short > sched->win_long || sched->win_short <= 0))
    return fail(PAMC_ERR_INVALID_ARG, "history windows must satisfy 0 < short <= long <= 64");
  if (I->dense && sched->augmented)
    return fail(PAMC_ERR_UNSUPPORTED, "the augmented controller's cluster moves need a sparse instance");
  return PAMC_OK;
}

int32_t cluster_possible(const Schedule& s) {
  return (s.augmented && s.resample && s.n_top > 0 && s.mis_trials > 0) ? 1 : 0;
}

// Normalises the schedule and sizes the per-run buffers of one instance.
pamc_status prepare_run(pamc_instance* I, Schedule& s) {
  if (!s.augmented) s.win_long = std::min(std::max(s.win_long, 1), pamc::kHistCap);
  pamc_status st = ensure_trace(I, std::max(s.steps, 1));
  if (!st) st = ensure_order(I, std::max(s.sweeps, 1));
  if (!st && cluster_possible(s)) st = ensure_cluster_scratch(I, s.n_top, s.mis_trials);
  return st;
}

void fill_result(const pamc_instance* I, const pamc::RunState& r, pamc_result* out) {
  memset(out, 0, sizeof *out);
  out->best_cut = r.mstar;
  out->best_energy = I->W - 2 * r.mstar;
  out->steps_run = r.steps_run;
  out->step_reached = r.step_reached;
  out->sum_lnq = r.sum_lnq;
  out->n_cluster_moves = r.n_cluster_moves;
  out->n_reheats = r.n_reheats;
  out->n_reversals = r.n_reversals;
  out->n_restarts = r.n_restarts;
  out->seconds_total = r.steps_run > 0 ? (double)(r.t_last - r.t_start) / I->clock_hz : 0.0;
  out->seconds_to_target = r.step_reached >= 0 ? (double)(r.t_reached - r.t_start) / I->clock_hz : -1.0;
}

}  // namespace

extern "C" {

const char* pamc_last_error(void) { return g_err.c_str(); }

pamc_status pamc_create_instance_csr(int32_t n, const int32_t* row_ptr, const int32_t* col,
                                     const int32_t* w, pamc_mem where, int32_t objective,
                                     const pamc_config* cfg, pamc_instance** out) {
  if (!out) return fail(PAMC_ERR_INVALID_ARG, "NULL out");
  *out = nullptr;
  pamc_status st = check_cfg(cfg);
  if (st) return st;
  if (objective != PAMC_OBJ_MAXCUT && objective != PAMC_OBJ_ISING)
    return fail(PAMC_ERR_INVALID_ARG, "unknown objective");
  if (n <= 0 || !row_ptr) return fail(PAMC_ERR_INVALID_ARG, "n must be positive");
  std::vector<int32_t> hrp, hcol, hw;
  const int32_t *rp = row_ptr, *cl = col, *ww = w;
  if (where == PAMC_MEM_DEVICE) {
    hrp.resize(n + 1);
    if (hipMemcpy(hrp.data(), row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(PAMC_ERR_INVALID_ARG, "cannot read device row_ptr");
    const int32_t nnz = hrp[n];
    if (nnz < 0) return fail(PAMC_ERR_INVALID_ARG, "negative nnz");
    hcol.resize(std::max(nnz, 1));
    hw.resize(std::max(nnz, 1));
    if (nnz && (hipMemcpy(hcol.data(), col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(hw.data(), w, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost) != hipSuccess))
      return fail(PAMC_ERR_INVALID_ARG, "cannot read device CSR");
    rp = hrp.data();
    cl = hcol.data();
    ww = hw.data();
  } else if (where != PAMC_MEM_HOST) {
    return fail(PAMC_ERR_INVALID_ARG, "bad memory kind");
  }
  st = validate_csr(n, rp, cl, ww, false);
  if (st) return st;
  std::vector<int32_t> J(std::max(rp[n], 1));
  for (int32_t e = 0; e < rp[n]; ++e) J[e] = objective == PAMC_OBJ_MAXCUT ? -ww[e] : ww[e];
  pamc_instance* I = new (std::nothrow) pamc_instance();
  if (!I) return fail(PAMC_ERR_OUT_OF_MEMORY, "host allocation");
  st = open_device(I, cfg);
  if (!st) st = build_sparse(I, n, rp, cl, J);
  if (st) {
    free_instance(I);
    return st;
  }
  *out = I;
  return PAMC_OK;
}

pamc_status pamc_create_instance_potts(int32_t n, const int32_t* row_ptr, const int32_t* col,
                                       const int32_t* w, int32_t K, int32_t potts_rule, double gamma,
                                       const pamc_config* cfg, pamc_instance** out) {
  if (!out) return fail(PAMC_ERR_INVALID_ARG, "NULL out");
  *out = nullptr;
  pamc_status st = check_cfg(cfg);
  if (st) return st;
  if (K < 2) return fail(PAMC_ERR_INVALID_ARG, "K must be at least 2");
  if (K > 4) return fail(PAMC_ERR_UNSUPPORTED, "K > 4");
  if (potts_rule != PAMC_POTTS_SOFTMAX && potts_rule != PAMC_POTTS_CASCADE)
    return fail(PAMC_ERR_INVALID_ARG, "unknown Potts rule");
  if (potts_rule == PAMC_POTTS_CASCADE && K != 3) return fail(PAMC_ERR_INVALID_ARG, "the cascade is for K = 3");
  if (!std::isfinite(gamma) || gamma < 0) return fail(PAMC_ERR_INVALID_ARG, "gamma must be finite and >= 0");
  if (n <= 0 || !row_ptr) return fail(PAMC_ERR_INVALID_ARG, "n must be positive");
  st = validate_csr(n, row_ptr, col, w, false);
  if (st) return st;
  std::vector<int32_t> J(std::max(row_ptr[n], 1));
  for (int32_t e = 0; e < row_ptr[n]; ++e) J[e] = -w[e];
  pamc_instance* I = new (std::nothrow) pamc_instance();
  if (!I) return fail(PAMC_ERR_OUT_OF_MEMORY, "host allocation");
  I->potts_K = K;
  I->potts_rule = potts_rule;
  I->potts_gamma = gamma;
  st = open_device(I, cfg);
  if (!st) st = build_sparse(I, n, row_ptr, col, J);
  if (st) {
    free_instance(I);
    return st;
  }
  *out = I;
  return PAMC_OK;
}

pamc_status pamc_create_instance_max3cut(int32_t n, const int32_t* row_ptr, const int32_t* col,
                                         const int32_t* w, const pamc_config* cfg,
                                         pamc_instance** out) {
  if (!out) return fail(PAMC_ERR_INVALID_ARG, "NULL out");
  *out = nullptr;
  pamc_status st = check_cfg(cfg);
  if (st) return st;
  st = validate_csr(n, row_ptr, col, w, true);
  if (st) return st;
  if ((int64_t)3 * n + 1 > INT32_MAX / 4) return fail(PAMC_ERR_UNSUPPORTED, "graph too large");
  // one-hot embedding with an ancilla (see pamc.h)
  const int32_t N = 3 * n + 1, anc = 3 * n;
  std::vector<int64_t> deg(n, 0), pen(n, 0);
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) deg[i] += w[e];
    pen[i] = deg[i] / 3 + 1;
  }
  std::vector<std::vector<std::pair<int32_t, int64_t>>> adj(N);
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t a = 0; a < 3; ++a) {
      const int32_t u = 3 * i + a;
      for (int32_t b = 0; b < 3; ++b)
        if (b != a) adj[u].push_back({3 * i + b, -2 * pen[i]});
      for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) adj[u].push_back({3 * col[e] + a, -(int64_t)w[e]});
      adj[u].push_back({anc, -(2 * pen[i] + deg[i])});
      adj[anc].push_back({u, -(2 * pen[i] + deg[i])});
    }
  }
  std::vector<int32_t> rp(N + 1, 0), cl, J;
  for (int32_t u = 0; u < N; ++u) {
    std::sort(adj[u].begin(), adj[u].end());
    int64_t ab = 0;
    for (auto& p : adj[u]) {
      ab += std::llabs(p.second);
      cl.push_back(p.first);
      J.push_back((int32_t)p.second);
    }
    if (2 * ab >= INT32_MAX) return fail(PAMC_ERR_INVALID_ARG, "local field range exceeds int32");
    rp[u + 1] = (int32_t)cl.size();
  }
  // the embedding's colour classes from the base graph's colouring c with
  // k colours: spin (i, a) takes (c(i) + a) mod max(k, 3) (the spins of one
  // vertex differ by 1 or 2, those of an edge ij by c(i) != c(j)), the
  // ancilla a class of its own: max(k, 3) classes of about 3n / max(k, 3)
  // spins instead of the long tail of small classes a colouring of the
  // embedding itself gives
  std::vector<int32_t> base, m3colour(N);
  const int32_t k = dsatur_colour(n, row_ptr, col, base), m = std::max(k, 3);
  for (int32_t i = 0; i < n; ++i)
    for (int32_t a = 0; a < 3; ++a) m3colour[3 * i + a] = (base[i] + a) % m;
  m3colour[anc] = m;
  pamc_instance* I = new (std::nothrow) pamc_instance();
  if (!I) return fail(PAMC_ERR_OUT_OF_MEMORY, "host allocation");
  st = open_device(I, cfg);
  if (!st) st = build_sparse(I, N, rp.data(), cl.data(), J, &m3colour);
  if (!st) {
    I->m3_n = n;
    const int32_t nnz = row_ptr[n];
    if (dalloc(I, &I->m3_row_ptr, n + 1) || dalloc(I, &I->m3_col, std::max(nnz, 1)) ||
        dalloc(I, &I->m3_w, std::max(nnz, 1)) || dalloc(I, &I->m3_labels, n) || dalloc(I, &I->m3_cut, 1) ||
        hipMemcpy(I->m3_row_ptr, row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice) ||
        (nnz && hipMemcpy(I->m3_col, col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice)) ||
        (nnz && hipMemcpy(I->m3_w, w, sizeof(int32_t) * nnz, hipMemcpyHostToDevice)))
      st = fail(PAMC_ERR_OUT_OF_MEMORY, "Max-3-Cut buffers");
  }
  if (st) {
    free_instance(I);
    return st;
  }
  *out = I;
  return PAMC_OK;
}

pamc_status pamc_create_instance_dense_i8(int32_t n, const int8_t* J, int64_t ld, pamc_mem where,
                                          int32_t objective, const pamc_config* cfg,
                                          pamc_instance** out) {
  if (!out) return fail(PAMC_ERR_INVALID_ARG, "NULL out");
  *out = nullptr;
  pamc_status st = check_cfg(cfg);
  if (st) return st;
  if (n <= 0 || !J || ld < n) return fail(PAMC_ERR_INVALID_ARG, "bad dense matrix arguments");
  if (objective != PAMC_OBJ_MAXCUT && objective != PAMC_OBJ_ISING)
    return fail(PAMC_ERR_INVALID_ARG, "unknown objective");
  std::vector<int8_t> hj;
  const int8_t* src = J;
  if (where == PAMC_MEM_DEVICE) {
    hj.resize((size_t)n * ld);
    if (hipMemcpy(hj.data(), J, hj.size(), hipMemcpyDeviceToHost) != hipSuccess)
      return fail(PAMC_ERR_INVALID_ARG, "cannot read device matrix");
    src = hj.data();
  } else if (where != PAMC_MEM_HOST) {
    return fail(PAMC_ERR_INVALID_ARG, "bad memory kind");
  }
  int64_t W = 0, X = 0;
  int32_t maxabs = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (src[(size_t)i * ld + i] != 0) return fail(PAMC_ERR_INVALID_ARG, "nonzero diagonal");
    int64_t ab = 0;
    for (int32_t j = 0; j < n; ++j) {
      const int8_t v = src[(size_t)i * ld + j];
      if (v == -128) return fail(PAMC_ERR_INVALID_ARG, "entries must lie in [-127, 127]");
      if (v != src[(size_t)j * ld + i]) return fail(PAMC_ERR_INVALID_ARG, "matrix is not symmetric");
      maxabs = std::max(maxabs, (int32_t)(v < 0 ? -v : v));
      ab += v < 0 ? -v : v;
      if (j > i) W += objective == PAMC_OBJ_MAXCUT ? v : -v;
    }
    X = std::max(X, ab);
  }
  if (2 * X >= INT32_MAX) return fail(PAMC_ERR_INVALID_ARG, "local field range exceeds int32");
  // the dense sweep sums a block's 64 energy changes in 32 bits
  if (X >= (1 << 25)) return fail(PAMC_ERR_UNSUPPORTED, "dense couplings with max_v sum_j |J_vj| >= 2^25");
  pamc_instance* I = new (std::nothrow) pamc_instance();
  if (!I) return fail(PAMC_ERR_OUT_OF_MEMORY, "host allocation");
  st = open_device(I, cfg);
  if (!st) st = build_dense_common(I, n);
  if (!st) {
    I->W = W;
    I->X = X;
    I->dense_j4 = maxabs <= 7;  // stored couplings are v or -v
    const size_t np = (size_t)I->dn_pad;
    std::vector<int8_t> row(np);
    hipError_t e = hipMemsetAsync(I->Jd, 0, np * np, I->stream);
    for (int32_t i = 0; i < n && e == hipSuccess; ++i) {
      std::fill(row.begin(), row.end(), 0);
      for (int32_t j = 0; j < n; ++j) {
        const int8_t v = src[(size_t)i * ld + j];
        row[j] = objective == PAMC_OBJ_MAXCUT ? (int8_t)-v : v;
      }
      e = hipMemcpy(I->Jd + (size_t)i * np, row.data(), np, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) st = dev_fail(e, "upload couplings");
  }
  if (!st) st = finish_dense(I);
  if (st) {
    free_instance(I);
    return st;
  }
  *out = I;
  return PAMC_OK;
}

pamc_status pamc_create_instance_dense_random(int32_t n, uint64_t graph_seed, const pamc_config* cfg,
                                              pamc_instance** out) {
  if (!out) return fail(PAMC_ERR_INVALID_ARG, "NULL out");
  *out = nullptr;
  pamc_status st = check_cfg(cfg);
  if (st) return st;
  if (n <= 1) return fail(PAMC_ERR_INVALID_ARG, "n must be at least 2");
  if (n > 400000) return fail(PAMC_ERR_UNSUPPORTED, "n too large for one device");
  pamc_instance* I = new (std::nothrow) pamc_instance();
  if (!I) return fail(PAMC_ERR_OUT_OF_MEMORY, "host allocation");
  st = open_device(I, cfg);
  if (!st) st = build_dense_common(I, n);
  if (!st) {
    I->X = n - 1;
    I->dense_j4 = 1;  // +-1 couplings
    hipError_t e = pamc::launch_dense_generate(I, graph_seed);
    int64_t W = 0;
    if (e == hipSuccess) e = hipStreamSynchronize(I->stream);
    if (e == hipSuccess) e = hipMemcpy(&W, I->flip_ctr + 400, sizeof(int64_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) st = dev_fail(e, "generate couplings");
    I->W = W;
  }
  if (!st) st = finish_dense(I);
  if (st) {
    free_instance(I);
    return st;
  }
  *out = I;
  return PAMC_OK;
}

void pamc_destroy_instance(pamc_instance* inst) { free_instance(inst); }

pamc_status pamc_reset_population(pamc_instance* I, uint64_t seed) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  hipSetDevice(I->device);
  I->seed = seed;
  I->self_dirty = true;  // the descriptor carries the key
  SELF_BATCH(I, b);
  if (I->dense) {
    HIP_TRY(pamc::launch_init_dense(I), "init kernels");
  } else {
    HIP_TRY(pamc::batch_init(*b), "init kernels");
  }
  return PAMC_OK;
}

pamc_status pamc_get_info(const pamc_instance* I, pamc_info* out) {
  if (!I || !out) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  out->n = I->n;
  out->replicas = I->R;
  out->num_classes = I->ncls;
  out->dense = I->dense;
  out->pull = I->pull;
  out->nnz = I->nnz;
  out->W = I->W;
  out->X = I->X;
  out->device_bytes = I->device_bytes;
  out->tiles_per_wave = I->tpw;
  out->quads_per_wave = I->qpw;
  out->coupling_mode = I->jmode;
  out->potts_K = I->potts_K;
  out->tile_sweeps = I->tile;
  out->hubs = I->nhub;
  return PAMC_OK;
}

pamc_status pamc_sweep(pamc_instance* I, double beta, int32_t nsweeps) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  if (nsweeps < 0 || !std::isfinite(beta)) return fail(PAMC_ERR_INVALID_ARG, "bad sweep arguments");
  if (I->potts_K && beta < 0) return fail(PAMC_ERR_INVALID_ARG, "negative beta on Potts labels");
  if (nsweeps == 0) return PAMC_OK;
  hipSetDevice(I->device);
  SELF_BATCH(I, b);
  if (I->dense) {
    HIP_TRY(pamc::launch_dense_prim_sweep(*b, beta, nsweeps), "dense sweep");
    return PAMC_OK;
  }
  HIP_TRY(pamc::prim_sweep(*b, beta, nsweeps), "sweep");
  return PAMC_OK;
}

pamc_status pamc_resample(pamc_instance* I, double delta, double* log_q) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  if (!std::isfinite(delta)) return fail(PAMC_ERR_INVALID_ARG, "delta must be finite");
  hipSetDevice(I->device);
  SELF_BATCH(I, b);
  if (I->dense) {
    HIP_TRY(pamc::launch_dense_prim_resample(*b, delta), "dense resample");
  } else {
    HIP_TRY(pamc::prim_resample(*b, delta), "resample");
  }
  if (log_q) {
    pamc::RunState s;
    pamc_status r = read_state(I, &s);
    if (r) return r;
    *log_q = s.last_lnq;
  }
  return PAMC_OK;
}

pamc_status pamc_cluster_move(pamc_instance* I, int32_t n_top, int32_t mis_trials, int32_t* flipped) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  if (n_top < 0 || mis_trials < 0) return fail(PAMC_ERR_INVALID_ARG, "negative argument");
  if (I->dense) return fail(PAMC_ERR_UNSUPPORTED, "cluster moves on dense instances");
  if (I->potts_K) return fail(PAMC_ERR_UNSUPPORTED, "cluster moves on Potts labels");
  hipSetDevice(I->device);
  pamc_status st = ensure_cluster_scratch(I, n_top, mis_trials);
  if (st) return st;
  int64_t* ctr = I->flip_ctr + 256;
  SELF_BATCH(I, b);
  HIP_TRY(hipMemsetAsync(ctr, 0, sizeof(int64_t), I->stream), "memset");
  HIP_TRY(pamc::prim_cluster(*b, n_top, mis_trials), "cluster move");
  if (flipped) {
    int64_t f = 0;
    HIP_TRY(hipStreamSynchronize(I->stream), "cluster move");
    HIP_TRY(hipMemcpy(&f, ctr, sizeof(int64_t), hipMemcpyDeviceToHost), "readback");
    *flipped = (int32_t)f;
  }
  return PAMC_OK;
}

pamc_status pamc_update_best(pamc_instance* I) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  hipSetDevice(I->device);
  SELF_BATCH(I, b);
  if (I->dense) {
    HIP_TRY(pamc::launch_dense_prim_update_best(*b), "best");
  } else {
    HIP_TRY(pamc::prim_update_best(*b), "best");
  }
  return PAMC_OK;
}

pamc_status pamc_best(pamc_instance* I, int64_t* cut, int64_t* energy, int8_t* spins) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  hipSetDevice(I->device);
  pamc::RunState s;
  pamc_status r = read_state(I, &s);
  if (r) return r;
  if (cut) *cut = s.mstar;
  if (energy) *energy = I->W - 2 * s.mstar;
  if (spins) {
    std::vector<int8_t> b(I->np);
    HIP_TRY(hipMemcpy(b.data(), I->best, I->np, hipMemcpyDeviceToHost), "readback");
    for (int32_t v = 0; v < I->n; ++v) spins[v] = b[I->dense ? v : I->to_internal[v]];
  }
  return PAMC_OK;
}

pamc_status pamc_get_state(pamc_instance* I, int8_t* spins, int32_t* fields, int64_t* energies,
                           int32_t* family) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  hipSetDevice(I->device);
  pamc::RunState s;
  pamc_status r = read_state(I, &s);
  if (r) return r;
  const int b = s.cur;
  if (I->dense) {
    const size_t np = (size_t)I->dn_pad;
    if (spins) {
      std::vector<int8_t> S((size_t)I->R * np);
      HIP_TRY(hipMemcpy(S.data(), b ? I->Sd2 : I->Sd, S.size(), hipMemcpyDeviceToHost), "readback");
      for (int32_t rr = 0; rr < I->R; ++rr) memcpy(spins + (size_t)rr * I->n, &S[(size_t)rr * np], I->n);
    }
    if (fields) {
      if (!I->H_scratch) HIP_TRY(dalloc(I, &I->H_scratch, (size_t)I->R * np), "alloc fields");
      HIP_TRY(pamc::launch_dense_fields(I, I->H_scratch), "fields");
      std::vector<int32_t> H((size_t)I->R * np);
      HIP_TRY(hipStreamSynchronize(I->stream), "fields");
      HIP_TRY(hipMemcpy(H.data(), I->H_scratch, H.size() * 4, hipMemcpyDeviceToHost), "readback");
      for (int32_t rr = 0; rr < I->R; ++rr)
        memcpy(fields + (size_t)rr * I->n, &H[(size_t)rr * np], sizeof(int32_t) * I->n);
    }
    if (energies) HIP_TRY(hipMemcpy(energies, I->pop.E[b], sizeof(int64_t) * I->R, hipMemcpyDeviceToHost), "readback");
    if (family) HIP_TRY(hipMemcpy(family, I->pop.fam[b], sizeof(int32_t) * I->R, hipMemcpyDeviceToHost), "readback");
    return PAMC_OK;
  }
  const int n = I->n, R = I->R;
  if (spins) {
    std::vector<uint32_t> S((size_t)I->T * I->nq * 64);
    HIP_TRY(hipMemcpy(S.data(), I->pop.S[b], S.size() * 4, hipMemcpyDeviceToHost), "readback");
    for (int32_t rr = 0; rr < R; ++rr)
      for (int32_t v = 0; v < n; ++v) {
        const int32_t iv = I->to_internal[v];
        const uint32_t w = S[((size_t)(rr >> 6) * I->nq + (iv >> 2)) * 64 + (rr & 63)];
        spins[(size_t)rr * n + v] = (int8_t)(w >> (8 * (iv & 3)));
      }
  }
  if (fields) {
    std::vector<int32_t> H((size_t)I->T * I->np * 64);
    const int32_t* src = I->pop.H[b];
    if (I->pull) {
      if (!I->H_scratch) HIP_TRY(dalloc(I, &I->H_scratch, H.size()), "alloc fields");
      SELF_BATCH(I, sb);
      HIP_TRY(pamc::launch_fields(*sb, b, I->H_scratch), "fields");
      HIP_TRY(hipStreamSynchronize(I->stream), "fields");
      src = I->H_scratch;
    }
    HIP_TRY(hipMemcpy(H.data(), src, H.size() * 4, hipMemcpyDeviceToHost), "readback");
    for (int32_t rr = 0; rr < R; ++rr)
      for (int32_t v = 0; v < n; ++v)
        fields[(size_t)rr * n + v] = H[((size_t)(rr >> 6) * I->np + I->to_internal[v]) * 64 + (rr & 63)];
  }
  if (energies) HIP_TRY(hipMemcpy(energies, I->pop.E[b], sizeof(int64_t) * R, hipMemcpyDeviceToHost), "readback");
  if (family) HIP_TRY(hipMemcpy(family, I->pop.fam[b], sizeof(int32_t) * R, hipMemcpyDeviceToHost), "readback");
  return PAMC_OK;
}

// An instance keeping both field forms (hub graphs) switches between them:
// the fields the new form keeps are recomputed from the current population,
// so the trajectory is the same in either (the fields are exact integers).
static pamc_status set_field_mode(pamc_instance* I, bool pull) {
  if (!I->dual || (I->pull != 0) == pull) return PAMC_OK;
  const int32_t was_pull = I->pull, was_tpw = I->tpw, was_qpw = I->qpw;
  I->pull = pull ? 1 : 0;
  I->tpw = pull ? I->hub_tpw : I->push_tpw;
  I->qpw = pull ? I->hub_qpw : I->push_qpw;
  I->self_dirty = true;
  hipError_t e;
  pamc::Batch* b = self_batch(I, &e);
  if (b) e = pamc::launch_refresh_fields(*b);
  if (e != hipSuccess) {  // the previous form's fields are still current: keep it
    I->pull = was_pull;
    I->tpw = was_tpw;
    I->qpw = was_qpw;
    I->self_dirty = true;
    return dev_fail(e, "field form switch");
  }
  return PAMC_OK;
}

// The steps a run of an instance keeping both field forms makes with
// gathered fields (the hubs' fields kept) before it switches to incremental
// ones: those whose scheduled beta, beta0 + k dbeta (before any reheat),
// lies below kDualSwitchBeta.  At low beta a hub flips often, and with
// incremental fields every such flip walks the hub's whole row from one
// wavefront; at higher beta incremental fields cost less per attempt.  On
// the Max-3-Cut embedding of G(7000, 21000) the per-step times of the two
// forms cross near beta 0.7-0.8 (PAMC_HUB_SWITCH_BETA overrides).  Resumed
// runs keep the current form.
constexpr double kDualSwitchBeta = 0.8;
static int32_t dual_field_steps(const pamc_instance* I, const Schedule& s) {
  if (!I->dual || s.resume || s.steps <= 0) return 0;
  double bsw = kDualSwitchBeta;
  if (const char* e = getenv("PAMC_HUB_SWITCH_BETA")) bsw = atof(e);
  if (!(s.dbeta > 0.0)) return s.beta0 < bsw ? s.steps : 0;
  const double k = std::ceil((bsw - s.beta0) / s.dbeta);
  return (int32_t)std::max(0.0, std::min((double)s.steps, k));
}

pamc_status pamc_anneal(pamc_instance* I, const pamc_schedule* sched, pamc_result* out) {
  if (!I || !sched || !out) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  pamc_status st = check_schedule(I, sched);
  if (st) return st;
  hipSetDevice(I->device);
  Schedule s = to_sched(sched);
  st = prepare_run(I, s);
  if (st) return st;
  const int32_t kd = dual_field_steps(I, s);
  if (kd > 0) {
    st = set_field_mode(I, true);
    if (st) return st;
  }
  SELF_BATCH(I, b);
  auto run_flags = [&](pamc::Batch* x) {
    x->max_sweeps = std::max(s.sweeps, 1);
    x->any_cluster = cluster_possible(s);
    x->any_dh = s.dh_every > 0 && x->dh.grid > 0;
  };
  run_flags(b);
  if (!I->d_sched) HIP_TRY(dev_alloc(I, &I->d_sched, sizeof(Schedule)), "alloc");
  HIP_TRY(hipMemcpyAsync(I->d_sched, &s, sizeof(Schedule), hipMemcpyHostToDevice, I->stream), "upload");
  HIP_TRY(pamc::batch_anneal_setup(*b, (const Schedule*)I->d_sched, nullptr, 1), "anneal setup");
  // steps in chunks of 16 between polls of the stop flag when stopping at
  // the target, else all at once (and the switch of field form, if any)
  const int32_t chunk = s.stop_at_target ? 16 : std::max(s.steps, 1);
  for (int32_t done = 0; done < s.steps;) {
    int32_t k = std::min(chunk, s.steps - done);
    if (kd > done) k = std::min(k, kd - done);
    if (I->dense) {
      for (int32_t i = 0; i < k; ++i) HIP_TRY(pamc::launch_dense_step(*b, s.sweeps, s.resample), "dense step");
    } else {
      HIP_TRY(pamc::batch_run_steps(*b, k), "step");
    }
    done += k;
    if (done == kd && I->pull) {
      st = set_field_mode(I, false);
      if (st) return st;
      hipError_t e2;
      b = self_batch(I, &e2);
      if (!b) return dev_fail(e2, "batch descriptors");
      run_flags(b);
    }
    if (s.stop_at_target && done < s.steps) {
      HIP_TRY(hipMemcpyAsync(I->pinned, &I->st->stopped, sizeof(int32_t), hipMemcpyDeviceToHost, I->stream), "poll");
      HIP_TRY(hipStreamSynchronize(I->stream), "poll");
      if (*(volatile int32_t*)I->pinned) break;
    }
  }
  if (I->dual && I->pull) {  // a run that stopped before the switch
    st = set_field_mode(I, false);
    if (st) return st;
  }
  pamc::RunState r;
  st = read_state(I, &r);
  if (!st && I->prof) st = resolve_events(I);
  if (st) return st;
  I->trace_ok = true;
  fill_result(I, r, out);
  return PAMC_OK;
}

pamc_status pamc_anneal_batch(pamc_instance* const* insts, const pamc_schedule* scheds, int32_t count,
                              pamc_result* out) {
  if (count < 0 || (count > 0 && (!insts || !scheds || !out))) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  if (count == 0) return PAMC_OK;
  std::vector<pamc_instance*> v(insts, insts + count);
  for (int32_t i = 0; i < count; ++i) {
    if (!v[i]) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
    if (v[i]->dense) return fail(PAMC_ERR_UNSUPPORTED, "batched runs take sparse instances");
    if (v[i]->device != v[0]->device) return fail(PAMC_ERR_INVALID_ARG, "instances on different devices");
    for (int32_t j = 0; j < i; ++j)
      if (v[j] == v[i]) return fail(PAMC_ERR_INVALID_ARG, "an instance appears twice");
    pamc_status st = check_schedule(v[i], &scheds[i]);
    if (st) return st;
  }
  hipSetDevice(v[0]->device);
  std::vector<Schedule> s(count);
  int32_t max_steps = 0, any_stop = 0;
  for (int32_t i = 0; i < count; ++i) {
    s[i] = to_sched(&scheds[i]);
    pamc_status st = prepare_run(v[i], s[i]);
    if (st) return st;
    max_steps = std::max(max_steps, s[i].steps);
    any_stop |= s[i].stop_at_target;
  }
  // instances keeping both field forms start in the gathered one and switch
  // at their own step (dual_field_steps); the batch is rebuilt there
  std::vector<int32_t> kd(count), cuts;
  for (int32_t i = 0; i < count; ++i) {
    kd[i] = dual_field_steps(v[i], s[i]);
    if (kd[i] > 0) {
      pamc_status st = set_field_mode(v[i], true);
      if (st) return st;
      if (kd[i] < max_steps) cuts.push_back(kd[i]);
    }
  }
  std::sort(cuts.begin(), cuts.end());
  cuts.erase(std::unique(cuts.begin(), cuts.end()), cuts.end());
  // every instance's queued work is finished before the batch takes over
  for (pamc_instance* I : v) HIP_TRY(hipStreamSynchronize(I->stream), "sync");
  pamc::Batch b;
  if (v[0]->use_al) b.al = &v[0]->al;  // the batch's memory from the first instance's provider
  HIP_TRY(pamc::batch_build(b, v, &s), "batch descriptors");
  Schedule* d_sched = nullptr;
  int32_t* d_status = nullptr;
  hipError_t e = pamc::batch_alloc(b, (void**)&d_sched, sizeof(Schedule) * count);
  if (e == hipSuccess) e = pamc::batch_alloc(b, (void**)&d_status, sizeof(int32_t) * count);
  if (e == hipSuccess) e = hipMemcpyAsync(d_sched, s.data(), sizeof(Schedule) * count, hipMemcpyHostToDevice, b.stream);
  if (e == hipSuccess) e = pamc::batch_anneal_setup(b, d_sched, nullptr, count);
  std::vector<int32_t> status(count);
  const int32_t chunk = any_stop ? 16 : std::max(max_steps, 1);
  size_t next_cut = 0;
  pamc_status sw = PAMC_OK;
  for (int32_t done = 0; done < max_steps && e == hipSuccess && !sw;) {
    int32_t k = std::min(chunk, max_steps - done);
    if (next_cut < cuts.size()) k = std::min(k, cuts[next_cut] - done);
    e = pamc::batch_run_steps(b, k);
    done += k;
    if (e == hipSuccess && next_cut < cuts.size() && done == cuts[next_cut]) {
      // the instances whose switch falls here take incremental fields
      e = hipStreamSynchronize(b.stream);
      for (int32_t i = 0; i < count && e == hipSuccess && !sw; ++i)
        if (kd[i] == done) {
          sw = set_field_mode(v[i], false);
          if (!sw) e = hipStreamSynchronize(v[i]->stream);
        }
      if (e == hipSuccess && !sw) e = pamc::batch_build(b, v, &s);
      ++next_cut;
    }
    if (e == hipSuccess && !sw && any_stop && done < max_steps) {
      e = pamc::batch_status(b, d_status);
      if (e == hipSuccess) e = hipMemcpyAsync(status.data(), d_status, sizeof(int32_t) * count, hipMemcpyDeviceToHost, b.stream);
      if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
      bool all = true;
      for (int32_t x : status) all = all && (x & 1);
      if (all) break;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
  // instances that stopped before their switch
  for (int32_t i = 0; i < count && e == hipSuccess && !sw; ++i)
    if (v[i]->dual && v[i]->pull) sw = set_field_mode(v[i], false);
  for (void* p : {(void*)d_sched, (void*)d_status}) {
    if (!p) continue;
    if (b.al)
      b.al->free(b.al->ctx, p, (void*)b.stream);
    else
      hipFree(p);
  }
  if (sw) return sw;
  if (e != hipSuccess) return dev_fail(e, "batched run");
  for (int32_t i = 0; i < count; ++i) {
    pamc::RunState r;
    pamc_status st = read_state(v[i], &r);
    if (st) return st;
    v[i]->trace_ok = true;
    fill_result(v[i], r, &out[i]);
  }
  return PAMC_OK;
}

pamc_status pamc_anneal_batch_noalloc(pamc_instance* const* insts, const pamc_schedule* scheds, int32_t count,
                                      pamc_result* out) {
  if (count < 0 || (count > 0 && (!insts || !scheds || !out))) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  if (count == 0) return PAMC_OK;
  std::vector<pamc_instance*> v(insts, insts + count);
  for (int32_t i = 0; i < count; ++i) {
    if (!v[i]) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
    if (v[i]->dense) return fail(PAMC_ERR_UNSUPPORTED, "batched runs take sparse instances");
    if (v[i]->device != v[0]->device) return fail(PAMC_ERR_INVALID_ARG, "instances on different devices");
    for (int32_t j = 0; j < i; ++j)
      if (v[j] == v[i]) return fail(PAMC_ERR_INVALID_ARG, "an instance appears twice");
    pamc_status st = check_schedule(v[i], &scheds[i]);
    if (st) return st;
  }
  hipSetDevice(v[0]->device);
  std::vector<Schedule> s(count);
  int32_t max_steps = 0, any_stop = 0;
  for (int32_t i = 0; i < count; ++i) {
    s[i] = to_sched(&scheds[i]);
    if (!s[i].augmented) s[i].win_long = std::min(std::max(s[i].win_long, 1), pamc::kHistCap);
    if (cluster_possible(s[i]) && !v[i]->potts_K) {
      if (v[i]->n > pamc::cluster_max_n()) return fail(PAMC_ERR_UNSUPPORTED, "cluster moves need n <= 26000");
      if (s[i].mis_trials > 64) return fail(PAMC_ERR_UNSUPPORTED, "mis_trials > 64");
    }
    max_steps = std::max(max_steps, s[i].steps);
    any_stop |= s[i].stop_at_target;
  }
  void* scratch = nullptr;
  size_t cap = 0;
  HIP_TRY(pamc::fixed_scratch(&scratch, &cap), "hipGetSymbolAddress");
  for (pamc_instance* I : v) HIP_TRY(hipStreamSynchronize(I->stream), "sync");
  pamc::Batch b;
  b.arena = (char*)scratch;
  b.arena_cap = cap;
  hipError_t e = pamc::batch_build(b, v, &s);
  pamc::Schedule* d_sched = nullptr;
  int32_t* d_status = nullptr;
  if (e == hipSuccess) e = pamc::batch_alloc(b, (void**)&d_sched, sizeof(Schedule) * count);
  if (e == hipSuccess) e = pamc::batch_alloc(b, (void**)&d_status, sizeof(int32_t) * count);
  if (e == hipErrorOutOfMemory)
    return fail(PAMC_ERR_UNSUPPORTED, "this batch needs " + std::to_string(b.arena_need) +
                                          " bytes of device scratch; the fixed scratch holds " +
                                          std::to_string(cap));
  if (e != hipSuccess) return dev_fail(e, "batch descriptors");
  e = hipMemcpyAsync(d_sched, s.data(), sizeof(Schedule) * count, hipMemcpyHostToDevice, b.stream);
  if (e == hipSuccess) e = pamc::batch_anneal_setup(b, d_sched, nullptr, count);
  std::vector<int32_t> status(count);
  const int32_t chunk = any_stop ? 16 : std::max(max_steps, 1);
  for (int32_t done = 0; done < max_steps && e == hipSuccess; done += chunk) {
    e = pamc::batch_run_steps(b, std::min(chunk, max_steps - done));
    if (e == hipSuccess && any_stop && done + chunk < max_steps) {
      e = pamc::batch_status(b, d_status);
      if (e == hipSuccess) e = hipMemcpyAsync(status.data(), d_status, sizeof(int32_t) * count, hipMemcpyDeviceToHost, b.stream);
      if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
      bool all = true;
      for (int32_t x : status) all = all && (x & 1);
      if (all) break;
    }
  }
  // the scratch is reused by the next call: nothing may still read it
  if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
  if (e != hipSuccess) return dev_fail(e, "batched run");
  for (int32_t i = 0; i < count; ++i) {
    pamc::RunState r;
    pamc_status st = read_state(v[i], &r);
    if (st) return st;
    v[i]->trace_ok = false;  // no trace was recorded
    fill_result(v[i], r, &out[i]);
  }
  return PAMC_OK;
}

pamc_status pamc_get_trace(pamc_instance* I, int32_t capacity, int64_t* mstar, double* beta, double* lnq,
                           int32_t* events, double* seconds, int32_t* steps) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  hipSetDevice(I->device);
  pamc::RunState r;
  pamc_status st = read_state(I, &r);
  if (st) return st;
  const int32_t k = I->trace_ok ? std::min(std::min(capacity, r.steps_run), I->tr_cap) : 0;
  if (steps) *steps = k;
  if (k <= 0) return PAMC_OK;
  if (mstar) HIP_TRY(hipMemcpy(mstar, I->tr_mstar, sizeof(int64_t) * k, hipMemcpyDeviceToHost), "readback");
  if (beta) HIP_TRY(hipMemcpy(beta, I->tr_beta, sizeof(double) * k, hipMemcpyDeviceToHost), "readback");
  if (lnq) HIP_TRY(hipMemcpy(lnq, I->tr_lnq, sizeof(double) * k, hipMemcpyDeviceToHost), "readback");
  if (events) HIP_TRY(hipMemcpy(events, I->tr_events, sizeof(int32_t) * k, hipMemcpyDeviceToHost), "readback");
  if (seconds) {
    std::vector<uint64_t> t(k);
    HIP_TRY(hipMemcpy(t.data(), I->tr_time, sizeof(uint64_t) * k, hipMemcpyDeviceToHost), "readback");
    for (int32_t i = 0; i < k; ++i) seconds[i] = (double)(t[i] - r.t_start) / I->clock_hz;
  }
  return PAMC_OK;
}

pamc_status pamc_max3cut_decode(pamc_instance* I, const int8_t* spins, int32_t* labels, int64_t* cut3) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  if (I->m3_n <= 0) return fail(PAMC_ERR_STATE, "not a Max-3-Cut instance");
  hipSetDevice(I->device);
  int8_t* src = I->best;
  int8_t* tmp = nullptr;
  if (spins) {
    std::vector<int8_t> internal(I->np, 1);
    for (int32_t v = 0; v < I->n; ++v) internal[I->to_internal[v]] = spins[v];
    HIP_TRY(dev_alloc(I, (void**)&tmp, I->np), "alloc");
    HIP_TRY(hipMemcpyAsync(tmp, internal.data(), I->np, hipMemcpyHostToDevice, I->stream), "upload");
    src = tmp;
  }
  hipError_t e = pamc::launch_m3_decode(I, src);
  if (e == hipSuccess) e = hipStreamSynchronize(I->stream);
  if (e == hipSuccess && labels) e = hipMemcpy(labels, I->m3_labels, sizeof(int32_t) * I->m3_n, hipMemcpyDeviceToHost);
  if (e == hipSuccess && cut3) e = hipMemcpy(cut3, I->m3_cut, sizeof(int64_t), hipMemcpyDeviceToHost);
  dev_free(I, tmp);
  if (e != hipSuccess) return dev_fail(e, "max3cut decode");
  return PAMC_OK;
}

pamc_status pamc_pair_distance(pamc_instance* I, double* mean) {
  if (!I || !mean) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  if (I->dense) return fail(PAMC_ERR_UNSUPPORTED, "pair distance on dense instances");
  if (I->potts_K) return fail(PAMC_ERR_UNSUPPORTED, "pair distance on Potts labels");
  hipSetDevice(I->device);
  double* d = (double*)(I->flip_ctr + 300);
  HIP_TRY(pamc::launch_pair_distance(I, d), "pair distance");
  double v = 0.0;
  HIP_TRY(hipStreamSynchronize(I->stream), "pair distance");
  HIP_TRY(hipMemcpy(&v, d, sizeof(double), hipMemcpyDeviceToHost), "readback");
  *mean = I->R > 1 ? v / ((double)I->R * (I->R - 1) / 2.0) : 0.0;
  return PAMC_OK;
}

}  // extern "C"

namespace {

// Population from the host (spins [R][n] in caller ids, lineage [R]) into
// buffer 0, fields and energies recomputed on the device; waits.
pamc_status load_population(pamc_instance* I, const int8_t* spins, const int32_t* family) {
  const int32_t n = I->n, R = I->R;
  for (size_t k = 0; k < (size_t)R * n; ++k) {
    const int8_t x = spins[k];
    if (I->potts_K ? (x < 0 || x >= I->potts_K) : (x != 1 && x != -1))
      return fail(PAMC_ERR_INVALID_ARG, I->potts_K ? "label out of range" : "spins must be -1 or +1");
  }
  std::vector<int32_t> fam(R);
  for (int32_t r = 0; r < R; ++r) fam[r] = family ? family[r] : r;
  HIP_TRY(hipStreamSynchronize(I->stream), "sync");
  if (I->dense) {
    const size_t np = (size_t)I->dn_pad;
    std::vector<int8_t> S((size_t)R * np, 0);
    for (int32_t r = 0; r < R; ++r) memcpy(&S[(size_t)r * np], spins + (size_t)r * n, n);
    HIP_TRY(hipMemcpy(I->Sd, S.data(), S.size(), hipMemcpyHostToDevice), "upload");
    HIP_TRY(hipMemcpy(I->pop.fam[0], fam.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice), "upload");
    HIP_TRY(pamc::launch_dense_load(I), "energies");
  } else {
    std::vector<uint32_t> S((size_t)I->T * I->nq * 64, 0u);
    for (int32_t r = 0; r < R; ++r)
      for (int32_t v = 0; v < n; ++v) {
        const int32_t iv = I->to_internal[v];
        uint32_t& w = S[((size_t)(r >> 6) * I->nq + (iv >> 2)) * 64 + (r & 63)];
        w |= (uint32_t)(uint8_t)spins[(size_t)r * n + v] << (8 * (iv & 3));
      }
    HIP_TRY(hipMemcpy(I->pop.S[0], S.data(), S.size() * 4, hipMemcpyHostToDevice), "upload");
    HIP_TRY(hipMemcpy(I->pop.fam[0], fam.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice), "upload");
    SELF_BATCH(I, b);
    HIP_TRY(pamc::launch_load_population(*b), "fields and energies");
  }
  HIP_TRY(hipStreamSynchronize(I->stream), "fields and energies");
  return PAMC_OK;
}

pamc_status write_state(pamc_instance* I, const pamc::RunState& r) {
  HIP_TRY(hipMemcpy(I->st, &r, sizeof(pamc::RunState), hipMemcpyHostToDevice), "upload");
  return PAMC_OK;
}

int64_t checkpoint_bytes(const pamc_instance* I) {
  return PAMC_CHECKPOINT_HEADER_BYTES + (int64_t)I->R * I->n + 4 * (int64_t)I->R + I->n;
}

uint32_t checkpoint_kind(const pamc_instance* I) { return I->dense ? 2u : (I->potts_K ? 1u : 0u); }

template <typename T>
void put(uint8_t* buf, size_t off, T v) {
  memcpy(buf + off, &v, sizeof(T));
}
template <typename T>
T get(const uint8_t* buf, size_t off) {
  T v;
  memcpy(&v, buf + off, sizeof(T));
  return v;
}

}  // namespace

extern "C" {

pamc_status pamc_set_state(pamc_instance* I, const int8_t* spins, const int32_t* family, const uint32_t* counters) {
  if (!I || !spins) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  hipSetDevice(I->device);
  pamc_status st = load_population(I, spins, family);
  if (st) return st;
  pamc::RunState r;
  st = read_state(I, &r);
  if (st) return st;
  if (counters) {
    r.gs = counters[0];
    r.g_rs = counters[1];
    r.g_cl = counters[2];
  }
  r.cur = 0;
  return write_state(I, r);
}

pamc_status pamc_checkpoint_size(const pamc_instance* I, int64_t* bytes) {
  if (!I || !bytes) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  *bytes = checkpoint_bytes(I);
  return PAMC_OK;
}

pamc_status pamc_get_checkpoint(pamc_instance* I, void* buf, int64_t bytes) {
  if (!I || !buf) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  const int64_t need = checkpoint_bytes(I);
  if (bytes < need) return fail(PAMC_ERR_INVALID_ARG, "checkpoint buffer too small");
  hipSetDevice(I->device);
  pamc::RunState r;
  pamc_status st = read_state(I, &r);
  if (st) return st;
  const int32_t n = I->n, R = I->R;
  uint8_t* b = (uint8_t*)buf;
  memset(b, 0, PAMC_CHECKPOINT_HEADER_BYTES);
  memcpy(b, "PAMCCKP1", 8);
  put<uint32_t>(b, 8, 1u);
  put<uint32_t>(b, 12, checkpoint_kind(I));
  put<int32_t>(b, 16, n);
  put<int32_t>(b, 20, R);
  put<uint64_t>(b, 24, I->seed);
  put<uint32_t>(b, 32, r.gs);
  put<uint32_t>(b, 36, r.g_rs);
  put<uint32_t>(b, 40, r.g_cl);
  put<int64_t>(b, 48, r.mstar);
  put<double>(b, 56, r.beta);
  put<double>(b, 64, r.delta);
  const int32_t ints[12] = {r.z, r.cycle, r.cooldown, r.enable ? 1 : 0, r.hist_len, r.steps_run, r.step_reached,
                            r.n_cluster_moves, r.n_reheats, r.n_reversals, r.n_restarts, 0};
  memcpy(b + 72, ints, sizeof ints);
  put<double>(b, 120, r.sum_lnq);
  for (int i = 0; i < pamc::kHistCap; ++i) put<int64_t>(b, 128 + 8 * (size_t)i, i < r.hist_len ? r.hist[i] : 0);
  std::vector<int32_t> fam(R);
  st = pamc_get_state(I, (int8_t*)b + PAMC_CHECKPOINT_HEADER_BYTES, nullptr, nullptr, fam.data());
  if (st) return st;
  memcpy(b + PAMC_CHECKPOINT_HEADER_BYTES + (size_t)R * n, fam.data(), 4 * (size_t)R);
  return pamc_best(I, nullptr, nullptr, (int8_t*)b + PAMC_CHECKPOINT_HEADER_BYTES + (size_t)R * n + 4 * (size_t)R);
}

pamc_status pamc_set_checkpoint(pamc_instance* I, const void* buf, int64_t bytes) {
  if (!I || !buf) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  const uint8_t* b = (const uint8_t*)buf;
  if (bytes < PAMC_CHECKPOINT_HEADER_BYTES || memcmp(b, "PAMCCKP1", 8) != 0 || get<uint32_t>(b, 8) != 1u)
    return fail(PAMC_ERR_INVALID_ARG, "not a version 1 checkpoint");
  if (get<uint32_t>(b, 12) != checkpoint_kind(I) || get<int32_t>(b, 16) != I->n || get<int32_t>(b, 20) != I->R)
    return fail(PAMC_ERR_INVALID_ARG, "checkpoint of another kind of instance, n or R");
  if (bytes < checkpoint_bytes(I)) return fail(PAMC_ERR_INVALID_ARG, "checkpoint truncated");
  int32_t ints[12];
  memcpy(ints, b + 72, sizeof ints);
  if (ints[4] < 0 || ints[4] > pamc::kHistCap || ints[0] < 1 || ints[5] < 0)
    return fail(PAMC_ERR_INVALID_ARG, "checkpoint controller out of range");
  const int32_t n = I->n, R = I->R;
  const int8_t* spins = (const int8_t*)b + PAMC_CHECKPOINT_HEADER_BYTES;
  std::vector<int32_t> fam(R);
  memcpy(fam.data(), b + PAMC_CHECKPOINT_HEADER_BYTES + (size_t)R * n, 4 * (size_t)R);
  const int8_t* best = spins + (size_t)R * n + 4 * (size_t)R;
  for (int32_t v = 0; v < n; ++v)
    if (I->potts_K ? (best[v] < 0 || best[v] >= I->potts_K) : (best[v] != 1 && best[v] != -1))
      return fail(PAMC_ERR_INVALID_ARG, "checkpoint configuration out of range");
  hipSetDevice(I->device);
  const uint64_t seed = get<uint64_t>(b, 24);
  if (seed != I->seed) {
    I->seed = seed;
    I->self_dirty = true;  // the descriptor carries the key
  }
  pamc_status st = load_population(I, spins, fam.data());
  if (st) return st;
  std::vector<int8_t> bi(I->np, I->potts_K ? 0 : 1);
  for (int32_t v = 0; v < n; ++v) bi[I->dense ? v : I->to_internal[v]] = best[v];
  HIP_TRY(hipMemcpy(I->best, bi.data(), I->np, hipMemcpyHostToDevice), "upload");
  pamc::RunState r;
  st = read_state(I, &r);
  if (st) return st;
  r.gs = get<uint32_t>(b, 32);
  r.g_rs = get<uint32_t>(b, 36);
  r.g_cl = get<uint32_t>(b, 40);
  r.mstar = get<int64_t>(b, 48);
  r.beta = get<double>(b, 56);
  r.delta = get<double>(b, 64);
  r.z = ints[0];
  r.cycle = ints[1];
  r.cooldown = ints[2];
  r.enable = ints[3] ? 1 : 0;
  r.hist_len = ints[4];
  r.steps_run = ints[5];
  r.step_reached = ints[6];
  r.n_cluster_moves = ints[7];
  r.n_reheats = ints[8];
  r.n_reversals = ints[9];
  r.n_restarts = ints[10];
  r.sum_lnq = get<double>(b, 120);
  for (int i = 0; i < pamc::kHistCap; ++i) r.hist[i] = get<int64_t>(b, 128 + 8 * (size_t)i);
  r.cur = 0;
  r.stopped = 0;
  r.active = 0;
  I->trace_ok = false;
  return write_state(I, r);
}

}  // extern "C"

namespace {


// The population buffers a sweep changes (spins, kept fields, energies)
// and their byte sizes.
std::vector<std::pair<void*, size_t>> sweep_state(pamc_instance* I, int cur) {
  std::vector<std::pair<void*, size_t>> v;
  v.push_back({I->pop.S[cur], sizeof(uint32_t) * (size_t)I->T * I->nq * 64});
  if (I->pop.H[cur]) v.push_back({I->pop.H[cur], sizeof(int32_t) * (size_t)I->T * I->np * 64});
  if (I->pop.HF[cur]) v.push_back({I->pop.HF[cur], sizeof(int32_t) * (size_t)pamc::kMaxHubs * I->R});
  v.push_back({I->pop.E[cur], sizeof(int64_t) * (size_t)I->R});
  return v;
}

}  // namespace

extern "C" {

pamc_status pamc_autotune(pamc_instance* I, double beta, int32_t sweeps, int32_t force, pamc_tune_result* out) {
  if (!I || !out) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  if (I->dense) return fail(PAMC_ERR_UNSUPPORTED, "the autotuner is for sparse instances");
  if (sweeps <= 0 || !std::isfinite(beta) || (I->potts_K && beta < 0))
    return fail(PAMC_ERR_INVALID_ARG, "bad tuning sweeps or beta");
  hipSetDevice(I->device);
  memset(out, 0, sizeof *out);
  const TuneShape initial{I->tile, I->tpw, I->qpw};
  const std::string key = tune_key(I);
  if (!force) {
    std::lock_guard<std::mutex> g(g_tune_mutex);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      apply_shape(I, it->second);
      out->tile_sweeps = I->tile;
      out->tiles_per_wave = I->tpw;
      out->quads_per_wave = I->qpw;
      out->cached = 1;
      return PAMC_OK;
    }
  }
  std::vector<TuneShape> cand;
  if (I->tmma_ok) cand.push_back({2, initial.tpw, initial.qpw});  // matrix-core fields
  for (int tile : {0, 1}) {
    if (tile && !I->tile_ok) continue;
    if (tile) {
      cand.push_back({1, initial.tpw, initial.qpw});  // the tile-resident sweep ignores the wave shape
      continue;
    }
    for (int tpw : {1, 2, 4}) {
      if (tpw > 1 && (!I->pull || I->potts_K || I->T % tpw)) continue;
      for (int qpw : {1, 2, 4}) cand.push_back({0, tpw, qpw});
    }
  }
  // scratch copy of the run state and of what sweeps change
  pamc::RunState st0;
  pamc_status st = read_state(I, &st0);
  if (st) return st;
  auto bufs = sweep_state(I, st0.cur);
  std::vector<void*> saved(bufs.size(), nullptr);
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < bufs.size() && e == hipSuccess; ++i) {
    e = dev_alloc(I, &saved[i], bufs[i].second);
    if (e == hipSuccess) e = hipMemcpyAsync(saved[i], bufs[i].first, bufs[i].second, hipMemcpyDeviceToDevice, I->stream);
  }
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (e == hipSuccess) e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  const bool prof = I->prof;
  I->prof = false;  // no library events inside the timed region
  auto restore = [&]() -> hipError_t {
    hipError_t r = hipSuccess;
    for (size_t i = 0; i < bufs.size() && r == hipSuccess; ++i)
      r = hipMemcpyAsync(bufs[i].first, saved[i], bufs[i].second, hipMemcpyDeviceToDevice, I->stream);
    if (r == hipSuccess) r = hipStreamSynchronize(I->stream);
    if (r == hipSuccess) r = hipMemcpy(I->st, &st0, sizeof st0, hipMemcpyHostToDevice);
    return r;
  };
  double best = 1e300, dflt = -1.0;
  TuneShape best_shape = initial;
  for (const TuneShape& c : cand) {
    if (e != hipSuccess) break;
    apply_shape(I, c);
    hipError_t be;
    pamc::Batch* b = self_batch(I, &be);
    if (!b) {
      e = be;
      break;
    }
    float ms = 1e30f;
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {  // the second of two timings
      e = hipEventRecord(ev[0], I->stream);
      if (e == hipSuccess) e = pamc::prim_sweep(*b, beta, sweeps);
      if (e == hipSuccess) e = hipEventRecord(ev[1], I->stream);
      if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
      if (e == hipSuccess) e = restore();
    }
    if (e != hipSuccess) break;
    const double per = ms / sweeps;
    if (c.tile == initial.tile && c.tpw == initial.tpw && c.qpw == initial.qpw) dflt = per;
    if (per < best) {
      best = per;
      best_shape = c;
    }
    out->candidates += 1;
  }
  I->prof = prof;
  for (hipEvent_t x : ev)
    if (x) hipEventDestroy(x);
  for (void* p : saved) dev_free(I, p);
  if (e != hipSuccess) {
    apply_shape(I, initial);
    return dev_fail(e, "autotune");
  }
  apply_shape(I, best_shape);
  {
    std::lock_guard<std::mutex> g(g_tune_mutex);
    g_tune_cache[key] = best_shape;
  }
  out->tile_sweeps = I->tile;
  out->tiles_per_wave = I->tpw;
  out->quads_per_wave = I->qpw;
  out->best_ms_per_sweep = best;
  out->default_ms_per_sweep = dflt;
  return PAMC_OK;
}

pamc_status pamc_pair_distance_hist(pamc_instance* I, int32_t nbins, int64_t* counts, double* mean) {
  if (!I || !counts) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  if (nbins < 1 || nbins > 4096) return fail(PAMC_ERR_INVALID_ARG, "nbins must lie in [1, 4096]");
  if (I->dense) return fail(PAMC_ERR_UNSUPPORTED, "pair distance on dense instances");
  if (I->potts_K) return fail(PAMC_ERR_UNSUPPORTED, "pair distance on Potts labels");
  hipSetDevice(I->device);
  int64_t* d = nullptr;
  HIP_TRY(dev_alloc(I, (void**)&d, sizeof(int64_t) * (nbins + 1)), "alloc");
  hipError_t e = pamc::launch_pair_hist(I, nbins, d, d + nbins);
  int64_t sum = 0;
  if (e == hipSuccess) e = hipStreamSynchronize(I->stream);
  if (e == hipSuccess) e = hipMemcpy(counts, d, sizeof(int64_t) * nbins, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&sum, d + nbins, sizeof(int64_t), hipMemcpyDeviceToHost);
  dev_free(I, d);
  if (e != hipSuccess) return dev_fail(e, "pair distance histogram");
  if (mean) *mean = I->R > 1 ? (double)sum / ((double)I->n * (0.5 * (double)I->R * (double)(I->R - 1))) : 0.0;
  return PAMC_OK;
}

pamc_status pamc_get_dh_trace(pamc_instance* I, int32_t capacity, double* dh, int32_t* steps) {
  if (!I || !dh) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  hipSetDevice(I->device);
  pamc::RunState r;
  pamc_status st = read_state(I, &r);
  if (st) return st;
  const int32_t k = (I->trace_ok && r.dh_every > 0) ? std::min(std::min(capacity, r.steps_run), I->tr_cap) : 0;
  if (steps) *steps = k;
  if (k > 0) HIP_TRY(hipMemcpy(dh, I->tr_dh, sizeof(double) * k, hipMemcpyDeviceToHost), "readback");
  return PAMC_OK;
}

pamc_status pamc_profile_enable(pamc_instance* I, int32_t on) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  hipSetDevice(I->device);
  HIP_TRY(hipStreamSynchronize(I->stream), "sync");
  I->prof = on != 0;
  I->ev_used = 0;
  I->prof_ms = 0.0;
  I->prof_launches = 0;
  I->prof_attempts = 0;
  HIP_TRY(hipMemset(I->flip_ctr, 0, sizeof(int64_t) * 256), "memset");
  I->self_dirty = true;  // the descriptor carries the flip counters iff profiling
  return PAMC_OK;
}

pamc_status pamc_profile_read(pamc_instance* I, double* ms, int64_t* launches, int64_t* attempts,
                              int64_t* flips) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  hipSetDevice(I->device);
  HIP_TRY(hipStreamSynchronize(I->stream), "sync");
  pamc_status st = resolve_events(I);
  if (st) return st;
  if (ms) *ms = I->prof_ms;
  if (launches) *launches = I->prof_launches;
  if (attempts) *attempts = I->prof_attempts;
  if (flips) {
    std::vector<int64_t> c(256);
    HIP_TRY(hipMemcpy(c.data(), I->flip_ctr, sizeof(int64_t) * 256, hipMemcpyDeviceToHost), "readback");
    int64_t t = 0;
    for (int64_t x : c) t += x;
    *flips = t;
  }
  return PAMC_OK;
}

pamc_status pamc_synchronize(pamc_instance* I) {
  if (!I) return fail(PAMC_ERR_INVALID_ARG, "NULL instance");
  hipSetDevice(I->device);
  HIP_TRY(hipStreamSynchronize(I->stream), "kernel execution");
  return PAMC_OK;
}


// ===========================================================================
// Continuous-batching server
// ===========================================================================
}  // extern "C"

// Host preparation of one request (validation, colouring, relabelled CSR),
// done on a worker thread while the device runs other requests.
struct ServerPrep {
  int32_t n = 0, objective = 0;
  std::vector<int32_t> rp, col, w;
  HostSparse h;
  pamc_status status = PAMC_OK;
  std::string error;
  double seconds = 0.0;
  std::mutex m;
  std::condition_variable cv;
  bool ready = false;
};

// Fixed pool of host threads for request preparation.
class ServerWorkers {
 public:
  void start(int n) {
    for (int i = 0; i < n; ++i) th_.emplace_back([this] { loop(); });
  }
  void push(std::function<void()> f) {
    {
      std::lock_guard<std::mutex> g(m_);
      q_.push_back(std::move(f));
    }
    cv_.notify_one();
  }
  ~ServerWorkers() {
    {
      std::lock_guard<std::mutex> g(m_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }

 private:
  void loop() {
    for (;;) {
      std::function<void()> f;
      {
        std::unique_lock<std::mutex> g(m_);
        cv_.wait(g, [this] { return stop_ || !q_.empty(); });
        if (q_.empty()) return;  // stopping
        f = std::move(q_.front());
        q_.pop_front();
      }
      f();
    }
  }
  std::vector<std::thread> th_;
  std::mutex m_;
  std::condition_variable cv_;
  std::deque<std::function<void()>> q_;
  bool stop_ = false;
};

struct pamc_server {
  struct Req {
    uint64_t ticket;
    std::shared_ptr<ServerPrep> prep;
    uint64_t seed;
    pamc_schedule sched;
    int64_t est;
    double t_submit;
  };
  struct Act {
    uint64_t ticket;
    pamc_instance* I;
    Schedule s;
    int32_t launched;
    int32_t fresh;  // controller not yet set up
    double t_submit, t_admit;
  };
  struct Fin {
    pamc_status status = PAMC_OK;
    std::string error;
    pamc_result res{};
    std::vector<int8_t> spins;
    double t_submit = 0, t_admit = 0, t_done = 0;
  };
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int64_t budget = 0, in_use = 0;
  int32_t max_slots = 0;
  pamc_config cfg{};
  uint64_t next_ticket = 1;
  std::deque<Req> queue;
  std::vector<Act> active;
  std::unordered_map<uint64_t, Fin> done;
  std::unordered_map<uint64_t, int> pending;  // ticket -> 0 queued, 1 active
  pamc::Batch batch;
  bool dirty = true;
  Schedule* d_sched = nullptr;
  int32_t* d_idx = nullptr;
  int32_t* d_status = nullptr;
  int32_t cap = 0;
  pamc_server_stats stats{};
  pamc_allocator al{};  // the caller's provider (copied), if any
  bool use_al = false;
  void* dmalloc(size_t bytes) {
    if (use_al) return al.alloc(al.ctx, bytes, (void*)stream);
    void* p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
  }
  void dmfree(void* p) {
    if (!p) return;
    if (use_al)
      al.free(al.ctx, p, (void*)stream);
    else
      hipFree(p);
  }
  std::unique_ptr<ServerWorkers> workers;  // declared last: joined first
};

namespace {

double now_seconds() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Device bytes a sparse instance of this graph will hold: the allocation
// plan of upload_sparse and prepare_run term by term (each allocation counts
// at least 16 bytes, as dalloc does), with the colour-class count bounded by
// the largest degree + 1.  It is an upper bound of the instance's
// device_bytes, so admission against it never overruns the budget.  The
// threshold table has 2X + 1 entries, X = max_v sum_j |w_vj| of this graph.
int64_t estimate_bytes(int32_t n, const int32_t* rp, const int32_t* w, const pamc_config& cfg,
                       const pamc_schedule& sc) {
  auto a = [](int64_t bytes) { return std::max<int64_t>(bytes, 16); };
  const int64_t R = cfg.replicas, np = (n + 3) & ~3, nnz = rp[n];
  int64_t maxdeg = 0, X = 0, gathered = 0;
  for (int32_t v = 0; v < n; ++v) {
    const int64_t deg = rp[v + 1] - rp[v];
    maxdeg = std::max(maxdeg, deg);
    gathered += (deg + 3) & ~3;
    int64_t ab = 0;
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) ab += std::llabs((long long)w[e]);
    X = std::max(X, ab);
  }
  std::vector<int32_t> hubs;
  bool pull = choose_fields(n, rp, cfg.flags, false, &hubs);
  const bool tile = !(cfg.flags & PAMC_FLAG_FIELDS_PUSH) && tile_fits(np / 4, X);
  const int64_t ncls = maxdeg + 1;
  int64_t b = a(4 * (int64_t)(n + 1)) + 2 * a(4 * (nnz + 16));                 // CSR
  if (pull || tile) b += a(4 * (int64_t)(n + 1)) + 2 * a(4 * std::max<int64_t>(gathered, 4));  // gathered CSR
  if (pull && !hubs.empty()) b += a(4 * np * pamc::kMaxHubs) + 2 * a(4 * pamc::kMaxHubs * R);  // hubs
  b += a(4 * (ncls + 1));                                                      // class_ptr
  b += 2 * (a(R * np) + (pull ? 0 : a(4 * R * np)) + a(8 * R) + a(4 * R));     // two populations
  b += a(np) + a(4 * (int64_t)n) + a((int64_t)sizeof(pamc::RunState));        // best, ids, run state
  b += a(4 * (2 * X + 1));                                                     // threshold table
  b += a(4 * std::max<int64_t>(64, sc.sweeps) * ncls);                        // class orders
  b += a(4 * R) + a(8 * 512);                                                  // parents, counters
  b += 4 * a(8 * (int64_t)std::max(sc.steps, 1)) + a(4 * (int64_t)std::max(sc.steps, 1)) +
       a(8 * (int64_t)std::max(sc.steps, 1));                                  // trace
  if (sc.augmented && sc.resample && sc.n_top > 0 && sc.mis_trials > 0) {    // cluster scratch
    const int64_t t = std::min<int64_t>(sc.n_top, R);
    b += a(4 * t) + a(t * sc.mis_trials * np) + a(4 * t * sc.mis_trials);
  }
  return b;
}

void server_prepare(ServerPrep& p, uint32_t flags, int32_t T) {
  const double t0 = now_seconds();
  pamc_status st = validate_csr(p.n, p.rp.data(), p.col.data(), p.w.data(), false);
  if (!st) {
    std::vector<int32_t> J(std::max(p.rp[p.n], 1));
    for (int32_t e = 0; e < p.rp[p.n]; ++e) J[e] = p.objective == PAMC_OBJ_MAXCUT ? -p.w[e] : p.w[e];
    st = prepare_sparse(p.h, p.n, p.rp.data(), p.col.data(), J, flags, T, false);
  }
  std::lock_guard<std::mutex> g(p.m);
  p.status = st;
  if (st) p.error = g_err;  // this worker's message
  p.rp = std::vector<int32_t>();
  p.col = std::vector<int32_t>();
  p.w = std::vector<int32_t>();
  p.seconds = now_seconds() - t0;
  p.ready = true;
  p.cv.notify_all();
}

// Admits queued requests in order while slots and memory allow.  A request
// whose host preparation is still running stops admission, unless nothing
// runs, in which case it is waited for.
pamc_status server_admit(pamc_server* S) {
  while (!S->queue.empty() && (int32_t)S->active.size() < S->max_slots &&
         S->in_use + S->queue.front().est <= S->budget) {
    pamc_server::Req& front = S->queue.front();
    ServerPrep& p = *front.prep;
    {
      std::unique_lock<std::mutex> g(p.m);
      if (!p.ready) {
        if (!S->active.empty()) break;
        p.cv.wait(g, [&p] { return p.ready; });
      }
    }
    pamc_server::Req q = std::move(front);
    S->queue.pop_front();
    const double t0 = now_seconds();
    S->stats.prep_seconds += p.seconds;
    pamc_status st = p.status;
    std::string err = p.error;
    pamc_instance* I = nullptr;
    Schedule s = to_sched(&q.sched);
    if (!st) {
      I = new (std::nothrow) pamc_instance();
      if (!I) st = fail(PAMC_ERR_OUT_OF_MEMORY, "host allocation");
      pamc_config c = S->cfg;
      c.seed = q.seed;
      c.stream = S->stream;
      if (!st) st = open_device(I, &c);
      if (!st) st = upload_sparse(I, p.h);
      if (!st) st = prepare_run(I, s);
      if (st) err = g_err;
    }
    q.prep.reset();
    if (st) {
      if (I) free_instance(I);
      S->pending.erase(q.ticket);
      pamc_server::Fin f;
      f.status = st;
      f.error = err;
      f.t_submit = f.t_admit = q.t_submit;
      f.t_done = now_seconds();
      S->done.emplace(q.ticket, std::move(f));
      S->stats.failed += 1;
      continue;
    }
    S->in_use += I->device_bytes;
    S->stats.peak_bytes = std::max(S->stats.peak_bytes, S->in_use);
    S->active.push_back({q.ticket, I, s, 0, 1, q.t_submit, now_seconds()});
    S->stats.peak_active = std::max<int64_t>(S->stats.peak_active, (int64_t)S->active.size());
    S->pending[q.ticket] = 1;
    S->dirty = true;
    S->stats.admit_seconds += now_seconds() - t0;
  }
  return PAMC_OK;
}

// Retires the finished requests.  Every finished request leaves the running
// set and has its memory freed even when reading its result fails (it then
// finishes with that error); the first such error is returned once the
// running set is consistent again.
pamc_status server_retire(pamc_server* S, const std::vector<int32_t>& status) {
  std::vector<pamc_server::Act> keep;
  keep.reserve(S->active.size());
  pamc_status first = PAMC_OK;
  std::string first_msg;
  for (size_t i = 0; i < S->active.size(); ++i) {
    pamc_server::Act& a = S->active[i];
    if (!(status[i] & 1)) {
      keep.push_back(a);
      continue;
    }
    pamc_server::Fin f;
    pamc::RunState r;
    pamc_status st = read_state(a.I, &r);
    if (!st) {
      fill_result(a.I, r, &f.res);
      f.spins.resize(a.I->n);
      st = pamc_best(a.I, nullptr, nullptr, f.spins.data());
    }
    if (st) {
      f.status = st;
      f.error = g_err;
      f.spins.clear();
      if (!first) {
        first = st;
        first_msg = g_err;
      }
      S->stats.failed += 1;
    } else {
      S->stats.finished += 1;
    }
    f.t_submit = a.t_submit;
    f.t_admit = a.t_admit;
    f.t_done = now_seconds();
    S->in_use -= a.I->device_bytes;
    free_instance(a.I);
    S->pending.erase(a.ticket);
    S->done.emplace(a.ticket, std::move(f));
    S->dirty = true;
  }
  S->active.swap(keep);
  if (first) return fail(first, first_msg);
  return PAMC_OK;
}

}  // namespace

extern "C" {

pamc_status pamc_server_create(int64_t hbm_budget_bytes, int32_t max_slots, const pamc_config* cfg,
                               pamc_server** out) {
  if (!out) return fail(PAMC_ERR_INVALID_ARG, "NULL out");
  *out = nullptr;
  pamc_status st = check_cfg(cfg);
  if (st) return st;
  if (hbm_budget_bytes <= 0 || max_slots <= 0) return fail(PAMC_ERR_INVALID_ARG, "budget and slots must be positive");
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count), "hipGetDeviceCount");
  if (cfg->device < 0 || cfg->device >= count) return fail(PAMC_ERR_INVALID_ARG, "bad device");
  pamc_server* S = new (std::nothrow) pamc_server();
  if (!S) return fail(PAMC_ERR_OUT_OF_MEMORY, "host allocation");
  S->device = cfg->device;
  S->budget = hbm_budget_bytes;
  S->max_slots = max_slots;
  S->cfg = *cfg;
  if (cfg->alloc) {
    if (!cfg->alloc->alloc || !cfg->alloc->free) {
      delete S;
      return fail(PAMC_ERR_INVALID_ARG, "allocator without functions");
    }
    S->al = *cfg->alloc;
    S->use_al = true;
    S->cfg.alloc = &S->al;  // requests copy it from here
    S->batch.al = &S->al;
  }
  int nthreads = 8;
  if (const char* e = getenv("PAMC_SERVER_THREADS")) nthreads = std::max(1, std::min(64, atoi(e)));
  S->workers.reset(new ServerWorkers());
  S->workers->start(nthreads);
  hipSetDevice(S->device);
  if (cfg->stream) {
    S->stream = (hipStream_t)cfg->stream;
  } else if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) == hipSuccess) {
    S->own_stream = true;
  } else {
    delete S;
    return fail(PAMC_ERR_DEVICE, "hipStreamCreate");
  }
  *out = S;
  return PAMC_OK;
}

pamc_status pamc_server_submit(pamc_server* S, int32_t n, const int32_t* row_ptr, const int32_t* col,
                               const int32_t* w, int32_t objective, uint64_t seed,
                               const pamc_schedule* sched, uint64_t* ticket) {
  if (!S || !sched || !ticket || !row_ptr) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  if (objective != PAMC_OBJ_MAXCUT && objective != PAMC_OBJ_ISING)
    return fail(PAMC_ERR_INVALID_ARG, "unknown objective");
  if (n <= 0) return fail(PAMC_ERR_INVALID_ARG, "n must be positive");
  if (row_ptr[0] != 0) return fail(PAMC_ERR_INVALID_ARG, "row_ptr[0] must be 0");
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return fail(PAMC_ERR_INVALID_ARG, "row_ptr must be non-decreasing");
  if (row_ptr[n] > 0 && (!col || !w)) return fail(PAMC_ERR_INVALID_ARG, "NULL CSR array");
  pamc_instance probe;  // schedule checks only look at the kind of instance
  pamc_status st = check_schedule(&probe, sched);
  if (st) return st;
  pamc_server::Req q;
  q.est = estimate_bytes(n, row_ptr, w ? w : row_ptr, S->cfg, *sched);
  if (q.est > S->budget) return fail(PAMC_ERR_OUT_OF_MEMORY, "request larger than the server's memory budget");
  auto prep = std::make_shared<ServerPrep>();
  prep->n = n;
  prep->objective = objective;
  prep->rp.assign(row_ptr, row_ptr + n + 1);
  prep->col.assign(col ? col : row_ptr, (col ? col : row_ptr) + row_ptr[n]);
  prep->w.assign(w ? w : row_ptr, (w ? w : row_ptr) + row_ptr[n]);
  q.prep = prep;
  q.ticket = S->next_ticket++;
  q.seed = seed;
  q.sched = *sched;
  q.t_submit = now_seconds();
  const uint32_t flags = S->cfg.flags;
  const int32_t T = S->cfg.replicas / 64;
  S->workers->push([prep, flags, T] { server_prepare(*prep, flags, T); });
  S->pending[q.ticket] = 0;
  *ticket = q.ticket;
  S->queue.push_back(std::move(q));
  S->stats.submitted += 1;
  return PAMC_OK;
}

pamc_status pamc_server_tick(pamc_server* S, int32_t max_steps, int32_t* n_active, int32_t* n_queued) {
  if (!S) return fail(PAMC_ERR_INVALID_ARG, "NULL server");
  hipSetDevice(S->device);
  pamc_status st = server_admit(S);
  if (st) return st;
  if (!S->active.empty()) {
    const int32_t na = (int32_t)S->active.size();
    if (S->dirty) {
      std::vector<pamc_instance*> v;
      std::vector<Schedule> sc;
      for (auto& a : S->active) {
        v.push_back(a.I);
        sc.push_back(a.s);
      }
      HIP_TRY(pamc::batch_build(S->batch, v, &sc), "batch descriptors");
      S->dirty = false;
      if (na > S->cap) {
        const int32_t cap = std::max(na, 2 * S->cap);
        S->dmfree(S->d_sched);
        S->dmfree(S->d_idx);
        S->dmfree(S->d_status);
        S->d_sched = nullptr;
        S->d_idx = S->d_status = nullptr;
        S->cap = 0;
        S->d_sched = (Schedule*)S->dmalloc(sizeof(Schedule) * cap);
        S->d_idx = (int32_t*)S->dmalloc(sizeof(int32_t) * cap);
        S->d_status = (int32_t*)S->dmalloc(sizeof(int32_t) * cap);
        if (!S->d_sched || !S->d_idx || !S->d_status) return fail(PAMC_ERR_OUT_OF_MEMORY, "server buffers");
        S->cap = cap;
      }
    }
    // controllers of the newly admitted requests (they sit at the end)
    std::vector<Schedule> ns;
    std::vector<int32_t> idx;
    for (int32_t i = 0; i < na; ++i)
      if (S->active[i].fresh) {
        ns.push_back(S->active[i].s);
        idx.push_back(i);
        S->active[i].fresh = 0;
      }
    if (!idx.empty()) {
      HIP_TRY(hipMemcpy(S->d_sched, ns.data(), sizeof(Schedule) * ns.size(), hipMemcpyHostToDevice), "upload");
      HIP_TRY(hipMemcpy(S->d_idx, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice), "upload");
      HIP_TRY(pamc::batch_anneal_setup(S->batch, S->d_sched, S->d_idx, (int32_t)idx.size()), "anneal setup");
    }
    // run until the first request can finish (or max_steps)
    int32_t k = INT32_MAX;
    for (auto& a : S->active) k = std::min(k, std::max(a.s.steps - a.launched, 1));
    if (max_steps > 0) k = std::min(k, max_steps);
    const double t_step = now_seconds();
    HIP_TRY(pamc::batch_run_steps(S->batch, k), "step");
    for (auto& a : S->active) a.launched += k;
    HIP_TRY(pamc::batch_status(S->batch, S->d_status), "status");
    std::vector<int32_t> status(na);
    HIP_TRY(hipMemcpyAsync(status.data(), S->d_status, sizeof(int32_t) * na, hipMemcpyDeviceToHost, S->stream), "readback");
    HIP_TRY(hipStreamSynchronize(S->stream), "batched steps");
    S->stats.step_seconds += now_seconds() - t_step;
    S->stats.ticks += 1;
    S->stats.steps += k;
    S->stats.request_steps += (int64_t)k * na;
    st = server_retire(S, status);
    if (st) return st;
  }
  if (n_active) *n_active = (int32_t)S->active.size();
  if (n_queued) *n_queued = (int32_t)S->queue.size();
  return PAMC_OK;
}

pamc_status pamc_server_drain(pamc_server* S) {
  if (!S) return fail(PAMC_ERR_INVALID_ARG, "NULL server");
  while (!S->active.empty() || !S->queue.empty()) {
    pamc_status st = pamc_server_tick(S, 0, nullptr, nullptr);
    if (st) return st;
  }
  return PAMC_OK;
}

pamc_status pamc_server_poll(pamc_server* S, uint64_t ticket, int32_t* done, pamc_result* out, int8_t* spins) {
  if (!S || !done) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  auto it = S->done.find(ticket);
  if (it == S->done.end()) {
    if (!S->pending.count(ticket)) return fail(PAMC_ERR_INVALID_ARG, "unknown ticket");
    *done = 0;
    return PAMC_OK;
  }
  *done = 1;
  if (it->second.status) return fail(it->second.status, it->second.error);
  if (out) *out = it->second.res;
  if (spins) memcpy(spins, it->second.spins.data(), it->second.spins.size());
  return PAMC_OK;
}

pamc_status pamc_server_get_stats(pamc_server* S, pamc_server_stats* out) {
  if (!S || !out) return fail(PAMC_ERR_INVALID_ARG, "NULL argument");
  *out = S->stats;
  out->in_use_bytes = S->in_use;
  out->active = (int64_t)S->active.size();
  out->queued = (int64_t)S->queue.size();
  return PAMC_OK;
}

pamc_status pamc_server_latency(pamc_server* S, uint64_t ticket, double* queued_seconds, double* total_seconds) {
  if (!S) return fail(PAMC_ERR_INVALID_ARG, "NULL server");
  auto it = S->done.find(ticket);
  if (it == S->done.end()) return fail(PAMC_ERR_STATE, "request not finished");
  if (queued_seconds) *queued_seconds = it->second.t_admit - it->second.t_submit;
  if (total_seconds) *total_seconds = it->second.t_done - it->second.t_submit;
  return PAMC_OK;
}

pamc_status pamc_server_forget(pamc_server* S, uint64_t ticket) {
  if (!S) return fail(PAMC_ERR_INVALID_ARG, "NULL server");
  if (!S->done.erase(ticket)) return fail(PAMC_ERR_STATE, "request not finished");
  return PAMC_OK;
}

void pamc_server_destroy(pamc_server* S) {
  if (!S) return;
  S->workers.reset();  // finishes the preparations in flight
  hipSetDevice(S->device);
  hipStreamSynchronize(S->stream);
  for (auto& a : S->active) free_instance(a.I);
  S->active.clear();
  S->batch.free_device();
  S->dmfree(S->d_sched);
  S->dmfree(S->d_idx);
  S->dmfree(S->d_status);
  if (S->own_stream) hipStreamDestroy(S->stream);
  delete S;
}

}  // extern "C"
