// instance.hpp -- host-side instance record and the launch entry points of
// the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pamc.h"
#include "pamc_device.hpp"

namespace pamc {

struct Batch;

// Population layout.  Replicas are grouped in tiles of 64 (one wavefront, one
// replica per lane).  Spins are quad-interleaved: the 32-bit word
// S[(t*nq + q)*64 + l] holds the spins of vertices 4q..4q+3 of replica
// 64t+l (byte k = vertex 4q+k), so a lane reads the four spins that share one
// Philox block with one load.  Fields are H[(t*np + v)*64 + l] (int32), so a
// neighbour update is one coalesced 64-lane row.
struct Pop {
  uint32_t* S[2] = {nullptr, nullptr};
  int32_t* H[2] = {nullptr, nullptr};
  int32_t* HF[2] = {nullptr, nullptr};  // hub fields [kMaxHubs][R] (gathered-field mode with hubs)
  int64_t* E[2] = {nullptr, nullptr};
  int32_t* fam[2] = {nullptr, nullptr};
};

struct GraphDev {
  int32_t* row_ptr = nullptr;
  int32_t* col = nullptr;
  int32_t* J = nullptr;
  // gathered-field copy of the CSR: rows padded to multiples of 4 entries
  // (vertex 0, coupling 0); columns as spin-word byte offsets 256 (v >> 2)
  // (+ (v & 3) in coupling modes 0 and 1); couplings as the sweep kernel's
  // coupling mode wants them (mode 2: int8 shifted to the neighbour's byte)
  int32_t* grow = nullptr;
  int32_t* gcol = nullptr;
  int32_t* gJ = nullptr;
  int32_t* class_ptr = nullptr;
  // small int8-coupling instances: J as 16-row x 64-column matrix-core A
  // fragments, [row tile][column step][lane][16 bytes]
  int8_t* Jt = nullptr;
  // hubs of the gathered-field mode: J between each vertex and each hub
  // [np][kMaxHubs] (0 where not adjacent)
  int32_t* hubJ = nullptr;
};

}  // namespace pamc

struct pamc_instance {
  pamc_allocator al{};  // device memory provider (use_al), else hipMalloc
  bool use_al = false;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int32_t n = 0, np = 0, nq = 0, R = 0, T = 0, rule = 0, dense = 0, ncls = 0;
  uint32_t flags = 0;
  uint64_t seed = 0;
  int64_t nnz = 0, W = 0, X = 0;
  int64_t device_bytes = 0;
  std::vector<int32_t> to_internal, to_input, class_ptr;
  int32_t max_class_quads = 0;
  int32_t pull = 0;       // 1: fields gathered at visit time (no field array)
  int32_t tile = 0;       // a step's sweeps of a replica tile in one work-group (small pull instances):
                          // 1 fields gathered from LDS, 2 fields from matrix-core products
  int32_t tmma_ok = 0;    // the matrix-core tile form possible (int8 couplings, n <= 1024)
  int32_t nks = 0;        // its 64-column steps
  int32_t tile_rows = 0;  // gathered-CSR entries of the largest colour class (staged in LDS by tile sweeps)
  int32_t tile_ok = 0;    // tile-resident sweeps possible
  int32_t nhub = 0;       // hubs (pull mode): vertices whose fields are kept incrementally
  int32_t hub_v[pamc::kMaxHubs] = {-1, -1};  // their internal ids
  int32_t dual = 0;       // both field forms kept: pull (with kept hub fields) and push
  int32_t hub_tpw = 1, hub_qpw = 1, push_tpw = 1, push_qpw = 1;  // wave shapes of the two forms
  int32_t tpw = 1;        // replica tiles per wavefront in the gathered-field sweep
  int32_t qpw = 1;        // vertex quads per wavefront in a sweep work-group (1, 2, 4)
  int32_t small_j = 0;    // 1: every |J| < 2^23 (24-bit multiplies are exact)
  int32_t jmode = 0;      // gathered-field coupling mode: 0 32-bit, 1 24-bit, 2 packed int8
  int32_t host_cur = 0;   // population buffer index last read back
  int32_t* H_scratch = nullptr;  // fields for snapshots in pull mode
  pamc::GraphDev g;
  pamc::Pop pop;
  int8_t* best = nullptr;  // [np] internal ids
  int32_t* to_internal_dev = nullptr;  // [n] caller id -> internal id
  pamc::RunState* st = nullptr;
  uint32_t* thr = nullptr;  // threshold table, 2X+1 entries
  int32_t potts_K = 0, potts_rule = 0;  // Potts labels (2 <= K <= 4), else 0
  double potts_gamma = 0.0;
  double* ptab = nullptr;   // Potts weight table, 2X+1 entries
  int32_t* order = nullptr; // [order_cap][ncls]
  int32_t order_cap = 0;
  // resampling scratch
  int32_t* rs_parent = nullptr;
  // cluster scratch
  int32_t* cl_targets = nullptr;
  uint8_t* cl_sel = nullptr;
  int32_t* cl_sizes = nullptr;
  int32_t cl_cap_top = 0, cl_cap_trials = 0;
  // per-step trace
  int64_t* tr_mstar = nullptr;
  double* tr_beta = nullptr;
  double* tr_lnq = nullptr;
  int32_t* tr_events = nullptr;
  uint64_t* tr_time = nullptr;
  double* tr_dh = nullptr;  // mean pair distance per step (-1: not measured)
  int32_t tr_cap = 0;
  bool trace_ok = false;  // the trace describes the last run (not one without a trace)
  double clock_hz = 100e6;
  // Max-3-Cut source graph (host and device)
  int32_t m3_n = 0;
  int32_t *m3_row_ptr = nullptr, *m3_col = nullptr, *m3_w = nullptr;
  int32_t* m3_labels = nullptr;
  int64_t* m3_cut = nullptr;
  // dense instance
  int8_t* Jd = nullptr;  // [np_pad][ld] row-major
  int64_t ldj = 0;
  int32_t dn_pad = 0;    // padded dimension of the dense matrix
  int32_t dense_j4 = 0;  // every dense coupling in [-8, 7] (four-bit dot products)
  int8_t* Sd = nullptr;  // [R][dn_pad] replica-major spins (dense)
  int8_t* Sd2 = nullptr; // resampling buffer
  int32_t* Gd = nullptr; // super-block field buffers [2][rows][R]
  int32_t* Cd = nullptr; // critical fields of a sweep [dn_pad / 4][R][4]
  int64_t* Ed[2] = {nullptr, nullptr};
  // profiling
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  double prof_ms = 0.0;
  int64_t prof_launches = 0, prof_attempts = 0;
  int64_t* flip_ctr = nullptr; // [256]
  // scratch for small readbacks
  void* pinned = nullptr;
  // the instance as a batch of one (rebuilt when a buffer it names changes)
  pamc::Batch* self = nullptr;
  bool self_dirty = true;
  void* d_sched = nullptr;  // device copy of the run's schedule
};

namespace pamc {

struct Schedule {
  double beta0, dbeta, reheat;
  int64_t target;
  int32_t steps, sweeps, z_rst, augmented, resample;
  int32_t win_short, win_long, max_ds, max_dl, tau, n_top, mis_trials;
  int32_t stop_at_target, literal_break;
  int32_t resume, dh_every;
};

// Per-instance descriptor read by every batched kernel: the device pointers
// and sizes of one instance (copied to the device once per batch).
struct Desc {
  const int32_t* row_ptr;
  const int32_t* col;
  const int32_t* J;
  const int32_t* grow;
  const int32_t* gcol;
  const int32_t* gJ;
  const int32_t* class_ptr;
  const int32_t* hubJ;    // [np][kMaxHubs] couplings to the hubs (gathered-field mode)
  int32_t *HF0, *HF1;     // hub fields [kMaxHubs][R], one per population buffer
  int32_t nhub, hub_v0, hub_v1;
  int32_t tile_rows;      // tile sweeps: gathered-CSR entries of the largest class
  const int8_t* Jt;       // matrix-core tile sweeps: J fragments
  int32_t nks;            // their 64-column steps
  int32_t* order;
  uint32_t* thr;
  uint32_t *S0, *S1;
  int32_t *H0, *H1;
  int64_t *E0, *E1;
  int32_t *F0, *F1;
  int8_t* best;
  RunState* st;
  int32_t* rs_parent;
  int32_t* cl_targets;
  uint8_t* cl_sel;
  int32_t* cl_sizes;
  int64_t* cl_flipped;
  int64_t* tr_mstar;
  double* tr_beta;
  double* tr_lnq;
  int32_t* tr_events;
  uint64_t* tr_time;
  double* tr_dh;
  int64_t* flip_ctr;      // null unless profiling
  const int8_t *D0, *D1;  // dense instances: replica-major spins [R][np]
  double* ptab;           // Potts labels: e^{-beta d}, d = 0..table_x
  double potts_gamma;     // softmax noise amplitude (Eq. 9)
  int32_t potts_K;        // 0: Ising spins; 2..4: Potts labels
  int32_t potts_rule;     // 0 softmax-perturbed argmax, 1 cascaded p-bits (K = 3)
  int64_t W, X;
  int32_t n, np, nq, R, T, ncls, rule, pull, dense, shuffle, tr_cap, order_cap, qpw;
  int32_t sweep_stride;   // incremental-field sweeps: a tile's work-groups take chunks c, c + stride, ...
  uint32_t k0, k1;
};

// A set of instances advanced by the same launches.  Grid kernels read a map
// of (instance << 32 | local block) words; one map per launch kind.
struct Batch {
  static constexpr int kGroups = 40;  // sweep kernel variants (37 spin, 3 Potts label)
  static int group_of(const pamc_instance* I);
  struct Launch {
    uint64_t* map = nullptr;
    int32_t grid = 0;
  };
  Launch init_spins, init_fields, thr, thr_dense, gather, cl_mis, cl_apply, dh;
  Launch sweep[kGroups];
  Launch tile[4];          // tile-resident sweeps: per coupling mode, then the matrix-core form
  int64_t tile_lds[4] = {0, 0, 0, 0};  // their dynamic LDS bytes
  int32_t tmma_waves = 16;             // waves per work-group of the matrix-core form (16 or 8)
  bool tmma_groups = false;            // matrix-core form: one work-group per 16-replica group
  Desc* d_desc = nullptr;
  int32_t n = 0;
  hipStream_t stream = nullptr;
  std::vector<pamc_instance*> I;
  int32_t max_ncls = 0, max_sweeps = 1, any_cluster = 0, any_dh = 0;
  int32_t group_ncls[kGroups] = {};  // most colour classes of an instance in each sweep group
  int64_t max_lds = 0;
  int32_t max_R = 0;  // most replicas of an instance (resampling LDS)
  hipGraphExec_t step_graph = nullptr;  // one captured beta step (batch_run_steps)
  int64_t graph_key = -1;
  bool graph_failed = false;
  // Arena mode (arena != nullptr): the descriptors, maps and per-run scratch
  // of batch_build are carved from [arena, arena + arena_cap) instead of
  // hipMalloc, never freed by the batch, and the batch launches eagerly
  // (no graph capture, no profiling events).  arena_need: bytes the last
  // build asked for (set also when it did not fit).
  char* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0, arena_need = 0;
  // outside arena mode: the provider of the batch's device memory (null:
  // hipMalloc); it must outlive the batch
  const pamc_allocator* al = nullptr;
  void free_device();
  Batch() = default;
  Batch(const Batch&) = delete;
  Batch& operator=(const Batch&) = delete;
  ~Batch() { free_device(); }
};

Desc make_desc(const pamc_instance* I);
// Device memory of the batch: hipMalloc, or in arena mode the next 256-byte
// aligned piece of the arena (hipErrorOutOfMemory once it is full).
hipError_t batch_alloc(Batch& b, void** p, size_t bytes);
// The library's fixed device scratch on the current device (a file-scope
// __device__ array; its address is looked up once per device).
hipError_t fixed_scratch(void** ptr, size_t* bytes);
// (Re)builds the batch's descriptors and maps; scheds (optional) give the
// sweeps per step and whether cluster moves can occur.  Synchronises the
// stream.  In arena mode scheds are required and each instance's class
// orders and cluster-move scratch come from the arena too, sized for its
// schedule (the instance's own buffers of those kinds are not used, and no
// per-step trace is recorded).
hipError_t batch_build(Batch& b, const std::vector<pamc_instance*>& insts, const std::vector<Schedule>* scheds);
hipError_t batch_init(Batch& b);                               // sparse instances
// Loads schedules and clears the controller of the listed instances (all if
// idx is null): instance idx[i] (or i) gets d_sched[i].
hipError_t batch_anneal_setup(Batch& b, const Schedule* d_sched, const int32_t* d_idx, int32_t count);
hipError_t batch_step(Batch& b);                               // one beta step of every live instance
hipError_t batch_run_steps(Batch& b, int32_t k);               // k steps, replaying a captured step graph
hipError_t batch_status(Batch& b, int32_t* d_out);             // (steps_run << 1) | stopped
hipError_t prim_sweep(Batch& b, double beta, int32_t nsweeps);
hipError_t prim_resample(Batch& b, double delta);
hipError_t prim_cluster(Batch& b, int32_t n_top, int32_t trials);
hipError_t prim_update_best(Batch& b);
hipError_t launch_fields(Batch& b, int32_t buf, int32_t* H);
// Fields and energies of population buffer 0 recomputed from its spins
// (spins uploaded by the host); the current buffer becomes 0.
hipError_t launch_load_population(Batch& b);
hipError_t launch_m3_decode(pamc_instance* I, const int8_t* spins_internal_dev);
hipError_t launch_pair_distance(pamc_instance* I, double* out_dev);
// histogram of min(d, n - d) over all replica pairs into nbins bins of
// [0, 1/2] (bin = floor(2 nbins min(d, n-d) / n), capped) plus its sum
hipError_t launch_refresh_fields(Batch& b);
hipError_t launch_pair_hist(pamc_instance* I, int32_t nbins, int64_t* hist_dev, int64_t* sum_dev);
int32_t cluster_max_n();
int32_t sweep_waves();  // wavefronts per sweep work-group
int32_t tile_max_quads();  // vertex quads a tile-resident sweep holds in LDS
int64_t tile_lds_bytes(int32_t nq, int32_t rows);  // its LDS: spins, table, a class's gathered rows
int32_t tmma_max_n();                               // largest padded n of the matrix-core tile form
int64_t tmma_lds_bytes(int32_t nks, int32_t rows);                // its LDS: replica-major spins, table
int64_t tile_lds_limit();
hipError_t prepare_kernel_lds();

// controller pieces (sparse.hip) shared with the dense path
hipError_t ctl_step_begin(Batch& b);
hipError_t ctl_resample_select(Batch& b);
hipError_t ctl_commit(Batch& b, int32_t in_run);
hipError_t ctl_thresholds(Batch& b);
hipError_t ctl_step_end(Batch& b, int32_t in_run);
hipError_t ctl_prim_set(Batch& b, int32_t kind, double value, int32_t nsweeps);
hipError_t ctl_advance(Batch& b, int32_t nsweeps);
hipError_t ctl_deactivate(Batch& b);
hipEvent_t ctl_event(pamc_instance* I);

// dense path launchers (dense.hip); b is the instance's batch of one
int32_t dense_superblock_rows();
int32_t dense_field_buffers();  // super-block field buffers (the next one is filled during a pass)
hipError_t launch_dense_fields(pamc_instance* I, int32_t* H_rmajor);
hipError_t launch_dense_generate(pamc_instance* I, uint64_t graph_seed);
hipError_t launch_init_dense(pamc_instance* I);
hipError_t launch_dense_load(pamc_instance* I);  // energies of uploaded spins (buffer 0)
hipError_t launch_dense_step(Batch& b, int32_t sweeps, int32_t resample);
hipError_t launch_dense_prim_sweep(Batch& b, double beta, int32_t nsweeps);
hipError_t launch_dense_prim_resample(Batch& b, double delta);
hipError_t launch_dense_prim_update_best(Batch& b);

}  // namespace pamc
