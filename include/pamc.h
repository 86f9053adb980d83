/*
 * pamc.h -- C ABI of the MI355X (gfx950) augmented Population Annealing Monte
 * Carlo library.
 *
 * Method: "Leveraging Population Dynamics to Steer Efficient Search in
 * Large-Scale Combinatorial Optimization" (Khan, Redding, Shukla).  A
 * population of R replicas of the Ising Hamiltonian H(s) = -sum_{i<j} J_ij
 * s_i s_j (Introduction) is swept with the single-spin rule of Eq. 4 on the
 * local fields of Eq. 3, resampled with the Boltzmann weights of Eqs. 1-2,
 * and steered by the stagnation-driven controller and the energy-preserving
 * cluster moves of Algorithm 1 (Sec. "Augmented PAMC").
 *
 * Conventions
 *  - Every call returns pamc_status; nothing throws or aborts across the ABI.
 *    On failure pamc_last_error() (thread-local) describes the cause.
 *  - Vertex ids at the ABI are the caller's ids (0..n-1).  Spin arrays are
 *    int8 in {-1,+1} (Potts instances: labels 0..K-1); populations are
 *    slot-major [R][n].
 *  - Input arrays are copied; the caller keeps ownership.  The instance owns
 *    its device memory (from cfg->alloc, else hipMalloc on cfg->device)
 *    until pamc_destroy_instance.
 *  - One host thread at a time per instance; distinct instances may be used
 *    concurrently.  Device work is enqueued on the instance's stream
 *    (cfg->stream, or a stream the library creates).  pamc_sweep,
 *    pamc_resample (log_q == NULL) and pamc_cluster_move (flipped == NULL)
 *    are asynchronous; pamc_best, pamc_get_state, pamc_anneal and
 *    pamc_synchronize wait for the stream.  An asynchronous device error is
 *    reported by the next waiting call as PAMC_ERR_DEVICE.
 *  - Randomness is a counter-based Philox4x32-10 stream keyed by cfg->seed.
 *    Each instance keeps monotone counters of sweeps, resamplings and cluster
 *    moves, so any sequence of calls is reproducible, and pamc_anneal is the
 *    sequence of primitive calls Algorithm 1 describes.
 */
#ifndef PAMC_H
#define PAMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pamc_instance pamc_instance;

typedef enum {
  PAMC_OK = 0,
  PAMC_ERR_INVALID_ARG = 1,   /* malformed instance, bad size, NULL pointer */
  PAMC_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed */
  PAMC_ERR_DEVICE = 3,        /* HIP runtime or kernel error */
  PAMC_ERR_STATE = 4,         /* call not valid for this instance */
  PAMC_ERR_UNSUPPORTED = 5    /* valid request outside the supported range */
} pamc_status;

/* Single-spin acceptance rule.  HEATBATH is Eq. 4 (flip probability
 * 1/(1+e^{2 beta s h})); METROPOLIS accepts with min(1, e^{-2 beta s h}). */
typedef enum { PAMC_RULE_HEATBATH = 0, PAMC_RULE_METROPOLIS = 1 } pamc_rule;

/* MAXCUT: weights w are edge weights, J = -w, cut = (W - H)/2 with
 * W = sum_{i<j} w_ij.  ISING: w are the couplings J themselves; the reported
 * "cut" is (sum_{i<j} (-J_ij) - H)/2. */
typedef enum { PAMC_OBJ_MAXCUT = 0, PAMC_OBJ_ISING = 1 } pamc_objective;

/* Where caller arrays live. */
typedef enum { PAMC_MEM_HOST = 0, PAMC_MEM_DEVICE = 1 } pamc_mem;

/* pamc_config.flags */
#define PAMC_FLAG_FIXED_CLASS_ORDER 1u /* do not shuffle colour classes per sweep */
/* Local-field storage of sparse instances.  PUSH keeps every field (Eq. 3)
 * in an int32 array updated by each flip; PULL keeps no field array and sums
 * the neighbours' spins when a spin is visited.  The integer fields, hence
 * every decision and the trajectory, are the same; the default picks PULL
 * when the average degree is at most 16 and no vertex has more than 64
 * neighbours.  PULL with at most two longer rows ("hubs") keeps the hubs'
 * fields.  With neither flag, a graph whose only long rows are one or two
 * hubs keeps both forms: pamc_anneal and pamc_anneal_batch sweep with PULL
 * while the scheduled beta is below 0.8 and with PUSH after, recomputing
 * the fields at the switch (pamc_get_info reports the form in use, PUSH
 * between runs). */
#define PAMC_FLAG_FIELDS_PUSH 2u
#define PAMC_FLAG_FIELDS_PULL 4u

/* Device memory provider.  alloc returns device memory of at least bytes
 * bytes for use on stream (NULL on failure, which the library reports as
 * PAMC_ERR_OUT_OF_MEMORY after returning everything it already holds);
 * free gives a block back after the library has waited for the stream.
 * ctx is passed through.  The Python binding can hand torch's caching
 * allocator here, so that the library's buffers come from torch's pool. */
typedef struct {
  void* ctx;
  void* (*alloc)(void* ctx, size_t bytes, void* stream);
  void (*free)(void* ctx, void* ptr, void* stream);
} pamc_allocator;

typedef struct {
  uint64_t seed;     /* Philox key */
  int32_t replicas;  /* R, a positive multiple of 64 */
  int32_t rule;      /* pamc_rule */
  int32_t device;    /* HIP device ordinal */
  void* stream;      /* hipStream_t or NULL (library-owned stream) */
  uint32_t flags;
  /* NULL: hipMalloc / hipFree.  Otherwise every device buffer the instance
   * (or server) holds comes from it; the struct is copied, its functions and
   * ctx must stay valid until the instance (server) is destroyed. */
  const pamc_allocator* alloc;
} pamc_config;

/* Sparse instance from a symmetric CSR graph (both directions stored, no
 * self loops, no duplicate or zero entries, symmetric weights).
 * row_ptr[n+1], col[nnz], w[nnz] with nnz = row_ptr[n], int32.  Vertices are
 * coloured by saturation degree (DSATUR: next the uncoloured vertex with the
 * most distinct neighbour colours, ties to the larger degree, then the lower
 * id; it takes the least colour free among its neighbours) and swept class
 * by class (spins of a class are mutually uncoupled, so this equals a
 * one-spin-at-a-time sweep in that order; Eq. 4, with the class sequence
 * reshuffled every sweep).  Fails with
 * PAMC_ERR_INVALID_ARG if 2*max_v sum_j |J_vj| does not fit int32. */
pamc_status pamc_create_instance_csr(int32_t n, const int32_t* row_ptr, const int32_t* col,
                                     const int32_t* w, pamc_mem where, int32_t objective,
                                     const pamc_config* cfg, pamc_instance** out);

/* Dense instance from an int8 coupling matrix J[n][ld] (row-major,
 * symmetric, zero diagonal, entries in [-127, 127]).  Spins are visited in
 * the fixed order 0..n-1; local fields are recomputed exactly with int8 x
 * int8 -> int32 matrix-core products (Scalability section: fully connected
 * instance).  Device memory: the padded matrix (n_pad^2 bytes, n_pad = n
 * rounded up to 64), two populations (2 n_pad R bytes), and per sweep each
 * visit's precomputed critical field (4 n_pad R bytes).  Instances whose
 * couplings all lie in [-7, 7] use four-bit products inside a block (same
 * results). */
pamc_status pamc_create_instance_dense_i8(int32_t n, const int8_t* J, int64_t ld, pamc_mem where,
                                          int32_t objective, const pamc_config* cfg,
                                          pamc_instance** out);

/* Dense +-1 instance generated on the device: J_ij = J_ji = +1 if the low bit
 * of word 0 of Philox(key = graph_seed, counter = (i, j, 0, 5)) is 1, else -1,
 * for i < j; zero diagonal; objective ISING.  Used for instances too large to
 * upload (n = 100,000 is 10^10 bytes). */
pamc_status pamc_create_instance_dense_random(int32_t n, uint64_t graph_seed,
                                              const pamc_config* cfg, pamc_instance** out);

/* Max-3-Cut through an Ising embedding (the paper notes that K > 2 needs
 * auxiliary spins and edges; Sec. "Max-3-Cut").  Vertex i of the input graph
 * (positive weights) becomes three one-hot spins (i,a) with ids 3i+a, plus
 * one ancilla with id 3n.  With weighted degree d_i and A_i = floor(d_i/3)+1:
 * J_{(i,a),anc} = -(2A_i + d_i), J_{(i,a),(i,b)} = -2A_i,
 * J_{(i,a),(j,a)} = -w_ij.  Ground states are one-hot and decode to maximum
 * 3-cuts (see pamc_max3cut_decode).  The sweep's colour classes come from
 * the input graph's colouring c (as for pamc_create_instance_csr, k colours):
 * spin (i,a) is in class (c(i) + a) mod max(k, 3), the ancilla in class
 * max(k, 3). */
pamc_status pamc_create_instance_max3cut(int32_t n, const int32_t* row_ptr, const int32_t* col,
                                         const int32_t* w, const pamc_config* cfg,
                                         pamc_instance** out);

/* Max-K-Cut with K-state Potts labels, the paper's own formulation (Sec.
 * "Max-3-Cut", Eqs. 6-9): one label per vertex, no auxiliary spins.  The
 * graph is given as for pamc_create_instance_csr (host memory, nonzero
 * symmetric weights w, J = -w).  Wherever the ABI returns spins
 * (pamc_best, pamc_get_state) it returns the labels, int8 in 0..K-1; fields
 * are returned as 0.  The energy is Eq. 6,
 * E = -sum_{i<j} J_ij (2 delta(s_i, s_j) - 1) = W - 2 cut, so the reported
 * cut is the weight of the edges whose ends carry different labels.
 * Visiting vertex i with the K-label field syn_k(i) = sum_j J_ij delta(s_j,
 * k) (Eq. 7) and omega_k = e^{beta (syn_k - max_m syn_m)} (binary64), the new
 * label is
 *   PAMC_POTTS_SOFTMAX: the k with the largest P_k - gamma U_k, P_k =
 *     omega_k / S, S = sum_m omega_m (Eqs. 8-9), U_k = u_k / 2^32, lowest k
 *     on ties; compared as omega_k - (gamma U_k) S;
 *   PAMC_POTTS_CASCADE (K = 3 only): the two binary p-bits of the cascaded
 *     sampler (Supplement): label 0 if tanh(Delta_1) = (omega_0 - s12) /
 *     (omega_0 + s12), s12 = omega_1 + omega_2, exceeds eta_1 = u_0/2^31 - 1,
 *     else label 1 if tanh(Delta_2) = (omega_1 - omega_2) / s12 exceeds
 *     eta_2 = u_1/2^31 - 1, else label 2 (exact Gibbs); each compared as
 *     numerator > eta * denominator.
 * u_0.. are the visit's W words (W = K, or 2 for the cascade): the four
 * vertices of a quad (id / 4, internal ids) share the W Philox blocks
 * (quad, sweep, replica, 6 | b << 8), b = 0..W-1, read as one sequence of 4W
 * words, vertex id % 4 = k taking words kW .. kW + W - 1.  This update
 * at beta leaves e^{-(beta/2) E} invariant, so resampling weighs replicas by
 * e^{-(Delta/2) (E - E_ref)} (ln Q likewise).  Cluster moves and the pair
 * distance are not defined for labels (PAMC_ERR_UNSUPPORTED; pamc_anneal
 * makes no moves, its controller still reheats).  cfg->rule is ignored.
 * Errors: K < 2, an unknown rule, the cascade with K != 3, gamma < 0 or not
 * finite: PAMC_ERR_INVALID_ARG; K > 4: PAMC_ERR_UNSUPPORTED. */
typedef enum { PAMC_POTTS_SOFTMAX = 0, PAMC_POTTS_CASCADE = 1 } pamc_potts_rule;
pamc_status pamc_create_instance_potts(int32_t n, const int32_t* row_ptr, const int32_t* col,
                                       const int32_t* w, int32_t K, int32_t potts_rule, double gamma,
                                       const pamc_config* cfg, pamc_instance** out);

void pamc_destroy_instance(pamc_instance* inst);

/* Re-draws the population from a new Philox key (Algorithm 1,
 * initialization: random spins, their fields and energies, M* = 0) and
 * resets the RNG counters, keeping the instance's graph and buffers. */
pamc_status pamc_reset_population(pamc_instance* inst, uint64_t seed);

/* Instance facts.  pull: fields gathered at visit time (1) or kept
 * incrementally (0).  The sweep kernel's shape for sparse instances:
 * tiles_per_wave replica tiles of 64 per wavefront, quads_per_wave vertex
 * quads per wavefront in a work-group, coupling_mode 0 (32-bit products),
 * 1 (24-bit) or 2 (int8 couplings with 4-way dot products); tile_sweeps 1:
 * small instance whose step's sweeps run in one launch, one work-group per
 * replica tile holding the tile's spins in LDS and gathering its neighbours;
 * tile_sweeps 2: one launch per step as well, with each colour class's
 * fields computed on the matrix cores as int8 products of 16 x 64 coupling
 * blocks with the spins (n <= 1024, int8 couplings), one work-group per
 * 16-replica group of a tile while the launch has at most 128 tiles, else
 * one per tile; hubs: vertices whose fields are kept while the others are
 * gathered. */
typedef struct {
  int32_t n, replicas, num_classes, dense, pull;
  int64_t nnz, W, X; /* X = max_v sum_j |J_vj| */
  int64_t device_bytes;
  int32_t tiles_per_wave, quads_per_wave, coupling_mode;
  int32_t potts_K; /* labels per vertex of a Potts instance, else 0 */
  int32_t tile_sweeps, hubs;
} pamc_info;
pamc_status pamc_get_info(const pamc_instance* inst, pamc_info* out);

/* Algorithm 1 inputs.  controller: augmented = 1 turns on the adaptive
 * temperature rule and cluster moves (Sec. "Augmented PAMC"); with 0 the run
 * is conventional PAMC on beta0, beta0+dbeta, ...; resample = 0 gives
 * independent chains (simulated annealing).  z_rst <= 0 never restarts. */
typedef struct {
  double beta0, dbeta;
  int32_t steps, sweeps;
  int32_t z_rst;
  int32_t augmented;
  int32_t resample;
  int32_t win_short, win_long, max_distinct_short, max_distinct_long; /* 25, 40, 3, 5 */
  double reheat;                                                      /* 0.8 */
  int32_t tau, n_top, mis_trials;
  int64_t target;         /* MC* */
  int32_t stop_at_target; /* 1: loop "while M* < MC*" */
  int32_t literal_break;  /* 1: end the run where Algorithm 1 prints "break" */
  /* 1: continue the run the instance holds (restored by pamc_set_checkpoint,
   * or left by a pamc_anneal that ended at its step count) instead of
   * starting Algorithm 1 afresh: the controller, M*, its configuration, the
   * history, the counts and the steps run are kept, and the run goes on
   * until the steps run reach steps (or M* reaches the target).  The trace
   * holds this call's steps at their absolute step indices. */
  int32_t resume;
  /* > 0: record the population's mean normalised pair distance d_H (see
   * pamc_pair_distance) every dh_every steps, after the step's sweeps
   * (pamc_get_dh_trace).  Each sample compares all R(R-1)/2 pairs:
   * O(R^2 n / 32) word reads. */
  int32_t dh_every;
} pamc_schedule;

typedef struct {
  int64_t best_cut, best_energy;
  int32_t steps_run, step_reached; /* first step with M* >= target, or -1 */
  double sum_lnq;                  /* sum of ln Q over resamplings */
  int32_t n_cluster_moves, n_reheats, n_reversals, n_restarts;
  double seconds_total, seconds_to_target; /* device clock; -1 if never */
} pamc_result;

/* Runs Algorithm 1 from the instance's current population and counters and
 * waits for it.  The controller runs on the device; the host only enqueues. */
pamc_status pamc_anneal(pamc_instance* inst, const pamc_schedule* sched, pamc_result* out);

/* nsweeps Monte Carlo sweeps at inverse temperature beta (Eqs. 3-4). */
pamc_status pamc_sweep(pamc_instance* inst, double beta, int32_t nsweeps);

/* Boltzmann resampling with increment delta (Eqs. 1-2): R multinomial draws
 * of parents with probability proportional to e^{-delta E_j}; children are
 * ordered by parent.  log_q (may be NULL) receives ln Q of Eq. 2. */
pamc_status pamc_resample(pamc_instance* inst, double delta, double* log_q);

/* Non-local cluster move (Algorithm 1; Sec. "Augmented PAMC") on the n_top
 * lowest-energy replicas, mis_trials randomized greedy independent sets of
 * iso-sites each, the largest flipped.  flipped (may be NULL) receives the
 * total number of spins flipped.  Requires n <= 26,000 (the independent-set
 * search is held in local data share). */
pamc_status pamc_cluster_move(pamc_instance* inst, int32_t n_top, int32_t mis_trials,
                              int32_t* flipped);

/* M* <- max(M*, max_r cut_r) with its configuration (Algorithm 1). */
pamc_status pamc_update_best(pamc_instance* inst);

/* Best cut M*, its energy and spins (n, may be NULL).  Waits. */
pamc_status pamc_best(pamc_instance* inst, int64_t* cut, int64_t* energy, int8_t* spins);

/* Population snapshot (each may be NULL): spins [R][n], fields [R][n],
 * energies [R], family (ancestor slot at creation) [R].  Waits. */
pamc_status pamc_get_state(pamc_instance* inst, int8_t* spins, int32_t* fields,
                           int64_t* energies, int32_t* family);

/* Per-step trace of the last pamc_anneal (arrays of length capacity, each may
 * be NULL): M* after the step, beta used for the sweeps, ln Q, event bits
 * (1 resampled, 2 cluster move, 4 strong reheat, 8 reversal, 16 restart) and
 * seconds since the start of the run.  *steps receives the number recorded. */
pamc_status pamc_get_trace(pamc_instance* inst, int32_t capacity, int64_t* mstar, double* beta,
                           double* lnq, int32_t* events, double* seconds, int32_t* steps);

/* Max-3-Cut decode (instances from pamc_create_instance_max3cut): undo the
 * global-flip gauge with the ancilla; the label of vertex i is the a with
 * spin (i,a) = +1, the lowest such a if several, 0 if none.  spins: the
 * embedded configuration (3n+1, caller ids) or NULL for the best one.
 * labels: n entries (may be NULL).  cut3: the 3-cut of the labelling. */
pamc_status pamc_max3cut_decode(pamc_instance* inst, const int8_t* spins, int32_t* labels,
                                int64_t* cut3);

/* Mean normalised pairwise Hamming distance d_H = min(d, 1-d) over all
 * replica pairs (Supplement, Hamming distance).  Waits. */
pamc_status pamc_pair_distance(pamc_instance* inst, double* mean);

/* The distribution of d_H over all R(R-1)/2 replica pairs (the diversity
 * histograms of the Supplement's Hamming-distance method): counts[nbins]
 * receives the number of pairs with floor(2 nbins min(d, n-d) / n) = k
 * (the last bin also takes d_H = 1/2), i.e. bins of width 1/(2 nbins) on
 * [0, 1/2]; mean (may be NULL) the mean d_H.  1 <= nbins <= 4096; Ising
 * spins only.  Waits. */
pamc_status pamc_pair_distance_hist(pamc_instance* inst, int32_t nbins, int64_t* counts, double* mean);

/* Per-step mean d_H of the last pamc_anneal run with dh_every > 0: dh
 * (capacity entries) receives, per step, the mean over all pairs after the
 * step's sweeps, or -1 on steps not sampled; *steps the number recorded. */
pamc_status pamc_get_dh_trace(pamc_instance* inst, int32_t capacity, double* dh, int32_t* steps);

/* ---------------------------------------------------------------------------
 * Checkpoint and resume.  A run of Algorithm 1 is a function of the
 * population, the controller variables and the stream counters, so a run
 * stopped after any beta step continues bit for bit from them, on the same
 * instance or on a new one built from the same graph.
 * ------------------------------------------------------------------------- */

/* Replaces the population: spins [R][n] in caller ids (labels 0..K-1 for
 * Potts instances), lineage ids [R] (NULL: 0..R-1) and the stream counters
 * {sweeps, resamplings, cluster moves} (NULL: unchanged).  Local fields and
 * energies are recomputed from the spins (Eq. 3 and H = -1/2 sum s h; Eq. 6
 * for labels).  M*, its configuration and the controller are not changed.
 * A spin outside {-1, +1} (a label outside 0..K-1): PAMC_ERR_INVALID_ARG,
 * nothing changed.  Waits. */
pamc_status pamc_set_state(pamc_instance* inst, const int8_t* spins, const int32_t* family,
                           const uint32_t* counters);

/* Checkpoint byte format, version 1: little-endian, fields packed in this
 * order at these offsets.
 *     0  char[8]  "PAMCCKP1"
 *     8  uint32   version = 1
 *    12  uint32   kind: 0 Ising spins on a CSR graph (also Max-3-Cut
 *                 embeddings), 1 Potts labels, 2 dense couplings
 *    16  int32    n              20  int32  R
 *    24  uint64   seed (the Philox key)
 *    32  uint32   sweeps, resamplings, cluster moves made (stream counters),
 *                 then a zero word
 *    48  int64    M*
 *    56  double   beta           64  double Delta   (controller, Algorithm 1)
 *    72  int32    z, cycle, cooldown, cluster move armed (0/1), history
 *                 length, steps run, first step with M* >= target (-1:
 *                 never), cluster moves, reheats, reversals, restarts, 0
 *   120  double   sum of ln Q
 *   128  int64    history[64]: the last (history length) values of M*,
 *                 oldest first, then zeros
 *   640  int8     spins [R][n], caller ids (labels for Potts instances)
 *   640 + R n         int32  lineage [R]
 *   640 + R n + 4 R   int8   configuration of M* [n], caller ids
 * Size: 640 + R n + 4 R + n bytes. */
#define PAMC_CHECKPOINT_HEADER_BYTES 640
pamc_status pamc_checkpoint_size(const pamc_instance* inst, int64_t* bytes);
/* Writes the instance's checkpoint into buf (bytes >= the size).  Waits. */
pamc_status pamc_get_checkpoint(pamc_instance* inst, void* buf, int64_t bytes);
/* Loads a checkpoint into an instance of the same kind, n and R (its graph
 * must be the one the checkpoint was taken on): the seed, the population
 * (fields and energies recomputed), the lineage, M* and its configuration,
 * the controller and the stream counters.  pamc_anneal with resume = 1 then
 * continues the run.  A malformed or mismatched buffer:
 * PAMC_ERR_INVALID_ARG, nothing changed.  Waits. */
pamc_status pamc_set_checkpoint(pamc_instance* inst, const void* buf, int64_t bytes);

/* Kernel timing: when enabled, the library records HIP events on the
 * instance stream around the sweep kernels: for sparse couplings one pair
 * around each step's consecutive sweep launches (so the mean launch time
 * includes the launch boundaries), for dense couplings one pair around each
 * launch of the field product.  Enabling it also turns on the flip counters
 * and turns off graph replay of beta steps. */
pamc_status pamc_profile_enable(pamc_instance* inst, int32_t on);
/* Sum of event-measured sweep-kernel time (ms), number of launches, and the
 * attempts (replica x vertex visits) they made since enabling.  Waits. */
pamc_status pamc_profile_read(pamc_instance* inst, double* ms, int64_t* launches,
                              int64_t* attempts, int64_t* flips);

pamc_status pamc_synchronize(pamc_instance* inst);

/* Autotuner of the sweep kernels' shape.  Candidates: tile-resident sweeps
 * on or off (where the instance allows them), 1, 2 or 4 replica tiles per
 * wavefront (gathered fields), 1, 2 or 4 vertex quads per wavefront.  Each
 * is timed on `sweeps` sweeps at `beta` run on the instance's own
 * population, which is saved first and restored, with the stream counters,
 * after every candidate, so tuning never changes a trajectory.  The fastest
 * shape is kept and remembered per instance shape (n, edges, replicas,
 * colour classes, field mode, coupling mode) for this process: a later call
 * for an instance of the same shape takes it without timing unless force is
 * set.  Sparse instances only; waits. */
typedef struct {
  int32_t tile_sweeps, tiles_per_wave, quads_per_wave; /* the chosen shape */
  int32_t candidates;                                   /* shapes timed (0 if taken from the cache) */
  int32_t cached;                                       /* 1: the shape came from the cache */
  double best_ms_per_sweep, default_ms_per_sweep;       /* chosen and creation-time shapes */
} pamc_tune_result;
pamc_status pamc_autotune(pamc_instance* inst, double beta, int32_t sweeps, int32_t force,
                          pamc_tune_result* out);

/* ---------------------------------------------------------------------------
 * Batched and served runs.  Many independent runs share every kernel launch:
 * each kernel reads a per-instance descriptor and a block-to-instance map,
 * so instances of different sizes, schedules and seeds advance together.
 * A run's result does not depend on what it is batched with: the cut, the
 * trace and the final population are bit-identical to pamc_anneal on the
 * same instance.
 * ------------------------------------------------------------------------- */

/* Runs Algorithm 1 on count sparse instances of one device at once, each
 * with its own schedule, and waits.  Instances must be distinct; each
 * instance's queued work is finished first, and the batch runs on the first
 * instance's stream.  out: count results. */
pamc_status pamc_anneal_batch(pamc_instance* const* insts, const pamc_schedule* scheds, int32_t count,
                              pamc_result* out);

/* The same batched run for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It calls no hipMalloc, hipFree or other allocating routine:
 * the batch's descriptors, launch maps and schedules, each instance's class
 * orders and its cluster-move scratch (n_top x mis_trials x n bytes) are
 * carved from a fixed 16 MiB device array that every GPU the library runs
 * on holds until the process ends.  A batch that needs more returns
 * PAMC_ERR_UNSUPPORTED (pamc_last_error() states the bytes needed) before
 * any device work.  Results and final populations equal pamc_anneal_batch's
 * bit for bit; no per-step trace is recorded (pamc_get_trace then reports
 * 0 steps), beta steps are launched one by one (no graph), and profiling is
 * off.  All calls on one GPU share the array, so calls that overlap on one
 * GPU (other threads) race; a call returns only after its device work is
 * done. */
pamc_status pamc_anneal_batch_noalloc(pamc_instance* const* insts, const pamc_schedule* scheds,
                                      int32_t count, pamc_result* out);

typedef struct pamc_server pamc_server;

/* Continuous-batching server on cfg->device: requests (a graph, a seed and a
 * schedule) wait in a FIFO queue; a request is admitted when fewer than
 * max_slots run and its device memory fits in hbm_budget_bytes next to the
 * running ones.  Each tick advances every running request by the same number
 * of beta steps in shared launches, then retires the finished ones and frees
 * their memory.  cfg gives replicas, rule, flags and stream (the seed comes
 * with each request).  One thread at a time per server. */
pamc_status pamc_server_create(int64_t hbm_budget_bytes, int32_t max_slots, const pamc_config* cfg,
                               pamc_server** out);

/* Queues a Max-Cut (objective PAMC_OBJ_MAXCUT) or Ising request on a host CSR
 * graph (copied now; the caller keeps its arrays).  The graph is validated,
 * coloured and relabelled on one of the server's host threads (8, or
 * PAMC_SERVER_THREADS) while the device runs other requests; a request that
 * fails there finishes with that error (pamc_server_poll returns it).
 * Returns PAMC_ERR_OUT_OF_MEMORY if the request alone exceeds the budget.
 * *ticket identifies the request. */
pamc_status pamc_server_submit(pamc_server* srv, int32_t n, const int32_t* row_ptr, const int32_t* col,
                               const int32_t* w, int32_t objective, uint64_t seed,
                               const pamc_schedule* sched, uint64_t* ticket);

/* Admits what fits (in submission order; a request still being prepared
 * holds back the ones after it, and is waited for only when nothing runs),
 * advances the running requests by min(max_steps, steps left of the nearest
 * one) beta steps (max_steps <= 0: no cap), waits, and retires finished
 * requests.  n_active / n_queued (may be NULL) receive the counts after the
 * tick. */
pamc_status pamc_server_tick(pamc_server* srv, int32_t max_steps, int32_t* n_active, int32_t* n_queued);

/* Ticks until nothing is queued or running. */
pamc_status pamc_server_drain(pamc_server* srv);

/* *done = 1 and the result (and best spins, n entries, may be NULL) once
 * the request has finished, else *done = 0.  A request that failed (invalid
 * graph, out of memory) has *done = 1 and its error as the return value. */
pamc_status pamc_server_poll(pamc_server* srv, uint64_t ticket, int32_t* done, pamc_result* out,
                             int8_t* spins);

/* Host wall-clock seconds from submission to admission and to retirement. */
pamc_status pamc_server_latency(pamc_server* srv, uint64_t ticket, double* queued_seconds,
                                double* total_seconds);

/* Server counters: requests submitted / finished / failed, ticks, beta
 * steps (per tick, and summed over running requests), host seconds spent
 * preparing requests on the worker threads (colouring, relabelling),
 * admitting them (device buffers, upload, initial population) and
 * stepping, peak running requests and device bytes, and the current state. */
typedef struct {
  int64_t submitted, finished, failed, ticks, steps, request_steps;
  double prep_seconds, admit_seconds, step_seconds;
  int64_t peak_active, peak_bytes, in_use_bytes, active, queued;
} pamc_server_stats;
pamc_status pamc_server_get_stats(pamc_server* srv, pamc_server_stats* out);

/* Drops a finished request's stored result. */
pamc_status pamc_server_forget(pamc_server* srv, uint64_t ticket);

/* Frees the server and every request still queued or running. */
void pamc_server_destroy(pamc_server* srv);

const char* pamc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PAMC_H */
