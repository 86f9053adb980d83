/*
 * pamc_oracle.h -- plain, slow, single-threaded CPU oracle for augmented
 * Population Annealing Monte Carlo (PAMC).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists so that the GPU library can be
 * checked against an obviously-correct implementation of the same method.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or constant generator with
 * the GPU library: every routine here (Philox, the exponential, colouring,
 * sweep, resampling, cluster move, controller, dense path, Max-3-Cut
 * embedding) is written independently from the paper and from the published
 * definitions it names.
 *
 * Paper: "Leveraging Population Dynamics to Steer Efficient Search in
 * Large-Scale Combinatorial Optimization" (Khan, Redding, Shukla).
 *
 * Conventions fixed by the paper or, where it is silent, by the readings
 * listed in the design notes:
 *   - H(s) = -sum_{i<j} J_ij s_i s_j  (Introduction; each pair once).
 *   - Max-Cut: J = -w, cut = (W - H)/2 with W = sum_{i<j} w_ij.
 *   - local field h_k = sum_j J_kj s_j (Eq. 3); flipping s_k changes H by
 *     2 s_k h_k.
 *   - heat-bath update of Eq. 4 flips with probability 1/(1+e^{2 beta s h}).
 *   - resampling weights of Eqs. 1-2, multinomial, population size kept at R.
 *   - control loop of Algorithm 1 with the adaptive rule of Sec. "Augmented
 *     PAMC" (windows 25/40, <=3 distinct / >5 distinct, factor 0.8).
 */
#ifndef PAMC_ORACLE_H
#define PAMC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* RNG stream tags (fourth Philox counter word). */
enum { ORC_TAG_INIT = 0, ORC_TAG_SWEEP = 1, ORC_TAG_RS = 2, ORC_TAG_CL = 3,
       ORC_TAG_ORDER = 4, ORC_TAG_DENSE = 5, ORC_TAG_POTTS = 6 };

/* Potts label updates (Sec. "Max-3-Cut"): softmax probabilities perturbed by
 * gamma-scaled uniform noise, then argmax (Eqs. 8-9); or the cascade of two
 * binary p-bits for K = 3 (Supplement, cascaded sampler). */
enum { ORC_POTTS_SOFTMAX = 0, ORC_POTTS_CASCADE = 1 };

enum { ORC_RULE_HEATBATH = 0, ORC_RULE_METROPOLIS = 1 };
enum { ORC_OBJ_MAXCUT = 0, ORC_OBJ_ISING = 1 };

typedef struct orc orc;

typedef struct {
  double beta0, dbeta;
  int32_t steps, sweeps;
  int32_t z_rst;          /* restart period (Algorithm 1); <=0 means never */
  int32_t augmented;      /* 1: adaptive control + cluster moves */
  int32_t resample;       /* 1: PAMC, 0: independent chains (SA) */
  int32_t win_short, win_long, max_distinct_short, max_distinct_long;
  double reheat;          /* 0.8 */
  int32_t tau, n_top, mis_trials;
  int64_t target;         /* target cut MC* */
  int32_t stop_at_target; /* 1: loop "while M* < MC*" */
  int32_t literal_break;  /* 1: end the run where Algorithm 1 prints "break" */
  int32_t resume;         /* 1: continue the run the instance holds (controller,
                             M*, history, counts and steps run kept) */
  int32_t dh_every;       /* > 0: record the mean pair distance every dh_every steps */
} orc_schedule;

typedef struct {
  int64_t best_cut, best_energy;
  int32_t steps_run, step_reached;
  double sum_lnq;
  int32_t n_cluster_moves, n_reheats, n_reversals, n_restarts;
} orc_result;

/* Optional per-step trace (arrays of length steps, may be NULL). */
typedef struct {
  int64_t* mstar;     /* M* after the step */
  double* beta;       /* beta used for the sweeps of the step */
  double* lnq;        /* ln Q of the step's resampling (0 if none) */
  int32_t* events;    /* bit0 resampled, bit1 cluster move, bit2 strong, bit3 mild, bit4 restart */
  double* dh;         /* mean pair distance after the step's sweeps (-1 if not sampled) */
} orc_trace;

/* ---- primitives exposed for pins ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_pexp(double x);
uint32_t orc_threshold(double beta, int32_t rule, int64_t x);
/* Saturation-degree (DSATUR) colouring: the uncoloured vertex with the most
 * distinct neighbour colours next (ties: larger degree, then lower id), the
 * least colour free among its neighbours; colour[v] out; returns the number
 * of classes. */
int32_t orc_colour(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* colour);
/* The Max-3-Cut embedding's colouring (3n + 1 spins, spin 3i + a, ancilla
 * 3n) from the base graph's colouring c (orc_colour) with k colours: (c(i) + a)
 * mod max(k, 3), the ancilla max(k, 3).  Returns the class count. */
int32_t orc_max3cut_colour(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* colour);
/* dense +-1 couplings from a counter-based hash of (seed, i, j) */
void orc_dense_random(int32_t n, uint64_t seed, int8_t* J);

/* ---- instances ---- */
/* Sparse symmetric CSR (both directions stored, no self loops, no
 * duplicates, no zero weights).  Returns NULL on invalid input (err filled). */
orc* orc_create_sparse(int32_t n, const int32_t* row_ptr, const int32_t* col,
                       const int32_t* w, int32_t objective, int32_t replicas,
                       uint64_t seed, int32_t rule, int32_t shuffle_classes,
                       char* err, int32_t errlen);
/* Dense int8 couplings J (n*n, row-major, symmetric, zero diagonal);
 * sequential vertex order 0..n-1. */
orc* orc_create_dense(int32_t n, const int8_t* J, int32_t objective,
                      int32_t replicas, uint64_t seed, int32_t rule,
                      char* err, int32_t errlen);
/* Max-3-Cut through a one-hot Ising embedding with one ancilla spin. */
orc* orc_create_max3cut(int32_t n, const int32_t* row_ptr, const int32_t* col,
                        const int32_t* w, int32_t replicas, uint64_t seed,
                        int32_t rule, int32_t shuffle_classes,
                        char* err, int32_t errlen);
/* Max-K-Cut with K-state Potts labels (Sec. "Max-3-Cut", Eqs. 6-9; the
 * cascaded K = 3 sampler of the Supplement), 2 <= K <= 4.  J = -w; the
 * energy is Eq. 6, E = -sum_{edges} J_ij (2 delta(s_i, s_j) - 1), so the
 * K-cut is (W - E)/2.  A label update draws P(k) from Eq. 8 with the
 * K-label field syn_k(i) = sum_j J_ij delta(s_j, k) at the step's beta. */
orc* orc_create_potts(int32_t n, const int32_t* row_ptr, const int32_t* col,
                      const int32_t* w, int32_t K, int32_t replicas, uint64_t seed,
                      int32_t potts_rule, double gamma, int32_t shuffle_classes,
                      char* err, int32_t errlen);
/* Eq. 6 energy of replica r recomputed from its labels. */
int64_t orc_potts_energy(const orc* o, int32_t r);
/* The label a Potts update picks for K-label field syn (length K) and four
 * uniform words u, at inverse temperature beta. */
int32_t orc_potts_choose(int32_t K, int32_t potts_rule, double gamma, double beta,
                         const int64_t* syn, const uint32_t* u);
void orc_destroy(orc* o);

/* Instance facts. */
int32_t orc_n(const orc* o);
int32_t orc_replicas(const orc* o);
int32_t orc_num_classes(const orc* o);
int64_t orc_W(const orc* o);
int64_t orc_X(const orc* o);
/* internal id of each input vertex (the sweep order key) */
void orc_internal_ids(const orc* o, int32_t* to_internal);
void orc_class_ptr(const orc* o, int32_t* class_ptr);

/* ---- steps of the method ---- */
void orc_sweep(orc* o, double beta, int32_t nsweeps);
double orc_resample(orc* o, double delta, int32_t* parents /* R, may be NULL */);
int32_t orc_cluster(orc* o, int32_t n_top, int32_t mis_trials,
                    int32_t* chosen_sizes /* n_top, may be NULL */);
int64_t orc_update_best(orc* o);
void orc_best(const orc* o, int64_t* cut, int64_t* energy, int8_t* spins);
void orc_get_state(const orc* o, int8_t* spins, int32_t* fields, int64_t* energies,
                   int32_t* family);
void orc_counters(const orc* o, uint32_t* c3 /* gs, g_rs, g_cl */);
void orc_anneal(orc* o, const orc_schedule* s, orc_result* r, orc_trace* t);

/* Max-3-Cut decode of a spin vector of the embedded instance (input order of
 * the embedded vertices).  labels: n entries in {0,1,2}.  Returns the 3-cut. */
int64_t orc_max3cut_decode(const orc* o, const int8_t* spins, int32_t* labels);
/* 3-cut of a labelling of the original graph. */
int64_t orc_max3cut_value(const orc* o, const int32_t* labels);

/* Controller: one application of the adaptive rule + schedule advance to a
 * state given explicitly (for table-driven tests). */
typedef struct {
  double beta, delta;
  int32_t z, cycle, cooldown, enable, hist_len, stop;
  int64_t hist[64];
} orc_ctrl;
int32_t orc_controller_step(orc_ctrl* c, const orc_schedule* s, int64_t mstar);

/* Hamming-distance diagnostic: normalised pairwise distance with the
 * global-flip symmetry folded in (Supplement, Hamming distance). */
double orc_mean_pair_distance(const orc* o);

/* Replaces the population: spins (labels for Potts instances) in input ids,
 * slot-major [R][n], and the lineage ids (NULL: unchanged).  Fields and
 * energies are recomputed from the spins (Eq. 3 and H = -1/2 sum s h; Eq. 6
 * for labels).  Returns 0, or -1 (nothing changed) for a value outside the
 * spin or label range. */
int32_t orc_set_population(orc* o, const int8_t* spins, const int32_t* family);

/* Checkpoints in the library's documented byte layout (version 1): header
 * of 640 bytes (magic "PAMCCKP1", version, kind, n, R, seed, the three stream
 * counters, M*, beta, Delta, twelve int32 controller and count fields, the
 * sum of ln Q, history[64]), then spins [R][n] in input ids, lineage [R]
 * (int32) and the configuration of M* [n].  orc_set_checkpoint returns 0, or
 * -1 (nothing changed) for a buffer that is not a checkpoint of an instance
 * of this kind, n and R. */
int64_t orc_checkpoint_size(const orc* o);
void orc_get_checkpoint(const orc* o, uint8_t* buf);
int32_t orc_set_checkpoint(orc* o, const uint8_t* buf, int64_t bytes);

/* Sets the stream counters (sweeps, resamplings, cluster moves). */
void orc_set_counters(orc* o, const uint32_t* c3);

/* All R(R-1)/2 normalised pair distances d_H = min(d, 1-d), pairs (a, b)
 * with a < b in row-major order. */
void orc_pair_distances(const orc* o, double* out);

#ifdef __cplusplus
}
#endif
#endif
