/*
 * pamc_oracle.c -- plain single-threaded CPU oracle for augmented PAMC.
 *
 * TEST INFRASTRUCTURE ONLY (see pamc_oracle.h).  Nothing here is tuned: each
 * step follows the paper's order and notation so that it can be read against
 * the paper.  Build with -ffp-contract=off: every floating-point value that
 * decides an integer (thresholds, resampling weights, the inverse
 * temperature) is produced by a fixed sequence of IEEE-754 operations.
 */
#include "pamc_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11).  Each round multiplies counter words 0 and 2   */
/* by the two round multipliers, xors the high halves with the other two    */
/* counter words and the round key, and the key advances by the two Weyl    */
/* constants between rounds.                                                */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * x0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * x2;
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)p0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                   uint32_t out[4]) {
  uint32_t ctr[4] = {c0, c1, c2, c3};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Exponential: Cody & Waite argument reduction (W. J. Cody, W. Waite,      */
/* "Software Manual for the Elementary Functions", 1980):                   */
/*   x = k ln2 + r, |r| <= ln2/2, with ln2 split in a high part whose       */
/*   product with k is exact and a low correction;                         */
/* e^r by its Taylor series to degree 13 in Horner form with fused          */
/* multiply-adds; then scaling by 2^k done in exact power-of-two steps so   */
/* that a subnormal result is rounded once.                                 */
/* ------------------------------------------------------------------------ */
static double pow2i(int k) { /* 2^k for -1022 <= k <= 1023 */
  uint64_t bits = (uint64_t)(k + 1023) << 52;
  double d;
  memcpy(&d, &bits, sizeof d);
  return d;
}

double orc_pexp(double x) {
  const double inv_ln2 = 1.4426950408889634;
  const double ln2_hi = 0.6931471803691238;     /* 32 significant bits */
  const double ln2_lo = 1.9082149292705877e-10;
  if (x != x) return x;
  if (x > 709.8) return INFINITY;
  if (x < -745.5) return 0.0;
  double k = rint(x * inv_ln2);
  double r = (x - k * ln2_hi) - k * ln2_lo;
  /* 1/j! for j = 13 .. 2 */
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
  int ki = (int)k;
  if (ki > 1000) return (p * pow2i(ki - 200)) * pow2i(200);
  if (ki < -1000) return (p * pow2i(ki + 200)) * pow2i(-200);
  return p * pow2i(ki);
}

/* ------------------------------------------------------------------------ */
/* Acceptance thresholds.  x = s_k h_k, the energy change of a flip is 2x.  */
/* Heat bath (Eq. 4): the new spin is +1 with probability                   */
/* (1 + tanh(beta h))/2, so the flip probability is 1/(1 + e^{2 beta x}).   */
/* Metropolis: min(1, e^{-2 beta x}).  A flip happens iff a uniform 32-bit  */
/* word u satisfies u < T, T = min(floor(p 2^32), 2^32 - 1); Metropolis     */
/* moves with x <= 0 are always taken.                                      */
/* ------------------------------------------------------------------------ */
uint32_t orc_threshold(double beta, int32_t rule, int64_t x) {
  double t = 2.0 * beta;
  double p;
  if (rule == ORC_RULE_METROPOLIS) {
    if (x <= 0) return 0xFFFFFFFFu;
    p = orc_pexp(-(t * (double)x));
  } else {
    double e = orc_pexp(t * (double)x);
    p = 1.0 / (1.0 + e);
  }
  double q = floor(p * 4294967296.0);
  if (q >= 4294967295.0) return 0xFFFFFFFFu;
  return (uint32_t)q;
}

static int flip_decision(uint32_t u, double beta, int32_t rule, int64_t x) {
  if (rule == ORC_RULE_METROPOLIS && x <= 0) return 1;
  return u < orc_threshold(beta, rule, x);
}

/* ------------------------------------------------------------------------ */
/* Instance                                                                 */
/* ------------------------------------------------------------------------ */
struct orc {
  int32_t n, nnz, R, rule, shuffle, dense;
  uint64_t seed;
  /* graph in internal ids */
  int32_t *row_ptr, *col, *J;
  int32_t ncls, *class_ptr;
  int32_t *to_input, *to_internal;
  int64_t W, X;
  /* population, slot-major [R][n] */
  int8_t* s;
  int32_t* h;
  int64_t* E;
  int32_t* family;
  uint32_t gs, g_rs, g_cl;
  int64_t mstar;
  int8_t* best; /* internal ids */
  /* Max-3-Cut embedding: original graph (input ids) */
  int32_t m3_n;
  int32_t *m3_row_ptr, *m3_col, *m3_w;
  /* Potts labels (potts_K > 0): s holds labels 0..K-1, h is unused */
  int32_t potts_K, potts_rule;
  double potts_gamma;
  /* Algorithm 1's controller and the run's counts, kept between calls so
   * that a run can be resumed */
  orc_ctrl ctrl;
  orc_result run;
};

static void set_err(char* err, int32_t errlen, const char* msg) {
  if (err && errlen > 0) {
    strncpy(err, msg, (size_t)errlen - 1);
    err[errlen - 1] = 0;
  }
}

int32_t orc_colour(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* colour) {
  /* Saturation-degree (DSATUR) colouring: repeatedly take the uncoloured
   * vertex with the most distinct colours among its neighbours, ties to the
   * larger degree, then to the lower id, and give it the least colour no
   * neighbour has.  A plain O(n^2) scan: the selection rule is written out
   * as stated. */
  int32_t ncls = 0;
  int32_t* sat = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
  int32_t* seen = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  for (int32_t v = 0; v < n; ++v) colour[v] = -1;
  for (int32_t k = 0; k <= n; ++k) seen[k] = -1;
  for (int32_t step = 0; step < n; ++step) {
    int32_t best = -1;
    for (int32_t v = 0; v < n; ++v) {
      if (colour[v] >= 0) continue;
      if (best < 0 || sat[v] > sat[best] ||
          (sat[v] == sat[best] && row_ptr[v + 1] - row_ptr[v] > row_ptr[best + 1] - row_ptr[best]))
        best = v;
    }
    const int32_t v = best;
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e)
      if (colour[col[e]] >= 0) seen[colour[col[e]]] = v;
    int32_t k = 0;
    while (seen[k] == v) ++k;
    colour[v] = k;
    if (k + 1 > ncls) ncls = k + 1;
    /* the neighbours' saturation: colour k is new to u unless another
     * coloured neighbour of u has it */
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      const int32_t u = col[e];
      if (colour[u] >= 0) continue;
      int has = 0;
      for (int32_t f = row_ptr[u]; f < row_ptr[u + 1] && !has; ++f)
        if (col[f] != v && colour[col[f]] == k) has = 1;
      if (!has) sat[u]++;
    }
  }
  free(seen);
  free(sat);
  return ncls;
}

static int validate_csr(int32_t n, const int32_t* row_ptr, const int32_t* col,
                        const int32_t* w, char* err, int32_t errlen) {
  if (n <= 0) { set_err(err, errlen, "n must be positive"); return 0; }
  if (row_ptr[0] != 0) { set_err(err, errlen, "row_ptr[0] != 0"); return 0; }
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) { set_err(err, errlen, "row_ptr not monotone"); return 0; }
  int32_t nnz = row_ptr[n];
  for (int32_t e = 0; e < nnz; ++e) {
    if (col[e] < 0 || col[e] >= n) { set_err(err, errlen, "column out of range"); return 0; }
    if (w[e] == 0) { set_err(err, errlen, "zero weight"); return 0; }
  }
  /* self loops, duplicates, symmetry: dense scan per row (slow and plain) */
  int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* wt = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  for (int32_t v = 0; v < n; ++v) mark[v] = -1;
  int ok = 1;
  for (int32_t v = 0; v < n && ok; ++v) {
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      int32_t u = col[e];
      if (u == v) { set_err(err, errlen, "self loop"); ok = 0; break; }
      if (mark[u] == v) { set_err(err, errlen, "duplicate edge"); ok = 0; break; }
      mark[u] = v;
      wt[u] = w[e];
    }
    if (!ok) break;
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1] && ok; ++e) {
      int32_t u = col[e];
      int found = 0;
      for (int32_t f = row_ptr[u]; f < row_ptr[u + 1]; ++f)
        if (col[f] == v) { found = (w[f] == wt[u]); break; }
      if (!found) { set_err(err, errlen, "not symmetric"); ok = 0; }
    }
  }
  free(mark);
  free(wt);
  return ok;
}

static orc* alloc_orc(int32_t n, int32_t R) {
  orc* o = (orc*)calloc(1, sizeof(orc));
  o->n = n;
  o->R = R;
  o->s = (int8_t*)calloc((size_t)R * n, 1);
  o->h = (int32_t*)calloc((size_t)R * n, sizeof(int32_t));
  o->E = (int64_t*)calloc((size_t)R, sizeof(int64_t));
  o->family = (int32_t*)calloc((size_t)R, sizeof(int32_t));
  o->best = (int8_t*)calloc((size_t)n, 1);
  o->to_input = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  o->to_internal = (int32_t*)calloc((size_t)n, sizeof(int32_t));
  return o;
}

/* Population initialisation (Algorithm 1, initialization): uniform random
 * spins, local fields by Eq. 3, energies H = -1/2 sum_v s_v h_v, M* = 0 with
 * the all-(+1) configuration (cut 0) as the best. */
static void init_population(orc* o) {
  int32_t n = o->n;
  for (int32_t r = 0; r < o->R; ++r) {
    int8_t* s = o->s + (size_t)r * n;
    for (int32_t v = 0; v < n; ++v) {
      uint32_t out[4];
      philox(o->seed, (uint32_t)(v >> 2), 0u, (uint32_t)r, ORC_TAG_INIT, out);
      s[v] = (out[v & 3] < 0x80000000u) ? 1 : -1;
    }
    int32_t* h = o->h + (size_t)r * n;
    int64_t twoE = 0;
    for (int32_t v = 0; v < n; ++v) {
      int64_t acc = 0;
      for (int32_t e = o->row_ptr[v]; e < o->row_ptr[v + 1]; ++e)
        acc += (int64_t)o->J[e] * s[o->col[e]];
      h[v] = (int32_t)acc;
      twoE += (int64_t)s[v] * acc;
    }
    o->E[r] = -twoE / 2;
    o->family[r] = r;
  }
  o->mstar = 0;
  for (int32_t v = 0; v < n; ++v) o->best[v] = 1;
  o->gs = o->g_rs = o->g_cl = 0;
}

/* Builds the internal graph from a validated CSR over input ids.  colour
 * classes give the sweep order; internal id = rank in (class, input id). */
int32_t orc_max3cut_colour(int32_t n, const int32_t* row_ptr, const int32_t* col, int32_t* colour) {
  /* The embedding's classes from the base graph's colouring c (orc_colour,
   * k colours): spin (i, a) takes (c(i) + a) mod m, m = max(k, 3), and the
   * ancilla colour m.  Spins of one vertex differ by 1 or 2 < m; spins
   * (i, a), (j, a) of an edge ij differ as c(i) != c(j) (both < m); the
   * ancilla meets every spin.  So the colouring is proper, with m + 1
   * classes of about 3n/m spins each and the ancilla alone. */
  int32_t* c = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t k = n > 0 ? orc_colour(n, row_ptr, col, c) : 0;
  int32_t m = k > 3 ? k : 3;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t a = 0; a < 3; ++a) colour[3 * i + a] = (c[i] + a) % m;
  colour[3 * n] = m;
  free(c);
  return m + 1;
}

/* The relabelled graph, from a given colouring (colour_in, ncls_in) or, with
 * colour_in NULL, orc_colour's (every vertex its own class when dense). */
static void build_graph(orc* o, const int32_t* row_ptr, const int32_t* col,
                        const int32_t* Jin, int32_t dense, const int32_t* colour_in, int32_t ncls_in) {
  int32_t n = o->n, nnz = row_ptr[n];
  o->nnz = nnz;
  o->dense = dense;
  int32_t* colour = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (colour_in) {
    for (int32_t v = 0; v < n; ++v) colour[v] = colour_in[v];
    o->ncls = ncls_in;
  } else if (dense) {
    for (int32_t v = 0; v < n; ++v) colour[v] = v;
    o->ncls = n;
  } else {
    o->ncls = orc_colour(n, row_ptr, col, colour);
  }
  o->class_ptr = (int32_t*)calloc((size_t)o->ncls + 1, sizeof(int32_t));
  for (int32_t v = 0; v < n; ++v) o->class_ptr[colour[v] + 1]++;
  for (int32_t k = 0; k < o->ncls; ++k) o->class_ptr[k + 1] += o->class_ptr[k];
  int32_t* fill = (int32_t*)malloc(sizeof(int32_t) * (size_t)o->ncls);
  for (int32_t k = 0; k < o->ncls; ++k) fill[k] = o->class_ptr[k];
  for (int32_t v = 0; v < n; ++v) { /* ascending input id within a class */
    int32_t iv = fill[colour[v]]++;
    o->to_internal[v] = iv;
    o->to_input[iv] = v;
  }
  free(fill);
  free(colour);
  o->row_ptr = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  o->col = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
  o->J = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
  o->row_ptr[0] = 0;
  int64_t W = 0, X = 0;
  for (int32_t iv = 0; iv < n; ++iv) {
    int32_t v = o->to_input[iv];
    int32_t base = o->row_ptr[iv];
    int32_t deg = row_ptr[v + 1] - row_ptr[v];
    int64_t absum = 0;
    for (int32_t e = 0; e < deg; ++e) {
      int32_t u = col[row_ptr[v] + e];
      o->col[base + e] = o->to_internal[u];
      o->J[base + e] = Jin[row_ptr[v] + e];
      absum += llabs((long long)Jin[row_ptr[v] + e]);
      if (u > v) W += -(int64_t)Jin[row_ptr[v] + e];
    }
    if (absum > X) X = absum;
    o->row_ptr[iv + 1] = base + deg;
  }
  o->W = W;
  o->X = X;
}

orc* orc_create_sparse(int32_t n, const int32_t* row_ptr, const int32_t* col,
                       const int32_t* w, int32_t objective, int32_t replicas,
                       uint64_t seed, int32_t rule, int32_t shuffle_classes,
                       char* err, int32_t errlen) {
  if (replicas <= 0) { set_err(err, errlen, "replicas must be positive"); return NULL; }
  if (!validate_csr(n, row_ptr, col, w, err, errlen)) return NULL;
  int32_t nnz = row_ptr[n];
  int32_t* Jin = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
  int64_t X = 0;
  for (int32_t v = 0; v < n; ++v) {
    int64_t a = 0;
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      Jin[e] = (objective == ORC_OBJ_MAXCUT) ? -w[e] : w[e];
      a += llabs((long long)w[e]);
    }
    if (a > X) X = a;
  }
  if (2 * X >= 2147483647LL) { free(Jin); set_err(err, errlen, "local field range exceeds int32"); return NULL; }
  orc* o = alloc_orc(n, replicas);
  o->seed = seed;
  o->rule = rule;
  o->shuffle = shuffle_classes;
  build_graph(o, row_ptr, col, Jin, 0, NULL, 0);
  free(Jin);
  init_population(o);
  return o;
}

/* ------------------------------------------------------------------------ */
/* Potts Max-K-Cut (Sec. "Max-3-Cut"; Eqs. 6-9; Supplement, cascaded         */
/* sampler).  Labels start uniform: label = floor(u K / 2^32) with u the     */
/* initialization word of the vertex.  E = -sum_{i<j} J_ij (2 delta - 1).    */
/* ------------------------------------------------------------------------ */
int64_t orc_potts_energy(const orc* o, int32_t r) {
  const int8_t* lab = o->s + (size_t)r * o->n;
  int64_t E = 0;
  for (int32_t v = 0; v < o->n; ++v)
    for (int32_t e = o->row_ptr[v]; e < o->row_ptr[v + 1]; ++e) {
      int32_t j = o->col[e];
      if (j > v) E -= (int64_t)o->J[e] * (lab[v] == lab[j] ? 1 : -1);
    }
  return E;
}

static void init_potts(orc* o) {
  int32_t n = o->n;
  for (int32_t r = 0; r < o->R; ++r) {
    int8_t* lab = o->s + (size_t)r * n;
    for (int32_t v = 0; v < n; ++v) {
      uint32_t out[4];
      philox(o->seed, (uint32_t)(v >> 2), 0u, (uint32_t)r, ORC_TAG_INIT, out);
      lab[v] = (int8_t)(((uint64_t)out[v & 3] * (uint64_t)o->potts_K) >> 32);
    }
    o->E[r] = orc_potts_energy(o, r);
    o->family[r] = r;
  }
  o->mstar = 0;
  for (int32_t v = 0; v < n; ++v) o->best[v] = 0;  /* all in one part: cut 0 */
  o->gs = o->g_rs = o->g_cl = 0;
}

orc* orc_create_potts(int32_t n, const int32_t* row_ptr, const int32_t* col,
                      const int32_t* w, int32_t K, int32_t replicas, uint64_t seed,
                      int32_t potts_rule, double gamma, int32_t shuffle_classes,
                      char* err, int32_t errlen) {
  if (replicas <= 0) { set_err(err, errlen, "replicas must be positive"); return NULL; }
  if (K < 2 || K > 4) { set_err(err, errlen, "K must be 2, 3 or 4"); return NULL; }
  if (potts_rule == ORC_POTTS_CASCADE && K != 3) { set_err(err, errlen, "the cascade is for K = 3"); return NULL; }
  if (potts_rule != ORC_POTTS_SOFTMAX && potts_rule != ORC_POTTS_CASCADE) { set_err(err, errlen, "bad rule"); return NULL; }
  if (!validate_csr(n, row_ptr, col, w, err, errlen)) return NULL;
  int32_t nnz = row_ptr[n];
  int32_t* Jin = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
  int64_t X = 0;
  for (int32_t v = 0; v < n; ++v) {
    int64_t a = 0;
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      Jin[e] = -w[e];
      a += llabs((long long)w[e]);
    }
    if (a > X) X = a;
  }
  if (2 * X >= 2147483647LL) { free(Jin); set_err(err, errlen, "local field range exceeds int32"); return NULL; }
  orc* o = alloc_orc(n, replicas);
  o->seed = seed;
  o->rule = ORC_RULE_HEATBATH;
  o->shuffle = shuffle_classes;
  o->potts_K = K;
  o->potts_rule = potts_rule;
  o->potts_gamma = gamma;
  build_graph(o, row_ptr, col, Jin, 0, NULL, 0);
  free(Jin);
  init_potts(o);
  return o;
}

orc* orc_create_dense(int32_t n, const int8_t* J, int32_t objective,
                      int32_t replicas, uint64_t seed, int32_t rule,
                      char* err, int32_t errlen) {
  if (n <= 0 || replicas <= 0) { set_err(err, errlen, "bad size"); return NULL; }
  for (int32_t i = 0; i < n; ++i) {
    if (J[(size_t)i * n + i] != 0) { set_err(err, errlen, "nonzero diagonal"); return NULL; }
    for (int32_t j = 0; j < i; ++j)
      if (J[(size_t)i * n + j] != J[(size_t)j * n + i]) { set_err(err, errlen, "not symmetric"); return NULL; }
  }
  int64_t nnz = 0;
  for (size_t k = 0; k < (size_t)n * n; ++k) nnz += (J[k] != 0);
  int32_t* rp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  int32_t* cl = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
  int32_t* jj = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
  int32_t p = 0;
  rp[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t j = 0; j < n; ++j) {
      int8_t v = J[(size_t)i * n + j];
      if (v) { cl[p] = j; jj[p] = (objective == ORC_OBJ_MAXCUT) ? -(int32_t)v : (int32_t)v; ++p; }
    }
    rp[i + 1] = p;
  }
  orc* o = alloc_orc(n, replicas);
  o->seed = seed;
  o->rule = rule;
  o->shuffle = 0;
  build_graph(o, rp, cl, jj, 1, NULL, 0);
  free(rp); free(cl); free(jj);
  init_population(o);
  return o;
}

void orc_dense_random(int32_t n, uint64_t seed, int8_t* J) {
  for (int32_t i = 0; i < n; ++i) {
    J[(size_t)i * n + i] = 0;
    for (int32_t j = i + 1; j < n; ++j) {
      uint32_t out[4];
      philox(seed, (uint32_t)i, (uint32_t)j, 0u, ORC_TAG_DENSE, out);
      int8_t v = (out[0] & 1u) ? 1 : -1;
      J[(size_t)i * n + j] = v;
      J[(size_t)j * n + i] = v;
    }
  }
}

/* Max-3-Cut as an Ising problem: spins x_{i,a} (a = 0,1,2) one-hot encode
 * the label of vertex i, plus one ancilla spin that carries the linear
 * terms.  With weighted degree d_i and penalty A_i = floor(d_i/3) + 1,
 * f = sum_i A_i (1 - sum_a x_ia)^2 + sum_{(i,j)} w_ij sum_a x_ia x_ja is
 * minimised only by one-hot states, where it equals W - cut3.  Writing
 * x = (1 + s)/2 and multiplying the linear terms by the ancilla gives
 * J_{(i,a),anc} = -(2 A_i + d_i), J_{(i,a),(i,b)} = -2 A_i,
 * J_{(i,a),(j,a)} = -w_ij, and H = 4 f - (4 sum A + 3 W) when s_anc = +1.
 * Embedded input ids: (i,a) -> 3i + a, ancilla -> 3n. */
orc* orc_create_max3cut(int32_t n, const int32_t* row_ptr, const int32_t* col,
                        const int32_t* w, int32_t replicas, uint64_t seed,
                        int32_t rule, int32_t shuffle_classes,
                        char* err, int32_t errlen) {
  if (!validate_csr(n, row_ptr, col, w, err, errlen)) return NULL;
  int32_t nnz = row_ptr[n];
  for (int32_t e = 0; e < nnz; ++e)
    if (w[e] <= 0) { set_err(err, errlen, "Max-3-Cut needs positive weights"); return NULL; }
  int32_t N = 3 * n + 1;
  int64_t* d = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  for (int32_t i = 0; i < n; ++i)
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) d[i] += w[e];
  /* per embedded vertex (i,a): 2 same-vertex partners + deg(i) + ancilla */
  int64_t enn = 0;
  for (int32_t i = 0; i < n; ++i) enn += 3 * (3 + (int64_t)(row_ptr[i + 1] - row_ptr[i]));
  enn += 3 * (int64_t)n; /* ancilla row */
  int32_t* rp = (int32_t*)malloc(sizeof(int32_t) * ((size_t)N + 1));
  int32_t* cl = (int32_t*)malloc(sizeof(int32_t) * (size_t)enn);
  int32_t* jj = (int32_t*)malloc(sizeof(int32_t) * (size_t)enn);
  int64_t p = 0;
  int64_t X = 0;
  rp[0] = 0;
  for (int32_t i = 0; i < n; ++i) {
    int64_t A = d[i] / 3 + 1;
    for (int32_t a = 0; a < 3; ++a) {
      int64_t absum = 0;
      for (int32_t b = 0; b < 3; ++b)
        if (b != a) { cl[p] = 3 * i + b; jj[p] = (int32_t)(-2 * A); absum += 2 * A; ++p; }
      for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        cl[p] = 3 * col[e] + a; jj[p] = -w[e]; absum += w[e]; ++p;
      }
      cl[p] = 3 * n; jj[p] = (int32_t)(-(2 * A + d[i])); absum += 2 * A + d[i]; ++p;
      if (absum > X) X = absum;
      rp[3 * i + a + 1] = (int32_t)p;
    }
  }
  int64_t absum = 0;
  for (int32_t i = 0; i < n; ++i) {
    int64_t A = d[i] / 3 + 1;
    for (int32_t a = 0; a < 3; ++a) { cl[p] = 3 * i + a; jj[p] = (int32_t)(-(2 * A + d[i])); absum += 2 * A + d[i]; ++p; }
  }
  if (absum > X) X = absum;
  rp[N] = (int32_t)p;
  free(d);
  if (2 * X >= 2147483647LL) {
    free(rp); free(cl); free(jj);
    set_err(err, errlen, "local field range exceeds int32");
    return NULL;
  }
  orc* o = alloc_orc(N, replicas);
  o->seed = seed;
  o->rule = rule;
  o->shuffle = shuffle_classes;
  int32_t* m3c = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  int32_t m3k = orc_max3cut_colour(n, row_ptr, col, m3c);
  build_graph(o, rp, cl, jj, 0, m3c, m3k);
  free(m3c);
  free(rp); free(cl); free(jj);
  o->m3_n = n;
  o->m3_row_ptr = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  o->m3_col = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
  o->m3_w = (int32_t*)malloc(sizeof(int32_t) * ((size_t)nnz + 1));
  memcpy(o->m3_row_ptr, row_ptr, sizeof(int32_t) * ((size_t)n + 1));
  memcpy(o->m3_col, col, sizeof(int32_t) * (size_t)nnz);
  memcpy(o->m3_w, w, sizeof(int32_t) * (size_t)nnz);
  init_population(o);
  return o;
}

void orc_destroy(orc* o) {
  if (!o) return;
  free(o->row_ptr); free(o->col); free(o->J); free(o->class_ptr);
  free(o->to_input); free(o->to_internal);
  free(o->s); free(o->h); free(o->E); free(o->family); free(o->best);
  free(o->m3_row_ptr); free(o->m3_col); free(o->m3_w);
  free(o);
}

int32_t orc_n(const orc* o) { return o->n; }
int32_t orc_replicas(const orc* o) { return o->R; }
int32_t orc_num_classes(const orc* o) { return o->ncls; }
int64_t orc_W(const orc* o) { return o->W; }
int64_t orc_X(const orc* o) { return o->X; }
void orc_internal_ids(const orc* o, int32_t* t) { memcpy(t, o->to_internal, sizeof(int32_t) * (size_t)o->n); }
void orc_class_ptr(const orc* o, int32_t* c) { memcpy(c, o->class_ptr, sizeof(int32_t) * ((size_t)o->ncls + 1)); }
void orc_counters(const orc* o, uint32_t* c) { c[0] = o->gs; c[1] = o->g_rs; c[2] = o->g_cl; }

/* ------------------------------------------------------------------------ */
/* Monte Carlo sweep (Eqs. 3-4, Algorithm 1): every spin is visited once per */
/* sweep, one at a time, in an order that changes from sweep to sweep.       */
/* Here the order is colour class by colour class.  A class holds mutually   */
/* uncoupled spins, so the visits inside it commute; the class sequence is a */
/* fresh Fisher-Yates permutation each sweep.  Dense instances use the fixed */
/* order 0..n-1.                                                             */
/* ------------------------------------------------------------------------ */
static void class_order(const orc* o, uint32_t gs, int32_t* order) {
  for (int32_t k = 0; k < o->ncls; ++k) order[k] = k;
  if (!o->shuffle) return;
  for (int32_t i = o->ncls - 1; i >= 1; --i) {
    uint32_t out[4];
    philox(o->seed, (uint32_t)i, gs, 0u, ORC_TAG_ORDER, out);
    int32_t j = (int32_t)(((uint64_t)out[0] * (uint64_t)(i + 1)) >> 32);
    int32_t t = order[i]; order[i] = order[j]; order[j] = t;
  }
}

static void flip_spin(orc* o, int32_t r, int32_t v) {
  int8_t* s = o->s + (size_t)r * o->n;
  int32_t* h = o->h + (size_t)r * o->n;
  s[v] = (int8_t)-s[v];
  for (int32_t e = o->row_ptr[v]; e < o->row_ptr[v + 1]; ++e)
    h[o->col[e]] += 2 * o->J[e] * s[v];
}

/* One Potts label update (Eqs. 7-9, or the Supplement's cascade).
 * omega_k = e^{beta (syn_k - max syn)}: the numerators of Eq. 8 scaled by a
 * common factor, so they do not overflow.  Both rules compare quantities
 * multiplied through by their positive denominators, which leaves every
 * comparison of the paper's formulas unchanged and needs no division:
 *   softmax: with S = sum_m omega_m (summed in label order), P_k - gamma U_k
 *     is compared as omega_k - (gamma U_k) S, U_k = u_k / 2^32; the largest
 *     wins, the lowest k on ties (Eq. 9).
 *   cascade (K = 3, labels alpha, beta, gamma = 0, 1, 2): tanh(Delta_1) =
 *     (w0 - s12) / (w0 + s12) with s12 = w1 + w2 and tanh(Delta_2) =
 *     (w1 - w2) / s12, since tanh(ln(a/b)/2) = (a - b)/(a + b); the p-bit
 *     b = [tanh(Delta) > eta], eta = u / 2^31 - 1 in [-1, 1), is taken as
 *     numerator > eta * denominator.  b1 = 1 picks label 0, else b2 picks
 *     label 1 (b2 = 1) or 2. */
int32_t orc_potts_choose(int32_t K, int32_t potts_rule, double gamma, double beta,
                         const int64_t* syn, const uint32_t* u) {
  int64_t m = syn[0];
  for (int32_t k = 1; k < K; ++k)
    if (syn[k] > m) m = syn[k];
  double om[4];
  for (int32_t k = 0; k < K; ++k) om[k] = orc_pexp(beta * (double)(syn[k] - m));
  if (potts_rule == ORC_POTTS_CASCADE) {
    double s12 = om[1] + om[2];
    double eta1 = (double)u[0] * (1.0 / 2147483648.0) - 1.0;
    if (om[0] - s12 > eta1 * (om[0] + s12)) return 0;
    double eta2 = (double)u[1] * (1.0 / 2147483648.0) - 1.0;
    return om[1] - om[2] > eta2 * s12 ? 1 : 2;
  }
  double S = 0.0;
  for (int32_t k = 0; k < K; ++k) S += om[k];
  int32_t best = 0;
  double bs = om[0] - (gamma * ((double)u[0] * (1.0 / 4294967296.0))) * S;
  for (int32_t k = 1; k < K; ++k) {
    double sc = om[k] - (gamma * ((double)u[k] * (1.0 / 4294967296.0))) * S;
    if (sc > bs) { bs = sc; best = k; }
  }
  return best;
}

/* Uniform words of a Potts visit: a visit takes W words (W = K for the
 * softmax, 2 for the cascade); the four vertices of a quad (v >> 2) share W
 * Philox blocks (quad, sweep, replica, POTTS | b << 8), b = 0..W-1, read as
 * one sequence of 4W words, of which vertex v takes words (v & 3) W ..
 * (v & 3) W + W - 1. */
static void potts_words(const orc* o, int32_t r, int32_t v, uint32_t* u) {
  int32_t W = o->potts_rule == ORC_POTTS_CASCADE ? 2 : o->potts_K;
  uint32_t blk[16];
  for (int32_t b = 0; b < W; ++b)
    philox(o->seed, (uint32_t)(v >> 2), o->gs, (uint32_t)r, ORC_TAG_POTTS | ((uint32_t)b << 8), blk + 4 * b);
  for (int32_t k = 0; k < W; ++k) u[k] = blk[(v & 3) * W + k];
}

/* Potts update of vertex v in replica r: the K-label field (Eq. 7), the
 * new label, and the Eq. 6 energy change -2 (syn_new - syn_old). */
static void potts_visit(orc* o, int32_t r, int32_t v, double beta) {
  int8_t* lab = o->s + (size_t)r * o->n;
  int64_t syn[4] = {0, 0, 0, 0};
  for (int32_t e = o->row_ptr[v]; e < o->row_ptr[v + 1]; ++e) syn[lab[o->col[e]]] += o->J[e];
  uint32_t u[4] = {0, 0, 0, 0};
  potts_words(o, r, v, u);
  int32_t old = lab[v];
  int32_t nw = orc_potts_choose(o->potts_K, o->potts_rule, o->potts_gamma, beta, syn, u);
  if (nw != old) {
    o->E[r] += -2 * (syn[nw] - syn[old]);
    lab[v] = (int8_t)nw;
  }
}

void orc_sweep(orc* o, double beta, int32_t nsweeps) {
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)o->ncls);
  for (int32_t sw = 0; sw < nsweeps; ++sw) {
    class_order(o, o->gs, order);
    for (int32_t ci = 0; ci < o->ncls; ++ci) {
      int32_t c = order[ci];
      for (int32_t v = o->class_ptr[c]; v < o->class_ptr[c + 1]; ++v) {
        if (o->potts_K) {
          for (int32_t r = 0; r < o->R; ++r) potts_visit(o, r, v, beta);
          continue;
        }
        for (int32_t r = 0; r < o->R; ++r) {
          int64_t x = (int64_t)o->s[(size_t)r * o->n + v] * o->h[(size_t)r * o->n + v];
          uint32_t out[4];
          philox(o->seed, (uint32_t)(v >> 2), o->gs, (uint32_t)r, ORC_TAG_SWEEP, out);
          if (flip_decision(out[v & 3], beta, o->rule, x)) {
            o->E[r] += 2 * x;
            flip_spin(o, r, v);
          }
        }
      }
    }
    o->gs++;
  }
  free(order);
}

/* ------------------------------------------------------------------------ */
/* Resampling (Eqs. 1-2).  Replica j receives on average                    */
/* tau_j = e^{-Delta E_j} / Q copies with Q = (1/R) sum_j e^{-Delta E_j}, so */
/* sum_j tau_j = R and the population size stays R.  Multinomial: R         */
/* independent draws of a parent with probability proportional to its       */
/* weight.  Weights are shifted by the extreme energy (exact in exponent    */
/* arithmetic) and quantised to q_j = floor(w_j 2^48) so that the draw is   */
/* an exact integer computation; children are ordered by parent.            */
/* ------------------------------------------------------------------------ */
double orc_resample(orc* o, double delta_in, int32_t* parents_out) {
  int32_t R = o->R, n = o->n;
  /* Potts labels: the update of Eq. 8 at beta leaves e^{-(beta/2) E}
   * invariant for the Eq. 6 energy, so the weights use Delta/2. */
  double delta = o->potts_K ? 0.5 * delta_in : delta_in;
  int64_t Eref = o->E[0];
  for (int32_t r = 1; r < R; ++r) {
    if (delta >= 0 ? (o->E[r] < Eref) : (o->E[r] > Eref)) Eref = o->E[r];
  }
  double* w = (double*)malloc(sizeof(double) * (size_t)R);
  uint64_t* P = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)R);
  double wsum = 0.0;
  uint64_t Q = 0;
  for (int32_t r = 0; r < R; ++r) {
    double a = delta * (double)(o->E[r] - Eref);
    w[r] = orc_pexp(-a);
    wsum += w[r];
    uint64_t q = (uint64_t)floor(w[r] * 281474976710656.0); /* 2^48 */
    Q += q;
    P[r] = Q;
  }
  double lnq = -delta * (double)Eref + log(wsum) - log((double)R);
  int32_t* parent = (int32_t*)malloc(sizeof(int32_t) * (size_t)R);
  for (int32_t k = 0; k < R; ++k) {
    uint32_t out[4];
    philox(o->seed, (uint32_t)(k >> 1), o->g_rs, 0u, ORC_TAG_RS, out);
    uint64_t u = (k & 1) ? ((uint64_t)out[2] | ((uint64_t)out[3] << 32))
                         : ((uint64_t)out[0] | ((uint64_t)out[1] << 32));
    uint64_t y = (uint64_t)(((unsigned __int128)u * Q) >> 64);
    int32_t j = 0;
    while (P[j] <= y) ++j; /* least j with P_j > y */
    parent[k] = j;
  }
  /* order children by parent (counting sort) */
  int32_t* cnt = (int32_t*)calloc((size_t)R, sizeof(int32_t));
  for (int32_t k = 0; k < R; ++k) cnt[parent[k]]++;
  int32_t k = 0;
  for (int32_t j = 0; j < R; ++j)
    for (int32_t c = 0; c < cnt[j]; ++c) parent[k++] = j;
  free(cnt);
  int8_t* s2 = (int8_t*)malloc((size_t)R * n);
  int32_t* h2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)R * n);
  int64_t* E2 = (int64_t*)malloc(sizeof(int64_t) * (size_t)R);
  int32_t* f2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)R);
  for (int32_t c = 0; c < R; ++c) {
    int32_t p = parent[c];
    memcpy(s2 + (size_t)c * n, o->s + (size_t)p * n, (size_t)n);
    memcpy(h2 + (size_t)c * n, o->h + (size_t)p * n, sizeof(int32_t) * (size_t)n);
    E2[c] = o->E[p];
    f2[c] = o->family[p];
  }
  free(o->s); free(o->h); free(o->E); free(o->family);
  o->s = s2; o->h = h2; o->E = E2; o->family = f2;
  if (parents_out) memcpy(parents_out, parent, sizeof(int32_t) * (size_t)R);
  free(parent); free(w); free(P);
  o->g_rs++;
  return lnq;
}

/* ------------------------------------------------------------------------ */
/* Non-local cluster move (Sec. "Augmented PAMC", NCM; Algorithm 1).  Target */
/* replicas: the n_top lowest (E, slot).  A spin whose local field is 0 (an  */
/* iso-site) can be flipped at zero energy cost, and so can any set of them  */
/* with no coupling inside the set.  Trial t orders the iso-sites by a       */
/* Philox key and builds such a set greedily in that order (a site joins    */
/* unless it is coupled to one already taken).  Of the mis_trials sets the   */
/* largest is flipped, the earliest trial winning a tie; H is unchanged.     */
/* ------------------------------------------------------------------------ */
typedef struct { uint32_t key; int32_t v; } keyed;
static int cmp_keyed(const void* a, const void* b) {
  const keyed* x = (const keyed*)a;
  const keyed* y = (const keyed*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->v < y->v ? -1 : (x->v > y->v);
}
typedef struct { int64_t E; int32_t r; } eslot;
static int cmp_eslot(const void* a, const void* b) {
  const eslot* x = (const eslot*)a;
  const eslot* y = (const eslot*)b;
  if (x->E != y->E) return x->E < y->E ? -1 : 1;
  return x->r < y->r ? -1 : (x->r > y->r);
}

int32_t orc_cluster(orc* o, int32_t n_top, int32_t mis_trials, int32_t* chosen_sizes) {
  if (o->potts_K) return 0;  /* defined for Ising spins only */
  int32_t R = o->R, n = o->n;
  if (n_top > R) n_top = R;
  if (n_top < 0) n_top = 0;
  eslot* es = (eslot*)malloc(sizeof(eslot) * (size_t)R);
  for (int32_t r = 0; r < R; ++r) { es[r].E = o->E[r]; es[r].r = r; }
  qsort(es, (size_t)R, sizeof(eslot), cmp_eslot);
  keyed* iso = (keyed*)malloc(sizeof(keyed) * (size_t)n);
  int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* sel = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t* best = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  int32_t total = 0;
  for (int32_t i = 0; i < n_top; ++i) {
    int32_t r = es[i].r;
    int32_t* h = o->h + (size_t)r * n;
    int32_t nbest = 0;
    for (int32_t t = 0; t < mis_trials; ++t) {
      int32_t m = 0;
      for (int32_t v = 0; v < n; ++v) {
        if (h[v] != 0) continue;
        uint32_t out[4];
        philox(o->seed, (uint32_t)v, o->g_cl, (uint32_t)r, (uint32_t)ORC_TAG_CL | ((uint32_t)t << 8), out);
        iso[m].key = out[0];
        iso[m].v = v;
        ++m;
      }
      qsort(iso, (size_t)m, sizeof(keyed), cmp_keyed);
      for (int32_t v = 0; v < n; ++v) mark[v] = 0;
      int32_t ns = 0;
      for (int32_t q = 0; q < m; ++q) {
        int32_t v = iso[q].v;
        int ok = 1;
        for (int32_t e = o->row_ptr[v]; e < o->row_ptr[v + 1]; ++e)
          if (mark[o->col[e]]) { ok = 0; break; }
        if (ok) { mark[v] = 1; sel[ns++] = v; }
      }
      if (ns > nbest) { nbest = ns; memcpy(best, sel, sizeof(int32_t) * (size_t)ns); }
    }
    int64_t dE = 0;
    for (int32_t q = 0; q < nbest; ++q) {
      int32_t v = best[q];
      dE += 2 * (int64_t)o->s[(size_t)r * n + v] * h[v];
      flip_spin(o, r, v);
    }
    if (dE != 0) { fprintf(stderr, "oracle: cluster move changed the energy\n"); abort(); }
    if (chosen_sizes) chosen_sizes[i] = nbest;
    total += nbest;
  }
  free(es); free(iso); free(mark); free(sel); free(best);
  o->g_cl++;
  return total;
}

/* ------------------------------------------------------------------------ */
/* Best cut (Algorithm 1: M* <- max(M*, max Cut(P))).  Lowest slot on ties.  */
/* ------------------------------------------------------------------------ */
int64_t orc_update_best(orc* o) {
  int32_t rbest = 0;
  int64_t m = (o->W - o->E[0]) / 2;
  for (int32_t r = 1; r < o->R; ++r) {
    int64_t c = (o->W - o->E[r]) / 2;
    if (c > m) { m = c; rbest = r; }
  }
  if (m > o->mstar) {
    o->mstar = m;
    memcpy(o->best, o->s + (size_t)rbest * o->n, (size_t)o->n);
  }
  return o->mstar;
}

void orc_best(const orc* o, int64_t* cut, int64_t* energy, int8_t* spins) {
  if (cut) *cut = o->mstar;
  if (energy) *energy = o->W - 2 * o->mstar;
  if (spins)
    for (int32_t v = 0; v < o->n; ++v) spins[v] = o->best[o->to_internal[v]];
}

void orc_get_state(const orc* o, int8_t* spins, int32_t* fields, int64_t* energies,
                   int32_t* family) {
  int32_t n = o->n;
  for (int32_t r = 0; r < o->R; ++r) {
    for (int32_t v = 0; v < n; ++v) {
      int32_t iv = o->to_internal[v];
      if (spins) spins[(size_t)r * n + v] = o->s[(size_t)r * n + iv];
      if (fields) fields[(size_t)r * n + v] = o->h[(size_t)r * n + iv];
    }
    if (energies) energies[r] = o->E[r];
    if (family) family[r] = o->family[r];
  }
}

/* ------------------------------------------------------------------------ */
/* Adaptive temperature control (Algorithm 1; Sec. "Augmented PAMC").        */
/* The controller keeps the last win_long values of M*.  Once the window is  */
/* full and no cooldown runs, the history is classified by how many distinct */
/* values its two tails hold, and each class maps to one action:            */
/*                                                                           */
/*   class     | condition (ds, dl: distinct in short / long tail) | action  */
/*   STRONG    | ds <= max_s and dl <= max_l    | beta *= reheat, +dbeta, arm NCM */
/*   MILD      | ds <= max_s and dl >  max_l    | -dbeta if beta > beta0, else    */
/*             |                                | +dbeta (or stop: literal_break) */
/*   PROGRESS  | ds >  max_s                    | +dbeta                          */
/*   NONE      | cooldown or short history      | keep Delta                      */
/*                                                                           */
/* After the action the schedule moves on: a restart every z_rst steps       */
/* (beta, Delta, NCM arming, cooldown and the history reset), otherwise     */
/* beta += Delta and the cooldown counts down.  Event bits: 4 strong, 8 a    */
/* reversal, 16 a restart.                                                   */
/* ------------------------------------------------------------------------ */
enum { STAG_NONE = 0, STAG_PROGRESS = 1, STAG_MILD = 2, STAG_STRONG = 3 };

static int32_t distinct_tail(const int64_t* hist, int32_t len, int32_t w) {
  int32_t d = 0;
  for (int32_t i = len - w; i < len; ++i) {
    int dup = 0;
    for (int32_t j = len - w; j < i; ++j)
      if (hist[j] == hist[i]) { dup = 1; break; }
    if (!dup) ++d;
  }
  return d;
}

static void record_mstar(orc_ctrl* c, const orc_schedule* s, int64_t mstar) {
  if (c->hist_len == s->win_long) { /* the oldest value leaves */
    memmove(c->hist, c->hist + 1, sizeof(int64_t) * (size_t)(s->win_long - 1));
    c->hist_len--;
  }
  c->hist[c->hist_len++] = mstar;
}

static int32_t classify(const orc_ctrl* c, const orc_schedule* s) {
  if (!s->augmented || c->cooldown != 0 || c->hist_len < s->win_long) return STAG_NONE;
  int32_t ds = distinct_tail(c->hist, c->hist_len, s->win_short);
  int32_t dl = distinct_tail(c->hist, c->hist_len, s->win_long);
  if (ds > s->max_distinct_short) return STAG_PROGRESS;
  return dl <= s->max_distinct_long ? STAG_STRONG : STAG_MILD;
}

static int32_t act(orc_ctrl* c, const orc_schedule* s, int32_t cls) {
  switch (cls) {
    case STAG_STRONG:
      c->beta = s->reheat * c->beta;
      c->delta = s->dbeta;
      c->enable = 1;
      return 4;
    case STAG_MILD:
      if (c->beta > s->beta0) { c->delta = -s->dbeta; return 8; }
      if (s->literal_break) { c->stop = 1; return 0; }
      c->delta = s->dbeta;
      return 0;
    case STAG_PROGRESS:
      c->delta = s->dbeta;
      return 0;
    default:
      return 0;
  }
}

static int32_t advance_schedule(orc_ctrl* c, const orc_schedule* s) {
  if (s->z_rst > 0 && c->z >= s->z_rst) {
    c->cycle++;
    c->z = 1;
    c->beta = s->beta0;
    c->delta = s->dbeta;
    c->enable = 0;
    c->cooldown = 0;
    c->hist_len = 0;
    return 16;
  }
  c->z++;
  c->beta = c->beta + c->delta;
  if (c->cooldown > 0) c->cooldown--;
  return 0;
}

int32_t orc_controller_step(orc_ctrl* c, const orc_schedule* s, int64_t mstar) {
  record_mstar(c, s, mstar);
  int32_t ev = act(c, s, classify(c, s));
  return ev | advance_schedule(c, s);
}

/* ------------------------------------------------------------------------ */
/* Algorithm 1 (augmented PAMC); with augmented = 0 it is conventional PAMC  */
/* on the schedule beta0, beta0 + dbeta, ...; with resample = 0 it is        */
/* independent chains (SA).                                                  */
/* ------------------------------------------------------------------------ */
void orc_anneal(orc* o, const orc_schedule* s, orc_result* res, orc_trace* tr) {
  orc_ctrl* c = &o->ctrl;
  orc_result* run = &o->run;
  if (!s->resume) { /* a fresh run: Algorithm 1's initial controller */
    memset(c, 0, sizeof *c);
    c->z = 1;
    c->beta = s->beta0;
    c->delta = s->dbeta;
    memset(run, 0, sizeof *run);
    run->step_reached = -1;
  }
  c->stop = 0;
  int32_t step;
  for (step = run->steps_run; step < s->steps; ++step) {
    if (s->stop_at_target && o->mstar >= s->target) break;
    int32_t ev = 0;
    double lnq = 0.0;
    if (c->z > 1 && s->resample) {
      lnq = orc_resample(o, c->delta, NULL);
      run->sum_lnq += lnq;
      ev |= 1;
      if (s->augmented && c->enable && c->cooldown == 0 && !o->potts_K) {
        orc_cluster(o, s->n_top, s->mis_trials, NULL);
        c->enable = 0;
        c->cooldown = s->tau;
        ev |= 2;
        run->n_cluster_moves++;
      }
    }
    double beta_used = c->beta;
    orc_sweep(o, c->beta, s->sweeps);
    if (tr && tr->dh && s->dh_every > 0)
      tr->dh[step] = (step % s->dh_every == 0) ? orc_mean_pair_distance(o) : -1.0;
    int64_t m = orc_update_best(o);
    if (run->step_reached < 0 && m >= s->target) run->step_reached = step;
    ev |= orc_controller_step(c, s, m);
    if (ev & 4) run->n_reheats++;
    if (ev & 8) run->n_reversals++;
    if (ev & 16) run->n_restarts++;
    if (tr) {
      if (tr->mstar) tr->mstar[step] = m;
      if (tr->beta) tr->beta[step] = beta_used;
      if (tr->lnq) tr->lnq[step] = lnq;
      if (tr->events) tr->events[step] = ev;
    }
    if (c->stop) { ++step; break; }
  }
  run->steps_run = step;
  run->best_cut = o->mstar;
  run->best_energy = o->W - 2 * o->mstar;
  *res = *run;
}

/* ------------------------------------------------------------------------ */
/* Checkpoints (the library's byte layout, version 1; see the header).      */
/* ------------------------------------------------------------------------ */
static int32_t ckp_kind(const orc* o) { return o->dense ? 2 : (o->potts_K ? 1 : 0); }

int64_t orc_checkpoint_size(const orc* o) {
  return 640 + (int64_t)o->R * o->n + 4 * (int64_t)o->R + o->n;
}

static void wr(uint8_t* b, size_t at, const void* v, size_t len) { memcpy(b + at, v, len); }
static void rd(const uint8_t* b, size_t at, void* v, size_t len) { memcpy(v, b + at, len); }

void orc_get_checkpoint(const orc* o, uint8_t* b) {
  int32_t n = o->n, R = o->R;
  memset(b, 0, 640);
  memcpy(b, "PAMCCKP1", 8);
  uint32_t u32[4] = {1u, (uint32_t)ckp_kind(o), 0u, 0u};
  wr(b, 8, u32, 8);
  wr(b, 16, &n, 4);
  wr(b, 20, &R, 4);
  wr(b, 24, &o->seed, 8);
  uint32_t ctr[4] = {o->gs, o->g_rs, o->g_cl, 0u};
  wr(b, 32, ctr, 16);
  wr(b, 48, &o->mstar, 8);
  wr(b, 56, &o->ctrl.beta, 8);
  wr(b, 64, &o->ctrl.delta, 8);
  int32_t f[12] = {o->ctrl.z, o->ctrl.cycle, o->ctrl.cooldown, o->ctrl.enable ? 1 : 0, o->ctrl.hist_len,
                   o->run.steps_run, o->run.step_reached, o->run.n_cluster_moves, o->run.n_reheats,
                   o->run.n_reversals, o->run.n_restarts, 0};
  wr(b, 72, f, sizeof f);
  wr(b, 120, &o->run.sum_lnq, 8);
  for (int32_t i = 0; i < o->ctrl.hist_len && i < 64; ++i) wr(b, 128 + 8 * (size_t)i, &o->ctrl.hist[i], 8);
  size_t at = 640;
  for (int32_t r = 0; r < R; ++r)
    for (int32_t v = 0; v < n; ++v) b[at + (size_t)r * n + v] = (uint8_t)o->s[(size_t)r * n + o->to_internal[v]];
  at += (size_t)R * n;
  wr(b, at, o->family, 4 * (size_t)R);
  at += 4 * (size_t)R;
  for (int32_t v = 0; v < n; ++v) b[at + v] = (uint8_t)o->best[o->to_internal[v]];
}

int32_t orc_set_checkpoint(orc* o, const uint8_t* b, int64_t bytes) {
  int32_t n = o->n, R = o->R;
  if (bytes < orc_checkpoint_size(o) || memcmp(b, "PAMCCKP1", 8) != 0) return -1;
  uint32_t ver, kind;
  int32_t cn, cR;
  rd(b, 8, &ver, 4);
  rd(b, 12, &kind, 4);
  rd(b, 16, &cn, 4);
  rd(b, 20, &cR, 4);
  if (ver != 1u || kind != (uint32_t)ckp_kind(o) || cn != n || cR != R) return -1;
  int32_t f[12];
  rd(b, 72, f, sizeof f);
  if (f[4] < 0 || f[4] > 64) return -1;
  const int8_t* spins = (const int8_t*)b + 640;
  int32_t* fam = (int32_t*)malloc(sizeof(int32_t) * (size_t)R);
  rd(b, 640 + (size_t)R * n, fam, 4 * (size_t)R);
  if (orc_set_population(o, spins, fam) != 0) { free(fam); return -1; }
  free(fam);
  const int8_t* best = spins + (size_t)R * n + 4 * (size_t)R;
  for (int32_t v = 0; v < n; ++v) o->best[o->to_internal[v]] = best[v];
  rd(b, 24, &o->seed, 8);
  uint32_t ctr[3];
  rd(b, 32, ctr, 12);
  o->gs = ctr[0];
  o->g_rs = ctr[1];
  o->g_cl = ctr[2];
  rd(b, 48, &o->mstar, 8);
  memset(&o->ctrl, 0, sizeof o->ctrl);
  rd(b, 56, &o->ctrl.beta, 8);
  rd(b, 64, &o->ctrl.delta, 8);
  o->ctrl.z = f[0];
  o->ctrl.cycle = f[1];
  o->ctrl.cooldown = f[2];
  o->ctrl.enable = f[3];
  o->ctrl.hist_len = f[4];
  for (int32_t i = 0; i < f[4]; ++i) rd(b, 128 + 8 * (size_t)i, &o->ctrl.hist[i], 8);
  memset(&o->run, 0, sizeof o->run);
  o->run.steps_run = f[5];
  o->run.step_reached = f[6];
  o->run.n_cluster_moves = f[7];
  o->run.n_reheats = f[8];
  o->run.n_reversals = f[9];
  o->run.n_restarts = f[10];
  rd(b, 120, &o->run.sum_lnq, 8);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Max-3-Cut decode: undo the global-flip gauge with the ancilla, then the   */
/* label of vertex i is the a with x_{i,a} = +1 (the lowest such a if more   */
/* than one, 0 if none).                                                     */
/* ------------------------------------------------------------------------ */
int64_t orc_max3cut_value(const orc* o, const int32_t* labels) {
  int64_t cut = 0;
  for (int32_t i = 0; i < o->m3_n; ++i)
    for (int32_t e = o->m3_row_ptr[i]; e < o->m3_row_ptr[i + 1]; ++e) {
      int32_t j = o->m3_col[e];
      if (j > i && labels[i] != labels[j]) cut += o->m3_w[e];
    }
  return cut;
}

int64_t orc_max3cut_decode(const orc* o, const int8_t* spins, int32_t* labels) {
  int32_t n = o->m3_n;
  int g = spins[3 * n] < 0 ? -1 : 1;
  for (int32_t i = 0; i < n; ++i) {
    int32_t lab = 0;
    for (int32_t a = 2; a >= 0; --a)
      if (g * spins[3 * i + a] > 0) lab = a;
    labels[i] = lab;
  }
  return orc_max3cut_value(o, labels);
}

/* Mean normalised pairwise Hamming distance with d_H = min(d, 1 - d)
 * (Supplement, Hamming distance). */
double orc_mean_pair_distance(const orc* o) {
  int32_t R = o->R, n = o->n;
  if (R < 2) return 0.0;
  double acc = 0.0;
  for (int32_t a = 0; a < R; ++a)
    for (int32_t b = a + 1; b < R; ++b) {
      int32_t dd = 0;
      for (int32_t v = 0; v < n; ++v) dd += o->s[(size_t)a * n + v] != o->s[(size_t)b * n + v];
      double d = (double)dd / n;
      acc += d < 1.0 - d ? d : 1.0 - d;
    }
  return acc / ((double)R * (R - 1) / 2.0);
}

int32_t orc_set_population(orc* o, const int8_t* spins, const int32_t* family) {
  int32_t n = o->n;
  for (size_t k = 0; k < (size_t)o->R * n; ++k) {
    int8_t x = spins[k];
    if (o->potts_K ? (x < 0 || x >= o->potts_K) : (x != 1 && x != -1)) return -1;
  }
  for (int32_t r = 0; r < o->R; ++r) {
    for (int32_t v = 0; v < n; ++v)
      o->s[(size_t)r * n + o->to_internal[v]] = spins[(size_t)r * n + v];
    if (family) o->family[r] = family[r];
    if (o->potts_K) {
      o->E[r] = orc_potts_energy(o, r);
      continue;
    }
    const int8_t* s = o->s + (size_t)r * n;
    int32_t* h = o->h + (size_t)r * n;
    int64_t twoE = 0;
    for (int32_t v = 0; v < n; ++v) {
      int64_t acc = 0;
      for (int32_t e = o->row_ptr[v]; e < o->row_ptr[v + 1]; ++e) acc += (int64_t)o->J[e] * s[o->col[e]];
      h[v] = (int32_t)acc;
      twoE += (int64_t)s[v] * acc;
    }
    o->E[r] = -twoE / 2;
  }
  return 0;
}

void orc_set_counters(orc* o, const uint32_t* c3) {
  o->gs = c3[0];
  o->g_rs = c3[1];
  o->g_cl = c3[2];
}

void orc_pair_distances(const orc* o, double* out) {
  int32_t R = o->R, n = o->n;
  size_t k = 0;
  for (int32_t a = 0; a < R; ++a)
    for (int32_t b = a + 1; b < R; ++b) {
      int32_t dd = 0;
      for (int32_t v = 0; v < n; ++v) dd += o->s[(size_t)a * n + v] != o->s[(size_t)b * n + v];
      double d = (double)dd / n;
      out[k++] = d < 1.0 - d ? d : 1.0 - d;
    }
}
