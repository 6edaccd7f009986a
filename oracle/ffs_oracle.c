/*
 * CPU oracle for the EDFFS hybrid parallel GA (arXiv 1903.10741).
 *
 * TEST INFRASTRUCTURE ONLY: see ffs_oracle.h. Everything here is written for
 * a reader checking it against the paper, not for speed: each step is the
 * plain statement of the rule it cites, in the order the paper gives it.
 *
 * Readings where the paper is silent, garbled or lost (its figures 2, 5, 9,
 * 10, 13 are not available) are marked "Reading:" at the point of use.
 */
#include "ffs_oracle.h"

#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAX32(a, b) ((a) > (b) ? (a) : (b))

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2, 3", */
/* SC'11): 10 rounds of two 64x64->128 multiplies; the key is bumped by the    */
/* two Weyl constants between rounds.                                          */
/* ------------------------------------------------------------------------ */
static void mul_hi_lo(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t hi0, lo0, hi1, lo1;
    mul_hi_lo(M0, x0, &hi0, &lo0);
    mul_hi_lo(M1, x2, &hi1, &lo1);
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Reading: the paper does not name its generator. Draws are keyed by
 * (seed, shop) and counted by (individual, generation, event,
 * purpose * 2^32 + block). Purposes: 0 init, 1 crossover, 2 mutation. */
static void rng_block(uint64_t seed, uint64_t shop, uint64_t idx, uint64_t gen,
                      uint64_t event, uint64_t purpose, uint64_t block, uint64_t out[4]) {
  uint64_t ctr[4] = {idx, gen, event, (purpose << 32) | block};
  uint64_t key[2] = {seed, shop};
  orc_philox4x64_10(ctr, key, out);
}

/* floor(hi32(w) * n / 2^32): an integer in [0, n). */
static uint32_t draw_below(uint64_t w, uint32_t n) {
  return (uint32_t)(((w >> 32) * (uint64_t)n) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Instance checks                                                           */
/* ------------------------------------------------------------------------ */
#define P_AT(in, j, s, m) ((in)->proc[((int64_t)(j) * (in)->n_stages + (s)) * (in)->o_max + (m)])
#define Q_AT(in, j, s, m) ((in)->power[((int64_t)(j) * (in)->n_stages + (s)) * (in)->o_max + (m)])

static int check_instance(const orc_instance *in) {
  if (in->n_stages < 1 || in->o_max < 1 || in->n_jobs < 0 || in->n_active < 0 ||
      in->n_active > in->n_jobs || in->n_running < 0 || in->q_max < 1 || in->n_fixed < 0 ||
      (in->n_fixed > 0 && !in->fixed))
    return ORC_E_INVAL;
  for (int r = 0; r < in->n_fixed; ++r) {
    const int32_t st = in->fixed[3 * r], end = in->fixed[3 * r + 1], q = in->fixed[3 * r + 2];
    if (st < in->rs || end <= st || q < 1) return ORC_E_INVAL;
    if (q > in->q_max) return ORC_E_INFEASIBLE;
  }
  for (int s = 0; s < in->n_stages; ++s)
    if (in->n_machines[s] < 1 || in->n_machines[s] > in->o_max) return ORC_E_INVAL;
  for (int k = 0; k < in->n_active; ++k) {
    int j = in->active[k];
    if (j < 0 || j >= in->n_jobs) return ORC_E_INVAL;
    int f = in->first_stage[j];
    if (f < 0 || f >= in->n_stages) return ORC_E_INVAL;
    for (int s = f; s < in->n_stages; ++s)
      for (int m = 0; m < in->n_machines[s]; ++m) {
        if (P_AT(in, j, s, m) < 1 || Q_AT(in, j, s, m) < 1) return ORC_E_INVAL;
        /* A placement needs Q_jsm <= Q_max, eq. (7); otherwise the push-right
         * of the decoding rule never ends. */
        if (Q_AT(in, j, s, m) > in->q_max) return ORC_E_INFEASIBLE;
      }
  }
  /* Every job with first_stage < g must be in the active list exactly once. */
  int n_unfrozen = 0;
  for (int j = 0; j < in->n_jobs; ++j)
    if (in->first_stage[j] < in->n_stages) ++n_unfrozen;
  if (n_unfrozen != in->n_active) return ORC_E_INVAL;
  return ORC_OK;
}

/* Latest completion any decode can reach, in slots after RS. Every start is
 * at most max(earliest start, machine free time, end of the latest placed op)
 * because past the latest placed op only the running ops (all ending by
 * `base`) use power; so every end is at most base + the sum of the longest
 * processing time of every op placed so far. */
int64_t orc_horizon_bound(const orc_instance *in) {
  int64_t base = in->rs;
  for (int k = 0; k < in->n_active; ++k) base = MAX32(base, (int64_t)in->ready[in->active[k]]);
  for (int s = 0; s < in->n_stages; ++s)
    for (int m = 0; m < in->n_machines[s]; ++m)
      base = MAX32(base, (int64_t)in->machine_free[s * in->o_max + m]);
  for (int r = 0; r < in->n_running; ++r) base = MAX32(base, (int64_t)in->running[2 * r]);
  for (int r = 0; r < in->n_fixed; ++r) base = MAX32(base, (int64_t)in->fixed[3 * r + 1]);
  int64_t sum = 0;
  for (int k = 0; k < in->n_active; ++k) {
    int j = in->active[k];
    for (int s = in->first_stage[j]; s < in->n_stages; ++s) {
      int32_t pmax = 0;
      for (int m = 0; m < in->n_machines[s]; ++m) pmax = MAX32(pmax, P_AT(in, j, s, m));
      sum += pmax;
    }
  }
  return base - in->rs + sum + 1;
}

/* ------------------------------------------------------------------------ */
/* Decoding (Section 4.3, Algorithm 2, eqs. (4)-(10))                        */
/* ------------------------------------------------------------------------ */
typedef struct {
  const orc_instance *in;
  int64_t horizon;      /* profile slots: index tau <-> time RS + tau */
  int32_t *profile;     /* [horizon] total power in use, eq. (8) */
  int32_t *free_at;     /* [g][o_max] end of the last op placed on each machine */
  int32_t *next_stage;  /* [n_jobs] next stage of each job still to place */
  int32_t *done_at;     /* [n_jobs] completion of the job's last placed stage */
  int64_t work;
} decoder;

static void decoder_free(decoder *d) {
  free(d->profile);
  free(d->free_at);
  free(d->next_stage);
  free(d->done_at);
}

/* The state at RS: frozen running ops hold their power on [RS, end), each
 * machine is busy until its last frozen op ends, each job resumes at its
 * first unfrozen stage no earlier than `ready`. */
static int decoder_init(decoder *d, const orc_instance *in) {
  memset(d, 0, sizeof(*d));
  d->in = in;
  d->horizon = orc_horizon_bound(in);
  d->profile = (int32_t *)calloc((size_t)d->horizon, sizeof(int32_t));
  d->free_at = (int32_t *)malloc(sizeof(int32_t) * (size_t)in->n_stages * in->o_max);
  d->next_stage = (int32_t *)malloc(sizeof(int32_t) * (size_t)(in->n_jobs + 1));
  d->done_at = (int32_t *)malloc(sizeof(int32_t) * (size_t)(in->n_jobs + 1));
  if (!d->profile || !d->free_at || !d->next_stage || !d->done_at) {
    decoder_free(d);
    return ORC_E_NOMEM;
  }
  memcpy(d->free_at, in->machine_free, sizeof(int32_t) * (size_t)in->n_stages * in->o_max);
  for (int j = 0; j < in->n_jobs; ++j) {
    d->next_stage[j] = in->first_stage[j];
    d->done_at[j] = in->ready[j];
  }
  for (int r = 0; r < in->n_running; ++r) {
    int32_t end = in->running[2 * r], q = in->running[2 * r + 1];
    for (int64_t tau = 0; tau < (int64_t)end - in->rs; ++tau) d->profile[tau] += q;
  }
  /* planned ops kept in place (static approach): power on their own window */
  for (int r = 0; r < in->n_fixed; ++r) {
    const int32_t st = in->fixed[3 * r], end = in->fixed[3 * r + 1], q = in->fixed[3 * r + 2];
    for (int64_t tau = (int64_t)st - in->rs; tau < (int64_t)end - in->rs; ++tau)
      d->profile[tau] += q;
  }
  return ORC_OK;
}

/* Push right (Algorithm 2, eqs. (7)-(9)): the earliest t >= t0 such that the
 * power over [t, t+p) plus q stays within Q_max; a window that breaks the
 * limit at tau cannot start at or before tau, so the search jumps past its
 * last breaking slot. */
static int32_t push_right(const decoder *d, int32_t t0, int32_t p, int32_t q) {
  const orc_instance *in = d->in;
  int32_t t = t0;
  for (;;) {
    int64_t last_bad = -1;
    for (int64_t tau = t; tau < (int64_t)t + p; ++tau)
      if (d->profile[tau - in->rs] + q > in->q_max) last_bad = tau;
    if (last_bad < 0) return t;
    t = (int32_t)(last_bad + 1);
  }
}

/* Place op (j, s). machine -1: the machine with the earliest completion time
 * max(est, free) + P, ties to the lowest index (reading: machine first, then
 * time, as X(k) is fixed before Algorithm 2 runs); -2: the machine of earliest
 * completion after its push-right (ORC_RULE_POWER_ECT). The start is the
 * earliest t >= max(RS, previous stage end or release, machine free) such that
 * the power over [t, t+p) plus q stays within Q_max (eqs. (7)-(9), half-open
 * per eq. (9)). Machines are append-only: an op goes after every op placed on
 * that machine before it. */
static int place_op(decoder *d, int32_t j, int32_t s, int32_t machine,
                    int32_t *start_out, int32_t *mach_out) {
  const orc_instance *in = d->in;
  if (j < 0 || j >= in->n_jobs || s < 0 || s >= in->n_stages) return ORC_E_INVAL;
  if (d->next_stage[j] != s) return ORC_E_INVAL;  /* route order, eqs. (4)-(5) */
  const int32_t o_s = in->n_machines[s];
  int32_t *free_s = d->free_at + (int64_t)s * in->o_max;
  const int32_t est = MAX32(in->rs, d->done_at[j]);  /* eqs. (4), (5), (10) */

  int32_t m = machine;
  if (m == -1) {
    int32_t best_end = 0;
    m = -1;
    for (int32_t c = 0; c < o_s; ++c) {
      int32_t end = MAX32(est, free_s[c]) + P_AT(in, j, s, c);
      d->work += 3;
      if (m < 0 || end < best_end) {
        best_end = end;
        m = c;
      }
    }
  }
  if (m == -2) {
    /* power-aware: the earliest completion after each machine's push-right, ties
     * to the lowest index. A push-right only delays, so max(est, free) + P
     * bounds a machine's completion from below: the machine of least bound
     * (ties to the lowest index) is pushed right first, then, in index order,
     * only the machines whose (bound, index) is below the best (completion,
     * index) found so far; the others cannot win. Work: 3 per machine for its
     * bound, plus the examined slots and p of every machine pushed right. */
    int32_t first = -1, first_lb = 0;
    for (int32_t c = 0; c < o_s; ++c) {
      if (Q_AT(in, j, s, c) > in->q_max) return ORC_E_INFEASIBLE;
      const int32_t lb = MAX32(est, free_s[c]) + P_AT(in, j, s, c);
      d->work += 3;
      if (first < 0 || lb < first_lb) {
        first = c;
        first_lb = lb;
      }
    }
    int32_t best_end = 0;
    m = -1;
    for (int32_t k = -1; k < o_s; ++k) {
      const int32_t c = k < 0 ? first : k;
      if (k >= 0 && c == first) continue;
      const int32_t t0c = MAX32(est, free_s[c]), pc = P_AT(in, j, s, c);
      if (m >= 0 && !(t0c + pc < best_end || (t0c + pc == best_end && c < m))) continue;
      const int32_t tc = push_right(d, t0c, pc, Q_AT(in, j, s, c));
      d->work += (int64_t)(tc - t0c) + pc;
      if (m < 0 || tc + pc < best_end || (tc + pc == best_end && c < m)) {
        best_end = tc + pc;
        m = c;
      }
    }
  }
  if (m < 0 || m >= o_s) return ORC_E_INVAL;
  const int32_t p = P_AT(in, j, s, m), q = Q_AT(in, j, s, m);
  if (q > in->q_max) return ORC_E_INFEASIBLE;

  const int32_t t0 = MAX32(est, free_s[m]);  /* eq. (6): after the machine's last op */
  const int32_t t = push_right(d, t0, p, q);
  if ((int64_t)t - in->rs + p > d->horizon) abort(); /* horizon bound broken */
  for (int64_t tau = t; tau < (int64_t)t + p; ++tau) d->profile[tau - in->rs] += q;
  /* every slot of [t0, t+p) needs examining once, then p slots are updated (the
   * power-aware choice has counted its examinations already) */
  d->work += machine == -2 ? (int64_t)p : (int64_t)(t - t0) + 2 * (int64_t)p;

  free_s[m] = t + p;
  d->done_at[j] = t + p;
  d->next_stage[j] = s + 1;
  if (start_out) start_out[(int64_t)j * in->n_stages + s] = t;
  if (mach_out) mach_out[(int64_t)j * in->n_stages + s] = m;
  return ORC_OK;
}

/* Objective eq. (1) with eqs. (2)-(3), summed over every job in J u J'. Jobs
 * frozen entirely contribute through frozen_tardiness / frozen_cmax. */
static int64_t objective(const decoder *d) {
  const orc_instance *in = d->in;
  int64_t tardiness = in->frozen_tardiness;
  int32_t cmax = in->frozen_cmax;
  for (int k = 0; k < in->n_active; ++k) {
    int j = in->active[k];
    int32_t c = d->done_at[j];
    int32_t late = c - in->due[j];
    tardiness += late > 0 ? late : 0;
    cmax = MAX32(cmax, c);
  }
  return (int64_t)in->wt * tardiness + cmax;
}

int orc_decode(const orc_instance *in, const int32_t *prio, int64_t *obj,
               int32_t *start, int32_t *mach, int64_t *work) {
  int rc = check_instance(in);
  if (rc) return rc;
  const int32_t n = in->n_active;
  /* Reading: the chromosome is one priority per job, larger = higher
   * (Section 4.3); the op order is stage-major, the same job order at every
   * stage. order[n - prio_k] = active[k] lists jobs by decreasing priority. */
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  if (!order) return ORC_E_NOMEM;
  for (int k = 0; k < n; ++k) order[k] = -1;
  for (int k = 0; k < n; ++k) {
    int32_t pk = prio[k];
    if (pk < 1 || pk > n || order[n - pk] >= 0) {
      free(order);
      return ORC_E_INVAL;
    }
    order[n - pk] = in->active[k];
  }
  decoder d;
  rc = decoder_init(&d, in);
  if (rc) {
    free(order);
    return rc;
  }
  const int32_t rule_m = (in->decode_rules & ORC_RULE_POWER_ECT) ? -2 : -1;
  int32_t *stage = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
  for (int s = 0; s < in->n_stages && rc == ORC_OK; ++s) {
    /* the jobs reaching stage s, in priority order ... */
    int32_t cnt = 0;
    for (int k = 0; k < n; ++k)
      if (in->first_stage[order[k]] <= s) stage[cnt++] = order[k];
    /* ... or (FIFO) by when their previous stage ended, ties kept in priority
     * order (a stable insertion sort) */
    if (in->decode_rules & ORC_RULE_FIFO)
      for (int a = 1; a < cnt; ++a) {
        const int32_t j = stage[a];
        int b = a - 1;
        while (b >= 0 && d.done_at[stage[b]] > d.done_at[j]) {
          stage[b + 1] = stage[b];
          --b;
        }
        stage[b + 1] = j;
      }
    for (int k = 0; k < cnt && rc == ORC_OK; ++k) rc = place_op(&d, stage[k], s, rule_m, start, mach);
  }
  free(stage);
  if (rc == ORC_OK) {
    *obj = objective(&d);
    if (work) *work = d.work;
  }
  decoder_free(&d);
  free(order);
  return rc;
}

int orc_decode_pop(const orc_instance *in, const int32_t *prio, int32_t pop,
                   int64_t *obj, int64_t *work, int32_t n_threads) {
  int rc = check_instance(in);
  if (rc) return rc;
  int bad = 0;
  const int64_t n = in->n_active;
#pragma omp parallel for schedule(dynamic, 8) num_threads(n_threads > 0 ? n_threads : 1) reduction(| : bad)
  for (int32_t i = 0; i < pop; ++i) {
    int r = orc_decode(in, prio + (int64_t)i * n, &obj[i], NULL, NULL, work ? &work[i] : NULL);
    if (r) bad |= 1;
  }
  return bad ? ORC_E_INVAL : ORC_OK;
}

int orc_decode_ops(const orc_instance *in, int32_t n_ops, const int32_t *ops,
                   int64_t *obj, int32_t *start, int32_t *mach) {
  int rc = check_instance(in);
  if (rc) return rc;
  decoder d;
  rc = decoder_init(&d, in);
  if (rc) return rc;
  for (int i = 0; i < n_ops && rc == ORC_OK; ++i)
    rc = place_op(&d, ops[3 * i], ops[3 * i + 1], ops[3 * i + 2], start, mach);
  if (rc == ORC_OK) {
    int complete = 1;
    for (int k = 0; k < in->n_active; ++k)
      if (d.next_stage[in->active[k]] != in->n_stages) complete = 0;
    *obj = complete ? objective(&d) : -1;
  }
  decoder_free(&d);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* The X/Y chromosome (Section 4.3, eqs. (10)-(12), Algorithms 1 and 2)      */
/* ------------------------------------------------------------------------ */
int32_t orc_xy_ops(const orc_instance *in) {
  int32_t R = 0;
  for (int x = 0; x < in->n_active; ++x) R += in->n_stages - in->first_stage[in->active[x]];
  return R;
}

/* Op of gene k: the active jobs in turn, each with its unfrozen stages. */
static void xy_gene_op(const orc_instance *in, int32_t k, int32_t *job, int32_t *stage) {
  for (int x = 0; x < in->n_active; ++x) {
    const int32_t j = in->active[x], len = in->n_stages - in->first_stage[j];
    if (k < len) {
      *job = j;
      *stage = in->first_stage[j] + k;
      return;
    }
    k -= len;
  }
  *job = -1;
  *stage = -1;
}

/* Gene of op (j, s): the genes of the active jobs before j, then s's place. */
static int32_t xy_op_gene(const orc_instance *in, int32_t j, int32_t s) {
  int32_t k = 0;
  for (int x = 0; x < in->n_active && in->active[x] != j; ++x)
    k += in->n_stages - in->first_stage[in->active[x]];
  return k + s - in->first_stage[j];
}

int orc_xy_order(const orc_instance *in, const int32_t *y, int32_t *order) {
  const int32_t R = orc_xy_ops(in), n = in->n_active;
  /* y is a permutation of 1..R, unique priorities (eq. (11)) */
  uint8_t *seen = (uint8_t *)calloc((size_t)R + 1, 1);
  int32_t *placed = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  if (!seen || !placed) {
    free(seen);
    free(placed);
    return ORC_E_NOMEM;
  }
  for (int k = 0; k < R; ++k) {
    if (y[k] < 1 || y[k] > R || seen[y[k]]) {
      free(seen);
      free(placed);
      return ORC_E_INVAL;
    }
    seen[y[k]] = 1;
  }
  /* Algorithm 1, greedy reading: the next op in Z is the one of largest y
   * among each job's first op not yet ordered (its earlier stages are
   * ordered or frozen, so the route order of eqs. (4)-(5) holds). */
  for (int32_t z = 0; z < R; ++z) {
    int32_t best = -1, best_y = 0, k0 = 0;
    for (int x = 0; x < n; ++x) {
      const int32_t j = in->active[x], len = in->n_stages - in->first_stage[j];
      if (placed[x] < len && y[k0 + placed[x]] > best_y) {
        best_y = y[k0 + placed[x]];
        best = x;
      }
      k0 += len;
    }
    const int32_t j = in->active[best];
    order[2 * z] = j;
    order[2 * z + 1] = in->first_stage[j] + placed[best];
    ++placed[best];
  }
  free(seen);
  free(placed);
  return ORC_OK;
}

int orc_decode_xy(const orc_instance *in, const int32_t *genes, int64_t *obj,
                  int32_t *start, int32_t *mach, int64_t *work) {
  int rc = check_instance(in);
  if (rc) return rc;
  const int32_t R = orc_xy_ops(in);
  const int32_t *xg = genes, *yg = genes + R;
  for (int32_t k = 0; k < R; ++k) {  /* x_k is a machine of its op's stage (eq. (10)) */
    int32_t j, s;
    xy_gene_op(in, k, &j, &s);
    if (xg[k] < 0 || xg[k] >= in->n_machines[s]) return ORC_E_INVAL;
  }
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * 2 * ((size_t)R + 1));
  if (!order) return ORC_E_NOMEM;
  if ((rc = orc_xy_order(in, yg, order))) {
    free(order);
    return rc;
  }
  decoder d;
  if ((rc = decoder_init(&d, in))) {
    free(order);
    return rc;
  }
  /* Algorithm 2 in Z order: each op on its target machine x_js. */
  for (int32_t z = 0; z < R && rc == ORC_OK; ++z) {
    const int32_t j = order[2 * z], s = order[2 * z + 1];
    rc = place_op(&d, j, s, xg[xy_op_gene(in, j, s)], start, mach);
  }
  if (rc == ORC_OK) {
    *obj = objective(&d);
    if (work) *work = d.work;
  }
  decoder_free(&d);
  free(order);
  return rc;
}

int orc_decode_xy_pop(const orc_instance *in, const int32_t *genes, int32_t pop,
                      int64_t *obj, int64_t *work, int32_t n_threads) {
  int rc = check_instance(in);
  if (rc) return rc;
  int bad = 0;
  const int64_t L = 2 * (int64_t)orc_xy_ops(in);
#pragma omp parallel for schedule(dynamic, 8) num_threads(n_threads > 0 ? n_threads : 1) reduction(| : bad)
  for (int32_t i = 0; i < pop; ++i) {
    int r = orc_decode_xy(in, genes + (int64_t)i * L, &obj[i], NULL, NULL, work ? &work[i] : NULL);
    if (r) bad |= 1;
  }
  return bad ? ORC_E_INVAL : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* GA operators (Section 4.4)                                                */
/* ------------------------------------------------------------------------ */

/* Single-point crossover: child_a = a[0:cut] ++ b[cut:], child_b the mirror,
 * each then corrected (Fig. 11). */
void orc_crossover(int32_t n, const int32_t *a, const int32_t *b, int32_t cut,
                   int32_t *child_a, int32_t *child_b) {
  for (int k = 0; k < n; ++k) {
    child_a[k] = k < cut ? a[k] : b[k];
    child_b[k] = k < cut ? b[k] : a[k];
  }
  orc_correct(n, child_a);
  orc_correct(n, child_b);
}

/* X/Y crossover (Section 4.4, Fig. 11): the single-point crossover on both
 * matrices, at the same row-major point (the figure's children are both
 * matrices cut after their second entry); the Y children are then corrected
 * like a priority vector. */
void orc_crossover_xy(int32_t R, const int32_t *a, const int32_t *b, int32_t cut,
                      int32_t *child_a, int32_t *child_b) {
  for (int k = 0; k < R; ++k) {
    child_a[k] = k < cut ? a[k] : b[k];
    child_b[k] = k < cut ? b[k] : a[k];
    child_a[R + k] = k < cut ? a[R + k] : b[R + k];
    child_b[R + k] = k < cut ? b[R + k] : a[R + k];
  }
  orc_correct(R, child_a + R);
  orc_correct(R, child_b + R);
}

/* Priority correction (Section 4.4, Fig. 11): scanning left to right, the
 * first occurrence of a value stays; every later duplicate receives the
 * values missing from 1..n, smallest first. */
void orc_correct(int32_t n, int32_t *v) {
  uint8_t *seen = (uint8_t *)calloc((size_t)n + 2, 1);
  uint8_t *dup = (uint8_t *)calloc((size_t)n + 1, 1);
  for (int k = 0; k < n; ++k) {
    if (v[k] >= 1 && v[k] <= n && !seen[v[k]]) seen[v[k]] = 1;
    else dup[k] = 1;
  }
  int32_t missing = 1;
  for (int k = 0; k < n; ++k) {
    if (!dup[k]) continue;
    while (missing <= n && seen[missing]) ++missing;
    v[k] = missing;
    seen[missing] = 1;
  }
  free(seen);
  free(dup);
}

/* Swap mutation (Section 4.4, Fig. 12): two distinct positions, the first
 * uniform over n, the second uniform over the other n-1, exchange values. */
void orc_mutate(int32_t n, int32_t *v, uint64_t w1, uint64_t w2) {
  int32_t x = (int32_t)draw_below(w1, (uint32_t)n);
  int32_t y = (int32_t)draw_below(w2, (uint32_t)(n - 1));
  if (y >= x) ++y;
  int32_t tmp = v[x];
  v[x] = v[y];
  v[y] = tmp;
}

static int check_ga(const orc_instance *in, const orc_ga_params *gp) {
  if (gp->islands < 1 || gp->rows < 1 || gp->cols < 1) return ORC_E_INVAL;
  if (gp->mig_k < 0 || gp->mig_k > gp->rows * gp->cols || gp->mig_interval < 0) return ORC_E_INVAL;
  if (gp->encoding != 0 && gp->encoding != 1) return ORC_E_INVAL;
  (void)in;
  return ORC_OK;
}

/* Genes per chromosome: one priority per active job, or X and Y (2R). */
static int64_t chrom_len(const orc_instance *in, const orc_ga_params *gp) {
  return gp->encoding == 1 ? 2 * (int64_t)orc_xy_ops(in) : in->n_active;
}

static int decode_chrom(const orc_instance *in, const orc_ga_params *gp, const int32_t *v,
                        int64_t *obj) {
  return gp->encoding == 1 ? orc_decode_xy(in, v, obj, NULL, NULL, NULL)
                           : orc_decode(in, v, obj, NULL, NULL, NULL);
}

/* Random unique priorities 1..n (Section 4.3): Fisher-Yates, the d-th draw
 * taken from word d % 4 of block d / 4 of purpose 0. */
static void fisher_yates(int32_t *v, int32_t n, uint64_t seed, uint64_t shop, int32_t i,
                         int32_t event) {
  for (int k = 0; k < n; ++k) v[k] = k + 1;
  uint64_t w[4] = {0, 0, 0, 0};
  for (int32_t pos = n - 1; pos >= 1; --pos) {
    int32_t d = n - 1 - pos;
    if (d % 4 == 0) rng_block(seed, shop, (uint64_t)i, 0, (uint64_t)event, 0, (uint64_t)(d / 4), w);
    int32_t r = (int32_t)draw_below(w[d % 4], (uint32_t)(pos + 1));
    int32_t tmp = v[pos];
    v[pos] = v[r];
    v[r] = tmp;
  }
}

int orc_ga_init(const orc_instance *in, const orc_ga_params *gp, uint64_t seed,
                uint64_t shop, int32_t event, int32_t *prio, int64_t *obj,
                int32_t *elite, int64_t *elite_obj, int32_t n_threads) {
  int rc = check_instance(in);
  if (rc) return rc;
  if ((rc = check_ga(in, gp))) return rc;
  const int64_t n = chrom_len(in, gp);
  const int32_t K = gp->rows * gp->cols, pop = gp->islands * K;
  for (int32_t i = 0; i < pop; ++i) {
    int32_t *v = prio + (int64_t)i * n;
    if (gp->encoding == 0) {
      fisher_yates(v, in->n_active, seed, shop, i, event);
      continue;
    }
    /* X/Y (Section 4.3): each x a uniform machine of its stage, the k-th draw
     * from word k % 4 of block k / 4 of purpose 4 (reading: the paper says
     * only "a random integer"); y unique in 1..R by Fisher-Yates as above. */
    const int32_t R = (int32_t)(n / 2);
    uint64_t w[4] = {0, 0, 0, 0};
    for (int32_t k = 0; k < R; ++k) {
      int32_t j, st;
      xy_gene_op(in, k, &j, &st);
      if (k % 4 == 0) rng_block(seed, shop, (uint64_t)i, 0, (uint64_t)event, 4, (uint64_t)(k / 4), w);
      v[k] = (int32_t)draw_below(w[k % 4], (uint32_t)in->n_machines[st]);
    }
    fisher_yates(v + R, R, seed, shop, i, event);
  }
  rc = gp->encoding == 1 ? orc_decode_xy_pop(in, prio, pop, obj, NULL, n_threads)
                         : orc_decode_pop(in, prio, pop, obj, NULL, n_threads);
  if (rc) return rc;
  for (int32_t I = 0; I < gp->islands; ++I) {
    int32_t b = I * K;
    for (int32_t i = I * K; i < (I + 1) * K; ++i)
      if (obj[i] < obj[b]) b = i;
    memcpy(elite + (int64_t)I * n, prio + (int64_t)b * n, sizeof(int32_t) * (size_t)n);
    elite_obj[I] = obj[b];
  }
  return ORC_OK;
}

/* Selection (Section 4.4, Fig. 9 lost): the neighbourhood is the slot and its
 * four torus neighbours within the island; the lowest objective wins.
 * Reading: candidate order self, up, down, left, right; ties go to the first. */
static int32_t select_winner(const orc_ga_params *gp, const int64_t *obj, int32_t i) {
  const int32_t K = gp->rows * gp->cols, R = gp->rows, C = gp->cols;
  const int32_t base = (i / K) * K, r = (i % K) / C, c = (i % K) % C;
  int32_t cand[5] = {
      base + r * C + c,
      base + ((r - 1 + R) % R) * C + c,
      base + ((r + 1) % R) * C + c,
      base + r * C + (c - 1 + C) % C,
      base + r * C + (c + 1) % C,
  };
  int32_t w = cand[0];
  for (int k = 1; k < 5; ++k)
    if (obj[cand[k]] < obj[w]) w = cand[k];
  return w;
}

/* Islands whose children must be built: the selected ones, plus their ring
 * predecessors when generation gen migrates. Caller frees. */
static uint8_t *needed_islands(const orc_ga_params *gp, int32_t gen, const uint8_t *island_sel) {
  const int32_t I_n = gp->islands;
  const int migrate = gp->mig_interval > 0 && gp->mig_k > 0 && I_n > 1 && gen % gp->mig_interval == 0;
  uint8_t *need = (uint8_t *)calloc((size_t)I_n, 1);
  for (int32_t I = 0; I < I_n; ++I)
    if (!island_sel || island_sel[I]) {
      need[I] = 1;
      if (migrate) need[(I - 1 + I_n) % I_n] = 1;
    }
  return need;
}

int orc_ga_breed(const orc_instance *in, const orc_ga_params *gp,
                 uint64_t seed, uint64_t shop, int32_t event, int32_t gen, int32_t variant,
                 const int32_t *prio_in, const int64_t *obj_in, int32_t *prio_out,
                 const uint8_t *island_sel) {
  int rc = check_instance(in);
  if (rc) return rc;
  if ((rc = check_ga(in, gp))) return rc;
  if (gen < 1 || variant < 0) return ORC_E_INVAL;
  const int64_t n = chrom_len(in, gp);
  const int32_t R = gp->rows, C = gp->cols, K = R * C;
  const int32_t I_n = gp->islands;
  const int xy = gp->encoding == 1;
  const int32_t n_genes = xy ? (int32_t)(n / 2) : (int32_t)n;  /* genes per matrix */
  uint8_t *need = needed_islands(gp, gen, island_sel);

  for (int32_t I = 0; I < I_n; ++I) {
    if (!need[I]) continue;
    /* 1. Selection, from the previous generation's objectives. */
    for (int32_t i = I * K; i < (I + 1) * K; ++i) {
      int32_t w = select_winner(gp, obj_in, i);
      memcpy(prio_out + (int64_t)i * n, prio_in + (int64_t)w * n, sizeof(int32_t) * (size_t)n);
    }
    /* 2. Crossover of neighbour pairs (Fig. 10 lost). Reading: pairs are
     * horizontal ((r,2c),(r,2c+1)) on odd generations and vertical
     * ((2r,c),(2r+1,c)) on even ones; the lower slot draws the decision and
     * the cut 1 + floor(hi32 * (n-1) / 2^32) (X/Y: one cut for both matrices,
     * n = R). Variant v of the breeding
     * (the screened generation's v-th candidate) draws from block v. */
    if (n_genes >= 2) {
      int32_t *ta = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
      int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
      const int horizontal = gen % 2 == 1;
      const int32_t n_pairs = horizontal ? R * (C / 2) : (R / 2) * C;
      for (int32_t pr = 0; pr < n_pairs; ++pr) {
        int32_t a, b;
        if (horizontal) {
          int32_t r = pr / (C / 2), c2 = pr % (C / 2);
          a = I * K + r * C + 2 * c2;
          b = a + 1;
        } else {
          int32_t r2 = pr / C, c = pr % C;
          a = I * K + (2 * r2) * C + c;
          b = a + C;
        }
        uint64_t w[4];
        rng_block(seed, shop, (uint64_t)a, (uint64_t)gen, (uint64_t)event, 1, (uint64_t)variant, w);
        if ((uint32_t)(w[0] >> 32) < gp->pc) {
          int32_t cut = 1 + (int32_t)draw_below(w[1], (uint32_t)(n_genes - 1));
          int32_t *pa = prio_out + (int64_t)a * n, *pb = prio_out + (int64_t)b * n;
          if (xy)
            orc_crossover_xy(n_genes, pa, pb, cut, ta, tb);
          else
            orc_crossover((int32_t)n, pa, pb, cut, ta, tb);
          memcpy(pa, ta, sizeof(int32_t) * (size_t)n);
          memcpy(pb, tb, sizeof(int32_t) * (size_t)n);
        }
      }
      free(ta);
      free(tb);
    }
    /* 3. Mutation (Fig. 12): the swap of two priorities (n >= 2); with X/Y
     * every x is also redrawn to another machine of its stage (x + 1 +
     * draw(o_s - 1)) mod o_s, the k-th draw from word k % 4 of block
     * variant * ceil(R / 4) + k / 4 of purpose 5 (reading: the paper says
     * only "random values in the range, apart from the original ones"). */
    for (int32_t i = I * K; i < (I + 1) * K; ++i) {
      uint64_t w[4];
      rng_block(seed, shop, (uint64_t)i, (uint64_t)gen, (uint64_t)event, 2, (uint64_t)variant, w);
      if ((uint32_t)(w[0] >> 32) >= gp->pm) continue;
      int32_t *v = prio_out + (int64_t)i * n;
      if (n_genes >= 2) orc_mutate(n_genes, xy ? v + n_genes : v, w[1], w[2]);
      if (!xy) continue;
      const uint64_t b0 = (uint64_t)variant * (uint64_t)((n_genes + 3) / 4);
      uint64_t wx[4] = {0, 0, 0, 0};
      for (int32_t k = 0; k < n_genes; ++k) {
        int32_t j, st;
        xy_gene_op(in, k, &j, &st);
        if (k % 4 == 0) rng_block(seed, shop, (uint64_t)i, (uint64_t)gen, (uint64_t)event, 5, b0 + (uint64_t)(k / 4), wx);
        const int32_t o = in->n_machines[st];
        if (o > 1) v[k] = (v[k] + 1 + (int32_t)draw_below(wx[k % 4], (uint32_t)(o - 1))) % o;
      }
    }
  }
  free(need);
  return ORC_OK;
}

int orc_ga_generation(const orc_instance *in, const orc_ga_params *gp,
                      uint64_t seed, uint64_t shop, int32_t event, int32_t gen,
                      const int32_t *prio_in, const int64_t *obj_in,
                      const int32_t *elite_in, const int64_t *elite_obj_in,
                      int32_t *prio_out, int64_t *obj_out,
                      int32_t *elite_out, int64_t *elite_obj_out,
                      const uint8_t *island_sel, int32_t n_threads) {
  int rc = orc_ga_breed(in, gp, seed, shop, event, gen, 0, prio_in, obj_in, prio_out, island_sel);
  if (rc) return rc;
  return orc_ga_finish(in, gp, gen, prio_out, obj_out, elite_in, elite_obj_in, elite_out,
                       elite_obj_out, island_sel, n_threads);
}

int orc_ga_finish(const orc_instance *in, const orc_ga_params *gp, int32_t gen,
                  int32_t *prio_out, int64_t *obj_out,
                  const int32_t *elite_in, const int64_t *elite_obj_in,
                  int32_t *elite_out, int64_t *elite_obj_out,
                  const uint8_t *island_sel, int32_t n_threads) {
  int rc = check_instance(in);
  if (rc) return rc;
  if ((rc = check_ga(in, gp))) return rc;
  if (gen < 1) return ORC_E_INVAL;
  const int64_t n = chrom_len(in, gp);
  const int32_t K = gp->rows * gp->cols;
  const int32_t I_n = gp->islands;
  const int migrate = gp->mig_interval > 0 && gp->mig_k > 0 && I_n > 1 && gen % gp->mig_interval == 0;
  uint8_t *need = needed_islands(gp, gen, island_sel);

  /* 4. Decode every child of the needed islands, eq. (1). */
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 8) num_threads(n_threads > 0 ? n_threads : 1) reduction(| : bad)
  for (int32_t i = 0; i < I_n * K; ++i) {
    if (!need[i / K]) continue;
    if (decode_chrom(in, gp, prio_out + (int64_t)i * n, &obj_out[i])) bad |= 1;
  }
  if (bad) {
    free(need);
    return ORC_E_INVAL;
  }

  /* 5. Replacement (Section 4.4): the island's best-in-history (elite) is
   * refreshed by the island's best child, then overwrites the island's
   * worst. Fitness eq. (13) is a decreasing function of the objective, so
   * "largest fitness" is "smallest objective". Ties go to the lowest slot. */
  for (int32_t I = 0; I < I_n; ++I) {
    if (!need[I]) continue;
    int32_t *el = elite_out + (int64_t)I * n;
    memcpy(el, elite_in + (int64_t)I * n, sizeof(int32_t) * (size_t)n);
    elite_obj_out[I] = elite_obj_in[I];
    int32_t b = I * K, w = I * K;
    for (int32_t i = I * K; i < (I + 1) * K; ++i) {
      if (obj_out[i] < obj_out[b]) b = i;
      if (obj_out[i] > obj_out[w]) w = i;
    }
    if (obj_out[b] < elite_obj_out[I]) {
      memcpy(el, prio_out + (int64_t)b * n, sizeof(int32_t) * (size_t)n);
      elite_obj_out[I] = obj_out[b];
    }
    memcpy(prio_out + (int64_t)w * n, el, sizeof(int32_t) * (size_t)n);
    obj_out[w] = elite_obj_out[I];
  }

  /* 6. Ring migration every mig_interval generations (Section 4.4, Fig. 13
   * lost): island I's mig_k worst slots take island I-1's mig_k best, from a
   * snapshot taken before any island is overwritten. Reading: best sorted by
   * (objective, slot), worst by (objective descending, slot); the elite takes
   * an immigrant that beats it. */
  if (migrate) {
    const int32_t km = gp->mig_k;
    int32_t *imm = (int32_t *)malloc(sizeof(int32_t) * (size_t)I_n * km * (n > 0 ? n : 1));
    int64_t *imm_obj = (int64_t *)malloc(sizeof(int64_t) * (size_t)I_n * km);
    int32_t *worst = (int32_t *)malloc(sizeof(int32_t) * (size_t)km);
    uint8_t *taken = (uint8_t *)malloc((size_t)K);
    /* snapshot: the mig_k best of each sender */
    for (int32_t I = 0; I < I_n; ++I) {
      if (island_sel && !island_sel[I]) continue;
      const int32_t src = (I - 1 + I_n) % I_n;
      memset(taken, 0, (size_t)K);
      for (int32_t r = 0; r < km; ++r) {
        int32_t b = -1;
        for (int32_t i = 0; i < K; ++i)
          if (!taken[i] && (b < 0 || obj_out[src * K + i] < obj_out[src * K + b])) b = i;
        taken[b] = 1;
        memcpy(imm + ((int64_t)I * km + r) * n, prio_out + (int64_t)(src * K + b) * n,
               sizeof(int32_t) * (size_t)n);
        imm_obj[I * km + r] = obj_out[src * K + b];
      }
    }
    /* overwrite: the r-th worst of I takes the r-th best of I-1 */
    for (int32_t I = 0; I < I_n; ++I) {
      if (island_sel && !island_sel[I]) continue;
      memset(taken, 0, (size_t)K);
      for (int32_t r = 0; r < km; ++r) {
        int32_t w = -1;
        for (int32_t i = 0; i < K; ++i)
          if (!taken[i] && (w < 0 || obj_out[I * K + i] > obj_out[I * K + w])) w = i;
        taken[w] = 1;
        worst[r] = w;
      }
      for (int32_t r = 0; r < km; ++r) {
        const int32_t slot = I * K + worst[r];
        memcpy(prio_out + (int64_t)slot * n, imm + ((int64_t)I * km + r) * n, sizeof(int32_t) * (size_t)n);
        obj_out[slot] = imm_obj[I * km + r];
        if (obj_out[slot] < elite_obj_out[I]) {
          memcpy(elite_out + (int64_t)I * n, prio_out + (int64_t)slot * n, sizeof(int32_t) * (size_t)n);
          elite_obj_out[I] = obj_out[slot];
        }
      }
    }
    free(imm);
    free(imm_obj);
    free(worst);
    free(taken);
  }
  free(need);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Predictive-reactive complete rescheduling (Section 4.1, eq. (10))         */
/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* The comparison GAs of Section 5.2 (classical and cellular)                */
/* ------------------------------------------------------------------------ */
int64_t orc_emax(const int64_t *obj, int32_t pop) {
  int64_t e = 10;
  for (;;) {
    int below = 1;
    for (int32_t i = 0; i < pop; ++i)
      if (obj[i] >= e) below = 0;
    if (below || e > INT64_MAX / 10) return e;
    e *= 10;
  }
}

/* Roulette spin: the first i with prefix[i] (inclusive running sum of the
 * fitness, index order) above floor(hi32(w) * total / 2^32). */
static int32_t roulette(const uint64_t *prefix, int32_t pop, uint64_t total, uint64_t w) {
  if (total == 0) return (int32_t)draw_below(w, (uint32_t)pop);
  uint64_t hi, lo;
  mul_hi_lo((w >> 32) << 32, total, &hi, &lo);
  for (int32_t i = 0; i < pop; ++i)
    if (prefix[i] > hi) return i;
  return pop - 1;  /* unreachable: hi < total = prefix[pop - 1] */
}

int orc_ga_generation_scheme(const orc_instance *in, const orc_ga_params *gp, int32_t scheme,
                             int64_t e_max, uint64_t seed, uint64_t shop, int32_t event,
                             int32_t gen, const int32_t *prio_in, const int64_t *obj_in,
                             const int32_t *elite_in, const int64_t *elite_obj_in,
                             int32_t *prio_out, int64_t *obj_out, int32_t *elite_out,
                             int64_t *elite_obj_out, int32_t n_threads) {
  int rc = check_instance(in);
  if (rc) return rc;
  if ((rc = check_ga(in, gp))) return rc;
  if (gen < 1 || gp->islands != 1 || gp->encoding != 0 ||
      (scheme != ORC_GA_CLASSICAL && scheme != ORC_GA_CELLULAR))
    return ORC_E_INVAL;
  const int32_t n = in->n_active, R = gp->rows, C = gp->cols, pop = R * C;
  const size_t row = sizeof(int32_t) * (size_t)(n > 0 ? n : 1);
  int32_t *child = (int32_t *)malloc(row * (size_t)pop);
  int32_t *tb = (int32_t *)malloc(row);
  int64_t *cobj = (int64_t *)malloc(sizeof(int64_t) * (size_t)pop);
  uint64_t *prefix = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)pop);
  int32_t *par = (int32_t *)malloc(sizeof(int32_t) * (size_t)pop);
  if (!child || !tb || !cobj || !prefix || !par) {
    free(child); free(tb); free(cobj); free(prefix); free(par);
    return ORC_E_NOMEM;
  }
  uint64_t w[4];
  if (scheme == ORC_GA_CLASSICAL) {
    /* eq. (13) fitness and its running sums, index order */
    uint64_t total = 0;
    for (int32_t i = 0; i < pop; ++i) {
      const int64_t f = e_max - obj_in[i];
      total += f > 0 ? (uint64_t)f : 0;
      prefix[i] = total;
    }
    for (int32_t i = 0; i < pop; ++i) {
      rng_block(seed, shop, (uint64_t)i, (uint64_t)gen, (uint64_t)event, 6, 0, w);
      par[i] = roulette(prefix, pop, total, w[0]);
      memcpy(child + (int64_t)i * n, prio_in + (int64_t)par[i] * n, row);
    }
    for (int32_t a = 0; a + 1 < pop && n >= 2; a += 2) {
      rng_block(seed, shop, (uint64_t)a, (uint64_t)gen, (uint64_t)event, 1, 0, w);
      if ((uint32_t)(w[0] >> 32) >= gp->pc) continue;
      const int32_t cut = 1 + (int32_t)draw_below(w[1], (uint32_t)(n - 1));
      int32_t *ta = (int32_t *)malloc(row);
      orc_crossover(n, prio_in + (int64_t)par[a] * n, prio_in + (int64_t)par[a + 1] * n, cut, ta, tb);
      memcpy(child + (int64_t)a * n, ta, row);
      memcpy(child + (int64_t)(a + 1) * n, tb, row);
      free(ta);
    }
  } else {
    for (int32_t i = 0; i < pop; ++i) {
      const int32_t r = i / C, c = i % C;
      const int32_t cand[5] = {i, ((r - 1 + R) % R) * C + c, ((r + 1) % R) * C + c,
                               r * C + (c - 1 + C) % C, r * C + (c + 1) % C};
      /* best two entries by (objective, order) */
      int32_t b1 = 0, b2 = -1;
      for (int k = 1; k < 5; ++k)
        if (obj_in[cand[k]] < obj_in[cand[b1]]) b1 = k;
      for (int k = 0; k < 5; ++k)
        if (k != b1 && (b2 < 0 || obj_in[cand[k]] < obj_in[cand[b2]])) b2 = k;
      const int32_t *p1 = prio_in + (int64_t)cand[b1] * n, *p2 = prio_in + (int64_t)cand[b2] * n;
      int32_t *v = child + (int64_t)i * n;
      memcpy(v, p1, row);
      rng_block(seed, shop, (uint64_t)i, (uint64_t)gen, (uint64_t)event, 1, 0, w);
      if (n >= 2 && (uint32_t)(w[0] >> 32) < gp->pc) {
        const int32_t cut = 1 + (int32_t)draw_below(w[1], (uint32_t)(n - 1));
        orc_crossover(n, p1, p2, cut, v, tb);
      }
    }
  }
  /* swap mutation, as the hybrid GA */
  for (int32_t i = 0; i < pop; ++i) {
    rng_block(seed, shop, (uint64_t)i, (uint64_t)gen, (uint64_t)event, 2, 0, w);
    if ((uint32_t)(w[0] >> 32) < gp->pm && n >= 2) orc_mutate(n, child + (int64_t)i * n, w[1], w[2]);
  }
  rc = orc_decode_pop(in, child, pop, cobj, NULL, n_threads);
  if (rc) {
    free(child); free(tb); free(cobj); free(prefix); free(par);
    return rc;
  }
  memcpy(elite_out, elite_in, row);
  elite_obj_out[0] = elite_obj_in[0];
  if (scheme == ORC_GA_CLASSICAL) {
    memcpy(prio_out, child, row * (size_t)pop);
    memcpy(obj_out, cobj, sizeof(int64_t) * (size_t)pop);
    int32_t b = 0, wst = 0;
    for (int32_t i = 0; i < pop; ++i) {
      if (obj_out[i] < obj_out[b]) b = i;
      if (obj_out[i] > obj_out[wst]) wst = i;
    }
    if (obj_out[b] < elite_obj_out[0]) {
      memcpy(elite_out, prio_out + (int64_t)b * n, row);
      elite_obj_out[0] = obj_out[b];
    }
    memcpy(prio_out + (int64_t)wst * n, elite_out, row);
    obj_out[wst] = elite_obj_out[0];
  } else {
    for (int32_t i = 0; i < pop; ++i) {
      const int better = cobj[i] < obj_in[i];
      memcpy(prio_out + (int64_t)i * n, better ? child + (int64_t)i * n : prio_in + (int64_t)i * n, row);
      obj_out[i] = better ? cobj[i] : obj_in[i];
    }
    int32_t b = 0;
    for (int32_t i = 1; i < pop; ++i)
      if (obj_out[i] < obj_out[b]) b = i;
    if (obj_out[b] < elite_obj_out[0]) {
      memcpy(elite_out, prio_out + (int64_t)b * n, row);
      elite_obj_out[0] = obj_out[b];
    }
  }
  free(child); free(tb); free(cobj); free(prefix); free(par);
  return ORC_OK;
}

int orc_reschedule(const orc_instance *prev, const int32_t *plan_start,
                   const int32_t *plan_mach, int32_t rs, int32_t n_new,
                   const int32_t *new_proc, const int32_t *new_power,
                   const int32_t *new_release, const int32_t *new_due,
                   orc_resched_out *out) {
  const int32_t g = prev->n_stages, om = prev->o_max, n0 = prev->n_jobs;
  if (n_new < 0 || rs < prev->rs || g < 1 || om < 1) return ORC_E_INVAL;
  const int32_t n = n0 + n_new;
  const size_t per_job = (size_t)g * om;
  memcpy(out->proc, prev->proc, sizeof(int32_t) * per_job * n0);
  memcpy(out->power, prev->power, sizeof(int32_t) * per_job * n0);
  memcpy(out->proc + per_job * n0, new_proc, sizeof(int32_t) * per_job * n_new);
  memcpy(out->power + per_job * n0, new_power, sizeof(int32_t) * per_job * n_new);
  memcpy(out->release, prev->release, sizeof(int32_t) * n0);
  memcpy(out->due, prev->due, sizeof(int32_t) * n0);
  memcpy(out->release + n0, new_release, sizeof(int32_t) * n_new);
  memcpy(out->due + n0, new_due, sizeof(int32_t) * n_new);
  for (size_t k = 0; k < per_job; ++k) out->machine_free[k] = 0;
  out->n_jobs = n;
  out->n_running = 0;
  out->frozen_tardiness = 0;
  out->frozen_cmax = 0;

  for (int32_t j = 0; j < n0; ++j) {
    /* Reading: an op is frozen iff it started strictly before RS ("started or
     * completed before the rescheduling point", Section 4.3; eq. (10)). The
     * frozen ops of a job form a stage prefix because of eq. (5). */
    int32_t f = g;
    for (int32_t s = 0; s < g; ++s)
      if (plan_start[(int64_t)j * g + s] >= rs) {
        f = s;
        break;
      }
    for (int32_t s = f; s < g; ++s)
      if (plan_start[(int64_t)j * g + s] < rs) return ORC_E_INVAL;
    int32_t last_end = prev->release[j];
    for (int32_t s = 0; s < f; ++s) {
      int32_t m = plan_mach[(int64_t)j * g + s];
      if (m < 0 || m >= prev->n_machines[s]) return ORC_E_INVAL;
      int32_t st = plan_start[(int64_t)j * g + s];
      int32_t end = st + prev->proc[((int64_t)j * g + s) * om + m];
      if (end > out->machine_free[s * om + m]) out->machine_free[s * om + m] = end;
      if (end > rs) {  /* running at RS: Algorithm 1's z = 0 case */
        out->running[2 * out->n_running] = end;
        out->running[2 * out->n_running + 1] = prev->power[((int64_t)j * g + s) * om + m];
        out->n_running++;
      }
      last_end = end;
    }
    out->first_stage[j] = f;
    out->ready[j] = f == 0 ? prev->release[j] : last_end;
    if (f == g) {
      int32_t late = last_end - prev->due[j];
      out->frozen_tardiness += late > 0 ? late : 0;
      out->frozen_cmax = MAX32(out->frozen_cmax, last_end);
    }
  }
  for (int32_t i = 0; i < n_new; ++i) {
    out->first_stage[n0 + i] = 0;
    out->ready[n0 + i] = new_release[i];
  }
  out->n_active = 0;
  for (int32_t j = 0; j < n; ++j)
    if (out->first_stage[j] < g) out->active[out->n_active++] = j;
  return ORC_OK;
}

int orc_reschedule_static(const orc_instance *prev, const int32_t *plan_start,
                          const int32_t *plan_mach, int32_t rs, int32_t n_new,
                          const int32_t *new_proc, const int32_t *new_power,
                          const int32_t *new_release, const int32_t *new_due,
                          orc_resched_out *out) {
  const int32_t g = prev->n_stages, om = prev->o_max, n0 = prev->n_jobs;
  if (n_new < 0 || rs < prev->rs || g < 1 || om < 1) return ORC_E_INVAL;
  const int32_t n = n0 + n_new;
  const size_t per_job = (size_t)g * om;
  memcpy(out->proc, prev->proc, sizeof(int32_t) * per_job * n0);
  memcpy(out->power, prev->power, sizeof(int32_t) * per_job * n0);
  memcpy(out->proc + per_job * n0, new_proc, sizeof(int32_t) * per_job * n_new);
  memcpy(out->power + per_job * n0, new_power, sizeof(int32_t) * per_job * n_new);
  memcpy(out->release, prev->release, sizeof(int32_t) * n0);
  memcpy(out->due, prev->due, sizeof(int32_t) * n0);
  memcpy(out->release + n0, new_release, sizeof(int32_t) * n_new);
  memcpy(out->due + n0, new_due, sizeof(int32_t) * n_new);
  out->n_jobs = n;
  out->n_running = 0;
  out->n_fixed = 0;
  out->frozen_tardiness = 0;
  out->frozen_cmax = 0;
  /* completion of the plan's last op at each stage */
  int32_t *stage_end = (int32_t *)calloc((size_t)g, sizeof(int32_t));
  if (!stage_end) return ORC_E_NOMEM;
  for (int32_t j = 0; j < n0; ++j) {
    int32_t last_end = prev->release[j];
    for (int32_t s = 0; s < g; ++s) {
      const int32_t m = plan_mach[(int64_t)j * g + s], st = plan_start[(int64_t)j * g + s];
      if (m < 0 || m >= prev->n_machines[s] || st < 0) {
        free(stage_end);
        return ORC_E_INVAL;
      }
      const int32_t end = st + prev->proc[((int64_t)j * g + s) * om + m];
      const int32_t q = prev->power[((int64_t)j * g + s) * om + m];
      stage_end[s] = MAX32(stage_end[s], end);
      if (st < rs && end > rs) {  /* running at RS: power on [RS, end) */
        out->running[2 * out->n_running] = end;
        out->running[2 * out->n_running + 1] = q;
        out->n_running++;
      } else if (st >= rs) {      /* not started: power on its planned window */
        out->fixed[3 * out->n_fixed] = st;
        out->fixed[3 * out->n_fixed + 1] = end;
        out->fixed[3 * out->n_fixed + 2] = q;
        out->n_fixed++;
      }
      last_end = end;
    }
    out->first_stage[j] = g;
    out->ready[j] = last_end;
    const int32_t late = last_end - prev->due[j];
    out->frozen_tardiness += late > 0 ? late : 0;
    out->frozen_cmax = MAX32(out->frozen_cmax, last_end);
  }
  for (int32_t s = 0; s < g; ++s)
    for (int32_t m = 0; m < om; ++m) out->machine_free[s * om + m] = m < prev->n_machines[s] ? stage_end[s] : 0;
  free(stage_end);
  for (int32_t i = 0; i < n_new; ++i) {
    out->first_stage[n0 + i] = 0;
    out->ready[n0 + i] = new_release[i];
  }
  out->n_active = 0;
  for (int32_t j = 0; j < n; ++j)
    if (out->first_stage[j] < g) out->active[out->n_active++] = j;
  return ORC_OK;
}
