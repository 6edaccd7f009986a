/*
 * CPU oracle for the energy-efficient dynamic flexible flow shop (EDFFS) and
 * its priority-based hybrid parallel GA (Luo, Fujimura, El Baz,
 * arXiv 1903.10741).
 *
 * TEST INFRASTRUCTURE ONLY. This library is the plain, slow, obviously
 * correct statement of what the GPU path computes. Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it. The GPU
 * library never includes this header nor links this code, and this code never
 * includes anything from the GPU library.
 *
 * Conventions (all integer):
 *   times int32, objective int64, power int32;
 *   arrays row-major, caller-owned; no function keeps a pointer past return.
 *   Return 0 on success or a negative ORC_E_* code.
 */
#ifndef FFS_ORACLE_H
#define FFS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_E_INVAL (-1)       /* bad shape, not a permutation, order breaks route */
#define ORC_E_INFEASIBLE (-2)  /* some Q_jsm > Q_max: no start time can ever fit */
#define ORC_E_NOMEM (-3)

/* One event's instance: all jobs known so far (original and arrived, J u J'),
 * plus the state frozen at the rescheduling point RS (Section 4.1). */
typedef struct {
  int32_t n_jobs, n_stages, o_max;
  const int32_t *n_machines;   /* [g] machines per stage, 1 <= o_s <= o_max */
  const int32_t *proc;         /* [n_jobs][g][o_max] P_jsm >= 1 */
  const int32_t *power;        /* [n_jobs][g][o_max] Q_jsm >= 1 */
  const int32_t *release;      /* [n_jobs] R_j */
  const int32_t *due;          /* [n_jobs] D_j */
  int32_t q_max, wt, rs;       /* Q_max, WT, rescheduling point RS */
  const int32_t *first_stage;  /* [n_jobs] first stage not frozen; g = all frozen */
  const int32_t *ready;        /* [n_jobs] earliest start of stage first_stage */
  const int32_t *machine_free; /* [g][o_max] end of the last frozen op per machine */
  int32_t n_running;
  const int32_t *running;      /* [n_running][2] (end, q): power held on [RS, end) */
  int64_t frozen_tardiness;    /* sum of T_j over jobs with every op frozen */
  int32_t frozen_cmax;         /* max C_j over those jobs (0 if none) */
  int32_t n_active;
  const int32_t *active;       /* [n_active] job ids with first_stage < g; gene k <-> active[k] */
  int32_t decode_rules;        /* job-vector decode variants, ORC_RULE_* bits (0 = the default) */
  int32_t n_fixed;
  const int32_t *fixed;        /* [n_fixed][3] (start, end, q): planned ops that stay where the
                                  plan put them (the traditional static approach), power q held on
                                  [start, end) with RS <= start < end */
} orc_instance;

/* Variants of the job-vector decode (readings the paper leaves open):
 * ORC_RULE_FIFO: at each stage the jobs go in order of the completion of
 *   their previous stage (their `ready` time for the first unfrozen stage),
 *   earliest first, ties by priority; by default every stage takes the
 *   priority order.
 * ORC_RULE_POWER_ECT: the machine of earliest completion counting the power
 *   push-right on each machine (ties to the lowest index); by default the
 *   earliest completion ignoring power. Machines whose completion ignoring
 *   power cannot beat the best found so far are not pushed right (the
 *   machine of least such bound goes first). Work per op then counts 3 per
 *   machine, the examined slots + p of every machine pushed right, plus p
 *   updated.
 * X/Y chromosomes fix both order and machine and ignore these bits. */
#define ORC_RULE_FIFO 1
#define ORC_RULE_POWER_ECT 2

/* Counter-based generator Philox4x64 with 10 rounds (Salmon, Moraes, Dror,
 * Shaw, SC'11), written from its published description. */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Upper bound (slots after RS) on any completion time a decode can produce. */
int64_t orc_horizon_bound(const orc_instance *in);

/* Decode one job-priority vector prio[n_active] (a permutation of 1..n_active,
 * larger = higher priority) into a schedule and its objective, eq. (1).
 * start/mach ([n_jobs][g], may be NULL): entries of decoded ops are written,
 * entries of frozen ops are left untouched. work (may be NULL): algorithmic
 * operation count of this decode: per op 3*o_s for the machine choice, plus
 * (S - t0) + p slots examined by the push-right from its first candidate
 * start t0, plus p slots updated. */
int orc_decode(const orc_instance *in, const int32_t *prio, int64_t *obj,
               int32_t *start, int32_t *mach, int64_t *work);

/* Decode pop vectors prio[pop][n_active]; OpenMP over chromosomes. */
int orc_decode_pop(const orc_instance *in, const int32_t *prio, int32_t pop,
                   int64_t *obj, int64_t *work, int32_t n_threads);

/* Operation-level decode (the paper's own X/Z form): place ops[n_ops][3] =
 * (job, stage, machine) in the given order; machine -1 picks the earliest
 * completion machine. Every op must be its job's next unplaced stage. If
 * every unfrozen op is placed, *obj gets eq. (1); otherwise *obj = -1. */
int orc_decode_ops(const orc_instance *in, int32_t n_ops, const int32_t *ops,
                   int64_t *obj, int32_t *start, int32_t *mach);

/* The paper's own chromosome (Section 4.3, eqs. (10)-(12)): a target-machine
 * matrix X and a priority matrix Y over the operations. Only unfrozen ops
 * carry genes (the -1 entries of X and Y have none): R of them, row-major
 * over the active jobs in active order, stages first_stage..g-1. An X/Y
 * chromosome is genes[2R] = (x_0..x_{R-1}, y_0..y_{R-1}) with x_k a machine
 * of the op's stage and y a permutation of 1..R, larger = higher priority. */
int32_t orc_xy_ops(const orc_instance *in);

/* Assignment order Z (Algorithm 1). Reading: the two rules of Algorithm 1
 * can contradict each other; Z is built greedily, each step taking, among
 * the ops whose job's previous stage is already ordered (or frozen), the one
 * with the largest y. order[R][2] receives (job, stage) in that order. */
int orc_xy_order(const orc_instance *in, const int32_t *y, int32_t *order);

/* Decode genes[2R]: the ops in Z order, each on its X machine, with the
 * start rule of orc_decode (Algorithm 2). Outputs as orc_decode; work counts
 * (S - t0) + 2p per op (no machine choice). */
int orc_decode_xy(const orc_instance *in, const int32_t *genes, int64_t *obj,
                  int32_t *start, int32_t *mach, int64_t *work);
int orc_decode_xy_pop(const orc_instance *in, const int32_t *genes, int32_t pop,
                      int64_t *obj, int64_t *work, int32_t n_threads);

/* GA parameters. An island is a rows x cols torus; islands are contiguous.
 * encoding 0: one priority per job (n_active genes); 1: X/Y (2R genes). */
typedef struct {
  int32_t islands, rows, cols;
  uint32_t pc, pm;             /* crossover / mutation if hi32(draw) < threshold */
  int32_t mig_interval, mig_k; /* ring migration every mig_interval generations */
  int32_t encoding;
} orc_ga_params;

/* Population init (generation 0): Fisher-Yates from Philox purpose 0, decode,
 * elite = island best. Outputs prio[pop][n_active], obj[pop],
 * elite[islands][n_active], elite_obj[islands]. */
int orc_ga_init(const orc_instance *in, const orc_ga_params *gp, uint64_t seed,
                uint64_t shop, int32_t event, int32_t *prio, int64_t *obj,
                int32_t *elite, int64_t *elite_obj, int32_t n_threads);

/* One generation gen >= 1: selection, crossover + correction, mutation,
 * decode, replacement, then migration when gen % mig_interval == 0.
 * Reads *_in, writes *_out (distinct buffers). island_sel (may be NULL = all):
 * only islands with island_sel[i] != 0 are written to the outputs; the
 * entries of other islands in the outputs are unspecified. */
int orc_ga_generation(const orc_instance *in, const orc_ga_params *gp,
                      uint64_t seed, uint64_t shop, int32_t event, int32_t gen,
                      const int32_t *prio_in, const int64_t *obj_in,
                      const int32_t *elite_in, const int64_t *elite_obj_in,
                      int32_t *prio_out, int64_t *obj_out,
                      int32_t *elite_out, int64_t *elite_obj_out,
                      const uint8_t *island_sel, int32_t n_threads);

/* The two halves of orc_ga_generation. orc_ga_breed: selection, crossover +
 * correction and mutation of the needed islands into prio_out, the random
 * draws of crossover and mutation taken from block `variant` (0 = the plain
 * generation's). orc_ga_finish: decode of those children, replacement and
 * migration, in place on prio_out/obj_out. orc_ga_generation is breed
 * (variant 0) then finish. */
int orc_ga_breed(const orc_instance *in, const orc_ga_params *gp,
                 uint64_t seed, uint64_t shop, int32_t event, int32_t gen, int32_t variant,
                 const int32_t *prio_in, const int64_t *obj_in, int32_t *prio_out,
                 const uint8_t *island_sel);
int orc_ga_finish(const orc_instance *in, const orc_ga_params *gp, int32_t gen,
                  int32_t *prio_out, int64_t *obj_out,
                  const int32_t *elite_in, const int64_t *elite_obj_in,
                  int32_t *elite_out, int64_t *elite_obj_out,
                  const uint8_t *island_sel, int32_t n_threads);

/* GA building blocks, exposed for the tests. */
void orc_crossover(int32_t n, const int32_t *a, const int32_t *b, int32_t cut,
                   int32_t *child_a, int32_t *child_b);
/* X/Y crossover (Section 4.4, Fig. 11): both matrices spliced at gene `cut`,
 * the Y halves then corrected; genes as in orc_xy_ops (R per matrix). */
void orc_crossover_xy(int32_t R, const int32_t *a, const int32_t *b, int32_t cut,
                      int32_t *child_a, int32_t *child_b);
void orc_correct(int32_t n, int32_t *v);
void orc_mutate(int32_t n, int32_t *v, uint64_t w1, uint64_t w2);  /* n >= 2 */

/* The comparison GAs of Section 5.2 (Tables 8-9), on job-priority vectors, one
 * population of rows x cols individuals (islands must be 1), generation 0 by
 * orc_ga_init. Draws: purpose 1 crossover, 2 mutation (as the hybrid GA),
 * 6 the classical GA's roulette spins.
 *
 * orc_emax: E_max of eq. (13), 10^a with the least a >= 1 such that every
 * objective of the initial population is below it (Section 5.1).
 *
 * Classical GA (reading of "roulette wheel selection ... single point
 * crossover ... with randomly paired individuals ... mutation kept the same"):
 * fitness F_i = max(E_max - obj_i, 0) (eq. (13)); slot i's parent is the
 * first individual whose running fitness sum (index order) exceeds
 * floor(hi32(w) * sum F / 2^32), w word 0 of slot i's purpose-6 block (a
 * uniform individual, floor(hi32(w) * pop / 2^32), if every fitness is 0).
 * The spins are independent, so consecutive slots (2k, 2k+1) are a random
 * pairing of the selected parents: with p_c (slot 2k's purpose-1 block, as in
 * the hybrid GA) they exchange tails at the same cut with correction, else
 * they keep their parents; a last unpaired slot keeps its parent. Swap
 * mutation as the hybrid GA. Replacement as the hybrid GA's with the whole
 * population as one island (best-in-history kept, written over the worst).
 *
 * Cellular GA (reading of "two individuals are selected from a similar
 * neighborhood area as the local asteroid selection ... single point
 * crossover ... to generate a new individual ... same mutation ... replaces
 * the target individual if its solution is better"): cell i's neighbourhood is
 * itself and its four torus neighbours (order self, up, down, left, right);
 * the two parents are its best two entries by (objective, order); with p_c
 * (cell i's purpose-1 block) the child is the best's head and the second's
 * tail at the cut, corrected, else a copy of the best; swap mutation as the
 * hybrid GA; the child replaces cell i when its objective is strictly lower.
 * The elite (best in history) is the lowest objective, lowest cell on ties. */
#define ORC_GA_CLASSICAL 1
#define ORC_GA_CELLULAR 2
int64_t orc_emax(const int64_t *obj, int32_t pop);
int orc_ga_generation_scheme(const orc_instance *in, const orc_ga_params *gp, int32_t scheme,
                             int64_t e_max, uint64_t seed, uint64_t shop, int32_t event,
                             int32_t gen, const int32_t *prio_in, const int64_t *obj_in,
                             const int32_t *elite_in, const int64_t *elite_obj_in,
                             int32_t *prio_out, int64_t *obj_out, int32_t *elite_out,
                             int64_t *elite_obj_out, int32_t n_threads);

/* Predictive-reactive rescheduling (Section 4.1, eq. (10)): freeze every op of
 * the executed plan that started before rs, append the n_new arrived jobs and
 * produce the next event's instance. */
typedef struct {
  int32_t *proc, *power;       /* [n_jobs + n_new][g][o_max] */
  int32_t *release, *due, *first_stage, *ready;  /* [n_jobs + n_new] */
  int32_t *machine_free;       /* [g][o_max] */
  int32_t *running;            /* [g * o_max][2]: a machine runs at most one op at RS */
  int32_t *active;             /* [n_jobs + n_new] */
  int32_t n_jobs, n_running, n_active;
  int64_t frozen_tardiness;
  int32_t frozen_cmax;
  int32_t *fixed;              /* [n_jobs * g][3], orc_reschedule_static only */
  int32_t n_fixed;
} orc_resched_out;

int orc_reschedule(const orc_instance *prev, const int32_t *plan_start,
                   const int32_t *plan_mach, int32_t rs, int32_t n_new,
                   const int32_t *new_proc, const int32_t *new_power,
                   const int32_t *new_release, const int32_t *new_due,
                   orc_resched_out *out);

/* The traditional static approach (Section 4.3, Fig. 7; Section 5.3), the
 * comparison the paper draws against complete rescheduling: the executed
 * plan of every job known before rs stays as it is, started or not, and the
 * n_new arrivals are scheduled after it, a new job's op at stage s no earlier
 * than the completion of the plan's last op at stage s ("after completing the
 * operations of the original schedule at each stage"). Every old job is
 * frozen whole: its ops running at rs hold their power on [rs, end)
 * (running), those starting at or after rs on their planned window (fixed);
 * every machine of stage s is free from the stage's planned completion. The
 * next instance's active jobs are the arrivals. */
int orc_reschedule_static(const orc_instance *prev, const int32_t *plan_start,
                          const int32_t *plan_mach, int32_t rs, int32_t n_new,
                          const int32_t *new_proc, const int32_t *new_power,
                          const int32_t *new_release, const int32_t *new_due,
                          orc_resched_out *out);

#ifdef __cplusplus
}
#endif
#endif
