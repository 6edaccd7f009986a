/*
 * ffsga: MI355X (gfx950) library for the hot path of the priority-based hybrid
 * parallel GA for the energy-efficient dynamic flexible flow shop (EDFFS) of
 * Luo, Fujimura and El Baz (arXiv 1903.10741).
 *
 * The problem (Section 3): jobs J u J' go through g stages in order; stage s
 * has o_s parallel machines; op (j,s) on machine m takes P_jsm time and draws
 * Q_jsm power; the total power at every instant stays within Q_max (eqs.
 * (7)-(9)); the objective is WT * total tardiness + makespan (eq. (1)).
 * New jobs arriving at a rescheduling point RS trigger predictive-reactive
 * complete rescheduling (Section 4.1): ops started before RS are frozen, every
 * other op is rescheduled no earlier than RS (eq. (10)).
 *
 * The chromosome is one priority per unfrozen job (larger = higher, Section
 * 4.3); a decode places ops stage by stage in decreasing priority, each on
 * the machine of earliest completion, after that machine's earlier ops, at
 * the earliest start whose power window fits under Q_max (Algorithm 2).
 *
 * Conventions
 *   - Every pointer marked "device" is GPU memory owned by the caller; the
 *     library keeps no pointer past a call except inside a caller-owned
 *     ffs_ga. Arrays are row-major, int32 unless stated.
 *   - `stream` is a hipStream_t (NULL = default stream). Calls are
 *     asynchronous on it unless documented to synchronise.
 *   - Calls return FFS_OK (0) or a negative FFS_E_* code and never allocate
 *     device memory; scratch memory comes from the caller's workspace.
 *   - An error raised inside a kernel (bad input found on the device) is
 *     reported by the next synchronising call of the same workspace
 *     (ffs_status, ffs_prepare, reschedule) as FFS_E_INVAL/FFS_E_INFEASIBLE.
 *   - Limits of this build: o_max <= 16, g <= 127, n_jobs < 2^20,
 *     P_jsm and Q_jsm in [1, 65535], Q_max <= 255, n_active <= 4096,
 *     RS + horizon < 2^27. Larger instances get FFS_E_UNSUPPORTED.
 */
#ifndef FFSGA_H
#define FFSGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FFS_OK 0
#define FFS_E_INVAL (-1)        /* bad shape, not a permutation, plan breaks the rules */
#define FFS_E_INFEASIBLE (-2)   /* some Q_jsm > Q_max: no op start can ever fit */
#define FFS_E_WORKSPACE (-3)    /* workspace missing or too small */
#define FFS_E_DEVICE (-4)       /* HIP runtime error */
#define FFS_E_UNSUPPORTED (-5)  /* outside the limits of this build */

/* One event's instance (Section 3, Table 2): every job known so far and the
 * state frozen at the rescheduling point. */
typedef struct {
  int32_t n_jobs, n_stages, o_max;  /* |J u J'|, g, row width of proc/power */
  const int32_t *n_machines;        /* device [g]: o_s, 1 <= o_s <= o_max */
  const int32_t *proc;              /* device [n_jobs][g][o_max]: P_jsm (m < o_s read) */
  const int32_t *power;             /* device [n_jobs][g][o_max]: Q_jsm */
  const int32_t *release, *due;     /* device [n_jobs]: R_j, D_j */
  int32_t q_max, wt, rs;            /* Q_max, WT, RS (0 for the first plan) */
  const int32_t *first_stage;       /* device [n_jobs]: first unfrozen stage, g = none */
  const int32_t *ready;             /* device [n_jobs]: earliest start of that stage */
  const int32_t *machine_free;      /* device [g][o_max]: end of the last frozen op */
  int32_t n_running;
  const int32_t *running;           /* device [n_running][2]: (end, q) of ops running at RS */
  int64_t frozen_tardiness;         /* sum of T_j over jobs whose every op is frozen */
  int32_t frozen_cmax;              /* max C_j over those jobs, 0 if none */
  int32_t n_active;
  const int32_t *active;            /* device [n_active]: unfrozen jobs; gene k <-> active[k] */
  int32_t horizon;                  /* host: slots after RS bounding every completion;
                                       set by ffs_prepare and reschedule */
  int32_t n_ops;                    /* host: unfrozen operations R = sum over active jobs of
                                       g - first_stage; set by ffs_prepare and reschedule */
  int32_t decode_rules;             /* host: FFS_RULE_* bits, variants of the job-priority
                                       decode (0 = the default rules); reschedule copies it */
  int32_t n_fixed;                  /* planned ops kept where the plan put them (written by
                                       reschedule_static; 0 otherwise) */
  const int32_t *fixed;             /* device [n_fixed][3]: (start, end, q) with
                                       RS <= start < end: power q held on [start, end) */
} ffs_instance;

/* Variants of the job-priority decode, readings the paper leaves open (X/Y
 * chromosomes fix order and machines and ignore them):
 * FFS_RULE_FIFO: at each stage the jobs go in order of the completion of their
 *   previous stage (their `ready` time at their first unfrozen stage), earliest
 *   first, ties by priority; by default every stage takes the priority order.
 * FFS_RULE_POWER_ECT: each op takes the machine of earliest completion after
 *   that machine's power push-right (ties to the lowest index); by default the
 *   earliest completion ignoring power. A push-right only delays, so a machine
 *   whose completion ignoring power is not below the best found so far is not
 *   pushed right (the machine of least such bound goes first). Its work count
 *   per op is 3 per machine, plus the examined slots + p of every machine
 *   pushed right, plus p updated. */
#define FFS_RULE_FIFO 1
#define FFS_RULE_POWER_ECT 2

/* Workspace bytes any ffs_prepare / ffs_status call needs. */
#define FFS_PREPARE_WORKSPACE 256

/* Check `inst` on the device (shapes, P/Q ranges, Q_jsm <= Q_max, active list
 * consistent with first_stage) and set inst->horizon: an upper bound on
 * (completion - RS) of every op any decode can place. Synchronises `stream`.
 * workspace: device, >= FFS_PREPARE_WORKSPACE bytes.
 * Errors: FFS_E_INVAL, FFS_E_INFEASIBLE, FFS_E_UNSUPPORTED, FFS_E_DEVICE. */
int ffs_prepare(ffs_instance *inst, void *workspace, size_t workspace_bytes, void *stream);

/* Device workspace bytes for ffs_decode or ffs_decode_xy of `pop` chromosomes. lds_slots: the
 * power-profile slots kept on chip per chromosome (0 = library default);
 * decodes that need more fall back to a slower profile in this workspace. */
size_t ffs_decode_workspace_size(const ffs_instance *inst, int32_t pop, int32_t lds_slots);

/* Decode pop priority vectors (Section 4.3, Algorithm 2, eq. (1)).
 * prio: device [pop][n_active], each a permutation of 1..n_active.
 * obj: device int64 [pop], WT * sum_j T_j + C_max over J u J'.
 * start, mach: device [pop][n_jobs][g] or NULL: start time and machine of every
 *   decoded op; entries of frozen ops are not written.
 * work: device int64 [pop] or NULL: algorithmic operation count of each decode
 *   (per op: 3*o_s for the machine choice, S - t0 + p slots examined by the
 *   push-right from its first candidate start t0, p slots updated).
 * A vector that is not a permutation gets obj = -1 and is reported by
 * ffs_status. inst must have been through ffs_prepare.
 * Errors: FFS_E_INVAL, FFS_E_WORKSPACE, FFS_E_UNSUPPORTED, FFS_E_DEVICE. */
int ffs_decode(const ffs_instance *inst, const int32_t *prio, int32_t pop, int64_t *obj,
               int32_t *start, int32_t *mach, int64_t *work, int32_t lds_slots,
               void *workspace, size_t workspace_bytes, void *stream);

/* Bytes of the library-owned device buffer behind ffs_decode_noalloc (one copy
 * per GPU, held until the process ends). */
#define FFS_DECODE_SCRATCH_BYTES (16u << 20)

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. ffs_decode
 * with its workspace taken from a static device buffer of
 * FFS_DECODE_SCRATCH_BYTES bytes that the library holds on each GPU, instead
 * of from the caller. Arguments, outputs, kernels and results are those of
 * ffs_decode without workspace/workspace_bytes; the caller still owns prio,
 * obj, start, mach and work. The call allocates nothing (no hipMalloc, no
 * allocating library routine) and the buffer's header is cleared by a kernel,
 * not a memset. Every call on one GPU shares that GPU's buffer, which keeps
 * the last call's contents: calls that overlap on one GPU (on different
 * streams or host threads) race and must be ordered by the caller.
 * A chromosome the kernels reject gets obj = -1; the device-side flags that
 * ffs_status reads for a caller's workspace stay in the shared buffer.
 * Errors: as ffs_decode; FFS_E_WORKSPACE when ffs_decode_workspace_size(inst,
 * pop, lds_slots) exceeds FFS_DECODE_SCRATCH_BYTES (nothing is launched);
 * FFS_E_DEVICE when the buffer's device address cannot be obtained. */
int ffs_decode_noalloc(const ffs_instance *inst, const int32_t *prio, int32_t pop, int64_t *obj,
                       int32_t *start, int32_t *mach, int64_t *work, int32_t lds_slots,
                       void *stream);

/* Decode pop X/Y chromosomes (Section 4.3, eqs. (10)-(12), Algorithms 1-2):
 * the paper's own encoding, a target machine and a priority per operation.
 * genes: device [pop][2 * n_ops]. Genes cover the n_ops unfrozen ops only
 * (the -1 entries of the paper's matrices carry none), row-major over the
 * active jobs in `active` order, each job's stages first_stage..g-1; the
 * first n_ops genes are the machines x (0 <= x < o_s of the op's stage), the
 * last n_ops the priorities y (a permutation of 1..n_ops, larger = higher).
 * The assignment order Z takes, step by step, the op of largest y among each
 * job's next unordered op (the greedy reading of Algorithm 1); each op then
 * starts on machine x at the earliest time after its job's previous stage and
 * the machine's last op at which the power stays within Q_max (the start rule
 * of ffs_decode). Outputs, workspace (ffs_decode_workspace_size), lds_slots,
 * work (per op: slots examined from the first candidate start plus p slots
 * updated) and errors as ffs_decode; a gene out of range or a y that is not a
 * permutation sets obj = -1 and makes ffs_status return FFS_E_INVAL. */
int ffs_decode_xy(const ffs_instance *inst, const int32_t *genes, int32_t pop, int64_t *obj,
                  int32_t *start, int32_t *mach, int64_t *work, int32_t lds_slots,
                  void *workspace, size_t workspace_bytes, void *stream);

/* Read and clear the device-side error flags of a workspace used by
 * ffs_decode or the GA (any kernel that met a bad input sets them).
 * Synchronises `stream`. Returns FFS_OK, FFS_E_INVAL or FFS_E_INFEASIBLE. */
int ffs_status(void *workspace, void *stream);

/* GA parameters (Sections 4.2, 4.4, 5.1). The population is `islands`
 * islands of rows x cols individuals on a torus, contiguous per island.
 * pc, pm: crossover / mutation happen when the high 32 bits of a draw are
 * below the threshold (floor(p * 2^32)). Every mig_interval generations the
 * mig_k best of island i-1 replace the mig_k worst of island i. */
typedef struct {
  int32_t islands, rows, cols;
  uint32_t pc, pm;
  int32_t mig_interval, mig_k;
  int32_t lds_slots;                /* on-chip profile slots per decode, 0 = default (4096);
                                       FFS_LDS_AUTO: sized by ga_init from generation 0 */
  int32_t encoding;                 /* 0: one priority per active job (n_genes = n_active);
                                       1: the paper's X/Y matrices (n_genes = 2 * n_ops, see
                                       ffs_decode_xy). The batched GA and ga_step_screened
                                       take encoding 0 only (else FFS_E_UNSUPPORTED). */
  int32_t scheme;                   /* FFS_GA_HYBRID (0, the method), or one of the comparison
                                       GAs of Section 5.2 below */
} ffs_ga_params;

/* ffs_ga_params.scheme. FFS_GA_CLASSICAL and FFS_GA_CELLULAR are the comparison
 * GAs of Section 5.2 (Tables 8-9) on job-priority vectors (encoding 0), one
 * population of rows x cols individuals (islands must be 1; the migration
 * fields are ignored), generation 0 as the hybrid GA's. Draws: purpose 1
 * crossover, 2 mutation, as the hybrid GA; 6 the classical GA's roulette.
 * FFS_GA_CLASSICAL: ga_init also sets E_max of eq. (13), 10^a with the least a
 *   >= 1 above every objective of generation 0; each generation, slot i's
 *   parent is the first individual whose running sum of the fitness
 *   F = max(E_max - obj, 0) (index order) exceeds floor(hi32(w) * sum F /
 *   2^32), w word 0 of slot i's purpose-6 block (a uniform individual,
 *   floor(hi32(w) * pop / 2^32), if every fitness is 0) -- the roulette wheel;
 *   the independent spins make slots (2k, 2k+1) a random pairing: with p_c
 *   (slot 2k's purpose-1 block) they exchange tails at one cut with
 *   correction (Fig. 11); a last unpaired slot keeps its parent; swap mutation
 *   (Fig. 12); replacement as the hybrid GA's over the whole population.
 * FFS_GA_CELLULAR: cell i takes the best two of itself and its four torus
 *   neighbours (by objective, then in the order self, up, down, left, right),
 *   crosses them at its own cut with p_c (the best's head, the second's tail,
 *   corrected; else a copy of the best), applies the swap mutation, and the
 *   child replaces the cell only if its objective is strictly lower; the elite
 *   is the best in history (lowest cell on ties). */
#define FFS_GA_HYBRID 0
#define FFS_GA_CLASSICAL 1
#define FFS_GA_CELLULAR 2

/* ffs_ga_params.lds_slots = FFS_LDS_AUTO (job-priority vectors only; encoding 1
 * gets FFS_E_UNSUPPORTED): ga_init decodes generation 0 with as many on-chip
 * slots as one workgroup's LDS holds (at most 16384, no more than the horizon
 * needs; a longer schedule is redone off chip) and records the longest schedule
 * (end - RS). Every later generation
 * keeps that schedule plus 1/64 of it and 64 slots on chip, widened to the
 * most slots (a multiple of 64, at most 32768) at which a compute
 * unit still holds as many waves of the generation kernel (the runtime's
 * occupancy figure), so long schedules stay on chip and short ones leave LDS for
 * more waves. ga_init then synchronises its stream once and ffs_ga.lds_slots
 * holds the chosen slots. A later decode that outgrows them is redone off chip as
 * usual: results never depend on the choice. */
#define FFS_LDS_AUTO (-1)

/* GA state. Filled by ga_init; the caller owns the struct and the workspace.
 * The device pointers point into the workspace. ga_step must be given the
 * instance ga_init was given. */
typedef struct {
  ffs_ga_params params;
  int32_t n_genes, pop;
  uint64_t seed, shop;
  int32_t event, generation, cur;   /* cur: which of the two population buffers is live */
  int32_t lds_slots;                /* resolved on-chip profile slots */
  int32_t n_jobs, horizon;          /* of the instance given to ga_init */
  void *workspace;
  size_t workspace_bytes;
  int32_t *prio[2];                 /* device [pop][n_genes] */
  int64_t *obj[2];                  /* device [pop] */
  int32_t *elite;                   /* device [islands][n_genes] */
  int64_t *elite_obj;               /* device [islands] */
  int32_t island_groups;            /* island groups the last ga_step ran (1: one stream,
                                       0: none yet; ga_set_island_groups) */
  int32_t narrow_lds;               /* 1 if the last ga_step's generation kernel kept its
                                       ready times in 16 bits: under the default decode rules
                                       of the hybrid scheme, where that lets a compute unit
                                       hold more waves of a population larger than the chip
                                       holds at once (same results either way) */
} ffs_ga;

/* Device views of a GA state (pointers into its workspace). */
typedef struct {
  int32_t *prio;       /* [pop][n_genes] */
  int64_t *obj;        /* [pop] */
  int32_t *elite;      /* [islands][n_genes]: best-in-history per island */
  int64_t *elite_obj;  /* [islands] */
  int64_t *work;       /* [1]: algorithmic work summed over every decode since ga_init
                          (same count as ffs_decode's work output) */
  int64_t *e_max;      /* [1]: E_max of eq. (13) (FFS_GA_CLASSICAL; 0 otherwise) */
  int64_t *overflows;  /* [1]: job-vector decodes since ga_init whose schedule outgrew the
                          on-chip profile and were redone off chip (same results) */
} ffs_ga_view;

size_t ffs_ga_workspace_size(const ffs_instance *inst, const ffs_ga_params *params);

/* Generation 0 of one event: random unique priorities (Section 4.3) by a
 * Fisher-Yates shuffle driven by Philox4x64-10 keyed (seed, shop) with
 * counter (individual, 0, event, block), decode, elite = each island's best.
 * Errors: FFS_E_INVAL, FFS_E_WORKSPACE, FFS_E_UNSUPPORTED, FFS_E_DEVICE. */
int ga_init(ffs_ga *ga, const ffs_instance *inst, const ffs_ga_params *params, uint64_t seed,
            uint64_t shop, int32_t event, void *workspace, size_t workspace_bytes, void *stream);

/* Run n_generations generations in place (Section 4.4): local selection of the
 * best of self and four torus neighbours, neighbour-paired single-point
 * crossover with priority correction, swap mutation, decode, elitist
 * replacement, ring migration every mig_interval generations.
 * A decode that outgrows the on-chip slots is redone off chip by its own
 * wave when the workspace holds an off-chip profile for every individual
 * (pop x (horizon + 64) bytes rounded to 256, used up to 1 GiB and counted by
 * ffs_ga_workspace_size), else by a separate kernel after the generation;
 * the results are the same either way.
 * Errors: FFS_E_INVAL, FFS_E_DEVICE. */
int ga_step(ffs_ga *ga, const ffs_instance *inst, int32_t n_generations, void *stream);

/* How many island groups ga_step runs concurrently (process-wide; 0, the
 * default, means 4; 1 runs every launch on the caller's stream); unless
 * groups is 1, also creates the current device's group streams now. Between two
 * migrations the islands of the hybrid GA (Section 4.4) share nothing, so
 * ga_step splits them into `groups` contiguous groups (group g: islands
 * [islands * g / groups, islands * (g + 1) / groups)) and runs each group's
 * generations on a stream of its own: a group that has decoded and replaced
 * its islands starts its next generation while others still decode. The
 * library creates the extra streams (default priority) and events once per
 * device, here or at the first grouped ga_step; they fork from the caller's
 * stream, and ga_step joins them back into it before every migration and
 * before it returns, so the caller's stream orders everything as before. The
 * groups only overlap when their streams sit on hardware queues of their own:
 * the runtime spreads streams over a few queues per process in the order they
 * are created, so call this before creating other streams. Results are the
 * same for every grouping (draws are keyed by the global slot). Grouping
 * applies to the hybrid scheme whose overflowed decodes are redone by their
 * own waves (see ga_step), ga_step_screened's included, not to the comparison
 * GAs, and never to more groups than islands. Calls of ga_step from several host
 * threads take turns enqueueing on one device while grouping is in use.
 * Errors: FFS_E_INVAL (groups < 0 or > 4), FFS_E_DEVICE. */
int ga_set_island_groups(int32_t groups);

/* Copy the best elite (lowest island on ties) to prio_out (device
 * [n_genes]) and obj_out (device int64 [1]). */
int ga_best(const ffs_ga *ga, int32_t *prio_out, int64_t *obj_out, void *stream);

/* Device pointers of the live state (no copy). */
int ga_view(const ffs_ga *ga, ffs_ga_view *view);

/* Workspace bytes reschedule needs. */
size_t ffs_reschedule_workspace_size(int32_t n_jobs, int32_t n_new);

/* Predictive-reactive complete rescheduling (Section 4.1, eq. (10)): freeze
 * every op of the executed plan that started before rs (an op is running at
 * rs when it started before and ends after, Algorithm 1), append the n_new
 * arrivals and write the next event's instance into `next`.
 * prev: a prepared instance; plan_start/plan_mach: device [prev->n_jobs][g],
 *   the executed plan (start and machine of every op of every job).
 * new_proc/new_power: device [n_new][g][o_max]; new_release/new_due: device [n_new].
 * next: caller-filled device pointers with room for n_jobs + n_new jobs
 *   (proc, power, release, due, first_stage, ready, active), g*o_max
 *   (machine_free) and g*o_max pairs (running); the n_machines pointer may
 *   alias prev's. The library writes those arrays and every host field of
 *   `next`, horizon included. Synchronises `stream`.
 * Errors: FFS_E_INVAL (rs < prev->rs, plan out of range or not a stage
 *   prefix before rs), FFS_E_INFEASIBLE, FFS_E_WORKSPACE, FFS_E_DEVICE. */
int reschedule(const ffs_instance *prev, const int32_t *plan_start, const int32_t *plan_mach,
               int32_t rs, int32_t n_new, const int32_t *new_proc, const int32_t *new_power,
               const int32_t *new_release, const int32_t *new_due, ffs_instance *next,
               void *workspace, size_t workspace_bytes, void *stream);

/* The traditional static approach (Section 4.3, Fig. 7; Section 5.3), the
 * comparison the paper draws against complete rescheduling: the executed plan
 * of every job known before rs stays as it is, started or not, and the n_new
 * arrivals are scheduled after it: a new job's op at stage s starts no
 * earlier than the completion of the plan's last op at stage s. Every old
 * job is frozen whole (its objective terms go to frozen_tardiness and
 * frozen_cmax); its ops running at rs hold their power on [rs, end)
 * (running), those starting at or after rs on their planned windows
 * (fixed); every machine of stage s is free from the stage's planned
 * completion; the active jobs are the arrivals. Arguments, synchronisation and
 * errors as reschedule; next->fixed: caller-filled device pointer with room
 * for prev->n_jobs * g triples (the library writes next->n_fixed). */
int reschedule_static(const ffs_instance *prev, const int32_t *plan_start,
                      const int32_t *plan_mach, int32_t rs, int32_t n_new,
                      const int32_t *new_proc, const int32_t *new_power,
                      const int32_t *new_release, const int32_t *new_due, ffs_instance *next,
                      void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Batched GA: many independent instances (shops) advanced by the same
 * launches. The batch has n_slots slots of fixed room; each slot holds one
 * instance (sizes may differ, within the room) with its own population of
 * islands x rows x cols individuals, its own Philox key (seed, shop) and its
 * own generation count, kept on the device so that one generation is the
 * same launch sequence every time (it is captured once in a hipGraph when
 * use_graph is set and replayed). Every slot's results are bit-identical to
 * running its instance alone with ga_init / ga_step.
 * ------------------------------------------------------------------------ */
#define FFS_SCHEDULE_CHROMOSOME 0   /* one wave decodes one child */
#define FFS_SCHEDULE_ISLAND 1       /* one wave breeds, decodes and replaces one island */
#define FFS_BATCH_MAX_SLOTS 4096
#define FFS_BATCH_MAX_CLASSES 4

typedef struct {
  int32_t n_slots;         /* instances held at once, <= FFS_BATCH_MAX_SLOTS */
  int32_t max_jobs;        /* room per slot: n_jobs */
  int32_t max_genes;       /* room per slot: n_active */
  int32_t max_stages;      /* room per slot: g */
  int32_t o_max;           /* row width of every instance's proc/power, <= 16 */
  int32_t max_horizon;     /* room per slot: instance horizon (off-chip profile) */
  ffs_ga_params ga;        /* the same for every slot */
  int32_t schedule;        /* FFS_SCHEDULE_CHROMOSOME or FFS_SCHEDULE_ISLAND */
  int32_t blocks;          /* persistent grid size (resident waves), 0 = 8 per CU */
  int32_t use_graph;       /* capture one generation in a hipGraph and replay it */
  int32_t profile_classes; /* 0 or 1: every decode keeps ga.lds_slots profile slots on chip.
                              C in 2..FFS_BATCH_MAX_CLASSES: size classes lds_slots / 2^(C-1),
                              ..., lds_slots (rounded up to multiples of 64); each slot takes the
                              smallest class holding 5/4 of the longest schedule of its
                              generation 0 (measured on the device) and each generation launches
                              once per class with that class's LDS, so short schedules keep more
                              waves per CU. Results do not depend on it: a decode that outgrows
                              its class is redone off chip. */
} ffs_batch_params;

typedef struct {
  ffs_batch_params params;
  int32_t pop, lds_slots, blocks, omp;
  void *workspace;
  size_t workspace_bytes;
  void *graph, *graph_exec;            /* hipGraph_t / hipGraphExec_t of one generation */
  void *graph_stream;                  /* the stream the graph was captured on */
  int32_t active[FFS_BATCH_MAX_SLOTS];     /* host mirror: slot holds an instance */
  int32_t generation[FFS_BATCH_MAX_SLOTS]; /* host mirror: generations run since ga_batch_set */
  int32_t n_genes[FFS_BATCH_MAX_SLOTS];    /* host mirror: the slot's n_active */
} ffs_batch;

size_t ffs_batch_workspace_size(const ffs_batch_params *params);

/* Lay out an empty batch in the caller's workspace (every slot inactive). */
int ga_batch_create(ffs_batch *b, const ffs_batch_params *params, void *workspace,
                    size_t workspace_bytes, void *stream);

/* Load a prepared instance into a slot and run its generation 0 (as ga_init).
 * The instance's device arrays must stay valid while the slot is active.
 * Errors: FFS_E_INVAL, FFS_E_UNSUPPORTED (instance exceeds the slot's room). */
int ga_batch_set(ffs_batch *b, int32_t slot, const ffs_instance *inst, uint64_t seed,
                 uint64_t shop, int32_t event, void *stream);

/* Deactivate a slot (its buffers may then be reused by ga_batch_set). */
int ga_batch_clear(ffs_batch *b, int32_t slot, void *stream);

/* Every active slot runs n_generations generations. With use_graph the first
 * call captures one generation on `stream` (which must not be the legacy
 * default stream) and every later generation replays it. */
int ga_batch_step(ffs_batch *b, int32_t n_generations, void *stream);

int ga_batch_best(const ffs_batch *b, int32_t slot, int32_t *prio_out, int64_t *obj_out,
                  void *stream);
int ga_batch_view(const ffs_batch *b, int32_t slot, ffs_ga_view *view);

/* Release the graph (the workspace stays the caller's). */
int ga_batch_destroy(ffs_batch *b);

/* Kernel timing with HIP events around every launch of one kernel family:
 * 0 = decode (ffs_decode), 1 = GA generation (breed + decode), 2 = GA
 * replacement, 3 = overflow decode, 4 = batched generation (breed + decode,
 * outside graphs), 5 = screened generation (ffs_surrogate.h: candidate
 * breeding + scoring + decode). Family 6 times whole ga_step calls instead:
 * events on the caller's stream before its first launch and after its last
 * (island groups joined), every call, counted in generations, so its time over
 * its count is the time per generation of the whole population even when
 * island groups overlap their launches. families: 0 stops timing; otherwise
 * bit f selects family f (-1: all) and every family's count starts afresh.
 * Only the selected families get events, so untimed launches carry no event
 * overhead. ffs_timing_read synchronises and returns the summed time and the
 * number of launches (family 6: generations) since the call. */
int ffs_timing_enable(int32_t families);

/* Put events on one launch in `every` (>= 1, default 1) of each timed kernel
 * family (0-5), starting with the first after ffs_timing_enable;
 * ffs_timing_read then counts the timed launches only. Errors: FFS_E_INVAL. */
int ffs_timing_every(int32_t every);
int ffs_timing_read(int32_t family, double *total_ms, int64_t *launches);

const char *ffs_strerror(int code);

/* Identity of this build: the first 16 hex digits of the sha256 of the HIP
 * source and this header it was compiled from. */
const char *ffs_build_id(void);

#ifdef __cplusplus
}
#endif
#endif
