/*
 * ffs_surrogate: the learned offspring pre-screen of the EDFFS hybrid GA on
 * MI355X (gfx950). This addition has no counterpart in the paper: a small
 * DeepSets network predicts ln(objective) of a chromosome from its genes, and
 * a screened GA generation breeds several candidate children per cell, keeps
 * the one the network scores lowest and decodes only that one exactly; the
 * decoder of Section 4.3 (Algorithm 2, eq. (1)) remains the judge of every
 * fitness the GA uses.
 *
 * The network (H = 256 hidden units):
 *   per active job k (gene k), integers first, then one rounding to float32:
 *     tot_k   = sum over unfrozen stages s of min over machines of P_ksm
 *     slack_k = D_k - max(ready_k, RS) - tot_k,  rel_k = max(ready_k - RS, 0)
 *     scale   = max(1, max_k tot_k);  f_k = (tot, slack, rel) / scale
 *     rank_k  = gene value / n  (gene values are 1..n)
 *   c_k  = ((b1 + f0 W1[1]) + f1 W1[2]) + f2 W1[3]            (float32, no FMA)
 *   h1_k = bf16(max(c_k + rank_k W1[0], 0))
 *   h2_k = max(h1_k . bf16(W2) + b2, 0)                       (bf16 MFMA, fp32 accumulate)
 *   y    = b3 + mean over k of h2_k . w3     (predicts standardised ln obj, below)
 * The rank is the only input that varies between chromosomes of one
 * instance and takes n values, so layers 1 and 2 are evaluated once per
 * (job, rank) pair, an n^2 x 256 by 256 x 256 matrix-core product, and a
 * chromosome's score is a gather of n table entries.
 *
 * Parameters are float32, flat: [W1 (4 x H), b1 (H), W2 (H x H, row = input
 * unit), b2 (H), w3 (H), b3 (1)]; FFS_SG_PARAMS floats. The network predicts
 * ln(obj) standardised within the chromosome's population (screening only
 * compares the candidates of one cell, so a population's offset and spread
 * carry nothing it needs); training minimises mean (y - t)^2 over a batch
 * with Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 *
 * Conventions as in ffsga.h: device pointers are caller-owned GPU memory,
 * calls are asynchronous on `stream` (a hipStream_t, NULL = default), never
 * allocate, and return FFS_OK or a negative FFS_E_* code. Every reduction is
 * taken in a fixed order, so results repeat bit for bit from run to run.
 * Limits: 1 <= n_genes <= FFS_SG_MAX_GENES, 1 <= batch <= FFS_SG_MAX_BATCH.
 */
#ifndef FFS_SURROGATE_H
#define FFS_SURROGATE_H

#include "ffsga.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FFS_SG_HIDDEN 256
#define FFS_SG_PARAMS (4 * 256 + 256 + 256 * 256 + 256 + 256 + 1)
#define FFS_SG_MAX_GENES 256
#define FFS_SG_MAX_BATCH 8192
#define FFS_SG_MAX_VARIANTS 8

typedef struct {
  float *theta;          /* device [FFS_SG_PARAMS]: parameters, flat layout above */
  float *adam_m;         /* device [FFS_SG_PARAMS]: Adam first moment (caller zeroes it) */
  float *adam_v;         /* device [FFS_SG_PARAMS]: Adam second moment (caller zeroes it) */
  uint16_t *w2_bf16;     /* device [H][H]: bf16(W2), kept by sg_refresh and sg_train_step */
  uint16_t *w2t_bf16;    /* device [H][H]: its transpose */
  int32_t step;          /* host: Adam steps taken so far */
} ffs_surrogate;

/* bf16 copies of W2 from theta (call after writing theta). */
int sg_refresh(ffs_surrogate *model, void *stream);

/* Per-job features of a prepared instance: feats, device float32
 * [n_active][4] = (f0, f1, f2, 0) in gene order. workspace: device, at
 * least FFS_PREPARE_WORKSPACE bytes. Errors: FFS_E_INVAL (n_active outside
 * 1..FFS_SG_MAX_GENES), FFS_E_WORKSPACE, FFS_E_DEVICE. */
int sg_features(const ffs_instance *inst, float *feats, void *workspace, size_t workspace_bytes,
                void *stream);

/* Device workspace bytes of sg_score_table for n_genes. */
size_t sg_table_workspace_size(int32_t n_genes);

/* Score table of an instance: table, device float32 [n][n], table[k][v-1] =
 * h2(job k, rank v / n) . w3 (per-job dot products, summed in float32). */
int sg_score_table(const ffs_surrogate *model, const float *feats, int32_t n_genes, float *table,
                   void *workspace, size_t workspace_bytes, void *stream);

/* Scores of `count` chromosomes prio (device [count][n_genes], permutations
 * of 1..n): y[i] = b3 + (sum over k of table[k][prio[i][k]-1]) / n, the sum
 * taken in one fixed order (64 lane partials over k = lane, lane + 64, ...,
 * then a fixed pairwise tree), the same order ga_step_screened uses, so a
 * chromosome gets the same score bits from both. y: device float32 [count];
 * a chromosome with a gene outside 1..n gets NaN. */
int sg_score(const ffs_surrogate *model, const float *table, int32_t n_genes, const int32_t *prio,
             int32_t count, float *y, void *stream);

/* Training targets: t[i] = (ln obj[i] - mean) / sd over each group of `group`
 * consecutive entries (one population; the last group may be shorter), mean
 * and population standard deviation in float64 summed in a fixed order (256
 * runs of consecutive entries, each in index order, then a fixed pairwise
 * tree), the result rounded to float32; a group with sd = 0 gets 0. obj device int64
 * [count] (> 0), target device float32 [count]. workspace: device, at least
 * FFS_PREPARE_WORKSPACE bytes; an objective <= 0 is reported by the next
 * ffs_status(workspace) as FFS_E_INVAL. */
int sg_targets(const int64_t *obj, int32_t count, int32_t group, float *target, void *workspace,
               size_t workspace_bytes, void *stream);

/* Device workspace bytes of sg_train_step for n_genes and batch. */
size_t sg_train_workspace_size(int32_t n_genes, int32_t batch);

/* One Adam step on a batch of decoder-labelled chromosomes: prio device
 * [batch][n_genes], target device float32 [batch] (from sg_targets on the
 * exact eq. (1) objectives). The step minimises mean (y - t)^2 with learning
 * rate lr, increments model->step and refreshes the bf16 copies of W2.
 * loss (device float32 [1], may be NULL) receives the batch loss before the
 * step; grad (device float32 [FFS_SG_PARAMS], may be NULL) the gradient.
 * A batch holding a gene outside 1..n or a target that is not finite is found on the
 * device: the step then leaves the parameters and moments unchanged and the
 * next ffs_status(workspace) returns FFS_E_INVAL (model->step still counts
 * the call). The workspace starts with the 256-byte status block ffs_status
 * reads; its status is cleared at the start of every step.
 * Errors: FFS_E_INVAL, FFS_E_WORKSPACE, FFS_E_DEVICE. */
int sg_train_step(ffs_surrogate *model, const float *feats, int32_t n_genes, const int32_t *prio,
                  const float *target, int32_t batch, float lr, float *loss, float *grad,
                  void *workspace, size_t workspace_bytes, void *stream);

/* n_generations screened GA generations on ga (an ffs_ga of ffsga.h, set up
 * by ga_init on inst): in each, every cell breeds `variants` candidate
 * children (candidate v takes its crossover and mutation draws from Philox
 * block v; candidate 0 is the plain generation's child), scores them with
 * `table` (from sg_score_table on this instance and model), keeps the lowest
 * score (ties to the lowest v) and decodes it exactly; replacement and
 * migration follow as in ga_step, in island groups as ga_step's
 * (ga_set_island_groups). scores (device float32 [variants][pop])
 * and choice (device int32 [pop]), each may be NULL, receive the last
 * generation's candidate scores and kept candidates.
 * Errors: as ga_step, and FFS_E_INVAL for variants outside 1..FFS_SG_MAX_VARIANTS. */
int ga_step_screened(ffs_ga *ga, const ffs_instance *inst, const ffs_surrogate *model,
                     const float *table, int32_t variants, int32_t n_generations, float *scores,
                     int32_t *choice, void *stream);

#ifdef __cplusplus
}
#endif

#endif
