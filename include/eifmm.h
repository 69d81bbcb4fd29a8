/*
 * eifmm.h -- C ABI of the MI355X EIFMM evaluation library (libeifmm.so).
 *
 * The library computes the fast summation of F. Casenave, "A Fast Summation
 * Method for translation invariant kernels" (arXiv:1408.0210), eq. (1):
 *
 *     f(x_i) = sum_{j=1..N} sigma_j K(x_i, x_j),   i = 1..N,
 *
 * for translation-invariant 3D kernels K(x, y) = k(x - y), with targets equal
 * to sources (the N-body setting of Sec. 1) or, when the plan says so, at
 * n_targets separate target points x_i and N source points y_j:
 *
 *     f(x_i) = sum_{j=1..N} sigma_j K(x_i, y_j),   i = 1..n_targets.
 *
 * Following the problem statement of Sec. 1, the domain Omega and N are fixed
 * per plan while the points and the potentials change from query to query:
 *
 *     eifmm_plan_create   per-level EIM (Algorithm 1) and operator tables,
 *                         host FP64, uploaded once                (Sec. 2, 4.1, 4.2)
 *     eifmm_set_points    octree build on the GPU: Morton keys, stable sort,
 *                         leaf ranges, active boxes, near lists   (Sec. 3.3)
 *     eifmm_evaluate      Algorithm 3 steps 1-7 plus the near field of eq. (13),
 *                         all on the GPU                          (Sec. 3.3.4)
 *
 * Conventions
 *   - Device pointers are HIP device pointers (e.g. from PyTorch tensors).
 *     Points are SoA: coordinate a of point i at xyz[a * n + i], FP64.
 *     sigma and f are column-major n x nrhs FP64 blocks with leading
 *     dimensions ld and ldf (>= n).
 *   - The caller owns every buffer it passes; the library keeps no caller
 *     pointer after a call returns (points are copied into internal
 *     Morton-ordered storage).  The library owns its tables and workspaces
 *     until eifmm_plan_destroy.
 *   - Calls enqueue work on the given HIP stream (NULL = default stream) and
 *     return before it finishes, except the export calls, which copy to host
 *     memory and wait, and eifmm_set_points, which waits until the box counts
 *     of the tree are on the host (to report invalid points and size the
 *     pass); its last kernels (near lists, chunk table, M2L column order) are
 *     still in flight on its stream when it returns, so an evaluate on another
 *     stream must first wait for that stream.
 *   - Every call returns 0 (EIFMM_OK) or a negative status.  A failed call
 *     leaves the plan usable (or, for plan_create, nothing to destroy).
 *   - A plan is not thread-safe; distinct plans are independent.
 */
#ifndef EIFMM_H
#define EIFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define EIFMM_OK 0
#define EIFMM_EINVAL (-1)  /* null pointer, bad size, nrhs > max_rhs, struct_size mismatch */
#define EIFMM_EDOMAIN (-2) /* a point outside the closed domain, or not finite            */
#define EIFMM_ESTATE (-3)  /* evaluate before set_points, or a host-only plan             */
#define EIFMM_EEIM (-4)    /* EIM reached dmax before the tolerance                       */
#define EIFMM_ENOMEM (-5)  /* host or device allocation failed                            */
#define EIFMM_EHIP (-6)    /* a HIP call failed; eifmm_stats.hip_error holds the code     */

/* kernels k(z), r = |z| */
#define EIFMM_K_LAPLACE 0 /* 1/r, singular (pairs at r = 0 are skipped)          */
#define EIFMM_K_YUKAWA 1  /* exp(-a r)/r, a = kernel_param, singular             */
#define EIFMM_K_GAUSS 2   /* exp(-r^2/h2), h2 = kernel_param                     */
#define EIFMM_K_SQDIST 3  /* r^2: rank-5 test kernel, the EIM is exact           */
#define EIFMM_K_COSR 4    /* cos(w r)/r, w = kernel_param, singular (Sec. 5.4)   */
#define EIFMM_K_MQ 5      /* sqrt(r^2 + c), c = kernel_param > 0 (Sec. 5.4)       */
#define EIFMM_K_ADVDIFF 6 /* exp(a (z_x - r))/r, a = kernel_param >= 0, singular:
                             the steady advection-diffusion kernel (flow along x),
                             not symmetric, so two EIMs per level (Sec. 3.1)     */

/* precision of the pass */
#define EIFMM_PREC_FP64 0  /* every step in FP64                                   */
#define EIFMM_PREC_MIXED 1 /* M2L on FP32 MFMA (FP32 products, each offset's
                              contribution added in FP64); P2P with FP64
                              coordinate differences, FP32 kernel values and
                              compensated FP32 sums; EIM, triangular solves, M2M,
                              L2L, P2M, L2P and the final f in FP64              */

/* flags */
#define EIFMM_FLAG_HOST_ONLY 1 /* plan_create runs the host setup only (no device
                                  tables); only eifmm_get_level/get_stats work   */
#define EIFMM_FLAG_TWO_EIM 4    /* use the general form of Sec. 3.1 (a second EIM
                                   on D_x = J_0, D_y = I_0 per level) for a
                                   symmetric kernel too; kernels that are not
                                   symmetric always use it.  Not in batches.    */
#define EIFMM_FLAG_HOST_SETUP 2 /* run the Algorithm 1 iterations on the host even
                                   for a device plan (by default a device plan
                                   runs them on the GPU; both select the same
                                   points and factors, bit for bit)             */

#define EIFMM_MAX_DEPTH 8

typedef struct eifmm_plan_s *eifmm_plan; /* opaque, owned by the library */

typedef struct {
  int32_t struct_size;  /* sizeof(eifmm_config)                                    */
  int32_t kernel;       /* EIFMM_K_*                                               */
  double kernel_param;  /* a (Yukawa) or h2 (Gauss); ignored otherwise              */
  double lo[3];         /* domain [lo, lo+L]^3 (closed; Sec. 1: fixed per plan)     */
  double L;             /* side of the cube, > 0                                    */
  int64_t n;            /* N, fixed per plan (Sec. 1)                               */
  int32_t depth;        /* kappa: leaf level, 0..EIFMM_MAX_DEPTH; the far field uses
                           levels 2..kappa, kappa < 2 is near field only (Sec. 3.3) */
  int32_t max_rhs;      /* largest nrhs accepted by evaluate (>= 1)                 */
  double eim_tol;       /* tau > 0: the greedy stops when eps_k <= tau * scale       */
  int32_t tol_mode;     /* 0: scale = max |K| over the level's training grid;
                           1: scale = that of one level (scale_level, by default
                           the finest), for all levels                         */
  int32_t precision;    /* EIFMM_PREC_*                                             */
  int32_t dmax;         /* cap on d_k, 0..1024 (0 = 1024); reaching it is EIFMM_EEIM */
  int32_t flags;        /* EIFMM_FLAG_*                                             */
  double compress_tol;  /* > 0: compress the M2L matrices (Sec. 4.2, first stage):
                           SVD of [K^delta_1 .. K^delta_316] per level; the rank r
                           is the larger of the two filters (s_j/s_0 > eps, and the
                           prefix holding 1 - eps of the sum of singular values);
                           the device pads it to whole 16-row MFMA blocks with
                           zero rows and columns (eifmm_stats.rpad); 0 = off.
                           With two EIMs the stacked matrices give the basis of
                           the columns and r is the larger of the two ranks     */
  int64_t n_targets;    /* 0: the targets are the n sources; > 0: that many separate
                           target points (eifmm_set_points_targets), fixed per
                           plan; n + n_targets <= 2^30 - 1                       */
  double compress_tol2; /* > 0 (with compress_tol > 0): the second stage of Sec. 4.2,
                           each compressed matrix C^delta replaced by its rank-s
                           truncation, s from the same two filters on its own
                           singular values with this tolerance; 0 = off        */
  int32_t scale_level;  /* tol_mode 1: the level (2..EIFMM_MAX_DEPTH) whose training
                           grid's max |K| is the scale of every level's stopping
                           rule; 0 = the plan's depth.  Ignored with tol_mode 0  */
  int32_t reserved_cfg; /* must be 0                                             */
} eifmm_config;

/* evaluation phases timed when timing is enabled (eifmm_set_timing) */
#define EIFMM_PH_TREE 0  /* keys, sort, gather, leaf ranges, lists (set_points)   */
#define EIFMM_PH_P2P 1   /* near field, eq. (13)                                  */
#define EIFMM_PH_P2M 2   /* Algorithm 3 step 1                                    */
#define EIFMM_PH_M2M 3   /* step 2                                                */
#define EIFMM_PH_WHAT 4  /* step 3 (triangular solves)                            */
#define EIFMM_PH_M2L 5   /* step 4                                                */
#define EIFMM_PH_L2L 6   /* step 5                                                */
#define EIFMM_PH_LHAT 7  /* step 6 (triangular solves)                            */
#define EIFMM_PH_L2P 8   /* step 7 plus f = f_far + f_near in input order         */
#define EIFMM_PH_PROJ 9  /* compression projections U^T What and U g' (Sec. 4.2)  */
#define EIFMM_NPHASE 10

typedef struct {
  int32_t struct_size;               /* sizeof(eifmm_stats)                      */
  int32_t depth;
  int32_t d[EIFMM_MAX_DEPTH + 1];    /* d_k for k = 2..depth (0 elsewhere)        */
  int32_t dpad[EIFMM_MAX_DEPTH + 1]; /* padded row count used on the device       */
  int32_t rank[EIFMM_MAX_DEPTH + 1]; /* M2L compression rank per level (0 = none) */
  double eim_err[EIFMM_MAX_DEPTH + 1]; /* final training error / scale per level  */
  double setup_ms;                   /* plan_create host time                     */
  double phase_ms[EIFMM_NPHASE];     /* accumulated GPU time per phase            */
  int64_t phase_calls[EIFMM_NPHASE]; /* timed launches of each phase              */
  double m2l_flops;                  /* algorithmic M2L flops of the last evaluate
                                        (2 d_k^2, or 2 r_k^2 when compressed, per
                                        interaction pair per RHS)                 */
  double proj_flops;                 /* compression projections of the last
                                        evaluate (4 d_k r_k per box per RHS)      */
  int64_t active_boxes[EIFMM_MAX_DEPTH + 1]; /* non-empty boxes per level        */
  int64_t il_pairs[EIFMM_MAX_DEPTH + 1];     /* interaction-list pairs per level */
  int64_t near_pairs;                /* ordered leaf pairs in the near lists      */
  int32_t hip_error;                 /* last hipError_t seen (0 = none)           */
  int32_t scale_level;               /* tol_mode 1: the level whose training max |K|
                                        scales every stopping rule; 0 otherwise   */
  int64_t near_point_pairs;          /* ordered point pairs (targets x sources) of
                                        the near field, self pairs included      */
  int32_t d2[EIFMM_MAX_DEPTH + 1];   /* d of the second EIM per level (the size of
                                        g, l and lhat), 0 with one EIM           */
  int32_t rpad[EIFMM_MAX_DEPTH + 1]; /* compressed levels: the rank padded to whole
                                        16-row MFMA blocks, as the device runs it */
  int32_t near_mode;                 /* where the last evaluate ran the near
                                        field: 0 on the caller's stream; 1 on the
                                        plan's second stream from P2M on; 2 there
                                        from the M2L on                          */
  double m2l_flops_exec;             /* M2L flops the MFMAs of the last evaluate
                                        execute: padded rows and columns (rpad or
                                        dpad), and every one of the 189 offsets of
                                        a box's child class, sources outside the
                                        domain included                          */
} eifmm_stats;

/* Per-level EIM plan: runs Algorithm 1 for k = 2..depth on the training sets,
 * factors K(X^k, Y^k) = Gamma B^T (the Delta = B^{-T} Gamma^{-1} of eq. (5)),
 * builds the 8 M2M and 8 L2L operators per level by triangular solves (Sec. 4.1)
 * and the 316 translation-invariant M2L matrices per level (Sec. 4.2), then
 * uploads them and allocates workspaces for n points and max_rhs.  *out is set
 * only on success. */
int eifmm_plan_create(const eifmm_config *cfg, eifmm_plan *out);

/* Builds the octree for n points xyz (device, 3 x n SoA FP64): Morton keys of
 * the leaf cells, a stable sort by (key, input index), Morton-ordered copies,
 * leaf ranges, active boxes per level and the near lists.  Returns
 * EIFMM_EDOMAIN if a point is outside [lo, lo+L]^3 or not finite (the plan then
 * has no points).  Waits for the box counts (see the conventions above). */
int eifmm_set_points(eifmm_plan plan, const double *xyz_dev, void *hip_stream);

/* For a plan with n_targets > 0: builds one octree over the n sources
 * src_xyz_dev and the n_targets targets tgt_xyz_dev (both device, SoA FP64),
 * sorted by (leaf key, source before target, input index), so that every leaf
 * holds its sources, then its targets.  Boxes are those with any point; P2M and
 * the near field read the sources of a leaf, L2P and the near field write its
 * targets (eq. (13) with x_i a target).  A target that coincides with a source
 * skips that pair for singular kernels, as a source does with itself.  Errors
 * as eifmm_set_points; EIFMM_EINVAL on a plan with n_targets == 0 (and
 * eifmm_set_points is EIFMM_EINVAL on a plan with n_targets > 0). */
int eifmm_set_points_targets(eifmm_plan plan, const double *src_xyz_dev, const double *tgt_xyz_dev,
                             void *hip_stream);

/* f = K sigma for nrhs right-hand sides: sigma_dev (n x nrhs, column-major,
 * leading dimension ld >= n) in input order; f_dev (m x nrhs, leading dimension
 * ldf >= m, m = n_targets if > 0, else n) is overwritten in input order.
 * Requires set_points (set_points_targets); nrhs <= max_rhs.  The work is
 * ordered on hip_stream: the near field runs on a second stream owned by the
 * plan, forked from and joined back to hip_stream with events, so completion
 * of hip_stream's work implies completion of the pass.  Calls on one plan must
 * not overlap (they share its workspaces). */
int eifmm_evaluate(eifmm_plan plan, const double *sigma_dev, int32_t nrhs, int64_t ld,
                   double *f_dev, int64_t ldf, void *hip_stream);

/* eifmm_evaluate for callers that cannot allocate device memory during the call
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same pass and arguments, with no hipMalloc, hipFree or other
 * allocating call.  The plan's expansions and tables were allocated by
 * eifmm_plan_create; the partial tiles of the Stream-K tails of the gathered-GEMM
 * launches, which eifmm_evaluate keeps in a workspace of the plan, go to a
 * device array of the library instead: 32 MiB per device, held until the
 * process ends, each launch splitting its tail over as many workgroups as fit
 * it.  Every call on a device shares that array, so calls that overlap in time
 * on one device (on different streams or from different threads, any plans)
 * race and must be serialised by the caller; each launch writes every piece
 * it reads, so nothing must be cleared between calls.  Per-phase timing is not
 * recorded.  Errors as eifmm_evaluate, plus EIFMM_EINVAL for a plan with the
 * second compression stage (its factored M2L keeps a workspace of its own) and
 * EIFMM_EHIP if the array's device address cannot be obtained.  Results equal
 * eifmm_evaluate's up to the order in which split tiles are summed. */
int eifmm_evaluate_noalloc(eifmm_plan plan, const double *sigma_dev, int32_t nrhs, int64_t ld,
                           double *f_dev, int64_t ldf, void *hip_stream);

/* Enables per-phase HIP-event timing (1: every phase; 2: the M2L launch only, two
 * events per evaluation) or disables it (0); resets the totals. */
int eifmm_set_timing(eifmm_plan plan, int32_t enable);

/* Copies statistics (waits for pending timed work). */
int eifmm_get_stats(eifmm_plan plan, eifmm_stats *out);

/* Host copies of level k's EIM data: d, X (I_0 points) and Y (J_0 points) as
 * d x 3 physical coordinates, training indices ia/ib, B and Gamma (d x d
 * row-major).  Any output may be NULL; call with all NULL to get d. */
int eifmm_get_level(eifmm_plan plan, int32_t k, int32_t *d, double *X, double *Y, int64_t *ia,
                    int64_t *ib, double *B, double *Gamma);

/* The same for the second EIM of level k (Sec. 3.1: D_x = J_0, D_y = I_0, so X
 * holds J_0 points and Y holds I_0 points; its Delta is Delta^{J_0,I_0}).
 * EIFMM_EINVAL for a plan with one EIM per level. */
int eifmm_get_level2(eifmm_plan plan, int32_t k, int32_t *d, double *X, double *Y, int64_t *ia,
                     int64_t *ib, double *B, double *Gamma);

/* Host copies of level k's M2L compression (Sec. 4.2): *r (0 when off), the
 * singular values of K_fat = [K^delta_1 .. K^delta_316] in descending order, and
 * U (row-major: the kept left singular vectors, r columns).  K^delta has one row
 * per M2L row point: d_k of them with one EIM per level, the second EIM's size
 * with two (then the columns are projected on the right singular vectors of the
 * stacked matrices, which stay internal).  Outputs may be NULL. */
int eifmm_get_compression(eifmm_plan plan, int32_t k, int32_t *r, double *sv, double *U);

/* The ranks s of the second compression stage of level k, one per M2L offset
 * (316, offset-id order; all 0 when the stage is off). */
int eifmm_get_compression2(eifmm_plan plan, int32_t k, int32_t *s);

/* Host copies of the current tree: perm[n] (input index of each Morton-ordered
 * point), leaf_start[8^depth + 1], keys[n] (leaf key of each sorted point).
 * With separate targets the arrays cover n + n_targets points; perm holds n + t
 * for target t. */
int eifmm_export_tree(eifmm_plan plan, int32_t *perm, int64_t *leaf_start, uint32_t *keys);

/* Builds (on the device) and copies the lists of `level`: active boxes in key
 * order, near lists (Chebyshev distance <= 1) and, for level >= 2, interaction
 * lists with offset ids (rank of (dx+3)+7(dy+3)+49(dz+3) among the 316 offsets),
 * each sorted by source key.  Capacities: active 8^level, near 27 * 8^level,
 * il 189 * 8^level.  *nactive receives the active count. */
int eifmm_export_lists(eifmm_plan plan, int32_t level, int64_t *nactive, uint32_t *active,
                       int64_t *near_ptr, uint32_t *near_src, int64_t *il_ptr, uint32_t *il_src,
                       int16_t *il_off);

/* Host copy of one expansion of the last evaluate, right-hand side `rhs`, as a
 * dense 8^k x d_k array in key order (zeros for empty boxes).  which: 0 = W,
 * 1 = What (= Delta W), 2 = g (M2L output), 3 = l, 4 = lhat (level depth only);
 * with two EIMs per level, g, l and lhat have the second EIM's d_k values.
 * With M2L compression the pass applies the factor B^{-T} of Delta = B^{-T}
 * Gamma^{-1} inside the projection (What' = U^T B^{-T} (Gamma^{-1} W)), so What
 * of a compressed level is computed by this call, on the device, from W. */
int eifmm_export_expansion(eifmm_plan plan, int32_t which, int32_t k, int32_t rhs, double *out);

/* Releases the plan and all its device memory. */
int eifmm_plan_destroy(eifmm_plan plan);

/* ------------------------------------------------------------------ batches
 * Many independent problems, each the paper's problem (Sec. 1: its own points,
 * sigma, N, kernel and depth), evaluated together.  Every step of Algorithm 3
 * and the near field runs as one launch over all problems (once per kernel
 * kind for the leaf-level steps); the resulting fixed launch sequence is
 * captured once into a HIP graph and replayed by eifmm_batch_evaluate.
 *
 * Problems whose configurations agree on kernel, kernel_param, lo, L, eim_tol,
 * tol_mode, dmax, compress_tol and precision share one set of level tables
 * (Algorithm 1 and the operators of Sec. 3 and 4 depend on nothing else),
 * built down to the deepest level any of them may use; with tol_mode 1 the
 * absolute scale is that deepest level's.  All problems of a batch use one
 * precision; max_rhs must be 1; depth is 2..EIFMM_MAX_DEPTH, or -1 to let the
 * autotuner of eifmm_batch_set_points choose it.  A batch is not thread-safe. */
typedef struct eifmm_batch_s *eifmm_batch;

typedef struct {
  int32_t struct_size;  /* sizeof(eifmm_batch_info)                          */
  int32_t nprob;        /* problems                                          */
  int32_t ntables;      /* distinct level-table sets                         */
  int32_t graph_nodes;  /* nodes of the captured graph (0 before the first
                           evaluation after set_points)                      */
  int32_t m2l_rbt;      /* chosen M2L tile height, in 16-row MFMA blocks     */
  int32_t reserved0;
  double m2l_flops;     /* 2 r_k^2 per interaction pair, summed over problems */
  double tune_ms;       /* host time spent autotuning (depths, M2L tiles)    */
  double setup_ms;      /* host time of eifmm_batch_create (tables)          */
  double reserved[4];
} eifmm_batch_info;

/* cfgs: nprob configurations (host memory, copied; n may be 0).  Builds and
 * uploads the shared level tables.  Errors as eifmm_plan_create, and
 * EIFMM_EINVAL for nprob < 1, differing precisions, max_rhs != 1, the host-only
 * flag, n_targets != 0, or depth outside {-1, 2..EIFMM_MAX_DEPTH}.  On error
 * *out is NULL. */
int eifmm_batch_create(const eifmm_config *cfgs, int32_t nprob, eifmm_batch *out);

/* xyz[p]: device pointer to problem p's 3 x n_p SoA points (may be NULL when
 * n_p = 0).  Builds every tree (synchronises the host with `stream`, like
 * eifmm_set_points).  At the first call, a problem with depth -1 gets, among
 * the depths around log8(n_p / 32) (at most 4 of them, within 2..8), the one
 * whose evaluation runs fastest here; later calls keep it.  The first call also
 * times the fused M2L launch with tiles of 3, 4, 5 and 6 MFMA row blocks and keeps
 * the fastest.  Drops the captured graph.  Errors as eifmm_set_points; after
 * an error the batch must get points again before evaluating. */
int eifmm_batch_set_points(eifmm_batch b, const double *const *xyz, void *stream);

/* sigma[p], f[p]: device pointers to n_p doubles each, input order (f is
 * overwritten).  Copies the pointer table to the device on `stream` and
 * replays the graph of the fused pass there (capturing it at the first call
 * after set_points).  Asynchronous.  EIFMM_ESTATE before set_points, EIFMM_EHIP
 * if capture or launch fails. */
int eifmm_batch_evaluate(eifmm_batch b, const double *const *sigma, double *const *f,
                         void *stream);

/* The same results without fusion or graph: each problem's own pass, one
 * after another on `stream` (the launches eifmm_evaluate makes).  For
 * measuring what the fused launches and the graph save, and for debugging. */
int eifmm_batch_evaluate_unfused(eifmm_batch b, const double *const *sigma, double *const *f,
                                 void *stream);

/* eifmm_export_expansion for problem p of the batch (right-hand side 0) after
 * an evaluation, fused or not. */
int eifmm_batch_export_expansion(eifmm_batch b, int32_t p, int32_t which, int32_t k,
                                 double *out);

/* Statistics of problem p (depth in use, d_k, ranks, counts, setup time of
 * its table set); EIFMM_EINVAL before its first set_points. */
int eifmm_batch_get_stats(eifmm_batch b, int32_t p, eifmm_stats *out);

/* Batch-wide information (out->struct_size must be set). */
int eifmm_batch_get_info(eifmm_batch b, eifmm_batch_info *out);

/* Releases the batch, its plans, tables, graph and device memory. */
int eifmm_batch_destroy(eifmm_batch b);

/* Static description of a status code. */
const char *eifmm_status_str(int status);

#ifdef __cplusplus
}
#endif
#endif /* EIFMM_H */
