// plan.hpp -- internal state of an EIFMM plan (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/eifmm.h"

namespace eifmm {

constexpr int kMaxLevels = EIFMM_MAX_DEPTH + 1;
// deepest level whose M2L columns are ordered by boundary faces (8^6 boxes)
constexpr int kMaxOrderLevel = 6;
constexpr int kNumOffsets = 316;  // 7^3 - 3^3 distinct M2L offsets (Sec. 4.2)
constexpr int kMaxRank2 = 96;     // largest second-stage rank the factored M2L takes
constexpr int kM2l2RbMin = 4, kM2l2RbMax = 16;  // 16-row blocks of r the factored M2L takes

// Host copy of one level's EIM data (Algorithm 1 and the factors of eq. (5)).
struct LevelHost {
  int d = 0;   // number of interpolation points d_k
  int dp = 0;  // d rounded up to a multiple of 16 (MFMA row blocks)
  // size of the local expansions g, l, lhat: the second EIM's d (kernels that
  // are not symmetric, Sec. 3.1), else d
  int dB = 0, dpB = 0;
  std::vector<double> XL;       // L2P points y^{I_0} (dB x 3): the second EIM's Y, else X
  double scale = 0, err = 0;
  std::vector<double> X, Y;     // d x 3, physical units: X in I_0^k, Y in J_0^k
  std::vector<int64_t> ia, ib;  // training-set indices of X and Y
  std::vector<double> B, G;     // d x d row-major: unit-lower B and lower Gamma
  // operator tables, padded to dp and laid out for the device (see setup.cpp)
  std::vector<double> kfrag;    // 316 M2L matrices K^delta, fragment order
  std::vector<double> m2m;      // level k < depth: 8 ops d_k x d_{k+1}, fragment order
  std::vector<double> l2l;      // level k < depth: 8 ops d_{k+1} x d_k, fragment order
  std::vector<double> tri[4];   // solve tables: Gamma, B^T, B, Gamma^T (setup.cpp)
  // M2L compression (Sec. 4.2): rank r (0 = off), padded rp; C^delta = U^T K^delta U
  int r = 0, rp = 0;
  std::vector<double> sv;       // singular values of [K^delta_1 .. K^delta_316]
  std::vector<double> U;        // dB x r, row-major: basis of the M2L rows (g) space
  std::vector<double> V;        // d x r basis of the columns' space (two EIMs; else V = U)
  std::vector<double> ufrag;    // U          (dpB x rp), fragment order: g = U g'
  std::vector<double> pfrag;    // V^T B^{-T} (rp x dp), fragment order: What' = V^T B^{-T} Gamma^{-1} W
  // pfrag holds V^T B^{-T} Gamma^{-1} (the pre-projection then reads W itself and the
  // pass takes no What solve on this level): plans with their own tables and one EIM
  bool fold_what = false;
  // second compression stage (Sec. 4.2): rank s2[o] of each C^delta (empty: off),
  // padded rank sp2[o] (multiple of 16, 0 when s2[o] = 0; empty when a rank exceeds
  // what the factored M2L takes, and the dense product serves) and the factors in
  // operand fragment order, offset after offset: vf2 = Vt (sp x rp, the k order of
  // the gathered loads), uf2 = Ut (rp x sp, the k order of MFMA results)
  std::vector<int> s2, sp2;
  // M2M / L2L operators of this (parent) level before their solves, for the device
  // solves: kernel rows padded to the child's dp (M2M, 8 d rows) and to this level's
  // dpB (L2L, 8 d_B(child) rows); with two EIMs also the solve tables they need
  // (M2M: the child's first-EIM B, Gamma^T; L2L: this level's B_B, Gamma_B^T)
  std::vector<double> m2m_rows, l2l_rows, op_tri[4];
  std::vector<int64_t> voff2, uoff2;
  std::vector<double> vf2, uf2;
};

// Device copy of one level's tables.
struct LevelDev {
  double *kfrag = nullptr;
  float *kfrag32 = nullptr;
  double *m2m = nullptr, *l2l = nullptr;
  double *tri[4] = {nullptr, nullptr, nullptr, nullptr};
  double *X = nullptr;   // d x 3 (leaf level: P2M)
  double *XL = nullptr;  // dB x 3 (leaf level: L2P); = X with one EIM
  // per-query workspaces
  size_t cap = 0;        // max active boxes at this level: min(8^k, n)
  uint32_t *act = nullptr;   // active box keys, ascending
  int *slot = nullptr;       // [8^k] slot of each key, -1 if empty
  int *cls = nullptr;        // slots grouped by child class (key & 7), ascending key
  // M2L target order: each class's slots grouped by which faces of the domain
  // the parent touches (so that a 16-column block shares its missing sources),
  // ascending key within a group; levels up to kMaxOrderLevel, else null
  int *ord = nullptr;
  double *W = nullptr, *Wh = nullptr, *g = nullptr, *l = nullptr;
  float *Wh32 = nullptr;  // FP32 copy of What (mixed precision M2L)
  // compressed M2L
  double *ufrag = nullptr, *pfrag = nullptr;
  // second compression stage (null: off)
  const int *sp2 = nullptr;
  const int64_t *voff2 = nullptr, *uoff2 = nullptr;
  const double *vf2 = nullptr, *uf2 = nullptr;
  double *Whp = nullptr, *gp = nullptr;  // What' = U^T What and g' (rp per box and RHS)
  float *Whp32 = nullptr;
};

// Packed M2L jobs of a batch: the columns of one job belong to several problems
// that share the level's operators; each column names its problem's arrays.
struct ColSrc {
  const uint32_t *keys;  // active keys of the level
  const int *slot;       // slot map of the level
  const void *B;         // source expansions (What or What')
  double *C;             // output (g or g')
};
struct ColRef {
  int rec;   // ColSrc record
  int slot;  // target slot
};

// One target group of a gathered GEMM launch (see pass.hip).
struct GemmJob {
  const void *A;        // fragment-ordered operand(s)
  const void *Bsrc;     // source expansions [slot * nrhs + r][dpk]
  double *C;            // output [slot * nrhs + r][dpm]
  float *C32;           // optional FP32 copy of the output
  const double *Cadd;   // added to the product (L2L: g), may be null
  const int *tgt;       // target slots
  const uint32_t *tgt_keys;  // active keys of the target level (indexed by slot)
  const int *src_slot;  // slot map of the source level (indexed by key)
  const int16_t *terms; // M2L: offset ids of the class; null otherwise
  int64_t a_stride;     // elements per operand matrix
  int ntgt, nterms, dpm, dpk;
  int level, cls, mode, nrhs;
  int tiles_start, ncoltiles, nrowtiles, src_level;
  int64_t units_start;  // first (tile, term) unit of the job within its launch
  const ColRef *colref;  // packed M2L: per target column (tgt, tgt_keys, src_slot,
  const ColSrc *colsrc;  // Bsrc and C unused); null otherwise
};

// One problem's leaf level as the near-field, P2M and L2P kernels read it.
struct LeafDesc {
  const uint32_t *act;      // active leaf keys
  const int *ls;            // leaf_start: points of leaf `key` are [ls[key], ls[key + 1])
  const int *se;            // sources of leaf key: [ls[key], se[key])
  const int *tb;            // targets of leaf key: [tb[key], ls[key + 1])
  const int *chunk_ptr;     // first 32-target chunk of each active leaf
  const int *near_ptr, *near_src;
  const int *perm;          // sorted position -> input index
  const double *xyz;        // sorted points
  const double *X;          // leaf-level EIM points X (d x 3): P2M
  const double *XL;         // leaf-level L2P points (dL x 3)
  const double *lhat;
  double *sig, *fnear, *W;  // sorted sigma, near field, leaf W
  int64_t n;
  int64_t nsrc;             // input indices below nsrc are sources (sigma rows)
  int64_t toff;             // target t has input index toff + t (f row t)
  int nleaf, nrhs, d, dp;
  int dL, dpL;              // size of lhat (L2P)
  double lo0, lo1, lo2, h, p;  // domain corner, leaf width, device kernel parameter
  int64_t chunk_base, leaf_base, pt_base;  // batch launches: first chunk / leaf / element
};

// Caller buffers of one evaluation: sigma (input order, column stride ld) and f.
struct IoDesc {
  const double *sigma;
  int64_t ld;
  double *f;
  int64_t ldf;
};

// A gathered-GEMM launch assembled from the jobs of several plans.
struct FusedGemm {
  GemmJob *dev = nullptr;
  int n = 0, tiles = 0, rbt = 6;
  int64_t units = 0;
};

// One (problem, level) of a blocked triangular-solve launch: columns of `in`
// (dp doubles each) solved into `out` (and an optional FP32 copy) with the
// fragment tables Tf (forward) and Tb (backward); blk_start = first workgroup.
struct SolveDesc {
  const double *in;
  double *out;
  float *out32;
  const double *Tf, *Tb;
  int ncols, dp, blk_start, pad;
};

// Problems of one kernel kind inside a batch (contiguous descriptor range).
struct BatchGroup {
  int kind = 0;
  int first = 0, count = 0;
  int64_t nchunk = 0, nleaf = 0;
  int dpmax = 0;
};

// The fused pass of a batch of plans: one launch per phase over all problems
// (per kernel kind for the leaf-level kernels).  Built by batch_prepare once the
// trees are known, replayed by batch_run.
struct BatchExec {
  int nprob = 0, maxdepth = 0;
  bool mixed = false;
  int64_t total_pts = 0;
  std::vector<int> order;          // descriptor slot -> problem index
  std::vector<BatchGroup> groups;
  LeafDesc *leaf_dev = nullptr;    // [nprob] in descriptor order
  IoDesc *io_dev = nullptr;        // [nprob] in descriptor order, written per evaluation
  SolveDesc *what_dev = nullptr, *lhat_dev = nullptr;
  int what_n = 0, what_blk = 0, lhat_n = 0, lhat_blk = 0;
  size_t what_shm = 0, lhat_shm = 0;
  FusedGemm m2m[kMaxLevels], l2l[kMaxLevels], pre, m2l, post;
  int sk_groups = 0;
  double *sk_ws = nullptr;
  const int8_t *dvec = nullptr;
  double m2l_flops = 0;
  std::vector<void *> track;       // device allocations of the tables above
};

// Factored M2L (second compression stage, Sec. 4.2) of one (level, child class):
// g'[:, col] += Ut_o (Vt_o What'[:, src(col, o)]) over the class's offsets o.
// Its 64-column tiles are split into kM2l2Parts term ranges (work items), each
// summed into its own workspace block and added up in part order afterwards.
constexpr int kM2l2Parts = 3;
struct M2l2Job {
  const int *tgt;             // target slots of the class
  const uint32_t *keys;       // active keys of the level (by slot)
  const int *slot;            // slot map of the level (by key)
  const double *B;            // What' [slot * nrhs + r][rp]
  double *C;                  // g'    [slot * nrhs + r][rp]
  const int16_t *terms;       // the class's 189 offset ids
  const double *vf, *uf;      // factor fragments of the level
  const int64_t *voff, *uoff; // first element of each offset's fragments
  const int *sp;              // padded rank of each offset (multiple of 16, 0 = none)
  int ntgt, nrhs, level, rp;
  int item_start, tile_start, ntiles;
};
struct M2l2Launch {           // jobs sharing rp (one kernel instance)
  int first_job, njobs, first_item, nitems, first_tile, ntiles, rb;
  size_t ws_off;              // first workspace element of its items
};

// Index ranges of the gathered-GEMM jobs of one (points, nrhs) pair.
struct JobTables {
  int nrhs = -1;
  int m2m_first[kMaxLevels] = {}, m2m_n[kMaxLevels] = {}, m2m_tiles[kMaxLevels] = {};
  int l2l_first[kMaxLevels] = {}, l2l_n[kMaxLevels] = {}, l2l_tiles[kMaxLevels] = {};
  int m2m_rbt[kMaxLevels] = {}, l2l_rbt[kMaxLevels] = {};
  int64_t m2m_units[kMaxLevels] = {}, l2l_units[kMaxLevels] = {};
  int64_t m2l_units = 0, pre_units = 0, post_units = 0;
  int m2l_first = 0, m2l_n = 0, m2l_tiles = 0, m2l_rbt = 6;
  int pre_first = 0, pre_n = 0, pre_tiles = 0, pre_rbt = 6;     // What' = U^T B^{-T} z
  int post_first = 0, post_n = 0, post_tiles = 0, post_rbt = 6; // g = U g'
};

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  int phase = 0;
};

struct Plan {
  eifmm_config cfg{};
  int device = 0;
  bool host_only = false;
  bool gpu_setup = false;  // Algorithm 1 iterations on the device
  bool gpu_ops = false;    // M2M / L2L operator solves on the device
  bool two_eim = false;    // second EIM per level (lhB): kernels that are not symmetric
  bool shared_tables = false;  // tables of a batch, used by problems of several depths
  // one EIM, compressed leaf level, own tables: the leaf's B^{-1} is folded into its
  // post-projection (U -> B^{-1} U) and into the L2L operators into it, so that the
  // leaf's g and l hold B^{-1} g and B^{-1} l and lhat takes the Gamma^T solve only
  bool fold_leaf = false;
  LevelHost lhB[kMaxLevels];  // the second EIM (D_x = J_0, D_y = I_0): X in J_0, Y in I_0
  int depth = 0;
  LevelHost lh[kMaxLevels];
  LevelDev ld[kMaxLevels];
  double setup_ms = 0;

  // tree / points (device).  With separate targets the tree holds n = ns + nt
  // points: input index i < ns is source i, ns + t is target t.
  int64_t n = 0;
  int64_t ns = 0, nt = 0;       // sources; separate targets (0: targets = sources)
  double *xin = nullptr;        // separate targets: sources then targets, SoA 3 x n
  int *tgt_begin = nullptr;     // separate targets: first target of each leaf [8^depth + 1]
  int ntiles_sort = 0;
  double *xyz = nullptr;        // sorted points, SoA 3 x n
  double *xyz4 = nullptr;       // tree build staging: (x, y, z, 0) per point, input order [4 n]
  uint32_t *keys = nullptr, *keys_tmp = nullptr;
  int *idx = nullptr, *idx_tmp = nullptr;  // idx = perm after the sort
  unsigned *hist = nullptr;
  int *leaf_start = nullptr;    // [8^depth + 1]
  int *scan_tmp = nullptr;       // block totals of the prefix sums
  int *blkcnt = nullptr;         // per-block counts of the active-box compaction
  int *list_cnt = nullptr;       // per-box entry counts of a list build
  int *counts_dev = nullptr;    // small counter block
  int *errflag = nullptr;       // counts_dev + 16 kMaxLevels
  int *counts_pin = nullptr;    // pinned host copy of counts_dev and errflag
  int *near_ptr = nullptr;      // leaf level near lists (CSR over active slots)
  int *near_src = nullptr;      // source leaf slots
  size_t near_cap = 0;
  int *chunk_ptr = nullptr;     // per active leaf: first 32-target chunk (prefix sum)
  int64_t nchunk = 0;           // bound on the 32-target chunks over all leaves
  unsigned long long *npairs_dev = nullptr;  // near-field work counters (2)
  int64_t near_point_pairs = 0;  // target x source point pairs of the near field
  int64_t near_lane_pairs = 0;   // the same with targets rounded up to 32-target chunks
  bool counts_pending = false;   // the three counts above are still on the device
  bool points_set = false;
  int64_t nact[kMaxLevels] = {0};
  int64_t cls_off[kMaxLevels][9] = {{0}};
  int64_t near_total = 0;
  int64_t il_pairs[kMaxLevels] = {0};
  // interaction-pair counts (statistics: M2L flops) counted on demand, when the
  // statistics are read, instead of with every tree (il_lazy); il_pending: the
  // current tree's counts are not taken yet
  bool il_lazy = false, il_pending = false;

  // per-evaluate buffers
  int max_rhs = 1;
  double *sig = nullptr;    // sorted sigma [n][nrhs]
  double *fnear = nullptr;  // near field [n][nrhs]
  double *lhat = nullptr;   // leaf level [slot][nrhs][dp]
  int16_t *dlist = nullptr; // [8][189] offset ids per child class
  int8_t *dvec = nullptr;   // [316][3]
  int16_t *code2id = nullptr; // [343] (dx+3)+7(dy+3)+49(dz+3) -> offset id or -1

  // gathered-GEMM job tables (rebuilt when the points or nrhs change)
  JobTables jobs;
  GemmJob *job_dev = nullptr;
  // factored M2L (second compression stage), FP64 passes
  std::vector<M2l2Job> m2l2_host;
  std::vector<M2l2Launch> m2l2_launch;
  M2l2Job *m2l2_dev = nullptr, *m2l2_pin = nullptr;
  size_t m2l2_cap = 0;
  double *m2l2_ws = nullptr;       // partial sums, one rp x 64 block per work item
  size_t m2l2_ws_cap = 0;          // in doubles
  size_t job_cap = 0;             // jobs job_dev and job_pin hold
  GemmJob *job_pin = nullptr;     // pinned staging copy of the job table
  hipEvent_t job_evt = nullptr;   // recorded after the last copy from job_pin
  hipEvent_t ev_counts = nullptr; // recorded after the tree's counts are copied to counts_pin
  // second stream of the pass: the near field runs on it beside the upward pass
  // (fork after the potentials are gathered, join before L2P)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int near_mode = 0;  // the last pass's near-field placement (eifmm_stats.near_mode)
  std::vector<GemmJob> jobs_host;  // host copy of the job table (batches concatenate it)
  int sk_groups = 512;       // persistent workgroups of a gathered-GEMM launch
  double *sk_ws = nullptr;   // Stream-K pieces and tail counter, stream_k_ws_len doubles
  // a Stream-K workspace lent for one pass (null: sk_ws), run_ws_len doubles
  double *run_ws = nullptr;
  size_t run_ws_len = 0;
  double m2l_flops = 0, proj_flops = 0;
  double m2l_flops_exec = 0;  // what the M2L MFMAs execute (padding, empty sources)

  // stats
  int timing = 0;  // per-phase events: 0 off, 1 every phase, 2 the M2L launch only
  std::vector<EventPair> ev_free, ev_pending;
  double phase_ms[EIFMM_NPHASE] = {0};
  int64_t phase_calls[EIFMM_NPHASE] = {0};
  int last_hip_error = 0;
  int last_rhs = 0;
};

// Stream-K workspace of `groups` persistent workgroups: 2 pieces of the largest
// tile (6 x 16 x 128 doubles) each
// (2 pieces per workgroup for the even split, and room for the M2L tail's finer
// pieces: 4 tiles of 6 x 16 x 128 doubles per workgroup, 201 MB for 512 groups)
inline size_t stream_k_ws_len(int groups) { return (size_t)4 * groups * 6 * 16 * 128; }
// the last doubles of a Stream-K workspace hold the gathered GEMM's tail counter
// (zero when the workspace is made)
constexpr size_t kCounterDoubles = 32;
// gathered-GEMM jobs a plan of this depth can have: M2M and the two projections
// one per level, M2L and L2L one per level and child class
inline size_t max_gemm_jobs(int depth) { return (size_t)19 * (depth > 0 ? depth : 1) + 16; }

// setup.cpp
int build_tables(Plan &P);
// Algorithm 1 iterations on the device (eim_gpu.hip): training matrix R (nx x ny,
// row-major), stopping rule |pivot| <= tau scale with scale = abs_scale if > 0,
// else the first pivot's magnitude; at most dmax points (then EIFMM_EEIM)
struct EimResult {
  std::vector<int64_t> ia, ib;  // selected rows / columns
  double scale = 0, emax = 0;   // scale, largest |residual| left
  int status = EIFMM_OK;
};
int eim_iterate_gpu(const std::vector<double> &R, int64_t nx, int64_t ny, double tau,
                    double abs_scale, int dmax, EimResult &res);
int pick_rbt(int nrb);

// device-side entry points (tree.hip, pass.hip)
int tree_build(Plan &P, const double *xyz_in, hipStream_t s);
int tree_counts(Plan &P);
int lists_export(Plan &P, int level, int64_t *nactive, uint32_t *active, int64_t *near_ptr,
                 uint32_t *near_src, int64_t *il_ptr, uint32_t *il_src, int16_t *il_off);
int build_jobs(Plan &P, int nrhs, hipStream_t s);
void timing_drain(Plan &P);
int pass_run(Plan &P, const double *sigma, int nrhs, int64_t ld, double *f, int64_t ldf,
             hipStream_t s);
// Writes an expansion of the last pass that the pass itself skipped (What of a
// compressed level), on the null stream.
int materialize_expansion(Plan &P, int which, int k);
// algorithmic M2L flops of one evaluation with nrhs right-hand sides, from the
// interaction-pair counts
double m2l_flops_of(const Plan &P, int nrhs);
// solves the M2M / L2L operator rows of parent level k on the device
// (LevelHost::m2m_rows, l2l_rows, solved in place)
int solve_operators_gpu(Plan &P, int k);
// packs the solved rows into the operator tables (fragment order) and frees them
void pack_operators(Plan &P, int k);
// On a compressed level the solve for What stops at z = Gamma^{-1} W: the
// projection applies U^T B^{-T} (pass.hip)
inline bool solves_what(const Plan &P, int k) { return P.lh[k].r == 0; }
// the pass's What phase touches level k (no solve where the pre-projection folds it)
inline bool what_level(const Plan &P, int k) { return !P.lh[k].fold_what; }
// the FP64 pass applies the second compression stage as two factor products
inline bool uses_m2l2(const Plan &P, int k) {
  return P.cfg.precision == EIFMM_PREC_FP64 && P.lh[k].r > 0 && !P.lh[k].sp2.empty();
}
// batches (pass.hip): m2l_rbt <= 0 picks the M2L tile height from the operators
int batch_prepare(BatchExec &B, const std::vector<Plan *> &plans, int m2l_rbt, int sk_groups,
                  double *sk_ws);
void batch_release(BatchExec &B);
// mark: null, or batch_marks(B) events recorded at the phase boundaries: start,
// after the sigma gather, after the near field of each kernel kind, after P2M of
// each kind, after M2M, What, the first projection, M2L, the second projection,
// L2L, lhat, and after L2P of each kind
void batch_run(const BatchExec &B, hipStream_t s, const hipEvent_t *mark = nullptr);
int batch_marks(const BatchExec &B);
void batch_run_m2l(const BatchExec &B, hipStream_t s);

}  // namespace eifmm
