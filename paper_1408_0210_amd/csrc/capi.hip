// capi.hip -- the extern "C" entry points of libeifmm.so (declared in include/eifmm.h).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <chrono>
#include <cstring>
#include <new>
#include <mutex>
#include <vector>

#include "devutil.hpp"
#include "plan.hpp"

using namespace eifmm;

struct eifmm_plan_s {
  Plan P;
  std::vector<void *> track;  // device allocations owned by the plan
};

namespace {

template <typename T>
int dalloc(T **p, size_t count, std::vector<void *> &track) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)p, sizeof(T) * count);
  if (e != hipSuccess) {
    hipGetLastError();
    if (std::getenv("EIFMM_DEBUG"))
      std::fprintf(stderr, "eifmm: hipMalloc(%zu bytes) failed: %s\n", sizeof(T) * count,
                   hipGetErrorString(e));
    return EIFMM_ENOMEM;
  }
  track.push_back((void *)*p);
  return EIFMM_OK;
}

template <typename T>
int upload(T **p, const T *src, size_t count, std::vector<void *> &track) {
  int st = dalloc(p, count, track);
  if (st) return st;
  if (count && hipMemcpy(*p, src, sizeof(T) * count, hipMemcpyHostToDevice) != hipSuccess)
    return EIFMM_EHIP;
  return EIFMM_OK;
}

// the general form of Sec. 3.1 (two EIMs per level)
bool uses_two_eim(const eifmm_config &c) {
  return c.kernel == EIFMM_K_ADVDIFF || (c.flags & EIFMM_FLAG_TWO_EIM);
}

int validate(const eifmm_config *c) {
  if (!c || c->struct_size != (int32_t)sizeof(eifmm_config)) return EIFMM_EINVAL;
  if (c->kernel < EIFMM_K_LAPLACE || c->kernel > EIFMM_K_ADVDIFF) return EIFMM_EINVAL;
  if ((c->kernel == EIFMM_K_GAUSS && !(c->kernel_param > 0)) ||
      (c->kernel == EIFMM_K_MQ && !(c->kernel_param > 0)) ||
      ((c->kernel == EIFMM_K_YUKAWA || c->kernel == EIFMM_K_ADVDIFF) && !(c->kernel_param >= 0)) ||
      !std::isfinite(c->kernel_param))
    return EIFMM_EINVAL;
  if (!(c->L > 0) || !std::isfinite(c->L)) return EIFMM_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(c->lo[a])) return EIFMM_EINVAL;
  if (c->n < 0 || c->n_targets < 0 || c->n > (int64_t)INT32_MAX / 2 ||
      c->n_targets > (int64_t)INT32_MAX / 2 - c->n)
    return EIFMM_EINVAL;
  if (c->depth < 0 || c->depth > EIFMM_MAX_DEPTH) return EIFMM_EINVAL;
  if (c->max_rhs < 1 || c->max_rhs > 4096) return EIFMM_EINVAL;
  if (!(c->eim_tol > 0) || !std::isfinite(c->eim_tol)) return EIFMM_EINVAL;
  if (c->tol_mode < 0 || c->tol_mode > 1) return EIFMM_EINVAL;
  if (c->scale_level != 0 && (c->scale_level < 2 || c->scale_level > EIFMM_MAX_DEPTH))
    return EIFMM_EINVAL;
  if (c->reserved_cfg != 0) return EIFMM_EINVAL;
  if (c->precision != EIFMM_PREC_FP64 && c->precision != EIFMM_PREC_MIXED) return EIFMM_EINVAL;
  // d_k <= 1024: the triangular solves keep a wave's 16 solved columns in LDS
  // (128 dp bytes) and the near-field / L2P launches stage d_k points
  if (c->dmax < 0 || c->dmax > 1024) return EIFMM_EINVAL;
  if (!(c->compress_tol >= 0) || !std::isfinite(c->compress_tol)) return EIFMM_EINVAL;
  if (!(c->compress_tol2 >= 0) || !std::isfinite(c->compress_tol2) ||
      (c->compress_tol2 > 0 && !(c->compress_tol > 0)))
    return EIFMM_EINVAL;
  return EIFMM_OK;
}

}  // namespace

namespace {
std::vector<void *> &owned(eifmm_plan h) { return h->track; }

void release(eifmm_plan h) {
  Plan &P = h->P;
  timing_drain(P);
  for (auto &e : P.ev_free) {
    hipEventDestroy(e.a);
    hipEventDestroy(e.b);
  }
  for (void *p : owned(h)) hipFree(p);
  if (P.side) {
    hipStreamSynchronize(P.side);
    hipStreamDestroy(P.side);
  }
  if (P.ev_fork) hipEventDestroy(P.ev_fork);
  if (P.ev_join) hipEventDestroy(P.ev_join);
  if (P.job_evt) {
    hipEventSynchronize(P.job_evt);
    hipEventDestroy(P.job_evt);
  }
  if (P.ev_counts) {
    hipEventSynchronize(P.ev_counts);
    hipEventDestroy(P.ev_counts);
  }
  if (P.job_dev) hipFree(P.job_dev);
  if (P.job_pin) hipHostFree(P.job_pin);
  if (P.counts_pin) hipHostFree(P.counts_pin);
  if (P.m2l2_dev) hipFree(P.m2l2_dev);
  if (P.m2l2_pin) hipHostFree(P.m2l2_pin);
  if (P.m2l2_ws) hipFree(P.m2l2_ws);
  delete h;
}

int stream_k_groups(int device) {
  int cus = 0;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  return std::max(8, 2 * cus);
}


#define TRY(x)            \
  do {                    \
    if ((st = (x)) != 0) return st; \
  } while (0)

// device copies of the plan's tables (offset lists, per-level operators)
int setup_tables(eifmm_plan h) {
  Plan &P = h->P;
  auto &tr = owned(h);
  const int depth = P.depth;
  const bool mixed = P.cfg.precision == EIFMM_PREC_MIXED;
  int st;
  // offset tables: 316 offsets, per-class lists of 189 (Sec. 3.3.2), code -> id
  {
    std::vector<int8_t> dvec(3 * kNumOffsets);
    std::vector<int16_t> code2id(343, -1), dlist(8 * 189);
    int id = 0;
    for (int code = 0; code < 343; ++code) {
      int dx = code % 7 - 3, dy = (code / 7) % 7 - 3, dz = code / 49 - 3;
      if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) < 2) continue;
      dvec[3 * id] = (int8_t)dx;
      dvec[3 * id + 1] = (int8_t)dy;
      dvec[3 * id + 2] = (int8_t)dz;
      code2id[code] = (int16_t)id;
      ++id;
    }
    for (int c = 0; c < 8; ++c) {
      int q = 0;
      for (int o = 0; o < kNumOffsets; ++o) {
        bool in = true;
        for (int a = 0; a < 3; ++a) {
          int ca = (c >> a) & 1, da = dvec[3 * o + a];
          if (da < -2 - ca || da > 3 - ca) in = false;
        }
        if (in) dlist[189 * c + q++] = (int16_t)o;
      }
      if (q != 189) return EIFMM_EINVAL;
    }
    TRY(upload(&P.dvec, dvec.data(), dvec.size(), tr));
    TRY(upload(&P.code2id, code2id.data(), code2id.size(), tr));
    TRY(upload(&P.dlist, dlist.data(), dlist.size(), tr));
  }
  // level tables
  for (int k = 2; k <= depth; ++k) {
    LevelHost &H = P.lh[k];
    LevelDev &D = P.ld[k];
    if (mixed) {
      std::vector<float> f32(H.kfrag.begin(), H.kfrag.end());
      TRY(upload(&D.kfrag32, f32.data(), f32.size(), tr));
    } else {
      TRY(upload(&D.kfrag, H.kfrag.data(), H.kfrag.size(), tr));
    }
    std::vector<double>().swap(H.kfrag);
    for (int q = 0; q < 4; ++q) TRY(upload(&D.tri[q], H.tri[q].data(), H.tri[q].size(), tr));
    if (k < depth && !P.gpu_ops) {
      TRY(upload(&D.m2m, H.m2m.data(), H.m2m.size(), tr));
      TRY(upload(&D.l2l, H.l2l.data(), H.l2l.size(), tr));
    }
    TRY(upload(&D.X, H.X.data(), H.X.size(), tr));
    if (P.two_eim)
      TRY(upload(&D.XL, H.XL.data(), H.XL.size(), tr));
    else
      D.XL = D.X;
    if (H.r > 0) {
      TRY(upload(&D.ufrag, H.ufrag.data(), H.ufrag.size(), tr));
      TRY(upload(&D.pfrag, H.pfrag.data(), H.pfrag.size(), tr));
      if (!H.sp2.empty()) {
        int *sp = nullptr;
        int64_t *vo = nullptr, *uo = nullptr;
        double *vf = nullptr, *uf = nullptr;
        TRY(upload(&sp, H.sp2.data(), H.sp2.size(), tr));
        TRY(upload(&vo, H.voff2.data(), H.voff2.size(), tr));
        TRY(upload(&uo, H.uoff2.data(), H.uoff2.size(), tr));
        TRY(upload(&vf, H.vf2.data(), H.vf2.size(), tr));
        TRY(upload(&uf, H.uf2.data(), H.uf2.size(), tr));
        D.sp2 = sp;
        D.voff2 = vo;
        D.uoff2 = uo;
        D.vf2 = vf;
        D.uf2 = uf;
        std::vector<double>().swap(H.vf2);
        std::vector<double>().swap(H.uf2);
      }
    }
  }
  // M2M / L2L operators (Sec. 4.1): solved on the device with the solve tables
  // just uploaded, packed on the host, uploaded
  if (P.gpu_ops)
    for (int k = 2; k < depth; ++k) {
      TRY(solve_operators_gpu(P, k));
      pack_operators(P, k);
      TRY(upload(&P.ld[k].m2m, P.lh[k].m2m.data(), P.lh[k].m2m.size(), tr));
      TRY(upload(&P.ld[k].l2l, P.lh[k].l2l.data(), P.lh[k].l2l.size(), tr));
    }
  return EIFMM_OK;
}

// per-query workspaces of a plan: points, tree, lists, expansions; sk_ws, when
// given, is a Stream-K workspace shared with other plans of a batch
int setup_workspaces(eifmm_plan h, double *shared_ws) {
  Plan &P = h->P;
  auto &tr = owned(h);
  const int depth = P.depth;
  const bool mixed = P.cfg.precision == EIFMM_PREC_MIXED;
  const int64_t n = P.n;
  const int R = P.cfg.max_rhs;
  int st;
  // point workspaces
  const int64_t nn = std::max<int64_t>(n, 1);
  P.ntiles_sort = (int)((nn + 1023) / 1024);
  TRY(dalloc(&P.xyz, 3 * nn, tr));
  TRY(dalloc(&P.xyz4, 4 * nn, tr));
  TRY(dalloc(&P.keys, nn, tr));
  TRY(dalloc(&P.keys_tmp, nn, tr));
  TRY(dalloc(&P.idx, nn, tr));
  TRY(dalloc(&P.idx_tmp, nn, tr));
  TRY(dalloc(&P.hist, (size_t)256 * P.ntiles_sort, tr));
  const int64_t nleaf = (int64_t)1 << (3 * depth);
  TRY(dalloc(&P.leaf_start, nleaf + 1, tr));
  if (P.nt) {
    TRY(dalloc(&P.tgt_begin, nleaf + 1, tr));
    TRY(dalloc(&P.xin, 3 * nn, tr));
  }
  size_t maxcap = 1;
  for (int k = 0; k <= depth; ++k) {
    LevelDev &D = P.ld[k];
    const int64_t nb = (int64_t)1 << (3 * k);
    D.cap = (size_t)std::max<int64_t>(1, std::min<int64_t>(nb, n));
    maxcap = std::max(maxcap, D.cap);
    TRY(dalloc(&D.act, D.cap, tr));
    TRY(dalloc(&D.slot, nb, tr));
    TRY(dalloc(&D.cls, D.cap, tr));
    if (k >= 2 && k <= kMaxOrderLevel) TRY(dalloc(&D.ord, D.cap, tr));
  }
  const size_t scan_len = std::max<size_t>((size_t)256 * P.ntiles_sort, maxcap + 2);
  TRY(dalloc(&P.scan_tmp, scan_len / 1024 + 64, tr));
  {
    size_t blocks = 1;  // blocks of 256 boxes over the levels of the active-box compaction
    for (int k = std::min(2, depth); k <= depth; ++k) blocks += ((size_t)1 << (3 * k)) / 256 + 1;
    TRY(dalloc(&P.blkcnt, blocks * 9, tr));
  }
  TRY(dalloc(&P.list_cnt, maxcap + 2, tr));
  // the counter block and, right after it, the tree's error flag (one clear and
  // one copy to the host cover both)
  TRY(dalloc(&P.counts_dev, (size_t)16 * kMaxLevels + 1, tr));
  P.errflag = P.counts_dev + 16 * kMaxLevels;
  P.near_cap = (size_t)27 * P.ld[depth].cap;
  TRY(dalloc(&P.near_ptr, P.ld[depth].cap + 2, tr));
  TRY(dalloc(&P.near_src, P.near_cap, tr));
  TRY(dalloc(&P.chunk_ptr, P.ld[depth].cap + 2, tr));
  TRY(dalloc(&P.npairs_dev, 2, tr));
  TRY(dalloc(&P.sig, (size_t)nn * R, tr));
  TRY(dalloc(&P.fnear, (size_t)nn * R, tr));
  for (int k = 2; k <= depth; ++k) {
    LevelDev &D = P.ld[k];
    const size_t m = D.cap * (size_t)R * (size_t)P.lh[k].dp;
    TRY(dalloc(&D.W, m, tr));
    TRY(dalloc(&D.Wh, m, tr));
    const size_t mr = D.cap * (size_t)R * (size_t)P.lh[k].rp;
    if (P.lh[k].r > 0) {
      TRY(dalloc(&D.Whp, mr, tr));
      TRY(dalloc(&D.gp, mr, tr));
      if (mixed) TRY(dalloc(&D.Whp32, mr, tr));
    } else if (mixed) {
      TRY(dalloc(&D.Wh32, m, tr));
    }
    // g and l have the second EIM's size (the first's with one EIM)
    const size_t mb = D.cap * (size_t)R * (size_t)P.lh[k].dpB;
    TRY(dalloc(&D.g, mb, tr));
    if (k == 2)
      D.l = D.g;  // l^2 = g^2 (Algorithm 3, step 5)
    else
      TRY(dalloc(&D.l, mb, tr));
  }
  P.sk_groups = stream_k_groups(P.device);
  if (shared_ws)
    P.sk_ws = shared_ws;
  else
    TRY(dalloc(&P.sk_ws, stream_k_ws_len(P.sk_groups), tr));
  // the gathered GEMM's tail counter, at the end of the workspace, starts at zero
  if (!shared_ws &&
      hipMemset(P.sk_ws + stream_k_ws_len(P.sk_groups) - kCounterDoubles, 0,
                kCounterDoubles * sizeof(double)) != hipSuccess)
    return EIFMM_EHIP;
  if (depth >= 2)
    TRY(dalloc(&P.lhat, P.ld[depth].cap * (size_t)R * (size_t)P.lh[depth].dpB, tr));
  // the gathered-GEMM job table at its largest size, so that no evaluation
  // allocates (build_jobs grows it only past this bound, which it cannot reach)
  {
    const size_t cap = max_gemm_jobs(depth);
    if (hipMalloc(&P.job_dev, sizeof(GemmJob) * cap) != hipSuccess ||
        hipHostMalloc((void **)&P.job_pin, sizeof(GemmJob) * cap) != hipSuccess ||
        hipHostMalloc((void **)&P.counts_pin, sizeof(int) * (16 * kMaxLevels + 1)) !=
            hipSuccess) {
      hipGetLastError();
      return EIFMM_ENOMEM;
    }
    P.job_cap = cap;
    if (hipEventCreateWithFlags(&P.job_evt, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&P.ev_counts, hipEventDisableTiming) != hipSuccess)
      return EIFMM_EHIP;
  }
#undef TRY
  return EIFMM_OK;
}

}  // namespace

struct eifmm_batch_s {
  std::vector<eifmm_config> cfg;     // as given (depth -1: autotuned)
  std::vector<int> depth;            // depth in use per problem (-1 until chosen)
  std::vector<eifmm_plan> plans;     // one per problem, sharing the level tables
  std::vector<eifmm_plan> tables;    // one per distinct table key
  std::vector<int> table_of;         // problem -> tables index
  BatchExec ex;
  bool ready = false;
  int m2l_rbt = 0;                   // 0 until tuned
  int device = 0;
  int sk_groups = 0;
  double *sk_ws = nullptr;           // Stream-K workspace shared by every launch
  double *scratch = nullptr;         // zero sigma and f for the autotuning runs
  int64_t scratch_n = 0;
  IoDesc *staging = nullptr;         // pinned host copy of the pointer table
  hipEvent_t staged = nullptr;
  hipStream_t cap = nullptr;         // capture stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int graph_nodes = 0;
  double tune_ms = 0, setup_ms = 0;
  // depth autotuning: per problem, the work of each candidate depth
  // (cand_lo + i), and the rates of the fused pass that turn work into time
  bool tuned = false;
  std::vector<int> cand_lo;
  std::vector<std::vector<std::array<double, 4>>> cand;
  double rate_near[EIFMM_K_MQ + 1] = {};  // near-field lane pairs / ms, per kernel kind
  double rate_m2l = 0;                 // M2L flops / ms
  double rate_leaf = 0;                // P2M + L2P kernel evaluations / ms
  double rate_box = 0;                 // box-level d^2 units / ms (M2M, L2L, solves)
};

namespace {

bool same_tables(const eifmm_config &a, const eifmm_config &b) {
  return a.kernel == b.kernel && a.kernel_param == b.kernel_param && a.lo[0] == b.lo[0] &&
         a.lo[1] == b.lo[1] && a.lo[2] == b.lo[2] && a.L == b.L && a.eim_tol == b.eim_tol &&
         a.tol_mode == b.tol_mode && a.dmax == b.dmax && a.compress_tol == b.compress_tol &&
         a.precision == b.precision && (a.tol_mode == 0 || a.scale_level == b.scale_level);
}

// depths the autotuner tries for n points: around log8(n / 32), within 2..8
void depth_candidates(int64_t n, int &lo, int &hi) {
  const double c = std::log(std::max<double>((double)n, 1.0) / 32.0) / std::log(8.0);
  const int k0 = (int)std::lround(c);
  lo = std::max(2, std::min(EIFMM_MAX_DEPTH, k0 - 1));
  hi = std::max(lo, std::min(EIFMM_MAX_DEPTH, k0 + 2));
}

// a plan of problem p at `depth` that uses the batch's level tables
int shared_plan(eifmm_batch b, int p, int depth, eifmm_plan *out) {
  const Plan &T = b->tables[b->table_of[p]]->P;
  eifmm_plan h = new (std::nothrow) eifmm_plan_s();
  if (!h) return EIFMM_ENOMEM;
  Plan &P = h->P;
  P.cfg = b->cfg[p];
  P.cfg.depth = depth;
  // the absolute stopping rule of the shared tables takes its scale from their
  // deepest level unless the configuration names one
  if (P.cfg.tol_mode == 1 && P.cfg.scale_level == 0) P.cfg.scale_level = T.depth;
  P.depth = depth;
  P.n = P.ns = P.cfg.n;
  P.max_rhs = 1;
  P.device = T.device;
  P.setup_ms = 0;
  for (int k = 2; k <= depth; ++k) {
    LevelHost &H = P.lh[k];
    const LevelHost &TH = T.lh[k];
    H.d = TH.d;
    H.dp = TH.dp;
    H.dB = TH.dB;
    H.dpB = TH.dpB;
    H.scale = TH.scale;
    H.err = TH.err;
    H.r = TH.r;
    H.rp = TH.rp;
    LevelDev &D = P.ld[k];
    const LevelDev &TD = T.ld[k];
    D.kfrag = TD.kfrag;
    D.kfrag32 = TD.kfrag32;
    D.m2m = TD.m2m;
    D.l2l = TD.l2l;
    for (int q = 0; q < 4; ++q) D.tri[q] = TD.tri[q];
    D.X = TD.X;
    D.XL = TD.XL;
    D.ufrag = TD.ufrag;
    D.pfrag = TD.pfrag;
    D.sp2 = TD.sp2;
    D.voff2 = TD.voff2;
    D.uoff2 = TD.uoff2;
    D.vf2 = TD.vf2;
    D.uf2 = TD.uf2;
  }
  P.dvec = T.dvec;
  P.code2id = T.code2id;
  P.dlist = T.dlist;
  int st = setup_workspaces(h, b->sk_ws);
  if (st) {
    release(h);
    return st;
  }
  *out = h;
  return EIFMM_OK;
}

// work of one problem's pass at its current depth, in the units of the rates:
// near-field lane pairs, M2L flops (2 r_k^2 per interaction pair), P2M + L2P
// kernel evaluations, and sum over levels of active boxes x d_k^2
std::array<double, 4> work_of(Plan &P) {
  tree_counts(P);
  std::array<double, 4> w{};
  w[0] = (double)P.near_lane_pairs;
  if (P.depth >= 2) {
    for (int k = 2; k <= P.depth; ++k) {
      const double rk = P.lh[k].r > 0 ? P.lh[k].r : P.lh[k].d;
      w[1] += 2.0 * rk * rk * (double)P.il_pairs[k];
      w[3] += (double)P.nact[k] * P.lh[k].d * P.lh[k].d;
    }
    w[2] = 2.0 * (double)P.n * P.lh[P.depth].d;
  }
  return w;
}

// the candidate depth with the smallest modelled time, as an offset from cand_lo
int pick_depth(eifmm_batch b, int p) {
  const int kind = b->cfg[p].kernel;
  int best = 0;
  double tbest = 0;
  for (size_t i = 0; i < b->cand[p].size(); ++i) {
    const auto &w = b->cand[p][i];
    const double t = w[0] / b->rate_near[kind] + w[1] / b->rate_m2l + w[2] / b->rate_leaf +
                     w[3] / b->rate_box;
    if (i == 0 || t < tbest) {
      best = (int)i;
      tbest = t;
    }
  }
  return best;
}

int stage_io(eifmm_batch b, const double *const *sigma, double *const *f, hipStream_t s);

// one fused pass with zero sigma and phase marks; rates = work / time, summed over
// the problems of the batch (keeps the previous rate where a phase had no work)
int calibrate(eifmm_batch b, hipStream_t s) {
  const BatchExec &B = b->ex;
  const int nm = batch_marks(B);
  std::vector<hipEvent_t> ev(nm, nullptr);
  for (auto &e : ev) hipEventCreate(&e);
  int st = stage_io(b, nullptr, nullptr, s);
  if (!st) {
    batch_run(B, s);  // warm-up
    batch_run(B, s, ev.data());
    if (hipEventSynchronize(ev.back()) != hipSuccess) st = EIFMM_EHIP;
  }
  if (!st) {
    const int G = (int)B.groups.size();
    auto dt = [&](int a) {
      float ms = 0;
      hipEventElapsedTime(&ms, ev[a], ev[a + 1]);
      return (double)ms;
    };
    // marks: 0 start, 1 gather, 2..G+1 near, G+2..2G+1 P2M, 2G+2 M2M, 2G+3 What,
    // 2G+4 pre, 2G+5 M2L, 2G+6 post, 2G+7 L2L, 2G+8 lhat, 2G+9.. L2P
    std::array<double, 4> wk[EIFMM_K_MQ + 1] = {};
    double leaf = 0, box = 0, m2l = 0;
    for (int p = 0; p < (int)b->plans.size(); ++p) {
      const auto w = work_of(b->plans[p]->P);
      wk[b->cfg[p].kernel][0] += w[0];
      m2l += w[1];
      leaf += w[2];
      box += w[3];
    }
    double t_leaf = 0;
    for (int g = 0; g < G; ++g) {
      const double t = dt(1 + g);
      if (t > 0 && wk[B.groups[g].kind][0] > 0) b->rate_near[B.groups[g].kind] = wk[B.groups[g].kind][0] / t;
      t_leaf += dt(1 + G + g) + dt(2 * G + 8 + g);
    }
    const double t_box = dt(2 * G + 1) + dt(2 * G + 2) + dt(2 * G + 3) + dt(2 * G + 5) +
                         dt(2 * G + 6) + dt(2 * G + 7);
    const double t_m2l = dt(2 * G + 4);
    if (t_m2l > 0 && m2l > 0) b->rate_m2l = m2l / t_m2l;
    if (t_leaf > 0 && leaf > 0) b->rate_leaf = leaf / t_leaf;
    if (t_box > 0 && box > 0) b->rate_box = box / t_box;
  }
  for (auto &e : ev) hipEventDestroy(e);
  return st;
}

void drop_graph(eifmm_batch b) {
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->graph_nodes = 0;
}

// copy the pointer table (descriptor order) to the device, on stream s
int stage_io(eifmm_batch b, const double *const *sigma, double *const *f, hipStream_t s) {
  if (hipEventSynchronize(b->staged) != hipSuccess) return EIFMM_EHIP;
  const BatchExec &B = b->ex;
  for (int q = 0; q < B.nprob; ++q) {
    const int p = B.order[q];
    const int64_t n = b->cfg[p].n;
    b->staging[q] = IoDesc{sigma ? sigma[p] : b->scratch, n, f ? f[p] : b->scratch + b->scratch_n, n};
  }
  if (hipMemcpyAsync(B.io_dev, b->staging, sizeof(IoDesc) * B.nprob, hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return EIFMM_EHIP;
  hipEventRecord(b->staged, s);
  return EIFMM_OK;
}

int prepare(eifmm_batch b, int rbt) {
  std::vector<Plan *> pl;
  for (auto h : b->plans) pl.push_back(&h->P);
  return batch_prepare(b->ex, pl, rbt, b->sk_groups, b->sk_ws);
}

double elapsed_ms(hipEvent_t a, hipEvent_t c) {
  float ms = 0;
  hipEventSynchronize(c);
  hipEventElapsedTime(&ms, a, c);
  return ms;
}

void batch_free(eifmm_batch b) {
  if (!b) return;
  hipDeviceSynchronize();
  drop_graph(b);
  for (auto h : b->plans)
    if (h) release(h);
  for (auto h : b->tables)
    if (h) release(h);
  batch_release(b->ex);
  if (b->sk_ws) hipFree(b->sk_ws);
  if (b->scratch) hipFree(b->scratch);
  if (b->staging) hipHostFree(b->staging);
  if (b->staged) hipEventDestroy(b->staged);
  if (b->cap) hipStreamDestroy(b->cap);
  delete b;
}

}  // namespace

extern "C" {

int eifmm_plan_create(const eifmm_config *cfg, eifmm_plan *out) {
  if (!out) return EIFMM_EINVAL;
  int st = validate(cfg);
  if (st) return st;
  eifmm_plan h = new (std::nothrow) eifmm_plan_s();
  if (!h) return EIFMM_ENOMEM;
  Plan &P = h->P;
  P.cfg = *cfg;
  P.depth = cfg->depth;
  P.ns = cfg->n;
  P.nt = cfg->n_targets;
  P.n = P.ns + P.nt;
  P.max_rhs = cfg->max_rhs;
  P.host_only = (cfg->flags & EIFMM_FLAG_HOST_ONLY) != 0;
  P.gpu_setup = !P.host_only && !(cfg->flags & EIFMM_FLAG_HOST_SETUP);
  P.gpu_ops = P.gpu_setup;
  P.il_lazy = true;  // a single plan counts its interaction pairs when asked
  P.two_eim = uses_two_eim(*cfg);
  if (!P.host_only) hipGetDevice(&P.device);
  st = build_tables(P);
  if (st == EIFMM_OK && !P.host_only) {
    st = setup_tables(h);
    if (st == EIFMM_OK) st = setup_workspaces(h, nullptr);
    if (st == EIFMM_OK &&
        (hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking) != hipSuccess ||
         hipEventCreateWithFlags(&P.ev_fork, hipEventDisableTiming) != hipSuccess ||
         hipEventCreateWithFlags(&P.ev_join, hipEventDisableTiming) != hipSuccess))
      st = EIFMM_EHIP;
    if (st == EIFMM_OK) {
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) st = EIFMM_EHIP;
    }
  }
  if (st != EIFMM_OK) {
    release(h);
    return st;
  }
  *out = h;
  return EIFMM_OK;
}

namespace {
// tree build over xyz (n points, SoA); with separate targets the sources and
// the targets are first copied into one array (sources first)
int set_points_impl(eifmm_plan h, const double *xyz, const double *tgt, void *stream) {
  Plan &P = h->P;
  hipSetDevice(P.device);
  P.points_set = false;
  P.jobs.nrhs = -1;
  hipStream_t s = (hipStream_t)stream;
  if (P.nt) {
    for (int a = 0; a < 3; ++a) {
      if (P.ns > 0 &&
          hipMemcpyAsync(P.xin + a * P.n, xyz + a * P.ns, sizeof(double) * P.ns,
                         hipMemcpyDeviceToDevice, s) != hipSuccess)
        return EIFMM_EHIP;
      if (hipMemcpyAsync(P.xin + a * P.n + P.ns, tgt + a * P.nt, sizeof(double) * P.nt,
                         hipMemcpyDeviceToDevice, s) != hipSuccess)
        return EIFMM_EHIP;
    }
    xyz = P.xin;
  }
  if (P.timing == 1) {
    // tree time is recorded as one phase
    EventPair e;
    if (P.ev_free.empty()) {
      hipEventCreate(&e.a);
      hipEventCreate(&e.b);
    } else {
      e = P.ev_free.back();
      P.ev_free.pop_back();
    }
    e.phase = EIFMM_PH_TREE;
    hipEventRecord(e.a, s);
    int st = tree_build(P, xyz, s);
    hipEventRecord(e.b, s);
    P.ev_pending.push_back(e);
    if (st) return st;
  } else {
    int st = tree_build(P, xyz, s);
    if (st) return st;
  }
  P.points_set = true;
  return EIFMM_OK;
}
}  // namespace

int eifmm_set_points(eifmm_plan h, const double *xyz, void *stream) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (P.host_only) return EIFMM_ESTATE;
  if (P.nt || (P.n > 0 && !xyz)) return EIFMM_EINVAL;
  return set_points_impl(h, xyz, nullptr, stream);
}

int eifmm_set_points_targets(eifmm_plan h, const double *src_xyz, const double *tgt_xyz,
                             void *stream) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (P.host_only) return EIFMM_ESTATE;
  if (!P.nt || !tgt_xyz || (P.ns > 0 && !src_xyz)) return EIFMM_EINVAL;
  return set_points_impl(h, src_xyz, tgt_xyz, stream);
}

int eifmm_evaluate(eifmm_plan h, const double *sigma, int32_t nrhs, int64_t ld, double *f,
                   int64_t ldf, void *stream) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (P.host_only || !P.points_set) return EIFMM_ESTATE;
  if (nrhs < 1 || nrhs > P.max_rhs) return EIFMM_EINVAL;
  const int64_t nout = P.nt ? P.nt : P.ns;
  if ((P.ns > 0 && (!sigma || ld < P.ns)) || (nout > 0 && (!f || ldf < nout)))
    return EIFMM_EINVAL;
  hipSetDevice(P.device);
  return pass_run(P, sigma, nrhs, ld, f, ldf, (hipStream_t)stream);
}

// ------------------------------------------------------------------ no allocation
// Scratch of eifmm_evaluate_noalloc: the partial tiles of the Stream-K tails of
// its gathered-GEMM launches (M2M, the projections, M2L, L2L), in place of the
// plan's own workspace.  One copy per device, held until the process ends.
// Host code must not use the name `scratch` as a device address: it takes the
// address that hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchDoubles = (size_t)4 << 20;  // 32 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on `dev` (taken once per device, with that
// device current); nullptr if the runtime cannot give it
double *scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != dev) return nullptr;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = (double *)ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

int eifmm_evaluate_noalloc(eifmm_plan h, const double *sigma, int32_t nrhs, int64_t ld,
                           double *f, int64_t ldf, void *stream) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (P.host_only || !P.points_set) return EIFMM_ESTATE;
  if (nrhs < 1 || nrhs > P.max_rhs) return EIFMM_EINVAL;
  const int64_t nout = P.nt ? P.nt : P.ns;
  if ((P.ns > 0 && (!sigma || ld < P.ns)) || (nout > 0 && (!f || ldf < nout)))
    return EIFMM_EINVAL;
  // the factored M2L of the second compression stage keeps a workspace of its own
  for (int k = 2; k <= P.depth; ++k)
    if (uses_m2l2(P, k)) return EIFMM_EINVAL;
  if (hipSetDevice(P.device) != hipSuccess) return EIFMM_EHIP;
  double *ws = scratch_on(P.device);
  if (!ws) return EIFMM_EHIP;
  // the scratch replaces the plan's Stream-K workspace for this pass; the
  // per-phase timing events (created on demand) stay off
  const int timing = P.timing;
  P.timing = 0;
  P.run_ws = ws;
  P.run_ws_len = kNoAllocScratchDoubles;
  const int st = pass_run(P, sigma, nrhs, ld, f, ldf, (hipStream_t)stream);
  P.run_ws = nullptr;
  P.run_ws_len = 0;
  P.timing = timing;
  return st;
}

int eifmm_set_timing(eifmm_plan h, int32_t enable) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  timing_drain(P);
  P.timing = enable == 2 ? 2 : (enable != 0 ? 1 : 0);
  for (int q = 0; q < EIFMM_NPHASE; ++q) {
    P.phase_ms[q] = 0;
    P.phase_calls[q] = 0;
  }
  return EIFMM_OK;
}

int eifmm_get_stats(eifmm_plan h, eifmm_stats *out) {
  if (!h || !out || out->struct_size != (int32_t)sizeof(eifmm_stats)) return EIFMM_EINVAL;
  Plan &P = h->P;
  timing_drain(P);
  if (!P.host_only && P.points_set) {
    hipSetDevice(P.device);
    if (tree_counts(P) != EIFMM_OK) return EIFMM_EHIP;
  }
  eifmm_stats s;
  std::memset(&s, 0, sizeof(s));
  s.struct_size = sizeof(eifmm_stats);
  s.depth = P.depth;
  for (int k = 2; k <= P.depth; ++k) {
    s.d[k] = P.lh[k].d;
    s.dpad[k] = P.lh[k].dp;
    s.rank[k] = P.lh[k].r;
    s.rpad[k] = P.lh[k].rp;
    s.d2[k] = P.two_eim ? P.lhB[k].d : 0;
    s.eim_err[k] = P.lh[k].err;
  }
  s.setup_ms = P.setup_ms;
  for (int q = 0; q < EIFMM_NPHASE; ++q) {
    s.phase_ms[q] = P.phase_ms[q];
    s.phase_calls[q] = P.phase_calls[q];
  }
  s.m2l_flops = P.m2l_flops;
  s.m2l_flops_exec = P.m2l_flops_exec;
  s.near_mode = P.near_mode;
  s.proj_flops = P.proj_flops;
  if (P.cfg.tol_mode == 1) s.scale_level = P.cfg.scale_level > 0 ? P.cfg.scale_level : P.depth;
  for (int k = 0; k <= P.depth; ++k) {
    s.active_boxes[k] = P.nact[k];
    s.il_pairs[k] = P.il_pairs[k];
  }
  s.near_pairs = P.near_total;
  s.near_point_pairs = P.near_point_pairs;
  s.hip_error = P.last_hip_error;
  *out = s;
  return EIFMM_OK;
}

namespace {
int get_level_impl(const LevelHost &L, int32_t *d, double *X, double *Y, int64_t *ia,
                   int64_t *ib, double *B, double *G) {
  if (d) *d = L.d;
  if (X) std::memcpy(X, L.X.data(), sizeof(double) * L.X.size());
  if (Y) std::memcpy(Y, L.Y.data(), sizeof(double) * L.Y.size());
  if (ia) std::memcpy(ia, L.ia.data(), sizeof(int64_t) * L.ia.size());
  if (ib) std::memcpy(ib, L.ib.data(), sizeof(int64_t) * L.ib.size());
  if (B) std::memcpy(B, L.B.data(), sizeof(double) * L.B.size());
  if (G) std::memcpy(G, L.G.data(), sizeof(double) * L.G.size());
  return EIFMM_OK;
}
}  // namespace

int eifmm_get_level(eifmm_plan h, int32_t k, int32_t *d, double *X, double *Y, int64_t *ia,
                    int64_t *ib, double *B, double *G) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (k < 2 || k > P.depth) return EIFMM_EINVAL;
  return get_level_impl(P.lh[k], d, X, Y, ia, ib, B, G);
}

int eifmm_get_level2(eifmm_plan h, int32_t k, int32_t *d, double *X, double *Y, int64_t *ia,
                     int64_t *ib, double *B, double *G) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (!P.two_eim || k < 2 || k > P.depth) return EIFMM_EINVAL;
  return get_level_impl(P.lhB[k], d, X, Y, ia, ib, B, G);
}

int eifmm_get_compression(eifmm_plan h, int32_t k, int32_t *r, double *sv, double *U) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (k < 2 || k > P.depth) return EIFMM_EINVAL;
  const LevelHost &L = P.lh[k];
  if (r) *r = L.r;
  if (sv && !L.sv.empty()) std::memcpy(sv, L.sv.data(), sizeof(double) * L.sv.size());
  if (U && L.r > 0) std::memcpy(U, L.U.data(), sizeof(double) * L.U.size());
  return EIFMM_OK;
}

int eifmm_get_compression2(eifmm_plan h, int32_t k, int32_t *s) {
  if (!h || !s) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (k < 2 || k > P.depth) return EIFMM_EINVAL;
  const LevelHost &L = P.lh[k];
  for (int o = 0; o < kNumOffsets; ++o) s[o] = L.s2.empty() ? 0 : L.s2[o];
  return EIFMM_OK;
}

int eifmm_export_tree(eifmm_plan h, int32_t *perm, int64_t *leaf_start, uint32_t *keys) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (P.host_only || !P.points_set) return EIFMM_ESTATE;
  hipSetDevice(P.device);
  if (hipDeviceSynchronize() != hipSuccess) return EIFMM_EHIP;
  if (perm && P.n) hipMemcpy(perm, P.idx, sizeof(int) * P.n, hipMemcpyDeviceToHost);
  if (keys && P.n) {
    hipMemcpy(keys, P.keys, sizeof(uint32_t) * P.n, hipMemcpyDeviceToHost);
    if (P.nt)  // drop the source/target bit of the sort key
      for (int64_t q = 0; q < P.n; ++q) keys[q] >>= 1;
  }
  if (leaf_start) {
    const int64_t nl = ((int64_t)1 << (3 * P.depth)) + 1;
    std::vector<int> tmp(nl);
    hipMemcpy(tmp.data(), P.leaf_start, sizeof(int) * nl, hipMemcpyDeviceToHost);
    for (int64_t q = 0; q < nl; ++q) leaf_start[q] = tmp[q];
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    P.last_hip_error = (int)e;
    return EIFMM_EHIP;
  }
  return EIFMM_OK;
}

int eifmm_export_lists(eifmm_plan h, int32_t level, int64_t *nactive, uint32_t *active,
                       int64_t *near_ptr, uint32_t *near_src, int64_t *il_ptr, uint32_t *il_src,
                       int16_t *il_off) {
  if (!h || !nactive) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (P.host_only || !P.points_set) return EIFMM_ESTATE;
  hipSetDevice(P.device);
  if (hipDeviceSynchronize() != hipSuccess) return EIFMM_EHIP;
  return lists_export(P, level, nactive, active, near_ptr, near_src, il_ptr, il_src, il_off);
}

int eifmm_export_expansion(eifmm_plan h, int32_t which, int32_t k, int32_t rhs, double *out) {
  if (!h || !out) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (P.host_only || !P.points_set || P.last_rhs == 0) return EIFMM_ESTATE;
  if (k < 2 || k > P.depth || which < 0 || which > 4 || (which == 4 && k != P.depth))
    return EIFMM_EINVAL;
  if (rhs < 0 || rhs >= P.last_rhs) return EIFMM_EINVAL;
  hipSetDevice(P.device);
  if (hipDeviceSynchronize() != hipSuccess) return EIFMM_EHIP;
  int st = materialize_expansion(P, which, k);
  if (st) return st;
  const LevelDev &D = P.ld[k];
  // W and What have the first EIM's size, g, l and lhat the second's
  const bool second = which >= 2;
  const int d = second ? P.lh[k].dB : P.lh[k].d, dp = second ? P.lh[k].dpB : P.lh[k].dp,
            R = P.last_rhs;
  const int64_t na = P.nact[k];
  std::vector<double> buf((size_t)na * R * dp);
  const double *src = nullptr;
  switch (which) {
    case 0: src = D.W; break;
    case 1: src = D.Wh; break;
    case 2: src = D.g; break;
    case 3: src = D.l; break;
    default: src = P.lhat; break;
  }
  hipMemcpy(buf.data(), src, sizeof(double) * buf.size(), hipMemcpyDeviceToHost);
  std::vector<uint32_t> act(na);
  hipMemcpy(act.data(), D.act, sizeof(uint32_t) * na, hipMemcpyDeviceToHost);
  const int64_t nb = (int64_t)1 << (3 * k);
  std::memset(out, 0, sizeof(double) * (size_t)nb * d);
  // the leaf's g and l of a plan that folds B^{-1} into them: g = B (B^{-1} g)
  const bool unfold = P.fold_leaf && k == P.depth && (which == 2 || which == 3);
  const std::vector<double> &Bl = P.lh[k].B;  // unit lower triangular, d x d
  for (int64_t j = 0; j < na; ++j) {
    const double *v = &buf[((size_t)j * R + rhs) * dp];
    for (int m = 0; m < d; ++m) {
      double t = v[m];
      if (unfold)
        for (int q = 0; q < m; ++q) t += Bl[(size_t)m * d + q] * v[q];
      out[(size_t)act[j] * d + m] = t;
    }
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    P.last_hip_error = (int)e;
    return EIFMM_EHIP;
  }
  return EIFMM_OK;
}

int eifmm_plan_destroy(eifmm_plan h) {
  if (!h) return EIFMM_EINVAL;
  if (!h->P.host_only) {
    hipSetDevice(h->P.device);
    hipDeviceSynchronize();
  }
  release(h);
  return EIFMM_OK;
}

int eifmm_batch_create(const eifmm_config *cfgs, int32_t nprob, eifmm_batch *out) {
  if (!out || !cfgs || nprob < 1) return EIFMM_EINVAL;
  *out = nullptr;
  for (int p = 0; p < nprob; ++p) {
    eifmm_config c = cfgs[p];
    if (c.depth == -1) c.depth = 2;
    int st = validate(&c);
    if (st) return st;
    if (c.depth < 2 || c.max_rhs != 1 || (c.flags & EIFMM_FLAG_HOST_ONLY) ||
        c.precision != cfgs[0].precision || c.n_targets != 0 || uses_two_eim(c))
      return EIFMM_EINVAL;
  }
  eifmm_batch b = new (std::nothrow) eifmm_batch_s();
  if (!b) return EIFMM_ENOMEM;
  const auto t0 = std::chrono::steady_clock::now();
  hipGetDevice(&b->device);
  b->cfg.assign(cfgs, cfgs + nprob);
  b->depth.assign(nprob, -1);
  b->plans.assign(nprob, nullptr);
  b->table_of.assign(nprob, -1);
  b->cand_lo.assign(nprob, 2);
  b->cand.assign(nprob, {});
  // starting rates, per millisecond, of the phases of a fused pass on MI355X
  // (FP64, one right-hand side); the first set_points measures the batch's own
  for (int k = 0; k <= EIFMM_K_MQ; ++k) b->rate_near[k] = 4.0e8;
  b->rate_m2l = 3.0e10;
  b->rate_leaf = 6.0e8;
  b->rate_box = 1.5e9;
  int st = EIFMM_OK;
  // one table set per key, down to the deepest level any of its problems may use
  std::vector<int> kmax, rep;  // per table set: deepest level, a problem that uses it
  int64_t nmax = 1;
  for (int p = 0; p < nprob; ++p) {
    const eifmm_config &c = b->cfg[p];
    nmax = std::max<int64_t>(nmax, c.n);
    int lo = c.depth, hi = c.depth;
    if (c.depth < 0) depth_candidates(c.n, lo, hi);
    int t = -1;
    for (size_t q = 0; q < rep.size() && t < 0; ++q)
      if (same_tables(b->cfg[rep[q]], c)) t = (int)q;
    if (t < 0) {
      t = (int)rep.size();
      rep.push_back(p);
      kmax.push_back(hi);
    }
    kmax[t] = std::max(kmax[t], hi);
    b->table_of[p] = t;
  }
  for (size_t t = 0; t < rep.size() && !st; ++t) {
    const int p = rep[t];
    eifmm_plan h = new (std::nothrow) eifmm_plan_s();
    if (!h) {
      st = EIFMM_ENOMEM;
      break;
    }
    b->tables.push_back(h);
    Plan &P = h->P;
    P.cfg = b->cfg[p];
    P.cfg.depth = kmax[t];
    P.cfg.n = 0;
    P.depth = kmax[t];
    P.n = 0;
    P.max_rhs = 1;
    P.device = b->device;
    P.gpu_setup = !(P.cfg.flags & EIFMM_FLAG_HOST_SETUP);
    P.shared_tables = true;
    st = build_tables(P);
    if (!st) st = setup_tables(h);
  }
  if (!st) {
    b->sk_groups = stream_k_groups(b->device);
    if (hipMalloc(&b->sk_ws, sizeof(double) * stream_k_ws_len(b->sk_groups)) != hipSuccess ||
        hipMemset(b->sk_ws + stream_k_ws_len(b->sk_groups) - kCounterDoubles, 0,
                  kCounterDoubles * sizeof(double)) !=
            hipSuccess)
      st = EIFMM_ENOMEM;
  }
  if (!st) {
    b->scratch_n = nmax;
    if (hipMalloc(&b->scratch, sizeof(double) * 2 * nmax) != hipSuccess ||
        hipMemset(b->scratch, 0, sizeof(double) * 2 * nmax) != hipSuccess)
      st = EIFMM_ENOMEM;
  }
  if (!st && (hipHostMalloc((void **)&b->staging, sizeof(IoDesc) * nprob) != hipSuccess ||
              hipEventCreate(&b->staged) != hipSuccess || hipStreamCreate(&b->cap) != hipSuccess))
    st = EIFMM_EHIP;
  if (!st && hipDeviceSynchronize() != hipSuccess) st = EIFMM_EHIP;
  if (st) {
    hipGetLastError();
    batch_free(b);
    return st;
  }
  b->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                    .count();
  *out = b;
  return EIFMM_OK;
}

int eifmm_batch_set_points(eifmm_batch b, const double *const *xyz, void *stream) {
  if (!b || !xyz) return EIFMM_EINVAL;
  const int np = (int)b->cfg.size();
  for (int p = 0; p < np; ++p)
    if (b->cfg[p].n > 0 && !xyz[p]) return EIFMM_EINVAL;
  hipSetDevice(b->device);
  hipStream_t s = (hipStream_t)stream;
  b->ready = false;
  drop_graph(b);
  const auto t0 = std::chrono::steady_clock::now();
  const bool first = !b->tuned;
  int st = EIFMM_OK;
  // trees; at the first call, the work of every candidate depth of the autotuned
  // problems (their trees are built once per candidate, then dropped)
  for (int p = 0; p < np && !st; ++p) {
    const eifmm_config &c = b->cfg[p];
    if (b->plans[p]) {
      st = eifmm_set_points(b->plans[p], xyz[p], s);
      continue;
    }
    if (c.depth < 0) {
      int lo, hi;
      depth_candidates(c.n, lo, hi);
      b->cand_lo[p] = lo;
      b->cand[p].clear();
      for (int k = lo; k <= hi && !st; ++k) {
        eifmm_plan h = nullptr;
        if ((st = shared_plan(b, p, k, &h))) break;
        st = eifmm_set_points(h, xyz[p], s);
        if (!st) b->cand[p].push_back(work_of(h->P));
        release(h);
      }
      if (st) break;
      b->depth[p] = b->cand_lo[p] + pick_depth(b, p);
    } else {
      b->depth[p] = c.depth;
    }
    if (!(st = shared_plan(b, p, b->depth[p], &b->plans[p])))
      st = eifmm_set_points(b->plans[p], xyz[p], s);
  }
  if (!st) st = prepare(b, b->m2l_rbt > 0 ? b->m2l_rbt : 0);
  if (!st && first) {
    // measure the fused pass once (zero sigma), turn the phase times into rates,
    // choose the depths again with them and rebuild the problems that change
    st = calibrate(b, s);
    bool changed = false;
    for (int p = 0; p < np && !st; ++p) {
      if (b->cfg[p].depth >= 0 || b->cand[p].empty()) continue;
      const int k = b->cand_lo[p] + pick_depth(b, p);
      if (k == b->depth[p]) continue;
      changed = true;
      release(b->plans[p]);
      b->plans[p] = nullptr;
      b->depth[p] = k;
      if (!(st = shared_plan(b, p, k, &b->plans[p])))
        st = eifmm_set_points(b->plans[p], xyz[p], s);
    }
    if (!st && changed) st = prepare(b, 0);
    // tile height of the fused M2L launch: the M2L launch alone for 3, 4, 5 and 6
    // row blocks, after one full pass that fills the expansions
    if (!st) st = stage_io(b, nullptr, nullptr, s);
    if (!st) batch_run(b->ex, s);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    double best = 0;
    int pick = 6;
    for (int rbt = 3; rbt <= 6 && !st; ++rbt) {
      if ((st = prepare(b, rbt))) break;
      batch_run_m2l(b->ex, s);
      hipEventRecord(e0, s);
      for (int rep = 0; rep < 3; ++rep) batch_run_m2l(b->ex, s);
      hipEventRecord(e1, s);
      const double ms = elapsed_ms(e0, e1);
      if (rbt == 4 || ms < best) {
        best = ms;
        pick = rbt;
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    b->m2l_rbt = pick;
    if (!st) st = prepare(b, pick);
    if (!st) b->tuned = true;
  }
  if (!st) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = EIFMM_EHIP;
  }
  if (first)
    b->tune_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                      .count();
  if (st) return st;
  b->ready = true;
  return EIFMM_OK;
}

int eifmm_batch_evaluate(eifmm_batch b, const double *const *sigma, double *const *f,
                         void *stream) {
  if (!b || !sigma || !f) return EIFMM_EINVAL;
  if (!b->ready) return EIFMM_ESTATE;
  const int np = (int)b->cfg.size();
  for (int p = 0; p < np; ++p)
    if (b->cfg[p].n > 0 && (!sigma[p] || !f[p])) return EIFMM_EINVAL;
  hipSetDevice(b->device);
  hipStream_t s = (hipStream_t)stream;
  int st = stage_io(b, sigma, f, s);
  if (st) return st;
  if (!b->gexec) {
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return EIFMM_EHIP;
    batch_run(b->ex, b->cap);
    if (hipStreamEndCapture(b->cap, &b->graph) != hipSuccess) {
      hipGetLastError();
      b->graph = nullptr;
      return EIFMM_EHIP;
    }
    if (hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0) != hipSuccess) {
      hipGetLastError();
      drop_graph(b);
      return EIFMM_EHIP;
    }
    size_t nodes = 0;
    hipGraphGetNodes(b->graph, nullptr, &nodes);
    b->graph_nodes = (int)nodes;
  }
  if (hipGraphLaunch(b->gexec, s) != hipSuccess) return EIFMM_EHIP;
  for (auto h : b->plans) h->P.last_rhs = 1;
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? EIFMM_OK : EIFMM_EHIP;
}

int eifmm_batch_evaluate_unfused(eifmm_batch b, const double *const *sigma, double *const *f,
                                 void *stream) {
  if (!b || !sigma || !f) return EIFMM_EINVAL;
  if (!b->ready) return EIFMM_ESTATE;
  const int np = (int)b->cfg.size();
  for (int p = 0; p < np; ++p)
    if (b->cfg[p].n > 0 && (!sigma[p] || !f[p])) return EIFMM_EINVAL;
  for (int p = 0; p < np; ++p) {
    const int64_t n = b->cfg[p].n;
    if (n == 0) continue;
    int st = eifmm_evaluate(b->plans[p], sigma[p], 1, n, f[p], n, stream);
    if (st) return st;
  }
  return EIFMM_OK;
}

int eifmm_batch_export_expansion(eifmm_batch b, int32_t p, int32_t which, int32_t k,
                                 double *out) {
  if (!b || p < 0 || p >= (int)b->cfg.size() || !b->plans[p]) return EIFMM_EINVAL;
  return eifmm_export_expansion(b->plans[p], which, k, 0, out);
}

int eifmm_batch_get_stats(eifmm_batch b, int32_t p, eifmm_stats *out) {
  if (!b || p < 0 || p >= (int)b->cfg.size() || !b->plans[p]) return EIFMM_EINVAL;
  int st = eifmm_get_stats(b->plans[p], out);
  if (!st) out->setup_ms = b->tables[b->table_of[p]]->P.setup_ms;
  return st;
}

int eifmm_batch_get_info(eifmm_batch b, eifmm_batch_info *out) {
  if (!b || !out || out->struct_size != (int32_t)sizeof(eifmm_batch_info)) return EIFMM_EINVAL;
  eifmm_batch_info i;
  std::memset(&i, 0, sizeof(i));
  i.struct_size = sizeof(i);
  i.nprob = (int32_t)b->cfg.size();
  i.ntables = (int32_t)b->tables.size();
  i.graph_nodes = b->graph_nodes;
  i.m2l_rbt = b->m2l_rbt;
  i.m2l_flops = b->ex.m2l_flops;
  i.tune_ms = b->tune_ms;
  i.setup_ms = b->setup_ms;
  *out = i;
  return EIFMM_OK;
}

int eifmm_batch_destroy(eifmm_batch b) {
  if (!b) return EIFMM_EINVAL;
  hipSetDevice(b->device);
  batch_free(b);
  return EIFMM_OK;
}

const char *eifmm_status_str(int status) {
  switch (status) {
    case EIFMM_OK: return "ok";
    case EIFMM_EINVAL: return "invalid argument";
    case EIFMM_EDOMAIN: return "point outside the domain or not finite";
    case EIFMM_ESTATE: return "call out of order (no points set, or host-only plan)";
    case EIFMM_EEIM: return "EIM reached dmax before the tolerance";
    case EIFMM_ENOMEM: return "out of memory";
    case EIFMM_EHIP: return "HIP runtime error";
  }
  return "unknown status";
}

}  // extern "C"
