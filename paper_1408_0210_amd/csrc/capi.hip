// capi.hip -- the extern "C" entry points of libeifmm.so (declared in include/eifmm.h).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
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

int validate(const eifmm_config *c) {
  if (!c || c->struct_size != (int32_t)sizeof(eifmm_config)) return EIFMM_EINVAL;
  if (c->kernel < EIFMM_K_LAPLACE || c->kernel > EIFMM_K_SQDIST) return EIFMM_EINVAL;
  if ((c->kernel == EIFMM_K_GAUSS && !(c->kernel_param > 0)) ||
      (c->kernel == EIFMM_K_YUKAWA && !(c->kernel_param >= 0)) || !std::isfinite(c->kernel_param))
    return EIFMM_EINVAL;
  if (!(c->L > 0) || !std::isfinite(c->L)) return EIFMM_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(c->lo[a])) return EIFMM_EINVAL;
  if (c->n < 0 || c->n > (int64_t)INT32_MAX / 2) return EIFMM_EINVAL;
  if (c->depth < 0 || c->depth > EIFMM_MAX_DEPTH) return EIFMM_EINVAL;
  if (c->max_rhs < 1 || c->max_rhs > 4096) return EIFMM_EINVAL;
  if (!(c->eim_tol > 0) || !std::isfinite(c->eim_tol)) return EIFMM_EINVAL;
  if (c->tol_mode < 0 || c->tol_mode > 1) return EIFMM_EINVAL;
  if (c->precision != EIFMM_PREC_FP64 && c->precision != EIFMM_PREC_MIXED) return EIFMM_EINVAL;
  if (c->dmax < 0 || c->dmax > 4096) return EIFMM_EINVAL;
  if (!(c->compress_tol >= 0) || !std::isfinite(c->compress_tol)) return EIFMM_EINVAL;
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
  if (P.job_dev) hipFree(P.job_dev);
  delete h;
}

int device_setup(eifmm_plan h) {
  Plan &P = h->P;
  auto &tr = owned(h);
  const int depth = P.depth;
  const bool mixed = P.cfg.precision == EIFMM_PREC_MIXED;
  const int64_t n = P.n;
  const int R = P.cfg.max_rhs;
  int st;
#define TRY(x)            \
  do {                    \
    if ((st = (x)) != 0) return st; \
  } while (0)
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
    if (k < depth) {
      TRY(upload(&D.m2m, H.m2m.data(), H.m2m.size(), tr));
      TRY(upload(&D.l2l, H.l2l.data(), H.l2l.size(), tr));
    }
    TRY(upload(&D.X, H.X.data(), H.X.size(), tr));
    if (H.r > 0) {
      TRY(upload(&D.ufrag, H.ufrag.data(), H.ufrag.size(), tr));
      TRY(upload(&D.utfrag, H.utfrag.data(), H.utfrag.size(), tr));
    }
  }
  // point workspaces
  const int64_t nn = std::max<int64_t>(n, 1);
  P.ntiles_sort = (int)((nn + 1023) / 1024);
  TRY(dalloc(&P.xyz, 3 * nn, tr));
  TRY(dalloc(&P.keys, nn, tr));
  TRY(dalloc(&P.keys_tmp, nn, tr));
  TRY(dalloc(&P.idx, nn, tr));
  TRY(dalloc(&P.idx_tmp, nn, tr));
  TRY(dalloc(&P.hist, (size_t)256 * P.ntiles_sort, tr));
  const int64_t nleaf = (int64_t)1 << (3 * depth);
  TRY(dalloc(&P.leaf_start, nleaf + 1, tr));
  size_t maxcap = 1;
  for (int k = 0; k <= depth; ++k) {
    LevelDev &D = P.ld[k];
    const int64_t nb = (int64_t)1 << (3 * k);
    D.cap = (size_t)std::max<int64_t>(1, std::min<int64_t>(nb, n));
    maxcap = std::max(maxcap, D.cap);
    TRY(dalloc(&D.act, D.cap, tr));
    TRY(dalloc(&D.slot, nb, tr));
    TRY(dalloc(&D.cls, D.cap, tr));
  }
  const size_t scan_len = std::max<size_t>((size_t)256 * P.ntiles_sort, maxcap + 2);
  TRY(dalloc(&P.scan_tmp, scan_len / 1024 + 64, tr));
  TRY(dalloc(&P.blkcnt, ((size_t)(nleaf + 255) / 256 + 1) * 9, tr));
  TRY(dalloc(&P.list_cnt, maxcap + 2, tr));
  TRY(dalloc(&P.counts_dev, (size_t)16 * kMaxLevels, tr));
  TRY(dalloc(&P.errflag, 1, tr));
  P.near_cap = (size_t)27 * P.ld[depth].cap;
  TRY(dalloc(&P.near_ptr, P.ld[depth].cap + 2, tr));
  TRY(dalloc(&P.near_src, P.near_cap, tr));
  TRY(dalloc(&P.chunk_ptr, P.ld[depth].cap + 2, tr));
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
    TRY(dalloc(&D.g, m, tr));
    if (k == 2)
      D.l = D.g;  // l^2 = g^2 (Algorithm 3, step 5)
    else
      TRY(dalloc(&D.l, m, tr));
  }
  {
    int cus = 0;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, P.device);
    P.sk_groups = std::max(8, 2 * cus);
    TRY(dalloc(&P.sk_ws, (size_t)2 * P.sk_groups * 6 * 16 * 128, tr));
  }
  if (depth >= 2)
    TRY(dalloc(&P.lhat, P.ld[depth].cap * (size_t)R * (size_t)P.lh[depth].dp, tr));
#undef TRY
  return EIFMM_OK;
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
  P.n = cfg->n;
  P.max_rhs = cfg->max_rhs;
  P.host_only = (cfg->flags & EIFMM_FLAG_HOST_ONLY) != 0;
  st = build_tables(P);
  if (st == EIFMM_OK && !P.host_only) {
    hipGetDevice(&P.device);
    st = device_setup(h);
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

int eifmm_set_points(eifmm_plan h, const double *xyz, void *stream) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (P.host_only) return EIFMM_ESTATE;
  if (P.n > 0 && !xyz) return EIFMM_EINVAL;
  hipSetDevice(P.device);
  P.points_set = false;
  P.jobs.nrhs = -1;
  hipStream_t s = (hipStream_t)stream;
  if (P.timing) {
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

int eifmm_evaluate(eifmm_plan h, const double *sigma, int32_t nrhs, int64_t ld, double *f,
                   int64_t ldf, void *stream) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (P.host_only || !P.points_set) return EIFMM_ESTATE;
  if (nrhs < 1 || nrhs > P.max_rhs) return EIFMM_EINVAL;
  if (P.n > 0 && (!sigma || !f || ld < P.n || ldf < P.n)) return EIFMM_EINVAL;
  hipSetDevice(P.device);
  return pass_run(P, sigma, nrhs, ld, f, ldf, (hipStream_t)stream);
}

int eifmm_set_timing(eifmm_plan h, int32_t enable) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  timing_drain(P);
  P.timing = enable != 0;
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
  eifmm_stats s;
  std::memset(&s, 0, sizeof(s));
  s.struct_size = sizeof(eifmm_stats);
  s.depth = P.depth;
  for (int k = 2; k <= P.depth; ++k) {
    s.d[k] = P.lh[k].d;
    s.dpad[k] = P.lh[k].dp;
    s.rank[k] = P.lh[k].r;
    s.eim_err[k] = P.lh[k].err;
  }
  s.setup_ms = P.setup_ms;
  for (int q = 0; q < EIFMM_NPHASE; ++q) {
    s.phase_ms[q] = P.phase_ms[q];
    s.phase_calls[q] = P.phase_calls[q];
  }
  s.m2l_flops = P.m2l_flops;
  s.proj_flops = P.proj_flops;
  for (int k = 0; k <= P.depth; ++k) {
    s.active_boxes[k] = P.nact[k];
    s.il_pairs[k] = P.il_pairs[k];
  }
  s.near_pairs = P.near_total;
  s.hip_error = P.last_hip_error;
  *out = s;
  return EIFMM_OK;
}

int eifmm_get_level(eifmm_plan h, int32_t k, int32_t *d, double *X, double *Y, int64_t *ia,
                    int64_t *ib, double *B, double *G) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (k < 2 || k > P.depth) return EIFMM_EINVAL;
  const LevelHost &L = P.lh[k];
  if (d) *d = L.d;
  if (X) std::memcpy(X, L.X.data(), sizeof(double) * L.X.size());
  if (Y) std::memcpy(Y, L.Y.data(), sizeof(double) * L.Y.size());
  if (ia) std::memcpy(ia, L.ia.data(), sizeof(int64_t) * L.ia.size());
  if (ib) std::memcpy(ib, L.ib.data(), sizeof(int64_t) * L.ib.size());
  if (B) std::memcpy(B, L.B.data(), sizeof(double) * L.B.size());
  if (G) std::memcpy(G, L.G.data(), sizeof(double) * L.G.size());
  return EIFMM_OK;
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

int eifmm_export_tree(eifmm_plan h, int32_t *perm, int64_t *leaf_start, uint32_t *keys) {
  if (!h) return EIFMM_EINVAL;
  Plan &P = h->P;
  if (P.host_only || !P.points_set) return EIFMM_ESTATE;
  hipSetDevice(P.device);
  if (hipDeviceSynchronize() != hipSuccess) return EIFMM_EHIP;
  if (perm && P.n) hipMemcpy(perm, P.idx, sizeof(int) * P.n, hipMemcpyDeviceToHost);
  if (keys && P.n) hipMemcpy(keys, P.keys, sizeof(uint32_t) * P.n, hipMemcpyDeviceToHost);
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
  const LevelDev &D = P.ld[k];
  const int d = P.lh[k].d, dp = P.lh[k].dp, R = P.last_rhs;
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
  for (int64_t j = 0; j < na; ++j)
    for (int m = 0; m < d; ++m)
      out[(size_t)act[j] * d + m] = buf[((size_t)j * R + rhs) * dp + m];
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
