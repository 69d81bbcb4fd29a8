// pass.hip -- the EIFMM evaluation pass (Algorithm 3 plus the near field).
//
// Expansions of level k live in slot-major arrays [slot][rhs][dp_k] (slot =
// rank of a non-empty box in key order; dp_k = d_k padded to 16 with zeros).
// Steps and kernels:
//   near field, eq. (13)        k_p2p64 / k_p2p32   one wave per 64 targets of a leaf
//   1  P2M                      k_p2m               one workgroup per leaf
//   2  M2M (Sec. 4.1 operators) k_gemm<MODE_M2M>    MFMA, 8 children per parent
//   3  What = Delta W           k_trsm              blocked triangular solves (MFMA)
//   4  M2L (Sec. 4.2 matrices)  k_gemm<MODE_M2L>    MFMA, 189 offsets per class
//   5  L2L                      k_gemm<MODE_L2L>    MFMA, adds g
//   6  lhat = Delta^T l         k_trsm
//   7  L2P and f = f_far + f_near, input order  k_l2p  one wave per 64 targets
#include <algorithm>
#include <climits>
#include <cstring>
#include <type_traits>
#include <vector>

#include "devutil.hpp"
#include "plan.hpp"

namespace eifmm {

// ------------------------------------------------------------------ kernels k
// 1/sqrt(r2) for r2 > 0: the hardware reciprocal square root y, refined with
// t = 1 - r2 y^2 by the series (1 - t)^(-1/2) = 1 + t/2 + 3 t^2 / 8 + ...,
// i.e. y (1 + t (1/2 + 3 t / 8)).  r2 = 0 gives NaN; the callers that can meet
// it (the near field of a singular kernel) replace the value.
__device__ inline double rsq_refined(double r2) {
  const double y = __builtin_amdgcn_rsq(r2);
  const double t = fma(-r2 * y, y, 1.0);
  return fma(y * t, fma(t, 0.375, 0.5), y);
}

template <int KIND>
struct KF {
  static constexpr bool singular = (KIND == EIFMM_K_LAPLACE || KIND == EIFMM_K_YUKAWA ||
                                     KIND == EIFMM_K_COSR || KIND == EIFMM_K_ADVDIFF);
  // k at z with r2 = |z|^2 and zx its first component (read by the kernel that
  // is not radial); p: Yukawa a, Gauss 1/h2, cos(w r)/r w, multiquadric c,
  // advection-diffusion a
  __device__ static inline double eval(double r2, double zx, double p) {
    if constexpr (KIND == EIFMM_K_LAPLACE) {
      return rsq_refined(r2);
    } else if constexpr (KIND == EIFMM_K_YUKAWA) {
      double ri = rsq_refined(r2);
      return exp(-p * (r2 * ri)) * ri;
    } else if constexpr (KIND == EIFMM_K_GAUSS) {
      return exp(-r2 * p);
    } else if constexpr (KIND == EIFMM_K_COSR) {
      double ri = rsq_refined(r2);
      return cos(p * (r2 * ri)) * ri;
    } else if constexpr (KIND == EIFMM_K_MQ) {
      return sqrt(r2 + p);
    } else if constexpr (KIND == EIFMM_K_ADVDIFF) {
      double ri = rsq_refined(r2);
      return exp(p * (zx - r2 * ri)) * ri;
    } else {
      return r2;
    }
  }
  __device__ static inline float evalf(float r2, float zx, float p) {
    if constexpr (KIND == EIFMM_K_LAPLACE) {
      return rsqrtf(r2);
    } else if constexpr (KIND == EIFMM_K_YUKAWA) {
      float ri = rsqrtf(r2);
      return expf(-p * (r2 * ri)) * ri;
    } else if constexpr (KIND == EIFMM_K_GAUSS) {
      return expf(-r2 * p);
    } else if constexpr (KIND == EIFMM_K_COSR) {
      float ri = rsqrtf(r2);
      return cosf(p * (r2 * ri)) * ri;
    } else if constexpr (KIND == EIFMM_K_MQ) {
      return sqrtf(r2 + p);
    } else if constexpr (KIND == EIFMM_K_ADVDIFF) {
      float ri = rsqrtf(r2);
      return expf(p * (zx - r2 * ri)) * ri;
    } else {
      return r2;
    }
  }
};

__host__ __device__ inline double dev_param(int kind, double p) {
  return kind == EIFMM_K_GAUSS ? 1.0 / p : p;
}

// ------------------------------------------------------------------ leaf level
// The kernels of the leaf level (sigma gather, near field, P2M, L2P) read one
// problem's arrays from a LeafDesc.  A plan launches them with its descriptor by
// value (BATCH = false); a batch of problems launches each kernel once over the
// chunks / leaves / points of all its problems with an array of descriptors in
// device memory (BATCH = true): each workgroup finds its problem by a binary
// search over the first chunk (leaf, point) of every problem.
//
// Near field and L2P work on chunks of up to 32 consecutive targets of a leaf
// (chunk_ptr: exclusive prefix sum of ceil(count / 32) over the active leaves),
// one chunk per 64-lane workgroup whose two halves share the chunk's work, so
// a crowded leaf of a clustered cloud spreads over many workgroups and a sparse
// one (~30 points) does not idle half a wave.

template <typename F>
__device__ inline int find_last_le(int n, int64_t v, F key) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (key(mid) <= v)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline int chunk_leaf(const int *__restrict__ chunk_ptr, int nleaf, int c) {
  return find_last_le(nleaf, c, [&](int m) { return (int64_t)chunk_ptr[m]; });
}

// the descriptor of work item b (a chunk or a leaf of the launch) and b's index
// within its problem
template <bool BATCH, int WHICH>  // WHICH: 0 chunk, 1 leaf
__device__ inline void pick_desc_at(const LeafDesc &one, const LeafDesc *__restrict__ many,
                                    int nmany, int b, LeafDesc &D, int &local, int &prob) {
  if constexpr (BATCH) {
    prob = find_last_le(nmany, b, [&](int m) {
      return WHICH == 0 ? many[m].chunk_base : many[m].leaf_base;
    });
    D = many[prob];
    local = b - (int)(WHICH == 0 ? D.chunk_base : D.leaf_base);
  } else {
    prob = 0;
    D = one;
    local = b;
  }
}

template <bool BATCH, int WHICH>
__device__ inline void pick_desc(const LeafDesc &one, const LeafDesc *__restrict__ many,
                                 int nmany, LeafDesc &D, int &local, int &prob) {
  pick_desc_at<BATCH, WHICH>(one, many, nmany, (int)blockIdx.x, D, local, prob);
}

// ------------------------------------------------------------------ sigma
// sig[s][r] = sigma[perm[s] + r ld] (sorted order; 0 at targets)
template <bool BATCH>
__global__ void k_gather_sigma(LeafDesc one, IoDesc ione, const LeafDesc *__restrict__ many,
                               const IoDesc *__restrict__ io, int nmany, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  LeafDesc D;
  IoDesc O;
  int64_t el = e;
  if constexpr (BATCH) {
    const int pr = find_last_le(nmany, e, [&](int m) { return many[m].pt_base; });
    D = many[pr];
    O = io[pr];
    el = e - D.pt_base;
  } else {
    D = one;
    O = ione;
  }
  const int64_t s = el / D.nrhs;
  const int r = (int)(el - s * D.nrhs);
  const int64_t src = D.perm[s];  // a target (src >= nsrc) carries no potential
  D.sig[el] = src < D.nsrc ? O.sigma[src + (int64_t)r * O.ld] : 0.0;
}

// ------------------------------------------------------------------ near field
// One 64-lane workgroup per chunk of up to 32 targets.  The sources of the
// chunk's neighbour leaves are numbered consecutively (a prefix sum over the
// near list, in LDS) and staged 64 at a time, so every batch is full whatever
// the leaf sizes; lane l and lane l + 32 hold the same target and take the
// first and the second half of each batch, and their sums are added at the end.
// The next batch is loaded into registers while the current one is used.
struct NearSrc {
  int nq;        // neighbour leaves
  int total;     // sources over all of them
  // source numbers of the chunk's own leaf, the one neighbour with pairs at r = 0
  // (a target and itself, or coincident points)
  int own_lo, own_hi;
};

// pre[e] = first source number of neighbour e, start[e] = its first point
__device__ inline NearSrc near_sources(const LeafDesc &D, int j, int *pre, int *start) {
  const int lane = threadIdx.x;
  const int q0 = D.near_ptr[j], nq = D.near_ptr[j + 1] - q0;
  int cnt = 0;
  bool own = false;
  if (lane < nq) {
    const int a = D.near_src[q0 + lane];
    const uint32_t sk = D.act[a];
    start[lane] = D.ls[sk];
    cnt = D.se[sk] - D.ls[sk];
    own = a == j;
  }
  const unsigned long long ob = __ballot(own);
  // inclusive scan of cnt over the (at most 27) lanes
  int v = cnt;
#pragma unroll
  for (int o = 1; o < 32; o <<= 1) {
    const int u = __shfl_up(v, o);
    if ((lane & 31) >= o) v += u;
  }
  if (lane < nq) pre[lane + 1] = v;
  if (lane == 0) pre[0] = 0;
  __syncthreads();
  const int eo = __ffsll(ob) - 1;  // the own leaf's place in the list (-1: absent)
  return NearSrc{nq, pre[nq], eo >= 0 ? pre[eo] : 0, eo >= 0 ? pre[eo + 1] : 0};
}

// point index of source number v (0 <= v < total); e is the neighbour of the
// lane's previous (smaller) source number, so the search resumes there
__device__ inline int near_point(int v, int nq, const int *pre, const int *start, int &e) {
  while (e + 1 < nq && pre[e + 1] <= v) ++e;
  return start[e] + (v - pre[e]);
}

// The lanes of chunk c of leaf j: with k targets (a chunk holds up to 32) and P
// the smallest power of two >= k, lane l holds target l mod P and takes sources
// [P (l / P), P (l / P + 1)) of every 64-source batch, so that a chunk of few
// targets (the last of a leaf) spreads each target's sources over 64 / P lanes
// instead of leaving lanes idle.  A full chunk has P = 32: lanes l and l + 32
// share a target and take the two halves of each batch.
struct ChunkLanes {
  int i;     // the lane's target point
  bool tv;   // the target exists
  int P;     // targets' lane period
  int u0;    // first source of the lane's range in a batch
};
// (spread: false keeps P = 32: the FP64 near field with several right-hand
// sides, whose RB sums per pair already fill the lanes' registers)
__device__ inline ChunkLanes chunk_lanes(const LeafDesc &D, int j, int c, int lane, bool spread) {
  const uint32_t key = D.act[j];
  const int i0 = D.tb[key] + 32 * (c - D.chunk_ptr[j]);
  const int k = min(32, D.ls[key + 1] - i0);
  const int P = !spread ? 32 : k <= 1 ? 1 : 1 << (32 - __clz(k - 1));
  const int ti = lane & (P - 1);
  return ChunkLanes{i0 + ti, ti < k, P, lane - ti};
}

// (cos(wr)/r asks for three waves per SIMD: its kernel value would otherwise
// take registers for two only)
template <int KIND, int RB, bool BATCH>
__global__ __launch_bounds__(64, KIND == EIFMM_K_COSR ? 3 : 1) void k_p2p64(
    LeafDesc one, const LeafDesc *__restrict__ many, int nmany) {
  __shared__ double sx[64], sy[64], sz[64], ss[64 * RB];
  __shared__ int pre[28], start[27];
  LeafDesc D;
  int c, prob;
  pick_desc<BATCH, 0>(one, many, nmany, D, c, prob);
  if (c >= D.chunk_ptr[D.nleaf]) return;  // past the last chunk (the grid is a bound)
  const int lane = threadIdx.x;
  const int64_t n = D.n;
  const int nrhs = D.nrhs;
  const double *__restrict__ xyz = D.xyz;
  const double *__restrict__ sig = D.sig;
  const int j = chunk_leaf(D.chunk_ptr, D.nleaf, c);
  const ChunkLanes CL = chunk_lanes(D, j, c, lane, RB == 1);
  const int i = CL.i;
  const bool tv = CL.tv;
  const double xi = tv ? xyz[i] : 0.0, yi = tv ? xyz[n + i] : 0.0, zi = tv ? xyz[2 * n + i] : 0.0;
  const NearSrc S = near_sources(D, j, pre, start);
  for (int r0 = 0; r0 < nrhs; r0 += RB) {
    double acc[RB];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) acc[rr] = 0.0;
    double px = 0, py = 0, pz = 0, ps[RB];
    // a block past the end is padded with the last source at zero potential, so
    // every block has 64 sources and the pair loop a fixed trip count
    int ecur = 0;  // neighbour of this lane's last source number
    auto load = [&](int base) {
      const int v = base + lane;
      if (S.total > 0) {
        const int sidx = near_point(v < S.total ? v : S.total - 1, S.nq, pre, start, ecur);
        px = xyz[sidx];
        py = xyz[n + sidx];
        pz = xyz[2 * n + sidx];
#pragma unroll
        for (int rr = 0; rr < RB; ++rr)
          ps[rr] = (v < S.total && r0 + rr < nrhs) ? sig[(int64_t)sidx * nrhs + r0 + rr] : 0.0;
      }
    };
    load(0);
    for (int base = 0; base < S.total; base += 64) {
      __syncthreads();
      sx[lane] = px;
      sy[lane] = py;
      sz[lane] = pz;
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) ss[lane * RB + rr] = ps[rr];
      __syncthreads();
      if (base + 64 < S.total) load(base + 64);
      // r = 0 (a pair the sum leaves out) needs the mask only in the batches that
      // hold sources of the own leaf: points of two different leaves are apart (a
      // leaf boundary lies between them), so r2 > 0 there, unless both lie within
      // about 1e-154 of a boundary at the origin, which the library does not
      // support.  The padding past the end repeats the last source, so it needs
      // the mask only when that source is the own leaf's, whose batch has it.
      // (several RHS share each pair's mask: they keep the one loop)
      const bool own =
          KF<KIND>::singular && (RB > 1 || (base < S.own_hi && base + 64 > S.own_lo));
      // (a full chunk's loop has a fixed trip count of 32)
      // (several RHS hold RB sums per pair already; a partial chunk's loop runs
      // at most 16 times)
      auto pairs = [&](auto masked, auto full) {
        constexpr bool F = decltype(full)::value;
        constexpr int kUnroll = RB > 1 ? 2 : (F ? 8 : 1);
        const int cnt = F ? 32 : CL.P;
#pragma unroll kUnroll
        for (int q = 0; q < cnt; ++q) {
          const int u = CL.u0 + q;
          const double dx = xi - sx[u], dy = yi - sy[u], dz = zi - sz[u];
          const double r2 = dx * dx + dy * dy + dz * dz;
          double kv = KF<KIND>::eval(r2, dx, D.p);
          if constexpr (decltype(masked)::value) kv = (r2 == 0.0) ? 0.0 : kv;
#pragma unroll
          for (int rr = 0; rr < RB; ++rr) acc[rr] += ss[u * RB + rr] * kv;
        }
      };
      if (RB > 1 || CL.P == 32) {
        if (own)
          pairs(std::true_type{}, std::true_type{});
        else
          pairs(std::false_type{}, std::true_type{});
      } else {
        if (own)
          pairs(std::true_type{}, std::false_type{});
        else
          pairs(std::false_type{}, std::false_type{});
      }
    }
    // the target's 64 / P partial sums (lanes l, l + P, ...)
    for (int o = CL.P; o < 64; o <<= 1) {
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) acc[rr] += __shfl_xor(acc[rr], o);
    }
    if (tv && lane < CL.P) {
#pragma unroll
      for (int rr = 0; rr < RB; ++rr)
        if (r0 + rr < nrhs) D.fnear[(int64_t)i * nrhs + r0 + rr] = acc[rr];
    }
  }
}

// Mixed-precision near field: the coordinate differences are taken in FP64 and
// rounded once to FP32 (so a close pair keeps its relative accuracy however
// crowded the leaf), kernel values and products in FP32, two-sum-compensated
// FP32 sums per half, the two halves and their compensations added in FP64.
template <int KIND, int RB, bool BATCH>
__global__ __launch_bounds__(64) void k_p2p32(LeafDesc one, const LeafDesc *__restrict__ many,
                                              int nmany) {
  __shared__ double sx[64], sy[64], sz[64];
  __shared__ float ss[64 * RB];
  __shared__ int pre[28], start[27];
  LeafDesc D;
  int c, prob;
  pick_desc<BATCH, 0>(one, many, nmany, D, c, prob);
  if (c >= D.chunk_ptr[D.nleaf]) return;  // past the last chunk (the grid is a bound)
  const int lane = threadIdx.x;
  const int64_t n = D.n;
  const int nrhs = D.nrhs;
  const float p = (float)D.p;
  const double *__restrict__ xyz = D.xyz;
  const double *__restrict__ sig = D.sig;
  const int j = chunk_leaf(D.chunk_ptr, D.nleaf, c);
  // (several RHS too: 64 RHS on 2^20 points, 264 -> 261 ms)
  const ChunkLanes CL = chunk_lanes(D, j, c, lane, true);
  const int i = CL.i;
  const bool tv = CL.tv;
  const double xi = tv ? xyz[i] : 0.0, yi = tv ? xyz[n + i] : 0.0, zi = tv ? xyz[2 * n + i] : 0.0;
  const NearSrc S = near_sources(D, j, pre, start);
  for (int r0 = 0; r0 < nrhs; r0 += RB) {
    float sum[RB], cmp[RB];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) sum[rr] = cmp[rr] = 0.f;
    double px = 0, py = 0, pz = 0;
    float ps[RB];
    // padding past the end as in k_p2p64 (zero potential adds exactly zero to
    // the compensated sums)
    int ecur = 0;  // neighbour of this lane's last source number
    auto load = [&](int base) {
      const int v = base + lane;
      if (S.total > 0) {
        const int sidx = near_point(v < S.total ? v : S.total - 1, S.nq, pre, start, ecur);
        px = xyz[sidx];
        py = xyz[n + sidx];
        pz = xyz[2 * n + sidx];
#pragma unroll
        for (int rr = 0; rr < RB; ++rr)
          ps[rr] = (v < S.total && r0 + rr < nrhs) ? (float)sig[(int64_t)sidx * nrhs + r0 + rr]
                                                   : 0.f;
      }
    };
    load(0);
    for (int base = 0; base < S.total; base += 64) {
      __syncthreads();
      sx[lane] = px;
      sy[lane] = py;
      sz[lane] = pz;
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) ss[lane * RB + rr] = ps[rr];
      __syncthreads();
      if (base + 64 < S.total) load(base + 64);
      // the r = 0 mask only in batches with the own leaf's sources, as in
      // k_p2p64 (here r2 is FP32: two points of different leaves give r2 = 0
      // only when under about 1e-22 apart, next to a boundary at the origin)
      // (several RHS share each pair's mask: they keep the one loop)
      const bool own =
          KF<KIND>::singular && (RB > 1 || (base < S.own_hi && base + 64 > S.own_lo));
      auto pairs = [&](auto masked, auto full) {
        constexpr bool F = decltype(full)::value;
        constexpr int kUnroll = RB > 1 ? 2 : (F ? 4 : 2);
        const int cnt = F ? 32 : CL.P;
#pragma unroll kUnroll
        for (int q = 0; q < cnt; ++q) {
          const int u = CL.u0 + q;
          const float dx = (float)(xi - sx[u]), dy = (float)(yi - sy[u]),
                      dz = (float)(zi - sz[u]);
          const float r2 = dx * dx + dy * dy + dz * dz;
          float kv = KF<KIND>::evalf(r2, dx, p);
          if constexpr (decltype(masked)::value) kv = (r2 == 0.f) ? 0.f : kv;
#pragma unroll
          for (int rr = 0; rr < RB; ++rr) {
            // the rounding error of sum + w, exactly, by the branch-free two-sum
            // (Knuth): no magnitude comparison as in Neumaier's form
            const float w = ss[u * RB + rr] * kv;
            const float tsum = sum[rr] + w;
            const float bv = tsum - sum[rr];
            cmp[rr] += (sum[rr] - (tsum - bv)) + (w - bv);
            sum[rr] = tsum;
          }
        }
      };
      if (CL.P == 32) {
        if (own)
          pairs(std::true_type{}, std::true_type{});
        else
          pairs(std::false_type{}, std::true_type{});
      } else {
        if (own)
          pairs(std::true_type{}, std::false_type{});
        else
          pairs(std::false_type{}, std::false_type{});
      }
    }
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) {
      // the target's 64 / P partial sums (lanes l, l + P, ...), in FP64
      double mine = (double)sum[rr] + (double)cmp[rr];
      for (int o = CL.P; o < 64; o <<= 1) mine += __shfl_xor(mine, o);
      if (tv && lane < CL.P && r0 + rr < nrhs) D.fnear[(int64_t)i * nrhs + r0 + rr] = mine;
    }
  }
}

// ------------------------------------------------------------------ P2M
// W^I_m = sum_{y_j in I} sigma_j K(x_m^{I_0}, y_j - c_I)  (Algorithm 3, step 1)
// One NT-thread workgroup per leaf; rows are taken in groups of 4 NT, thread t
// owning rows m0 + t + NT u, u < 4, of group m0.  NT = 0: the launch's block size
// (one right-hand side on leaves of many points: a whole number of waves
// covering d_p, up to 1024, so that every wave takes one row per lane and none
// waits at the batch barriers for a wave with two); otherwise 256 threads
// (several right-hand sides: their registers rule out 1024-thread blocks), or
// one wave when d_p <= 64.
template <int KIND, int RB, bool BATCH, int NT>
__global__ __launch_bounds__(NT ? NT : 1024) void k_p2m(LeafDesc one,
                                                        const LeafDesc *__restrict__ many,
                                                        int nmany) {
  __shared__ double px[64], py[64], pz[64], ps[64 * RB];
  LeafDesc D;
  int j, prob;
  pick_desc<BATCH, 1>(one, many, nmany, D, j, prob);
  const int t = threadIdx.x;
  const int nt = NT ? NT : (int)blockDim.x;
  const int64_t n = D.n;
  const int nrhs = D.nrhs, d = D.d, dp = D.dp;
  const double *__restrict__ xyz = D.xyz;
  const double *__restrict__ sig = D.sig;
  const uint32_t key = D.act[j];
  const int a = D.ls[key], b = D.se[key];
  const double cx = D.lo0 + ((double)morton_axis(key, 0) + 0.5) * D.h;
  const double cy = D.lo1 + ((double)morton_axis(key, 1) + 0.5) * D.h;
  const double cz = D.lo2 + ((double)morton_axis(key, 2) + 0.5) * D.h;
  for (int m0 = 0; m0 < dp; m0 += 4 * nt) {
    const int nu = min(4, (dp - m0 + nt - 1) / nt);
    double xm[4], ym[4], zm[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int m = m0 + t + nt * u;
      const bool ok = u < nu && m < d;
      xm[u] = ok ? D.X[3 * m] : 0.0;
      ym[u] = ok ? D.X[3 * m + 1] : 0.0;
      zm[u] = ok ? D.X[3 * m + 2] : 0.0;
    }
    for (int r0 = 0; r0 < nrhs; r0 += RB) {
      double acc[4][RB];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int rr = 0; rr < RB; ++rr) acc[u][rr] = 0.0;
      for (int s0 = a; s0 < b; s0 += 64) {
        const int cnt = min(64, b - s0);
        __syncthreads();
        if (t < cnt) {
          const int s = s0 + t;
          px[t] = xyz[s] - cx;
          py[t] = xyz[n + s] - cy;
          pz[t] = xyz[2 * n + s] - cz;
#pragma unroll
          for (int rr = 0; rr < RB; ++rr)
            ps[t * RB + rr] = (r0 + rr < nrhs) ? sig[(int64_t)s * nrhs + r0 + rr] : 0.0;
        }
        __syncthreads();
        for (int q = 0; q < cnt; ++q) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            // skipped by a whole wave whose rows all lie past d (rows d..dp-1
            // are stored as zeros)
            if (u < nu && m0 + nt * u + (t & ~63) < d) {
              const double dx = xm[u] - px[q], dy = ym[u] - py[q], dz = zm[u] - pz[q];
              const double kv = KF<KIND>::eval(dx * dx + dy * dy + dz * dz, dx, D.p);
#pragma unroll
              for (int rr = 0; rr < RB; ++rr) acc[u][rr] += ps[q * RB + rr] * kv;
            }
          }
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int m = m0 + t + nt * u;
        if (u < nu && m < dp) {
#pragma unroll
          for (int rr = 0; rr < RB; ++rr)
            if (r0 + rr < nrhs)
              D.W[((int64_t)j * nrhs + r0 + rr) * dp + m] = m < d ? acc[u][rr] : 0.0;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ L2P + combine
// f(x_i) = sum_{l'} K(x_i - c_I, y_{l'}^{I_0}) lhat_{l'}^I + f_near(x_i), written to
// the input position of x_i (Algorithm 3, step 7).  One 64-lane workgroup per
// chunk of up to 32 targets: lane l and lane l + 32 hold the same target and sum
// the first and the second half of the d terms (a chunk of fewer targets
// spreads each over more lanes: chunk_lanes).
template <int KIND, int RB, bool BATCH>
__global__ __launch_bounds__(64) void k_l2p(LeafDesc one, IoDesc ione,
                                            const LeafDesc *__restrict__ many,
                                            const IoDesc *__restrict__ io, int nmany) {
  extern __shared__ double sm[];
  LeafDesc D;
  int c, prob;
  pick_desc<BATCH, 0>(one, many, nmany, D, c, prob);
  if (c >= D.chunk_ptr[D.nleaf]) return;  // past the last chunk (the grid is a bound)
  IoDesc O;
  if constexpr (BATCH)
    O = io[prob];
  else
    O = ione;
  // lhat and its points: the second EIM's size and y^{I_0} with two EIMs per level
  const int dp = D.dpL, d = D.dL, nrhs = D.nrhs;
  const int64_t n = D.n;
  double *sX = sm, *sl = sm + 3 * dp;
  const int lane = threadIdx.x;
  const int j = chunk_leaf(D.chunk_ptr, D.nleaf, c);
  const uint32_t key = D.act[j];
  // the chunk's lanes as in the near field: 64 / P lanes per target, each
  // summing one of 64 / P equal ranges of the d terms (P = 32: two halves)
  const ChunkLanes CL = chunk_lanes(D, j, c, lane, true);
  const int i = CL.i;
  const double cx = D.lo0 + ((double)morton_axis(key, 0) + 0.5) * D.h;
  const double cy = D.lo1 + ((double)morton_axis(key, 1) + 0.5) * D.h;
  const double cz = D.lo2 + ((double)morton_axis(key, 2) + 0.5) * D.h;
  for (int e = lane; e < 3 * d; e += 64) sX[e] = D.XL[e];
  const bool tv = CL.tv;
  const double xc = tv ? D.xyz[i] - cx : 0.0, yc = tv ? D.xyz[n + i] - cy : 0.0,
               zc = tv ? D.xyz[2 * n + i] - cz : 0.0;
  const int ng = 64 / CL.P, grp = lane / CL.P;
  const int dh = (d + ng - 1) / ng, l0 = grp * dh, l1 = min(d, l0 + dh);
  for (int r0 = 0; r0 < nrhs; r0 += RB) {
    __syncthreads();
    for (int e = lane; e < RB * d; e += 64) {
      const int rr = e / d, l = e - rr * d;
      sl[rr * dp + l] = (r0 + rr < nrhs) ? D.lhat[((int64_t)j * nrhs + r0 + rr) * dp + l] : 0.0;
    }
    __syncthreads();
    double acc[RB];
#pragma unroll
    for (int rr = 0; rr < RB; ++rr) acc[rr] = 0.0;
#pragma unroll 4
    for (int l = l0; l < l1; ++l) {
      const double dx = xc - sX[3 * l], dy = yc - sX[3 * l + 1], dz = zc - sX[3 * l + 2];
      const double kv = KF<KIND>::eval(dx * dx + dy * dy + dz * dz, dx, D.p);
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) acc[rr] += kv * sl[rr * dp + l];
    }
    for (int o = CL.P; o < 64; o <<= 1) {
#pragma unroll
      for (int rr = 0; rr < RB; ++rr) acc[rr] += __shfl_xor(acc[rr], o);
    }
    if (tv && lane < CL.P) {
      const int64_t o = D.perm[i] - D.toff;
#pragma unroll
      for (int rr = 0; rr < RB; ++rr)
        if (r0 + rr < nrhs)
          O.f[o + (int64_t)(r0 + rr) * O.ldf] = acc[rr] + D.fnear[(int64_t)i * nrhs + r0 + rr];
    }
  }
}

// depth < 2: no far field, f = f_near in input order
// (targets only: input indices from toff on)
__global__ void k_combine_near(int64_t n, int nrhs, const double *__restrict__ fnear,
                               const int *__restrict__ perm, int64_t toff, double *__restrict__ f,
                               int64_t ldf) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nrhs) return;
  int64_t s = e / nrhs;
  int r = (int)(e - s * nrhs);
  const int64_t o = (int64_t)perm[s] - toff;
  if (o >= 0) f[o + (int64_t)r * ldf] = fnear[e];
}

// ------------------------------------------------------------------ triangular solves
// One wave per 16 columns (box, rhs).  Forward substitution with the lower
// factor, then backward substitution with the upper factor, in 16-row tiles:
//   r_bi = v_bi - sum_{bj < bi} T[bi][bj] z_bj        (MFMA, -T tiles in the table)
//   z_bi = T[bi][bi]^{-1} r_bi                       (MFMA with the inverted tile)
// The solved tiles of the 16 columns stay in LDS.  In the FP64 16x16x4 MFMA the
// result register q of lane l holds row (l / 16) + 4 q of column l % 16, which
// is exactly the B operand that lane supplies at k-step q, so tiles feed the
// next product without data movement.
//   Delta   v: Gamma z = v, then B^T w = z
//   Delta^T v: B z = v,     then Gamma^T w = z
struct SolveArgs {
  SolveDesc lv[kMaxLevels];
  int nlev;
};

__device__ inline void trsm_body(const SolveDesc &D, double *zs) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x;
  const int c = ((int)blockIdx.x - D.blk_start) * 16 + (lane & 15);
  const bool cv = c < D.ncols;
  const int dp = D.dp, nb = dp >> 4, rs = lane >> 4;
  const double *x = D.in + (int64_t)(cv ? c : 0) * dp;
  double *y = D.out + (int64_t)(cv ? c : 0) * dp;
  // acc += sum over tiles j in [j0, j1) of row Ar's tile j times z_j, in two
  // accumulation chains (even and odd tiles).  The operator fragments of a pair
  // of tiles are loaded a pair ahead; past the end the loads read the row's last
  // tile, so the loads in flight do not depend on the data.
  auto row_sum = [&](const double *Ar, int j0, int j1, v4 &acc) {
    v4 acc2 = {0, 0, 0, 0};
    const int npair = (j1 - j0) >> 1;
    double fa[2][4], fb[2][4];
    auto load = [&](double(&f)[2][4], int j) {
      const int ja = min(j, nb - 1), jb = min(j + 1, nb - 1);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        f[0][ks] = Ar[ja * 256 + ks * 64];
        f[1][ks] = Ar[jb * 256 + ks * 64];
      }
    };
    auto mul = [&](const double(&f)[2][4], int j) {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(f[0][ks], zs[(j * 4 + ks) * 64 + lane], acc, 0,
                                                   0, 0);
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(f[1][ks], zs[((j + 1) * 4 + ks) * 64 + lane],
                                                    acc2, 0, 0, 0);
      }
    };
    int p = 0, j = j0;
    load(fa, j);
    for (; p + 2 <= npair; p += 2, j += 4) {
      load(fb, j + 2);
      mul(fa, j);
      load(fa, j + 4);
      mul(fb, j + 2);
    }
    if (p < npair) {
      mul(fa, j);
      j += 2;
    }
    if (j < j1) {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Ar[j * 256 + ks * 64],
                                                   zs[(j * 4 + ks) * 64 + lane], acc, 0, 0, 0);
    }
    acc += acc2;
  };
  if (!D.Tf) {
    // no forward factor (folded into the producers of the input): z = v
    for (int bi = 0; bi < nb; ++bi)
#pragma unroll
      for (int q = 0; q < 4; ++q) zs[(bi * 4 + q) * 64 + lane] = cv ? x[16 * bi + rs + 4 * q] : 0.0;
  }
  v4 xn;
#pragma unroll
  for (int q = 0; q < 4; ++q) xn[q] = (cv && D.Tf) ? x[rs + 4 * q] : 0.0;
  for (int bi = 0; D.Tf && bi < nb; ++bi) {
    v4 acc = xn;
    // the next row's right-hand side, loaded during this row's products
    const int bn = min(bi + 1, nb - 1);
#pragma unroll
    for (int q = 0; q < 4; ++q) xn[q] = cv ? x[16 * bn + rs + 4 * q] : 0.0;
    const double *Ar = D.Tf + (int64_t)bi * nb * 256 + lane;
    double dg[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) dg[ks] = Ar[bi * 256 + ks * 64];
    row_sum(Ar, 0, bi, acc);
    v4 z = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) z = __builtin_amdgcn_mfma_f64_16x16x4f64(dg[ks], acc[ks], z, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) zs[(bi * 4 + q) * 64 + lane] = z[q];
    if (!D.Tb && cv) {
#pragma unroll
      for (int q = 0; q < 4; ++q) y[16 * bi + rs + 4 * q] = z[q];
    }
  }
  if (!D.Tb) return;  // forward solve only
  for (int bi = nb - 1; bi >= 0; --bi) {
    v4 acc;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = zs[(bi * 4 + q) * 64 + lane];
    const double *Ar = D.Tb + (int64_t)bi * nb * 256 + lane;
    double dg[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) dg[ks] = Ar[bi * 256 + ks * 64];
    row_sum(Ar, bi + 1, nb, acc);
    v4 w = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) w = __builtin_amdgcn_mfma_f64_16x16x4f64(dg[ks], acc[ks], w, 0, 0, 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) zs[(bi * 4 + q) * 64 + lane] = w[q];
    if (cv) {
#pragma unroll
      for (int q = 0; q < 4; ++q) y[16 * bi + rs + 4 * q] = w[q];
      if (D.out32) {
        float *y32 = D.out32 + (int64_t)c * dp;
#pragma unroll
        for (int q = 0; q < 4; ++q) y32[16 * bi + rs + 4 * q] = (float)w[q];
      }
    }
  }
}

// LDS bytes of a solve launch: the solved tiles of the 16 columns
inline size_t trsm_shm(int dp) { return sizeof(double) * 4 * 64 * (size_t)(dp / 16); }

// one plan: up to one descriptor per level, passed by value
__global__ __launch_bounds__(64) void k_trsm(SolveArgs A) {
  extern __shared__ double zs[];  // [nb][4][64]
  int li = 0;
  for (int q = 1; q < A.nlev; ++q)
    if ((int)blockIdx.x >= A.lv[q].blk_start) li = q;
  trsm_body(A.lv[li], zs);
}

// a batch: every (problem, level) of the launch, descriptors in device memory
__global__ __launch_bounds__(64) void k_trsm_list(const SolveDesc *__restrict__ L, int n) {
  extern __shared__ double zs[];
  const int li = find_last_le(n, blockIdx.x, [&](int m) { return (int64_t)L[m].blk_start; });
  const SolveDesc D = L[li];
  trsm_body(D, zs);
}

// ------------------------------------------------------------------ gathered GEMM
// C[:, col] (+)= sum_t A_t B_t[:, col] for the columns (box, RHS) of a target
// group, where B_t[:, col] is the expansion of the source box that term t pairs
// with the column's target box: M2L the box at offset delta; M2M child t; L2L the
// parent; PROJ the box itself (compression projections).  A workgroup computes a
// (16 RBT)-row tile, 128 columns wide for 3 and 4 row blocks and 64 for 5 and 6,
// with 16x16x4 MFMAs; each of the 4 waves owns a quarter of the columns and all
// RBT row blocks.  The operator chunks of 16 k values pass through LDS in MFMA
// fragment order, loaded two chunks ahead of their products.  With FOLD (FP32
// operands) each term's product is accumulated by the MFMA in FP32 and then
// added to an FP64 sum over the terms, so FP32 rounding grows with one matrix
// product (d_k terms) rather than with the whole interaction list.
constexpr int MODE_M2M = 0, MODE_M2L = 1, MODE_L2L = 2, MODE_PROJ = 3;
// 16-column blocks per wave: 2 (128-column tiles) for 3- and 4-block tiles, 1
// (64 columns) for taller ones, whose accumulators and three sets of prefetched
// operands would not fit the registers of two waves per SIMD otherwise
__host__ __device__ constexpr int gemm_cpw(int rbt) { return rbt >= 5 ? 1 : 2; }
static_assert(gemm_cpw(6) == 1 && gemm_cpw(4) == 2 && gemm_cpw(3) == 2, "tile widths");
__host__ __device__ constexpr int gemm_cols(int rbt) { return 64 * gemm_cpw(rbt); }
constexpr int kMaxTerms = 189;   // terms of one job (M2L: the offsets of a child class)
// M2L: the tiles left after the whole-tile rounds are split in `parts` term
// ranges each (as many as the workspace holds pieces for, up to kMaxTailParts),
// taken by the workgroups from a counter as they finish, so that workgroups
// whose tiles skipped products take more of them.  The counter sits in the last
// kCounterDoubles of the Stream-K workspace; it is zero when a workspace is
// made, and the fixup that follows each such launch zeroes it.
constexpr int kMaxTailParts = 16;
// zeros, read in place of a missing source column or of operator rows past the
// operator, so that every chunk issues the same loads (static device memory is
// zero-initialized; 1024 covers the longest column, d_k <= 1024)
__device__ double g_gemm_zero[1024];
// the slots read for a missing source: no box (one per column of a lane, so that
// the dummy loads stay distinct loads)
__device__ int g_slot_none[2] = {-1, -1};

// Operand layouts (both types): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16].
// Result layouts differ: FP64 keeps rows (l / 16) + 4 q of column l % 16 in
// register q, FP32 rows 4 (l / 16) + q.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  typedef d2v p2;
  __device__ static inline v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int q) { return (lane >> 4) + 4 * q; }
};
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  typedef f2v p2;
  __device__ static inline v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};

// Where the slot of the source box that term `term` pairs with target (tkey, ts)
// is read: M2L the box at offset delta, M2M child `term`, L2L the parent (entries
// of the source level's slot map, which holds -1 for an empty box); PROJ needs
// no read (the box itself).  For a missing column or a source outside the
// domain the address is g_slot_none[jj] (-1, no box), so that every lane reads,
// the number of loads in flight does not depend on the data, and the value read
// needs no select (a select right after the load would wait for it).
template <int MODE>
__device__ inline const int *gemm_source_addr(const GemmJob &J, int term, bool cvalid,
                                              uint32_t tkey, const int *sdel,
                                              const int *__restrict__ src_slot, int jj) {
  uint32_t skey;
  bool v = cvalid;
  if constexpr (MODE == MODE_M2L) {
    const int pk = sdel[term];  // the term's offset, packed (LDS)
    const int side = 1 << J.level;
    const int m0 = (int)morton_axis(tkey, 0) + (pk & 7) - 3;
    const int m1 = (int)morton_axis(tkey, 1) + ((pk >> 3) & 7) - 3;
    const int m2 = (int)morton_axis(tkey, 2) + ((pk >> 6) & 7) - 3;
    v = v && m0 >= 0 && m1 >= 0 && m2 >= 0 && m0 < side && m1 < side && m2 < side;
    skey = morton_encode((uint32_t)m0, (uint32_t)m1, (uint32_t)m2);
  } else if constexpr (MODE == MODE_M2M) {
    skey = tkey * 8u + (uint32_t)term;
  } else {
    skey = tkey >> 3;
  }
  return (v && src_slot) ? src_slot + skey : &g_slot_none[jj];
}

template <typename T>
__device__ inline const T *gemm_source_ptr(const GemmJob &J, int s, int r, const T *Bsrc) {
  return s < 0 ? nullptr : Bsrc + ((int64_t)s * J.nrhs + r) * J.dpk;
}

template <typename T, int MODE>
__device__ inline const T *gemm_operand(const GemmJob &J, int term, const int *sdel) {
  int64_t idx;
  if constexpr (MODE == MODE_M2L)
    idx = sdel[term] >> 9;  // the offset id, from the LDS term table
  else if constexpr (MODE == MODE_M2M)
    idx = term;
  else if constexpr (MODE == MODE_L2L)
    idx = J.cls;
  else
    idx = 0;
  return (const T *)J.A + idx * J.a_stride;
}

// Schedule (data-parallel + Stream-K): the units of a launch are (tile, term)
// pairs numbered job by job, tile by tile, term by term.  With G persistent
// workgroups, the first F = floor(T / G) G tiles run whole, G at a time, all
// workgroups walking the terms in the same order (so the operators they read are
// shared in L2); within a round the tiles of one XCD are contiguous in space.
// The R units of the remaining tiles are split evenly over G_t = min(G, R)
// workgroups: workgroup g < G_t takes [S + B_g, S + B_{g+1}) with
// B_g = floor(g R / G_t) and S the first remaining unit.  A tile split between
// workgroups is stored in pieces (slot 2g for the first remaining tile of g,
// 2g + 1 for its last) that k_gemm_fixup adds in workgroup order, so results do
// not depend on timing.
__device__ inline int64_t sk_bound(int64_t g, int64_t units, int G) { return g * units / G; }

__device__ inline int find_job_units(const GemmJob *__restrict__ jobs, int njobs, int64_t u) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].units_start <= u)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline int find_job_tiles(const GemmJob *__restrict__ jobs, int njobs, int tile) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tiles_start <= tile)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// Source metadata of one target column of a gathered-GEMM tile.
struct ColState {
  const int *slot_map;  // slot map of the source level
  const void *B;        // source expansions
  uint32_t tkey;        // target key
  int tsl, r;           // target slot, right-hand side
  int valid;
};

// terms [term0, term1) of one tile; writes the result (part == nullptr) or a piece.
// A (the operators) is shared by the 4 waves and staged through LDS; each wave
// multiplies its own 32 columns, so B (the gathered source expansions) goes
// straight from memory to registers: within each 16-k chunk lane l supplies
// k = 4 (l / 16) + ks at k-step ks, four consecutive elements of its column, and
// the operator tables use the same k order (setup.cpp).
template <typename T, int MODE, bool FOLD, int RBT>
__device__ inline void gemm_tile(const GemmJob &J, int tile_local, int term0, int term1,
                                 double *__restrict__ part, const int8_t *__restrict__ dvec,
                                 T (*As)[RBT * 4 * 64], ColState *cst, int *sdel) {
  typedef typename Mfma<T>::v4 V4;
  typedef typename Mfma<T>::p2 P2;
  typedef double D4 __attribute__((ext_vector_type(4)));
  constexpr int CPW = gemm_cpw(RBT), COLS = 64 * CPW;
  constexpr int NA = RBT * 128;         // A chunk, in pairs
  constexpr int QA = (NA + 255) / 256;  // pairs per thread
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int rowtile = tile_local % J.nrowtiles, coltile = tile_local / J.nrowtiles;
  const int rb0 = rowtile * RBT, col0 = coltile * COLS;
  const int nrb = J.dpm >> 4, nks = J.dpk >> 2, nkc = J.dpk >> 4;
  const int ncols = J.ntgt * J.nrhs;
  const int koff = 4 * (lane >> 4);

  // the CPW columns of this lane (one per 16-column block of the wave); their
  // source metadata waits in LDS (this thread's own slots) until each term
  // starts, which keeps it out of the registers the accumulators need
  ColState *my = cst + CPW * t;
#pragma unroll
  for (int jj = 0; jj < CPW; ++jj) {
    const int jc = col0 + 16 * (CPW * w + jj) + (lane & 15);
    ColState c{};
    c.valid = jc < ncols;
    c.slot_map = J.src_slot;
    c.B = J.Bsrc;
    if (c.valid) {
      const int tt = jc / J.nrhs;
      c.r = jc - tt * J.nrhs;
      if (MODE == MODE_M2L && J.colref) {
        const ColRef cr = J.colref[tt];
        const ColSrc &cs = J.colsrc[cr.rec];
        c.tsl = cr.slot;
        c.tkey = ldg(cs.keys + cr.slot);
        c.slot_map = cs.slot;
        c.B = cs.B;
      } else {
        c.tsl = J.tgt ? ldg(J.tgt + tt) : tt;
        if (MODE != MODE_PROJ) c.tkey = ldg(J.tgt_keys + c.tsl);
      }
    }
    my[jj] = c;
  }
  // the job's terms in LDS, packed (dx+3) | (dy+3) << 3 | (dz+3) << 6 | id << 9
  // (offset and offset id): a source lookup then waits on no global load but
  // the slot map's, and the operator address on none.  Only the terms of
  // [term0, term1) whose source box lies inside the domain for some column of
  // the tile are kept, in order (the others would add zeros): the tile's target
  // boxes span [lo, hi] per axis, and offset delta reaches inside for some of
  // them on an axis when hi + delta >= 0 and lo + delta < side.  Boxes of one
  // child class and one face signature (the M2L column order) share their
  // missing offsets, so a tile of them drops those terms whole: their loads,
  // LDS staging and barriers as well as their products.
  if constexpr (MODE == MODE_M2L) {
    __shared__ int sbox[4][6];
    __shared__ int snk;
    int bb[6] = {INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
    for (int jj = 0; jj < CPW; ++jj) {
      const ColState c = my[jj];
      if (c.valid) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int m = (int)morton_axis(c.tkey, a);
          bb[a] = min(bb[a], m);
          bb[3 + a] = max(bb[3 + a], m);
        }
      }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        bb[a] = min(bb[a], __shfl_xor(bb[a], o));
        bb[3 + a] = max(bb[3 + a], __shfl_xor(bb[3 + a], o));
      }
    }
    if (lane < 6) sbox[w][lane] = bb[lane];
    lds_barrier();
    if (w == 0) {
      int lo[3], hi[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        lo[a] = min(min(sbox[0][a], sbox[1][a]), min(sbox[2][a], sbox[3][a]));
        hi[a] = max(max(sbox[0][3 + a], sbox[1][3 + a]), max(sbox[2][3 + a], sbox[3][3 + a]));
      }
      const int side = 1 << J.level;
      const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
      int nk = 0;
      for (int b = term0; b < term1; b += 64) {
        const int i = b + lane;
        bool keep = false;
        int pk = 0;
        if (i < term1) {
          const int id = ldg(J.terms + i);
          const int d0 = dvec[3 * id], d1 = dvec[3 * id + 1], d2 = dvec[3 * id + 2];
          pk = (d0 + 3) | ((d1 + 3) << 3) | ((d2 + 3) << 6) | (id << 9);
          keep = hi[0] + d0 >= 0 && lo[0] + d0 < side && hi[1] + d1 >= 0 && lo[1] + d1 < side &&
                 hi[2] + d2 >= 0 && lo[2] + d2 < side;
        }
        const uint64_t m = __ballot(keep);
        if (keep) sdel[nk + (int)__popcll(m & below)] = pk;
        nk += (int)__popcll(m);
      }
      if (lane == 0) snk = nk;
    }
    lds_barrier();
    term0 = 0;
    term1 = snk;
  }
  V4 acc[RBT][CPW];
  D4 sum[RBT][CPW];
  bool rowok[RBT];
#pragma unroll
  for (int i = 0; i < RBT; ++i) {
    rowok[i] = rb0 + i < nrb;
#pragma unroll
    for (int jj = 0; jj < CPW; ++jj) {
      acc[i][jj] = V4{0, 0, 0, 0};
      if constexpr (FOLD) sum[i][jj] = D4{0, 0, 0, 0};
    }
  }
  // Chunks are loaded two ahead of their products: during the products of
  // chunk it, the loads of chunk it + 2 are in flight and chunk it + 1 goes from
  // registers into the LDS buffer that chunk it - 1 used.  The barriers order
  // LDS accesses only, so loads stay in flight across them.  Three register sets
  // (R, B) rotate by name over a loop unrolled by 3 (a copy from a register a
  // load is filling would wait for that load), and every chunk issues the same
  // loads, so that the waits for them are exact.
  P2 R0[QA], R1[QA], R2[QA];               // A of a chunk, on its way to LDS
  P2 B0[CPW][2], B1[CPW][2], B2[CPW][2];   // B of a chunk: [column][pair]
  const T *srcp[CPW];
  const T *Ap = nullptr;
  // source slots of the next term (-1: none): read by the fetch of a term's
  // last chunk (the other fetches read g_slot_none), used at the next term's
  // first chunk
  int nslot[CPW];
#pragma unroll
  for (int jj = 0; jj < CPW; ++jj) {
    srcp[jj] = nullptr;
    nslot[jj] = -1;
  }
  auto lookup = [&](int term, bool real) {
#pragma unroll
    for (int jj = 0; jj < CPW; ++jj) {
      const ColState c = my[jj];
      if constexpr (MODE == MODE_PROJ) {
        nslot[jj] = c.valid ? c.tsl : -1;
      } else {
        const int *addr = &g_slot_none[jj];
        if (real) addr = gemm_source_addr<MODE>(J, term, c.valid, c.tkey, sdel, c.slot_map, jj);
        nslot[jj] = ldg(addr);
      }
    }
  };
  // loads chunk (fterm, fkc), the next one in order, into raD and bD; with live
  // false (past the last chunk) the same loads read zeros
  int fterm = term0, fkc = 0;
  const T *zero = (const T *)g_gemm_zero;
  // M2L: 1 when none of this wave's columns has a source in the current fetch
  // term; the wave's products would add zeros and are skipped
  uint32_t curskip = 0;
  auto fetch = [&](P2(&raD)[QA], P2(&bD)[CPW][2], uint32_t &skD, bool live) {
    const int term = fterm, kc = fkc;
    if (live) {
      if (++fkc == nkc) {
        fkc = 0;
        ++fterm;
      }
      if (kc == 0) {
#pragma unroll
        for (int jj = 0; jj < CPW; ++jj) {
          const ColState c = my[jj];
          srcp[jj] = gemm_source_ptr<T>(J, nslot[jj], c.r, (const T *)c.B);
        }
        Ap = gemm_operand<T, MODE>(J, term, sdel);
        if constexpr (MODE == MODE_M2L) {
          bool any = false;
#pragma unroll
          for (int jj = 0; jj < CPW; ++jj) any = any || srcp[jj] != nullptr;
          curskip = __ballot(any) == 0 ? 1u : 0u;
        }
      }
    }
    skD = curskip;
    // the slots of the next term, at the term's last chunk
    lookup(term + 1, live && kc == nkc - 1 && term + 1 < term1);
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = t + 256 * q;  // pair index in the chunk
      const int rb = rb0 + (e >> 7);
      if (e < NA) {
        const T *src = (live && rb < nrb) ? Ap + ((int64_t)rb * nks + kc * 4) * 64 : zero;
        raD[q] = ldg((const P2 *)(src + 2 * (e & 127)));
      }
    }
#pragma unroll
    for (int jj = 0; jj < CPW; ++jj) {
      const T *col = (live && srcp[jj]) ? srcp[jj] + kc * 16 : zero;
      const P2 *s2 = (const P2 *)(col + koff);
      bD[jj][0] = ldg(s2);
      bD[jj][1] = ldg(s2 + 1);
    }
  };
  auto stash = [&](int buf, const P2(&raS)[QA]) {
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      const int e = t + 256 * q;
      if (e < NA) *(P2 *)(&As[buf][2 * e]) = raS[q];
    }
  };
  const int it0 = term0 * nkc, it1 = term1 * nkc;
  int mkc = 0;  // k chunk of the current term
  // the products of chunk it (its A in LDS buffer (it - it0) & 1, its B in Bc),
  // with the loads of chunk it + 2 into (Rf, Bf) and chunk it + 1 (Rn) stashed
  // The products of a chunk's last k-step are deferred to the start of the next
  // step, after the barrier, so that their MFMAs run while the wave issues the
  // next chunk's loads (a branch around the products, for the skipped terms,
  // would otherwise keep the compiler from moving them there); their operands
  // wait in registers.  With FOLD a term's sum is folded after them.
  T a3[RBT], b3[CPW];
  bool dpend = false, fpend = false;  // deferred products and fold pending (wave-uniform)
  auto deferred = [&]() {
    if (dpend) {
#pragma unroll
      for (int i = 0; i < RBT; ++i)
        if (RBT != 6 || rowok[i]) {
#pragma unroll
          for (int jj = 0; jj < CPW; ++jj) acc[i][jj] = Mfma<T>::op(a3[i], b3[jj], acc[i][jj]);
        }
    }
    if constexpr (FOLD) {
      if (fpend) {  // a term is complete
#pragma unroll
        for (int i = 0; i < RBT; ++i)
#pragma unroll
          for (int jj = 0; jj < CPW; ++jj) {
#pragma unroll
            for (int q = 0; q < 4; ++q) sum[i][jj][q] += (double)acc[i][jj][q];
            acc[i][jj] = V4{0, 0, 0, 0};
          }
      }
    }
    dpend = false;
    fpend = false;
  };
  // k-steps 0..2 of one chunk, and the operands of k-step 3
  auto products = [&](int cur, const P2(&Bc)[CPW][2]) {
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) {
      T a[RBT], b[CPW];
#pragma unroll
      for (int i = 0; i < RBT; ++i) a[i] = As[cur][(i * 4 + ks) * 64 + lane];
#pragma unroll
      for (int jj = 0; jj < CPW; ++jj) b[jj] = (ks & 1) ? Bc[jj][ks >> 1].y : Bc[jj][ks >> 1].x;
      // every row block is multiplied (except with 6 blocks): the A chunk holds
      // zeros beyond the operator's rows (their results are not stored), and a
      // branch per block would split the products into pieces that each wait for
      // their LDS reads.  With 6 blocks the unbranched form runs out of registers.
#pragma unroll
      for (int i = 0; i < RBT; ++i)
        if (RBT != 6 || rowok[i]) {
#pragma unroll
          for (int jj = 0; jj < CPW; ++jj) acc[i][jj] = Mfma<T>::op(a[i], b[jj], acc[i][jj]);
        }
    }
#pragma unroll
    for (int i = 0; i < RBT; ++i) a3[i] = As[cur][(i * 4 + 3) * 64 + lane];
#pragma unroll
    for (int jj = 0; jj < CPW; ++jj) b3[jj] = Bc[jj][1].y;
  };
  auto step = [&](int it, const P2(&Bc)[CPW][2], uint32_t skc, const P2(&Rn)[QA], P2(&Rf)[QA],
                  P2(&Bf)[CPW][2], uint32_t &skf) {
    const int cur = (it - it0) & 1;
    deferred();  // the previous chunk's last k-step
    fetch(Rf, Bf, skf, it + 2 < it1);
    stash(cur ^ 1, Rn);
    const bool run = MODE != MODE_M2L || skc == 0;
    if (run) products(cur, Bc);
    dpend = run;
    if (++mkc == nkc) {
      mkc = 0;
      fpend = FOLD;
    }
    lds_barrier();
  };

  if (it0 < it1) {
    lookup(term0, true);
    uint32_t S0 = 0, S1 = 0, S2 = 0;  // skip flags of the chunks in B0, B1, B2
    fetch(R0, B0, S0, true);
    stash(0, R0);
    fetch(R1, B1, S1, it0 + 1 < it1);
    lds_barrier();
    int it = it0;
    for (; it + 3 <= it1; it += 3) {
      step(it, B0, S0, R1, R2, B2, S2);
      step(it + 1, B1, S1, R2, R0, B0, S0);
      step(it + 2, B2, S2, R0, R1, B1, S1);
    }
    if (it < it1) step(it, B0, S0, R1, R2, B2, S2);
    if (it + 1 < it1) step(it + 1, B1, S1, R2, R0, B0, S0);
    deferred();
  }

#pragma unroll
  for (int jj = 0; jj < CPW; ++jj) {
    const int jt = 16 * (CPW * w + jj) + (lane & 15);
    const int jo = col0 + jt;
    if (jo >= ncols) continue;
    const int tt = jo / J.nrhs, ro = jo - tt * J.nrhs;
    int tso;
    double *Cout = J.C;
    if (MODE == MODE_M2L && J.colref) {
      const ColRef cr = J.colref[tt];
      tso = cr.slot;
      Cout = J.colsrc[cr.rec].C;
    } else {
      tso = J.tgt ? ldg(J.tgt + tt) : tt;
    }
    const int64_t cbase = ((int64_t)tso * J.nrhs + ro) * J.dpm;
#pragma unroll
    for (int i = 0; i < RBT; ++i) {
      if (!rowok[i]) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int rt = 16 * i + Mfma<T>::row(lane, q);
        double v;
        if constexpr (FOLD)
          v = sum[i][jj][q];
        else
          v = (double)acc[i][jj][q];
        if (part) {
          stg(part + (size_t)rt * COLS + jt, v);
        } else {
          const int64_t o = cbase + 16 * rb0 + rt;
          if constexpr (MODE == MODE_L2L) v += ldg(J.Cadd + o);
          stg(Cout + o, v);
          if (J.C32) stg(J.C32 + o, (float)v);
        }
      }
    }
  }
}

template <typename T, int MODE, bool FOLD, int RBT>
__global__ __launch_bounds__(256, 2) void k_gemm(const GemmJob *__restrict__ jobs, int njobs,
                                                 int ntiles, int64_t units, int G, int GT,
                                                 double *__restrict__ ws,
                                                 const int8_t *__restrict__ dvec, int dyn_items,
                                                 int parts, int *__restrict__ ctr) {
  constexpr int TILE = RBT * 16 * 64 * gemm_cpw(RBT);
  __shared__ T As[2][RBT * 4 * 64];
  __shared__ ColState cst[2 * 256];
  __shared__ int sdel[kMaxTerms];
  const int g = blockIdx.x;
  // whole tiles, G at a time; the tiles of one XCD (g mod 8) are contiguous
  const int full = (ntiles / G) * G;
  const int per = G / 8;
  const int gx = (G % 8 == 0) ? (g % 8) * per + g / 8 : g;
  for (int t0 = 0; t0 < full; t0 += G) {
    const int tile = t0 + gx;
    const GemmJob J = jobs[find_job_tiles(jobs, njobs, tile)];
    gemm_tile<T, MODE, FOLD, RBT>(J, tile - J.tiles_start, 0, J.nterms, nullptr, dvec, As,
                                  cst, sdel);
  }
  if (full == ntiles) return;
  if (MODE == MODE_M2L && dyn_items > 0) {
    // the remaining tiles, `parts` pieces each, taken in order from the counter
    __shared__ int item_sh;
    for (;;) {
      if (threadIdx.x == 0) item_sh = atomicAdd(ctr, 1);
      __syncthreads();
      const int item = item_sh;
      __syncthreads();
      if ((unsigned)item >= (unsigned)dyn_items) return;  // done (or a stale counter)
      const int tile = full + item / parts, q = item % parts;
      const GemmJob J = jobs[find_job_tiles(jobs, njobs, tile)];
      gemm_tile<T, MODE, FOLD, RBT>(J, tile - J.tiles_start, q * J.nterms / parts,
                                    (q + 1) * J.nterms / parts, ws + (size_t)item * TILE,
                                    dvec, As, cst, sdel);
    }
  }
  // the remaining units, split evenly
  const GemmJob Jr = jobs[find_job_tiles(jobs, njobs, full)];
  const int64_t S = Jr.units_start + (int64_t)(full - Jr.tiles_start) * Jr.nterms;
  const int64_t R = units - S;
  // workgroups sharing the tail (at most GT, so that the 2 GT pieces fit the
  // workspace): each owns >= 1 unit
  const int Gt = (int)min((int64_t)GT, R);
  if (g >= Gt) return;
  const int64_t ua = S + sk_bound(g, R, Gt), ub = S + sk_bound(g + 1, R, Gt);
  for (int64_t u = ua; u < ub;) {
    const GemmJob J = jobs[find_job_units(jobs, njobs, u)];
    const int64_t local = u - J.units_start;
    const int tile_local = (int)(local / J.nterms);
    const int term0 = (int)(local - (int64_t)tile_local * J.nterms);
    const int64_t ts = J.units_start + (int64_t)tile_local * J.nterms;
    const int term1 = (int)(min(ts + J.nterms, ub) - ts);
    u = ts + term1;
    const bool whole = term0 == 0 && term1 == J.nterms;
    double *part = whole ? nullptr : ws + (size_t)(2 * g + (ua >= ts ? 0 : 1)) * TILE;
    gemm_tile<T, MODE, FOLD, RBT>(J, tile_local, term0, term1, part, dvec, As, cst, sdel);
  }
}

// Adds the pieces of the tiles split between workgroups; kFixupSplit blocks per
// tile, each adding a slice of its elements.  The workgroups meeting a tile are
// consecutive, glo..ghi: glo's piece is in slot 2 glo + 1 unless glo starts at
// the tile (then 2 glo), the others start inside it (slot 2 g).  The pieces are
// added in workgroup order, 8 loads in flight at a time.
constexpr int kFixupSplit = 4;
template <int RBT>
__global__ __launch_bounds__(256) void k_gemm_fixup(const GemmJob *__restrict__ jobs, int njobs,
                                                    int ntiles, int64_t units, int G, int GT,
                                                    const double *__restrict__ ws, int dyn_items,
                                                    int parts, int *__restrict__ ctr) {
  constexpr int COLS = 64 * gemm_cpw(RBT), TILE = RBT * 16 * COLS;
  constexpr int SLICE = TILE / kFixupSplit;
  static_assert(SLICE % 256 == 0 && 256 % COLS == 0, "fixup slices");
  const int full = (ntiles / G) * G;
  const int tile = full + (int)(blockIdx.x / kFixupSplit);
  const int slice = (int)(blockIdx.x % kFixupSplit);
  if (dyn_items > 0 && blockIdx.x == 0 && threadIdx.x == 0) stg(ctr, 0);  // for the next launch
  if (tile >= ntiles) return;
  const GemmJob J = jobs[find_job_tiles(jobs, njobs, tile)];
  const int tile_local = tile - J.tiles_start;
  int64_t glo;
  int np, first;
  if (dyn_items > 0) {
    // `parts` pieces in slots (tile - full) parts + q
    np = parts;
    first = (tile - full) * parts;
    glo = 0;
  } else {
    const GemmJob Jr = jobs[find_job_tiles(jobs, njobs, full)];
    const int64_t S = Jr.units_start + (int64_t)(full - Jr.tiles_start) * Jr.nterms;
    const int64_t R = units - S;
    const int Gt = (int)min((int64_t)GT, R);
    // unit range of the tile relative to S; workgroup g starts at unit
    // sk_bound(g) = floor(g R / Gt), so the last one starting at or before ts is
    // floor(((ts + 1) Gt - 1) / R) and the last one starting before te is
    // floor((te Gt - 1) / R)
    const int64_t ts = J.units_start + (int64_t)tile_local * J.nterms - S, te = ts + J.nterms;
    glo = min(((ts + 1) * Gt - 1) / R, (int64_t)Gt - 1);
    const int64_t ghi = min((te * Gt - 1) / R, (int64_t)Gt - 1);
    if (ghi == glo) return;  // written directly
    np = (int)(ghi - glo + 1);
    first = (int)(2 * glo + (sk_bound(glo, R, Gt) == ts ? 0 : 1));
  }
  // slot of piece i: consecutive slots for the counter's pieces; for the even
  // split, glo's piece then the first slot of each later workgroup
  const bool dyn = dyn_items > 0;
  auto slot_of = [&](int i) { return dyn ? first + i : (i == 0 ? first : (int)(2 * (glo + i))); };
  const int rowtile = tile_local % J.nrowtiles, coltile = tile_local / J.nrowtiles;
  const int rb0 = rowtile * RBT, col0 = coltile * COLS;
  const int nrows = min(RBT * 16, J.dpm - 16 * rb0);
  const int ncols = J.ntgt * J.nrhs;
  // this thread's column (the same for all its elements, 256 being a multiple of COLS)
  const int jt = (int)threadIdx.x % COLS;
  const int jo = col0 + jt;
  if (jo >= ncols) return;
  const int tt = jo / J.nrhs, ro = jo - tt * J.nrhs;
  int tso;
  double *Cout = J.C;
  if (J.colref) {
    const ColRef cr = J.colref[tt];
    tso = cr.slot;
    Cout = J.colsrc[cr.rec].C;
  } else {
    tso = J.tgt ? ldg(J.tgt + tt) : tt;
  }
  const int64_t obase = ((int64_t)tso * J.nrhs + ro) * J.dpm + 16 * rb0;
  for (int e = slice * SLICE + (int)threadIdx.x; e < (slice + 1) * SLICE; e += 256) {
    const int rt = e / COLS;
    if (rt >= nrows) break;
    double v = 0.0;
    int i = 0;
    for (; i + 8 <= np; i += 8) {
      double p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) p[u] = ldg(ws + (size_t)slot_of(i + u) * TILE + e);
#pragma unroll
      for (int u = 0; u < 8; ++u) v += p[u];
    }
    for (; i < np; ++i) v += ldg(ws + (size_t)slot_of(i) * TILE + e);
    const int64_t o = obase + rt;
    if (J.mode == MODE_L2L) v += ldg(J.Cadd + o);
    stg(Cout + o, v);
    if (J.C32) stg(J.C32 + o, (float)v);
  }
}

// ------------------------------------------------------------------ factored M2L
// Second compression stage (Sec. 4.2): per offset o the r x r matrix C^delta is
// the product Ut_o Vt_o of an r x s_o and an s_o x r factor, so a column's
// contribution is Ut_o (Vt_o w), w the What' column of its source.  A work item is
// (64-column tile, range of terms); each of the 4 waves owns 16 columns and all
// rp rows of g'.  Per term a wave forms t = Vt_o w (s_o x 16) on FP64 MFMA, with
// w loaded straight from memory in the gathered GEMM's k order, then
// g' += Ut_o t, feeding t from its result registers as the B operand: result
// register q of lane l holds row (l / 16) + 4 q, the k order of the Ut fragments.
// Factor fragments are read from memory; the tiles of a class walk the same terms
// in the same order, so they stay in L1 / L2.
constexpr int kM2l2Sb = kMaxRank2 / 16;  // most 16-row blocks of t

template <int RB>
__global__ __launch_bounds__(256, 2) void k_m2l2(const M2l2Job *__restrict__ jobs, int njobs,
                                                 int nitems, const int8_t *__restrict__ dvec,
                                                 double *__restrict__ ws) {
  typedef double v4 __attribute__((ext_vector_type(4)));
  constexpr int rp = 16 * RB;
  const int item = blockIdx.x;
  if (item >= nitems) return;
  const int ji = find_last_le(njobs, item, [&](int m) { return (int64_t)jobs[m].item_start; });
  const M2l2Job J = jobs[ji];
  const int local = item - J.item_start;
  const int tile = local / kM2l2Parts, part = local - tile * kM2l2Parts;
  const int term0 = 189 * part / kM2l2Parts, term1 = 189 * (part + 1) / kM2l2Parts;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = tile * 64 + 16 * w + (lane & 15);
  const bool cv = col < J.ntgt * J.nrhs;
  const int tt = cv ? col / J.nrhs : 0;
  const int rr = cv ? col - tt * J.nrhs : 0;
  const int tsl = cv ? J.tgt[tt] : 0;
  const uint32_t tkey = cv ? J.keys[tsl] : 0u;
  const int side = 1 << J.level;
  const int c0 = (int)morton_axis(tkey, 0), c1 = (int)morton_axis(tkey, 1),
            c2 = (int)morton_axis(tkey, 2);
  const int g4 = 4 * (lane >> 4);
  v4 acc[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) acc[rb] = v4{0, 0, 0, 0};
  for (int term = term0; term < term1; ++term) {
    const int o = J.terms[term];
    const int sp = J.sp[o];
    if (sp == 0) continue;
    const int nsb = sp >> 4;
    int sl = -1;
    if (cv) {
      const int m0 = c0 + dvec[3 * o], m1 = c1 + dvec[3 * o + 1], m2 = c2 + dvec[3 * o + 2];
      if (m0 >= 0 && m1 >= 0 && m2 >= 0 && m0 < side && m1 < side && m2 < side)
        sl = J.slot[morton_encode((uint32_t)m0, (uint32_t)m1, (uint32_t)m2)];
    }
    const double *src = sl >= 0 ? J.B + ((int64_t)sl * J.nrhs + rr) * rp : nullptr;
    const double *V = J.vf + J.voff[o] + lane;
    const double *U = J.uf + J.uoff[o] + lane;
    v4 t[kM2l2Sb];
#pragma unroll
    for (int sb = 0; sb < kM2l2Sb; ++sb) t[sb] = v4{0, 0, 0, 0};
    // t = Vt_o w
#pragma unroll
    for (int kc = 0; kc < RB; ++kc) {
      double b[4] = {0, 0, 0, 0};
      if (src) {
        const double2 *s2 = (const double2 *)(src + kc * 16 + g4);
        const double2 x = s2[0], y = s2[1];
        b[0] = x.x;
        b[1] = x.y;
        b[2] = y.x;
        b[3] = y.y;
      }
#pragma unroll
      for (int sb = 0; sb < kM2l2Sb; ++sb)
        if (sb < nsb) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            t[sb] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                V[((int64_t)sb * (rp / 4) + kc * 4 + q) * 64], b[q], t[sb], 0, 0, 0);
        }
    }
    // g' += Ut_o t
#pragma unroll
    for (int sb = 0; sb < kM2l2Sb; ++sb)
      if (sb < nsb) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
            acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                U[((int64_t)rb * (sp / 4) + sb * 4 + q) * 64], t[sb][q], acc[rb], 0, 0, 0);
      }
  }
  // partial block of the item, column-major: ws[item][column][row]
  double *out = ws + (size_t)item * rp * 64 + (size_t)(16 * w + (lane & 15)) * rp;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int q = 0; q < 4; ++q) out[16 * rb + (lane >> 4) + 4 * q] = acc[rb][q];
}

// g' of each tile: the kM2l2Parts partial blocks added in part order
__global__ __launch_bounds__(256) void k_m2l2_sum(const M2l2Job *__restrict__ jobs, int njobs,
                                                  int ntiles, const double *__restrict__ ws) {
  const int tg = blockIdx.x;
  if (tg >= ntiles) return;
  const int ji = find_last_le(njobs, tg, [&](int m) { return (int64_t)jobs[m].tile_start; });
  const M2l2Job J = jobs[ji];
  const int tile = tg - J.tile_start, rp = J.rp;
  const int ncols = J.ntgt * J.nrhs;
  const size_t blk = (size_t)rp * 64;
  const double *base = ws + (size_t)(J.item_start + tile * kM2l2Parts) * blk;
  for (int e = threadIdx.x; e < rp * 64; e += 256) {
    const int jc = e / rp, row = e - jc * rp;
    const int col = tile * 64 + jc;
    if (col >= ncols) continue;
    double v = 0.0;
#pragma unroll
    for (int p = 0; p < kM2l2Parts; ++p) v += base[p * blk + e];
    const int tt = col / J.nrhs, r = col - tt * J.nrhs;
    J.C[((int64_t)J.tgt[tt] * J.nrhs + r) * rp + row] = v;
  }
}

template <int RB>
void launch_m2l2_rb(const M2l2Job *jobs, const M2l2Launch &L, const int8_t *dvec, double *ws,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_m2l2<RB>, dim3(L.nitems), dim3(256), 0, s, jobs + L.first_job, L.njobs,
                     L.nitems, dvec, ws + L.ws_off);
  hipLaunchKernelGGL(k_m2l2_sum, dim3(L.ntiles), dim3(256), 0, s, jobs + L.first_job, L.njobs,
                     L.ntiles, ws + L.ws_off);
}

void launch_m2l2(const M2l2Job *jobs, const M2l2Launch &L, const int8_t *dvec, double *ws,
                 hipStream_t s) {
  if (L.nitems == 0) return;
  switch (L.rb) {
    case 4: launch_m2l2_rb<4>(jobs, L, dvec, ws, s); break;
    case 5: launch_m2l2_rb<5>(jobs, L, dvec, ws, s); break;
    case 6: launch_m2l2_rb<6>(jobs, L, dvec, ws, s); break;
    case 7: launch_m2l2_rb<7>(jobs, L, dvec, ws, s); break;
    case 8: launch_m2l2_rb<8>(jobs, L, dvec, ws, s); break;
    case 9: launch_m2l2_rb<9>(jobs, L, dvec, ws, s); break;
    case 10: launch_m2l2_rb<10>(jobs, L, dvec, ws, s); break;
    case 11: launch_m2l2_rb<11>(jobs, L, dvec, ws, s); break;
    case 12: launch_m2l2_rb<12>(jobs, L, dvec, ws, s); break;
    case 13: launch_m2l2_rb<13>(jobs, L, dvec, ws, s); break;
    case 14: launch_m2l2_rb<14>(jobs, L, dvec, ws, s); break;
    case 15: launch_m2l2_rb<15>(jobs, L, dvec, ws, s); break;
    default: launch_m2l2_rb<16>(jobs, L, dvec, ws, s); break;
  }
}

// ------------------------------------------------------------------ host side
namespace {

// Per-phase HIP events; elapsed times are collected by timing_drain.
struct Timer {
  Plan &P;
  hipStream_t s;
  EventPair ep;
  bool on;
  Timer(Plan &P_, hipStream_t s_, int ph)
      : P(P_), s(s_), on(P_.timing == 1 || (P_.timing == 2 && ph == EIFMM_PH_M2L)) {
    if (!on) return;
    if (P.ev_pending.size() > 4096) timing_drain(P);
    if (P.ev_free.empty()) {
      EventPair e;
      hipEventCreate(&e.a);
      hipEventCreate(&e.b);
      P.ev_free.push_back(e);
    }
    ep = P.ev_free.back();
    P.ev_free.pop_back();
    ep.phase = ph;
    hipEventRecord(ep.a, s);
  }
  ~Timer() {
    if (!on) return;
    hipEventRecord(ep.b, s);
    P.ev_pending.push_back(ep);
  }
};

int tiles_of(const GemmJob &J) { return J.ncoltiles * J.nrowtiles; }

void finish_job(GemmJob &J, int &tiles, int rbt) {
  const int ncols = J.ntgt * J.nrhs;
  J.ncoltiles = (ncols + gemm_cols(rbt) - 1) / gemm_cols(rbt);
  J.nrowtiles = (J.dpm / 16 + rbt - 1) / rbt;
  J.tiles_start = tiles;
  tiles += tiles_of(J);
}

// unit offsets (tile x term) of the jobs of one launch group
int64_t finish_units(std::vector<GemmJob> &h, int first) {
  int64_t u = 0;
  for (size_t j = first; j < h.size(); ++j) {
    h[j].units_start = u;
    u += (int64_t)tiles_of(h[j]) * h[j].nterms;
  }
  return u;
}

}  // namespace

// Job tables of a (points, nrhs) pair, uploaded once and reused.
int build_jobs(Plan &P, int nrhs, hipStream_t s) {
  const int depth = P.depth;
  const bool mixed = P.cfg.precision == EIFMM_PREC_MIXED;
  std::vector<GemmJob> h;
  auto &jt = P.jobs;
  jt = JobTables{};
  // M2M, one job per parent level k = depth-1 .. 2
  for (int k = depth - 1; k >= 2; --k) {
    int tiles = 0;
    GemmJob J{};
    J.A = P.ld[k].m2m;
    J.Bsrc = P.ld[k + 1].W;
    J.C = P.ld[k].W;
    J.tgt = nullptr;
    J.tgt_keys = P.ld[k].act;
    J.src_slot = P.ld[k + 1].slot;
    J.a_stride = (int64_t)P.lh[k].dp * P.lh[k + 1].dp;
    J.ntgt = (int)P.nact[k];
    J.nterms = 8;
    J.dpm = P.lh[k].dp;
    J.dpk = P.lh[k + 1].dp;
    J.level = k;
    J.mode = MODE_M2M;
    J.nrhs = nrhs;
    jt.m2m_rbt[k] = pick_rbt(J.dpm / 16);
    finish_job(J, tiles, jt.m2m_rbt[k]);
    jt.m2m_first[k] = (int)h.size();
    jt.m2m_n[k] = 1;
    jt.m2m_tiles[k] = tiles;
    h.push_back(J);
    jt.m2m_units[k] = finish_units(h, jt.m2m_first[k]);
  }
  // compression projections What' = U^T B^{-T} z with z = Gamma^{-1} W from the
  // forward solve, one job per compressed level (What' = (U^T B^{-T} Gamma^{-1}) W
  // from W itself where the operator folds the solve in)
  {
    int tiles = 0;
    jt.pre_first = (int)h.size();
    jt.pre_rbt = pick_rbt(P.lh[depth].rp / 16 > 0 ? P.lh[depth].rp / 16 : 1);
    double pf = 0;
    for (int k = depth; k >= 2; --k) {
      if (P.lh[k].r == 0 || P.nact[k] == 0) continue;
      GemmJob J{};
      J.A = P.ld[k].pfrag;
      J.Bsrc = P.lh[k].fold_what ? P.ld[k].W : P.ld[k].Wh;
      J.C = P.ld[k].Whp;
      J.C32 = mixed ? P.ld[k].Whp32 : nullptr;
      J.ntgt = (int)P.nact[k];
      J.nterms = 1;
      J.dpm = P.lh[k].rp;
      J.dpk = P.lh[k].dp;
      J.level = k;
      J.mode = MODE_PROJ;
      J.nrhs = nrhs;
      finish_job(J, tiles, jt.pre_rbt);
      h.push_back(J);
      pf += 2.0 * (P.lh[k].d + P.lh[k].dB) * (double)P.lh[k].r * (double)P.nact[k] * nrhs;
    }
    jt.pre_n = (int)h.size() - jt.pre_first;
    jt.pre_tiles = tiles;
    jt.pre_units = finish_units(h, jt.pre_first);
    P.proj_flops = pf;
  }
  // M2L, every level in one launch, finest level first
  {
    int tiles = 0;
    jt.m2l_first = (int)h.size();
    const LevelHost &F = P.lh[depth];
    jt.m2l_rbt = pick_rbt((F.r ? F.rp : F.dpB) / 16);
    for (int k = depth; k >= 2; --k) {
      if (uses_m2l2(P, k)) continue;  // the factored M2L below
      const bool cz = P.lh[k].r > 0;
      // rows: g (the second EIM's size); columns: What
      const int dm = cz ? P.lh[k].rp : P.lh[k].dpB, dk = cz ? P.lh[k].rp : P.lh[k].dp;
      for (int c = 0; c < 8; ++c) {
        const int64_t nt = P.cls_off[k][c + 1] - P.cls_off[k][c];
        if (nt == 0) continue;
        GemmJob J{};
        J.A = mixed ? (const void *)P.ld[k].kfrag32 : (const void *)P.ld[k].kfrag;
        if (cz)
          J.Bsrc = mixed ? (const void *)P.ld[k].Whp32 : (const void *)P.ld[k].Whp;
        else
          J.Bsrc = mixed ? (const void *)P.ld[k].Wh32 : (const void *)P.ld[k].Wh;
        J.C = cz ? P.ld[k].gp : P.ld[k].g;
        J.tgt = (P.ld[k].ord ? P.ld[k].ord : P.ld[k].cls) + P.cls_off[k][c];
        J.tgt_keys = P.ld[k].act;
        J.src_slot = P.ld[k].slot;
        J.terms = P.dlist + 189 * c;
        J.a_stride = (int64_t)dm * dk;
        J.ntgt = (int)nt;
        J.nterms = 189;
        J.dpm = dm;
        J.dpk = dk;
        J.level = k;
        J.cls = c;
        J.mode = MODE_M2L;
        J.nrhs = nrhs;
        finish_job(J, tiles, jt.m2l_rbt);
        h.push_back(J);
      }
    }
    jt.m2l_n = (int)h.size() - jt.m2l_first;
    jt.m2l_tiles = tiles;
    jt.m2l_units = finish_units(h, jt.m2l_first);
    // executed work: every column walks all terms of its class, over whole row
    // tiles of the padded operators
    double fx = 0;
    for (int j = jt.m2l_first; j < jt.m2l_first + jt.m2l_n; ++j)
      fx += 2.0 * (double)h[j].nrowtiles * 16 * jt.m2l_rbt * h[j].dpk * (double)h[j].ntgt *
            h[j].nrhs * h[j].nterms;
    P.m2l_flops_exec = fx;
    // factored M2L levels: one job per child class, grouped by rp; algorithmic
    // flops 2 (r s_o + s_o r) per interaction pair, with the mean s_o over the
    // 316 offsets standing in for the offsets the pairs actually use
    auto &mj = P.m2l2_host;
    auto &ml = P.m2l2_launch;
    mj.clear();
    ml.clear();
    int item = 0, tilec = 0;
    for (int rb = kM2l2RbMin; rb <= kM2l2RbMax; ++rb) {
      M2l2Launch L{(int)mj.size(), 0, item, 0, tilec, 0, rb};
      for (int k = depth; k >= 2; --k) {
        if (!uses_m2l2(P, k) || P.lh[k].rp != 16 * rb) continue;
        for (int c = 0; c < 8; ++c) {
          const int64_t nt = P.cls_off[k][c + 1] - P.cls_off[k][c];
          if (nt == 0) continue;
          M2l2Job J{};
          J.tgt = P.ld[k].cls + P.cls_off[k][c];
          J.keys = P.ld[k].act;
          J.slot = P.ld[k].slot;
          J.B = P.ld[k].Whp;
          J.C = P.ld[k].gp;
          J.terms = P.dlist + 189 * c;
          J.vf = P.ld[k].vf2;
          J.uf = P.ld[k].uf2;
          J.voff = P.ld[k].voff2;
          J.uoff = P.ld[k].uoff2;
          J.sp = P.ld[k].sp2;
          J.ntgt = (int)nt;
          J.nrhs = nrhs;
          J.level = k;
          J.rp = P.lh[k].rp;
          J.ntiles = (int)((nt * nrhs + 63) / 64);
          J.tile_start = tilec - L.first_tile;
          J.item_start = item - L.first_item;
          tilec += J.ntiles;
          item += J.ntiles * kM2l2Parts;
          mj.push_back(J);
        }
      }
      L.njobs = (int)mj.size() - L.first_job;
      L.nitems = item - L.first_item;
      L.ntiles = tilec - L.first_tile;
      if (L.njobs) ml.push_back(L);
    }
    P.m2l_flops = m2l_flops_of(P, nrhs);
  }
  // g = U g' on compressed levels
  {
    int tiles = 0;
    jt.post_first = (int)h.size();
    jt.post_rbt = pick_rbt(P.lh[depth].dpB / 16);
    for (int k = depth; k >= 2; --k) {
      if (P.lh[k].r == 0 || P.nact[k] == 0) continue;
      GemmJob J{};
      J.A = P.ld[k].ufrag;
      J.Bsrc = P.ld[k].gp;
      J.C = P.ld[k].g;
      J.ntgt = (int)P.nact[k];
      J.nterms = 1;
      J.dpm = P.lh[k].dpB;
      J.dpk = P.lh[k].rp;
      J.level = k;
      J.mode = MODE_PROJ;
      J.nrhs = nrhs;
      finish_job(J, tiles, jt.post_rbt);
      h.push_back(J);
    }
    jt.post_n = (int)h.size() - jt.post_first;
    jt.post_tiles = tiles;
    jt.post_units = finish_units(h, jt.post_first);
  }
  // L2L, per child level k = 3 .. depth, one job per child class
  for (int k = 3; k <= depth; ++k) {
    int tiles = 0;
    jt.l2l_first[k] = (int)h.size();
    for (int c = 0; c < 8; ++c) {
      const int64_t nt = P.cls_off[k][c + 1] - P.cls_off[k][c];
      if (nt == 0) continue;
      GemmJob J{};
      J.A = P.ld[k - 1].l2l;
      J.Bsrc = P.ld[k - 1].l;
      J.C = P.ld[k].l;
      J.Cadd = P.ld[k].g;
      J.tgt = P.ld[k].cls + P.cls_off[k][c];
      J.tgt_keys = P.ld[k].act;
      J.src_slot = P.ld[k - 1].slot;
      J.a_stride = (int64_t)P.lh[k].dpB * P.lh[k - 1].dpB;
      J.ntgt = (int)nt;
      J.nterms = 1;
      J.dpm = P.lh[k].dpB;
      J.dpk = P.lh[k - 1].dpB;
      J.level = k;
      J.cls = c;
      J.mode = MODE_L2L;
      J.nrhs = nrhs;
      jt.l2l_rbt[k] = pick_rbt(J.dpm / 16);
      finish_job(J, tiles, jt.l2l_rbt[k]);
      h.push_back(J);
    }
    jt.l2l_n[k] = (int)h.size() - jt.l2l_first[k];
    jt.l2l_tiles[k] = tiles;
    jt.l2l_units[k] = finish_units(h, jt.l2l_first[k]);
  }
  P.jobs_host = h;
  if (!h.empty()) {
    // the table goes to the device from pinned memory, asynchronously on the
    // stream of the evaluation; buffers grow only when the job count does
    if (h.size() > P.job_cap) {
      if (P.job_evt) hipEventSynchronize(P.job_evt);
      if (P.job_dev) hipFree(P.job_dev);
      if (P.job_pin) hipHostFree(P.job_pin);
      P.job_dev = nullptr;
      P.job_pin = nullptr;
      P.job_cap = 0;
      const size_t cap = h.size() + h.size() / 2 + 16;
      if (hipMalloc(&P.job_dev, sizeof(GemmJob) * cap) != hipSuccess ||
          hipHostMalloc((void **)&P.job_pin, sizeof(GemmJob) * cap) != hipSuccess) {
        hipGetLastError();
        return EIFMM_ENOMEM;
      }
      P.job_cap = cap;
      if (!P.job_evt && hipEventCreateWithFlags(&P.job_evt, hipEventDisableTiming) != hipSuccess)
        return EIFMM_EHIP;
    }
    if (hipEventSynchronize(P.job_evt) != hipSuccess) return EIFMM_EHIP;
    std::memcpy(P.job_pin, h.data(), sizeof(GemmJob) * h.size());
    if (hipMemcpyAsync(P.job_dev, P.job_pin, sizeof(GemmJob) * h.size(), hipMemcpyHostToDevice,
                       s) != hipSuccess ||
        hipEventRecord(P.job_evt, s) != hipSuccess)
      return EIFMM_EHIP;
  }
  if (!P.m2l2_host.empty()) {
    // factored M2L jobs: the same pinned, asynchronous upload; the workspace
    // holds one rp x 64 block per work item, launch after launch
    const size_t nj = P.m2l2_host.size();
    size_t need = 0;
    for (auto &L : P.m2l2_launch) {
      L.ws_off = need;
      need += (size_t)L.nitems * 16 * L.rb * 64;
    }
    if (P.job_evt) hipEventSynchronize(P.job_evt);
    if (nj > P.m2l2_cap) {
      if (P.m2l2_dev) hipFree(P.m2l2_dev);
      if (P.m2l2_pin) hipHostFree(P.m2l2_pin);
      P.m2l2_dev = nullptr;
      P.m2l2_pin = nullptr;
      P.m2l2_cap = 0;
      const size_t cap = nj + nj / 2 + 8;
      if (hipMalloc(&P.m2l2_dev, sizeof(M2l2Job) * cap) != hipSuccess ||
          hipHostMalloc((void **)&P.m2l2_pin, sizeof(M2l2Job) * cap) != hipSuccess) {
        hipGetLastError();
        return EIFMM_ENOMEM;
      }
      P.m2l2_cap = cap;
    }
    if (need > P.m2l2_ws_cap) {
      if (P.m2l2_ws) hipFree(P.m2l2_ws);
      P.m2l2_ws = nullptr;
      P.m2l2_ws_cap = 0;
      if (hipMalloc(&P.m2l2_ws, sizeof(double) * need) != hipSuccess) {
        hipGetLastError();
        return EIFMM_ENOMEM;
      }
      P.m2l2_ws_cap = need;
    }
    if (!P.job_evt && hipEventCreateWithFlags(&P.job_evt, hipEventDisableTiming) != hipSuccess)
      return EIFMM_EHIP;
    std::memcpy(P.m2l2_pin, P.m2l2_host.data(), sizeof(M2l2Job) * nj);
    if (hipMemcpyAsync(P.m2l2_dev, P.m2l2_pin, sizeof(M2l2Job) * nj, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipEventRecord(P.job_evt, s) != hipSuccess)
      return EIFMM_EHIP;
  }
  jt.nrhs = nrhs;
  return EIFMM_OK;
}

namespace {

// ws holds ws_len doubles: the pieces of the Stream-K tail, TILE doubles each, 2
// per tail workgroup, so the tail is split over at most ws_len / (2 TILE)
// workgroups (G itself for the plan's own workspace, fewer for a smaller one)
template <typename T, int MODE, int RBT>
void launch_gemm_rbt(const GemmJob *jobs, int n, int tiles, int64_t units, int gmax,
                     double *ws, size_t ws_len, const int8_t *dvec, hipStream_t s) {
  const size_t TILE = (size_t)RBT * 16 * gemm_cols(RBT);
  int *ctr = (int *)(ws + ws_len - kCounterDoubles);
  const size_t len = ws_len - kCounterDoubles;  // pieces
  const int G = (int)std::min<int64_t>(units, gmax);
  const int GT = (int)std::min<size_t>((size_t)G, len / (2 * TILE));
  const int rest = tiles - (tiles / G) * G;
  // the counter's split of the remaining tiles (M2L, when its pieces fit)
  int dyn = 0;
  int parts = 0;
  if (MODE == MODE_M2L && G > 1 && rest > 0) {
    // (an M2L job has 189 terms, more than kMaxTailParts)
    parts = (int)std::min<size_t>(kMaxTailParts, len / ((size_t)rest * TILE));
    if (parts >= 2) dyn = rest * parts;
  }
  constexpr bool fold = sizeof(T) == 4;
  hipLaunchKernelGGL((k_gemm<T, MODE, fold, RBT>), dim3(G), dim3(256), 0, s, jobs, n, tiles,
                     units, G, GT, ws, dvec, dyn, parts, ctr);
  if (G > 1 && rest > 0)
    hipLaunchKernelGGL((k_gemm_fixup<RBT>), dim3(rest * kFixupSplit), dim3(256), 0, s, jobs, n,
                       tiles, units, G, GT, ws, dyn, parts, ctr);
}

template <typename T, int MODE>
void launch_gemm_tab(const GemmJob *jobs, int n, int tiles, int64_t units, int rbt, int gmax,
                     double *ws, size_t ws_len, const int8_t *dvec, hipStream_t s) {
  if (n == 0 || tiles == 0 || units == 0) return;
  switch (rbt) {
    case 4: launch_gemm_rbt<T, MODE, 4>(jobs, n, tiles, units, gmax, ws, ws_len, dvec, s); break;
    case 3: launch_gemm_rbt<T, MODE, 3>(jobs, n, tiles, units, gmax, ws, ws_len, dvec, s); break;
    case 5: launch_gemm_rbt<T, MODE, 5>(jobs, n, tiles, units, gmax, ws, ws_len, dvec, s); break;

    default: launch_gemm_rbt<T, MODE, 6>(jobs, n, tiles, units, gmax, ws, ws_len, dvec, s); break;
  }
}

// a plan's launch: its Stream-K workspace, or the one its caller lends for this
// pass (P.run_ws, P.run_ws_len)
template <typename T, int MODE>
void launch_gemm(Plan &P, int first, int n, int tiles, int64_t units, hipStream_t s,
                 int rbt = 6) {
  double *ws = P.run_ws ? P.run_ws : P.sk_ws;
  const size_t len = P.run_ws ? P.run_ws_len : stream_k_ws_len(P.sk_groups);
  launch_gemm_tab<T, MODE>(P.job_dev + first, n, tiles, units, rbt, P.sk_groups, ws, len, P.dvec,
                           s);
}

void launch_gemm_fused(const FusedGemm &F, int mode, bool fp32, int gmax, double *ws,
                       const int8_t *dvec, hipStream_t s) {
  const size_t len = stream_k_ws_len(gmax);
  switch (mode) {
    case MODE_M2M:
      launch_gemm_tab<double, MODE_M2M>(F.dev, F.n, F.tiles, F.units, F.rbt, gmax, ws, len, dvec,
                                        s);
      break;
    case MODE_L2L:
      launch_gemm_tab<double, MODE_L2L>(F.dev, F.n, F.tiles, F.units, F.rbt, gmax, ws, len, dvec,
                                        s);
      break;
    case MODE_PROJ:
      launch_gemm_tab<double, MODE_PROJ>(F.dev, F.n, F.tiles, F.units, F.rbt, gmax, ws, len, dvec,
                                         s);
      break;
    default:
      if (fp32)
        launch_gemm_tab<float, MODE_M2L>(F.dev, F.n, F.tiles, F.units, F.rbt, gmax, ws, len, dvec,
                                         s);
      else
        launch_gemm_tab<double, MODE_M2L>(F.dev, F.n, F.tiles, F.units, F.rbt, gmax, ws, len, dvec,
                                          s);
  }
}

// ---- leaf-level launches (one plan: BATCH = false; a batch group: BATCH = true)
// workgroups of a chunk launch: one per 32-target chunk
unsigned chunk_grid(int64_t nchunk) { return (unsigned)nchunk; }

template <int KIND, bool BATCH>
void launch_p2p(bool mixed, int nrhs, int64_t nchunk, const LeafDesc &one, const LeafDesc *many,
                int nmany, hipStream_t s) {
  const unsigned grid = chunk_grid(nchunk);
  if (grid == 0) return;
  if (mixed) {
    if (nrhs == 1)
      hipLaunchKernelGGL((k_p2p32<KIND, 1, BATCH>), dim3(grid), dim3(64), 0, s, one, many, nmany);
    else
      hipLaunchKernelGGL((k_p2p32<KIND, 8, BATCH>), dim3(grid), dim3(64), 0, s, one, many, nmany);
  } else {
    if (nrhs == 1)
      hipLaunchKernelGGL((k_p2p64<KIND, 1, BATCH>), dim3(grid), dim3(64), 0, s, one, many, nmany);
    else
      hipLaunchKernelGGL((k_p2p64<KIND, 8, BATCH>), dim3(grid), dim3(64), 0, s, one, many, nmany);
  }
}

// crowded: the leaves hold more than 64 points on average, so that a workgroup
// spends its time in the batch loop (1e6 clustered points at depth 5: P2M 2.95
// -> 2.66 ms); on leaves of a few dozen points the 256-thread form is faster
// (1e6 uniform points at depth 5: 0.21 against 0.25 ms)
template <int KIND, bool BATCH>
void launch_p2m(int nrhs, unsigned grid, int dpmax, const LeafDesc &one, const LeafDesc *many,
                int nmany, hipStream_t s, bool crowded = false) {
  if (grid == 0) return;
  if (dpmax <= 64) {  // one row per thread: a 64-lane workgroup wastes no lanes on small d
    if (nrhs == 1)
      hipLaunchKernelGGL((k_p2m<KIND, 1, BATCH, 64>), dim3(grid), dim3(64), 0, s, one, many,
                         nmany);
    else
      hipLaunchKernelGGL((k_p2m<KIND, 8, BATCH, 64>), dim3(grid), dim3(64), 0, s, one, many,
                         nmany);
  } else {
    if (nrhs == 1 && crowded) {
      const int nt = std::min(1024, (dpmax + 63) / 64 * 64);
      hipLaunchKernelGGL((k_p2m<KIND, 1, BATCH, 0>), dim3(grid), dim3(nt), 0, s, one, many,
                         nmany);
    } else if (nrhs == 1) {
      hipLaunchKernelGGL((k_p2m<KIND, 1, BATCH, 256>), dim3(grid), dim3(256), 0, s, one, many,
                         nmany);
    } else {
      hipLaunchKernelGGL((k_p2m<KIND, 8, BATCH, 256>), dim3(grid), dim3(256), 0, s, one, many,
                         nmany);
    }
  }
}

size_t l2p_shm(int nrhs, int dpmax) {
  const int rb = nrhs == 1 ? 1 : 8;
  return sizeof(double) * (3 * (size_t)dpmax + (size_t)rb * dpmax);
}

template <int KIND, bool BATCH>
void launch_l2p(int nrhs, int64_t nchunk, int dpmax, const LeafDesc &one, const IoDesc &ione,
                const LeafDesc *many, const IoDesc *io, int nmany, hipStream_t s) {
  const unsigned grid = chunk_grid(nchunk);
  if (grid == 0) return;
  const size_t shm = l2p_shm(nrhs, dpmax);
  if (nrhs == 1)
    hipLaunchKernelGGL((k_l2p<KIND, 1, BATCH>), dim3(grid), dim3(64), shm, s, one, ione, many, io,
                       nmany);
  else
    hipLaunchKernelGGL((k_l2p<KIND, 8, BATCH>), dim3(grid), dim3(64), shm, s, one, ione, many, io,
                       nmany);
}

LeafDesc leaf_desc(const Plan &P, int nrhs) {
  const int depth = P.depth;
  LeafDesc D{};
  D.act = P.ld[depth].act;
  D.ls = P.leaf_start;
  // targets = sources: every point of a leaf is both; otherwise each leaf holds
  // its sources, then its targets
  D.se = P.nt ? P.tgt_begin : P.leaf_start + 1;
  D.tb = P.nt ? P.tgt_begin : P.leaf_start;
  D.chunk_ptr = P.chunk_ptr;
  D.near_ptr = P.near_ptr;
  D.near_src = P.near_src;
  D.perm = P.idx;
  D.xyz = P.xyz;
  D.X = P.ld[depth].X;
  D.XL = P.ld[depth].XL;
  D.lhat = P.lhat;
  D.sig = P.sig;
  D.fnear = P.fnear;
  D.W = P.ld[depth].W;
  D.n = P.n;
  D.nsrc = P.nt ? P.ns : P.n;
  D.toff = P.nt ? P.ns : 0;
  D.nleaf = (int)P.nact[depth];
  D.nrhs = nrhs;
  D.d = depth >= 2 ? P.lh[depth].d : 0;
  D.dp = depth >= 2 ? P.lh[depth].dp : 0;
  D.dL = depth >= 2 ? P.lh[depth].dB : 0;
  D.dpL = depth >= 2 ? P.lh[depth].dpB : 0;
  D.lo0 = P.cfg.lo[0];
  D.lo1 = P.cfg.lo[1];
  D.lo2 = P.cfg.lo[2];
  D.h = std::ldexp(P.cfg.L, -depth);
  D.p = dev_param(P.cfg.kernel, P.cfg.kernel_param);
  return D;
}

template <int KIND>
void run_kind(Plan &P, int nrhs, const IoDesc &io, hipStream_t s) {
  const int depth = P.depth;
  const bool mixed = P.cfg.precision == EIFMM_PREC_MIXED;
  const int64_t n = P.n;
  const int nleafa = (int)P.nact[depth];
  const int64_t nchunk = P.nchunk;
  const LeafDesc LD = leaf_desc(P, nrhs);
  LevelDev &LL = P.ld[depth];
  // near field: with a far field to compute it runs on the plan's second stream
  // and L2P waits for it. In FP64 it starts after P2M, so that it overlaps M2M,
  // the solves and the projections (small MFMA launches that leave the vector
  // units idle); the FP64 M2L holds 230 VGPRs per lane at two waves per SIMD,
  // which leaves no room for the near-field waves beside it. In mixed precision
  // it starts just before M2L: the FP32 M2L and FP32 near-field waves fit on a
  // SIMD together, and the near field then fills the M2L's ramp-down as well.
  // With many right-hand sides the near field is long enough to take CUs from
  // the M2L's persistent workgroups when it is dispatched first (the order of
  // the two streams' first dispatches is not fixed), so it starts after P2M.
  const bool fork = depth >= 2 && nleafa > 0 && P.side;
  const bool fork_late = fork && mixed && nrhs == 1;
  P.near_mode = fork_late ? 2 : fork ? 1 : 0;
  auto near_field = [&](hipStream_t sn) {
    if (sn != s) {
      hipEventRecord(P.ev_fork, s);
      hipStreamWaitEvent(sn, P.ev_fork, 0);
    }
    {
      Timer tm(P, sn, EIFMM_PH_P2P);
      launch_p2p<KIND, false>(mixed, nrhs, nchunk, LD, nullptr, 0, sn);
    }
    if (sn != s) hipEventRecord(P.ev_join, sn);
  };
  if (nleafa > 0 && !fork) near_field(s);
  if (depth < 2) {
    const int64_t m = n * nrhs;
    if (m > 0)
      hipLaunchKernelGGL(k_combine_near, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, n,
                         nrhs, P.fnear, P.idx, LD.toff, io.f, io.ldf);
    return;
  }
  const LevelHost &HL = P.lh[depth];
  // step 1: P2M
  if (nleafa > 0) {
    Timer tm(P, s, EIFMM_PH_P2M);
    launch_p2m<KIND, false>(nrhs, (unsigned)nleafa, HL.dp, LD, nullptr, 0, s,
                            n > 64 * (int64_t)nleafa);
  }
  if (fork && !fork_late) near_field(P.side);
  // step 2: M2M
  {
    Timer tm(P, s, EIFMM_PH_M2M);
    for (int k = depth - 1; k >= 2; --k)
      launch_gemm<double, MODE_M2M>(P, P.jobs.m2m_first[k], P.jobs.m2m_n[k], P.jobs.m2m_tiles[k],
                                    P.jobs.m2m_units[k], s, P.jobs.m2m_rbt[k]);
  }
  // step 3: What = Delta W = B^{-T} Gamma^{-1} W on uncompressed levels; on
  // compressed ones z = Gamma^{-1} W (the projection applies U^T B^{-T}), or
  // nothing where the projection's operator holds Gamma^{-1} too (fold_what)
  {
    Timer tm(P, s, EIFMM_PH_WHAT);
    SolveArgs A{};
    int blk = 0, q = 0;
    size_t shm = 0;
    for (int k = 2; k <= depth; ++k) {
      const int nc = (int)(P.nact[k] * nrhs);
      if (nc == 0 || !what_level(P, k)) continue;
      SolveDesc &D = A.lv[q++];
      D.in = P.ld[k].W;
      D.out = P.ld[k].Wh;
      D.out32 = (mixed && P.lh[k].r == 0) ? P.ld[k].Wh32 : nullptr;
      D.Tf = P.ld[k].tri[0];
      D.Tb = solves_what(P, k) ? P.ld[k].tri[1] : nullptr;
      D.ncols = nc;
      D.dp = P.lh[k].dp;
      D.blk_start = blk;
      blk += (nc + 15) / 16;
      shm = std::max(shm, trsm_shm(P.lh[k].dp));
    }
    A.nlev = q;
    if (blk > 0) hipLaunchKernelGGL(k_trsm, dim3(blk), dim3(64), shm, s, A);
  }
  // step 4: M2L (with the compression projections around it when enabled)
  if (P.jobs.pre_n) {
    Timer tm(P, s, EIFMM_PH_PROJ);
    launch_gemm<double, MODE_PROJ>(P, P.jobs.pre_first, P.jobs.pre_n, P.jobs.pre_tiles,
                                   P.jobs.pre_units, s, P.jobs.pre_rbt);
  }
  if (fork_late) hipEventRecord(P.ev_fork, s);
  {
    Timer tm(P, s, EIFMM_PH_M2L);
    if (mixed)
      launch_gemm<float, MODE_M2L>(P, P.jobs.m2l_first, P.jobs.m2l_n, P.jobs.m2l_tiles,
                                   P.jobs.m2l_units, s, P.jobs.m2l_rbt);
    else
      launch_gemm<double, MODE_M2L>(P, P.jobs.m2l_first, P.jobs.m2l_n, P.jobs.m2l_tiles,
                                    P.jobs.m2l_units, s, P.jobs.m2l_rbt);
    for (const M2l2Launch &L : P.m2l2_launch) launch_m2l2(P.m2l2_dev, L, P.dvec, P.m2l2_ws, s);
  }
  // launched after the M2L so that the M2L's workgroups are dispatched first
  if (fork_late) {
    hipStreamWaitEvent(P.side, P.ev_fork, 0);
    {
      Timer tm(P, P.side, EIFMM_PH_P2P);
      launch_p2p<KIND, false>(mixed, nrhs, nchunk, LD, nullptr, 0, P.side);
    }
    hipEventRecord(P.ev_join, P.side);
  }
  if (P.jobs.post_n) {
    Timer tm(P, s, EIFMM_PH_PROJ);
    launch_gemm<double, MODE_PROJ>(P, P.jobs.post_first, P.jobs.post_n, P.jobs.post_tiles,
                                   P.jobs.post_units, s, P.jobs.post_rbt);
  }
  // step 5: l^2 = g^2, then L2L downwards
  {
    Timer tm(P, s, EIFMM_PH_L2L);
    for (int k = 3; k <= depth; ++k)
      launch_gemm<double, MODE_L2L>(P, P.jobs.l2l_first[k], P.jobs.l2l_n[k], P.jobs.l2l_tiles[k],
                                    P.jobs.l2l_units[k], s, P.jobs.l2l_rbt[k]);
  }
  // step 6: lhat = Delta^{J_0,I_0} l on the leaf level (Delta^T l with one EIM)
  {
    Timer tm(P, s, EIFMM_PH_LHAT);
    SolveArgs A{};
    const int nc = nleafa * nrhs;
    A.lv[0].in = LL.l;
    A.lv[0].out = P.lhat;
    A.lv[0].out32 = nullptr;
    A.lv[0].Tf = P.fold_leaf ? nullptr : LL.tri[2];  // B^{-1} folded into l (the Gamma^T solve only)
    A.lv[0].Tb = LL.tri[3];
    A.lv[0].ncols = nc;
    A.lv[0].dp = HL.dpB;
    A.lv[0].blk_start = 0;
    A.nlev = 1;
    if (nc > 0)
      hipLaunchKernelGGL(k_trsm, dim3((nc + 15) / 16), dim3(64), trsm_shm(HL.dpB), s, A);
  }
  // step 7: L2P and the final sum (after the near field)
  if (fork) hipStreamWaitEvent(s, P.ev_join, 0);
  if (nleafa > 0) {
    Timer tm(P, s, EIFMM_PH_L2P);
    launch_l2p<KIND, false>(nrhs, nchunk, HL.dpB, LD, io, nullptr, nullptr, 0, s);
  }
}

}  // namespace

void timing_drain(Plan &P) {
  for (auto &e : P.ev_pending) {
    hipEventSynchronize(e.b);
    float ms = 0;
    hipEventElapsedTime(&ms, e.a, e.b);
    P.phase_ms[e.phase] += ms;
    P.phase_calls[e.phase] += 1;
    P.ev_free.push_back(e);
  }
  P.ev_pending.clear();
}

int pass_run(Plan &P, const double *sigma, int nrhs, int64_t ld, double *f, int64_t ldf,
             hipStream_t s) {
  if (P.jobs.nrhs != nrhs) {
    int st = build_jobs(P, nrhs, s);
    if (st != EIFMM_OK) return st;
  }
  const int64_t m = P.n * nrhs;
  const IoDesc io{sigma, ld, f, ldf};
  if (m > 0)
    hipLaunchKernelGGL((k_gather_sigma<false>), dim3((unsigned)((m + 255) / 256)), dim3(256), 0,
                       s, leaf_desc(P, nrhs), io, nullptr, nullptr, 0, m);
  switch (P.cfg.kernel) {
    case EIFMM_K_LAPLACE:
      run_kind<EIFMM_K_LAPLACE>(P, nrhs, io, s);
      break;
    case EIFMM_K_YUKAWA:
      run_kind<EIFMM_K_YUKAWA>(P, nrhs, io, s);
      break;
    case EIFMM_K_GAUSS:
      run_kind<EIFMM_K_GAUSS>(P, nrhs, io, s);
      break;
    case EIFMM_K_COSR:
      run_kind<EIFMM_K_COSR>(P, nrhs, io, s);
      break;
    case EIFMM_K_MQ:
      run_kind<EIFMM_K_MQ>(P, nrhs, io, s);
      break;
    case EIFMM_K_ADVDIFF:
      run_kind<EIFMM_K_ADVDIFF>(P, nrhs, io, s);
      break;
    default:
      run_kind<EIFMM_K_SQDIST>(P, nrhs, io, s);
      break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    P.last_hip_error = (int)e;
    return EIFMM_EHIP;
  }
  P.last_rhs = nrhs;
  return EIFMM_OK;
}

// 2 (rows x columns) per interaction pair on dense and stage-1 levels (the
// compressed sizes where compressed); 2 (r s + s r) with the factored M2L, s the
// mean second-stage rank over the 316 offsets standing in for the offsets the
// pairs actually use
double m2l_flops_of(const Plan &P, int nrhs) {
  double f = 0;
  for (int k = 2; k <= P.depth; ++k) {
    const LevelHost &L = P.lh[k];
    const double pairs = (double)P.il_pairs[k] * nrhs;
    if (uses_m2l2(P, k)) {
      double smean = 0;
      for (int o = 0; o < kNumOffsets; ++o) smean += L.s2[o];
      smean /= kNumOffsets;
      f += 4.0 * L.r * smean * pairs;
    } else {
      const bool cz = L.r > 0;
      const double rm = cz ? L.r : L.dB, rk = cz ? L.r : L.d;
      f += 2.0 * rm * rk * pairs;
    }
  }
  return f;
}

int materialize_expansion(Plan &P, int which, int k) {
  const int nrhs = P.jobs.nrhs;
  if (nrhs < 1 || k < 2 || k > P.depth || P.nact[k] == 0) return EIFMM_OK;
  hipStream_t s = nullptr;
  if (which == 1 && !solves_what(P, k)) {
    // What = Delta W, as the pass computes it on uncompressed levels
    SolveArgs A{};
    SolveDesc &D = A.lv[0];
    D.in = P.ld[k].W;
    D.out = P.ld[k].Wh;
    D.out32 = nullptr;
    D.Tf = P.ld[k].tri[0];
    D.Tb = P.ld[k].tri[1];
    D.ncols = (int)(P.nact[k] * nrhs);
    D.dp = P.lh[k].dp;
    D.blk_start = 0;
    A.nlev = 1;
    hipLaunchKernelGGL(k_trsm, dim3((D.ncols + 15) / 16), dim3(64), trsm_shm(D.dp), s, A);
  } else {
    return EIFMM_OK;
  }
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    P.last_hip_error = (int)e;
    return EIFMM_EHIP;
  }
  return EIFMM_OK;
}

// M2M and L2L operators of parent level k (Sec. 4.1) by the blocked MFMA solves of
// the pass, one launch for both: the M2M rows K(X^k - s_i, Y^{k+1}) times
// M^{-1} of the child, i.e. M^{-T} applied to each row (B forward, Gamma^T
// backward); the L2L rows times the parent's Delta^T (one EIM: M^{-1} applied to
// each row, Gamma forward, B^T backward) or M_B^{-1} (two EIMs: M_B^{-T} applied,
// B_B forward, Gamma_B^T backward).  Rows are padded to the solve's dp with
// zeros, which the identity-padded tables keep at zero.
int solve_operators_gpu(Plan &P, int k) {
  LevelHost &lp = P.lh[k], &lc = P.lh[k + 1];
  const int n0 = 8 * lp.d, n1 = 8 * lc.dB;
  const int dp0 = lc.dp, dp1 = lp.dpB;
  const size_t sz0 = (size_t)n0 * dp0, sz1 = (size_t)n1 * dp1;
  if (lp.m2m_rows.size() != sz0 || lp.l2l_rows.size() != sz1) return EIFMM_EINVAL;
  double *rows = nullptr, *tabs[4] = {nullptr, nullptr, nullptr, nullptr};
  hipError_t e = hipMalloc(&rows, sizeof(double) * (sz0 + sz1 > 0 ? sz0 + sz1 : 1));
  if (e == hipSuccess && sz0) e = hipMemcpy(rows, lp.m2m_rows.data(), sizeof(double) * sz0, hipMemcpyHostToDevice);
  if (e == hipSuccess && sz1)
    e = hipMemcpy(rows + sz0, lp.l2l_rows.data(), sizeof(double) * sz1, hipMemcpyHostToDevice);
  const double *T[4];
  if (P.two_eim) {
    for (int q = 0; q < 4 && e == hipSuccess; ++q) {
      e = hipMalloc(&tabs[q], sizeof(double) * std::max<size_t>(lp.op_tri[q].size(), 1));
      if (e == hipSuccess && !lp.op_tri[q].empty())
        e = hipMemcpy(tabs[q], lp.op_tri[q].data(), sizeof(double) * lp.op_tri[q].size(),
                      hipMemcpyHostToDevice);
      T[q] = tabs[q];
    }
  } else {
    T[0] = P.ld[k + 1].tri[2];  // the child's Delta^T tables: B, Gamma^T
    T[1] = P.ld[k + 1].tri[3];
    T[2] = P.ld[k].tri[0];      // the parent's Delta tables: Gamma, B^T
    T[3] = P.ld[k].tri[1];
  }
  if (e == hipSuccess) {
    SolveArgs A{};
    A.lv[0] = SolveDesc{rows, rows, nullptr, T[0], T[1], n0, dp0, 0, 0};
    A.lv[1] = SolveDesc{rows + sz0, rows + sz0, nullptr, T[2], T[3], n1, dp1, (n0 + 15) / 16, 0};
    A.nlev = 2;
    const int blk = (n0 + 15) / 16 + (n1 + 15) / 16;
    // in place: a wave reads all tiles of its columns (forward pass) before it
    // writes any (backward pass)
    if (blk > 0) {
      hipLaunchKernelGGL(k_trsm, dim3(blk), dim3(64), trsm_shm(std::max(dp0, dp1)), nullptr, A);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess && sz0)
    e = hipMemcpy(lp.m2m_rows.data(), rows, sizeof(double) * sz0, hipMemcpyDeviceToHost);
  if (e == hipSuccess && sz1)
    e = hipMemcpy(lp.l2l_rows.data(), rows + sz0, sizeof(double) * sz1, hipMemcpyDeviceToHost);
  hipFree(rows);
  for (double *t : tabs) hipFree(t);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? EIFMM_ENOMEM : EIFMM_EHIP;
  }
  return EIFMM_OK;
}

// ------------------------------------------------------------------ batches
// A batch runs the pass of many independent problems (one plan each) as a fixed,
// short sequence of launches, each covering every problem: the leaf-level
// kernels once per kernel kind with an array of LeafDesc, the triangular solves
// once per step with a list of SolveDesc, and each gathered-GEMM step once with
// the concatenated jobs of all plans (re-tiled for the fused launch).  The
// sequence contains no host synchronisation and no allocation, so it can be
// captured once into a HIP graph and replayed.

namespace {

template <typename T>
int bupload(T **p, const std::vector<T> &v, std::vector<void *> &track) {
  *p = nullptr;
  if (v.empty()) return EIFMM_OK;
  if (hipMalloc((void **)p, sizeof(T) * v.size()) != hipSuccess) {
    hipGetLastError();
    return EIFMM_ENOMEM;
  }
  track.push_back((void *)*p);
  if (hipMemcpy(*p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
    return EIFMM_EHIP;
  return EIFMM_OK;
}

// concatenate the job ranges [first, first + n) of every plan into one launch
int fuse_jobs(FusedGemm &F, const std::vector<Plan *> &plans,
              const std::vector<std::pair<int, int>> &ranges, int rbt,
              std::vector<void *> &track) {
  std::vector<GemmJob> h;
  int dmax = 16;
  for (size_t q = 0; q < plans.size(); ++q)
    for (int j = ranges[q].first; j < ranges[q].first + ranges[q].second; ++j) {
      const GemmJob &J = plans[q]->jobs_host[j];
      if (J.ntgt == 0) continue;
      h.push_back(J);
      dmax = std::max(dmax, J.dpm);
    }
  F = FusedGemm{};
  F.rbt = rbt > 0 ? rbt : pick_rbt(dmax / 16);
  int tiles = 0;
  for (auto &J : h) finish_job(J, tiles, F.rbt);
  F.units = finish_units(h, 0);
  F.tiles = tiles;
  F.n = (int)h.size();
  return bupload(&F.dev, h, track);
}

// Packed M2L: one job per (operator set, level, child class) whose columns are
// the targets of that class in every problem using the set, so the coarse
// levels of small problems (a few boxes per class each) fill whole tiles.
int pack_m2l(FusedGemm &F, const std::vector<Plan *> &plans, int rbt, bool mixed,
             std::vector<void *> &track) {
  struct Key {
    const void *A;
    int k, c;
  };
  std::vector<Key> keys;
  std::vector<GemmJob> jobs;
  std::vector<std::vector<ColRef>> refs;
  std::vector<ColSrc> srcs;
  std::vector<int> cls;
  int dmax = 16;
  for (Plan *Pp : plans) {
    const Plan &P = *Pp;
    for (int k = P.depth; k >= 2; --k) {
      const int64_t na = P.nact[k];
      if (na == 0) continue;
      cls.resize(na);
      if (hipMemcpy(cls.data(), P.ld[k].cls, sizeof(int) * na, hipMemcpyDeviceToHost) !=
          hipSuccess)
        return EIFMM_EHIP;
      const bool cz = P.lh[k].r > 0;
      const int dm = cz ? P.lh[k].rp : P.lh[k].dp;
      dmax = std::max(dmax, dm);
      const void *A = mixed ? (const void *)P.ld[k].kfrag32 : (const void *)P.ld[k].kfrag;
      ColSrc cs;
      cs.keys = P.ld[k].act;
      cs.slot = P.ld[k].slot;
      if (cz)
        cs.B = mixed ? (const void *)P.ld[k].Whp32 : (const void *)P.ld[k].Whp;
      else
        cs.B = mixed ? (const void *)P.ld[k].Wh32 : (const void *)P.ld[k].Wh;
      cs.C = cz ? P.ld[k].gp : P.ld[k].g;
      const int rec = (int)srcs.size();
      srcs.push_back(cs);
      for (int c = 0; c < 8; ++c) {
        const int64_t c0 = P.cls_off[k][c], c1 = P.cls_off[k][c + 1];
        if (c1 == c0) continue;
        size_t j = 0;
        while (j < keys.size() && !(keys[j].A == A && keys[j].k == k && keys[j].c == c)) ++j;
        if (j == keys.size()) {
          keys.push_back(Key{A, k, c});
          GemmJob J{};
          J.A = A;
          J.terms = P.dlist + 189 * c;
          J.a_stride = (int64_t)dm * dm;
          J.nterms = 189;
          J.dpm = J.dpk = dm;
          J.level = k;
          J.cls = c;
          J.mode = MODE_M2L;
          J.nrhs = 1;
          jobs.push_back(J);
          refs.emplace_back();
        }
        for (int64_t i = c0; i < c1; ++i) refs[j].push_back(ColRef{rec, cls[i]});
      }
    }
  }
  F = FusedGemm{};
  F.rbt = rbt > 0 ? rbt : pick_rbt(dmax / 16);
  if (jobs.empty()) return EIFMM_OK;
  // finest level first (as in a plan's own launch), then operator set and class
  std::vector<int> order(jobs.size());
  for (size_t j = 0; j < jobs.size(); ++j) order[j] = (int)j;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return jobs[a].level > jobs[b].level; });
  std::vector<ColRef> all;
  std::vector<GemmJob> h;
  std::vector<size_t> off;
  for (int j : order) {
    off.push_back(all.size());
    all.insert(all.end(), refs[j].begin(), refs[j].end());
    GemmJob J = jobs[j];
    J.ntgt = (int)refs[j].size();
    h.push_back(J);
  }
  ColSrc *srcs_dev = nullptr;
  ColRef *refs_dev = nullptr;
  int st = bupload(&srcs_dev, srcs, track);
  if (!st) st = bupload(&refs_dev, all, track);
  if (st) return st;
  int tiles = 0;
  for (size_t j = 0; j < h.size(); ++j) {
    h[j].colsrc = srcs_dev;
    h[j].colref = refs_dev + off[j];
    finish_job(h[j], tiles, F.rbt);
  }
  F.units = finish_units(h, 0);
  F.tiles = tiles;
  F.n = (int)h.size();
  return bupload(&F.dev, h, track);
}

template <int KIND>
void run_group(const BatchExec &B, const BatchGroup &g, int phase, hipStream_t s) {
  const LeafDesc *many = B.leaf_dev + g.first;
  const LeafDesc none{};
  const IoDesc inone{};
  if (phase == 0)
    launch_p2p<KIND, true>(B.mixed, 1, g.nchunk, none, many, g.count, s);
  else if (phase == 1)
    launch_p2m<KIND, true>(1, (unsigned)g.nleaf, g.dpmax, none, many, g.count, s);
  else
    launch_l2p<KIND, true>(1, g.nchunk, g.dpmax, none, inone, many, B.io_dev + g.first, g.count,
                           s);
}

void run_groups(const BatchExec &B, int phase, hipStream_t s, const hipEvent_t *mark,
                int &m) {
  for (const BatchGroup &g : B.groups) {
    switch (g.kind) {
      case EIFMM_K_LAPLACE: run_group<EIFMM_K_LAPLACE>(B, g, phase, s); break;
      case EIFMM_K_YUKAWA: run_group<EIFMM_K_YUKAWA>(B, g, phase, s); break;
      case EIFMM_K_GAUSS: run_group<EIFMM_K_GAUSS>(B, g, phase, s); break;
      case EIFMM_K_COSR: run_group<EIFMM_K_COSR>(B, g, phase, s); break;
      case EIFMM_K_MQ: run_group<EIFMM_K_MQ>(B, g, phase, s); break;
      default: run_group<EIFMM_K_SQDIST>(B, g, phase, s); break;
    }
    if (mark) hipEventRecord(mark[m++], s);
  }
}

}  // namespace

void batch_release(BatchExec &B) {
  if (!B.track.empty()) hipDeviceSynchronize();  // launches may still read the tables
  for (void *p : B.track) hipFree(p);
  B = BatchExec{};
}

int batch_prepare(BatchExec &B, const std::vector<Plan *> &plans_in, int m2l_rbt, int sk_groups,
                  double *sk_ws) {
  batch_release(B);
  const int np = (int)plans_in.size();
  if (np == 0) return EIFMM_EINVAL;
  B.nprob = np;
  B.mixed = plans_in[0]->cfg.precision == EIFMM_PREC_MIXED;
  for (Plan *P : plans_in) {
    if (!P->points_set || P->depth < 2) return EIFMM_ESTATE;
    if ((P->cfg.precision == EIFMM_PREC_MIXED) != B.mixed) return EIFMM_EINVAL;
    if (P->jobs.nrhs != 1) {
      int st = build_jobs(*P, 1, nullptr);
      if (st) return st;
    }
    B.maxdepth = std::max(B.maxdepth, P->depth);
  }
  // descriptor order: problems grouped by kernel kind, batch order inside a group
  std::vector<Plan *> plans;
  for (int kind = EIFMM_K_LAPLACE; kind <= EIFMM_K_MQ; ++kind) {
    BatchGroup g;
    g.kind = kind;
    g.first = (int)plans.size();
    for (int q = 0; q < np; ++q)
      if (plans_in[q]->cfg.kernel == kind) {
        B.order.push_back(q);
        plans.push_back(plans_in[q]);
      }
    g.count = (int)plans.size() - g.first;
    if (g.count) B.groups.push_back(g);
  }
  std::vector<LeafDesc> leaf(np);
  int64_t pts = 0;
  for (BatchGroup &g : B.groups) {
    int64_t ch = 0, lf = 0;
    for (int q = g.first; q < g.first + g.count; ++q) {
      const Plan &P = *plans[q];
      LeafDesc D = leaf_desc(P, 1);
      D.chunk_base = ch;
      D.leaf_base = lf;
      D.pt_base = pts;
      ch += P.nchunk;
      lf += P.nact[P.depth];
      pts += P.n;
      g.dpmax = std::max(g.dpmax, std::max(P.lh[P.depth].dp, P.lh[P.depth].dpB));
      leaf[q] = D;
    }
    g.nchunk = ch;
    g.nleaf = lf;
  }
  B.total_pts = pts;
  int st = bupload(&B.leaf_dev, leaf, B.track);
  if (st) return st;
  {
    std::vector<IoDesc> io(np, IoDesc{nullptr, 0, nullptr, 0});
    if ((st = bupload(&B.io_dev, io, B.track))) return st;
  }
  // triangular solves: What (z on compressed levels) on every level, lhat on the leaf level
  {
    std::vector<SolveDesc> w, l;
    int bw = 0, bl = 0;
    for (Plan *Pp : plans) {
      const Plan &P = *Pp;
      for (int k = 2; k <= P.depth; ++k) {
        const int nc = (int)P.nact[k];
        if (nc == 0) continue;
        SolveDesc D{};
        D.in = P.ld[k].W;
        D.out = P.ld[k].Wh;
        D.out32 = (B.mixed && P.lh[k].r == 0) ? P.ld[k].Wh32 : nullptr;
        D.Tf = P.ld[k].tri[0];
        D.Tb = solves_what(P, k) ? P.ld[k].tri[1] : nullptr;
        D.ncols = nc;
        D.dp = P.lh[k].dp;
        D.blk_start = bw;
        bw += (nc + 15) / 16;
        B.what_shm = std::max(B.what_shm, trsm_shm(D.dp));
        w.push_back(D);
      }
      const int k = P.depth, nc = (int)P.nact[k];
      if (nc == 0) continue;
      SolveDesc D{};
      D.in = P.ld[k].l;
      D.out = P.lhat;
      D.out32 = nullptr;
      D.Tf = P.ld[k].tri[2];
      D.Tb = P.ld[k].tri[3];
      D.ncols = nc;
      D.dp = P.lh[k].dpB;
      D.blk_start = bl;
      bl += (nc + 15) / 16;
      B.lhat_shm = std::max(B.lhat_shm, trsm_shm(D.dp));
      l.push_back(D);
    }
    B.what_n = (int)w.size();
    B.what_blk = bw;
    B.lhat_n = (int)l.size();
    B.lhat_blk = bl;
    if ((st = bupload(&B.what_dev, w, B.track))) return st;
    if ((st = bupload(&B.lhat_dev, l, B.track))) return st;
  }
  // gathered GEMMs
  const int nq = (int)plans.size();
  std::vector<std::pair<int, int>> r(nq);
  for (int k = B.maxdepth - 1; k >= 2; --k) {
    for (int q = 0; q < nq; ++q)
      r[q] = {plans[q]->jobs.m2m_first[k], k < plans[q]->depth ? plans[q]->jobs.m2m_n[k] : 0};
    if ((st = fuse_jobs(B.m2m[k], plans, r, 0, B.track))) return st;
  }
  for (int q = 0; q < nq; ++q) r[q] = {plans[q]->jobs.pre_first, plans[q]->jobs.pre_n};
  if ((st = fuse_jobs(B.pre, plans, r, 0, B.track))) return st;
  if ((st = pack_m2l(B.m2l, plans, m2l_rbt, B.mixed, B.track))) return st;
  for (int q = 0; q < nq; ++q) r[q] = {plans[q]->jobs.post_first, plans[q]->jobs.post_n};
  if ((st = fuse_jobs(B.post, plans, r, 0, B.track))) return st;
  for (int k = 3; k <= B.maxdepth; ++k) {
    for (int q = 0; q < nq; ++q)
      r[q] = {plans[q]->jobs.l2l_first[k], k <= plans[q]->depth ? plans[q]->jobs.l2l_n[k] : 0};
    if ((st = fuse_jobs(B.l2l[k], plans, r, 0, B.track))) return st;
  }
  B.m2l_flops = 0;
  for (Plan *P : plans) B.m2l_flops += P->m2l_flops;
  B.sk_groups = sk_groups;
  B.sk_ws = sk_ws;
  B.dvec = plans[0]->dvec;
  hipError_t e = hipDeviceSynchronize();
  return e == hipSuccess ? EIFMM_OK : EIFMM_EHIP;
}

void batch_run_m2l(const BatchExec &B, hipStream_t s) {
  launch_gemm_fused(B.m2l, MODE_M2L, B.mixed, B.sk_groups, B.sk_ws, B.dvec, s);
}

int batch_marks(const BatchExec &B) { return 9 + 3 * (int)B.groups.size(); }

void batch_run(const BatchExec &B, hipStream_t s, const hipEvent_t *mark) {
  int m = 0;
  auto tick = [&]() {
    if (mark) hipEventRecord(mark[m++], s);
  };
  tick();
  if (B.total_pts > 0)
    hipLaunchKernelGGL((k_gather_sigma<true>), dim3((unsigned)((B.total_pts + 255) / 256)),
                       dim3(256), 0, s, LeafDesc{}, IoDesc{}, B.leaf_dev, B.io_dev, B.nprob,
                       B.total_pts);
  tick();
  run_groups(B, 0, s, mark, m);  // near field, one mark per kernel kind
  run_groups(B, 1, s, mark, m);  // P2M
  for (int k = B.maxdepth - 1; k >= 2; --k)
    launch_gemm_fused(B.m2m[k], MODE_M2M, false, B.sk_groups, B.sk_ws, B.dvec, s);
  tick();
  if (B.what_blk > 0)
    hipLaunchKernelGGL(k_trsm_list, dim3(B.what_blk), dim3(64), B.what_shm, s, B.what_dev,
                       B.what_n);
  tick();
  launch_gemm_fused(B.pre, MODE_PROJ, false, B.sk_groups, B.sk_ws, B.dvec, s);
  tick();
  batch_run_m2l(B, s);
  tick();
  launch_gemm_fused(B.post, MODE_PROJ, false, B.sk_groups, B.sk_ws, B.dvec, s);
  tick();
  for (int k = 3; k <= B.maxdepth; ++k)
    launch_gemm_fused(B.l2l[k], MODE_L2L, false, B.sk_groups, B.sk_ws, B.dvec, s);
  tick();
  if (B.lhat_blk > 0)
    hipLaunchKernelGGL(k_trsm_list, dim3(B.lhat_blk), dim3(64), B.lhat_shm, s, B.lhat_dev,
                       B.lhat_n);
  tick();
  run_groups(B, 2, s, mark, m);  // L2P and the final sum
}

}  // namespace eifmm
