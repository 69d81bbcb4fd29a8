// eim_gpu.hip -- the EIM greedy (Algorithm 1) on the GPU.
//
// Algorithm 1 in the L-infinity norm on a training matrix R (rows: points of
// D_x, columns: points of D_y) is cross approximation with complete pivoting:
// take the entry of largest magnitude (lowest row, then lowest column on ties),
// stop when it is <= tau * scale, else record it and subtract the rank-1 term
//   R[a][b] -= R[a][bs] * (R[as][b] / R[as][bs]).
// Each step reads and writes all of R once: the update is HBM-bound, and it
// also reduces the magnitudes of the values it writes, so the next pivot comes
// from the same pass.  Two buffers alternate so that every thread reads the
// pivot row and column as they were before the step.  Products and
// differences are separate correctly rounded operations (no contraction) and
// the quotient is a correctly rounded division, as in the host greedy, so both
// select the same points and leave the same residual, bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "plan.hpp"

namespace eifmm {
namespace {

constexpr int kEimThreads = 256;

struct EimPivot {
  double v;     // largest |R|
  int64_t idx;  // its linear index (row-major), lowest on ties
  double piv;   // R at idx (signed)
};

// (value, index) pair that wins: larger value, then lower index.  NaN never wins.
__device__ inline bool better(double v, int64_t i, double bv, int64_t bi) {
  return v > bv || (v == bv && i < bi);
}

__device__ inline void block_best(double v, int64_t i, double *sv, int64_t *si,
                                  double *ov, int64_t *oi) {
  const int t = threadIdx.x;
  sv[t] = v;
  si[t] = i;
  __syncthreads();
  for (int o = kEimThreads / 2; o > 0; o >>= 1) {
    if (t < o && better(sv[t + o], si[t + o], sv[t], si[t])) {
      sv[t] = sv[t + o];
      si[t] = si[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    *ov = sv[0];
    *oi = si[0];
  }
}

// per-block best |R| over a grid-stride range
__global__ __launch_bounds__(kEimThreads) void k_eim_amax(const double *__restrict__ R,
                                                          int64_t total, double *__restrict__ bv,
                                                          int64_t *__restrict__ bi) {
  __shared__ double sv[kEimThreads];
  __shared__ int64_t si[kEimThreads];
  double v = -1.0;
  int64_t i = INT64_MAX;
  for (int64_t e = (int64_t)blockIdx.x * kEimThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kEimThreads) {
    const double a = fabs(R[e]);
    if (better(a, e, v, i)) {
      v = a;
      i = e;
    }
  }
  block_best(v, i, sv, si, bv + blockIdx.x, bi + blockIdx.x);
}

// one block: best over the block results, and the pivot value
__global__ __launch_bounds__(kEimThreads) void k_eim_final(const double *__restrict__ bv,
                                                           const int64_t *__restrict__ bi, int nb,
                                                           const double *__restrict__ R,
                                                           EimPivot *__restrict__ out) {
  __shared__ double sv[kEimThreads];
  __shared__ int64_t si[kEimThreads];
  double v = -1.0;
  int64_t i = INT64_MAX;
  for (int b = threadIdx.x; b < nb; b += kEimThreads)
    if (better(bv[b], bi[b], v, i)) {
      v = bv[b];
      i = bi[b];
    }
  __shared__ double fv;
  __shared__ int64_t fi;
  block_best(v, i, sv, si, &fv, &fi);
  __syncthreads();
  if (threadIdx.x == 0) {
    out->v = fv;
    out->idx = fi;
    out->piv = fi != INT64_MAX ? R[fi] : 0.0;
  }
}

// Rout = Rin - Rin[:, bs] (Rin[as, :] / piv), and the per-block best |Rout|
__global__ __launch_bounds__(kEimThreads) void k_eim_update(const double *__restrict__ Rin,
                                                            double *__restrict__ Rout, int64_t ny,
                                                            int64_t total,
                                                            const EimPivot *__restrict__ pv,
                                                            double *__restrict__ bv,
                                                            int64_t *__restrict__ bi) {
#pragma clang fp contract(off)
  __shared__ double sv[kEimThreads];
  __shared__ int64_t si[kEimThreads];
  const int64_t as = pv->idx / ny, bs = pv->idx - (pv->idx / ny) * ny;
  const double piv = pv->piv;
  const double *prow = Rin + as * ny;
  double v = -1.0;
  int64_t i = INT64_MAX;
  for (int64_t e = (int64_t)blockIdx.x * kEimThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kEimThreads) {
    const int64_t a = e / ny, b = e - a * ny;
    const double q = prow[b] / piv;
    const double c = Rin[a * ny + bs];
    const double prod = c * q;
    const double r = Rin[e] - prod;
    Rout[e] = r;
    const double m = fabs(r);
    if (better(m, e, v, i)) {
      v = m;
      i = e;
    }
  }
  block_best(v, i, sv, si, bv + blockIdx.x, bi + blockIdx.x);
}

int hip_status(hipError_t e) {
  if (e == hipSuccess) return EIFMM_OK;
  (void)hipGetLastError();
  return e == hipErrorOutOfMemory ? EIFMM_ENOMEM : EIFMM_EHIP;
}

}  // namespace

int eim_iterate_gpu(const std::vector<double> &R, int64_t nx, int64_t ny, double tau,
                    double abs_scale, int dmax, EimResult &res) {
  res = EimResult{};
  const int64_t total = nx * ny;
  if (total == 0) return EIFMM_OK;
  double *buf[2] = {nullptr, nullptr};
  double *bv = nullptr;
  int64_t *bi = nullptr;
  EimPivot *pv = nullptr;
  int dev = 0, ncu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const int nb = (int)std::min<int64_t>(std::max(1, 4 * ncu), (total + kEimThreads - 1) / kEimThreads);
  int st = hip_status(hipMalloc(&buf[0], sizeof(double) * total));
  if (!st) st = hip_status(hipMalloc(&buf[1], sizeof(double) * total));
  if (!st) st = hip_status(hipMalloc(&bv, sizeof(double) * nb));
  if (!st) st = hip_status(hipMalloc(&bi, sizeof(int64_t) * nb));
  if (!st) st = hip_status(hipMalloc(&pv, sizeof(EimPivot)));
  if (!st) st = hip_status(hipMemcpy(buf[0], R.data(), sizeof(double) * total, hipMemcpyHostToDevice));
  if (!st) {
    hipLaunchKernelGGL(k_eim_amax, dim3(nb), dim3(kEimThreads), 0, nullptr, buf[0], total, bv, bi);
    hipLaunchKernelGGL(k_eim_final, dim3(1), dim3(kEimThreads), 0, nullptr, bv, bi, nb, buf[0], pv);
  }
  int cur = 0;
  while (!st) {
    EimPivot h{};
    st = hip_status(hipMemcpy(&h, pv, sizeof(h), hipMemcpyDeviceToHost));
    if (st) break;
    if (res.ia.empty()) res.scale = abs_scale > 0 ? abs_scale : h.v;
    res.emax = h.v;
    if (h.v <= tau * res.scale) break;
    if ((int)res.ia.size() == dmax) {
      res.status = EIFMM_EEIM;
      break;
    }
    res.ia.push_back(h.idx / ny);
    res.ib.push_back(h.idx - (h.idx / ny) * ny);
    hipLaunchKernelGGL(k_eim_update, dim3(nb), dim3(kEimThreads), 0, nullptr, buf[cur],
                       buf[cur ^ 1], ny, total, pv, bv, bi);
    hipLaunchKernelGGL(k_eim_final, dim3(1), dim3(kEimThreads), 0, nullptr, bv, bi, nb,
                       buf[cur ^ 1], pv);
    cur ^= 1;
    st = hip_status(hipGetLastError());
  }
  hipFree(buf[0]);
  hipFree(buf[1]);
  hipFree(bv);
  hipFree(bi);
  hipFree(pv);
  return st;
}

}  // namespace eifmm
