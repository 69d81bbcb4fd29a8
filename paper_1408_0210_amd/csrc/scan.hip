// scan.hip -- exclusive prefix sums (three launches: block scans, a scan of the
// block totals by one workgroup, and the final add).
#include "devutil.hpp"

namespace eifmm {

constexpr int kScanBlock = 1024;  // 256 threads x 4 entries

template <typename T>
__global__ __launch_bounds__(256) void k_scan_blocks(const T *__restrict__ in, T *__restrict__ out,
                                                     int64_t n, int *__restrict__ tot) {
  __shared__ T part[256];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * t;
  T v[4];
  T s = 0;
  for (int q = 0; q < 4; ++q) {
    v[q] = (base + q < n) ? in[base + q] : T(0);
    s += v[q];
  }
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    T u = t >= off ? part[t - off] : T(0);
    __syncthreads();
    part[t] += u;
    __syncthreads();
  }
  T run = part[t] - s;
  for (int q = 0; q < 4; ++q) {
    if (base + q < n) out[base + q] = run;
    run += v[q];
  }
  if (t == 255) tot[blockIdx.x] = (int)part[255];
}

// one workgroup: exclusive scan of the nb block totals, in chunks of 1024
__global__ __launch_bounds__(1024) void k_scan_tops(int *__restrict__ tot, int nb) {
  __shared__ int part[1024];
  __shared__ int carry;
  const int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nb; c0 += 1024) {
    int v = (c0 + t < nb) ? tot[c0 + t] : 0;
    part[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int u = t >= off ? part[t - off] : 0;
      __syncthreads();
      part[t] += u;
      __syncthreads();
    }
    if (c0 + t < nb) tot[c0 + t] = carry + part[t] - v;
    __syncthreads();
    if (t == 1023) carry += part[1023];
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_add(T *__restrict__ out, int64_t n,
                                                  const int *__restrict__ tot) {
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * threadIdx.x;
  const T add = (T)tot[blockIdx.x];
  for (int q = 0; q < 4; ++q)
    if (base + q < n) out[base + q] += add;
}

template <typename T>
static void scan_impl(const T *in, T *out, int64_t n, int *tmp, hipStream_t s) {
  if (n <= 0) return;
  const int nb = (int)((n + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_scan_blocks<T>, dim3(nb), dim3(256), 0, s, in, out, n, tmp);
  hipLaunchKernelGGL(k_scan_tops, dim3(1), dim3(1024), 0, s, tmp, nb);
  hipLaunchKernelGGL(k_scan_add<T>, dim3(nb), dim3(256), 0, s, out, n, tmp);
}

void scan_exclusive_i32(const int *in, int *out, int64_t n, int *tmp, hipStream_t s) {
  scan_impl<int>(in, out, n, tmp, s);
}

void scan_exclusive_u32(const unsigned *in, unsigned *out, int64_t n, int *tmp, hipStream_t s) {
  scan_impl<unsigned>(in, out, n, tmp, s);
}

}  // namespace eifmm
