// devutil.hpp -- small device helpers shared by the library's kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace eifmm {

// Morton interleave of three 10-bit indices: bit b of v goes to bit 3b.
__host__ __device__ inline uint32_t spread3(uint32_t v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__host__ __device__ inline uint32_t compact3(uint32_t v) {
  v &= 0x09249249u;
  v = (v ^ (v >> 2)) & 0x030C30C3u;
  v = (v ^ (v >> 4)) & 0x0300F00Fu;
  v = (v ^ (v >> 8)) & 0xFF0000FFu;
  v = (v ^ (v >> 16)) & 0x000003FFu;
  return v;
}

__host__ __device__ inline uint32_t morton_encode(uint32_t x, uint32_t y, uint32_t z) {
  return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// Loads and stores through global-memory (address space 1) pointers.  A pointer
// the kernel reads from memory (a job table, a descriptor) is generic to the
// compiler, which then emits flat instructions; those count against the LDS wait
// counter as well, so waiting for an LDS read would also wait for every memory
// load in flight, the prefetches included.  T must be a scalar or an
// ext_vector_type (HIP's double2 class copies through a generic pointer).
#define EIFMM_GLOBAL_AS __attribute__((address_space(1)))
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
template <typename T>
__device__ inline T ldg(const T *p) {
  return *(const EIFMM_GLOBAL_AS T *)p;
}
template <typename T>
__device__ inline void stg(T *p, T v) {
  *(EIFMM_GLOBAL_AS T *)p = v;
}

// Workgroup barrier for hand-offs through LDS: a release/acquire on the LDS
// address space only, so the compiler waits for the LDS accesses before the
// barrier but leaves global loads in flight (a full __syncthreads waits for
// every outstanding memory operation, which ends any prefetch at the barrier).
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// index along axis a (0 = x, 1 = y, 2 = z) of a Morton key
__host__ __device__ inline uint32_t morton_axis(uint32_t key, int a) { return compact3(key >> a); }

// Exclusive prefix sums over n entries (in may equal out); tmp needs
// (n + 1023) / 1024 + 1 ints.  Enqueued on stream s.
void scan_exclusive_i32(const int *in, int *out, int64_t n, int *tmp, hipStream_t s);
void scan_exclusive_u32(const unsigned *in, unsigned *out, int64_t n, int *tmp, hipStream_t s);

}  // namespace eifmm
