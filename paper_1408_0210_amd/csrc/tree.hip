// tree.hip -- octree build on the GPU (Sec. 3.3: a 2^D-tree with depth+1 levels).
//
// Points are binned into the leaf cells of a uniform octree over [lo, lo+L]^3,
// keyed by Morton order (bit b of the x index at bit 3b, y at 3b+1, z at 3b+2),
// sorted stably by (key, input index) with an LSD radix sort, gathered into
// Morton order, and summarised per level:
//   leaf_start[key]  first sorted point of each leaf (boxes of any level are
//                    contiguous ranges of sorted points);
//   act[k]           keys of the non-empty boxes of level k, ascending;
//   slot[k][key]     position of a box in act[k], or -1 when empty;
//   cls[k]           slots grouped by child class (key & 7), ascending key;
//   near lists       boxes at Chebyshev index distance <= 1 (Sec. 3.2);
//   interaction lists (export only) children of the parent's neighbours that
//                    are well separated (Sec. 3.3.2).
#include <algorithm>
#include <cstring>

#include "devutil.hpp"
#include "plan.hpp"

namespace eifmm {

// ---------------------------------------------------------------- keys
// With separate targets (tbit = 1) the sort key is 2 * leaf key + (i >= tsplit),
// so each leaf's sources precede its targets.  Each point is also written as one
// 32-byte record (x, y, z, 0) to x4, so that the gather into Morton order reads
// one cache line per point instead of one per coordinate.
__global__ void k_keys(int64_t n, const double *__restrict__ xyz, double lo0, double lo1,
                       double lo2, double L, double scale, int side, int64_t tsplit, int tbit,
                       uint32_t *__restrict__ keys, int *__restrict__ idx,
                       int *__restrict__ err, double *__restrict__ x4) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lo[3] = {lo0, lo1, lo2};
  const double xv[3] = {xyz[i], xyz[n + i], xyz[2 * n + i]};
  double2 *rec = reinterpret_cast<double2 *>(x4 + 4 * i);
  rec[0] = make_double2(xv[0], xv[1]);
  rec[1] = make_double2(xv[2], 0.0);
  uint32_t c[3];
  bool bad = false;
  for (int a = 0; a < 3; ++a) {
    double x = xv[a];
    // closed domain [lo, lo+L]; NaN and +-inf fail the comparison
    if (!(x >= lo[a] && x <= lo[a] + L)) {
      bad = true;
      c[a] = 0;
      continue;
    }
    // one FP64 subtraction and one FP64 multiplication, then floor and clamp
    double t = floor(__dmul_rn(__dsub_rn(x, lo[a]), scale));
    int q = (int)t;
    q = q > side - 1 ? side - 1 : (q < 0 ? 0 : q);
    c[a] = (uint32_t)q;
  }
  if (bad) atomicOr(err, 1);
  keys[i] = (morton_encode(c[0], c[1], c[2]) << tbit) | (uint32_t)(tbit && i >= tsplit);
  idx[i] = (int)i;
}

// ---------------------------------------------------------------- radix sort
// Tile of kSortTile keys per block (256 threads x 4 rounds); digits of 8 bits.
constexpr int kSortTile = 1024;

__global__ __launch_bounds__(256) void k_sort_hist(const uint32_t *__restrict__ keys, int64_t n,
                                                   int shift, unsigned *__restrict__ hist,
                                                   int ntiles) {
  __shared__ unsigned cnt[256];
  const int t = threadIdx.x, tile = blockIdx.x;
  cnt[t] = 0;
  __syncthreads();
  for (int r = 0; r < kSortTile / 256; ++r) {
    int64_t e = (int64_t)tile * kSortTile + r * 256 + t;
    if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)t * ntiles + tile] = cnt[t];
}

// Stable scatter: within a round, lanes of a wave with equal digits are ranked
// by lane order (ballot match), waves by wave order, rounds by round order.
__global__ __launch_bounds__(256) void k_sort_scatter(const uint32_t *__restrict__ kin,
                                                      const int *__restrict__ iin,
                                                      uint32_t *__restrict__ kout,
                                                      int *__restrict__ iout, int64_t n,
                                                      int shift,
                                                      const unsigned *__restrict__ hist,
                                                      int ntiles) {
  __shared__ unsigned run[256];
  __shared__ unsigned wcnt[4][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, tile = blockIdx.x;
  run[t] = hist[(int64_t)t * ntiles + tile];
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kSortTile / 256; ++r) {
    for (int q = 0; q < 4; ++q) wcnt[q][t] = 0;
    __syncthreads();
    int64_t e = (int64_t)tile * kSortTile + r * 256 + t;
    bool valid = e < n;
    uint32_t key = valid ? kin[e] : 0u;
    int id = valid ? iin[e] : 0;
    unsigned dig = (key >> shift) & 255u;
    uint64_t mask = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      bool bit = (dig >> b) & 1u;
      uint64_t bal = __ballot(bit);
      mask &= bit ? bal : ~bal;
    }
    unsigned rank = (unsigned)__popcll(mask & lt);
    if (valid && rank == 0) wcnt[w][dig] = (unsigned)__popcll(mask);
    __syncthreads();
    unsigned pos = 0;
    if (valid) {
      pos = run[dig] + rank;
      for (int q = 0; q < w; ++q) pos += wcnt[q][dig];
    }
    __syncthreads();
    run[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
    if (valid) {
      kout[pos] = key;
      iout[pos] = id;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- gather
// xs (SoA 3 x n, Morton order) from the records k_keys wrote in input order
__global__ void k_gather_points(int64_t n, const double *__restrict__ x4,
                                const int *__restrict__ perm, double *__restrict__ xs) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double2 *rec = reinterpret_cast<const double2 *>(x4 + 4 * (int64_t)perm[s]);
  const double2 a = rec[0], b = rec[1];
  xs[s] = a.x;
  xs[n + s] = a.y;
  xs[2 * n + s] = b.x;
}

// ls[k] = first sorted position with key >= (k << shift) + add, k = 0..nleaf
// (leaf_start: shift = tbit, add = 0; first target of a leaf: shift 1, add 1)
__global__ void k_leaf_start(int64_t n, const uint32_t *__restrict__ keys, int64_t nleaf,
                             int shift, int add, int *__restrict__ ls) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > nleaf) return;
  const int64_t v = (k << shift) + add;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if ((int64_t)keys[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  ls[k] = (int)lo;
}

// ---------------------------------------------------------------- active boxes
__device__ inline bool box_active(const int *__restrict__ ls, int shift, int64_t b) {
  return ls[(b + 1) << shift] > ls[b << shift];
}

// per block of 256 boxes: active count per child class and in total
// near-field work: out[0] = point pairs (count(leaf) x the point count of its
// near list, summed over active leaves), out[1] = the same with count(leaf)
// rounded up to 32-target chunks (the sweeps the near-field kernels make);
// integer atomics, so the totals are exact
// (targets of the leaf [tb[key], ls[key + 1]), sources of a neighbour [ls, se))
__global__ __launch_bounds__(256) void k_near_pairs(const uint32_t *__restrict__ act,
                                                    const int *__restrict__ ls,
                                                    const int *__restrict__ se,
                                                    const int *__restrict__ tb,
                                                    const int *__restrict__ near_ptr,
                                                    const int *__restrict__ near_src, int nact,
                                                    unsigned long long *__restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nact) return;
  const uint32_t key = act[j];
  long long src = 0;
  for (int q = near_ptr[j]; q < near_ptr[j + 1]; ++q) {
    const uint32_t sk = act[near_src[q]];
    src += se[sk] - ls[sk];
  }
  const long long cnt = ls[key + 1] - tb[key];
  atomicAdd(out, (unsigned long long)(cnt * src));
  atomicAdd(out + 1, (unsigned long long)(((cnt + 31) / 32) * 32 * src));
}

// number of 32-target chunks of each active leaf (targets [tb[key], ls[key + 1]));
// 0 past the active count
__global__ __launch_bounds__(256) void k_chunk_count(const uint32_t *__restrict__ act,
                                                     const int *__restrict__ ls,
                                                     const int *__restrict__ tb,
                                                     const int *__restrict__ nact, int64_t len,
                                                     int *__restrict__ cnt) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= len) return;
  int c = 0;
  if (j < *nact) {
    const uint32_t key = act[j];
    c = (ls[key + 1] - tb[key] + 31) >> 5;
  }
  cnt[j] = c;
}

// The active boxes of every level from 2 to the leaf level, in three launches
// for all levels: a box is active when its subtree holds a point (a non-empty
// range of leaf_start).  Blocks of 256 boxes; block numbers run over the levels
// one after another (blk0), and blkcnt holds 9 counts per block (one per child
// class, then the total).
struct ActLevels {
  int n;                        // levels
  int shift[kMaxLevels];        // 3 (depth - k)
  int64_t nb[kMaxLevels];       // 8^k boxes
  int blk0[kMaxLevels + 1];     // first block of each level; blk0[n] = all blocks
  uint32_t *act[kMaxLevels];    // compact keys, ascending
  int *slot[kMaxLevels];        // dense map key -> compact index or -1
  int *cls[kMaxLevels];         // compact indices grouped by child class
  int *counts[kMaxLevels];      // class offsets [0, 8) and the total [8]
};

__device__ inline int act_level(const ActLevels &L, int blk) {
  int q = 0;
  while (q + 1 < L.n && L.blk0[q + 1] <= blk) ++q;
  return q;
}

__global__ __launch_bounds__(256) void k_act_count(const int *__restrict__ ls, ActLevels L,
                                                   int *__restrict__ blkcnt) {
  __shared__ int c[9];
  const int t = threadIdx.x;
  if (t < 9) c[t] = 0;
  __syncthreads();
  const int q = act_level(L, blockIdx.x);
  const int64_t b = (int64_t)(blockIdx.x - L.blk0[q]) * 256 + t;
  if (b < L.nb[q] && box_active(ls, L.shift[q], b)) {
    atomicAdd(&c[8], 1);
    atomicAdd(&c[b & 7], 1);
  }
  __syncthreads();
  if (t < 9) blkcnt[(int64_t)blockIdx.x * 9 + t] = c[t];
}

// one block per level: exclusive scan of the 9 columns over the level's blocks
// (in place); the class offsets and the total go to the level's counts
__global__ __launch_bounds__(1024) void k_act_scan(int *__restrict__ blkcnt, ActLevels L) {
  __shared__ int part[9][1024];
  const int q = blockIdx.x, t = threadIdx.x;
  const int b0 = L.blk0[q], nblk = L.blk0[q + 1] - b0;
  const int per = (nblk + 1023) / 1024;
  const int a = min(nblk, t * per), b = min(nblk, a + per);
  int s[9], run[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) s[c] = 0;
  for (int i = a; i < b; ++i)
#pragma unroll
    for (int c = 0; c < 9; ++c) s[c] += blkcnt[(int64_t)(b0 + i) * 9 + c];
#pragma unroll
  for (int c = 0; c < 9; ++c) part[c][t] = s[c];
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) v[c] = t >= off ? part[c][t - off] : 0;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 9; ++c) part[c][t] += v[c];
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < 9; ++c) run[c] = part[c][t] - s[c];
  for (int i = a; i < b; ++i)
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const int64_t o = (int64_t)(b0 + i) * 9 + c;
      const int v = blkcnt[o];
      blkcnt[o] = run[c];
      run[c] += v;
    }
  if (t == 0) {
    int off = 0;
    for (int c = 0; c < 8; ++c) {
      L.counts[q][c] = off;
      off += part[c][1023];
    }
    L.counts[q][8] = part[8][1023];
  }
}

__global__ __launch_bounds__(256) void k_act_scatter(const int *__restrict__ ls, ActLevels L,
                                                     const int *__restrict__ blkoff) {
  __shared__ int wtot[4][9];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int q = act_level(L, blockIdx.x);
  const int64_t b = (int64_t)(blockIdx.x - L.blk0[q]) * 256 + t;
  const bool a = b < L.nb[q] && box_active(ls, L.shift[q], b);
  const int c = (int)(b & 7);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint64_t ball = __ballot(a);
  uint64_t bc[8];
  for (int k = 0; k < 8; ++k) bc[k] = __ballot(a && c == k);
  if (lane == 0) {
    wtot[w][8] = (int)__popcll(ball);
    for (int k = 0; k < 8; ++k) wtot[w][k] = (int)__popcll(bc[k]);
  }
  __syncthreads();
  if (b >= L.nb[q]) return;
  if (!a) {
    L.slot[q][b] = -1;
    return;
  }
  int rt = (int)__popcll(ball & lt), rc = (int)__popcll(bc[c] & lt);
  for (int k = 0; k < w; ++k) {
    rt += wtot[k][8];
    rc += wtot[k][c];
  }
  const int64_t bo = (int64_t)blockIdx.x * 9;
  const int pos = blkoff[bo + 8] + rt;
  L.act[q][pos] = (uint32_t)b;
  L.slot[q][b] = pos;
  L.cls[q][L.counts[q][c] + blkoff[bo + c] + rc] = pos;
}

// M2L target order (levels 2..kMaxOrderLevel).  A box of class c at level k has
// parent coordinates p_a, and its sources lie at 2 p_a - 2 .. 2 p_a + 3 per axis,
// so a source falls outside the domain only for p_a = 0 (below) or p_a =
// 2^(k-1) - 1 (above): the boxes of one class and one face signature (3 states
// per axis) miss the same offsets.  One block per (level, class): a stable
// counting sort of the class's slots by signature.
struct OrdLevels {
  int n;
  int level[kMaxLevels];
  const uint32_t *act[kMaxLevels];
  const int *cls[kMaxLevels];
  const int *counts[kMaxLevels];  // class offsets [0, 8) and the total [8]
  int *ord[kMaxLevels];
};

__device__ inline int face_signature(uint32_t key, int last) {
  int s = 0, m = 1;
  for (int a = 0; a < 3; ++a) {
    const int p = (int)morton_axis(key, a) >> 1;
    s += m * (p == 0 ? 0 : (p == last ? 2 : 1));
    m *= 3;
  }
  return s;
}

__global__ __launch_bounds__(1024) void k_m2l_order(OrdLevels L) {
  __shared__ int base[27];
  __shared__ int wcnt[16][27];
  const int q = (int)blockIdx.x >> 3, c = (int)blockIdx.x & 7;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int last = (1 << (L.level[q] - 1)) - 1;
  const int *cnt = L.counts[q];
  const int beg = cnt[c], end = c < 7 ? cnt[c + 1] : cnt[8];
  const uint32_t *act = L.act[q];
  const int *cls = L.cls[q];
  int *ord = L.ord[q];
  if (t < 27) base[t] = 0;
  __syncthreads();
  for (int i = beg + t; i < end; i += 1024) atomicAdd(&base[face_signature(act[cls[i]], last)], 1);
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int b = 0; b < 27; ++b) {
      const int v = base[b];
      base[b] = run;
      run += v;
    }
  }
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int c0 = beg; c0 < end; c0 += 1024) {
    const int i = c0 + t;
    const bool v = i < end;
    const int sl = v ? cls[i] : 0;
    const int b = v ? face_signature(act[sl], last) : -1;
    int rk = 0;
    for (int bb = 0; bb < 27; ++bb) {
      const uint64_t m = __ballot(b == bb);
      if (b == bb) rk = (int)__popcll(m & lt);
      if (lane == 0) wcnt[w][bb] = (int)__popcll(m);
    }
    __syncthreads();
    if (v) {
      int o = base[b] + rk;
      for (int ww = 0; ww < w; ++ww) o += wcnt[ww][b];
      ord[beg + o] = sl;
    }
    __syncthreads();
    if (t < 27) {
      int sum = 0;
      for (int ww = 0; ww < 16; ++ww) sum += wcnt[ww][t];
      base[t] += sum;
    }
    __syncthreads();
  }
}

// interaction-list entries of level `level` summed into *out (statistics):
// for a box of child class c the offsets are delta_a in [-2-c_a, 3-c_a] with
// ||delta||_inf >= 2 (the children of the parent's neighbours that are well
// separated, Sec. 3.3.2)
__global__ __launch_bounds__(256) void k_il_count(int level, const uint32_t *__restrict__ act,
                                                  const int *__restrict__ nact,
                                                  const int *__restrict__ slot,
                                                  unsigned long long *__restrict__ out) {
  __shared__ int tot;
  if (threadIdx.x == 0) tot = 0;
  __syncthreads();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  int c = 0;
  if (j < *nact) {
    const int side = 1 << level;
    const uint32_t key = act[j];
    int n[3], p[3];
    for (int a = 0; a < 3; ++a) {
      n[a] = (int)morton_axis(key, a);
      p[a] = n[a] & 1;
    }
    for (int dz = -2 - p[2]; dz <= 3 - p[2]; ++dz)
      for (int dy = -2 - p[1]; dy <= 3 - p[1]; ++dy)
        for (int dx = -2 - p[0]; dx <= 3 - p[0]; ++dx) {
          if (max(abs(dx), max(abs(dy), abs(dz))) < 2) continue;
          const int m0 = n[0] + dx, m1 = n[1] + dy, m2 = n[2] + dz;
          if (m0 < 0 || m1 < 0 || m2 < 0 || m0 >= side || m1 >= side || m2 >= side) continue;
          if (slot[morton_encode((uint32_t)m0, (uint32_t)m1, (uint32_t)m2)] >= 0) ++c;
        }
  }
  if (c) atomicAdd(&tot, c);
  __syncthreads();
  if (threadIdx.x == 0 && tot) atomicAdd(out, (unsigned long long)tot);
}

// ---------------------------------------------------------------- lists
// mode 0: near list (Chebyshev <= 1, self included); mode 1: interaction list.
// Entries are source slots (ascending slot = ascending key) and, for mode 1,
// offset ids.
template <int MODE>
__global__ void k_list(int level, const uint32_t *__restrict__ act, const int *__restrict__ nact,
                       const int *__restrict__ slot, const int *__restrict__ ptr,
                       int *__restrict__ cnt, int *__restrict__ src,
                       int16_t *__restrict__ off, const int16_t *__restrict__ code2id) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= *nact) {
    if (cnt && j == *nact) cnt[j] = 0;
    return;
  }
  const int side = 1 << level;
  const uint32_t key = act[j];
  const int n0 = (int)morton_axis(key, 0), n1 = (int)morton_axis(key, 1),
            n2 = (int)morton_axis(key, 2);
  int s_loc[189];
  int16_t o_loc[189];
  int c = 0;
  const int R = MODE == 0 ? 1 : 3;
  for (int dz = -R; dz <= R; ++dz)
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        const int m0 = n0 + dx, m1 = n1 + dy, m2 = n2 + dz;
        if (m0 < 0 || m1 < 0 || m2 < 0 || m0 >= side || m1 >= side || m2 >= side) continue;
        if (MODE == 1) {
          int cheb = max(abs(dx), max(abs(dy), abs(dz)));
          if (cheb < 2) continue;
          int pc = max(abs((m0 >> 1) - (n0 >> 1)),
                       max(abs((m1 >> 1) - (n1 >> 1)), abs((m2 >> 1) - (n2 >> 1))));
          if (pc > 1) continue;
        }
        int sl = slot[morton_encode((uint32_t)m0, (uint32_t)m1, (uint32_t)m2)];
        if (sl < 0) continue;
        if (src) {
          s_loc[c] = sl;
          if (MODE == 1) o_loc[c] = code2id[(dx + 3) + 7 * (dy + 3) + 49 * (dz + 3)];
        }
        ++c;
      }
  if (cnt) {
    cnt[j] = c;
    return;
  }
  // insertion sort by source slot
  for (int a = 1; a < c; ++a) {
    int s = s_loc[a];
    int16_t o = MODE == 1 ? o_loc[a] : 0;
    int b = a - 1;
    while (b >= 0 && s_loc[b] > s) {
      s_loc[b + 1] = s_loc[b];
      if (MODE == 1) o_loc[b + 1] = o_loc[b];
      --b;
    }
    s_loc[b + 1] = s;
    if (MODE == 1) o_loc[b + 1] = o;
  }
  const int base = ptr[j];
  for (int a = 0; a < c; ++a) {
    src[base + a] = s_loc[a];
    if (MODE == 1) off[base + a] = o_loc[a];
  }
}

// ---------------------------------------------------------------- host side
namespace {

int sort_points(Plan &P, hipStream_t s) {
  const int64_t n = P.n;
  const int bits = 3 * P.depth + (P.nt ? 1 : 0);
  const int ntiles = (int)((n + kSortTile - 1) / kSortTile);
  uint32_t *ka = P.keys, *kb = P.keys_tmp;
  int *ia = P.idx, *ib = P.idx_tmp;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_sort_hist, dim3(ntiles), dim3(256), 0, s, ka, n, shift, P.hist, ntiles);
    scan_exclusive_u32(P.hist, P.hist, (int64_t)256 * ntiles, P.scan_tmp, s);
    hipLaunchKernelGGL(k_sort_scatter, dim3(ntiles), dim3(256), 0, s, ka, ia, kb, ib, n, shift,
                       P.hist, ntiles);
    std::swap(ka, kb);
    std::swap(ia, ib);
  }
  if (ka != P.keys) {  // odd pass count: result sits in the tmp buffers
    std::swap(P.keys, P.keys_tmp);
    std::swap(P.idx, P.idx_tmp);
  }
  return EIFMM_OK;
}

// active boxes of levels k0..k1
void build_active(Plan &P, int k0, int k1, hipStream_t s) {
  ActLevels L{};
  int blk = 0;
  for (int k = k0; k <= k1; ++k) {
    const int q = L.n++;
    L.shift[q] = 3 * (P.depth - k);
    L.nb[q] = (int64_t)1 << (3 * k);
    L.blk0[q] = blk;
    blk += (int)((L.nb[q] + 255) / 256);
    L.act[q] = P.ld[k].act;
    L.slot[q] = P.ld[k].slot;
    L.cls[q] = P.ld[k].cls;
    L.counts[q] = P.counts_dev + 16 * k;
  }
  L.blk0[L.n] = blk;
  hipLaunchKernelGGL(k_act_count, dim3(blk), dim3(256), 0, s, P.leaf_start, L, P.blkcnt);
  hipLaunchKernelGGL(k_act_scan, dim3(L.n), dim3(1024), 0, s, P.blkcnt, L);
  hipLaunchKernelGGL(k_act_scatter, dim3(blk), dim3(256), 0, s, P.leaf_start, L, P.blkcnt);
}

// CSR list for level k into (ptr, src, off).  bounded: the entry count cannot
// exceed cap (27 near entries per box), so it is not read back and 0 is
// returned; otherwise returns the entry count, or -1 if it exceeds cap.
int64_t build_list(Plan &P, int k, int mode, int *ptr, int *src, int16_t *off, size_t cap,
                   bool bounded, hipStream_t s) {
  LevelDev &L = P.ld[k];
  const int *nact = P.counts_dev + 16 * k + 8;
  const int grid = (int)((L.cap + 1 + 127) / 128);
  int *cnt = P.list_cnt;
  if (mode == 0)
    hipLaunchKernelGGL(k_list<0>, dim3(grid), dim3(128), 0, s, k, L.act, nact, L.slot, nullptr,
                       cnt, nullptr, nullptr, nullptr);
  else
    hipLaunchKernelGGL(k_list<1>, dim3(grid), dim3(128), 0, s, k, L.act, nact, L.slot, nullptr,
                       cnt, nullptr, nullptr, P.code2id);
  scan_exclusive_i32(cnt, ptr, (int64_t)L.cap + 1, P.scan_tmp, s);
  int total = 0;
  if (!bounded) {
    hipMemcpyAsync(&total, ptr + P.nact[k], sizeof(int), hipMemcpyDeviceToHost, s);
    hipStreamSynchronize(s);
    if ((size_t)total > cap) return -1;
  }
  if (mode == 0)
    hipLaunchKernelGGL(k_list<0>, dim3(grid), dim3(128), 0, s, k, L.act, nact, L.slot, ptr,
                       nullptr, src, nullptr, nullptr);
  else
    hipLaunchKernelGGL(k_list<1>, dim3(grid), dim3(128), 0, s, k, L.act, nact, L.slot, ptr,
                       nullptr, src, off, P.code2id);
  return total;
}

}  // namespace

// interaction-list pairs of levels 2..depth (64-bit count in ints 10-11 of each
// level's block of counts_dev, zeroed with the tree)
void il_count_launch(Plan &P, hipStream_t s) {
  for (int k = 2; k <= P.depth; ++k) {
    const int grid = (int)((P.ld[k].cap + 255) / 256);
    hipLaunchKernelGGL(k_il_count, dim3(grid), dim3(256), 0, s, k, P.ld[k].act,
                       P.counts_dev + 16 * k + 8, P.ld[k].slot,
                       (unsigned long long *)(P.counts_dev + 16 * k + 10));
  }
}

int tree_build(Plan &P, const double *xyz_in, hipStream_t s) {
  const int64_t n = P.n;
  const int depth = P.depth;
  const int side = 1 << depth;
  const double scale = std::ldexp(1.0, depth) / P.cfg.L;
  const int tbit = P.nt ? 1 : 0;
  const int *tb = tbit ? P.tgt_begin : P.leaf_start;
  // the counter block and the error flag after it
  hipMemsetAsync(P.counts_dev, 0, sizeof(int) * (16 * kMaxLevels + 1), s);
  if (n > 0) {
    hipLaunchKernelGGL(k_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, xyz_in,
                       P.cfg.lo[0], P.cfg.lo[1], P.cfg.lo[2], P.cfg.L, scale, side, P.ns, tbit,
                       P.keys, P.idx, P.errflag, P.xyz4);
    sort_points(P, s);
    hipLaunchKernelGGL(k_gather_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       P.xyz4, P.idx, P.xyz);
  }
  const int64_t nleaf = (int64_t)1 << (3 * depth);
  hipLaunchKernelGGL(k_leaf_start, dim3((unsigned)((nleaf + 1 + 255) / 256)), dim3(256), 0, s, n,
                     P.keys, nleaf, tbit, 0, P.leaf_start);
  if (tbit)
    hipLaunchKernelGGL(k_leaf_start, dim3((unsigned)((nleaf + 1 + 255) / 256)), dim3(256), 0, s,
                       n, P.keys, nleaf, 1, 1, P.tgt_begin);
  build_active(P, std::min(2, depth), depth, s);
  if (!P.il_lazy) il_count_launch(P, s);
  // the counts and the error flag, into pinned memory; the host waits for this
  // copy only, while the order, the near lists and the chunks below (which read
  // the counts on the device) run
  int *host_counts = P.counts_pin;
  hipMemcpyAsync(host_counts, P.counts_dev, sizeof(int) * (16 * kMaxLevels + 1),
                 hipMemcpyDeviceToHost, s);
  hipEventRecord(P.ev_counts, s);
  // M2L target order of the levels that keep one
  {
    OrdLevels L{};
    for (int k = 2; k <= std::min(depth, kMaxOrderLevel); ++k) {
      if (!P.ld[k].ord) continue;
      const int q = L.n++;
      L.level[q] = k;
      L.act[q] = P.ld[k].act;
      L.cls[q] = P.ld[k].cls;
      L.counts[q] = P.counts_dev + 16 * k;
      L.ord[q] = P.ld[k].ord;
    }
    if (L.n) hipLaunchKernelGGL(k_m2l_order, dim3(8 * L.n), dim3(1024), 0, s, L);
  }
  // near lists of the leaf level (used by the near-field pass); at most 27
  // entries per box, within near_cap = 27 cap
  build_list(P, depth, 0, P.near_ptr, P.near_src, nullptr, P.near_cap, true, s);
  // 32-target chunks of the leaves (the work of the near-field and L2P kernels).
  // The grid is launched with the bound nact + ceil(n / 32) on the chunk count,
  // and workgroups past chunk_ptr[nact] exit, so the count is not read back.
  {
    const int64_t cap = P.ld[depth].cap;
    hipLaunchKernelGGL(k_chunk_count, dim3((unsigned)((cap + 1 + 255) / 256)), dim3(256), 0, s,
                       P.ld[depth].act, P.leaf_start, tb, P.counts_dev + 16 * depth + 8, cap + 1,
                       P.list_cnt);
    scan_exclusive_i32(P.list_cnt, P.chunk_ptr, cap + 1, P.scan_tmp, s);
  }
  hipError_t e = hipEventSynchronize(P.ev_counts);
  const int err = host_counts[16 * kMaxLevels];
  if (e != hipSuccess) {
    P.last_hip_error = (int)e;
    return EIFMM_EHIP;
  }
  if (err) return EIFMM_EDOMAIN;
  for (int k = std::min(2, depth); k <= depth; ++k) {
    P.nact[k] = host_counts[16 * k + 8];
    for (int c = 0; c < 8; ++c) P.cls_off[k][c] = host_counts[16 * k + c];
    P.cls_off[k][8] = P.nact[k];
    if (!P.il_lazy) {
      unsigned long long ilp = 0;
      std::memcpy(&ilp, &host_counts[16 * k + 10], sizeof(ilp));
      P.il_pairs[k] = k >= 2 ? (int64_t)ilp : 0;
    }
  }
  P.il_pending = P.il_lazy;
  P.nchunk = P.nact[depth] > 0 ? P.nact[depth] + (n + 31) / 32 : 0;  // the near-field pair counts (statistics) are taken when they are read
  P.counts_pending = true;
  e = hipGetLastError();
  if (e != hipSuccess) {
    P.last_hip_error = (int)e;
    return EIFMM_EHIP;
  }
  return EIFMM_OK;
}

// Copies the counts the tree build leaves on the device (near-list entries,
// near-field point pairs) to the plan; synchronises the host with the device.
int tree_counts(Plan &P) {
  if (P.il_pending) {
    // the tree's interaction pairs, counted now (the tree is complete once the
    // device is idle), and the M2L flops of the jobs built on it
    int hc[16 * kMaxLevels];
    if (hipDeviceSynchronize() != hipSuccess) return EIFMM_EHIP;
    il_count_launch(P, nullptr);
    if (hipMemcpy(hc, P.counts_dev, sizeof(hc), hipMemcpyDeviceToHost) != hipSuccess)
      return EIFMM_EHIP;
    for (int k = 2; k <= P.depth; ++k) {
      unsigned long long ilp = 0;
      std::memcpy(&ilp, &hc[16 * k + 10], sizeof(ilp));
      P.il_pairs[k] = (int64_t)ilp;
    }
    P.il_pending = false;
    if (P.jobs.nrhs > 0) P.m2l_flops = m2l_flops_of(P, P.jobs.nrhs);
  }
  if (!P.counts_pending) return EIFMM_OK;
  const int depth = P.depth;
  int total = 0;
  unsigned long long npairs[2] = {0, 0};
  if (P.nact[depth] > 0) {
    // the tree is complete once the device is idle
    if (hipDeviceSynchronize() != hipSuccess) return EIFMM_EHIP;
    const int *se = P.nt ? P.tgt_begin : P.leaf_start + 1;
    const int *tb = P.nt ? P.tgt_begin : P.leaf_start;
    hipMemsetAsync(P.npairs_dev, 0, 2 * sizeof(unsigned long long), nullptr);
    hipLaunchKernelGGL(k_near_pairs, dim3((unsigned)((P.nact[depth] + 255) / 256)), dim3(256), 0,
                       nullptr, P.ld[depth].act, P.leaf_start, se, tb, P.near_ptr, P.near_src,
                       (int)P.nact[depth], P.npairs_dev);
  }
  if (P.nact[depth] > 0 &&
      (hipMemcpy(&total, P.near_ptr + P.nact[depth], sizeof(int), hipMemcpyDeviceToHost) !=
           hipSuccess ||
       hipMemcpy(npairs, P.npairs_dev, sizeof(npairs), hipMemcpyDeviceToHost) != hipSuccess))
    return EIFMM_EHIP;
  P.near_total = total;
  P.near_point_pairs = (int64_t)npairs[0];
  P.near_lane_pairs = (int64_t)npairs[1];
  P.counts_pending = false;
  return EIFMM_OK;
}

int lists_export(Plan &P, int level, int64_t *nactive, uint32_t *active, int64_t *near_ptr,
                 uint32_t *near_src, int64_t *il_ptr, uint32_t *il_src, int16_t *il_off) {
  hipStream_t s = nullptr;
  if (level < 0 || level > P.depth) return EIFMM_EINVAL;
  const int lo_level = std::min(2, P.depth);
  if (level < lo_level) {
    // levels 0 and 1 are not kept per query; build them on the fly
    build_active(P, level, level, s);
    int hc[16];
    hipMemcpy(hc, P.counts_dev + 16 * level, sizeof(int) * 16, hipMemcpyDeviceToHost);
    P.nact[level] = hc[8];
  }
  LevelDev &L = P.ld[level];
  const int64_t na = P.nact[level];
  *nactive = na;
  std::vector<uint32_t> act(na);
  hipMemcpy(act.data(), L.act, sizeof(uint32_t) * na, hipMemcpyDeviceToHost);
  if (active) std::memcpy(active, act.data(), sizeof(uint32_t) * na);
  const size_t cap_near = (size_t)27 * (na + 1), cap_il = (size_t)189 * (na + 1);
  int *dptr = nullptr, *dsrc = nullptr;
  int16_t *doff = nullptr;
  if (hipMalloc(&dptr, sizeof(int) * (L.cap + 2)) != hipSuccess) return EIFMM_ENOMEM;
  if (hipMalloc(&dsrc, sizeof(int) * std::max(cap_near, cap_il)) != hipSuccess ||
      hipMalloc(&doff, sizeof(int16_t) * cap_il) != hipSuccess) {
    hipFree(dptr);
    hipFree(dsrc);
    return EIFMM_ENOMEM;
  }
  int rc = EIFMM_OK;
  for (int mode = 0; mode < 2 && rc == EIFMM_OK; ++mode) {
    int64_t *optr = mode == 0 ? near_ptr : il_ptr;
    uint32_t *osrc = mode == 0 ? near_src : il_src;
    if (!optr) continue;
    if (mode == 1 && level < 2) {
      for (int64_t j = 0; j <= na; ++j) optr[j] = 0;
      continue;
    }
    int64_t tot =
        build_list(P, level, mode, dptr, dsrc, doff, mode == 0 ? cap_near : cap_il, false, s);
    if (tot < 0) {
      rc = EIFMM_ENOMEM;
      break;
    }
    std::vector<int> hp(na + 1), hs(tot);
    hipMemcpy(hp.data(), dptr, sizeof(int) * (na + 1), hipMemcpyDeviceToHost);
    hipMemcpy(hs.data(), dsrc, sizeof(int) * tot, hipMemcpyDeviceToHost);
    for (int64_t j = 0; j <= na; ++j) optr[j] = hp[j];
    if (osrc)
      for (int64_t q = 0; q < tot; ++q) osrc[q] = act[hs[q]];
    if (mode == 1 && il_off) hipMemcpy(il_off, doff, sizeof(int16_t) * tot, hipMemcpyDeviceToHost);
  }
  hipFree(dptr);
  hipFree(dsrc);
  hipFree(doff);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    P.last_hip_error = (int)e;
    return EIFMM_EHIP;
  }
  return rc;
}

}  // namespace eifmm
