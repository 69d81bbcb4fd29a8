// setup.cpp -- host FP64 precomputation of a plan (runs once per plan).
//
//  * training sets: the paper leaves D_x,trial / D_y,trial open (Sec. 2); this
//    library uses cube-surface shells in I_0^k and the surface (or a volume
//    grid) of J_0^k, in units of l_k so that a homogeneous kernel selects the
//    same scaled points on every level;
//  * Algorithm 1 in the L-infinity norm, which is cross approximation with
//    complete pivoting on the training matrix: pick the largest residual
//    entry (lowest row, then lowest column on ties), subtract the rank-1 term,
//    stop once the largest residual is <= tau * scale (end of Sec. 2);
//  * M = K(X, Y) factored without pivoting as M = Gamma B^T (Crout), so that
//    Delta = B^{-T} Gamma^{-1} = M^{-1} (eq. (5));
//  * for a kernel that is not symmetric (or when asked), the second EIM of Sec.
//    3.1 per level, on D_x = J_0 and D_y = I_0 (the training sets exchanged): its
//    J_0 points are the rows of the M2L and L2L operators, its I_0 points the L2P
//    points, and its M_B^{-1} = Delta^{J_0,I_0} gives lhat and the L2L operators;
//  * M2M / L2L operators K M^{-1} and K M^{-T} formed row by row with
//    triangular solves, never with an explicit inverse (Sec. 4.1);
//  * the 316 M2L matrices K^delta = K(Y, Y + 2 l_k delta) (Sec. 4.2), and, when
//    asked for, their compression (Sec. 4.2, first stage): the leading left
//    singular vectors U of [K^delta_1 .. K^delta_316] (Householder QR of the
//    transpose, then a one-sided Jacobi SVD of R^T -- an exact SVD in place of the
//    paper's bivariate ACA) and C^delta = U^T K^delta U; the factor B^{-T} of
//    Delta = M^{-1} is folded into the projection before the M2L step, U^T B^{-T}
//    (the Gamma solve stays on the device).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>

#include "plan.hpp"

namespace eifmm {
namespace {

// Host kernel k(z); the squared norm is summed x, y, z.
inline double kern_host(int kind, double p, double zx, double zy, double zz) {
  double r2 = zx * zx + zy * zy + zz * zz;
  switch (kind) {
    case EIFMM_K_LAPLACE:
      return 1.0 / std::sqrt(r2);
    case EIFMM_K_YUKAWA: {
      double r = std::sqrt(r2);
      return std::exp(-p * r) / r;
    }
    case EIFMM_K_GAUSS:
      return std::exp(-r2 / p);
    case EIFMM_K_SQDIST:
      return r2;
    case EIFMM_K_COSR: {
      double r = std::sqrt(r2);
      return std::cos(p * r) / r;
    }
    case EIFMM_K_MQ:
      return std::sqrt(r2 + p);
    case EIFMM_K_ADVDIFF: {
      double r = std::sqrt(r2);
      return std::exp(p * (zx - r)) / r;
    }
  }
  return NAN;
}

int hw_threads() {
  unsigned t = std::thread::hardware_concurrency();
  if (t == 0) t = 4;
  if (t > 64) t = 64;
  return (int)t;
}

template <class F>
void parallel_for(int64_t n, F fn, bool small_ok = false) {
  if (n <= 0) return;
  int nt = hw_threads();
  if (small_ok)
    nt = (int)std::min<int64_t>(nt, n);  // each item is large work
  else if (n < 2 * nt)
    nt = 1;
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; t++) {
    int64_t a = t * chunk, b = std::min<int64_t>(n, a + chunk);
    if (a >= b) break;
    th.emplace_back([=, &fn]() { fn(a, b); });
  }
  for (auto &x : th) x.join();
}

// ---- training sets ---------------------------------------------------------
// Cube surface ||u||_inf = rho with an m x m grid per face.  Faces in the order
// x-, x+, y-, y+, z-, z+; on each face the lower free axis varies slowest; a
// grid point lying on several faces belongs to the face of the lowest axis.
void add_shell(double rho, int m, std::vector<double> &out) {
  static const int free_axes[3][2] = {{1, 2}, {0, 2}, {0, 1}};
  for (int ax = 0; ax < 3; ++ax) {
    const int a0 = free_axes[ax][0], a1 = free_axes[ax][1];
    for (int side = 0; side < 2; ++side) {
      const double face = side ? rho : -rho;
      for (int i = 0; i < m; ++i) {
        const bool edge0 = (i == 0 || i == m - 1);
        if (a0 < ax && edge0) continue;
        for (int j = 0; j < m; ++j) {
          const bool edge1 = (j == 0 || j == m - 1);
          if (a1 < ax && edge1) continue;
          double u[3];
          u[ax] = face;
          u[a0] = rho * double(2 * i - (m - 1)) / double(m - 1);
          u[a1] = rho * double(2 * j - (m - 1)) / double(m - 1);
          out.insert(out.end(), u, u + 3);
        }
      }
    }
  }
}

void add_volume(int m, std::vector<double> &out) {
  for (int iz = 0; iz < m; ++iz)
    for (int iy = 0; iy < m; ++iy)
      for (int ix = 0; ix < m; ++ix) {
        out.push_back(double(2 * ix - (m - 1)) / double(m - 1));
        out.push_back(double(2 * iy - (m - 1)) / double(m - 1));
        out.push_back(double(2 * iz - (m - 1)) / double(m - 1));
      }
}

// kernels without a maximum principle (no decay, oscillation or growth) are
// trained on a volume grid of J_0 rather than on its surface
bool volume_kernel(int kind) {
  return kind == EIFMM_K_GAUSS || kind == EIFMM_K_COSR || kind == EIFMM_K_MQ;
}

// Shell radii in units of l_k; level k keeps those below 2^(k+1) - 1 and then
// adds the outer boundary 2^(k+1) - 1 of I_0^k itself.
const double kShellsSurface[] = {3,   3.5, 4,   5,   6.5, 8.5, 11,  15,   20,   27,
                                 36,  48,  64,  86,  116, 155, 208, 279,  374,  502,
                                 673, 902, 1209, 1621, 2173};
const double kShellsVolume[] = {3,    3.25, 3.5, 3.75, 4,   4.5, 5,   5.5,  6,    6.5,
                                7.25, 8,    9,   10,   11,  12.5, 14, 16,   18,   20,
                                23,   27,   32,  38,   45,  54,  64,  76,   90,   108,
                                128,  152,  181, 215,  256, 304, 362, 431,  512,  609,
                                724,  861,  1024, 1218, 1448, 1722, 2048};

void training_sets(int kind, int level, double lk, std::vector<double> &tx,
                   std::vector<double> &ty) {
  const double outer = double((1 << (level + 1)) - 1);
  const bool vol = volume_kernel(kind);
  const double *radii = vol ? kShellsVolume : kShellsSurface;
  const size_t nr = vol ? sizeof(kShellsVolume) / sizeof(double)
                        : sizeof(kShellsSurface) / sizeof(double);
  tx.clear();
  ty.clear();
  for (size_t s = 0; s < nr; ++s)
    if (radii[s] < outer) add_shell(radii[s], radii[s] < 6.0 ? 19 : 9, tx);
  add_shell(outer, outer < 6.0 ? 19 : 9, tx);
  if (vol)
    add_volume(11, ty);
  else
    add_shell(1.0, 11, ty);
  for (auto &v : tx) v *= lk;
  for (auto &v : ty) v *= lk;
}

// ---- Algorithm 1 as complete-pivot cross approximation ----------------------
// d, scale, relative training error and the selected points from ia / ib
void finish_eim(const std::vector<double> &tx, const std::vector<double> &ty, double scale,
                double emax, LevelHost &out) {
  const int d = (int)out.ia.size();
  out.d = d;
  out.scale = scale;
  out.err = scale > 0 ? emax / scale : 0;
  out.X.resize(3 * (size_t)d);
  out.Y.resize(3 * (size_t)d);
  for (int i = 0; i < d; ++i)
    for (int c = 0; c < 3; ++c) {
      out.X[3 * i + c] = tx[3 * out.ia[i] + c];
      out.Y[3 * i + c] = ty[3 * out.ib[i] + c];
    }
}

// max |K| over the training grid of `level`: the scale of the absolute stopping
// rule (tol_mode 1); swap: the second EIM's grid (D_x = J_0, D_y = I_0).  The
// same kernel values the greedy of that level starts from, so its first pivot
// has this magnitude.
double training_scale(int kind, double p, int level, double L, bool swap) {
  const double lk = std::ldexp(L, -level - 1);
  std::vector<double> tx, ty;
  training_sets(kind, level, lk, tx, ty);
  if (swap) std::swap(tx, ty);
  const int64_t nx = (int64_t)tx.size() / 3, ny = (int64_t)ty.size() / 3;
  std::vector<double> rowmax((size_t)nx, 0.0);
  parallel_for(nx, [&](int64_t a0, int64_t a1) {
    for (int64_t a = a0; a < a1; ++a) {
      double m = 0.0;
      for (int64_t b = 0; b < ny; ++b)
        m = std::max(m, std::fabs(kern_host(kind, p, tx[3 * a] - ty[3 * b],
                                            tx[3 * a + 1] - ty[3 * b + 1],
                                            tx[3 * a + 2] - ty[3 * b + 2])));
      rowmax[(size_t)a] = m;
    }
  });
  double m = 0.0;
  for (double v : rowmax) m = std::max(m, v);
  return m;
}

// swap: the second EIM of Sec. 3.1, with D_x = J_0 and D_y = I_0 (X then holds
// J_0 points, Y holds I_0 points)
int greedy_eim(int kind, double p, int level, double L, double tau, int dmax, double abs_scale,
               bool gpu, bool swap, LevelHost &out) {
  const double lk = std::ldexp(L, -level - 1);
  std::vector<double> tx, ty;
  training_sets(kind, level, lk, tx, ty);
  if (swap) std::swap(tx, ty);
  const int64_t nx = (int64_t)tx.size() / 3, ny = (int64_t)ty.size() / 3;
  std::vector<double> R((size_t)(nx * ny));
  parallel_for(nx, [&](int64_t a0, int64_t a1) {
    for (int64_t a = a0; a < a1; ++a)
      for (int64_t b = 0; b < ny; ++b)
        R[a * ny + b] = kern_host(kind, p, tx[3 * a] - ty[3 * b], tx[3 * a + 1] - ty[3 * b + 1],
                                  tx[3 * a + 2] - ty[3 * b + 2]);
  });
  if (gpu) {
    // the same iterations on the device (eim_gpu.hip), bit for bit
    EimResult res;
    int st = eim_iterate_gpu(R, nx, ny, tau, abs_scale, dmax, res);
    if (st != EIFMM_OK) return st;
    out.ia = res.ia;
    out.ib = res.ib;
    finish_eim(tx, ty, res.scale, res.emax, out);
    return res.status;
  }
  const int nth = hw_threads();
  struct Best {
    double v;
    int64_t a, b;
  };
  std::vector<Best> part(nth);
  std::vector<double> qrow((size_t)ny);
  out.ia.clear();
  out.ib.clear();
  double scale = 0;
  int status = EIFMM_OK;
  for (;;) {
    // largest |residual|, lowest (row, column) on ties
    int64_t chunk = (nx + nth - 1) / nth;
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) {
      th.emplace_back([&, t]() {
        Best bt{-1.0, 0, 0};
        int64_t a0 = t * chunk, a1 = std::min(nx, a0 + chunk);
        for (int64_t a = a0; a < a1; ++a) {
          const double *row = &R[a * ny];
          for (int64_t b = 0; b < ny; ++b) {
            double v = std::fabs(row[b]);
            if (v > bt.v) bt = {v, a, b};
          }
        }
        part[t] = bt;
      });
    }
    for (auto &x : th) x.join();
    Best best{-1.0, 0, 0};
    for (int t = 0; t < nth; ++t)
      if (part[t].v > best.v) best = part[t];  // parts are in row order
    if (out.ia.empty()) scale = abs_scale > 0 ? abs_scale : best.v;
    if (best.v <= tau * scale) break;
    if ((int)out.ia.size() == dmax) {
      status = EIFMM_EEIM;
      break;
    }
    const int64_t as = best.a, bs = best.b;
    const double piv = R[as * ny + bs];
    out.ia.push_back(as);
    out.ib.push_back(bs);
    for (int64_t b = 0; b < ny; ++b) qrow[b] = R[as * ny + b] / piv;
    parallel_for(nx, [&](int64_t a0, int64_t a1) {
      for (int64_t a = a0; a < a1; ++a) {
        double *row = &R[a * ny];
        const double c = row[bs];
        for (int64_t b = 0; b < ny; ++b) row[b] -= c * qrow[b];
      }
    });
  }
  // training error left after the last accepted point
  double emax = 0;
  for (double v : R) emax = std::max(emax, std::fabs(v));
  finish_eim(tx, ty, scale, emax, out);
  return status;
}

// Crout factorisation M = Gamma B^T (Gamma lower, B unit lower), no pivoting:
// the greedy order already makes every leading minor nonzero.
void crout(int kind, double p, LevelHost &lv) {
  const int d = lv.d;
  std::vector<double> M((size_t)d * d), BT((size_t)d * d, 0.0);
  lv.G.assign((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      M[(size_t)i * d + j] =
          kern_host(kind, p, lv.X[3 * i] - lv.Y[3 * j], lv.X[3 * i + 1] - lv.Y[3 * j + 1],
                    lv.X[3 * i + 2] - lv.Y[3 * j + 2]);
  for (int j = 0; j < d; ++j) {
    for (int i = j; i < d; ++i) {
      double s = M[(size_t)i * d + j];
      for (int k = 0; k < j; ++k) s -= lv.G[(size_t)i * d + k] * BT[(size_t)k * d + j];
      lv.G[(size_t)i * d + j] = s;
    }
    BT[(size_t)j * d + j] = 1.0;
    for (int i = j + 1; i < d; ++i) {
      double s = M[(size_t)j * d + i];
      for (int k = 0; k < j; ++k) s -= lv.G[(size_t)j * d + k] * BT[(size_t)k * d + i];
      BT[(size_t)j * d + i] = s / lv.G[(size_t)j * d + j];
    }
  }
  lv.B.assign((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) lv.B[(size_t)i * d + j] = BT[(size_t)j * d + i];
}

// x <- M^{-1} x  (Gamma z = x, then B^T x = z)
void solve_minv(const LevelHost &lv, double *x) {
  const int d = lv.d;
  for (int i = 0; i < d; ++i) {
    double s = x[i];
    for (int j = 0; j < i; ++j) s -= lv.G[(size_t)i * d + j] * x[j];
    x[i] = s / lv.G[(size_t)i * d + i];
  }
  for (int i = d - 1; i >= 0; --i) {
    double s = x[i];
    for (int j = i + 1; j < d; ++j) s -= lv.B[(size_t)j * d + i] * x[j];
    x[i] = s;
  }
}

// x <- M^{-T} x  (B z = x, then Gamma^T x = z)
void solve_mtinv(const LevelHost &lv, double *x) {
  const int d = lv.d;
  for (int i = 0; i < d; ++i) {
    double s = x[i];
    for (int j = 0; j < i; ++j) s -= lv.B[(size_t)i * d + j] * x[j];
    x[i] = s;
  }
  for (int i = d - 1; i >= 0; --i) {
    double s = x[i];
    for (int j = i + 1; j < d; ++j) s -= lv.G[(size_t)j * d + i] * x[j];
    x[i] = s / lv.G[(size_t)i * d + i];
  }
}

// Dense rows x cols (row-major) -> MFMA fragment order for a 16x16x4 A operand:
// [rb = rows/16][ks = cols/4][lane 64], lane l holding row 16 rb + l % 16 and, within
// the 16-column chunk ks / 4, column 4 (l / 16) + ks % 4 (the gathered GEMM feeds B
// in the same k order); padded rows / columns are zero.
void to_fragments(const double *A, int rows, int cols, int rpad, int cpad, double *out) {
  const int nrb = rpad / 16, nks = cpad / 4;
  for (int rb = 0; rb < nrb; ++rb)
    for (int ks = 0; ks < nks; ++ks)
      for (int l = 0; l < 64; ++l) {
        int r = 16 * rb + (l & 15), c = 16 * (ks >> 2) + 4 * (l >> 4) + (ks & 3);
        out[((size_t)rb * nks + ks) * 64 + l] =
            (r < rows && c < cols) ? A[(size_t)r * cols + c] : 0.0;
      }
}

// The same with the k order of an MFMA result used as the B operand: within each
// 16-column chunk, k-step q of lane l takes column (l / 16) + 4 q.
void to_fragments_nat(const double *A, int rows, int cols, int rpad, int cpad, double *out) {
  const int nrb = rpad / 16, nks = cpad / 4;
  for (int rb = 0; rb < nrb; ++rb)
    for (int ks = 0; ks < nks; ++ks)
      for (int l = 0; l < 64; ++l) {
        int r = 16 * rb + (l & 15), c = 16 * (ks >> 2) + (l >> 4) + 4 * (ks & 3);
        out[((size_t)rb * nks + ks) * 64 + l] =
            (r < rows && c < cols) ? A[(size_t)r * cols + c] : 0.0;
      }
}

// Operand table of a blocked triangular solve with 16 x 16 tiles, for the MFMA
// solver: T (d x d, or its transpose) is padded to dp with the identity; tile
// (bi, bj) of the triangle holds -T[bi][bj] off the diagonal and the inverse of
// the diagonal tile T[bi][bi] on it (the inverse of a 16 x 16 triangular tile,
// by substitution; the full triangular factor is never inverted).  Tiles are
// stored in A-operand fragment order: out[((bi nb + bj) 4 + ks) 64 + lane] is
// element (lane % 16, 4 ks + lane / 16) of the tile.
void trsm_table(const std::vector<double> &T, int d, int dp, bool transpose, bool lower,
                std::vector<double> &out) {
  const int nb = dp / 16;
  auto at = [&](int r, int c) -> double {
    if (r < d && c < d) return transpose ? T[(size_t)c * d + r] : T[(size_t)r * d + c];
    return r == c ? 1.0 : 0.0;
  };
  out.assign((size_t)dp * dp, 0.0);
  double tile[16][16], inv[16][16];
  for (int bi = 0; bi < nb; ++bi)
    for (int bj = 0; bj < nb; ++bj) {
      if (lower ? bj > bi : bj < bi) continue;
      for (int i = 0; i < 16; ++i)
        for (int j = 0; j < 16; ++j) tile[i][j] = at(16 * bi + i, 16 * bj + j);
      if (bi == bj) {
        // columns of the inverse by substitution on the identity
        for (int c = 0; c < 16; ++c) {
          if (lower) {
            for (int i = 0; i < 16; ++i) {
              double s = (i == c) ? 1.0 : 0.0;
              for (int j = 0; j < i; ++j) s -= tile[i][j] * inv[j][c];
              inv[i][c] = s / tile[i][i];
            }
          } else {
            for (int i = 15; i >= 0; --i) {
              double s = (i == c) ? 1.0 : 0.0;
              for (int j = i + 1; j < 16; ++j) s -= tile[i][j] * inv[j][c];
              inv[i][c] = s / tile[i][i];
            }
          }
        }
      }
      double *o = &out[((size_t)bi * nb + bj) * 256];
      for (int ks = 0; ks < 4; ++ks)
        for (int l = 0; l < 64; ++l) {
          const int r = l & 15, c = 4 * ks + (l >> 4);
          o[ks * 64 + l] = (bi == bj) ? inv[r][c] : -tile[r][c];
        }
    }
}

void jacobi_left(std::vector<double> &G, int d, std::vector<double> &U, std::vector<double> &s);

// x . y with eight interleaved partial sums added in a fixed order (a long
// single accumulator chain is latency bound)
inline double dot8(const double *x, const double *y, int64_t n) {
  double p[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t i = 0;
  for (; i + 8 <= n; i += 8)
    for (int l = 0; l < 8; ++l) p[l] += x[i + l] * y[i + l];
  for (int l = 0; i < n; ++i, ++l) p[l] += x[i] * y[i];
  return ((p[0] + p[4]) + (p[1] + p[5])) + ((p[2] + p[6]) + (p[3] + p[7]));
}

// Singular values (descending) and left singular vectors (U, d x d row-major,
// column p = vector p) of the d x m matrix whose rows are given in A (row-major,
// m >= d; A is overwritten).  Householder QR of A^T = Q R, then a one-sided
// Jacobi SVD of R^T: R^T V = U diag(s), so A = R^T Q^T = U diag(s) (Q V)^T.
// The reflectors are formed in blocks of 16 columns: inside a block each one is
// applied to the block's remaining columns at once, and each column right of the
// block then receives the block's 16 reflectors in order while it is in cache.
void svd_rows(std::vector<double> &A, int d, int64_t m, std::vector<double> &U,
              std::vector<double> &s) {
  constexpr int kb = 16;
  std::vector<double> R((size_t)d * d, 0.0), vtv(kb);
  std::vector<std::vector<double>> vs(kb);
  // reflector j (slot jl of the block) applied to column cc, rows j..m-1
  auto apply = [&](int j, int jl, double *cc) {
    const double *v = vs[jl].data();
    const double f = 2.0 * dot8(v, cc + j, m - j) / vtv[jl];
    for (int64_t i = j; i < m; ++i) cc[i] -= f * v[i - j];
  };
  for (int j0 = 0; j0 < d; j0 += kb) {
    const int j1 = std::min(d, j0 + kb);
    for (int j = j0; j < j1; ++j) {
      double *cj = &A[(size_t)j * m];
      const double n2 = dot8(cj + j, cj + j, m - j);
      const double alpha = cj[j] >= 0 ? -std::sqrt(n2) : std::sqrt(n2);
      std::vector<double> &v = vs[j - j0];
      v.assign(cj + j, cj + m);
      v[0] -= alpha;
      vtv[j - j0] = dot8(v.data(), v.data(), m - j);
      R[(size_t)j * d + j] = alpha;
      if (vtv[j - j0] == 0.0) continue;
      parallel_for(
          j1 - j - 1,
          [&](int64_t a0, int64_t a1) {
            for (int64_t c = j + 1 + a0; c < j + 1 + a1; ++c) apply(j, j - j0, &A[(size_t)c * m]);
          },
          true);
    }
    // columns right of the block, two at a time so that each pass over a
    // reflector serves both (same arithmetic per column as apply)
    const int64_t npair = (d - j1 + 1) / 2;
    parallel_for(npair, [&](int64_t a0, int64_t a1) {
      for (int64_t q = a0; q < a1; ++q) {
        const int64_t c = j1 + 2 * q;
        double *c0 = &A[(size_t)c * m];
        if (c + 1 >= d) {
          for (int j = j0; j < j1; ++j)
            if (vtv[j - j0] != 0.0) apply(j, j - j0, c0);
          continue;
        }
        double *c1 = c0 + m;
        for (int j = j0; j < j1; ++j) {
          if (vtv[j - j0] == 0.0) continue;
          const double *v = vs[j - j0].data();
          const double f0 = 2.0 * dot8(v, c0 + j, m - j) / vtv[j - j0];
          const double f1 = 2.0 * dot8(v, c1 + j, m - j) / vtv[j - j0];
          for (int64_t i = j; i < m; ++i) {
            c0[i] -= f0 * v[i - j];
            c1[i] -= f1 * v[i - j];
          }
        }
      }
    });
    // row j of R is final once reflector j has reached the columns right of it
    for (int j = j0; j < j1; ++j)
      for (int c = j + 1; c < d; ++c) R[(size_t)j * d + c] = A[(size_t)c * m + j];
  }
  // columns of G = R^T are the rows of R
  jacobi_left(R, d, U, s);
}

// One-sided Jacobi on the d columns of a d x d matrix M, given as the rows of G
// (G[p][i] = M[i][p]; overwritten): M V = U diag(s), s descending, U d x d
// row-major (column p = vector p).  Serial.
void jacobi_left(std::vector<double> &G, int d, std::vector<double> &U, std::vector<double> &s) {
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < d - 1; ++p)
      for (int q = p + 1; q < d; ++q) {
        double *gp = &G[(size_t)p * d], *gq = &G[(size_t)q * d];
        const double a = dot8(gp, gp, d), b = dot8(gq, gq, d), c = dot8(gp, gq, d);
        if (std::fabs(c) <= 1e-15 * std::sqrt(a * b) || c == 0.0) continue;
        rotated = true;
        const double zeta = (b - a) / (2.0 * c);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int i = 0; i < d; ++i) {
          const double x = gp[i], y = gq[i];
          gp[i] = cs * x - sn * y;
          gq[i] = sn * x + cs * y;
        }
      }
    if (!rotated) break;
  }
  std::vector<std::pair<double, int>> order(d);
  for (int p = 0; p < d; ++p) {
    double n2 = 0;
    for (int i = 0; i < d; ++i) n2 += G[(size_t)p * d + i] * G[(size_t)p * d + i];
    order[p] = {std::sqrt(n2), p};
  }
  std::sort(order.begin(), order.end(),
            [](const std::pair<double, int> &x, const std::pair<double, int> &y) {
              return x.first > y.first || (x.first == y.first && x.second < y.second);
            });
  s.resize(d);
  U.assign((size_t)d * d, 0.0);
  for (int k = 0; k < d; ++k) {
    s[k] = order[k].first;
    const double *gp = &G[(size_t)order[k].second * d];
    for (int i = 0; i < d; ++i) U[(size_t)i * d + k] = s[k] > 0 ? gp[i] / s[k] : 0.0;
  }
}

// Rank kept by the two filters of Sec. 4.2 (the larger of the two): the values
// with s_j / s_0 > eps, and the shortest prefix holding 1 - eps of the sum.
int filter_rank(const std::vector<double> &s, double eps) {
  const int n = (int)s.size();
  int r1 = 0;
  for (int j = 0; j < n; ++j)
    if (s[j] / s[0] > eps) r1 = j + 1;
  double tot = 0;
  for (double x : s) tot += x;
  int r2 = n;
  double acc = 0;
  for (int j = 0; j < n; ++j) {
    acc += s[j];
    if (acc / tot >= 1.0 - eps) {
      r2 = j + 1;
      break;
    }
  }
  return std::max(r1, r2);
}

// Q R of the k columns of the r x k matrix A (row-major): modified Gram-Schmidt,
// each column orthogonalised twice; Q r x k row-major, R k x k upper triangular.
void qr_mgs(const std::vector<double> &A, int r, int k, std::vector<double> &Q,
            std::vector<double> &R) {
  Q = A;
  R.assign((size_t)k * k, 0.0);
  for (int j = 0; j < k; ++j) {
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        double dot = 0.0;
        for (int a = 0; a < r; ++a) dot += Q[(size_t)a * k + i] * Q[(size_t)a * k + j];
        R[(size_t)i * k + j] += dot;
        for (int a = 0; a < r; ++a) Q[(size_t)a * k + j] -= dot * Q[(size_t)a * k + i];
      }
    double n2 = 0.0;
    for (int a = 0; a < r; ++a) n2 += Q[(size_t)a * k + j] * Q[(size_t)a * k + j];
    const double nr = std::sqrt(n2);
    R[(size_t)j * k + j] = nr;
    for (int a = 0; a < r; ++a) Q[(size_t)a * k + j] = nr > 0 ? Q[(size_t)a * k + j] / nr : 0.0;
  }
}

// Second compression stage of Sec. 4.2 for one compressed M2L matrix C (r x r,
// row-major): cross approximation with complete pivoting C ~ U V (stopping at
// 1e-13 of max |C|, so it only fixes the numerical rank), QR of U and of V^T, an
// SVD of R_U R_V^T, the two filters with eps, and the kept singular values split
// between the factors: C ~ Ut Vt, Ut = Q_U P_s sqrt(S_s) (r x s),
// Vt = sqrt(S_s) (Q_V Q_s)^T (s x r).  Returns s.
int stage2_factors(const std::vector<double> &C, int r, double eps, std::vector<double> &Ut,
                   std::vector<double> &Vt) {
  std::vector<double> Rm(C), U, V;
  double cmax = 0.0;
  for (double x : C) cmax = std::max(cmax, std::fabs(x));
  int k = 0;
  while (k < r && cmax > 0) {
    int64_t best = 0;
    double bv = -1.0;
    for (int64_t e = 0; e < (int64_t)r * r; ++e)
      if (std::fabs(Rm[e]) > bv) {
        bv = std::fabs(Rm[e]);
        best = e;
      }
    if (bv <= 1e-13 * cmax) break;
    const int p = (int)(best / r), q = (int)(best % r);
    const double piv = Rm[best];
    std::vector<double> u(r), v(r);
    for (int a = 0; a < r; ++a) u[a] = Rm[(size_t)a * r + q];
    for (int b = 0; b < r; ++b) v[b] = Rm[(size_t)p * r + b] / piv;
    for (int a = 0; a < r; ++a)
      for (int b = 0; b < r; ++b) Rm[(size_t)a * r + b] -= u[a] * v[b];
    U.insert(U.end(), u.begin(), u.end());  // column k of U, stored k-major
    V.insert(V.end(), v.begin(), v.end());  // row k of V
    ++k;
  }
  if (k == 0) {
    Ut.clear();
    Vt.clear();
    return 0;
  }
  std::vector<double> Ua((size_t)r * k), Va((size_t)r * k), Qu, Ru, Qv, Rv;
  for (int j = 0; j < k; ++j)
    for (int a = 0; a < r; ++a) {
      Ua[(size_t)a * k + j] = U[(size_t)j * r + a];
      Va[(size_t)a * k + j] = V[(size_t)j * r + a];
    }
  qr_mgs(Ua, r, k, Qu, Ru);
  qr_mgs(Va, r, k, Qv, Rv);
  // M = R_U R_V^T (k x k); its SVD M = P S Qs^T
  std::vector<double> M((size_t)k * k, 0.0);
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      double t = 0.0;
      for (int l = 0; l < k; ++l) t += Ru[(size_t)i * k + l] * Rv[(size_t)j * k + l];
      M[(size_t)i * k + j] = t;
    }
  std::vector<double> G((size_t)k * k), P, sv;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) G[(size_t)j * k + i] = M[(size_t)i * k + j];
  jacobi_left(G, k, P, sv);
  const int so = sv[0] > 0 ? filter_rank(sv, eps) : 0;
  Ut.assign((size_t)r * so, 0.0);
  Vt.assign((size_t)so * r, 0.0);
  for (int a = 0; a < so; ++a) {
    const double h = std::sqrt(sv[a]);
    // Qs column a = M^T P_a / s_a
    std::vector<double> qs(k, 0.0);
    for (int j = 0; j < k; ++j) {
      double t = 0.0;
      for (int i = 0; i < k; ++i) t += M[(size_t)i * k + j] * P[(size_t)i * k + a];
      qs[j] = t / sv[a];
    }
    for (int i = 0; i < r; ++i) {
      double tu = 0.0, tv = 0.0;
      for (int l = 0; l < k; ++l) {
        tu += Qu[(size_t)i * k + l] * P[(size_t)l * k + a];
        tv += Qv[(size_t)i * k + l] * qs[l];
      }
      Ut[(size_t)i * so + a] = tu * h;
      Vt[(size_t)a * r + i] = tv * h;
    }
  }
  return so;
}

}  // namespace

// Row blocks per gathered-GEMM tile for nrb 16-row blocks: the height (3 to 6
// blocks; 3- and 4-block tiles are 128 columns wide, the others 64) that leaves
// the fewest idle blocks in the last row tile, the taller one on a tie.
int pick_rbt(int nrb) {
  int best = 6, waste = 1 << 30;
  for (int rbt = 6; rbt >= 3; --rbt) {
    const int w = (nrb + rbt - 1) / rbt * rbt - nrb;
    if (w < waste) {
      waste = w;
      best = rbt;
    }
  }
  return best;
}

// A <- L^{-1} A for L unit lower triangular (n x n, row-major) and A n x m
// (row-major): forward substitution down the rows, all m columns at once
void lower_unit_solve_rows(const std::vector<double> &Lm, int n, std::vector<double> &A, int m) {
  for (int i = 1; i < n; ++i) {
    double *ai = &A[(size_t)i * m];
    for (int j = 0; j < i; ++j) {
      const double l = Lm[(size_t)i * n + j];
      if (l == 0.0) continue;
      const double *aj = &A[(size_t)j * m];
      for (int c = 0; c < m; ++c) ai[c] -= l * aj[c];
    }
  }
}

int build_tables(Plan &P) {
  auto t0 = std::chrono::steady_clock::now();
  const eifmm_config &c = P.cfg;
  const int depth = c.depth, kind = c.kernel;
  const double p = c.kernel_param, L = c.L;
  const int dmax = c.dmax > 0 ? c.dmax : 1024;
  // absolute stopping rule: the scale of level scale_level (default: the finest)
  double abs_scale = 0, abs_scale2 = 0;
  if (c.tol_mode == 1 && depth >= 2) {
    const int ls = c.scale_level > 0 ? c.scale_level : depth;
    abs_scale = training_scale(kind, p, ls, L, false);
    if (P.two_eim) abs_scale2 = training_scale(kind, p, ls, L, true);
  }
  for (int k = depth; k >= 2; --k) {
    LevelHost &lv = P.lh[k];
    int st = greedy_eim(kind, p, k, L, c.eim_tol, dmax, c.tol_mode == 1 ? abs_scale : 0.0,
                        P.gpu_setup, false, lv);
    if (st != EIFMM_OK) return st;
    crout(kind, p, lv);
    lv.dp = ((lv.d + 15) / 16) * 16;
    if (lv.dp == 0) lv.dp = 16;
    lv.dB = lv.d;
    lv.dpB = lv.dp;
    if (P.two_eim) {
      // the second EIM (Sec. 3.1): its X (J_0) are the local expansions' check
      // points, its Y (I_0) the L2P points, its Delta = M_B^{-1} gives lhat
      LevelHost &lb = P.lhB[k];
      st = greedy_eim(kind, p, k, L, c.eim_tol, dmax, c.tol_mode == 1 ? abs_scale2 : 0.0,
                      P.gpu_setup, true, lb);
      if (st != EIFMM_OK) return st;
      crout(kind, p, lb);
      lb.dp = ((lb.d + 15) / 16) * 16;
      if (lb.dp == 0) lb.dp = 16;
      lv.dB = lb.d;
      lv.dpB = lb.dp;
      lv.XL = lb.Y;
    }
  }
  // translation-invariant M2L matrices K^delta (Sec. 4.2): rows m' (target check
  // points x^{J_0}_m': the second EIM's X, else Y), columns l (source equivalent
  // points Y_l + 2 l_k delta)
  int delta[kNumOffsets][3];
  {
    int id = 0;
    for (int dz = -3; dz <= 3; ++dz)
      for (int dy = -3; dy <= 3; ++dy)
        for (int dx = -3; dx <= 3; ++dx) {
          int m = std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz)));
          if (m < 2) continue;
          delta[id][0] = dx;
          delta[id][1] = dy;
          delta[id][2] = dz;
          ++id;
        }
  }
  for (int k = 2; k <= depth; ++k) {
    LevelHost &lv = P.lh[k];
    const int d = lv.d, dp = lv.dp, dB = lv.dB, dpB = lv.dpB;
    const double *xr = P.two_eim ? P.lhB[k].X.data() : lv.Y.data();  // row points
    const double h = std::ldexp(L, -k);  // box side 2 l_k
    auto kdelta = [&](int o, std::vector<double> &A) {  // dB x d
      const double sx = delta[o][0] * h, sy = delta[o][1] * h, sz = delta[o][2] * h;
      for (int i = 0; i < dB; ++i)
        for (int j = 0; j < d; ++j)
          A[(size_t)i * d + j] = kern_host(kind, p, xr[3 * i] - (lv.Y[3 * j] + sx),
                                           xr[3 * i + 1] - (lv.Y[3 * j + 1] + sy),
                                           xr[3 * i + 2] - (lv.Y[3 * j + 2] + sz));
    };
    lv.r = lv.rp = 0;
    if (c.compress_tol > 0 && d > 0 && dB > 0) {
      // K_fat = [K^delta_1 .. K^delta_316]: row i holds K^delta[i][:] for every delta.
      // With two EIMs the matrices are not symmetric: their common row space comes
      // from K_thin (the matrices stacked), taken as the rows of its transpose,
      // row j holding K^delta[:][j] for every delta
      const int64_t m = (int64_t)kNumOffsets * d, mt = (int64_t)kNumOffsets * dB;
      std::vector<double> Kfat((size_t)dB * m), Kthin(P.two_eim ? (size_t)d * mt : 0);
      parallel_for(kNumOffsets, [&](int64_t o0, int64_t o1) {
        std::vector<double> A((size_t)dB * d);
        for (int64_t o = o0; o < o1; ++o) {
          kdelta((int)o, A);
          for (int i = 0; i < dB; ++i)
            std::memcpy(&Kfat[(size_t)i * m + (size_t)o * d], &A[(size_t)i * d], sizeof(double) * d);
          if (P.two_eim)
            for (int i = 0; i < dB; ++i)
              for (int j = 0; j < d; ++j) Kthin[(size_t)j * mt + (size_t)o * dB + i] = A[(size_t)i * d + j];
        }
      });
      std::vector<double> Ufull, Vfull, sv2;
      svd_rows(Kfat, dB, m, Ufull, lv.sv);
      int fr = filter_rank(lv.sv, c.compress_tol);
      if (P.two_eim) {
        svd_rows(Kthin, d, mt, Vfull, sv2);
        fr = std::max(fr, filter_rank(sv2, c.compress_tol));
      }
      // the rank is the filters' rank; the device tables pad it with zero rows
      // and columns to whole 16-row MFMA blocks (rp), which changes no result
      lv.r = std::min(std::min(d, dB), fr);
      lv.rp = ((lv.r + 15) / 16) * 16;
      lv.U.assign((size_t)dB * lv.r, 0.0);
      for (int i = 0; i < dB; ++i)
        for (int a = 0; a < lv.r; ++a) lv.U[(size_t)i * lv.r + a] = Ufull[(size_t)i * dB + a];
      if (P.two_eim) {
        lv.V.assign((size_t)d * lv.r, 0.0);
        for (int i = 0; i < d; ++i)
          for (int a = 0; a < lv.r; ++a) lv.V[(size_t)i * lv.r + a] = Vfull[(size_t)i * d + a];
      }
      const std::vector<double> &Vb = P.two_eim ? lv.V : lv.U;  // d x r, column side
      // What' = V^T What = (V^T B^{-T}) (Gamma^{-1} W): the factor B^T is folded
      // into the projection (row a is (B^{-1} v_a)^T).  A plan with its own tables
      // and one EIM folds Gamma^{-T} in too (row a is (Gamma^{-T} B^{-1} v_a)^T), so
      // that the projection reads W and the pass takes no solve on this level.  With
      // the expansions the pass forms (smooth sums of the kernel over a box's
      // sources) both forms carry the same rounding: rel-L2 2e-11 folded, 3e-11
      // as solve-then-project, against an 80-bit evaluation, for 1/r at tau 1e-6
      // (Gamma's condition number 6e7), where the 1e-6 target leaves a wide margin.
      lv.fold_what = !P.shared_tables && !P.two_eim && lv.r > 0;
      std::vector<double> Pm((size_t)lv.r * d);
      for (int a = 0; a < lv.r; ++a) {
        double *row = &Pm[(size_t)a * d];
        for (int i = 0; i < d; ++i) row[i] = Vb[(size_t)i * lv.r + a];
        for (int i = 0; i < d; ++i) {  // B row = u_a, B unit lower
          double t = row[i];
          for (int j = 0; j < i; ++j) t -= lv.B[(size_t)i * d + j] * row[j];
          row[i] = t;
        }
        if (lv.fold_what) {
          for (int i = d - 1; i >= 0; --i) {  // Gamma^T row = (B^{-1} v_a), Gamma^T upper
            double t = row[i];
            for (int j = i + 1; j < d; ++j) t -= lv.G[(size_t)j * d + i] * row[j];
            row[i] = t / lv.G[(size_t)i * d + i];
          }
        }
      }
      lv.ufrag.assign((size_t)dpB * lv.rp, 0.0);
      lv.pfrag.assign((size_t)lv.rp * dp, 0.0);
      // the leaf level of a plan with its own tables and one EIM: g = U g' is
      // stored as B^{-1} g = (B^{-1} U) g', so that lhat = Gamma^{-T} (B^{-1} l)
      // takes the solve with Gamma only (B is well conditioned)
      if (k == depth && !P.shared_tables && !P.two_eim) {
        P.fold_leaf = true;
        std::vector<double> Uf(lv.U);
        lower_unit_solve_rows(lv.B, d, Uf, lv.r);
        to_fragments(Uf.data(), dB, lv.r, dpB, lv.rp, lv.ufrag.data());
      } else {
        to_fragments(lv.U.data(), dB, lv.r, dpB, lv.rp, lv.ufrag.data());
      }
      to_fragments(Pm.data(), lv.r, d, lv.rp, dp, lv.pfrag.data());
    }
    const int r = lv.r, rp = lv.rp;
    // rows (g) and columns (What) of the transferred expansions
    const int dmr = r > 0 ? rp : dpB, dmc = r > 0 ? rp : dp;
    lv.kfrag.assign((size_t)kNumOffsets * dmr * dmc, 0.0);
    if (r > 0 && c.compress_tol2 > 0) lv.s2.assign(kNumOffsets, 0);
    std::vector<std::vector<double>> fUt(lv.s2.empty() ? 0 : kNumOffsets),
        fVt(lv.s2.empty() ? 0 : kNumOffsets);
    parallel_for(kNumOffsets, [&](int64_t o0, int64_t o1) {
      std::vector<double> A((size_t)dB * d), KU, C;
      for (int64_t o = o0; o < o1; ++o) {
        kdelta((int)o, A);
        if (r == 0) {
          to_fragments(A.data(), dB, d, dpB, dp, &lv.kfrag[(size_t)o * dpB * dp]);
          continue;
        }
        // C^delta = U^T K^delta V (V = U for a symmetric kernel)
        const std::vector<double> &Vb = P.two_eim ? lv.V : lv.U;
        KU.assign((size_t)dB * r, 0.0);
        for (int i = 0; i < dB; ++i)
          for (int j = 0; j < d; ++j) {
            const double a = A[(size_t)i * d + j];
            const double *vj = &Vb[(size_t)j * r];
            double *ki = &KU[(size_t)i * r];
            for (int b = 0; b < r; ++b) ki[b] += a * vj[b];
          }
        C.assign((size_t)r * r, 0.0);
        for (int i = 0; i < dB; ++i) {
          const double *ui = &lv.U[(size_t)i * r];
          const double *ki = &KU[(size_t)i * r];
          for (int a = 0; a < r; ++a) {
            const double u = ui[a];
            double *ca = &C[(size_t)a * r];
            for (int b = 0; b < r; ++b) ca[b] += u * ki[b];
          }
        }
        if (c.compress_tol2 > 0) {
          // second stage (Sec. 4.2): C^delta ~ Ut Vt, applied as two products by
          // the FP64 pass; the dense product serves the FP32 pass
          std::vector<double> &Ut = fUt[o], &Vt = fVt[o];
          const int so = stage2_factors(C, r, c.compress_tol2, Ut, Vt);
          lv.s2[o] = so;
          for (int i = 0; i < r; ++i)
            for (int b = 0; b < r; ++b) {
              double t = 0.0;
              for (int a2 = 0; a2 < so; ++a2) t += Ut[(size_t)i * so + a2] * Vt[(size_t)a2 * r + b];
              C[(size_t)i * r + b] = t;
            }
        }
        to_fragments(C.data(), r, r, rp, rp, &lv.kfrag[(size_t)o * rp * rp]);
      }
    });
    if (!lv.s2.empty()) {
      // pack the factors in fragment order; a level whose ranks exceed the
      // kernel's bound (kMaxRank2) keeps only the dense product
      int smax = 0;
      for (int o = 0; o < kNumOffsets; ++o) smax = std::max(smax, lv.s2[o]);
      if (smax > kMaxRank2 || rp / 16 < kM2l2RbMin || rp / 16 > kM2l2RbMax) {
        lv.sp2.clear();  // the ranks stay (exported); the product serves the pass
      } else {
        lv.sp2.assign(kNumOffsets, 0);
        lv.voff2.assign(kNumOffsets, 0);
        lv.uoff2.assign(kNumOffsets, 0);
        int64_t tot = 0;
        for (int o = 0; o < kNumOffsets; ++o) {
          lv.sp2[o] = ((lv.s2[o] + 15) / 16) * 16;
          lv.voff2[o] = lv.uoff2[o] = tot;
          tot += (int64_t)lv.sp2[o] * rp;
        }
        lv.vf2.assign((size_t)std::max<int64_t>(tot, 1), 0.0);
        lv.uf2.assign((size_t)std::max<int64_t>(tot, 1), 0.0);
        for (int o = 0; o < kNumOffsets; ++o) {
          const int so = lv.s2[o], sp = lv.sp2[o];
          if (sp == 0) continue;
          to_fragments(fVt[o].data(), so, r, sp, rp, &lv.vf2[lv.voff2[o]]);
          to_fragments_nat(fUt[o].data(), r, so, rp, sp, &lv.uf2[lv.uoff2[o]]);
        }
      }
    }
    trsm_table(lv.G, d, dp, false, true, lv.tri[0]);   // Gamma    (forward, Delta)
    trsm_table(lv.B, d, dp, true, false, lv.tri[1]);   // B^T      (backward, Delta)
    if (P.two_eim) {  // lhat = Delta^{J_0,I_0} l = M_B^{-1} l: the second EIM's factors
      const LevelHost &lb = P.lhB[k];
      trsm_table(lb.G, dB, dpB, false, true, lv.tri[2]);  // Gamma_B  (forward)
      trsm_table(lb.B, dB, dpB, true, false, lv.tri[3]);  // B_B^T    (backward)
    } else {
      trsm_table(lv.B, d, dp, false, true, lv.tri[2]);   // B        (forward, Delta^T)
      trsm_table(lv.G, d, dp, true, false, lv.tri[3]);   // Gamma^T  (backward, Delta^T)
    }
  }
  // M2M (Sec. 4.1): for parent level k and child i with c_C - c_P = s_i,
  //   M2M_i = K(X^k - s_i, Y^{k+1}) (M^{k+1})^{-1}        (d_k x d_{k+1})
  // L2L: L2L_i = K(x^{J_0,k+1} + s_i, y^{I_0,k}) Delta^{J_0,I_0,k}, with the second
  // EIM's points and M_B^{-1}; one EIM: K(Y^{k+1} + s_i, X^k) (M^k)^{-T}
  for (int k = 2; k < depth; ++k) {
    LevelHost &lp = P.lh[k], &lc = P.lh[k + 1];
    const int dk = lp.d, dc = lc.d, dkB = lp.dB, dcB = lc.dB;
    const double *xbc = P.two_eim ? P.lhB[k + 1].X.data() : lc.Y.data();
    const double *ybp = P.two_eim ? P.lhB[k].Y.data() : lp.X.data();
    const double lc_half = std::ldexp(L, -k - 2);  // l_{k+1}
    // device solves: the kernel rows only, padded; the solves and the packing
    // follow once the solve tables are on the device
    const bool dev = P.gpu_ops;
    if (dev) {
      lp.m2m_rows.assign((size_t)8 * dk * lc.dp, 0.0);
      lp.l2l_rows.assign((size_t)8 * dcB * lp.dpB, 0.0);
      if (P.two_eim) {
        trsm_table(lc.B, dc, lc.dp, false, true, lp.op_tri[0]);                // B      (forward)
        trsm_table(lc.G, dc, lc.dp, true, false, lp.op_tri[1]);                // Gamma^T (backward)
        trsm_table(P.lhB[k].B, dkB, lp.dpB, false, true, lp.op_tri[2]);      // B_B
        trsm_table(P.lhB[k].G, dkB, lp.dpB, true, false, lp.op_tri[3]);      // Gamma_B^T
      }
    } else {
      lp.m2m.assign((size_t)8 * lp.dp * lc.dp, 0.0);
      lp.l2l.assign((size_t)8 * lc.dpB * lp.dpB, 0.0);
    }
    parallel_for(8, [&](int64_t i0, int64_t i1) {
      std::vector<double> A((size_t)dk * dc), Bm((size_t)dcB * dkB), row;
      for (int64_t i = i0; i < i1; ++i) {
        double s[3];
        for (int a = 0; a < 3; ++a) s[a] = ((i >> a) & 1) ? lc_half : -lc_half;
        for (int m = 0; m < dk; ++m) {
          row.assign((size_t)dc, 0.0);
          for (int q = 0; q < dc; ++q)
            row[q] = kern_host(kind, p, (lp.X[3 * m] - s[0]) - lc.Y[3 * q],
                               (lp.X[3 * m + 1] - s[1]) - lc.Y[3 * q + 1],
                               (lp.X[3 * m + 2] - s[2]) - lc.Y[3 * q + 2]);
          if (dev) {
            std::memcpy(&lp.m2m_rows[((size_t)i * dk + m) * lc.dp], row.data(), sizeof(double) * dc);
            continue;
          }
          solve_mtinv(lc, row.data());  // row M^{-1} = (M^{-T} row^T)^T
          std::memcpy(&A[(size_t)m * dc], row.data(), sizeof(double) * dc);
        }
        if (!dev)
          to_fragments(A.data(), dk, dc, lp.dp, lc.dp, &lp.m2m[(size_t)i * lp.dp * lc.dp]);
        for (int m = 0; m < dcB; ++m) {
          row.assign((size_t)dkB, 0.0);
          for (int q = 0; q < dkB; ++q)
            row[q] = kern_host(kind, p, (xbc[3 * m] + s[0]) - ybp[3 * q],
                               (xbc[3 * m + 1] + s[1]) - ybp[3 * q + 1],
                               (xbc[3 * m + 2] + s[2]) - ybp[3 * q + 2]);
          if (dev) {
            std::memcpy(&lp.l2l_rows[((size_t)i * dcB + m) * lp.dpB], row.data(),
                        sizeof(double) * dkB);
            continue;
          }
          if (P.two_eim)
            solve_mtinv(P.lhB[k], row.data());  // row M_B^{-1} = (M_B^{-T} row^T)^T
          else
            solve_minv(lp, row.data());  // row M^{-T} = (M^{-1} row^T)^T
          std::memcpy(&Bm[(size_t)m * dkB], row.data(), sizeof(double) * dkB);
        }
        if (!dev) {
          if (P.fold_leaf && k + 1 == depth) lower_unit_solve_rows(lc.B, dc, Bm, dkB);
          to_fragments(Bm.data(), dcB, dkB, lc.dpB, lp.dpB,
                       &lp.l2l[(size_t)i * lc.dpB * lp.dpB]);
        }
      }
    });
  }
  P.setup_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return EIFMM_OK;
}

void pack_operators(Plan &P, int k) {
  LevelHost &lp = P.lh[k], &lc = P.lh[k + 1];
  const int dk = lp.d, dc = lc.d, dkB = lp.dB, dcB = lc.dB;
  lp.m2m.assign((size_t)8 * lp.dp * lc.dp, 0.0);
  lp.l2l.assign((size_t)8 * lc.dpB * lp.dpB, 0.0);
  parallel_for(8, [&](int64_t i0, int64_t i1) {
    std::vector<double> A((size_t)dk * dc), Bm((size_t)dcB * dkB);
    for (int64_t i = i0; i < i1; ++i) {
      for (int m = 0; m < dk; ++m)
        std::memcpy(&A[(size_t)m * dc], &lp.m2m_rows[((size_t)i * dk + m) * lc.dp],
                    sizeof(double) * dc);
      to_fragments(A.data(), dk, dc, lp.dp, lc.dp, &lp.m2m[(size_t)i * lp.dp * lc.dp]);
      for (int m = 0; m < dcB; ++m)
        std::memcpy(&Bm[(size_t)m * dkB], &lp.l2l_rows[((size_t)i * dcB + m) * lp.dpB],
                    sizeof(double) * dkB);
      if (P.fold_leaf && k + 1 == P.depth) lower_unit_solve_rows(lc.B, dc, Bm, dkB);
      to_fragments(Bm.data(), dcB, dkB, lc.dpB, lp.dpB, &lp.l2l[(size_t)i * lc.dpB * lp.dpB]);
    }
  });
  std::vector<double>().swap(lp.m2m_rows);
  std::vector<double>().swap(lp.l2l_rows);
  for (auto &t : lp.op_tri) std::vector<double>().swap(t);
}

}  // namespace eifmm
