// The sparsifying Cartesian preconditioner S^(C) = (C^(C))^-1 A of the paper's Section 4
// (subsection "Sparsifying preconditioner", eqs. LS_eq_on_cartesian_points, cart_neighbors_LS,
// sparsifying_min, LC_def, S_minus_I), built per scatterer on its transfer grid.
//
// Cartesian system: L^(C) = I + k^2 V^(C) M^(C) on the grid nodes z_j, with M^(C) = diag(m(z_j)).
// V^(C) is the first-order rule (the paper's Duan-Rokhlin corrections are cited, not given):
// h^2 G(z_i, z_j) off the diagonal, and on it the integral of G over the disk of the cell's area,
// (-1 + (i pi / 2) k a H1(k a)) / k^2 with a = h / sqrt(pi).
//
// Construction (host, at setup):
//   * A: row j's weights are the unit vector v on its 3 x 3 neighbourhood N(j) within the grid
//     that minimises || v V(N(j), N(j)^c) || (eq. sparsifying_min): the left singular vector of
//     the smallest singular value.  The complement block is reduced to a square triangular
//     factor by Givens rotations row by row (QR of its transpose), whose left singular vectors
//     are those of the block; a one-sided Jacobi SVD of that small factor gives them.  Rows
//     with all 9 neighbours take the grid's central node's weights (translation invariance);
//     every edge and corner row solves its own problem (mirror-image rows share theirs).
//   * C^(C) = A L^(C) kept on the 3 x 3 pattern (eq. LC_def): 9 entries per row, from V^(C) at
//     the offsets of at most two steps.
//   * Block LU of C^(C) with grid rows as blocks (block tridiagonal, each block tridiagonal):
//     Sigma_0 = D_0, Sigma_i = D_i - L_i Sigma_{i-1}^-1 U_{i-1}; G_i = Sigma_i^-1 is kept dense
//     (Gauss-Jordan with partial pivoting inside a block, none across blocks).  A seeded
//     right-hand side solved through the factors reports ||C x - y|| / ||y||.
//
// Application (device): S c = C^-1 (A c): a 9-point stencil kernel and a block sweep kernel
// (one workgroup per right-hand side, the grid rows in order, one dense block product per row
// and direction).  S^H c = A^H (C^-H c) uses the same factors (C^H = U~^H L~^H).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <functional>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "host.h"
#include "internal.h"

namespace lsk {

namespace {

typedef std::complex<double> cplx;

constexpr int kBlock = 256;
constexpr int kMaxNx = 1536;   // grid row length the sweep kernel's LDS vectors hold (R = 1)

// stencil slot o = (dy + 1) * 3 + (dx + 1)
__device__ __host__ inline int slot(int dx, int dy) { return (dy + 1) * 3 + (dx + 1); }
__device__ __host__ inline int slot_dx(int o) { return o % 3 - 1; }
__device__ __host__ inline int slot_dy(int o) { return o / 3 - 1; }

// ---------------------------------------------------------------------------------------------
// host construction

// V^(C) between grid nodes (dx, dy) steps apart, |dx| < nx, |dy| < ny (translation invariant).
struct VTable {
  int nx = 0, ny = 0;
  std::vector<cplx> v;   // [|dy|][|dx|]
  cplx at(int dx, int dy) const { return v[(size_t)std::abs(dy) * nx + std::abs(dx)]; }
};

VTable cartesian_table(int nx, int ny, double h, double k) {
  VTable t;
  t.nx = nx;
  t.ny = ny;
  const size_t n = (size_t)nx * ny;
  std::vector<double> z2(n), g(2 * n);
  const double kh2 = (k * h) * (k * h);
  for (int dy = 0; dy < ny; ++dy)
    for (int dx = 0; dx < nx; ++dx) {
      const double d2 = (double)dx * dx + (double)dy * dy;
      z2[(size_t)dy * nx + dx] = kh2 * (d2 > 0 ? d2 : 1.0);
    }
  eval_green_host(z2.data(), g.data(), (int64_t)n);
  t.v.resize(n);
  for (size_t i = 0; i < n; ++i) t.v[i] = h * h * cplx(g[2 * i], g[2 * i + 1]);
  // the cell's own term: G integrated over the disk of area h^2 centred on the node
  const double a = h / std::sqrt(M_PI);
  const cplx h1(::j1(k * a), ::y1(k * a));
  t.v[0] = (-1.0 + cplx(0.0, 0.5 * M_PI) * (k * a) * h1) / (k * k);
  return t;
}

// Left singular vector of the smallest singular value of the m x m matrix A (column-major,
// a[c * m + r]), by one-sided Jacobi on its columns: A W = U Sigma.  Returns the unit vector and
// writes smallest / largest singular value to ratio.
std::vector<cplx> smallest_left_singular(std::vector<cplx> a, int m, double *ratio) {
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        cplx *ap = &a[(size_t)p * m], *aq = &a[(size_t)q * m];
        double al = 0, be = 0;
        cplx ga = 0;
        for (int r = 0; r < m; ++r) {
          al += std::norm(ap[r]);
          be += std::norm(aq[r]);
          ga += std::conj(ap[r]) * aq[r];
        }
        const double gm = std::abs(ga);
        if (!(gm > 1e-15 * std::sqrt(al * be))) continue;
        rotated = true;
        const cplx ph = ga / gm;   // rotate a_q by conj(ph) so that a_p^H a_q = |gamma|
        const double zeta = (be - al) / (2 * gm);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
        const double c = 1 / std::sqrt(1 + t * t), s = c * t;
        for (int r = 0; r < m; ++r) {
          const cplx x = ap[r], y = aq[r] * std::conj(ph);
          ap[r] = c * x - s * y;
          aq[r] = s * x + c * y;
        }
      }
    if (!rotated) break;
  }
  int imin = 0, imax = 0;
  std::vector<double> nrm(m);
  for (int p = 0; p < m; ++p) {
    double s2 = 0;
    for (int r = 0; r < m; ++r) s2 += std::norm(a[(size_t)p * m + r]);
    nrm[p] = std::sqrt(s2);
    if (nrm[p] < nrm[imin]) imin = p;
    if (nrm[p] > nrm[imax]) imax = p;
  }
  std::vector<cplx> u(m);
  for (int r = 0; r < m; ++r) u[r] = a[(size_t)imin * m + r] / nrm[imin];
  if (ratio) *ratio = nrm[imax] > 0 ? nrm[imin] / nrm[imax] : 0.0;
  return u;
}

// Row j = (ix, iy)'s weights (eq. sparsifying_min) on its neighbours within the grid: 9 slots,
// zero where a neighbour is off the grid.
std::vector<cplx> row_weights(const VTable &V, int ix, int iy, double *ratio) {
  const int nx = V.nx, ny = V.ny;
  int have[9], m = 0;
  for (int o = 0; o < 9; ++o) {
    const int x = ix + slot_dx(o), y = iy + slot_dy(o);
    if (x >= 0 && x < nx && y >= 0 && y < ny) have[m++] = o;
  }
  // R: upper triangular m x m factor of B^T, B = V(N(j), N(j)^c), fed one complement node at a
  // time (row a_l = V(n_a, l) of B^T) and rotated in by Givens rotations
  std::vector<cplx> R((size_t)m * m, cplx(0));   // row-major R[i * m + c]
  std::vector<cplx> row(m);
  for (int ly = 0; ly < ny; ++ly)
    for (int lx = 0; lx < nx; ++lx) {
      if (std::abs(lx - ix) <= 1 && std::abs(ly - iy) <= 1) continue;   // in N(j)
      for (int a = 0; a < m; ++a) row[a] = V.at(lx - (ix + slot_dx(have[a])), ly - (iy + slot_dy(have[a])));
      for (int i = 0; i < m; ++i) {
        const cplx a = R[(size_t)i * m + i], b = row[i];
        if (b == cplx(0)) continue;
        const double aa = std::abs(a), r = std::hypot(aa, std::abs(b));
        double c;
        cplx s;
        if (aa == 0) {
          c = 0;
          s = std::conj(b) / std::abs(b);
        } else {
          c = aa / r;
          s = (a / aa) * std::conj(b) / r;
        }
        for (int cc = i; cc < m; ++cc) {
          const cplx x = R[(size_t)i * m + cc], y = row[cc];
          R[(size_t)i * m + cc] = c * x + s * y;
          row[cc] = -std::conj(s) * x + c * y;
        }
      }
    }
  // B = R^T Q^T: the left singular vectors of B are those of R^T; column-major R^T is row-major R
  std::vector<cplx> u = smallest_left_singular(R, m, ratio);
  std::vector<cplx> w(9, cplx(0));
  for (int a = 0; a < m; ++a) w[have[a]] = std::conj(u[a]);
  return w;
}

void parallel_for(int n, int threads, const std::function<void(int)> &f);

}  // namespace

// W[j * 9 + o] = A[j, j + off(o)], E[j * 9 + o] = C^(C)[j, j + off(o)] (0 off the grid).
void sparsify_stencil(int nx, int ny, double h, double k, const cplx *m, int threads, std::vector<cplx> &W,
                      std::vector<cplx> &E, double *ratio) {
  const VTable V = cartesian_table(nx, ny, h, k);
  const size_t nc = (size_t)nx * ny;
  W.assign(nc * 9, cplx(0));
  E.assign(nc * 9, cplx(0));
  const std::vector<cplx> wc = row_weights(V, nx / 2, ny / 2, ratio);
  // boundary rows: by the grid's mirror symmetries only those with ix <= (nx-1)/2 and
  // iy <= (ny-1)/2 are solved; the mirror images take the reflected weights
  std::vector<std::pair<int, int>> todo;
  for (int iy = 0; iy <= (ny - 1) / 2; ++iy)
    for (int ix = 0; ix <= (nx - 1) / 2; ++ix)
      if (ix == 0 || iy == 0) todo.push_back({ix, iy});
  std::vector<std::vector<cplx>> wb(todo.size());
  parallel_for((int)todo.size(), threads, [&](int t) { wb[t] = row_weights(V, todo[t].first, todo[t].second, nullptr); });
  for (size_t j = 0; j < nc; ++j)
    for (int o = 0; o < 9; ++o) W[j * 9 + o] = wc[o];
  for (size_t t = 0; t < todo.size(); ++t) {
    const int ix = todo[t].first, iy = todo[t].second;
    for (int fy = 0; fy < 2; ++fy)
      for (int fx = 0; fx < 2; ++fx) {
        const int x = fx ? nx - 1 - ix : ix, y = fy ? ny - 1 - iy : iy;
        const size_t j = (size_t)y * nx + x;
        for (int o = 0; o < 9; ++o) {
          const int dx = slot_dx(o), dy = slot_dy(o);
          W[j * 9 + slot(fx ? -dx : dx, fy ? -dy : dy)] = wb[t][o];
        }
      }
  }
  // interior weights truncated nowhere; slots off the grid are zero
  for (int iy = 0; iy < ny; ++iy)
    for (int ix = 0; ix < nx; ++ix)
      for (int o = 0; o < 9; ++o) {
        const int x = ix + slot_dx(o), y = iy + slot_dy(o);
        if (x < 0 || x >= nx || y < 0 || y >= ny) W[((size_t)iy * nx + ix) * 9 + o] = 0;
      }
  // C^(C)[j, j2] = sum_o A[j, l] L^(C)[l, j2], l = j + off(o), j2 = j + off(o2),
  // L^(C)[l, j2] = [l == j2] + k^2 V^(C)(z_l - z_j2) m(z_j2)
  const double k2 = k * k;
  for (int iy = 0; iy < ny; ++iy)
    for (int ix = 0; ix < nx; ++ix) {
      const size_t j = (size_t)iy * nx + ix;
      for (int o2 = 0; o2 < 9; ++o2) {
        const int x2 = ix + slot_dx(o2), y2 = iy + slot_dy(o2);
        if (x2 < 0 || x2 >= nx || y2 < 0 || y2 >= ny) continue;
        const cplx mj2 = m[(size_t)y2 * nx + x2];
        cplx acc = 0;
        for (int o = 0; o < 9; ++o) {
          const cplx w = W[j * 9 + o];
          if (w == cplx(0)) continue;
          const int dx = slot_dx(o) - slot_dx(o2), dy = slot_dy(o) - slot_dy(o2);
          const cplx l = (o == o2 ? 1.0 : 0.0) + k2 * V.at(dx, dy) * mj2;
          acc += w * l;
        }
        E[j * 9 + o2] = acc;
      }
    }
}

namespace {

void parallel_for(int n, int threads, const std::function<void(int)> &f) {
  threads = std::max(1, std::min(threads, n));
  if (threads == 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&, t] {
      for (int i = t; i < n; i += threads) f(i);
    });
  for (auto &th : pool) th.join();
}

// Entry of the tridiagonal block (i, i + dy) of C^(C) at (r, r + dx).
inline cplx eblk(const std::vector<cplx> &E, int nx, int i, int r, int dx, int dy) {
  return E[((size_t)i * nx + r) * 9 + slot(dx, dy)];
}

}  // namespace

// A reusable barrier for the factorization's worker threads (spinning: the waits are a few
// microseconds, one per pivot).
struct SpinBarrier {
  explicit SpinBarrier(int n) : n_(n) {}
  void wait() {
    const int g = gen_.load(std::memory_order_acquire);
    if (count_.fetch_add(1, std::memory_order_acq_rel) + 1 == n_) {
      count_.store(0, std::memory_order_relaxed);
      gen_.fetch_add(1, std::memory_order_acq_rel);
    } else {
      while (gen_.load(std::memory_order_acquire) == g) std::this_thread::yield();
    }
  }
  int n_;
  std::atomic<int> count_{0}, gen_{0};
};

// Block LU of C^(C): G[i] = Sigma_i^-1 (row-major, nx x nx each), with `threads` host threads
// sharing each block's work by rows (the blocks themselves are sequential).  Gauss-Jordan with
// partial pivoting inside a block.  Returns false if a block is singular.
bool sparsify_factor(int nx, int ny, const std::vector<cplx> &E, std::vector<std::vector<cplx>> &G, int threads) {
  const size_t n2 = (size_t)nx * nx;
  G.assign(ny, std::vector<cplx>(n2));
  threads = std::max(1, std::min(threads, std::max(1, nx / 8)));
  std::vector<cplx> S(n2), T(n2);
  std::vector<int> piv(nx);
  std::atomic<bool> singular{false};
  SpinBarrier bar(threads);
  auto work = [&](int tid) {
    const int r0 = (int)((int64_t)nx * tid / threads), r1 = (int)((int64_t)nx * (tid + 1) / threads);
    for (int i = 0; i < ny; ++i) {
      // S = D_i - L_i G_{i-1} U_{i-1}, rows [r0, r1)
      for (int r = r0; r < r1; ++r) {
        cplx *sr = &S[(size_t)r * nx];
        std::fill(sr, sr + nx, cplx(0));
        for (int dx = -1; dx <= 1; ++dx)
          if (r + dx >= 0 && r + dx < nx) sr[r + dx] = eblk(E, nx, i, r, dx, 0);
      }
      if (i > 0) {
        // T = G_{i-1} U_{i-1}, U_{i-1}[q][q + dx] = C[(i-1, q), (i, q + dx)]
        const std::vector<cplx> &Gp = G[i - 1];
        for (int r = r0; r < r1; ++r)
          for (int c = 0; c < nx; ++c) {
            cplx acc = 0;
            for (int dx = -1; dx <= 1; ++dx) {
              const int q = c - dx;
              if (q >= 0 && q < nx) acc += Gp[(size_t)r * nx + q] * eblk(E, nx, i - 1, q, dx, 1);
            }
            T[(size_t)r * nx + c] = acc;
          }
        bar.wait();
        // S -= L_i T, L_i[r][r + dx] = C[(i, r), (i-1, r + dx)]
        for (int r = r0; r < r1; ++r)
          for (int dx = -1; dx <= 1; ++dx) {
            const int q = r + dx;
            if (q < 0 || q >= nx) continue;
            const cplx l = eblk(E, nx, i, r, dx, -1);
            if (l == cplx(0)) continue;
            cplx *sr = &S[(size_t)r * nx];
            const cplx *tq = &T[(size_t)q * nx];
            for (int c = 0; c < nx; ++c) sr[c] -= l * tq[c];
          }
      }
      bar.wait();
      // Gauss-Jordan: thread 0 picks and normalises the pivot row, every thread eliminates the
      // column from its own rows
      for (int c = 0; c < nx; ++c) {
        if (tid == 0) {
          int p = c;
          double best = std::abs(S[(size_t)c * nx + c]);
          for (int r = c + 1; r < nx; ++r)
            if (std::abs(S[(size_t)r * nx + c]) > best) {
              best = std::abs(S[(size_t)r * nx + c]);
              p = r;
            }
          if (!(best > 0)) {
            singular = true;
          } else {
            piv[c] = p;
            if (p != c)
              for (int q = 0; q < nx; ++q) std::swap(S[(size_t)c * nx + q], S[(size_t)p * nx + q]);
            cplx *rc = &S[(size_t)c * nx];
            const cplx inv = 1.0 / rc[c];
            rc[c] = 1.0;
            for (int q = 0; q < nx; ++q) rc[q] *= inv;
          }
        }
        bar.wait();
        if (singular) return;
        const cplx *rc = &S[(size_t)c * nx];
        for (int r = r0; r < r1; ++r) {
          if (r == c) continue;
          cplx *rr = &S[(size_t)r * nx];
          const cplx f = rr[c];
          if (f == cplx(0)) continue;
          rr[c] = 0.0;
          for (int q = 0; q < nx; ++q) rr[q] -= f * rc[q];
        }
        bar.wait();
      }
      // undo the row interchanges as column interchanges (last first), row by row, into G_i
      std::vector<cplx> &Gi = G[i];
      for (int r = r0; r < r1; ++r) {
        cplx *sr = &S[(size_t)r * nx];
        for (int c = nx - 1; c >= 0; --c)
          if (piv[c] != c) std::swap(sr[c], sr[piv[c]]);
        std::copy(sr, sr + nx, &Gi[(size_t)r * nx]);
      }
      bar.wait();
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto &th : pool) th.join();
  return !singular;
}

// x = C^-1 y through the factors on the host (the sweeps the device kernel performs).
void sparsify_solve_host(int nx, int ny, const std::vector<cplx> &E, const std::vector<std::vector<cplx>> &G,
                         const cplx *y, cplx *x) {
  std::vector<cplx> z(nx), t(nx);
  // forward: z_i = y_i - L_i w_{i-1}, w_i = G_i z_i (into x)
  for (int i = 0; i < ny; ++i) {
    for (int r = 0; r < nx; ++r) {
      cplx v = y[(size_t)i * nx + r];
      if (i > 0)
        for (int dx = -1; dx <= 1; ++dx)
          if (r + dx >= 0 && r + dx < nx) v -= eblk(E, nx, i, r, dx, -1) * x[(size_t)(i - 1) * nx + r + dx];
      z[r] = v;
    }
    for (int r = 0; r < nx; ++r) {
      cplx acc = 0;
      for (int c = 0; c < nx; ++c) acc += G[i][(size_t)r * nx + c] * z[c];
      x[(size_t)i * nx + r] = acc;
    }
  }
  // backward: x_i = w_i - G_i (U_i x_{i+1})
  for (int i = ny - 2; i >= 0; --i) {
    for (int r = 0; r < nx; ++r) {
      cplx v = 0;
      for (int dx = -1; dx <= 1; ++dx)
        if (r + dx >= 0 && r + dx < nx) v += eblk(E, nx, i, r, dx, 1) * x[(size_t)(i + 1) * nx + r + dx];
      t[r] = v;
    }
    for (int r = 0; r < nx; ++r) {
      cplx acc = 0;
      for (int c = 0; c < nx; ++c) acc += G[i][(size_t)r * nx + c] * t[c];
      x[(size_t)i * nx + r] -= acc;
    }
  }
}

// ---------------------------------------------------------------------------------------------
// device kernels

namespace {

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(std::fma(a.x, b.x, -a.y * b.y), std::fma(a.x, b.y, a.y * b.x));
}
__device__ inline double2 cmulc(double2 a, double2 b) {   // conj(a) b
  return make_double2(std::fma(a.x, b.x, a.y * b.y), std::fma(a.x, b.y, -a.y * b.x));
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// out[c][j] = (A c)[j] = sum_o W[o][j] in[c][j + off(o)], or with adjoint
// out[c][l] = (A^H c)[l] = sum_o conj(W[o][l - off(o)]) in[c][l - off(o)]; then multiplied by
// oscale[j] when given.  W is [9][nc] (slots off the grid hold zero).  grid (ceil(nc / kBlock), nrhs)
__global__ __launch_bounds__(kBlock) void stencil_kernel(int nx, int ny, const double2 *__restrict__ W,
                                                         const double2 *__restrict__ in, int64_t ldi,
                                                         double2 *__restrict__ out, int64_t ldo, int adjoint,
                                                         const double *__restrict__ oscale) {
  const int64_t nc = (int64_t)nx * ny;
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= nc) return;
  const int iy = (int)(j / nx), ix = (int)(j - (int64_t)iy * nx);
  const double2 *ic = in + (int64_t)blockIdx.y * ldi;
  double2 acc = make_double2(0.0, 0.0);
#pragma unroll
  for (int o = 0; o < 9; ++o) {
    const int dx = slot_dx(o), dy = slot_dy(o);
    if (!adjoint) {
      const int x = ix + dx, y = iy + dy;
      if (x >= 0 && x < nx && y >= 0 && y < ny) acc = cadd(acc, cmul(W[o * nc + j], ic[(int64_t)y * nx + x]));
    } else {
      const int x = ix - dx, y = iy - dy;
      if (x >= 0 && x < nx && y >= 0 && y < ny) {
        const int64_t r = (int64_t)y * nx + x;
        acc = cadd(acc, cmulc(W[o * nc + r], ic[r]));
      }
    }
  }
  if (oscale) {
    const double s = oscale[j];
    acc = make_double2(acc.x * s, acc.y * s);
  }
  out[(int64_t)blockIdx.y * ldo + j] = acc;
}

// x = C^-1 y (adjoint = 0) or x = C^-H y (adjoint = 1) through the block factors.  A workgroup
// serves R consecutive right-hand sides (c0 = blockIdx.x R); each (grid-row entry r, right-hand
// side k) pair has P threads that split the dense block product's columns (thread t: part
// t / (nx R), pair t mod (nx R), consecutive pairs in consecutive lanes for coalesced factor
// loads), so each thread's chain of dependent loads is nx / P long.  y may equal x.  E is
// [9][nc] (C^(C)'s stencil entries), Gc the blocks G_i column-major (element (r, c) at c nx + r),
// Gr the same blocks row-major.  With iscale, the input is read as iscale[j] y[j].
//   C^-1: forward  z_i = y_i - L_i w_{i-1}, w_i = G_i z_i;  backward x_i = w_i - G_i (U_i x_{i+1})
//   C^-H: forward  z_i = G_i^H (y_i - U_{i-1}^H z_{i-1});   backward x_i = z_i - G_i^H (L_{i+1}^H x_{i+1})
// with L_i = block (i, i - 1), U_i = block (i, i + 1), each tridiagonal.  LDS vectors are stored
// pair-major ([r][R]).
constexpr int kSweepBlock = 1024;
constexpr int kSweepLds = 1536;   // R nx <= kSweepLds complex values per LDS vector
__global__ __launch_bounds__(kSweepBlock) void block_sweep_kernel(int nx, int ny, int R, int P, int nrhs,
                                                                  const double2 *__restrict__ E,
                                                                  const double2 *__restrict__ Gc,
                                                                  const double2 *__restrict__ Gr, const double2 *y,
                                                                  int64_t ldy, double2 *x, int64_t ldx, int adjoint,
                                                                  const double *__restrict__ iscale) {
  // va: the previous row's result, and during a dense product its partial sums [part][pair] (the
  // product does not read va; each pair's sum reads its own slots before it writes slot 0 again);
  // vb: the current operand
  __shared__ double2 va[kSweepLds], vb[kSweepLds];
  const int64_t nc = (int64_t)nx * ny;
  const int c0 = blockIdx.x * R;
  const int nloc = min(R, nrhs - c0);
  const int64_t n2 = (int64_t)nx * nx;
  const int work = nx * R;
  const int chunk = (nx + P - 1) / P;
  const int t = threadIdx.x;
  // tridiagonal product of block (bi, bi + dy) (or its conjugate transpose) with va, entry r
  auto tri = [&](int bi, int dy, int r, int k, bool conjt) {
    double2 acc = make_double2(0.0, 0.0);
    for (int dx = -1; dx <= 1; ++dx) {
      if (!conjt) {
        const int q = r + dx;
        if (q >= 0 && q < nx) acc = cadd(acc, cmul(E[slot(dx, dy) * nc + (int64_t)bi * nx + r], va[q * R + k]));
      } else {
        // (B^H v)[r] = sum_q conj(B[q][r]) v[q], B[q][q + dx] nonzero: q = r - dx
        const int q = r - dx;
        if (q >= 0 && q < nx) acc = cadd(acc, cmulc(E[slot(dx, dy) * nc + (int64_t)bi * nx + q], va[q * R + k]));
      }
    }
    return acc;
  };
  // one part of the dense product of block i (or its conjugate transpose) with vb for pair
  // (r_me, k_me): columns [cb, ce), loads issued eight at a time
  auto dense_part = [&](int i, bool conjt, int r_me, int k_me, int cb, int ce) {
    double2 a0 = make_double2(0.0, 0.0), a1 = make_double2(0.0, 0.0);
    const double2 *g = (conjt ? Gr : Gc) + (int64_t)i * n2 + r_me;   // G[r][c] (or G[c][r]) at c nx + r
    int c = cb;
    for (; c + 8 <= ce; c += 8) {
      double2 gv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) gv[u] = g[(int64_t)(c + u) * nx];
#pragma unroll
      for (int u = 0; u < 8; u += 2) {
        const double2 v0 = vb[(c + u) * R + k_me], v1 = vb[(c + u + 1) * R + k_me];
        a0 = cadd(a0, conjt ? cmulc(gv[u], v0) : cmul(gv[u], v0));
        a1 = cadd(a1, conjt ? cmulc(gv[u + 1], v1) : cmul(gv[u + 1], v1));
      }
    }
    for (; c < ce; ++c) {
      const double2 gv = g[(int64_t)c * nx], v = vb[c * R + k_me];
      a0 = cadd(a0, conjt ? cmulc(gv, v) : cmul(gv, v));
    }
    return cadd(a0, a1);
  };
  // every (part, pair) of the dense product, partial sums into va
  auto dense_all = [&](int i, bool conjt) {
    for (int p = t; p < P * work; p += kSweepBlock) {
      const int part = p / work, pr = p - part * work;
      const int r = pr / R, k = pr - r * R;
      if (k >= nloc) continue;
      const int cb = part * chunk, ce = min(nx, cb + chunk);
      va[p] = dense_part(i, conjt, r, k, cb, ce);
    }
  };
  auto summed = [&](int p0) {
    double2 w = va[p0];
    for (int q = 1; q < P; ++q) w = cadd(w, va[q * work + p0]);
    return w;
  };
  auto yin = [&](int k, int64_t j) {
    double2 v = y[(int64_t)(c0 + k) * ldy + j];
    if (iscale) v = make_double2(v.x * iscale[j], v.y * iscale[j]);
    return v;
  };
  const bool conjt = adjoint != 0;
  // forward sweep
  for (int i = 0; i < ny; ++i) {
    for (int p0 = t; p0 < work; p0 += kSweepBlock) {
      const int r = p0 / R, k = p0 - r * R;
      if (k >= nloc) continue;
      double2 v = yin(k, (int64_t)i * nx + r);
      if (i > 0) v = csub(v, adjoint ? tri(i - 1, 1, r, k, true) : tri(i, -1, r, k, false));
      vb[p0] = v;
    }
    __syncthreads();
    dense_all(i, conjt);
    __syncthreads();
    for (int p0 = t; p0 < work; p0 += kSweepBlock) {
      const int r = p0 / R, k = p0 - r * R;
      if (k >= nloc) continue;
      const double2 w = summed(p0);
      x[(int64_t)(c0 + k) * ldx + (int64_t)i * nx + r] = w;
      va[p0] = w;
    }
    __syncthreads();
  }
  // backward sweep (va holds row i + 1's result)
  for (int i = ny - 2; i >= 0; --i) {
    for (int p0 = t; p0 < work; p0 += kSweepBlock) {
      const int r = p0 / R, k = p0 - r * R;
      if (k >= nloc) continue;
      vb[p0] = adjoint ? tri(i + 1, -1, r, k, true) : tri(i, 1, r, k, false);
    }
    __syncthreads();
    dense_all(i, conjt);
    __syncthreads();
    for (int p0 = t; p0 < work; p0 += kSweepBlock) {
      const int r = p0 / R, k = p0 - r * R;
      if (k >= nloc) continue;
      const int64_t j = (int64_t)(c0 + k) * ldx + (int64_t)i * nx + r;
      const double2 v = csub(x[j], summed(p0));
      x[j] = v;
      va[p0] = v;
    }
    __syncthreads();
  }
}

// Sweep shape for grid rows of nx entries and nrhs right-hand sides: R right-hand sides per
// workgroup and P threads per (entry, right-hand side) pair.  One right-hand side per workgroup at
// every nrhs: a sweep is bound by the latency of each thread's chain of block-factor loads (nx / P
// long), which several right-hand sides per workgroup lengthen.  Eight columns on a 99 x 197 grid:
// 6.46 ms per sweep with all eight in one workgroup, the solve of that scatterer 10.7 -> 6.6 s.
void sweep_shape(int nx, int nrhs, int *R, int *P) {
  (void)nrhs;
  *R = 1;
  *P = std::max(1, kSweepBlock / nx);   // P nx <= max(kSweepBlock, nx) <= kSweepLds
}

}  // namespace

hipError_t launch_sparsify(const SparsifyData &sp, const double2 *c, int64_t ldc, double2 *sc, int64_t ldo,
                           double2 *tmp, int64_t ldt, int nrhs, bool adjoint, bool dscale, hipStream_t st) {
  const int64_t nc = (int64_t)sp.nx * sp.ny;
  const dim3 gs((unsigned)((nc + kBlock - 1) / kBlock), (unsigned)nrhs);
  int R = 1, P = 1;
  sweep_shape(sp.nx, nrhs, &R, &P);
  const unsigned sweeps = (unsigned)((nrhs + R - 1) / R);
  if (!adjoint) {
    // S c = C^-1 (A c): the stencil into sc, the sweep in place
    stencil_kernel<<<gs, kBlock, 0, st>>>(sp.nx, sp.ny, sp.W, c, ldc, sc, ldo, 0, nullptr);
    block_sweep_kernel<<<sweeps, kSweepBlock, 0, st>>>(sp.nx, sp.ny, R, P, nrhs, sp.E, sp.Gc, sp.Gr, sc, ldo, sc, ldo,
                                                       0, nullptr);
  } else {
    // S^H c = A^H (C^-H c), or D^-1 S^H D c with dscale
    block_sweep_kernel<<<sweeps, kSweepBlock, 0, st>>>(sp.nx, sp.ny, R, P, nrhs, sp.E, sp.Gc, sp.Gr, c, ldc, tmp, ldt,
                                                       1, dscale ? sp.d : nullptr);
    stencil_kernel<<<gs, kBlock, 0, st>>>(sp.nx, sp.ny, sp.W, tmp, ldt, sc, ldo, 1, dscale ? sp.dinv : nullptr);
  }
  return hipGetLastError();
}

}  // namespace lsk

using lsk::Scat;
using lsk::SparsifyData;
using lsk::cplx;

namespace {

ls_status sfail(ls_ctx *h, ls_status st, const std::string &msg) { return lsk::setup_fail(h, st, msg.c_str()); }

bool grid_ok(const ls_grid *g) {
  return g && g->h > 0 && std::isfinite(g->h) && std::isfinite(g->x0) && std::isfinite(g->y0) && g->nx >= 3 &&
         g->ny >= 3 && g->nx <= lsk::kMaxNx && (int64_t)g->nx * g->ny < ((int64_t)1 << 31);
}

}  // namespace

extern "C" {

ls_status ls_sparsify_stencil_host(const ls_grid *g, double k, const double *m_grid, double *W, double *E,
                                   double *sv_ratio) {
  if (!grid_ok(g) || !(k > 0) || !std::isfinite(k) || !m_grid || !W || !E)
    return lsk::setup_fail(nullptr, LS_ERR_ARG, "bad argument");
  std::vector<cplx> w, e;
  lsk::sparsify_stencil(g->nx, g->ny, g->h, k, (const cplx *)m_grid,
                        lsk::host_threads(ls_options{}), w, e, sv_ratio);
  std::memcpy(W, w.data(), sizeof(cplx) * w.size());
  std::memcpy(E, e.data(), sizeof(cplx) * e.size());
  return LS_OK;
}

ls_status ls_sparsify_setup(ls_handle h, int32_t s, const ls_grid *g, const double *m_grid, ls_sparsify_info *info) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!h) return lsk::setup_fail(nullptr, LS_ERR_ARG, "null handle");
  if (s < 0 || s >= (int32_t)h->sc.size()) return sfail(h, LS_ERR_ARG, "bad scatterer index");
  if (!grid_ok(g)) return sfail(h, LS_ERR_ARG, "bad grid (3 <= nx <= 1536, ny >= 3)");
  if (!m_grid) return sfail(h, LS_ERR_ARG, "null contrast");
  const int64_t nc = (int64_t)g->nx * g->ny;
  for (int64_t j = 0; j < 2 * nc; ++j)
    if (!std::isfinite(m_grid[j])) return sfail(h, LS_ERR_NONFINITE, "non-finite grid contrast");
  ls_status st = ls_transfer_setup(h, s, g);
  if (st != LS_OK) return st;
  Scat &sc = h->sc[s];
  const int nx = g->nx, ny = g->ny;
  const int threads = lsk::host_threads(h->opt);
  std::vector<cplx> W, E;
  double ratio = 0;
  lsk::sparsify_stencil(nx, ny, g->h, sc.k, (const cplx *)m_grid, threads, W, E, &ratio);
  std::vector<std::vector<cplx>> G;
  if (!lsk::sparsify_factor(nx, ny, E, G, threads))
    return sfail(h, LS_ERR_BREAKDOWN, "singular block in the LU of C^(C)");
  // residual of a seeded right-hand side solved through the factors, C x applied by the stencil
  double lu_res = 0;
  {
    std::vector<cplx> y(nc), x(nc);
    uint64_t z = 0x9E3779B97F4A7C15ull;
    for (int64_t j = 0; j < nc; ++j) {
      z = z * 6364136223846793005ull + 1442695040888963407ull;
      const double a = (double)(z >> 11) * 0x1.0p-53 - 0.5;
      z = z * 6364136223846793005ull + 1442695040888963407ull;
      const double b = (double)(z >> 11) * 0x1.0p-53 - 0.5;
      y[j] = cplx(a, b);
    }
    lsk::sparsify_solve_host(nx, ny, E, G, y.data(), x.data());
    double r2 = 0, y2 = 0;
    for (int iy = 0; iy < ny; ++iy)
      for (int ix = 0; ix < nx; ++ix) {
        const int64_t j = (int64_t)iy * nx + ix;
        cplx acc = 0;
        for (int o = 0; o < 9; ++o) {
          const int x2 = ix + o % 3 - 1, y2_ = iy + o / 3 - 1;
          if (x2 >= 0 && x2 < nx && y2_ >= 0 && y2_ < ny) acc += E[j * 9 + o] * x[(int64_t)y2_ * nx + x2];
        }
        r2 += std::norm(acc - y[j]);
        y2 += std::norm(y[j]);
      }
    lu_res = std::sqrt(r2 / y2);
  }
  // device arrays: W and E as [9][nc], the blocks both column- and row-major, D and D^-1
  auto sp = std::make_shared<SparsifyData>();
  sp->nx = nx;
  sp->ny = ny;
  const size_t n2 = (size_t)nx * nx;
  std::vector<cplx> W9(9 * nc), E9(9 * nc), Gc(n2 * ny), Gr(n2 * ny);
  for (int64_t j = 0; j < nc; ++j)
    for (int o = 0; o < 9; ++o) {
      W9[(size_t)o * nc + j] = W[(size_t)j * 9 + o];
      E9[(size_t)o * nc + j] = E[(size_t)j * 9 + o];
    }
  for (int i = 0; i < ny; ++i)
    for (int r = 0; r < nx; ++r)
      for (int c = 0; c < nx; ++c) {
        Gr[(size_t)i * n2 + (size_t)r * nx + c] = G[i][(size_t)r * nx + c];
        Gc[(size_t)i * n2 + (size_t)c * nx + r] = G[i][(size_t)r * nx + c];
      }
  std::vector<double> d(sc.tr->colsum), dinv(nc);
  for (int64_t j = 0; j < nc; ++j) dinv[j] = 1.0 / d[j];
  auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
    if (lsk::dmalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) return false;
    sp->bufs.push_back(*dst);
    h->owned.push_back(*dst);
    sp->bytes += (int64_t)bytes;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  if (!up((void **)&sp->W, W9.data(), sizeof(cplx) * W9.size()) ||
      !up((void **)&sp->E, E9.data(), sizeof(cplx) * E9.size()) ||
      !up((void **)&sp->Gc, Gc.data(), sizeof(cplx) * Gc.size()) ||
      !up((void **)&sp->Gr, Gr.data(), sizeof(cplx) * Gr.size()) ||
      !up((void **)&sp->d, d.data(), sizeof(double) * nc) || !up((void **)&sp->dinv, dinv.data(), sizeof(double) * nc))
    return sfail(h, LS_ERR_ALLOC, "preconditioner tables");
  sp->sv_ratio = ratio;
  sp->lu_residual = lu_res;
  if (sc.sp) {
    (void)hipDeviceSynchronize();
    for (void *p : sc.sp->bufs) {
      h->owned.erase(std::remove(h->owned.begin(), h->owned.end(), p), h->owned.end());
      (void)hipFree(p);
    }
  }
  sc.sp = sp;
  if (info) {
    info->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    info->sv_ratio = ratio;
    info->lu_residual = lu_res;
    info->device_bytes = sp->bytes;
  }
  return LS_OK;
}

ls_status ls_sparsify_apply(ls_handle h, int32_t s, const double *c, int64_t ldc, double *sc_out, int32_t nrhs,
                            int32_t adjoint, hipStream_t stream) {
  if (!h) return lsk::setup_fail(nullptr, LS_ERR_ARG, "null handle");
  if (s < 0 || s >= (int32_t)h->sc.size()) return sfail(h, LS_ERR_ARG, "bad scatterer index");
  const Scat &sc = h->sc[s];
  if (!sc.sp) return sfail(h, LS_ERR_ARG, "no preconditioner for this scatterer (ls_sparsify_setup)");
  if (nrhs < 0 || nrhs > 65535) return sfail(h, LS_ERR_ARG, "bad nrhs");
  if (nrhs == 0) return LS_OK;
  if (!c || !sc_out) return sfail(h, LS_ERR_ARG, "null vector");
  const int64_t nc = (int64_t)sc.sp->nx * sc.sp->ny;
  if (ldc < nc) return sfail(h, LS_ERR_ARG, "ldc < number of grid nodes");
  if (c == sc_out) return sfail(h, LS_ERR_ARG, "c and sc must not alias");
  double2 *tmp = nullptr;
  if (adjoint) {
    const size_t need = sizeof(double2) * (size_t)nc * nrhs;
    if (need > h->ws_grid.bytes) {
      if (h->ws_grid.ptr) {
        if (hipStreamSynchronize(stream) != hipSuccess) return sfail(h, LS_ERR_HIP, "stream synchronize");
        (void)hipFree(h->ws_grid.ptr);
        h->ws_grid.ptr = nullptr;
        h->ws_grid.bytes = 0;
      }
      if (lsk::dmalloc(&h->ws_grid.ptr, need) != hipSuccess) return sfail(h, LS_ERR_ALLOC, "grid workspace");
      h->ws_grid.bytes = need;
    }
    tmp = (double2 *)h->ws_grid.ptr;
  }
  if (lsk::launch_sparsify(*sc.sp, (const double2 *)c, ldc, (double2 *)sc_out, ldc, tmp, nc, nrhs, adjoint != 0, false,
                           stream) != hipSuccess)
    return sfail(h, LS_ERR_HIP, "sparsify launch");
  return LS_OK;
}

}  // extern "C"
