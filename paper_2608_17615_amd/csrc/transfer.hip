// Transfer operators between a scatterer's quadrature nodes and a Cartesian grid, and the last
// step of the preconditioner built from them (paper, Section 4):
//   T_C^Q  grid -> nodes: bilinear hat functions of the node's cell (eq. psi_def), four entries
//          per row, applied as a gather of the four vertex values;
//   T_Q^C  nodes -> grid: the renormalized transpose D^-1 (T_C^Q)^T (Approach II, eqs. T_H^C_def
//          and D_def), a CSR over the grid nodes built on the host (rows in node order, so the
//          sums are deterministic);
//   P x = x + T_C^Q (S - I) T_Q^C x (eq. preconditioner_factored): the caller forms c = T_Q^C x,
//          applies its Cartesian approximate inverse S to c, and ls_precond_finish adds
//          T_C^Q (S c - c) to x.
// All three kernels are HBM-bound gathers: 16 B per complex value moved.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

namespace lsk {

namespace {

constexpr int kBlock = 256;

// Each thread serves one node (or grid node) for kCols consecutive right-hand sides, so the cell
// weights and the CSR rows are read once per kCols columns instead of once per column.
constexpr int kCols = 8;

// y[c][off + perm[i]] = (xa ? xa[c][off + perm[i]] : 0) + sum over the four vertices v of node i's
// cell of w_v(i) (g[c][j_v] - (g2 ? g2[c][j_v] : 0)); grid (ceil(n / kBlock), ceil(nrhs / kCols)).
__global__ __launch_bounds__(kBlock) void cart_to_quad_kernel(int64_t n, int nrhs, int nx,
                                                             const int32_t *__restrict__ cell,
                                                             const double4 *__restrict__ w,
                                                             const int32_t *__restrict__ perm, int64_t off,
                                                             const double2 *__restrict__ g,
                                                             const double2 *__restrict__ g2, int64_t ldg,
                                                             const double2 *xa, double2 *y, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t j = cell[i];
  const double4 wv = w[i];
  const int64_t dst = off + perm[i];
  const int c1 = min(nrhs, (int)(blockIdx.y + 1) * kCols);
  for (int64_t c = (int64_t)blockIdx.y * kCols; c < c1; ++c) {
    const double2 *gc = g + c * ldg;
    double2 v0 = gc[j], v1 = gc[j + 1], v2 = gc[j + nx], v3 = gc[j + nx + 1];
    if (g2) {
      const double2 *hc = g2 + c * ldg;
      const double2 u0 = hc[j], u1 = hc[j + 1], u2 = hc[j + nx], u3 = hc[j + nx + 1];
      v0 = make_double2(v0.x - u0.x, v0.y - u0.y);
      v1 = make_double2(v1.x - u1.x, v1.y - u1.y);
      v2 = make_double2(v2.x - u2.x, v2.y - u2.y);
      v3 = make_double2(v3.x - u3.x, v3.y - u3.y);
    }
    double re = wv.x * v0.x, im = wv.x * v0.y;
    re = std::fma(wv.y, v1.x, re);
    im = std::fma(wv.y, v1.y, im);
    re = std::fma(wv.z, v2.x, re);
    im = std::fma(wv.z, v2.y, im);
    re = std::fma(wv.w, v3.x, re);
    im = std::fma(wv.w, v3.y, im);
    const int64_t idx = c * ld + dst;
    if (xa) {
      const double2 a = xa[idx];
      re += a.x;
      im += a.y;
    }
    y[idx] = make_double2(re, im);
  }
}

// g[c][j] = sum over CSR row j of val * x[c][off + col]; grid (ceil(nc / kBlock), ceil(nrhs / kCols)).
// Rows of up to kRow entries are held in registers across the columns.
constexpr int kRow = 8;
__global__ __launch_bounds__(kBlock) void quad_to_cart_kernel(int64_t nc, int nrhs, const int64_t *__restrict__ rp,
                                                             const int32_t *__restrict__ col,
                                                             const double *__restrict__ val, int64_t off,
                                                             const double2 *__restrict__ x, int64_t ld,
                                                             double2 *__restrict__ g, int64_t ldg) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= nc) return;
  const int64_t e0 = rp[j], e1 = rp[j + 1];
  const int c1 = min(nrhs, (int)(blockIdx.y + 1) * kCols);
  if (e1 - e0 <= kRow) {
    const int m = (int)(e1 - e0);
    int32_t cl[kRow];
    double vl[kRow];
#pragma unroll
    for (int e = 0; e < kRow; ++e) {
      cl[e] = e < m ? col[e0 + e] : 0;
      vl[e] = e < m ? val[e0 + e] : 0.0;
    }
    for (int64_t c = (int64_t)blockIdx.y * kCols; c < c1; ++c) {
      const double2 *xc = x + c * ld + off;
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int e = 0; e < kRow; ++e)
        if (e < m) {
          const double2 a = xc[cl[e]];
          re = std::fma(vl[e], a.x, re);
          im = std::fma(vl[e], a.y, im);
        }
      g[c * ldg + j] = make_double2(re, im);
    }
  } else {
    for (int64_t c = (int64_t)blockIdx.y * kCols; c < c1; ++c) {
      const double2 *xc = x + c * ld + off;
      double re = 0.0, im = 0.0;
      for (int64_t e = e0; e < e1; ++e) {
        const double v = val[e];
        const double2 a = xc[col[e]];
        re = std::fma(v, a.x, re);
        im = std::fma(v, a.y, im);
      }
      g[c * ldg + j] = make_double2(re, im);
    }
  }
}

ls_status tfail(ls_ctx *h, ls_status st, const char *msg) { return setup_fail(h, st, msg); }

}  // namespace

hipError_t launch_quad_to_cart(const Scat &sc, const double2 *x, int64_t ld, double2 *c, int64_t ldc, int nrhs,
                               hipStream_t st) {
  const TransferData &t = *sc.tr;
  const int64_t nc = (int64_t)t.nx * t.ny;
  dim3 grid((unsigned)((nc + kBlock - 1) / kBlock), (unsigned)((nrhs + kCols - 1) / kCols));
  quad_to_cart_kernel<<<grid, kBlock, 0, st>>>(nc, nrhs, t.rp, t.col, t.val, sc.off, x, ld, c, ldc);
  return hipGetLastError();
}

hipError_t launch_precond_finish(const Scat &sc, const double2 *x, int64_t ld, const double2 *c, const double2 *s,
                                 int64_t ldc, double2 *y, int nrhs, hipStream_t st) {
  const TransferData &t = *sc.tr;
  dim3 grid((unsigned)((sc.n + kBlock - 1) / kBlock), (unsigned)((nrhs + kCols - 1) / kCols));
  cart_to_quad_kernel<<<grid, kBlock, 0, st>>>(sc.n, nrhs, t.nx, t.cell, t.w, sc.perm, sc.off, s, c, ldc, x, y, ld);
  return hipGetLastError();
}

}  // namespace lsk

using lsk::Scat;
using lsk::TransferData;

extern "C" {

ls_status ls_transfer_setup(ls_handle h, int32_t s, const ls_grid *g) {
  if (!h) return lsk::setup_fail(nullptr, LS_ERR_ARG, "null handle");
  if (s < 0 || s >= (int32_t)h->sc.size()) return lsk::tfail(h, LS_ERR_ARG, "bad scatterer index");
  if (!g || !(g->h > 0) || !std::isfinite(g->h) || !std::isfinite(g->x0) || !std::isfinite(g->y0) || g->nx < 2 ||
      g->ny < 2 || (int64_t)g->nx * g->ny >= ((int64_t)1 << 31))
    return lsk::tfail(h, LS_ERR_ARG, "bad grid");
  Scat &sc = h->sc[s];
  const double *px = lsk::geom_x(sc), *py = lsk::geom_y(sc);
  if (!px || !py) return lsk::tfail(h, LS_ERR_UNSUPPORTED, "no geometry for this scatterer");
  const int64_t n = sc.n, nx = g->nx, ny = g->ny, nc = nx * ny;
  // cell of each node (floor of the scaled coordinate, the last grid line taking the cell below)
  // and the hat functions of its four vertices, psi_j = (1 - |dx| / h)(1 - |dy| / h)
  std::vector<int32_t> cell(n);
  std::vector<double4> w(n);
  for (int64_t i = 0; i < n; ++i) {
    const double sx = (px[i] - g->x0) / g->h, sy = (py[i] - g->y0) / g->h;
    if (!(sx >= 0 && sy >= 0 && sx <= (double)(nx - 1) && sy <= (double)(ny - 1)))
      return lsk::tfail(h, LS_ERR_ARG, "a node lies outside the grid");
    const double fx = std::floor(sx), fy = std::floor(sy);
    const int64_t ix = std::min<int64_t>((int64_t)fx, nx - 2), iy = std::min<int64_t>((int64_t)fy, ny - 2);
    cell[i] = (int32_t)(iy * nx + ix);
    double wx[2], wy[2];
    for (int d = 0; d < 2; ++d) {
      const double tx = (double)(ix + d) * g->h;   // separate statements: no contraction into an FMA
      const double zx = g->x0 + tx;
      const double ty = (double)(iy + d) * g->h;
      const double zy = g->y0 + ty;
      wx[d] = 1.0 - std::fabs(px[i] - zx) / g->h;
      wy[d] = 1.0 - std::fabs(py[i] - zy) / g->h;
    }
    double4 v;
    v.x = wx[0] * wy[0];
    v.y = wx[1] * wy[0];
    v.z = wx[0] * wy[1];
    v.w = wx[1] * wy[1];
    w[i] = v;
  }
  // T_Q^C = D^-1 (T_C^Q)^T: rows over the grid nodes, entries in internal node order
  std::vector<int64_t> rp(nc + 1, 0);
  auto vidx = [&](int64_t i, int v) { return (int64_t)cell[i] + (v & 1) + (v >> 1) * nx; };
  for (int64_t i = 0; i < n; ++i)
    for (int v = 0; v < 4; ++v) ++rp[vidx(i, v) + 1];
  for (int64_t j = 0; j < nc; ++j) rp[j + 1] += rp[j];
  std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
  std::vector<int32_t> col(4 * n);
  std::vector<double> val(4 * n);
  for (int64_t i = 0; i < n; ++i) {
    const double wv[4] = {w[i].x, w[i].y, w[i].z, w[i].w};
    for (int v = 0; v < 4; ++v) {
      const int64_t e = fill[vidx(i, v)]++;
      col[e] = sc.perm_host[i];
      val[e] = wv[v];
    }
  }
  std::vector<double> colsum(nc);
  for (int64_t j = 0; j < nc; ++j) {
    double d = 0.0;
    for (int64_t e = rp[j]; e < rp[j + 1]; ++e) d += val[e];
    const double dj = d > 0 ? d : 1.0;   // D_jj = 1 where no node reaches j with a positive weight
    colsum[j] = dj;
    for (int64_t e = rp[j]; e < rp[j + 1]; ++e) val[e] /= dj;
  }
  // replace an earlier grid of this scatterer
  auto t = std::make_shared<TransferData>();
  t->x0 = g->x0;
  t->y0 = g->y0;
  t->h = g->h;
  t->nx = g->nx;
  t->ny = g->ny;
  t->colsum = std::move(colsum);
  auto up = [&](void **dst, const void *src, size_t bytes) -> bool {
    if (lsk::dmalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) return false;
    t->bufs.push_back(*dst);
    h->owned.push_back(*dst);
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  if (!up((void **)&t->cell, cell.data(), sizeof(int32_t) * n) || !up((void **)&t->w, w.data(), sizeof(double4) * n) ||
      !up((void **)&t->rp, rp.data(), sizeof(int64_t) * (nc + 1)) ||
      !up((void **)&t->col, col.data(), sizeof(int32_t) * col.size()) ||
      !up((void **)&t->val, val.data(), sizeof(double) * val.size()))
    return lsk::tfail(h, LS_ERR_ALLOC, "transfer tables");
  if (sc.tr || sc.sp) {
    (void)hipDeviceSynchronize();
    // the old grid's tables, and a sparsifying preconditioner built on that grid
    std::vector<void *> old;
    if (sc.tr) old = sc.tr->bufs;
    if (sc.sp) old.insert(old.end(), sc.sp->bufs.begin(), sc.sp->bufs.end());
    for (void *p : old) {
      h->owned.erase(std::remove(h->owned.begin(), h->owned.end(), p), h->owned.end());
      (void)hipFree(p);
    }
    sc.sp.reset();
  }
  sc.tr = t;
  return LS_OK;
}

static ls_status transfer_args(ls_handle h, int32_t s, int64_t ld, int64_t ldc, int32_t nrhs) {
  if (!h) return lsk::setup_fail(nullptr, LS_ERR_ARG, "null handle");
  if (s < 0 || s >= (int32_t)h->sc.size()) return lsk::tfail(h, LS_ERR_ARG, "bad scatterer index");
  if (!h->sc[s].tr) return lsk::tfail(h, LS_ERR_ARG, "no grid for this scatterer (ls_transfer_setup)");
  if (nrhs < 0 || nrhs > 65535) return lsk::tfail(h, LS_ERR_ARG, "bad nrhs");
  if (ld < h->n_total) return lsk::tfail(h, LS_ERR_ARG, "ld < number of nodes");
  const TransferData &t = *h->sc[s].tr;
  if (ldc < (int64_t)t.nx * t.ny) return lsk::tfail(h, LS_ERR_ARG, "ldc < number of grid nodes");
  return LS_OK;
}

ls_status ls_transfer_colsums(ls_handle h, int32_t s, double *d) {
  if (!h) return lsk::setup_fail(nullptr, LS_ERR_ARG, "null handle");
  if (s < 0 || s >= (int32_t)h->sc.size()) return lsk::tfail(h, LS_ERR_ARG, "bad scatterer index");
  if (!h->sc[s].tr) return lsk::tfail(h, LS_ERR_ARG, "no grid for this scatterer (ls_transfer_setup)");
  if (!d) return lsk::tfail(h, LS_ERR_ARG, "null output");
  const std::vector<double> &cs = h->sc[s].tr->colsum;
  std::copy(cs.begin(), cs.end(), d);
  return LS_OK;
}

ls_status ls_quad_to_cart(ls_handle h, int32_t s, const double *x, int64_t ld, double *c, int64_t ldc, int32_t nrhs,
                          hipStream_t stream) {
  ls_status st = transfer_args(h, s, ld, ldc, nrhs);
  if (st != LS_OK) return st;
  if (nrhs == 0) return LS_OK;
  if (!x || !c) return lsk::tfail(h, LS_ERR_ARG, "null vector");
  if (lsk::launch_quad_to_cart(h->sc[s], (const double2 *)x, ld, (double2 *)c, ldc, nrhs, stream) != hipSuccess)
    return lsk::tfail(h, LS_ERR_HIP, "quad_to_cart launch");
  return LS_OK;
}

ls_status ls_cart_to_quad(ls_handle h, int32_t s, const double *c, int64_t ldc, double *y, int64_t ld, int32_t nrhs,
                          hipStream_t stream) {
  ls_status st = transfer_args(h, s, ld, ldc, nrhs);
  if (st != LS_OK) return st;
  if (nrhs == 0) return LS_OK;
  if (!c || !y) return lsk::tfail(h, LS_ERR_ARG, "null vector");
  const Scat &sc = h->sc[s];
  const TransferData &t = *sc.tr;
  dim3 grid((unsigned)((sc.n + lsk::kBlock - 1) / lsk::kBlock), (unsigned)((nrhs + lsk::kCols - 1) / lsk::kCols));
  lsk::cart_to_quad_kernel<<<grid, lsk::kBlock, 0, stream>>>(sc.n, nrhs, t.nx, t.cell, t.w, sc.perm, sc.off,
                                                             (const double2 *)c, nullptr, ldc, nullptr,
                                                             (double2 *)y, ld);
  if (hipGetLastError() != hipSuccess) return lsk::tfail(h, LS_ERR_HIP, "cart_to_quad launch");
  return LS_OK;
}

ls_status ls_precond_finish(ls_handle h, int32_t s, const double *x, int64_t ld, const double *c, const double *sc_,
                            int64_t ldc, double *y, int32_t nrhs, hipStream_t stream) {
  ls_status st = transfer_args(h, s, ld, ldc, nrhs);
  if (st != LS_OK) return st;
  if (nrhs == 0) return LS_OK;
  if (!x || !c || !sc_ || !y) return lsk::tfail(h, LS_ERR_ARG, "null vector");
  if (lsk::launch_precond_finish(h->sc[s], (const double2 *)x, ld, (const double2 *)c, (const double2 *)sc_, ldc,
                                 (double2 *)y, nrhs, stream) != hipSuccess)
    return lsk::tfail(h, LS_ERR_HIP, "precond_finish launch");
  return LS_OK;
}

}  // extern "C"
