// Native assembly of the VDIM correction C (paper, Section 3, eq. DIM_decomp with the
// subdomain split of eq. vol_pot_decomp) for ls_setup.
//
// For node j and subdomain l, with tau the interpolation element (the node's own element when
// it lies in l, otherwise l's element whose node-mean centroid is nearest, ties to the smaller
// caller element index), centre c and scale s (largest node-to-node distance) of tau, and the
// scaled monomials P_a(y) = ((y - c)/s)^a, |a| <= 3:
//     D_a = E_l[P_a](y_j) - sum_{q in l, q != j} G(y_j, y_q) w_q P_a(y_q),
//     C_{j, nodes(tau)} = V_tau^{-T} D,   V_tau[i][a] = P_a(node i of tau),
// so that C applied to nodal values adds E_l[F] - sum G w F for the cubic interpolant F on tau.
//   * E_l[P](x) = -Phi(x) [x in Omega_l] + oint_{dOmega_l} (G d_nu Phi - Phi d_nu G) ds by Green's
//     third identity with the polynomial particular solution Phi = P/k^2 - Delta P / k^4
//     ((Delta + k^2) Phi = P for cubic P), integrated with adaptive 16-point Gauss-Legendre
//     panels on the exact curves: host threads, libm J0/Y0/J1/Y1 in long double.
//   * The punctured monomial sums (N^2 x 10 work) run on the GPU: one target per lane with its
//     own frame (c, 1/s), sources of subdomain l walked uniformly per wavefront, G from the same
//     in-register evaluation as the operator's far sum, compensated (TwoSum) accumulation.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "hankel.h"
#include "host.h"
#include "internal.h"

namespace lsk {

ls_status setup_fail(ls_ctx *h, ls_status st, const char *msg);
std::vector<int32_t> element_order(const ls_scatterer &s);
ls_status upload_nodes(ls_ctx *h, Scat &sc, const ls_scatterer &s, const std::vector<int32_t> &eord);
ls_status upload_correction(ls_ctx *h, Scat &sc, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci,
                            const std::vector<double> &cv);

struct CurveH {
  int kind, orient, sub;
  double cx, cy, a, b;
  void eval(double t, double &px, double &py, double &sp, double &nx, double &ny) const {
    const double ct = std::cos(t), st = std::sin(t);
    px = cx + a * ct;
    py = cy + b * st;
    const double tx = -a * st, ty = b * ct;
    sp = std::hypot(tx, ty);
    nx = orient * ty / sp;
    ny = -orient * tx / sp;
  }
};

namespace {

constexpr int kBlock = 256;
constexpr int NA = 10;
constexpr int AX[NA] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0};
constexpr int AY[NA] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3};

__constant__ HankelTable s_hankel = kHankelTable;
typedef __attribute__((address_space(4))) const HankelTable ConstTab;

__device__ __forceinline__ ConstTab &table() {
  ConstTab *t = (ConstTab *)&s_hankel;
  asm volatile("" : "+s"(t));
  return *t;
}

// out[split][j][a] = sum_{q in [q0, q1) of this split} G(x_j, y_q) w_q P_a((y_q - c_j)/s_j) for the
// targets x_j = (tx[j], ty[j]); PUNCT: the targets are the nodes themselves and q = j is left out
template <bool PUNCT>
__global__ __launch_bounds__(kBlock) void poly_sums_kernel(int n, const double *__restrict__ tx,
                                                           const double *__restrict__ ty,
                                                           const double2 *__restrict__ pos,
                                                           const double *__restrict__ w, int q0, int q1,
                                                           const double4 *__restrict__ frame, double k2,
                                                           int split_len, double2 *__restrict__ out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int ii = i < n ? i : n - 1;
  const double xt = tx[ii], yt = ty[ii];
  const double4 fr = frame[ii];   // (cx, cy, 1/s, unused)
  const int s0 = q0 + blockIdx.y * split_len;
  const int s1 = min(q1, s0 + split_len);
  // compensated accumulation (TwoSum: the rounding error of every addition is kept in cr, ci),
  // since the sums of far-away, large monomial values cancel against the exact potentials
  double ar[NA], ai[NA], cr[NA], ci[NA];
#pragma unroll
  for (int a = 0; a < NA; ++a) ar[a] = ai[a] = cr[a] = ci[a] = 0.0;
  auto two_sum = [](double &s, double &c, double t) {
#pragma clang fp contract(off)
    const double u = s + t;
    const double bp = u - s;
    c += (s - (u - bp)) + (t - bp);
    s = u;
  };
  for (int q = s0; q < s1; ++q) {
    const double2 p = pos[q];
    const double wq = w[q];
    const double dx = xt - p.x, dy = yt - p.y;
    const double A = k2 * std::fma(dx, dx, dy * dy);
    double gr, gi;
    green(A, gr, gi, table());
    const bool self = PUNCT && (q == i);
    gr = self ? 0.0 : gr * wq;
    gi = self ? 0.0 : gi * wq;
    const double u = (p.x - fr.x) * fr.z, v = (p.y - fr.y) * fr.z;
    const double u2 = u * u, v2 = v * v, uv = u * v;
    const double P[NA] = {1.0, u, v, u2, uv, v2, u2 * u, u2 * v, u * v2, v2 * v};
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      // the product is rounded on its own (no contraction into the sum)
      const double tr = __builtin_fma(gr, P[a], 0.0), ti = __builtin_fma(gi, P[a], 0.0);
      two_sum(ar[a], cr[a], tr);
      two_sum(ai[a], ci[a], ti);
    }
  }
  if (i < n) {
    double2 *o = out + ((int64_t)blockIdx.y * n + i) * NA;
#pragma unroll
    for (int a = 0; a < NA; ++a) o[a] = make_double2(ar[a] + cr[a], ai[a] + ci[a]);
  }
}

// ---------------------------------------------------------------- host quadrature
struct GaussLegendre {
  static constexpr int N = 16;
  double t[N], w[N];
  GaussLegendre() {
    for (int i = 0; i < N; ++i) {
      double x = std::cos(M_PI * (i + 0.75) / (N + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= N; ++k) {
          const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        const double dp = N * (x * p1 - p0) / (x * x - 1.0);
        const double dx = p1 / dp;
        x -= dx;
        if (std::fabs(dx) < 1e-17) {
          t[i] = x;
          w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
          break;
        }
        t[i] = x;
        w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
      }
    }
  }
};

inline double mono(double u, double v, int a, int b) {
  if (a < 0 || b < 0) return 0.0;
  double r = 1.0;
  for (int i = 0; i < a; ++i) r *= u;
  for (int i = 0; i < b; ++i) r *= v;
  return r;
}

// Phi_a and d_nu Phi_a at y for the 10 scaled monomials of frame (c, s)
inline void particular(double y1, double y2, double cx, double cy, double s, double k, double nx, double ny,
                       double *phi, double *dphi) {
  const double u = (y1 - cx) / s, v = (y2 - cy) / s;
  const double k2 = k * k, k4 = k2 * k2;
  for (int al = 0; al < NA; ++al) {
    const int a = AX[al], b = AY[al];
    const double P = mono(u, v, a, b);
    const double Pu = a * mono(u, v, a - 1, b), Pv = b * mono(u, v, a, b - 1);
    const double L = a * (a - 1) * mono(u, v, a - 2, b) + b * (b - 1) * mono(u, v, a, b - 2);
    const double Lu = a * (a - 1) * (a - 2) * mono(u, v, a - 3, b) + b * (b - 1) * a * mono(u, v, a - 1, b - 2);
    const double Lv = a * (a - 1) * b * mono(u, v, a - 2, b - 1) + b * (b - 1) * (b - 2) * mono(u, v, a, b - 3);
    phi[al] = P / k2 - L / (s * s * k4);
    const double gx = Pu / (s * k2) - Lu / (s * s * s * k4);
    const double gy = Pv / (s * k2) - Lv / (s * s * s * k4);
    dphi[al] = gx * nx + gy * ny;
  }
}

// E[P_a](x) for the 10 monomials over the subdomain bounded by `curves`.
void poly_potential(const std::vector<CurveH> &curves, bool inside, double x1, double x2, double cx, double cy,
                    double s, double k, const GaussLegendre &gl, double *Er, double *Ei) {
  double accr[NA] = {0}, acci[NA] = {0}, cr[NA] = {0}, cim[NA] = {0};   // Kahan-compensated
  auto add = [&](int a, double vr, double vi) {
    double y = vr - cr[a], t = accr[a] + y;
    cr[a] = (t - accr[a]) - y;
    accr[a] = t;
    y = vi - cim[a];
    t = acci[a] + y;
    cim[a] = (t - acci[a]) - y;
    acci[a] = t;
  };
  std::vector<std::pair<double, double>> stack, panels;
  for (const CurveH &cv : curves) {
    const double vmax = std::max(cv.a, cv.b);
    const int m0 = (int)std::max(16.0, std::ceil(k * 2 * M_PI * vmax / 4.0));
    stack.clear();
    panels.clear();
    for (int i = 0; i < m0; ++i) stack.push_back({2 * M_PI * i / m0, 2 * M_PI * (i + 1) / m0});
    while (!stack.empty()) {
      auto [t0, t1] = stack.back();
      stack.pop_back();
      const double tm = 0.5 * (t0 + t1);
      double mx, my, sp, nx, ny;
      cv.eval(tm, mx, my, sp, nx, ny);
      const double len = vmax * (t1 - t0);
      if (std::hypot(x1 - mx, x2 - my) < 1.5 * len && len > 1e-14) {
        stack.push_back({t0, tm});
        stack.push_back({tm, t1});
      } else {
        panels.push_back({t0, t1});
      }
    }
    double phi[NA], dphi[NA];
    for (auto [t0, t1] : panels) {
      const double hh = 0.5 * (t1 - t0), tc = 0.5 * (t0 + t1);
      for (int g = 0; g < GaussLegendre::N; ++g) {
        double py1, py2, sp, nx, ny;
        cv.eval(tc + hh * gl.t[g], py1, py2, sp, nx, ny);
        const double ds = sp * hh * gl.w[g];
        const double rx = py1 - x1, ry = py2 - x2;
        const double rho = std::hypot(rx, ry);
        const double z = k * rho;
        // extended-precision Bessel values (x87 long double), rounded once: their absolute error
        // multiplies the large polynomial densities of far-away panels
        const long double zl = (long double)z;
        const double J0 = (double)::j0l(zl), Y0 = (double)::y0l(zl), J1 = (double)::j1l(zl), Y1 = (double)::y1l(zl);
        // G = (i/4)(J0 + i Y0);  d_nu G = -(i k / 4)(J1 + i Y1) (y - x).nu / rho
        const double Gr = -0.25 * Y0 * ds, Gi = 0.25 * J0 * ds;
        const double f = (rx * nx + ry * ny) / rho * k * 0.25 * ds;
        // d_nu G ds = -i f (J1 + i Y1) = f Y1 - i f J1
        const double dGr = Y1 * f, dGi = -J1 * f;
        particular(py1, py2, cx, cy, s, k, nx, ny, phi, dphi);
        for (int a = 0; a < NA; ++a) add(a, Gr * dphi[a] - dGr * phi[a], Gi * dphi[a] - dGi * phi[a]);
      }
    }
  }
  double phix[NA], dummy[NA];
  particular(x1, x2, cx, cy, s, k, 0.0, 0.0, phix, dummy);
  for (int a = 0; a < NA; ++a) {
    Er[a] = accr[a] - (inside ? phix[a] : 0.0);
    Ei[a] = acci[a];
  }
}

// LU with partial pivoting of a 10x10 matrix (row-major), in place.
bool lu10(double *A, int *piv) {
  for (int c = 0; c < NA; ++c) {
    int p = c;
    for (int r = c + 1; r < NA; ++r)
      if (std::fabs(A[r * NA + c]) > std::fabs(A[p * NA + c])) p = r;
    if (A[p * NA + c] == 0.0) return false;
    piv[c] = p;
    if (p != c)
      for (int k = 0; k < NA; ++k) std::swap(A[c * NA + k], A[p * NA + k]);
    for (int r = c + 1; r < NA; ++r) {
      const double f = A[r * NA + c] / A[c * NA + c];
      A[r * NA + c] = f;
      for (int k = c + 1; k < NA; ++k) A[r * NA + k] -= f * A[c * NA + k];
    }
  }
  return true;
}

void lu10_solve(const double *LU, const int *piv, double *b) {
  for (int c = 0; c < NA; ++c) std::swap(b[c], b[piv[c]]);
  for (int r = 1; r < NA; ++r)
    for (int k = 0; k < r; ++k) b[r] -= LU[r * NA + k] * b[k];
  for (int r = NA - 1; r >= 0; --r) {
    for (int k = r + 1; k < NA; ++k) b[r] -= LU[r * NA + k] * b[k];
    b[r] /= LU[r * NA + r];
  }
}

template <class F>
void parallel_for(int64_t n, int threads, F f) {
  if (threads <= 1 || n < 64) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> pool;
  std::atomic<int64_t> next(0);
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&]() {
      for (;;) {
        const int64_t b = next.fetch_add(64);
        if (b >= n) break;
        for (int64_t i = b; i < std::min(n, b + 64); ++i) f(i);
      }
    });
  for (auto &th : pool) th.join();
}

}  // namespace

// Host geometry of a scatterer in the internal node order: element frames (node-mean centroid,
// largest node distance), LU factors of the transposed cubic Vandermonde matrices, subdomain
// node ranges and element lists, and the boundary curves of every subdomain.
struct GeomData {
  int64_t n = 0;
  int32_t ne = 0;
  int nsub = 1;
  double k = 0;
  std::vector<double> px, py;
  std::vector<int32_t> esub, ecaller;
  std::vector<double> ecx, ecy, esc, LU;
  std::vector<int> piv;
  std::vector<int64_t> sub_lo, sub_hi;
  std::vector<std::vector<int32_t>> sub_elems;
  std::vector<std::vector<CurveH>> curves;
};

const double *geom_x(const Scat &sc) { return sc.geom ? sc.geom->px.data() : nullptr; }
const double *geom_y(const Scat &sc) { return sc.geom ? sc.geom->py.data() : nullptr; }

ls_status build_geometry(ls_ctx *h, Scat &sc, const ls_scatterer &s, const std::vector<int32_t> &eord) {
  auto g = std::make_shared<GeomData>();
  const int64_t n = sc.n;
  const int32_t ne = (int32_t)(n / 10);
  g->n = n;
  g->ne = ne;
  g->nsub = sc.n_sub;
  g->k = sc.k;
  g->px.resize(n);
  g->py.resize(n);
  g->esub.resize(ne);
  g->ecaller.resize(ne);
  for (int32_t e = 0; e < ne; ++e) {
    g->esub[e] = s.elem_subdomain[eord[e]];
    g->ecaller[e] = eord[e];
  }
  for (int64_t i = 0; i < n; ++i) {
    g->px[i] = s.x[sc.perm_host[i]];
    g->py[i] = s.y[sc.perm_host[i]];
  }
  g->ecx.resize(ne);
  g->ecy.resize(ne);
  g->esc.resize(ne);
  g->LU.resize((size_t)ne * NA * NA);
  g->piv.resize((size_t)ne * NA);
  bool ok = true;
  for (int32_t e = 0; e < ne; ++e) {
    const double *X = &g->px[10 * (int64_t)e], *Y = &g->py[10 * (int64_t)e];
    double ax = 0, ay = 0, d = 0;
    for (int q = 0; q < 10; ++q) {
      ax += X[q];
      ay += Y[q];
    }
    g->ecx[e] = ax / 10;
    g->ecy[e] = ay / 10;
    for (int p = 0; p < 10; ++p)
      for (int q = 0; q < 10; ++q) d = std::max(d, std::hypot(X[p] - X[q], Y[p] - Y[q]));
    g->esc[e] = d;
    // V^T[a][i] = P_a(node i): factor V^T so that V^T r = D is one solve
    double *A = &g->LU[(size_t)e * NA * NA];
    for (int i = 0; i < 10; ++i) {
      const double u = (X[i] - g->ecx[e]) / d, v = (Y[i] - g->ecy[e]) / d;
      for (int a = 0; a < NA; ++a) A[a * NA + i] = mono(u, v, AX[a], AY[a]);
    }
    ok = ok && lu10(A, &g->piv[(size_t)e * NA]);
  }
  if (!ok) return setup_fail(h, LS_ERR_ARG, "an element's 10 nodes are not unisolvent for cubics");
  // subdomain ranges (internal order groups subdomains contiguously)
  const int nsub = g->nsub;
  g->sub_lo.assign(nsub, n);
  g->sub_hi.assign(nsub, 0);
  g->sub_elems.assign(nsub, {});
  for (int32_t e = 0; e < ne; ++e) {
    const int l = g->esub[e];
    g->sub_lo[l] = std::min<int64_t>(g->sub_lo[l], 10 * (int64_t)e);
    g->sub_hi[l] = std::max<int64_t>(g->sub_hi[l], 10 * (int64_t)e + 10);
    g->sub_elems[l].push_back(e);
  }
  for (int l = 0; l < nsub; ++l)
    if (g->sub_elems[l].empty()) return setup_fail(h, LS_ERR_ARG, "a subdomain has no elements");
  g->curves.assign(nsub, {});
  for (int c = 0; c < s.n_curves; ++c) {
    const ls_curve &cv = s.curves[c];
    g->curves[cv.subdomain].push_back({cv.kind, cv.orientation, cv.subdomain, cv.cx, cv.cy, cv.a, cv.b});
  }
  sc.geom = g;
  return LS_OK;
}

// Host stage of the correction rows for nt targets: the interpolation element tau of every
// (target, subdomain) and the exact polynomial potentials E[P_a] there (Er, Ei: [nt][nsub][10]).
//   nodes = true : the targets are the scatterer's own nodes (internal order); a node's own
//                  element serves its own subdomain, it lies inside that subdomain, and the
//                  monomial sums leave out the node itself;
//   nodes = false: external targets (tx, ty), all outside the scatterer: the nearest element
//                  serves every subdomain and nothing is left out.
void correction_potentials(const GeomData &g, int threads, int64_t nt, const double *tx, const double *ty,
                           bool nodes, std::vector<int32_t> &tau, std::vector<double> &Er, std::vector<double> &Ei) {
  const int nsub = g.nsub;
  // interpolation element for each (target, subdomain): the node's own element, else the
  // nearest centroid (uniform bucket grid per subdomain; ties to the smaller caller index)
  tau.assign((size_t)nt * nsub, 0);
  for (int l = 0; l < nsub; ++l) {
    const auto &E = g.sub_elems[l];
    double bx0 = 1e300, bx1 = -1e300, by0 = 1e300, by1 = -1e300;
    for (int32_t e : E) {
      bx0 = std::min(bx0, g.ecx[e]);
      bx1 = std::max(bx1, g.ecx[e]);
      by0 = std::min(by0, g.ecy[e]);
      by1 = std::max(by1, g.ecy[e]);
    }
    const int G = std::max(1, (int)std::sqrt((double)E.size() / 2));
    const double gx = std::max(bx1 - bx0, 1e-12) / G, gy = std::max(by1 - by0, 1e-12) / G;
    std::vector<std::vector<int32_t>> bucket((size_t)G * G);
    auto cell = [&](double x, double y, int &ix, int &iy) {
      ix = std::min(G - 1, std::max(0, (int)std::floor((x - bx0) / gx)));
      iy = std::min(G - 1, std::max(0, (int)std::floor((y - by0) / gy)));
    };
    for (int32_t e : E) {
      int ix, iy;
      cell(g.ecx[e], g.ecy[e], ix, iy);
      bucket[(size_t)iy * G + ix].push_back(e);
    }
    parallel_for(nt, threads, [&](int64_t j) {
      if (nodes && g.esub[j / 10] == l) {
        tau[(size_t)j * nsub + l] = (int32_t)(j / 10);
        return;
      }
      const double xj = nodes ? g.px[j] : tx[j], yj = nodes ? g.py[j] : ty[j];
      int ix, iy;
      cell(xj, yj, ix, iy);
      double best = 1e300;
      int32_t be = -1;
      for (int r = 0; r <= 2 * G; ++r) {
        // ring r around (ix, iy); stop once the ring is farther than the best distance
        const double ringd = (r - 1) * std::min(gx, gy);
        if (be >= 0 && ringd > best) break;
        for (int dy = -r; dy <= r; ++dy)
          for (int dx = -r; dx <= r; ++dx) {
            if (std::max(std::abs(dx), std::abs(dy)) != r) continue;
            const int cx = ix + dx, cy = iy + dy;
            if (cx < 0 || cy < 0 || cx >= G || cy >= G) continue;
            for (int32_t e : bucket[(size_t)cy * G + cx]) {
              const double d = std::hypot(g.ecx[e] - xj, g.ecy[e] - yj);
              if (d < best || (d == best && g.ecaller[e] < g.ecaller[be])) {
                best = d;
                be = e;
              }
            }
          }
      }
      tau[(size_t)j * nsub + l] = be;
    });
  }
  // exact polynomial potentials (host threads)
  GaussLegendre gl;
  Er.assign((size_t)nt * nsub * NA, 0.0);
  Ei.assign((size_t)nt * nsub * NA, 0.0);
  const double k = g.k;
  parallel_for(nt * nsub, threads, [&](int64_t jl) {
    const int64_t j = jl / nsub;
    const int l = (int)(jl % nsub);
    const int32_t e = tau[(size_t)jl];
    const bool inside = nodes && g.esub[j / 10] == l;
    const double xj = nodes ? g.px[j] : tx[j], yj = nodes ? g.py[j] : ty[j];
    poly_potential(g.curves[l], inside, xj, yj, g.ecx[e], g.ecy[e], g.esc[e], k, gl, &Er[(size_t)jl * NA],
                   &Ei[(size_t)jl * NA]);
  });
}

// Host stage closing the correction rows: per (target, subdomain) the solve V^T r = E - S with
// the interpolation element's factors, S the punctured monomial sums ([nt][nsub][10] complex).
void correction_solve(const GeomData &g, int threads, int64_t nt, const std::vector<int32_t> &tau,
                      const std::vector<double> &Er, const std::vector<double> &Ei, const std::vector<double> &S,
                      std::vector<int64_t> &rp, std::vector<int32_t> &ci, std::vector<double> &cv) {
  const int nsub = g.nsub;
  rp.resize(nt + 1);
  for (int64_t j = 0; j <= nt; ++j) rp[j] = j * NA * nsub;
  ci.resize((size_t)nt * NA * nsub);
  cv.resize((size_t)nt * NA * nsub * 2);
  parallel_for(nt, threads, [&](int64_t j) {
    for (int l = 0; l < nsub; ++l) {
      const size_t jl = (size_t)j * nsub + l;
      const int32_t e = tau[jl];
      double dr[NA], di[NA];
      for (int a = 0; a < NA; ++a) {
        dr[a] = Er[jl * NA + a] - S[(jl * NA + a) * 2];
        di[a] = Ei[jl * NA + a] - S[(jl * NA + a) * 2 + 1];
      }
      lu10_solve(&g.LU[(size_t)e * NA * NA], &g.piv[(size_t)e * NA], dr);
      lu10_solve(&g.LU[(size_t)e * NA * NA], &g.piv[(size_t)e * NA], di);
      for (int i = 0; i < NA; ++i) {
        const size_t d = (size_t)rp[j] + (size_t)l * NA + i;
        ci[d] = 10 * e + i;
        cv[2 * d] = dr[i];
        cv[2 * d + 1] = di[i];
      }
    }
  });
}

namespace {

// Correction rows (10 entries per subdomain) for nt targets, in CSR form on the host: the host
// potentials, the punctured monomial sums on the GPU, and the solves with the interpolation
// matrices (nodes as for correction_potentials).
ls_status correction_rows(ls_ctx *h, const Scat &sc, int64_t nt, const double *tx, const double *ty, bool nodes,
                          hipStream_t st, std::vector<int64_t> &rp, std::vector<int32_t> &ci,
                          std::vector<double> &cv) {
  const GeomData &g = *sc.geom;
  const int nsub = g.nsub;
  int threads = host_threads(h->opt);
  threads = std::max(1, std::min(threads, 64));
  std::vector<int32_t> tau;
  std::vector<double> Er, Ei;
  correction_potentials(g, threads, nt, tx, ty, nodes, tau, Er, Ei);
  const double k = g.k;
  // monomial sums on the GPU
  std::vector<double> S((size_t)nt * nsub * NA * 2);
  {
    const int nsplit = std::max(1, std::min(16, (int)(8192 / ((nt + 63) / 64))));
    void *dframe = nullptr, *dout = nullptr, *dtgt = nullptr;
    auto release = [&]() {
      if (dframe) (void)hipFree(dframe);
      if (dout) (void)hipFree(dout);
      if (dtgt) (void)hipFree(dtgt);
    };
    if (lsk::dmalloc(&dframe, sizeof(double4) * nt) != hipSuccess ||
        lsk::dmalloc(&dout, sizeof(double2) * NA * nt * (size_t)nsplit) != hipSuccess ||
        (!nodes && lsk::dmalloc(&dtgt, sizeof(double) * 2 * nt) != hipSuccess)) {
      release();
      return setup_fail(h, LS_ERR_ALLOC, "monomial sums");
    }
    const double *dtx = sc.px, *dty = sc.py;
    hipError_t err = hipSuccess;
    if (!nodes) {
      err = hipMemcpyAsync(dtgt, tx, sizeof(double) * nt, hipMemcpyHostToDevice, st);
      if (err == hipSuccess)
        err = hipMemcpyAsync((double *)dtgt + nt, ty, sizeof(double) * nt, hipMemcpyHostToDevice, st);
      dtx = (const double *)dtgt;
      dty = (const double *)dtgt + nt;
    }
    std::vector<double> frame(4 * nt), part((size_t)NA * 2 * nt * nsplit);
    for (int l = 0; l < nsub && err == hipSuccess; ++l) {
      for (int64_t j = 0; j < nt; ++j) {
        const int32_t e = tau[(size_t)j * nsub + l];
        frame[4 * j] = g.ecx[e];
        frame[4 * j + 1] = g.ecy[e];
        frame[4 * j + 2] = 1.0 / g.esc[e];
        frame[4 * j + 3] = 0.0;
      }
      err = hipMemcpyAsync(dframe, frame.data(), sizeof(double) * 4 * nt, hipMemcpyHostToDevice, st);
      const int q0 = (int)g.sub_lo[l], q1 = (int)g.sub_hi[l];
      const int split_len = (q1 - q0 + nsplit - 1) / nsplit;
      dim3 grid((unsigned)((nt + kBlock - 1) / kBlock), (unsigned)nsplit);
      if (err == hipSuccess) {
        if (nodes)
          poly_sums_kernel<true><<<grid, kBlock, 0, st>>>((int)nt, dtx, dty, sc.pos, sc.w, q0, q1,
                                                          (const double4 *)dframe, k * k, split_len, (double2 *)dout);
        else
          poly_sums_kernel<false><<<grid, kBlock, 0, st>>>((int)nt, dtx, dty, sc.pos, sc.w, q0, q1,
                                                           (const double4 *)dframe, k * k, split_len, (double2 *)dout);
        err = hipGetLastError();
      }
      if (err == hipSuccess)
        err = hipMemcpyAsync(part.data(), dout, sizeof(double) * part.size(), hipMemcpyDeviceToHost, st);
      if (err == hipSuccess) err = hipStreamSynchronize(st);
      if (err != hipSuccess) break;
      for (int64_t j = 0; j < nt; ++j)
        for (int a = 0; a < NA; ++a) {
          double sr = 0, si = 0;
          for (int sp = 0; sp < nsplit; ++sp) {
            sr += part[(((size_t)sp * nt + j) * NA + a) * 2];
            si += part[(((size_t)sp * nt + j) * NA + a) * 2 + 1];
          }
          S[(((size_t)j * nsub + l) * NA + a) * 2] = sr;
          S[(((size_t)j * nsub + l) * NA + a) * 2 + 1] = si;
        }
    }
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    release();
    if (err != hipSuccess) return setup_fail(h, LS_ERR_HIP, hipGetErrorString(err));
  }
  correction_solve(g, threads, nt, tau, Er, Ei, S, rp, ci, cv);
  return LS_OK;
}

}  // namespace

// Build the geometry and C for scatterer sc (nodes already uploaded in internal order) and
// upload C.
ls_status build_correction(ls_ctx *h, Scat &sc, const ls_scatterer &s, const std::vector<int32_t> &eord,
                           hipStream_t st) {
  ls_status rc = build_geometry(h, sc, s, eord);
  if (rc != LS_OK) return rc;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> cv;
  rc = correction_rows(h, sc, sc.n, nullptr, nullptr, true, st, rp, ci, cv);
  if (rc != LS_OK) return rc;
  return upload_correction(h, sc, rp, ci, cv);
}

// Correction rows of field-recovery targets outside the scatterer (CSR over the scatterer's
// internal node order).
ls_status field_correction(ls_ctx *h, const Scat &sc, int64_t nt, const double *tx, const double *ty,
                           hipStream_t st, std::vector<int64_t> &rp, std::vector<int32_t> &ci,
                           std::vector<double> &cv) {
  return correction_rows(h, sc, nt, tx, ty, false, st, rp, ci, cv);
}

// True when (x, y) lies outside every curve that encloses a subdomain of the scatterer.
bool outside_scatterer(const Scat &sc, double x, double y) {
  for (const auto &cl : sc.geom->curves)
    for (const CurveH &c : cl) {
      if (c.orient != 1) continue;
      const double u = (x - c.cx) / c.a, v = (y - c.cy) / c.b;
      if (u * u + v * v <= 1.0) return false;
    }
  return true;
}

}  // namespace lsk
