// Host stages of the setup under AddressSanitizer and UndefinedBehaviorSanitizer (built by
// tests/test_host_sanitize.py with the library's sources compiled for the host only): element
// order, geometry and interpolation factors, the exact polynomial potentials by Green's identity
// on the boundary curves (threads), the interpolation solves, and the sparsifying
// preconditioner's stencils, threaded block LU and host sweeps.  No GPU call is made.
//
// Usage: host_check <scatterer file> <threads>
// The scatterer file holds, little-endian: int64 n, int32 n_elems, int32 n_curves, double k, then
// x[n], y[n], w[n], m[2n] (double), elem_subdomain[n_elems] (int32), and n_curves records of
// (int32 kind, orientation, subdomain, pad; double cx, cy, a, b).
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "host.h"

namespace {

template <class T>
bool get(std::FILE *f, T *p, size_t n) {
  return std::fread(p, sizeof(T), n, f) == n;
}

int fail(const char *msg) {
  std::fprintf(stderr, "host_check: %s\n", msg);
  return 1;
}

}  // namespace

int main(int argc, char **argv) {
  if (argc < 3) return fail("usage: host_check <scatterer file> <threads>");
  const int threads = std::atoi(argv[2]);
  std::FILE *f = std::fopen(argv[1], "rb");
  if (!f) return fail("cannot open the scatterer file");
  int64_t n = 0;
  int32_t ne = 0, nc = 0;
  double k = 0;
  bool ok = get(f, &n, 1) && get(f, &ne, 1) && get(f, &nc, 1) && get(f, &k, 1);
  if (!ok || n != 10 * (int64_t)ne || nc < 1) return fail("bad header");
  std::vector<double> x(n), y(n), w(n), m(2 * n);
  std::vector<int32_t> esub(ne);
  std::vector<ls_curve> curves(nc);
  ok = get(f, x.data(), n) && get(f, y.data(), n) && get(f, w.data(), n) && get(f, m.data(), 2 * n) &&
       get(f, esub.data(), ne) && get(f, curves.data(), nc);
  std::fclose(f);
  if (!ok) return fail("short file");
  ls_scatterer s{};
  s.n_nodes = n;
  s.n_elems = ne;
  s.nq = 10;
  s.x = x.data();
  s.y = y.data();
  s.w = w.data();
  s.elem_subdomain = esub.data();
  s.m = m.data();
  s.k = k;
  s.n_curves = nc;
  s.curves = curves.data();

  // the internal order and geometry, as the setup builds them
  const std::vector<int32_t> eord = lsk::element_order(s);
  lsk::Scat sc;
  sc.n = n;
  sc.k = k;
  int32_t nsub = 0;
  for (int32_t e = 0; e < ne; ++e) nsub = std::max(nsub, esub[e] + 1);
  sc.n_sub = nsub;
  sc.perm_host.resize(n);
  for (size_t ie = 0; ie < eord.size(); ++ie)
    for (int q = 0; q < 10; ++q) sc.perm_host[10 * ie + q] = 10 * eord[ie] + q;
  ls_ctx ctx;
  if (lsk::build_geometry(&ctx, sc, s, eord) != LS_OK) return fail(ctx.err.c_str());

  // correction rows at the nodes and at external points; the monomial sums (a GPU stage) are
  // replaced by zeros, which leaves every host step and its memory accesses as in the setup
  std::vector<int32_t> tau;
  std::vector<double> Er, Ei;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> cv;
  lsk::correction_potentials(*sc.geom, threads, n, nullptr, nullptr, true, tau, Er, Ei);
  lsk::correction_solve(*sc.geom, threads, n, tau, Er, Ei, std::vector<double>(Er.size() * 2, 0.0), rp, ci, cv);
  bool finite = rp.back() == (int64_t)ci.size() && cv.size() == 2 * ci.size();
  for (double v : Er) finite = finite && std::isfinite(v);
  for (double v : cv) finite = finite && std::isfinite(v);
  const int nt = 37;
  std::vector<double> tx(nt), ty(nt);
  double rmax = 0;
  for (int64_t i = 0; i < n; ++i) rmax = std::max(rmax, std::hypot(x[i], y[i]));
  for (int j = 0; j < nt; ++j) {
    tx[j] = 1.3 * rmax * std::cos(0.17 * j);
    ty[j] = 1.3 * rmax * std::sin(0.17 * j);
  }
  lsk::correction_potentials(*sc.geom, threads, nt, tx.data(), ty.data(), false, tau, Er, Ei);
  lsk::correction_solve(*sc.geom, threads, nt, tau, Er, Ei, std::vector<double>(Er.size() * 2, 0.0), rp, ci, cv);
  for (double v : cv) finite = finite && std::isfinite(v);
  if (!finite) return fail("non-finite correction rows");

  // sparsifying preconditioner on a 23 x 19 grid: stencils, block LU, host sweeps, and the
  // residual of C^(C) x = y through the 9-point stencil E
  const int gx = 23, gy = 19;
  const int64_t ng = (int64_t)gx * gy;
  const double h = 0.3 / k;
  std::vector<std::complex<double>> mg(ng), W, E, yv(ng), xv(ng);
  for (int64_t j = 0; j < ng; ++j) {
    const double u = (double)(j % gx) / gx - 0.5, v = (double)(j / gx) / gy - 0.5;
    mg[j] = (u * u + v * v < 0.16) ? std::complex<double>(-1.0, 0.05) : 0.0;
    yv[j] = std::complex<double>(std::cos(0.7 * j), std::sin(0.3 * j));
  }
  double ratio = 0;
  lsk::sparsify_stencil(gx, gy, h, k, mg.data(), threads, W, E, &ratio);
  std::vector<std::vector<std::complex<double>>> G;
  if (!lsk::sparsify_factor(gx, gy, E, G, threads)) return fail("singular block in the LU");
  lsk::sparsify_solve_host(gx, gy, E, G, yv.data(), xv.data());
  double num = 0, den = 0;
  for (int64_t j = 0; j < ng; ++j) {
    const int ix = (int)(j % gx), iy = (int)(j / gx);
    std::complex<double> acc = 0;
    for (int o = 0; o < 9; ++o) {
      const int dx = o % 3 - 1, dy = o / 3 - 1;
      if (ix + dx < 0 || ix + dx >= gx || iy + dy < 0 || iy + dy >= gy) continue;
      acc += E[(size_t)j * 9 + o] * xv[(size_t)(j + dx + (int64_t)dy * gx)];
    }
    num = std::max(num, std::abs(acc - yv[j]));
    den = std::max(den, std::abs(yv[j]));
  }
  std::printf("host_check: n = %lld, %d subdomains, %zu correction entries at the nodes; grid %dx%d, "
              "stencil ratio %.3e, ||C x - y|| / ||y|| = %.2e\n",
              (long long)n, nsub, (size_t)(10 * nsub) * (size_t)n, gx, gy, ratio, num / den);
  return num / den <= 1e-11 ? 0 : fail("block LU residual too large");
}
