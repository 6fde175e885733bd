// C ABI entry points: argument validation, internal node ordering, device uploads, dispatch.
#include <sched.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "host.h"
#include "internal.h"

using lsk::Scat;

namespace {

thread_local std::string g_err;   // errors raised before a handle exists

ls_status fail(ls_ctx *h, ls_status st, const std::string &msg) {
  if (h) h->err = msg;
  g_err = msg;
  return st;
}

#define HIPCHK(h, call)                                                                   \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail((h), LS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

// Allocate max(count, 1) elements on the device and copy count elements from src.
template <class T>
ls_status upload(ls_ctx *h, T **dst, const T *src, size_t count) {
  *dst = nullptr;
  void *p = nullptr;
  if (lsk::dmalloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess)
    return fail(h, LS_ERR_ALLOC, "hipMalloc failed");
  h->owned.push_back(p);
  *dst = (T *)p;
  if (src && count) HIPCHK(h, hipMemcpy(p, src, count * sizeof(T), hipMemcpyHostToDevice));
  return LS_OK;
}

// Hilbert-curve index of (x, y) on a 2^16 x 2^16 grid.
uint64_t hilbert_index(uint32_t x, uint32_t y) {
  const uint32_t n = 1u << 16;
  uint64_t d = 0;
  for (uint32_t s = n / 2; s > 0; s /= 2) {
    const uint32_t rx = (x & s) ? 1u : 0u;
    const uint32_t ry = (y & s) ? 1u : 0u;
    d += (uint64_t)s * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = n - 1 - x;
        y = n - 1 - y;
      }
      std::swap(x, y);
    }
  }
  return d;
}

ls_status validate_scatterer(const ls_scatterer &s) {
  if (s.n_nodes <= 0 || s.nq != 10 || s.n_elems <= 0 || (int64_t)s.n_elems * 10 != s.n_nodes)
    return fail(nullptr, LS_ERR_ARG, "scatterer: need nq = 10 and n_nodes = 10 * n_elems > 0");
  if (s.n_nodes > (int64_t)INT32_MAX / 2) return fail(nullptr, LS_ERR_ARG, "scatterer: too many nodes");
  if (!s.x || !s.y || !s.w || !s.m || !s.elem_subdomain)
    return fail(nullptr, LS_ERR_ARG, "scatterer: null array");
  if (!(s.k > 0) || !std::isfinite(s.k)) return fail(nullptr, LS_ERR_ARG, "scatterer: k must be > 0");
  for (int64_t i = 0; i < s.n_nodes; ++i)
    if (!std::isfinite(s.x[i]) || !std::isfinite(s.y[i]) || !std::isfinite(s.w[i]) ||
        !std::isfinite(s.m[2 * i]) || !std::isfinite(s.m[2 * i + 1]))
      return fail(nullptr, LS_ERR_NONFINITE, "scatterer: non-finite node data");
  int32_t nsub = 0;
  for (int32_t e = 0; e < s.n_elems; ++e) {
    if (s.elem_subdomain[e] < 0) return fail(nullptr, LS_ERR_ARG, "scatterer: negative subdomain");
    nsub = std::max(nsub, s.elem_subdomain[e] + 1);
  }
  if (s.n_curves < 0 || (s.n_curves > 0 && !s.curves))
    return fail(nullptr, LS_ERR_ARG, "scatterer: bad curve list");
  for (int32_t c = 0; c < s.n_curves; ++c) {
    const ls_curve &cv = s.curves[c];
    if ((cv.kind != LS_CIRCLE && cv.kind != LS_ELLIPSE) || (cv.orientation != 1 && cv.orientation != -1) ||
        cv.subdomain < 0 || cv.subdomain >= nsub || !(cv.a > 0) || !(cv.b > 0))
      return fail(nullptr, LS_ERR_ARG, "scatterer: bad curve");
  }
  return LS_OK;
}

}  // namespace

namespace lsk {

ls_status setup_fail(ls_ctx *h, ls_status st, const char *msg) { return fail(h, st, msg); }
ls_status resolve_scratch(ls_ctx *h);
ls_status build_correction(ls_ctx *h, Scat &sc, const ls_scatterer &s, const std::vector<int32_t> &eord,
                           hipStream_t st);

// Element order: by subdomain, then along a Hilbert curve through element centroids.
std::vector<int32_t> element_order(const ls_scatterer &s) {
  const int32_t ne = s.n_elems;
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  std::vector<double> cx(ne), cy(ne);
  for (int32_t e = 0; e < ne; ++e) {
    double ax = 0, ay = 0;
    for (int q = 0; q < 10; ++q) {
      ax += s.x[10 * (int64_t)e + q];
      ay += s.y[10 * (int64_t)e + q];
    }
    cx[e] = ax / 10;
    cy[e] = ay / 10;
    x0 = std::min(x0, cx[e]);
    x1 = std::max(x1, cx[e]);
    y0 = std::min(y0, cy[e]);
    y1 = std::max(y1, cy[e]);
  }
  const double span = std::max(std::max(x1 - x0, y1 - y0), 1e-300);
  std::vector<uint64_t> key(ne);
  for (int32_t e = 0; e < ne; ++e) {
    const uint32_t gx = (uint32_t)std::min(65535.0, std::floor((cx[e] - x0) / span * 65535.0));
    const uint32_t gy = (uint32_t)std::min(65535.0, std::floor((cy[e] - y0) / span * 65535.0));
    key[e] = ((uint64_t)s.elem_subdomain[e] << 40) | hilbert_index(gx, gy);
  }
  std::vector<int32_t> ord(ne);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  return ord;
}

// Upload one scatterer's node data in internal order; fills perm and the geometry arrays.
ls_status upload_nodes(ls_ctx *h, Scat &sc, const ls_scatterer &s, const std::vector<int32_t> &eord) {
  const int64_t n = s.n_nodes;
  sc.n = n;
  sc.k = s.k;
  sc.perm_host.resize(n);
  std::vector<double> px(n), py(n), w(n), m(2 * n), pos(2 * n);
  int32_t nsub = 0;
  for (int32_t e = 0; e < s.n_elems; ++e) nsub = std::max(nsub, s.elem_subdomain[e] + 1);
  sc.n_sub = nsub;
  for (size_t ie = 0; ie < eord.size(); ++ie)
    for (int q = 0; q < 10; ++q) {
      const int64_t i = 10 * (int64_t)ie + q;
      const int64_t c = 10 * (int64_t)eord[ie] + q;
      sc.perm_host[i] = (int32_t)c;
      px[i] = s.x[c];
      py[i] = s.y[c];
      w[i] = s.w[c];
      m[2 * i] = s.m[2 * c];
      m[2 * i + 1] = s.m[2 * c + 1];
      pos[2 * i] = px[i];
      pos[2 * i + 1] = py[i];
    }
  sc.w_host = w;
  ls_status st;
  if ((st = upload(h, &sc.px, px.data(), n)) != LS_OK) return st;
  if ((st = upload(h, &sc.py, py.data(), n)) != LS_OK) return st;
  if ((st = upload(h, &sc.w, w.data(), n)) != LS_OK) return st;
  if ((st = upload(h, (double **)&sc.m, m.data(), 2 * n)) != LS_OK) return st;
  if ((st = upload(h, (double **)&sc.pos, pos.data(), 2 * n)) != LS_OK) return st;
  if ((st = upload(h, &sc.perm, sc.perm_host.data(), n)) != LS_OK) return st;
  return LS_OK;
}

// Upload C (internal order, CSR) and build/upload C^H.
// Source intervals of the FP64 near launch of scatterer sc (mixed-precision applications): for
// every tile of 16 consecutive targets (internal order), 4-aligned index intervals [begin, end)
// that hold every source n != j with z = k |y_j - y_n| < 1 of its targets j.  The pairs are
// classified with the far kernels' own A = k^2 fma(dx, dx, dy dy) < 1 test (the near launch and
// the mixed tiles apply the same test to the same FP64 positions, so each pair is taken exactly
// once).  Sources of one tile closer than 16 in the node order share an interval.  Skipped
// (near_ok false) when the options keep the pairs in the tiles or they exceed kNearPerNode per node.
ls_status build_near_lists(ls_ctx *h, Scat &sc) {
#pragma clang fp contract(off)
  sc.near_ok = false;
  sc.near_pairs = 0;
  if (h->opt.mixed_near == 1) return LS_OK;
  const int64_t n = sc.n;
  const double *px = geom_x(sc), *py = geom_y(sc);
  if (!px || !py || n < 2) return LS_OK;
  const double k = sc.k, k2 = k * k;
  // buckets of side 1 / k (slightly more): a pair with z < 1 lies in neighbouring buckets
  double x0 = px[0], x1 = px[0], y0 = py[0], y1 = py[0];
  for (int64_t i = 1; i < n; ++i) {
    x0 = std::min(x0, px[i]);
    x1 = std::max(x1, px[i]);
    y0 = std::min(y0, py[i]);
    y1 = std::max(y1, py[i]);
  }
  const double cell = 1.0001 / k;
  const double gxd = std::floor((x1 - x0) / cell) + 1, gyd = std::floor((y1 - y0) / cell) + 1;
  if (gxd * gyd > 16.0 * (double)n + 1e6) return LS_OK;   // a mesh coarse against 1 / k: hardly any pair
  const int64_t gx = (int64_t)gxd, gy = (int64_t)gyd;
  auto bucket_of = [&](double x, double y, int64_t &bx, int64_t &by) {
    bx = std::min(gx - 1, std::max<int64_t>(0, (int64_t)std::floor((x - x0) / cell)));
    by = std::min(gy - 1, std::max<int64_t>(0, (int64_t)std::floor((y - y0) / cell)));
  };
  std::vector<int64_t> bstart(gx * gy + 1, 0);
  std::vector<int32_t> border(n);
  for (int64_t i = 0; i < n; ++i) {
    int64_t bx, by;
    bucket_of(px[i], py[i], bx, by);
    ++bstart[by * gx + bx + 1];
  }
  for (int64_t b = 0; b < gx * gy; ++b) bstart[b + 1] += bstart[b];
  {
    std::vector<int64_t> fill(bstart.begin(), bstart.end() - 1);
    for (int64_t i = 0; i < n; ++i) {
      int64_t bx, by;
      bucket_of(px[i], py[i], bx, by);
      border[fill[by * gx + bx]++] = (int32_t)i;
    }
  }
  const int32_t ntiles = (int32_t)((n + 15) / 16);
  std::vector<std::vector<int2>> tiv(ntiles);
  std::vector<int64_t> tpairs(ntiles, 0);
  const int threads = std::max(1, std::min(host_threads(h->opt), 64));
  std::vector<std::thread> pool;
  std::atomic<int32_t> next(0);
  for (int th = 0; th < threads; ++th)
    pool.emplace_back([&]() {
      std::vector<int32_t> src;
      for (;;) {
        const int32_t t = next.fetch_add(16);
        if (t >= ntiles) break;
        for (int32_t tile = t; tile < std::min(ntiles, t + 16); ++tile) {
          src.clear();
          for (int64_t j = 16 * (int64_t)tile; j < std::min(n, 16 * (int64_t)tile + 16); ++j) {
            int64_t bx, by;
            bucket_of(px[j], py[j], bx, by);
            for (int64_t yb = std::max<int64_t>(0, by - 1); yb <= std::min(gy - 1, by + 1); ++yb)
              for (int64_t xb = std::max<int64_t>(0, bx - 1); xb <= std::min(gx - 1, bx + 1); ++xb)
                for (int64_t q = bstart[yb * gx + xb]; q < bstart[yb * gx + xb + 1]; ++q) {
                  const int32_t c = border[q];
                  if (c == j) continue;
                  const double dx = px[j] - px[c], dy = py[j] - py[c];
                  if (k2 * std::fma(dx, dx, dy * dy) < 1.0) {
                    src.push_back(c);
                    ++tpairs[tile];
                  }
                }
          }
          std::sort(src.begin(), src.end());
          src.erase(std::unique(src.begin(), src.end()), src.end());
          for (size_t e = 0; e < src.size();) {
            int64_t b = src[e] / 4 * 4, end = src[e] + 1;
            size_t f = e + 1;
            while (f < src.size() && src[f] < end + 16) end = src[f++] + 1;
            tiv[tile].push_back(make_int2((int)b, (int)std::min<int64_t>(n, (end + 3) / 4 * 4)));
            e = f;
          }
        }
      }
    });
  for (auto &t : pool) t.join();
  int64_t pairs = 0, niv = 0;
  for (int32_t t = 0; t < ntiles; ++t) {
    pairs += tpairs[t];
    niv += (int64_t)tiv[t].size();
  }
  if (pairs > Scat::kNearPerNode * n) return LS_OK;
  std::vector<int32_t> rp(ntiles + 1, 0);
  std::vector<int2> iv;
  iv.reserve(niv);
  for (int32_t t = 0; t < ntiles; ++t) {
    iv.insert(iv.end(), tiv[t].begin(), tiv[t].end());
    rp[t + 1] = (int32_t)iv.size();
  }
  ls_status st;
  if ((st = upload(h, &sc.near_rp, rp.data(), rp.size())) != LS_OK) return st;
  if ((st = upload(h, &sc.near_iv, iv.empty() ? nullptr : iv.data(), iv.size())) != LS_OK) return st;
  sc.near_ntiles = ntiles;
  sc.near_pairs = pairs;
  sc.near_ok = true;
  return LS_OK;
}

ls_status upload_correction(ls_ctx *h, Scat &sc, const std::vector<int64_t> &rp, const std::vector<int32_t> &ci,
                            const std::vector<double> &cv) {
  const int64_t n = sc.n, nnz = rp[n];
  sc.nnz = nnz;
  std::vector<int64_t> rpH(n + 1, 0);
  for (int64_t q = 0; q < nnz; ++q) rpH[ci[q] + 1]++;
  for (int64_t i = 0; i < n; ++i) rpH[i + 1] += rpH[i];
  std::vector<int32_t> ciH(nnz);
  std::vector<double> cvH(2 * nnz);
  std::vector<int64_t> fill(rpH.begin(), rpH.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
      const int64_t d = fill[ci[q]]++;
      ciH[d] = (int32_t)i;
      cvH[2 * d] = cv[2 * q];
      cvH[2 * d + 1] = -cv[2 * q + 1];
    }
  ls_status st;
  if ((st = upload(h, &sc.rp, rp.data(), n + 1)) != LS_OK) return st;
  if ((st = upload(h, &sc.ci, ci.data(), nnz)) != LS_OK) return st;
  if ((st = upload(h, (double **)&sc.cv, cv.data(), 2 * nnz)) != LS_OK) return st;
  if ((st = upload(h, &sc.rpH, rpH.data(), n + 1)) != LS_OK) return st;
  if ((st = upload(h, &sc.ciH, ciH.data(), nnz)) != LS_OK) return st;
  if ((st = upload(h, (double **)&sc.cvH, cvH.data(), 2 * nnz)) != LS_OK) return st;
  return build_near_lists(h, sc);
}

}  // namespace lsk

extern "C" {

const char *ls_status_str(ls_status s) {
  switch (s) {
    case LS_OK: return "ok";
    case LS_NOT_CONVERGED: return "not converged";
    case LS_ERR_ARG: return "invalid argument";
    case LS_ERR_HIP: return "HIP runtime error";
    case LS_ERR_ALLOC: return "allocation failed";
    case LS_ERR_BREAKDOWN: return "Krylov breakdown";
    case LS_ERR_NONFINITE: return "non-finite input";
    case LS_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char *ls_last_error(ls_handle h) { return h ? h->err.c_str() : g_err.c_str(); }

void ls_destroy(ls_handle h) {
  if (!h) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  for (void *p : h->owned) (void)hipFree(p);
  if (h->ws_apply.ptr) (void)hipFree(h->ws_apply.ptr);
  if (h->ws_ff.ptr) (void)hipFree(h->ws_ff.ptr);
  if (h->ws_grid.ptr) (void)hipFree(h->ws_grid.ptr);
  if (h->batch_tables) (void)hipFree(h->batch_tables);
  lsk::free_solve_ws(h);
  for (hipEvent_t e : h->ev_far) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->ev_apply) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->aux_join) (void)hipEventDestroy(e);
  if (h->aux_fork) (void)hipEventDestroy(h->aux_fork);
  for (hipStream_t q : h->aux_streams) (void)hipStreamDestroy(q);
  (void)hipSetDevice(cur);
  delete h;
}

ls_status ls_setup(const ls_scatterer *s, int32_t n_scatterers, const ls_options *opt, ls_handle *out) {
  if (!out) return fail(nullptr, LS_ERR_ARG, "out is null");
  *out = nullptr;
  if (!s || n_scatterers <= 0) return fail(nullptr, LS_ERR_ARG, "need at least one scatterer");
  for (int32_t i = 0; i < n_scatterers; ++i) {
    ls_status st = validate_scatterer(s[i]);
    if (st != LS_OK) return st;
    if (s[i].n_curves == 0) return fail(nullptr, LS_ERR_ARG, "ls_setup needs the boundary curves");
  }
  int64_t total = 0;
  for (int32_t i = 0; i < n_scatterers; ++i) total += s[i].n_nodes;
  if (total > (int64_t)INT32_MAX / 2) return fail(nullptr, LS_ERR_ARG, "too many nodes in total");
  ls_ctx *h = new ls_ctx();
  if (opt) h->opt = *opt;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return fail(nullptr, LS_ERR_HIP, "hipGetDevice failed");
  }
  hipStream_t st = nullptr;
  if (hipStreamCreate(&st) != hipSuccess) {
    delete h;
    return fail(nullptr, LS_ERR_HIP, "hipStreamCreate failed");
  }
  h->sc.resize(n_scatterers);
  int64_t off = 0;
  ls_status rc = LS_OK;
  for (int32_t i = 0; i < n_scatterers && rc == LS_OK; ++i) {
    Scat &sc = h->sc[i];
    sc.off = off;
    off += s[i].n_nodes;
    const std::vector<int32_t> eord = lsk::element_order(s[i]);
    rc = lsk::upload_nodes(h, sc, s[i], eord);
    if (rc == LS_OK) rc = lsk::build_correction(h, sc, s[i], eord, st);
  }
  (void)hipStreamDestroy(st);
  h->n_total = off;
  if (rc == LS_OK) rc = lsk::resolve_scratch(h);
  if (rc != LS_OK) {
    g_err = h->err;
    ls_destroy(h);
    return rc;
  }
  *out = h;
  return LS_OK;
}

ls_status ls_setup_from_csr(const ls_scatterer *s, const int64_t *rowptr, const int32_t *col, const double *val,
                            const ls_options *opt, ls_handle *out) {
  if (!out) return fail(nullptr, LS_ERR_ARG, "out is null");
  *out = nullptr;
  if (!s || !rowptr || (!col && rowptr[s->n_nodes] > 0) || (!val && rowptr[s->n_nodes] > 0))
    return fail(nullptr, LS_ERR_ARG, "null argument");
  ls_status st = validate_scatterer(*s);
  if (st != LS_OK) return st;
  const int64_t n = s->n_nodes;
  if (rowptr[0] != 0) return fail(nullptr, LS_ERR_ARG, "rowptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return fail(nullptr, LS_ERR_ARG, "rowptr not monotone");
  const int64_t nnz = rowptr[n];
  for (int64_t q = 0; q < nnz; ++q) {
    if (col[q] < 0 || col[q] >= n) return fail(nullptr, LS_ERR_ARG, "column index out of range");
    if (!std::isfinite(val[2 * q]) || !std::isfinite(val[2 * q + 1]))
      return fail(nullptr, LS_ERR_NONFINITE, "non-finite correction value");
  }
  ls_ctx *h = new ls_ctx();
  if (opt) h->opt = *opt;
  HIPCHK(nullptr, hipGetDevice(&h->device));
  h->sc.resize(1);
  Scat &sc = h->sc[0];
  sc.off = 0;
  h->n_total = n;
  const std::vector<int32_t> eord = lsk::element_order(*s);
  if ((st = lsk::upload_nodes(h, sc, *s, eord)) != LS_OK || (st = lsk::build_geometry(h, sc, *s, eord)) != LS_OK) {
    ls_destroy(h);
    return st;
  }
  std::vector<int32_t> inv(n);
  for (int64_t i = 0; i < n; ++i) inv[sc.perm_host[i]] = (int32_t)i;
  std::vector<int64_t> rp(n + 1, 0);
  std::vector<int32_t> ci(nnz);
  std::vector<double> cv(2 * nnz);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t r = sc.perm_host[i];
    rp[i + 1] = rp[i] + (rowptr[r + 1] - rowptr[r]);
    int64_t d = rp[i];
    for (int64_t q = rowptr[r]; q < rowptr[r + 1]; ++q, ++d) {
      ci[d] = inv[col[q]];
      cv[2 * d] = val[2 * q];
      cv[2 * d + 1] = val[2 * q + 1];
    }
  }
  if ((st = lsk::upload_correction(h, sc, rp, ci, cv)) != LS_OK || (st = lsk::resolve_scratch(h)) != LS_OK) {
    g_err = h->err;
    ls_destroy(h);
    return st;
  }
  *out = h;
  return LS_OK;
}

}  // extern "C"

namespace lsk {

namespace {
std::atomic<int64_t> g_device_allocations{0};

// The workspace of ls_apply_noalloc: a static device array, so that application allocates
// nothing.  In host code its name stands for a host-side symbol; its address on a device comes
// from hipGetSymbolAddress (resolved once per device by ls_setup, with that device current).
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kScratchBytes];
std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;   // per device ordinal
}  // namespace

// Resolves the address of the static workspace on the current device (once per device).
ls_status resolve_scratch(ls_ctx *h) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (h->device < 0) return fail(h, LS_ERR_HIP, "no device");
  if ((int)g_scratch_ptr.size() <= h->device) g_scratch_ptr.resize(h->device + 1, nullptr);
  if (g_scratch_ptr[h->device]) return LS_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return fail(h, LS_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
  g_scratch_ptr[h->device] = p;
  return LS_OK;
}

void *scratch_on(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && device < (int)g_scratch_ptr.size() ? g_scratch_ptr[device] : nullptr;
}

void count_device_allocation() { g_device_allocations.fetch_add(1, std::memory_order_relaxed); }

int host_threads(const ls_options &opt) {
  if (opt.n_threads_host > 0) return opt.n_threads_host;
  cpu_set_t set;
  int n = 0;
  if (sched_getaffinity(0, sizeof(set), &set) == 0) n = CPU_COUNT(&set);
  if (n <= 0) n = (int)std::thread::hardware_concurrency();
  return std::max(1, std::min(n, 16));
}

// How an application of nrhs columns in precision p runs: FP32 tiles (mixed), FP64 tiles
// (batched FP64 on the matrix cores) or the FP64 VALU sum, one persistent launch over several
// scatterers on the matrix cores, and the workspace it needs.
struct ApplyPlan {
  bool single, tiles, batch, h16;
  int tpl, chunk, bmt, bsplit;
  size_t need;
};

int plan_splits(const ls_ctx *h, const ApplyPlan &pl, const Scat &sc, int nrhs) {
  if (h->opt.source_split > 0) return h->opt.source_split;
  if (pl.tiles) return lsk::tile_source_split(sc.n, nrhs, pl.single);
  // one right-hand side, one target per lane: the sum over unordered pairs, one split per block,
  // once its nb (nb + 1) / 2 workgroups fill the chip several times over (N above ~16 000; at
  // N = 2 500 its 55 workgroups left most of the chip idle: 12.7 ms per solve of the unit disk at
  // k = 2 pi against 8.7 ms with the ordered-pair sum's source splits)
  if (nrhs == 1 && pl.tpl == 1) {
    const int64_t nb = lsk::fp64_sym_splits(sc.n);
    if (nb * (nb + 1) / 2 >= 2048) return (int)nb;
  }
  return lsk::auto_source_split(sc.n, nrhs, std::max(1, nrhs / pl.chunk), pl.tpl);
}

ApplyPlan apply_plan(const ls_ctx *h, int nrhs, ls_precision p) {
  ApplyPlan pl;
  pl.single = p == LS_MIXED;
  // FP64 on the matrix cores from 4 right-hand sides on: the VALU sum evaluates G once per pass of
  // rhs_chunk columns, the tiles once for all (16 scatterers, 8 columns: 374 -> 78 ms)
  pl.tiles = pl.single || h->opt.fp64_matrix == 2 || (h->opt.fp64_matrix == 0 && nrhs >= 4);
  pl.tpl = h->opt.targets_per_lane == 2 ? 2 : 1;
  pl.chunk = h->opt.rhs_chunk > 0 ? h->opt.rhs_chunk : 1;
  // mixed precision on split FP16 (one launch per scatterer) where a wave holds a 64-column group,
  // unless the option asks otherwise (1: always, 2: never)
  pl.h16 = pl.single && (h->opt.mixed_fp16 == 1 ||
                         (h->opt.mixed_fp16 == 0 && h->sc.size() == 1 && lsk::tile_ldx(nrhs) % 64 == 0));
  pl.batch = pl.tiles && h->sc.size() > 1 && !pl.h16;
  const lsk::TileTune &tt = h->tune[pl.single ? 1 : 0];
  pl.bmt = h->opt.mixed_tile > 0 ? h->opt.mixed_tile : (tt.mt > 0 ? tt.mt : lsk::tile_mt(nrhs, pl.single));
  pl.bsplit = tt.split_len > 0 ? tt.split_len : lsk::batch_default_split_len(h, pl.single);
  pl.need = 0;
  if (pl.batch) pl.need = lsk::batch_workspace_bytes(h, nrhs, pl.single, pl.bsplit);
  else
    for (const Scat &sc : h->sc) {
      const int nsplit = plan_splits(h, pl, sc, nrhs);
      // the mixed tiles' partial sums have one more split for the FP64 near launch
      const int near = (pl.single && sc.near_ok) ? 1 : 0;
      pl.need = std::max(pl.need, pl.h16     ? lsk::tile_h_workspace_bytes(sc.n, nrhs, nsplit)
                                  : pl.tiles ? lsk::tile_workspace_bytes(sc.n, nrhs, nsplit + near)
                                             : lsk::apply_workspace_bytes(sc.n, nrhs, nsplit));
    }
  return pl;
}

// Operator application without argument checks (callers validate).
ls_status apply_op(ls_ctx *h, const double *x, double *y, int nrhs, int64_t ld, Mode mode, ls_precision p,
                   hipStream_t stream, bool may_grow) {
  const ApplyPlan pl = apply_plan(h, nrhs, p);
  const bool single = pl.single, tiles = pl.tiles, batch = pl.batch;
  const int tpl = pl.tpl, chunk = pl.chunk, bmt = pl.bmt, bsplit = pl.bsplit;
  const size_t need = pl.need;
  if (need > h->ws_apply.bytes && !may_grow)
    return fail(h, LS_ERR_ARG, "the workspace is smaller than this application needs: call ls_reserve first");
  if (need > h->ws_apply.bytes) {
    if (h->ws_apply.ptr) {
      HIPCHK(h, hipStreamSynchronize(stream));
      HIPCHK(h, hipFree(h->ws_apply.ptr));
      h->ws_apply.ptr = nullptr;
      h->ws_apply.bytes = 0;
    }
    if (lsk::dmalloc(&h->ws_apply.ptr, need) != hipSuccess) return fail(h, LS_ERR_ALLOC, "workspace allocation failed");
    h->ws_apply.bytes = need;
  }
  hipEvent_t a0 = nullptr, a1 = nullptr;
  if (h->prof) {
    for (size_t si = 0; si < h->sc.size(); ++si)
      if (h->scat_skip.empty() || !h->scat_skip[si]) {
        const double pr = (double)h->sc[si].n * (double)(h->sc[si].n - 1) * nrhs;
        h->prof_pairs += pr;
        if (single) h->prof_pairs_mixed += pr;
        if (pl.h16) h->prof_pairs_h16 += pr;
      }
    HIPCHK(h, hipEventCreate(&a0));
    HIPCHK(h, hipEventCreate(&a1));
    HIPCHK(h, hipEventRecord(a0, stream));
  }
  if (batch) {
    hipEvent_t f0 = nullptr, f1 = nullptr;
    if (h->prof) {
      HIPCHK(h, hipEventCreate(&f0));
      HIPCHK(h, hipEventCreate(&f1));
      h->ev_far.push_back(f0);
      h->ev_far.push_back(f1);
      h->ev_far_mixed.push_back(single ? 1 : 0);
    }
    const hipError_t eb = lsk::launch_apply_batch(h, x, y, nrhs, ld, mode, single, bmt, bsplit, h->ws_apply.ptr,
                                                  stream, f0, f1, false, may_grow);
    if (eb == hipErrorOutOfMemory && !may_grow)
      return fail(h, LS_ERR_ARG, "the batch tables are smaller than this application needs: call ls_reserve first");
    HIPCHK(h, eb);
  }
  for (size_t si = 0; si < h->sc.size() && !batch; ++si) {
    if (!h->scat_skip.empty() && h->scat_skip[si]) continue;
    const Scat &sc = h->sc[si];
    const int nsplit = plan_splits(h, pl, sc, nrhs);
    hipEvent_t f0 = nullptr, f1 = nullptr;
    if (h->prof) {
      HIPCHK(h, hipEventCreate(&f0));
      HIPCHK(h, hipEventCreate(&f1));
      h->ev_far.push_back(f0);
      h->ev_far.push_back(f1);
      h->ev_far_mixed.push_back(pl.h16 ? 2 : (single ? 1 : 0));
    }
    if (pl.h16)
      HIPCHK(h, lsk::launch_apply_tile_h(sc, x, y, nrhs, ld, mode, nsplit, h->ws_apply.ptr, stream, f0, f1));
    else if (tiles)
      HIPCHK(h, lsk::launch_apply_tile(sc, x, y, nrhs, ld, mode, single, nsplit, h->ws_apply.ptr, stream, f0, f1));
    else
      HIPCHK(h, lsk::launch_apply_fp64(sc, x, y, nrhs, ld, mode, nsplit, chunk, tpl, h->ws_apply.ptr, stream, f0,
                                       f1));
  }
  if (h->prof) {
    HIPCHK(h, hipEventRecord(a1, stream));
    h->ev_apply.push_back(a0);
    h->ev_apply.push_back(a1);
  }
  return LS_OK;
}

}  // namespace lsk

extern "C" {

static ls_status apply_common(ls_handle h, const double *x, double *y, int32_t nrhs, int64_t ld, ls_precision p,
                              hipStream_t stream, lsk::Mode mode) {
  if (!h) return fail(nullptr, LS_ERR_ARG, "null handle");
  if (nrhs < 0) return fail(h, LS_ERR_ARG, "nrhs < 0");
  if (nrhs == 0) return LS_OK;
  if (!x || !y) return fail(h, LS_ERR_ARG, "null vector");
  if (x == y) return fail(h, LS_ERR_ARG, "x and y must not alias");
  if (ld < h->n_total) return fail(h, LS_ERR_ARG, "ld < number of nodes");
  if (p != LS_FP64 && p != LS_MIXED) return fail(h, LS_ERR_ARG, "bad precision");
  return lsk::apply_op(h, x, y, nrhs, ld, mode, p, stream, false);
}

ls_status ls_reserve(ls_handle h, int32_t nrhs, ls_precision p) {
  if (!h) return fail(nullptr, LS_ERR_ARG, "null handle");
  if (nrhs < 0 || nrhs > 65535) return fail(h, LS_ERR_ARG, "bad nrhs");
  if (p != LS_FP64 && p != LS_MIXED) return fail(h, LS_ERR_ARG, "bad precision");
  if (nrhs == 0) return LS_OK;
  const lsk::ApplyPlan pl = lsk::apply_plan(h, nrhs, p);
  if (pl.need > h->ws_apply.bytes) {
    HIPCHK(h, hipDeviceSynchronize());   // an earlier application may still use the old workspace
    if (h->ws_apply.ptr) HIPCHK(h, hipFree(h->ws_apply.ptr));
    h->ws_apply.ptr = nullptr;
    h->ws_apply.bytes = 0;
    if (lsk::dmalloc(&h->ws_apply.ptr, pl.need) != hipSuccess) return fail(h, LS_ERR_ALLOC, "workspace allocation failed");
    h->ws_apply.bytes = pl.need;
    h->batch_key = -1;
  }
  if (pl.batch) HIPCHK(h, lsk::reserve_batch_tables(h, nrhs, pl.single, pl.bmt, pl.bsplit));
  return LS_OK;
}

int64_t ls_device_allocations(void) { return lsk::g_device_allocations.load(); }

ls_status ls_apply_noalloc(ls_handle h, const double *x, double *y, int32_t nrhs, int64_t ld, ls_precision p,
                           hipStream_t stream) {
  if (!h) return fail(nullptr, LS_ERR_ARG, "null handle");
  if (nrhs < 0) return fail(h, LS_ERR_ARG, "nrhs < 0");
  if (nrhs == 0) return LS_OK;
  if (!x || !y) return fail(h, LS_ERR_ARG, "null vector");
  if (x == y) return fail(h, LS_ERR_ARG, "x and y must not alias");
  if (ld < h->n_total) return fail(h, LS_ERR_ARG, "ld < number of nodes");
  if (p != LS_FP64 && p != LS_MIXED) return fail(h, LS_ERR_ARG, "bad precision");
  void *ws = lsk::scratch_on(h->device);
  if (!ws) return fail(h, LS_ERR_HIP, "the allocation-free workspace is not resolved on this device");
  // each scatterer by itself (tile or VALU kernel) with as many source splits as the workspace
  // holds, at most the ones ls_apply takes; every size is checked before anything is enqueued
  lsk::ApplyPlan pl = lsk::apply_plan(h, nrhs, p);
  pl.batch = false;
  const size_t cap = lsk::kScratchBytes;
  std::vector<int> nsplit(h->sc.size());
  for (size_t si = 0; si < h->sc.size(); ++si) {
    const Scat &sc = h->sc[si];
    const size_t col = sizeof(double2) * (size_t)sc.n * nrhs;   // one [nrhs][n] complex block
    // blocks besides the far splits: f, and the FP64 near launch's split of mixed applications
    const int64_t extra = 1 + ((pl.single && sc.near_ok) ? 1 : 0);
    int64_t fit;
    if (pl.h16) {
      const size_t fixed = 2 * 6 * (size_t)((sc.n + 31) / 32 * 32) * lsk::tile_ldx(nrhs) + 16 * (size_t)lsk::tile_ldx(nrhs) + 1024;
      fit = cap > fixed ? (int64_t)((cap - fixed) / col) - extra : -1;
    } else if (pl.tiles) {
      const size_t fixed = sizeof(double2) * (size_t)sc.n * lsk::tile_ldx(nrhs) + 512;
      fit = cap > fixed ? (int64_t)((cap - fixed) / col) - extra : -1;
    } else {
      fit = cap > 256 ? (int64_t)((cap - 256) / col) - 2 : -1;
    }
    if (fit < 1)
      return fail(h, LS_ERR_ARG, "nrhs x nodes too large for the 64 MiB allocation-free workspace (scatterer " +
                                     std::to_string(si) + ", " + std::to_string(sc.n) + " nodes, " +
                                     std::to_string(nrhs) + " columns)");
    nsplit[si] = (int)std::min<int64_t>(lsk::plan_splits(h, pl, sc, nrhs), fit);
  }
  for (size_t si = 0; si < h->sc.size(); ++si) {
    const Scat &sc = h->sc[si];
    if (pl.h16)
      HIPCHK(h, lsk::launch_apply_tile_h(sc, x, y, nrhs, ld, lsk::Mode::Forward, nsplit[si], ws, stream, nullptr,
                                         nullptr));
    else if (pl.tiles)
      HIPCHK(h, lsk::launch_apply_tile(sc, x, y, nrhs, ld, lsk::Mode::Forward, pl.single, nsplit[si], ws, stream,
                                       nullptr, nullptr));
    else
      HIPCHK(h, lsk::launch_apply_fp64(sc, x, y, nrhs, ld, lsk::Mode::Forward, nsplit[si], pl.chunk, pl.tpl, ws,
                                       stream));
  }
  return LS_OK;
}

ls_status ls_solve_gmres(ls_handle h, const double *b, double *x, int32_t nrhs, int64_t ld, const ls_solve_opts *o,
                         ls_solve_info *info, hipStream_t stream) {
  if (!h) return fail(nullptr, LS_ERR_ARG, "null handle");
  if (!o) return fail(h, LS_ERR_ARG, "null options");
  if (nrhs < 0) return fail(h, LS_ERR_ARG, "nrhs < 0");
  if (nrhs == 0) return LS_OK;
  if (!b || !x) return fail(h, LS_ERR_ARG, "null vector");
  if (b == x) return fail(h, LS_ERR_ARG, "b and x must not alias");
  if (ld < h->n_total) return fail(h, LS_ERR_ARG, "ld < number of nodes");
  if (!(o->tol > 0) || !std::isfinite(o->tol)) return fail(h, LS_ERR_ARG, "tol must be > 0");
  if (o->maxit < 1) return fail(h, LS_ERR_ARG, "maxit must be >= 1");
  if (o->restart < 0) return fail(h, LS_ERR_ARG, "restart < 0");
  if (o->prec != LS_FP64 && o->prec != LS_MIXED) return fail(h, LS_ERR_ARG, "bad precision");
  return lsk::solve_gmres(h, b, x, nrhs, ld, *o, info, stream);
}

ls_status ls_solve_gmres_precond(ls_handle h, const double *b, double *x, int32_t nrhs, int64_t ld,
                                 const ls_solve_opts *o, int32_t s, ls_grid_op S, void *user, double *c, double *sc,
                                 int64_t ldc, ls_solve_info *info, hipStream_t stream) {
  if (!h) return fail(nullptr, LS_ERR_ARG, "null handle");
  if (!o) return fail(h, LS_ERR_ARG, "null options");
  if (nrhs < 0 || nrhs > 65535) return fail(h, LS_ERR_ARG, "bad nrhs");
  if (nrhs == 0) return LS_OK;
  if (!b || !x) return fail(h, LS_ERR_ARG, "null vector");
  if (b == x) return fail(h, LS_ERR_ARG, "b and x must not alias");
  if (ld < h->n_total) return fail(h, LS_ERR_ARG, "ld < number of nodes");
  if (!(o->tol > 0) || !std::isfinite(o->tol)) return fail(h, LS_ERR_ARG, "tol must be > 0");
  if (o->maxit < 1) return fail(h, LS_ERR_ARG, "maxit must be >= 1");
  if (o->restart < 0) return fail(h, LS_ERR_ARG, "restart < 0");
  if (o->prec != LS_FP64 && o->prec != LS_MIXED) return fail(h, LS_ERR_ARG, "bad precision");
  lsk::PrecondCb pc;
  if (s == -1 && !S) {
    // the library's sparsifying preconditioner on every scatterer that has one
    bool any = false;
    for (const Scat &q : h->sc) any = any || q.sp != nullptr;
    if (!any) return fail(h, LS_ERR_ARG, "no scatterer has a preconditioner (ls_sparsify_setup)");
    pc.s = -1;
    return lsk::solve_gmres(h, b, x, nrhs, ld, *o, info, stream, &pc);
  }
  if (s < 0 || s >= (int32_t)h->sc.size()) return fail(h, LS_ERR_ARG, "bad scatterer index");
  const Scat &sct = h->sc[s];
  if (!sct.tr) return fail(h, LS_ERR_ARG, "no grid for this scatterer (ls_transfer_setup)");
  if (!S || !c || !sc) return fail(h, LS_ERR_ARG, "null preconditioner argument");
  if (ldc < (int64_t)sct.tr->nx * sct.tr->ny) return fail(h, LS_ERR_ARG, "ldc < number of grid nodes");
  pc.s = s;
  pc.S = S;
  pc.user = user;
  pc.c = (double2 *)c;
  pc.sc = (double2 *)sc;
  pc.ldc = ldc;
  return lsk::solve_gmres(h, b, x, nrhs, ld, *o, info, stream, &pc);
}

ls_status ls_grad_contrast(ls_handle h, const double *u, const double *lam, const double *a, int32_t nrhs,
                           int64_t ld, double *grad, hipStream_t stream) {
  if (!h) return fail(nullptr, LS_ERR_ARG, "null handle");
  if (nrhs < 0) return fail(h, LS_ERR_ARG, "nrhs < 0");
  if (!u || !lam || !a || !grad) return fail(h, LS_ERR_ARG, "null vector");
  if (ld < h->n_total) return fail(h, LS_ERR_ARG, "ld < number of nodes");
  if (nrhs == 0) {
    HIPCHK(h, hipMemsetAsync(grad, 0, sizeof(double) * h->n_total, stream));
    return LS_OK;
  }
  return lsk::grad_contrast(h, u, lam, a, nrhs, ld, grad, stream);
}

ls_status ls_apply(ls_handle h, const double *x, double *y, int32_t nrhs, int64_t ld, ls_precision p,
                   hipStream_t stream) {
  return apply_common(h, x, y, nrhs, ld, p, stream, lsk::Mode::Forward);
}

ls_status ls_apply_adjoint(ls_handle h, const double *x, double *y, int32_t nrhs, int64_t ld, ls_precision p,
                           hipStream_t stream) {
  return apply_common(h, x, y, nrhs, ld, p, stream, lsk::Mode::Adjoint);
}

ls_status ls_profile_enable(ls_handle h, int32_t on) {
  if (!h) return fail(nullptr, LS_ERR_ARG, "null handle");
  h->prof = on != 0;
  return LS_OK;
}

ls_status ls_profile_query(ls_handle h, ls_profile *out, int32_t reset) {
  if (!h || !out) return fail(h, LS_ERR_ARG, "null argument");
  out->far_launches = (int64_t)h->ev_far.size() / 2;
  out->apply_calls = (int64_t)h->ev_apply.size() / 2;
  out->far_ms = out->apply_ms = 0.0;
  out->pair_rhs = h->prof_pairs;
  out->far_launches_mixed = 0;
  out->far_ms_mixed = 0.0;
  out->pair_rhs_mixed = h->prof_pairs_mixed;
  out->far_launches_h16 = 0;
  out->far_ms_h16 = 0.0;
  out->pair_rhs_h16 = h->prof_pairs_h16;
  for (size_t i = 0; i + 1 < h->ev_far.size(); i += 2) {
    float ms = 0.f;
    HIPCHK(h, hipEventSynchronize(h->ev_far[i + 1]));
    HIPCHK(h, hipEventElapsedTime(&ms, h->ev_far[i], h->ev_far[i + 1]));
    out->far_ms += ms;
    if (h->ev_far_mixed[i / 2]) {
      out->far_ms_mixed += ms;
      ++out->far_launches_mixed;
    }
    if (h->ev_far_mixed[i / 2] == 2) {
      out->far_ms_h16 += ms;
      ++out->far_launches_h16;
    }
  }
  for (size_t i = 0; i + 1 < h->ev_apply.size(); i += 2) {
    float ms = 0.f;
    HIPCHK(h, hipEventSynchronize(h->ev_apply[i + 1]));
    HIPCHK(h, hipEventElapsedTime(&ms, h->ev_apply[i], h->ev_apply[i + 1]));
    out->apply_ms += ms;
  }
  if (reset) {
    for (hipEvent_t e : h->ev_far) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->ev_apply) (void)hipEventDestroy(e);
    h->ev_far.clear();
    h->ev_far_mixed.clear();
    h->ev_apply.clear();
    h->prof_pairs = 0.0;
    h->prof_pairs_mixed = 0.0;
    h->prof_pairs_h16 = 0.0;
  }
  return LS_OK;
}

static ls_status ensure_ws(ls_ctx *h, lsk::Workspace &w, size_t need, hipStream_t st) {
  if (need <= w.bytes) return LS_OK;
  if (w.ptr) {
    HIPCHK(h, hipStreamSynchronize(st));
    HIPCHK(h, hipFree(w.ptr));
    w.ptr = nullptr;
    w.bytes = 0;
  }
  if (lsk::dmalloc(&w.ptr, need) != hipSuccess) return fail(h, LS_ERR_ALLOC, "workspace allocation failed");
  w.bytes = need;
  return LS_OK;
}

ls_status ls_farfield(ls_handle h, int32_t s, const double *u, int32_t nrhs, int64_t ld, const double *thetas,
                      int32_t R, const double *data, double *uinf, double *res, double *misfit, hipStream_t stream) {
  if (!h) return fail(nullptr, LS_ERR_ARG, "null handle");
  if (s < 0 || s >= (int32_t)h->sc.size()) return fail(h, LS_ERR_ARG, "bad scatterer index");
  if (nrhs < 1 || R < 1 || !u || !thetas || !uinf) return fail(h, LS_ERR_ARG, "bad argument");
  if (ld < h->n_total) return fail(h, LS_ERR_ARG, "ld < number of nodes");
  if ((res || misfit) && !data) return fail(h, LS_ERR_ARG, "res and misfit need data");
  for (int r = 0; r < R; ++r)
    if (!std::isfinite(thetas[r])) return fail(h, LS_ERR_NONFINITE, "non-finite angle");
  const Scat &sc = h->sc[s];
  const size_t need = lsk::farfield_workspace_bytes(sc.n, R, nrhs);
  ls_status st = ensure_ws(h, h->ws_ff, need, stream);
  if (st != LS_OK) return st;
  // angles at the end of the workspace, residual buffer before them when the caller gave none
  const size_t th_off = (need - sizeof(double) * R - 256) & ~(size_t)255;
  const size_t res_off = (th_off - sizeof(double2) * (size_t)R * nrhs - 256) & ~(size_t)255;
  double *th = (double *)((char *)h->ws_ff.ptr + th_off);
  double2 *res_tmp = (double2 *)((char *)h->ws_ff.ptr + res_off);
  HIPCHK(h, hipMemcpyAsync(th, thetas, sizeof(double) * R, hipMemcpyHostToDevice, stream));
  double *resp = res ? res : (data ? (double *)res_tmp : nullptr);
  HIPCHK(h, lsk::launch_farfield(sc, u, nrhs, ld, th, R, data, uinf, resp, h->ws_ff.ptr, stream));
  if (misfit) {
    std::vector<double> hr(2 * (size_t)R * nrhs);
    HIPCHK(h, hipMemcpyAsync(hr.data(), resp, sizeof(double) * hr.size(), hipMemcpyDeviceToHost, stream));
    HIPCHK(h, hipStreamSynchronize(stream));
    double J = 0.0;
    for (double v : hr) J += v * v;
    *misfit = 0.5 * J;
  }
  return LS_OK;
}

ls_status ls_field(ls_handle h, int32_t s, const double *tx, const double *ty, int64_t nt, const double *u,
                   int32_t nrhs, int64_t ld, double *out, hipStream_t stream) {
  if (!h) return fail(nullptr, LS_ERR_ARG, "null handle");
  if (s < 0 || s >= (int32_t)h->sc.size()) return fail(h, LS_ERR_ARG, "bad scatterer index");
  if (nrhs < 1 || nt < 1 || nt > (int64_t)INT32_MAX / 2 || !tx || !ty || !u || !out)
    return fail(h, LS_ERR_ARG, "bad argument");
  if (ld < h->n_total) return fail(h, LS_ERR_ARG, "ld < number of nodes");
  const Scat &sc = h->sc[s];
  if (!sc.geom) return fail(h, LS_ERR_UNSUPPORTED, "no geometry for this scatterer");
  for (int64_t t = 0; t < nt; ++t) {
    if (!std::isfinite(tx[t]) || !std::isfinite(ty[t])) return fail(h, LS_ERR_NONFINITE, "non-finite point");
    if (!lsk::outside_scatterer(sc, tx[t], ty[t])) return fail(h, LS_ERR_ARG, "a point lies inside the scatterer");
  }
  // correction rows of the targets (host threads and the GPU), then the sums
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> cv;
  ls_status st = lsk::field_correction(h, sc, nt, tx, ty, stream, rp, ci, cv);
  if (st != LS_OK) return st;
  const int nsplit = lsk::field_source_split(sc.n, nt, nrhs);
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t b_rp = al(sizeof(int64_t) * rp.size()), b_ci = al(sizeof(int32_t) * ci.size()),
               b_cv = al(sizeof(double) * cv.size()), b_t = al(sizeof(double) * 2 * nt);
  const size_t need = b_rp + b_ci + b_cv + b_t + lsk::field_workspace_bytes(sc.n, nrhs, nt, nsplit);
  void *ws = nullptr;
  if (lsk::dmalloc(&ws, need) != hipSuccess) return fail(h, LS_ERR_ALLOC, "field workspace");
  char *p = (char *)ws;
  int64_t *drp = (int64_t *)p;
  int32_t *dci = (int32_t *)(p + b_rp);
  double *dcv = (double *)(p + b_rp + b_ci);
  double *dt = (double *)(p + b_rp + b_ci + b_cv);
  void *rest = p + b_rp + b_ci + b_cv + b_t;
  hipError_t e = hipMemcpyAsync(drp, rp.data(), sizeof(int64_t) * rp.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dci, ci.data(), sizeof(int32_t) * ci.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dcv, cv.data(), sizeof(double) * cv.size(), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dt, tx, sizeof(double) * nt, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dt + nt, ty, sizeof(double) * nt, hipMemcpyHostToDevice, stream);
  hipEvent_t f0 = nullptr, f1 = nullptr;
  if (e == hipSuccess && h->prof) {
    (void)hipEventCreate(&f0);
    (void)hipEventCreate(&f1);
    h->ev_far.push_back(f0);
    h->ev_far.push_back(f1);
    h->ev_far_mixed.push_back(0);
    h->prof_pairs += (double)sc.n * (double)nt * nrhs;
  }
  if (e == hipSuccess)
    e = lsk::launch_field(sc, u, nrhs, ld, nt, dt, dt + nt, drp, dci, (const double2 *)dcv, nsplit, out, rest, stream,
                          f0, f1);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);   // host vectors and the workspace go away
  (void)hipFree(ws);
  if (e != hipSuccess) return fail(h, LS_ERR_HIP, hipGetErrorString(e));
  return LS_OK;
}

ls_status ls_farfield_adjoint(ls_handle h, int32_t s, const double *res, int32_t nrhs, int64_t ld,
                              const double *thetas, int32_t R, double *a, double *rhs, hipStream_t stream) {
  if (!h) return fail(nullptr, LS_ERR_ARG, "null handle");
  if (s < 0 || s >= (int32_t)h->sc.size()) return fail(h, LS_ERR_ARG, "bad scatterer index");
  if (nrhs < 1 || R < 1 || !res || !thetas || (!a && !rhs)) return fail(h, LS_ERR_ARG, "bad argument");
  if (ld < h->n_total) return fail(h, LS_ERR_ARG, "ld < number of nodes");
  const Scat &sc = h->sc[s];
  const size_t need = lsk::farfield_workspace_bytes(sc.n, R, nrhs);
  ls_status st = ensure_ws(h, h->ws_ff, need, stream);
  if (st != LS_OK) return st;
  double *th = (double *)((char *)h->ws_ff.ptr + ((need - sizeof(double) * R - 256) & ~(size_t)255));
  HIPCHK(h, hipMemcpyAsync(th, thetas, sizeof(double) * R, hipMemcpyHostToDevice, stream));
  HIPCHK(h, lsk::launch_farfield_adjoint(sc, res, nrhs, ld, th, R, a, rhs, stream));
  return LS_OK;
}

ls_status ls_autotune(ls_handle h, int32_t nrhs, ls_precision p, ls_tune_result *out, hipStream_t stream) {
  if (!h || nrhs < 1 || (p != LS_FP64 && p != LS_MIXED)) return fail(h, LS_ERR_ARG, "bad argument");
  const bool single = p == LS_MIXED;
  const int mts[2] = {single ? 2 : 1, single ? 4 : 2};
  // FP32 partial sums over more than 2 048 sources lose accuracy (see tile_source_split)
  const int lens_all[4] = {1024, 2048, 4096, 8192};
  const std::vector<int> lens(lens_all, lens_all + (single ? 2 : 4));
  size_t need = 0;
  for (int L : lens) need = std::max(need, lsk::batch_workspace_bytes(h, nrhs, single, L));
  ls_status st = ensure_ws(h, h->ws_apply, need, stream);
  if (st != LS_OK) return st;
  HIPCHK(h, hipMemsetAsync(h->ws_apply.ptr, 0, need, stream));
  hipEvent_t e0, e1;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  lsk::TileTune best;
  best.ms = 1e300;
  for (int mt : mts)
    for (int L : lens) {
      // one untimed launch, then the mean of two timed ones (far sum only, all scatterers)
      float ms = 0.f, tot = 0.f;
      for (int rep = 0; rep < 3; ++rep) {
        HIPCHK(h, lsk::launch_apply_batch(h, nullptr, nullptr, nrhs, h->n_total, lsk::Mode::Forward, single, mt, L,
                                          h->ws_apply.ptr, stream, rep ? e0 : nullptr, rep ? e1 : nullptr, true));
        if (rep) {
          HIPCHK(h, hipEventSynchronize(e1));
          HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
          tot += ms;
        }
      }
      if (tot / 2 < best.ms) best = lsk::TileTune{mt, L, tot / 2.0};
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->tune[single ? 1 : 0] = best;
  h->batch_key = -1;
  if (out) {
    out->mt = best.mt;
    out->split_len = best.split_len;
    out->far_ms = best.ms;
  }
  return LS_OK;
}

ls_status ls_set_tile_shape(ls_handle h, ls_precision p, int32_t mt, int32_t split_len) {
  if (!h || (p != LS_FP64 && p != LS_MIXED)) return fail(h, LS_ERR_ARG, "bad argument");
  const bool single = p == LS_MIXED;
  const bool mt_ok = single ? (mt == 2 || mt == 4) : (mt == 1 || mt == 2);
  if (!mt_ok || split_len < 64) return fail(h, LS_ERR_ARG, "unsupported tile shape");
  h->tune[single ? 1 : 0] = lsk::TileTune{mt, split_len, 0.0};
  h->batch_key = -1;
  return LS_OK;
}

ls_status ls_set_contrast(ls_handle h, const double *m, hipStream_t stream) {
  if (!h || !m) return fail(h, LS_ERR_ARG, "null argument");
  for (const Scat &sc : h->sc) HIPCHK(h, lsk::launch_set_contrast(sc, m, stream));
  return LS_OK;
}

int64_t ls_num_nodes(ls_handle h) { return h ? h->n_total : -1; }
int32_t ls_num_scatterers(ls_handle h) { return h ? (int32_t)h->sc.size() : -1; }
int64_t ls_scatterer_offset(ls_handle h, int32_t s) {
  return (h && s >= 0 && s < (int32_t)h->sc.size()) ? h->sc[s].off : -1;
}
int64_t ls_correction_nnz(ls_handle h, int32_t s) {
  return (h && s >= 0 && s < (int32_t)h->sc.size()) ? h->sc[s].nnz : -1;
}

int64_t ls_near_pairs(ls_handle h, int32_t s) {
  if (!h || s < 0 || s >= (int32_t)h->sc.size()) return -1;
  const lsk::Scat &sc = h->sc[s];
  return sc.near_ok ? sc.near_pairs : 0;
}

ls_status ls_export_correction(ls_handle h, int32_t s, int64_t *rowptr, int32_t *col, double *val) {
  if (!h || s < 0 || s >= (int32_t)h->sc.size() || !rowptr || !col || !val)
    return fail(h, LS_ERR_ARG, "bad argument");
  const Scat &sc = h->sc[s];
  const int64_t n = sc.n, nnz = sc.nnz;
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> ci(std::max<int64_t>(nnz, 1));
  std::vector<double> cv(2 * std::max<int64_t>(nnz, 1));
  HIPCHK(h, hipMemcpy(rp.data(), sc.rp, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
  if (nnz) {
    HIPCHK(h, hipMemcpy(ci.data(), sc.ci, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    HIPCHK(h, hipMemcpy(cv.data(), sc.cv, sizeof(double) * 2 * nnz, hipMemcpyDeviceToHost));
  }
  // back to caller order
  std::vector<int32_t> inv(n);
  for (int64_t i = 0; i < n; ++i) inv[sc.perm_host[i]] = (int32_t)i;
  rowptr[0] = 0;
  for (int64_t r = 0; r < n; ++r) {
    const int64_t i = inv[r];
    rowptr[r + 1] = rowptr[r] + (rp[i + 1] - rp[i]);
    int64_t d = rowptr[r];
    for (int64_t q = rp[i]; q < rp[i + 1]; ++q, ++d) {
      col[d] = sc.perm_host[ci[q]];
      val[2 * d] = cv[2 * q];
      val[2 * d + 1] = cv[2 * q + 1];
    }
  }
  return LS_OK;
}

ls_status ls_eval_green_host(const double *z2, double *g, int64_t n) {
  if (n < 0 || (n > 0 && (!z2 || !g))) return fail(nullptr, LS_ERR_ARG, "bad argument");
  lsk::eval_green_host(z2, g, n);
  return LS_OK;
}

ls_status ls_eval_green(const double *z2, double *g, int64_t n, int32_t single, hipStream_t stream) {
  if (n < 0 || (n > 0 && (!z2 || !g))) return fail(nullptr, LS_ERR_ARG, "bad argument");
  HIPCHK(nullptr, lsk::launch_eval_green(z2, g, n, single, stream));
  return LS_OK;
}

}  // extern "C"
