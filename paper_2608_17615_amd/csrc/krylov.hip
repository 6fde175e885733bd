// GMRES without restart (paper, Section 6 setup: the Nystrom system L u = b is solved by GMRES
// without restart; here unpreconditioned), per right-hand side, on the device, and the contrast
// gradient of a far-field misfit.
//
// Arnoldi: classical Gram-Schmidt with one re-orthogonalisation pass (CGS2) in FP64.  Every
// inner product is a two-stage deterministic reduction (fixed-order block partials, then a
// fixed-order sum), so results do not depend on scheduling.  The basis lives in chunks of
// device memory kept by the handle between solves.  Per iteration the host receives the new
// Hessenberg column (2 (j+1) + 1 values per RHS) and applies the complex Givens rotations;
// everything of size N stays on the device.
//
// Mixed precision (LS_MIXED): flexible GMRES (FP64 outer Arnoldi, FP64 applies for the outer
// Krylov vectors and for the residuals) whose preconditioner is an inner GMRES solve with the
// mixed-precision operator; the outer iteration removes the inner solve's error.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <vector>

#include "internal.h"

namespace lsk {

namespace {

constexpr int kBlock = 256;
constexpr int kEPT = 4;                      // elements per thread in the dot kernel
constexpr int kTile = kBlock * kEPT;
constexpr int kGroup = 8;                    // basis vectors per dot-product block

typedef std::complex<double> cplx;

__device__ __forceinline__ double2 block_sum2(double2 v, double2 *lds) {
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o);
    v.y += __shfl_xor(v.y, o);
  }
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  if (ln == 0) lds[wv] = v;
  __syncthreads();
  double2 r = make_double2(0.0, 0.0);
  if (threadIdx.x == 0)
    for (int k = 0; k < kBlock / 64; ++k) {
      r.x += lds[k].x;
      r.y += lds[k].y;
    }
  __syncthreads();
  return r;
}

// part[(tile * nrhs + c) * nv + i] = sum over the tile of conj(V_i[c][n]) w[c][n].
// grid (tiles, ceil(nv / kGroup), nrhs): each block forms kGroup inner products over one tile, so
// even a single short column (one right-hand side) spreads over many workgroups, and the
// kGroup x kEPT loads of a thread are independent.
__global__ __launch_bounds__(kBlock) void dots_kernel(int64_t n, int nrhs, int nv, const double2 *const *V,
                                                      int64_t ldv, const double2 *__restrict__ w, int64_t ldw,
                                                      double2 *__restrict__ part) {
  __shared__ double2 lds[kGroup][kBlock / 64];
  const int64_t t0 = (int64_t)blockIdx.x * kTile;
  const int i0 = blockIdx.y * kGroup;
  const int c = blockIdx.z;
  double2 wv[kEPT];
#pragma unroll
  for (int e = 0; e < kEPT; ++e) {
    const int64_t idx = t0 + e * kBlock + threadIdx.x;
    wv[e] = idx < n ? w[(int64_t)c * ldw + idx] : make_double2(0.0, 0.0);
  }
  double2 acc[kGroup];
#pragma unroll
  for (int g = 0; g < kGroup; ++g) {
    acc[g] = make_double2(0.0, 0.0);
    if (i0 + g < nv) {
      const double2 *v = V[i0 + g] + (int64_t)c * ldv;
#pragma unroll
      for (int e = 0; e < kEPT; ++e) {
        const int64_t idx = t0 + e * kBlock + threadIdx.x;
        if (idx < n) {
          const double2 a = v[idx];
          acc[g].x = std::fma(a.x, wv[e].x, std::fma(a.y, wv[e].y, acc[g].x));
          acc[g].y = std::fma(a.x, wv[e].y, std::fma(-a.y, wv[e].x, acc[g].y));
        }
      }
    }
  }
#pragma unroll
  for (int g = 0; g < kGroup; ++g) {
    double2 v = acc[g];
    for (int o = 32; o > 0; o >>= 1) {
      v.x += __shfl_xor(v.x, o);
      v.y += __shfl_xor(v.y, o);
    }
    if ((threadIdx.x & 63) == 0) lds[g][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < kGroup && i0 + (int)threadIdx.x < nv) {
    double2 r = make_double2(0.0, 0.0);
    for (int k = 0; k < kBlock / 64; ++k) {
      r.x += lds[threadIdx.x][k].x;
      r.y += lds[threadIdx.x][k].y;
    }
    part[((int64_t)blockIdx.x * nrhs + c) * nv + i0 + threadIdx.x] = r;
  }
}

// out[c * ldo + i] = sum_tile part[(tile * nrhs + c) * nv + i]  (fixed order); optionally also
// writes sqrt(real part) of entry 0 to beta[c] (norm mode)
__global__ void reduce_kernel(int ntiles, int nrhs, int nv, const double2 *__restrict__ part, double2 *out,
                              int64_t ldo, double *beta) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrhs * nv) return;
  const int c = t / nv, i = t - c * nv;
  double2 r = make_double2(0.0, 0.0);
  for (int k = 0; k < ntiles; ++k) {
    const double2 p = part[((int64_t)k * nrhs + c) * nv + i];
    r.x += p.x;
    r.y += p.y;
  }
  if (out) out[(int64_t)c * ldo + i] = r;
  if (beta) beta[c] = std::sqrt(r.x);
}

// w[c][n] += sign * sum_{i < nv} V_i[c][n] h[c * ldh + i]
__global__ __launch_bounds__(kBlock) void update_kernel(int64_t n, int nv, const double2 *const *V, int64_t ldv,
                                                        const double2 *__restrict__ hcoef, int64_t ldh,
                                                        double sign, double2 *__restrict__ w, int64_t ldw) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int c = blockIdx.y;
  if (idx >= n) return;
  double ar = 0.0, ai = 0.0;
  const double2 *hc = hcoef + (int64_t)c * ldh;
#pragma unroll 8
  for (int i = 0; i < nv; ++i) {
    const double2 v = V[i][(int64_t)c * ldv + idx];
    const double2 hh = hc[i];
    ar = std::fma(v.x, hh.x, std::fma(-v.y, hh.y, ar));
    ai = std::fma(v.x, hh.y, std::fma(v.y, hh.x, ai));
  }
  double2 &o = w[(int64_t)c * ldw + idx];
  o.x = std::fma(sign, ar, o.x);
  o.y = std::fma(sign, ai, o.y);
}

// y[c][n] = a[c][n] * (1 / beta[c])  (beta[c] > 0), with a and y possibly the same
__global__ __launch_bounds__(kBlock) void scale_kernel(int64_t n, const double *__restrict__ beta, const double2 *a,
                                                       int64_t lda, double2 *y, int64_t ldy) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int c = blockIdx.y;
  if (idx >= n) return;
  const double bt = beta[c];
  const double s = bt > 0.0 ? 1.0 / bt : 0.0;
  const double2 v = a[(int64_t)c * lda + idx];
  y[(int64_t)c * ldy + idx] = make_double2(v.x * s, v.y * s);
}

// y[c][n] = a[c][n] + alpha * b[c][n]
__global__ __launch_bounds__(kBlock) void axpy_kernel(int64_t n, const double2 *a, int64_t lda, double alpha,
                                                      const double2 *b, int64_t ldb, double2 *y, int64_t ldy) {
  const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int c = blockIdx.y;
  if (idx >= n) return;
  const double2 u = a[(int64_t)c * lda + idx], v = b[(int64_t)c * ldb + idx];
  y[(int64_t)c * ldy + idx] = make_double2(std::fma(alpha, v.x, u.x), std::fma(alpha, v.y, u.y));
}

// grad[j] = sum_d Re[ conj(a_dj - k^2 P_dj) u_dj ]  for j in one scatterer's segment
__global__ __launch_bounds__(kBlock) void grad_kernel(int64_t n, int64_t off, int nrhs, double k2,
                                                      const double2 *__restrict__ u, const double2 *__restrict__ a,
                                                      const double2 *__restrict__ P, int64_t ld, int64_t ldp,
                                                      double *__restrict__ grad) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n) return;
  double g = 0.0;
  for (int d = 0; d < nrhs; ++d) {
    const double2 av = a[(int64_t)d * ld + off + j], pv = P[(int64_t)d * ldp + off + j];
    const double2 uv = u[(int64_t)d * ld + off + j];
    const double qr = av.x - k2 * pv.x, qi = av.y - k2 * pv.y;
    g += qr * uv.x + qi * uv.y;   // Re(conj(q) u)
  }
  grad[off + j] = g;
}

// ---------------------------------------------------------------- host side
struct Basis {
  // Krylov vectors, each nrhs x n complex (ld = n), in chunks of kChunk vectors
  static constexpr int kChunk = 16;
  std::vector<void *> chunks;
  size_t chunk_bytes = 0;
  double2 *vec(int i, int64_t n, int nrhs) const {
    return (double2 *)chunks[i / kChunk] + (size_t)(i % kChunk) * n * nrhs;
  }
};

struct SolveWs {
  Basis V, Z;                // Z: flexible GMRES preconditioned vectors
  void *small = nullptr;     // h, y, beta, pointer table
  size_t small_bytes = 0;
  void *part = nullptr;      // per-tile partial inner products, grown with the basis
  size_t part_bytes = 0;
  void *vecs = nullptr;      // r, t, inner workspaces
  size_t vec_bytes = 0;
};

hipError_t ensure_chunks(Basis &B, int nvec, int64_t n, int nrhs) {
  const size_t cb = (size_t)Basis::kChunk * n * nrhs * sizeof(double2);
  if (B.chunk_bytes != cb) {
    for (void *p : B.chunks) (void)hipFree(p);
    B.chunks.clear();
    B.chunk_bytes = cb;
  }
  const int need = (nvec + Basis::kChunk - 1) / Basis::kChunk;
  while ((int)B.chunks.size() < need) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, cb);
    if (e != hipSuccess) return e;
    B.chunks.push_back(p);
  }
  return hipSuccess;
}

hipError_t ensure(void *&p, size_t &have, size_t need) {
  if (need <= have) return hipSuccess;
  if (p) (void)hipFree(p);
  p = nullptr;
  have = 0;
  hipError_t e = hipMalloc(&p, need);
  if (e == hipSuccess) have = need;
  return e;
}

SolveWs *solve_ws(ls_ctx *h, int level) {
  if (!h->ws_solve.ptr) h->ws_solve.ptr = new SolveWs[3]();
  return (SolveWs *)h->ws_solve.ptr + level;
}

unsigned tiles_of(int64_t n) { return (unsigned)((n + kTile - 1) / kTile); }
unsigned blocks_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// One GMRES cycle engine shared by the plain and the flexible variant.
struct Gmres {
  ls_ctx *h;
  hipStream_t st;
  int64_t n;
  int nrhs;
  Mode mode;
  SolveWs *ws;
  // device scratch
  double2 *part = nullptr, *hbuf = nullptr, *ybuf = nullptr;
  double *beta = nullptr;
  double2 **ptrs = nullptr;   // device table of basis pointers
  int max_vec = 0;

  hipError_t init(int maxvec) {
    max_vec = maxvec;
    const size_t need = 2 * sizeof(double2) * (size_t)nrhs * (maxvec + 1) +          // h, y
                        sizeof(double) * nrhs + sizeof(double2 *) * (size_t)(2 * maxvec + 8) + 1024;
    hipError_t e = ensure(ws->small, ws->small_bytes, need);
    if (e != hipSuccess) return e;
    e = ensure_part(16);
    if (e != hipSuccess) return e;
    char *p = (char *)ws->small;
    hbuf = (double2 *)p;
    p += sizeof(double2) * (size_t)nrhs * (maxvec + 1);
    ybuf = (double2 *)p;
    p += sizeof(double2) * (size_t)nrhs * (maxvec + 1);
    beta = (double *)p;
    p += sizeof(double) * nrhs;
    p = (char *)(((uintptr_t)p + 255) & ~(uintptr_t)255);
    ptrs = (double2 **)p;
    return hipSuccess;
  }

  // partials for nv inner products per column; grows geometrically, after the stream has drained
  // (the old buffer may still be read by a queued reduction)
  hipError_t ensure_part(int nv) {
    const size_t per = sizeof(double2) * tiles_of(n) * nrhs;
    if (per * nv <= ws->part_bytes) {
      part = (double2 *)ws->part;
      return hipSuccess;
    }
    const int cap = std::min(max_vec + 1, std::max(nv, 2 * (int)(ws->part_bytes / per)));
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    e = ensure(ws->part, ws->part_bytes, per * std::max(cap, nv));
    part = (double2 *)ws->part;
    return e;
  }

  // h[c][0..nv) = V[0..nv)^H w (device, hbuf), using the pointer table entries [0, nv)
  hipError_t dots(int nv, const double2 *w, double2 *out, int64_t ldo) {
    hipError_t e0 = ensure_part(nv);
    if (e0 != hipSuccess) return e0;
    dim3 g(tiles_of(n), (unsigned)((nv + kGroup - 1) / kGroup), nrhs);
    dots_kernel<<<g, kBlock, 0, st>>>(n, nrhs, nv, ptrs, n, w, n, part);
    reduce_kernel<<<(unsigned)((nrhs * nv + 255) / 256), 256, 0, st>>>((int)tiles_of(n), nrhs, nv, part, out, ldo,
                                                                       nullptr);
    return hipGetLastError();
  }

  // beta[c] = ||w_c||
  hipError_t norms(const double2 *w, double2 **tbl_slot) {
    (void)tbl_slot;
    dim3 g(tiles_of(n), 1, nrhs);
    dots_kernel<<<g, kBlock, 0, st>>>(n, nrhs, 1, ptrs + max_vec + 2, n, w, n, part);
    reduce_kernel<<<(unsigned)((nrhs + 255) / 256), 256, 0, st>>>((int)tiles_of(n), nrhs, 1, part, nullptr, 1, beta);
    return hipGetLastError();
  }
};

}  // namespace

struct CoreOpts {
  double tol;
  int maxit, restart;
  Mode mode;
  ls_precision matvec;   // precision of the Arnoldi operator applications
  bool flexible;         // FP64 flexible GMRES with an inner mixed-precision GMRES preconditioner
  double inner_tol;
  int inner_maxit;
  bool x0_given;
  double relax_eps;      // > 0: FP64 applies while the residual estimate exceeds tol / relax_eps, mixed after
};

struct CoreResult {
  std::vector<int> iters;
  std::vector<char> done;
  int64_t n_fp64 = 0, n_mixed = 0;
};

// GMRES on contiguous (ld = n) device vectors b, x of nrhs columns.  x holds the initial guess
// when o.x0_given, the approximate solution on return.  ws is this level's workspace; the
// flexible variant runs its inner solves with a second workspace.
ls_status gmres_core(ls_ctx *h, SolveWs *ws, SolveWs *ws_inner, const double2 *b, double2 *x, int nrhs,
                     const CoreOpts &o, CoreResult &res, hipStream_t st) {
  const int64_t n = h->n_total;
  const int maxit = o.maxit;
  const int cyc = (o.restart > 0 && o.restart < maxit) ? o.restart : maxit;
  Gmres G{h, st, n, nrhs, o.mode, ws};
#define HIPTRY(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) return setup_fail(h, LS_ERR_HIP, hipGetErrorString(e_)); \
  } while (0)
  HIPTRY(G.init(cyc + 1));
  const size_t vb = sizeof(double2) * (size_t)n * nrhs;
  HIPTRY(ensure(ws->vecs, ws->vec_bytes, 2 * vb));
  double2 *r = (double2 *)ws->vecs;
  double2 *t = r + (size_t)n * nrhs;
  // the basis grows chunk by chunk as the iteration needs it (a solve that converges early never
  // holds maxit vectors); new chunks enter the device pointer table as they arrive
  HIPTRY(ensure_chunks(ws->V, 1, n, nrhs));
  if (o.flexible) HIPTRY(ensure_chunks(ws->Z, 1, n, nrhs));
  std::vector<double2 *> tbl(2 * (cyc + 1) + 4, nullptr);
  int have = 0;   // basis vectors whose pointers are in tbl and on the device
  auto grow = [&](int nvec) -> hipError_t {
    nvec = std::min(nvec, cyc + 1);
    if (nvec <= have) return hipSuccess;
    hipError_t e = ensure_chunks(ws->V, nvec, n, nrhs);
    if (e != hipSuccess) return e;
    const int upto = std::min(cyc + 1, (int)ws->V.chunks.size() * Basis::kChunk);
    for (int i = have; i < upto; ++i) tbl[i] = ws->V.vec(i, n, nrhs);
    e = hipMemcpyAsync(G.ptrs + have, tbl.data() + have, sizeof(double2 *) * (upto - have), hipMemcpyHostToDevice,
                       st);
    have = upto;
    return e;
  };
  const int slot = G.max_vec + 2;
  std::vector<double> bnorm(nrhs);
  tbl[slot] = (double2 *)b;
  HIPTRY(hipMemcpyAsync(G.ptrs, tbl.data(), sizeof(double2 *) * tbl.size(), hipMemcpyHostToDevice, st));
  HIPTRY(grow(1));
  HIPTRY(G.norms(b, nullptr));
  HIPTRY(hipMemcpyAsync(bnorm.data(), G.beta, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
  HIPTRY(hipStreamSynchronize(st));
  for (int c = 0; c < nrhs; ++c)
    if (!std::isfinite(bnorm[c])) return setup_fail(h, LS_ERR_NONFINITE, "non-finite right-hand side");
  if (!o.x0_given) HIPTRY(hipMemsetAsync(x, 0, vb, st));
  res.iters.assign(nrhs, 0);
  res.done.assign(nrhs, 0);
  std::vector<double> est(nrhs, 1.0);
  int total_it = 0;
  bool first_cycle = true;
  // Hessenberg columns packed per right-hand side: column j (rows 0..j+1) starts at j (j + 3) / 2,
  // grown one column per step
  std::vector<std::vector<cplx>> H(nrhs);
  std::vector<cplx> cs, sn, g;
  std::vector<double2> hh((size_t)nrhs * (cyc + 1) * 2);
  std::vector<double> betah(nrhs);
  const dim3 gv(blocks_of(n), nrhs);
  while (total_it < maxit) {
    // r = b - L x (FP64), skipped while x = 0
    if (first_cycle && !o.x0_given) {
      HIPTRY(hipMemcpyAsync(r, b, vb, hipMemcpyDeviceToDevice, st));
    } else {
      const ls_precision pr = (o.flexible || o.relax_eps > 0) ? LS_FP64 : o.matvec;
      ls_status s2 = apply_op(h, (const double *)x, (double *)t, nrhs, n, o.mode, pr, st);
      if (s2 != LS_OK) return s2;
      if (pr == LS_FP64) ++res.n_fp64; else ++res.n_mixed;
      axpy_kernel<<<gv, kBlock, 0, st>>>(n, b, n, -1.0, t, n, r, n);
      HIPTRY(hipGetLastError());
    }
    first_cycle = false;
    tbl[slot] = r;
    HIPTRY(hipMemcpyAsync(G.ptrs, tbl.data(), sizeof(double2 *) * tbl.size(), hipMemcpyHostToDevice, st));
    HIPTRY(G.norms(r, nullptr));
    std::vector<double> rnorm(nrhs);
    HIPTRY(hipMemcpyAsync(rnorm.data(), G.beta, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    scale_kernel<<<gv, kBlock, 0, st>>>(n, G.beta, r, n, tbl[0], n);
    HIPTRY(hipGetLastError());
    HIPTRY(hipStreamSynchronize(st));
    bool all = true;
    for (int c = 0; c < nrhs; ++c) {
      est[c] = bnorm[c] > 0 ? rnorm[c] / bnorm[c] : 0.0;
      if (!std::isfinite(est[c])) return setup_fail(h, LS_ERR_NONFINITE, "non-finite residual");
      res.done[c] = est[c] <= o.tol;
      all = all && res.done[c];
    }
    if (all) break;
    const int m = cyc;
    for (auto &hc : H) hc.clear();
    cs.assign((size_t)nrhs * m, cplx(0));
    sn.assign((size_t)nrhs * m, cplx(0));
    g.assign((size_t)nrhs * (m + 1), cplx(0));
    std::vector<int> mc(nrhs, 0);
    std::vector<char> active(nrhs);
    for (int c = 0; c < nrhs; ++c) {
      g[(size_t)c * (m + 1)] = rnorm[c];
      active[c] = !res.done[c];
    }
    int j = 0;
    for (; j < m && total_it < maxit; ++j, ++total_it) {
      HIPTRY(grow(j + 2));
      double2 *vj = tbl[j];
      double2 *w = tbl[j + 1];
      if (o.flexible) {
        // z_j ~ L^{-1} v_j by an inner GMRES with the mixed-precision operator, then w = L z_j
        HIPTRY(ensure_chunks(ws->Z, j + 1, n, nrhs));
        double2 *zj = ws->Z.vec(j, n, nrhs);
        CoreOpts io{o.inner_tol, o.inner_maxit, 0, o.mode, LS_MIXED, false, 0.0, 0, false, 0.0};
        CoreResult ir;
        ls_status s2 = gmres_core(h, ws_inner, nullptr, vj, zj, nrhs, io, ir, st);
        if (s2 < 0) return s2;
        res.n_mixed += ir.n_mixed;
        res.n_fp64 += ir.n_fp64;
        s2 = apply_op(h, (const double *)zj, (double *)w, nrhs, n, o.mode, LS_FP64, st);
        if (s2 != LS_OK) return s2;
        ++res.n_fp64;
        tbl[slot] = r;   // the inner solve used its own pointer table; ours is intact
      } else {
        // relaxed inexact Arnoldi: an application error of relative size eps perturbs the
        // residual by about eps times the current residual, so once the largest active residual
        // estimate is below tol / eps the cheaper mixed-precision operator is accurate enough
        ls_precision pj = o.matvec;
        if (o.relax_eps > 0) {
          double worst = 0.0;
          for (int c = 0; c < nrhs; ++c)
            if (active[c]) worst = std::max(worst, est[c]);
          pj = worst * o.relax_eps <= o.tol ? LS_MIXED : LS_FP64;
        }
        ls_status s2 = apply_op(h, (const double *)vj, (double *)w, nrhs, n, o.mode, pj, st);
        if (s2 != LS_OK) return s2;
        if (pj == LS_FP64) ++res.n_fp64; else ++res.n_mixed;
      }
      // CGS2 against V[0..j]
      const int nv = j + 1;
      double2 *h1 = G.hbuf, *h2 = G.ybuf;
      HIPTRY(G.dots(nv, w, h1, nv));
      update_kernel<<<gv, kBlock, 0, st>>>(n, nv, G.ptrs, n, h1, nv, -1.0, w, n);
      HIPTRY(G.dots(nv, w, h2, nv));
      update_kernel<<<gv, kBlock, 0, st>>>(n, nv, G.ptrs, n, h2, nv, -1.0, w, n);
      tbl[slot] = w;
      HIPTRY(hipMemcpyAsync(G.ptrs + slot, &tbl[slot], sizeof(double2 *), hipMemcpyHostToDevice, st));
      HIPTRY(G.norms(w, nullptr));
      scale_kernel<<<gv, kBlock, 0, st>>>(n, G.beta, w, n, w, n);
      HIPTRY(hipMemcpyAsync(hh.data(), h1, sizeof(double2) * nrhs * nv, hipMemcpyDeviceToHost, st));
      HIPTRY(hipMemcpyAsync(hh.data() + (size_t)nrhs * nv, h2, sizeof(double2) * nrhs * nv, hipMemcpyDeviceToHost,
                            st));
      HIPTRY(hipMemcpyAsync(betah.data(), G.beta, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
      HIPTRY(hipStreamSynchronize(st));
      bool any = false;
      for (int c = 0; c < nrhs; ++c) {
        if (!active[c]) continue;
        std::vector<cplx> &Hv = H[c];
        Hv.resize((size_t)(j + 1) * (j + 4) / 2, cplx(0));
        cplx *Hc = Hv.data();
        auto Hat = [&](int r_, int c_) -> cplx & { return Hc[(size_t)c_ * (c_ + 3) / 2 + r_]; };
        for (int i = 0; i < nv; ++i) {
          const double2 a = hh[(size_t)c * nv + i], bq = hh[(size_t)nrhs * nv + (size_t)c * nv + i];
          Hat(i, j) = cplx(a.x + bq.x, a.y + bq.y);
        }
        Hat(j + 1, j) = betah[c];
        if (!std::isfinite(betah[c])) return setup_fail(h, LS_ERR_BREAKDOWN, "non-finite Arnoldi vector");
        cplx *csc = &cs[(size_t)c * m], *snc = &sn[(size_t)c * m], *gc = &g[(size_t)c * (m + 1)];
        for (int i = 0; i < j; ++i) {
          const cplx tq = csc[i] * Hat(i, j) + snc[i] * Hat(i + 1, j);
          Hat(i + 1, j) = -std::conj(snc[i]) * Hat(i, j) + std::conj(csc[i]) * Hat(i + 1, j);
          Hat(i, j) = tq;
        }
        const cplx a = Hat(j, j), bq = Hat(j + 1, j);
        const double den = std::sqrt(std::norm(a) + std::norm(bq));
        csc[j] = den > 0 ? std::conj(a) / den : cplx(1);
        snc[j] = den > 0 ? std::conj(bq) / den : cplx(0);
        Hat(j, j) = csc[j] * a + snc[j] * bq;
        Hat(j + 1, j) = 0.0;
        gc[j + 1] = -std::conj(snc[j]) * gc[j];
        gc[j] = csc[j] * gc[j];
        mc[c] = j + 1;
        res.iters[c]++;
        est[c] = bnorm[c] > 0 ? std::abs(gc[j + 1]) / bnorm[c] : 0.0;
        if (est[c] <= o.tol || betah[c] == 0.0) {
          active[c] = 0;
          res.done[c] = 1;
        } else {
          any = true;
        }
      }
      if (!any) {
        ++j;
        ++total_it;
        break;
      }
    }
    // x += V y (or Z y for the flexible variant) per column
    std::vector<double2> yv((size_t)nrhs * m, make_double2(0, 0));
    for (int c = 0; c < nrhs; ++c) {
      const int mm = mc[c];
      const cplx *Hc = H[c].data();
      auto Hat = [&](int r_, int c_) { return Hc[(size_t)c_ * (c_ + 3) / 2 + r_]; };
      std::vector<cplx> yc(mm);
      for (int i = mm - 1; i >= 0; --i) {
        cplx sacc = g[(size_t)c * (m + 1) + i];
        for (int k2 = i + 1; k2 < mm; ++k2) sacc -= Hat(i, k2) * yc[k2];
        yc[i] = sacc / Hat(i, i);
      }
      for (int i = 0; i < mm; ++i) yv[(size_t)c * m + i] = make_double2(yc[i].real(), yc[i].imag());
    }
    const int mmax = std::max(1, *std::max_element(mc.begin(), mc.end()));
    HIPTRY(hipMemcpyAsync(G.hbuf, yv.data(), sizeof(double2) * nrhs * m, hipMemcpyHostToDevice, st));
    if (o.flexible) {
      std::vector<double2 *> ztbl(mmax);
      for (int i = 0; i < mmax; ++i) ztbl[i] = ws->Z.vec(i, n, nrhs);
      HIPTRY(hipMemcpyAsync(G.ptrs + G.max_vec + 4, ztbl.data(), sizeof(double2 *) * mmax, hipMemcpyHostToDevice,
                            st));
      update_kernel<<<gv, kBlock, 0, st>>>(n, mmax, G.ptrs + G.max_vec + 4, n, G.hbuf, m, 1.0, x, n);
    } else {
      update_kernel<<<gv, kBlock, 0, st>>>(n, mmax, G.ptrs, n, G.hbuf, m, 1.0, x, n);
    }
    HIPTRY(hipGetLastError());
    HIPTRY(hipStreamSynchronize(st));
    bool all_done = true;
    for (int c = 0; c < nrhs; ++c) all_done = all_done && res.done[c];
    if (all_done || cyc >= maxit) break;
  }
  return LS_OK;
#undef HIPTRY
}

ls_status solve_gmres(ls_ctx *h, const double *b_in, double *x_out, int nrhs, int64_t ld, const ls_solve_opts &o,
                      ls_solve_info *info, hipStream_t st) {
  const auto t_start = std::chrono::steady_clock::now();
  const int64_t n = h->n_total;
  const Mode mode = o.adjoint ? Mode::Adjoint : Mode::Forward;
  SolveWs *ws = solve_ws(h, 0), *wi = solve_ws(h, 1), *wt = solve_ws(h, 2);
#define HIPTRY(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) return setup_fail(h, LS_ERR_HIP, hipGetErrorString(e_)); \
  } while (0)
  // contiguous copies of b and x plus the residual check buffers (top-level workspace)
  const size_t vb = sizeof(double2) * (size_t)n * nrhs;
  HIPTRY(ensure(wt->vecs, wt->vec_bytes, 4 * vb));
  double2 *bb = (double2 *)wt->vecs, *xs = bb + (size_t)n * nrhs, *r = xs + (size_t)n * nrhs,
          *t = r + (size_t)n * nrhs;
  HIPTRY(hipMemcpy2DAsync(bb, n * sizeof(double2), b_in, ld * sizeof(double2), n * sizeof(double2), nrhs,
                          hipMemcpyDeviceToDevice, st));
  if (o.x0_given)
    HIPTRY(hipMemcpy2DAsync(xs, n * sizeof(double2), x_out, ld * sizeof(double2), n * sizeof(double2), nrhs,
                            hipMemcpyDeviceToDevice, st));
  // LS_MIXED: with inner_maxit > 0, flexible GMRES whose preconditioner is inner_maxit steps of
  // mixed-precision GMRES (to inner_tol); otherwise relaxed GMRES switching to the mixed operator
  // once the residual is below tol / inner_tol (inner_tol = relative accuracy granted to it),
  // followed by FP64 refinement passes from the true residual if that missed tol
  const bool mixed = o.prec == LS_MIXED;
  const bool flexible = mixed && o.inner_maxit > 0;
  const double relax = (mixed && !flexible) ? (o.inner_tol > 0 ? o.inner_tol : 1e-3) : 0.0;
  // the relaxed iteration aims its residual estimate below 0.3 tol so that its FP64 residual,
  // perturbed by the mixed applications, still meets tol without a (Krylov-space-losing) restart
  CoreOpts co{relax > 0 ? 0.3 * o.tol : o.tol, o.maxit, o.restart, mode, LS_FP64, flexible,
              o.inner_tol > 0 ? o.inner_tol : 1e-12, o.inner_maxit, o.x0_given != 0, relax};
  CoreResult res;
  ls_status status = gmres_core(h, ws, wi, bb, xs, nrhs, co, res, st);
  if (status < 0) return status;
  for (int pass = 0; pass < 3 && relax > 0; ++pass) {
    // refinement from the FP64 residual for columns the relaxed iteration left above tol
    int used = 0;
    for (int c = 0; c < nrhs; ++c) used = std::max(used, res.iters[c]);
    if (used >= o.maxit) break;
    CoreOpts ro = co;
    ro.x0_given = true;
    ro.tol = o.tol;
    ro.maxit = o.maxit - used;
    CoreResult rr;
    status = gmres_core(h, ws, wi, bb, xs, nrhs, ro, rr, st);
    if (status < 0) return status;
    int more = 0;
    for (int c = 0; c < nrhs; ++c) {
      res.iters[c] += rr.iters[c];
      res.done[c] = rr.done[c];
      more += rr.iters[c];
    }
    res.n_fp64 += rr.n_fp64;
    res.n_mixed += rr.n_mixed;
    if (more == 0) break;   // every column met tol on its FP64 residual
  }
  // true residuals with the FP64 apply
  ls_status s2 = apply_op(h, (const double *)xs, (double *)t, nrhs, n, mode, LS_FP64, st);
  if (s2 != LS_OK) return s2;
  ++res.n_fp64;
  {
    Gmres G{h, st, n, nrhs, mode, ws};
    HIPTRY(G.init(std::max(1, (o.restart > 0 && o.restart < o.maxit) ? o.restart : o.maxit) + 1));
    const dim3 gv(blocks_of(n), nrhs);
    axpy_kernel<<<gv, kBlock, 0, st>>>(n, bb, n, -1.0, t, n, r, n);
    std::vector<double2 *> tbl(G.max_vec + 3, nullptr);
    tbl[G.max_vec + 2] = r;
    HIPTRY(hipMemcpyAsync(G.ptrs, tbl.data(), sizeof(double2 *) * tbl.size(), hipMemcpyHostToDevice, st));
    HIPTRY(G.norms(r, nullptr));
    std::vector<double> rn(nrhs), bn(nrhs);
    HIPTRY(hipMemcpyAsync(rn.data(), G.beta, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    HIPTRY(hipStreamSynchronize(st));
    tbl[G.max_vec + 2] = bb;
    HIPTRY(hipMemcpyAsync(G.ptrs, tbl.data(), sizeof(double2 *) * tbl.size(), hipMemcpyHostToDevice, st));
    HIPTRY(G.norms(bb, nullptr));
    HIPTRY(hipMemcpyAsync(bn.data(), G.beta, sizeof(double) * nrhs, hipMemcpyDeviceToHost, st));
    HIPTRY(hipMemcpy2DAsync(x_out, ld * sizeof(double2), xs, n * sizeof(double2), n * sizeof(double2), nrhs,
                            hipMemcpyDeviceToDevice, st));
    HIPTRY(hipStreamSynchronize(st));
    status = LS_OK;
    for (int c = 0; c < nrhs; ++c) {
      const double rr = bn[c] > 0 ? rn[c] / bn[c] : 0.0;
      if (info && info->relres) info->relres[c] = rr;
      if (info && info->iters) info->iters[c] = res.iters[c];
      if (!res.done[c]) status = LS_NOT_CONVERGED;
    }
  }
  if (info) {
    info->n_apply_fp64 = res.n_fp64 * nrhs;
    info->n_apply_mixed = res.n_mixed * nrhs;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  }
  return status;
#undef HIPTRY
}

ls_status grad_contrast(ls_ctx *h, const double *u, const double *lam, const double *a, int nrhs, int64_t ld,
                        double *grad, hipStream_t st) {
  const int64_t n = h->n_total;
  SolveWs *ws = solve_ws(h, 2);
  // P = V^H lam, written with the caller's leading dimension
  const size_t pb = sizeof(double2) * (size_t)ld * nrhs;
  if (ensure(ws->vecs, ws->vec_bytes, std::max(pb, 4 * sizeof(double2) * (size_t)n * nrhs)) != hipSuccess)
    return setup_fail(h, LS_ERR_ALLOC, "workspace");
  double2 *P = (double2 *)ws->vecs;
  ls_status s2 = apply_op(h, lam, (double *)P, nrhs, ld, Mode::AdjointPotential, LS_FP64, st);
  if (s2 != LS_OK) return s2;
  for (const Scat &sc : h->sc) {
    grad_kernel<<<blocks_of(sc.n), kBlock, 0, st>>>(sc.n, sc.off, nrhs, sc.k * sc.k, (const double2 *)u,
                                                   (const double2 *)a, P, ld, ld, grad);
  }
  if (hipGetLastError() != hipSuccess) return setup_fail(h, LS_ERR_HIP, "grad kernel launch");
  return LS_OK;
}

void free_solve_ws(ls_ctx *h) {
  SolveWs *all = (SolveWs *)h->ws_solve.ptr;
  if (!all) return;
  for (int l = 0; l < 3; ++l) {
    SolveWs *ws = all + l;
    for (void *p : ws->V.chunks) (void)hipFree(p);
    for (void *p : ws->Z.chunks) (void)hipFree(p);
    if (ws->small) (void)hipFree(ws->small);
    if (ws->part) (void)hipFree(ws->part);
    if (ws->vecs) (void)hipFree(ws->vecs);
  }
  delete[] all;
  h->ws_solve.ptr = nullptr;
}

}  // namespace lsk
