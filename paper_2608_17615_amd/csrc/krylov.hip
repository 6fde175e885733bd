// GMRES without restart (paper, Section 6 setup: the Nystrom system L u = b is solved by GMRES
// without restart; here unpreconditioned), per right-hand side, on the device, and the contrast
// gradient of a far-field misfit.
//
// Independent systems: with several scatterers in one handle the operator is block diagonal, so
// right-hand side c restricted to scatterer s is a system of its own (q = c * nseg + s) with its
// own Krylov space, Hessenberg matrix and convergence test.  All systems step together (one
// batched operator application per step covers every scatterer and column), but a converged
// system drops out of the orthogonalisation, and each one takes only the iterations its own
// scatterer needs.
//
// Arnoldi: classical Gram-Schmidt with one re-orthogonalisation pass (CGS2) in FP64.  Every
// inner product is a two-stage deterministic reduction (fixed-order partials over tiles that
// never straddle two scatterers, then a fixed-order sum), so results do not depend on
// scheduling.  The basis lives in chunks of device memory kept by the handle between solves and
// grows with the iteration.  Per iteration the host receives the new Hessenberg column
// (2 (j+1) + 1 values per system) and applies the complex Givens rotations; everything of size
// N stays on the device.
//
// Mixed precision (LS_MIXED): relaxed GMRES (FP64 applications until the residual is small
// enough for the mixed-precision operator's error, mixed after, FP64 refinement from the true
// residual), or flexible GMRES whose preconditioner is an inner GMRES solve with the
// mixed-precision operator; the outer FP64 iteration removes the inner solve's error.
//
// Progress: with the environment variable LS_PROGRESS=k the solver prints the step, the largest
// residual estimate and the number of active systems every k steps (flexible GMRES: every outer
// step) to stderr.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "internal.h"

namespace lsk {

namespace {

constexpr int kBlock = 256;
constexpr int kEPT = 4;                      // elements per thread in the dot kernel
constexpr int kTile = kBlock * kEPT;
constexpr int kGroup = 8;                    // basis vectors per dot-product block

typedef std::complex<double> cplx;

// A tile of at most kTile consecutive elements of one scatterer's segment.
struct TileDesc {
  int64_t start;
  int len, seg;
};

// part[(tile * nrhs + c) * nv + i] = sum over the tile of conj(V_i[c][n]) w[c][n].
// grid (tiles, ceil(nv / kGroup), nrhs): each block forms kGroup inner products over one tile, so
// even a single short column (one right-hand side) spreads over many workgroups, and the
// kGroup x kEPT loads of a thread are independent.  Blocks of inactive systems return at once.
__global__ __launch_bounds__(kBlock) void dots_kernel(int nrhs, int nv, int nseg, const TileDesc *__restrict__ tiles,
                                                      const int *__restrict__ active, const double2 *const *V,
                                                      int64_t ldv, const double2 *__restrict__ w, int64_t ldw,
                                                      double2 *__restrict__ part) {
  __shared__ double2 lds[kGroup][kBlock / 64];
  const TileDesc td = tiles[blockIdx.x];
  const int i0 = blockIdx.y * kGroup;
  const int c = blockIdx.z;
  if (!active[c * nseg + td.seg]) return;
  double2 wv[kEPT];
#pragma unroll
  for (int e = 0; e < kEPT; ++e) {
    const int loc = e * kBlock + threadIdx.x;
    wv[e] = loc < td.len ? w[(int64_t)c * ldw + td.start + loc] : make_double2(0.0, 0.0);
  }
  double2 acc[kGroup];
#pragma unroll
  for (int g = 0; g < kGroup; ++g) {
    acc[g] = make_double2(0.0, 0.0);
    if (i0 + g < nv) {
      const double2 *v = V[i0 + g] + (int64_t)c * ldv + td.start;
#pragma unroll
      for (int e = 0; e < kEPT; ++e) {
        const int loc = e * kBlock + threadIdx.x;
        if (loc < td.len) {
          const double2 a = v[loc];
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

// out[q * ldo + i] = sum over the tiles [seg_tiles[s].x, seg_tiles[s].y) of system q = c nseg + s
// (fixed order); zero for inactive systems.  Optionally writes sqrt(real part) of entry 0 to
// beta[q] (norm mode).
__global__ void reduce_kernel(int nrhs, int nv, int nseg, const int2 *__restrict__ seg_tiles,
                              const int *__restrict__ active, const double2 *__restrict__ part, double2 *out,
                              int64_t ldo, double *beta) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nrhs * nseg * nv) return;
  const int q = t / nv, i = t - q * nv;
  const int c = q / nseg, s = q - c * nseg;
  double2 r = make_double2(0.0, 0.0);
  if (active[q]) {
    const int2 tr = seg_tiles[s];
    for (int k = tr.x; k < tr.y; ++k) {
      const double2 p = part[((int64_t)k * nrhs + c) * nv + i];
      r.x += p.x;
      r.y += p.y;
    }
  }
  if (out) out[(int64_t)q * ldo + i] = r;
  if (beta) beta[q] = std::sqrt(r.x);
}

// w[c][n] += sign * sum_{i < nv} V_i[c][n] h[q * ldh + i] for the system q of element n
// (active systems only); grid (tiles * kEPT, nrhs)
__global__ __launch_bounds__(kBlock) void update_kernel(int nv, int nseg, const TileDesc *__restrict__ tiles,
                                                        const int *__restrict__ active, const double2 *const *V,
                                                        int64_t ldv, const double2 *__restrict__ hcoef, int64_t ldh,
                                                        double sign, double2 *__restrict__ w, int64_t ldw) {
  const TileDesc td = tiles[blockIdx.x / kEPT];
  const int loc = (blockIdx.x % kEPT) * kBlock + threadIdx.x;
  const int c = blockIdx.y;
  const int q = c * nseg + td.seg;
  if (loc >= td.len || !active[q]) return;
  const int64_t idx = td.start + loc;
  double ar = 0.0, ai = 0.0;
  const double2 *hc = hcoef + (int64_t)q * ldh;
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

// flag[q] = 1 for an active system whose vector w kept less than a twentieth of its norm after
// the first Gram-Schmidt projection h (h[q ldh + i], i < nv; h[q ldh + nv] = ||w||^2 before it):
// the test of Daniel, Gragg, Kaufman and Stewart with eta = 1/20, against a cancellation that
// would cost more than a digit of orthogonality.  Their usual eta = 1/sqrt(2) flags nearly every
// step of these solves (||w_after|| / ||w_before|| has a median of about 0.4).  One classical pass
// took the same steps as two in dense runs (N = 6 400, k = 20: 264 steps, basis orthogonal to
// 5e-7 at the end; N = 10 000, k = 40: 4e-13 after 3 000 steps), and the same 1 054 steps at
// N = 122 500, k = 40, with half the basis traffic.
__global__ void reorth_flags_kernel(int nsys, int nv, const int *__restrict__ active, const double2 *__restrict__ h,
                                    int64_t ldh, int *__restrict__ flag) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nsys) return;
  int f = 0;
  if (active[q]) {
    const double2 *hq = h + (int64_t)q * ldh;
    double proj = 0.0;
    for (int i = 0; i < nv; ++i) proj = std::fma(hq[i].x, hq[i].x, std::fma(hq[i].y, hq[i].y, proj));
    const double w0 = hq[nv].x;
    f = (w0 - proj) < (1.0 / 400.0) * w0 ? 1 : 0;
  }
  flag[q] = f;
}

// y[c][n] = a[c][n] * (1 / beta[q]) for active systems (beta[q] > 0), and 0 for inactive ones, a
// and y possibly the same; grid (tiles * kEPT, nrhs).  Zeroing keeps the vectors of a finished
// system bounded (the operator maps 0 to 0), so its later basis vectors, which enter the final
// update with zero weights, stay exactly zero.
__global__ __launch_bounds__(kBlock) void scale_kernel(int nseg, const TileDesc *__restrict__ tiles,
                                                       const int *__restrict__ active,
                                                       const double *__restrict__ beta, const double2 *a,
                                                       int64_t lda, double2 *y, int64_t ldy) {
  const TileDesc td = tiles[blockIdx.x / kEPT];
  const int loc = (blockIdx.x % kEPT) * kBlock + threadIdx.x;
  const int c = blockIdx.y;
  const int q = c * nseg + td.seg;
  if (loc >= td.len) return;
  const int64_t idx = td.start + loc;
  const double bt = beta[q];
  if (!active[q] || !(bt > 0.0)) {
    y[(int64_t)c * ldy + idx] = make_double2(0.0, 0.0);   // a may hold anything here
    return;
  }
  const double s = 1.0 / bt;
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
  void *meta = nullptr;      // tile table, per-scatterer tile ranges, active flags
  size_t meta_bytes = 0;
  void *vecs = nullptr;      // r, t, inner workspaces
  size_t vec_bytes = 0;
  void *grid = nullptr;      // grid vectors of the library's preconditioner (c, S c, temporary)
  size_t grid_bytes = 0;
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
    hipError_t e = lsk::dmalloc(&p, cb);
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
  hipError_t e = lsk::dmalloc(&p, need);
  if (e == hipSuccess) have = need;
  return e;
}

// three auxiliary streams at the default priority (a fourth chain goes back to the first), with
// their join events and the fork event, created once per handle
constexpr int kAuxStreams = 3;
hipError_t aux_streams_ready(ls_ctx *h) {
  if (!h->aux_streams.empty()) return hipSuccess;
  hipError_t e = hipEventCreateWithFlags(&h->aux_fork, hipEventDisableTiming);
  for (int a = 0; a < kAuxStreams && e == hipSuccess; ++a) {
    hipStream_t q = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
    if (e != hipSuccess) break;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      (void)hipStreamDestroy(q);
      break;
    }
    h->aux_streams.push_back(q);
    h->aux_join.push_back(ev);
  }
  return e;
}

SolveWs *solve_ws(ls_ctx *h, int level) {
  if (!h->ws_solve.ptr) h->ws_solve.ptr = new SolveWs[3]();
  return (SolveWs *)h->ws_solve.ptr + level;
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// One GMRES engine shared by the plain, relaxed and flexible variants.
struct Gmres {
  ls_ctx *h;
  hipStream_t st;
  int64_t n;
  int nrhs;
  Mode mode;
  SolveWs *ws;
  int nseg = 1, nsys = 1, ntile = 0;
  // device scratch
  double2 *part = nullptr, *hbuf = nullptr, *ybuf = nullptr;
  double *beta = nullptr;
  double2 **ptrs = nullptr;   // device table of basis pointers; entry max_vec + 2 is the norm slot
  TileDesc *tiles = nullptr;
  int2 *seg_tiles = nullptr;
  int *active = nullptr;
  int *reorth = nullptr;   // per system: a second Gram-Schmidt pass runs in this step
  int max_vec = 0;
  const double2 *slot_vec = nullptr;   // the vector in the norm slot (host copy of that entry)

  hipError_t init(int maxvec) {
    max_vec = maxvec;
    nseg = (int)h->sc.size();
    nsys = nrhs * nseg;
    // tiles of at most kTile elements inside each scatterer's segment
    std::vector<TileDesc> tl;
    std::vector<int2> sr(nseg);
    for (int s = 0; s < nseg; ++s) {
      const Scat &sc = h->sc[s];
      sr[s].x = (int)tl.size();
      for (int64_t a = 0; a < sc.n; a += kTile)
        tl.push_back(TileDesc{sc.off + a, (int)std::min<int64_t>(kTile, sc.n - a), s});
      sr[s].y = (int)tl.size();
    }
    ntile = (int)tl.size();
    const size_t need = 2 * sizeof(double2) * (size_t)nsys * (maxvec + 1) +          // h, y
                        sizeof(double) * nsys + sizeof(double2 *) * (size_t)(2 * maxvec + 8) + 1024;
    hipError_t e = ensure(ws->small, ws->small_bytes, need);
    if (e != hipSuccess) return e;
    const size_t mneed = sizeof(TileDesc) * tl.size() + sizeof(int2) * nseg + 2 * sizeof(int) * nsys + 1024;
    e = ensure(ws->meta, ws->meta_bytes, mneed);
    if (e != hipSuccess) return e;
    e = ensure_part(16);
    if (e != hipSuccess) return e;
    char *p = (char *)ws->small;
    hbuf = (double2 *)p;
    p += sizeof(double2) * (size_t)nsys * (maxvec + 1);
    ybuf = (double2 *)p;
    p += sizeof(double2) * (size_t)nsys * (maxvec + 1);
    beta = (double *)p;
    p += sizeof(double) * nsys;
    p = (char *)(((uintptr_t)p + 255) & ~(uintptr_t)255);
    ptrs = (double2 **)p;
    char *m = (char *)ws->meta;
    tiles = (TileDesc *)m;
    m += sizeof(TileDesc) * tl.size();
    m = (char *)(((uintptr_t)m + 255) & ~(uintptr_t)255);
    seg_tiles = (int2 *)m;
    m += sizeof(int2) * nseg;
    m = (char *)(((uintptr_t)m + 255) & ~(uintptr_t)255);
    active = (int *)m;
    m += sizeof(int) * nsys;
    m = (char *)(((uintptr_t)m + 255) & ~(uintptr_t)255);
    reorth = (int *)m;
    e = hipMemcpyAsync(tiles, tl.data(), sizeof(TileDesc) * tl.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(seg_tiles, sr.data(), sizeof(int2) * nseg, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // host tables go out of scope
    return e;
  }

  // device copy of the active flags (host vector of nsys entries)
  hipError_t set_active(const std::vector<int> &flags) {
    return hipMemcpyAsync(active, flags.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, st);
  }

  // partials for nv inner products per column; grows geometrically, after the stream has drained
  // (the old buffer may still be read by a queued reduction)
  hipError_t ensure_part(int nv) {
    const size_t per = sizeof(double2) * (size_t)(ntile > 0 ? ntile : 1) * nrhs;
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

  // out[q][0..nv) = V[0..nv)^H w per system flagged in mask (default: the active ones; zero for
  // the others), using the pointer table entries [0, nv)
  hipError_t dots(int nv, const double2 *w, double2 *out, int64_t ldo, const int *mask = nullptr) {
    hipError_t e0 = ensure_part(nv);
    if (e0 != hipSuccess) return e0;
    if (!mask) mask = active;
    dim3 g((unsigned)ntile, (unsigned)((nv + kGroup - 1) / kGroup), nrhs);
    dots_kernel<<<g, kBlock, 0, st>>>(nrhs, nv, nseg, tiles, mask, ptrs, n, w, n, part);
    reduce_kernel<<<(unsigned)((nsys * nv + 255) / 256), 256, 0, st>>>(nrhs, nv, nseg, seg_tiles, mask, part, out,
                                                                       ldo, nullptr);
    return hipGetLastError();
  }

  // puts v in the norm slot of the device pointer table
  hipError_t set_slot(const double2 *v) {
    slot_vec = v;
    return hipMemcpyAsync(ptrs + max_vec + 2, &slot_vec, sizeof(double2 *), hipMemcpyHostToDevice, st);
  }

  // beta[q] = ||v_q|| per active system for the vector v in the norm slot
  hipError_t norms() {
    dim3 g((unsigned)ntile, 1, nrhs);
    dots_kernel<<<g, kBlock, 0, st>>>(nrhs, 1, nseg, tiles, active, ptrs + max_vec + 2, n, slot_vec, n, part);
    reduce_kernel<<<(unsigned)((nsys + 255) / 256), 256, 0, st>>>(nrhs, 1, nseg, seg_tiles, active, part, nullptr, 1,
                                                                  beta);
    return hipGetLastError();
  }

  dim3 tile_grid() const { return dim3((unsigned)ntile * kEPT, nrhs); }
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
  int progress;          // > 0: print a progress line every this many steps
  const PrecondCb *pc = nullptr;   // flexible: z_j = P v_j instead of an inner solve
  bool all_mixed = false;          // every Arnoldi application in the mixed precision (the residual
                                   // at the start of a cycle stays FP64)
  double pass_reduce = 0.0;        // > 0: a cycle stops once its residual estimate is below
                                   // max(0.3 tol, pass_reduce x the largest starting residual)
  bool close_update = false;       // a refinement cycle that starts from a small FP64 residual
                                   // closes on r - L_mixed dx instead of a new FP64 residual
  bool close_relaxed = false;      // a relaxed flexible cycle (z_j = P v_j kept) closes on its
                                   // basis residual when the mixed steps' bound allows it
  double close_tol = 0.0;          // the caller's tolerance for these closing checks
  bool check_orth = false;         // measure each new basis vector's loss of orthogonality
};

// The closing check of a refinement cycle by the residual update r_new = r - L_mixed dx, with r
// the cycle's FP64 starting residual and dx the cycle's correction of x; r_new is formed from the
// Arnoldi basis (no operator application).  It differs from the FP64 residual b - L (x + dx) by
// (L - L_mixed) dx, i.e. by the mixed far sum's error on dx, at most kCloseEps (||L_mixed dx|| +
// ||dx||) (the far sum K = L - I is bounded by those two): 50 times the 2-norm error of the mixed
// operators measured on the workloads (split FP16 1.8e-7, FP32 tiles 2.9e-7).  A system is closed
// only if its updated residual plus that bound meets tol, and the check runs only when it can
// succeed (kCloseEps ||r|| <= tol ||b|| / 2), so it is not tried on the first pass from x = 0.
// A relaxed cycle (FP64 applications first, mixed ones once the residual allows) has
// r - sum_j y_j L_j z_j = V Q^H g_m e_m with L_j the operator of step j, so its basis residual
// differs from the FP64 one by (L_mixed - L) dm, dm = sum over the mixed steps of y_j z_j, at most
// kCloseEps (||L_mixed dm|| + ||dm||) with L_mixed dm = V sum_{j mixed} y_j h_j (h_j the unrotated
// Hessenberg column).
constexpr double kCloseEps = 1e-5;

struct CoreResult {
  std::vector<int> iters;   // per system
  std::vector<char> done;   // per system
  // the call ended at a cycle's start because every system met tol on its FP64 residual: the
  // residual and right-hand-side norms of that check (x has not changed since)
  bool start_done = false;
  std::vector<double> rn0, bn0;
  // the call closed every system by the residual update (CoreOpts::close_update); rn0 and bn0 then
  // hold the updated residuals' norms and those of b
  bool closed = false;
  int64_t n_fp64 = 0, n_mixed = 0;
  int64_t n_reorth = 0;     // system-steps that took a second Gram-Schmidt pass
  double orth_loss = 0.0;   // CoreOpts::check_orth: max |<v_i, v_j> - delta_ij| of the outer basis
};

// GMRES on contiguous (ld = n) device vectors b, x of nrhs columns, one independent system per
// (column, scatterer).  x holds the initial guess when o.x0_given, the approximate solution on
// return.  Systems with (*only)[q] == 0 (when given) are left alone.  ws is this level's
// workspace; the flexible variant runs its inner solves with a second workspace.
ls_status gmres_core(ls_ctx *h, SolveWs *ws, SolveWs *ws_inner, const double2 *b, double2 *x, int nrhs,
                     const CoreOpts &o, CoreResult &res, hipStream_t st, const std::vector<int> *only = nullptr) {
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
  const int nseg = G.nseg, nsys = G.nsys;
  const size_t vb = sizeof(double2) * (size_t)n * nrhs;
  const bool any_close = o.close_update || o.close_relaxed;
  HIPTRY(ensure(ws->vecs, ws->vec_bytes, (any_close ? 3 : 2) * vb));
  double2 *r = (double2 *)ws->vecs;
  double2 *t = r + (size_t)n * nrhs;
  double2 *d = any_close ? t + (size_t)n * nrhs : nullptr;   // the closing check's residual
  // the basis grows chunk by chunk as the iteration needs it (a solve that converges early never
  // holds maxit vectors); new chunks enter the device pointer table as they arrive
  HIPTRY(ensure_chunks(ws->V, 1, n, nrhs));
  if (o.flexible) HIPTRY(ensure_chunks(ws->Z, 1, n, nrhs));
  std::vector<double2 *> tbl(cyc + 1, nullptr);
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
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // tbl entries may move when tbl is reused
    have = upto;
    return e;
  };
  auto norms_of = [&](const double2 *v, std::vector<double> &out) -> hipError_t {
    hipError_t e = G.set_slot(v);
    if (e == hipSuccess) e = G.norms();
    if (e == hipSuccess) e = hipMemcpyAsync(out.data(), G.beta, sizeof(double) * nsys, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
  };
  HIPTRY(grow(1));
  // applications leave out scatterers none of whose systems is in play (cleared on every exit)
  struct SkipReset {
    ls_ctx *h;
    ~SkipReset() { h->scat_skip.clear(); }
  } skip_reset{h};
  auto set_skip = [&](const std::vector<int> &flags) {
    if (nseg == 1) return;
    h->scat_skip.assign(nseg, 1);
    for (int q = 0; q < nsys; ++q)
      if (flags[q]) h->scat_skip[q % nseg] = 0;
  };
  // systems in play: all, or those the caller names; the others count as done from the start
  std::vector<int> act(nsys, 1);
  if (only)
    for (int q = 0; q < nsys; ++q) act[q] = (*only)[q] ? 1 : 0;
  HIPTRY(G.set_active(act));
  std::vector<double> bnorm(nsys, 0.0);
  HIPTRY(norms_of(b, bnorm));
  for (int q = 0; q < nsys; ++q)
    if (act[q] && !std::isfinite(bnorm[q])) return setup_fail(h, LS_ERR_NONFINITE, "non-finite right-hand side");
  if (!o.x0_given) HIPTRY(hipMemsetAsync(x, 0, vb, st));
  res.iters.assign(nsys, 0);
  res.done.assign(nsys, 0);
  for (int q = 0; q < nsys; ++q) res.done[q] = act[q] ? 0 : 1;
  std::vector<double> est(nsys, 1.0);
  int total_it = 0;
  bool first_cycle = true;
  // Hessenberg columns packed per system: column j (rows 0..j+1) starts at j (j + 3) / 2, grown
  // one column per step
  std::vector<std::vector<cplx>> H(nsys);
  std::vector<cplx> cs, sn, g;
  std::vector<double2> hh((size_t)nsys * (cyc + 2) * 2);
  std::vector<int> rflag(nsys, 0);
  std::vector<double> betah(nsys), rnorm(nsys);
  std::vector<double2> oc;   // check_orth: the new basis vector's inner products, per system
  const dim3 gv(blocks_of(n), nrhs);
  const dim3 gt = G.tile_grid();
  while (total_it < maxit) {
    const bool first_of_call = first_cycle;
    // r = b - L x (FP64), skipped while x = 0
    if (first_cycle && !o.x0_given) {
      HIPTRY(hipMemcpyAsync(r, b, vb, hipMemcpyDeviceToDevice, st));
    } else {
      const ls_precision pr = (o.flexible || o.relax_eps > 0 || o.all_mixed) ? LS_FP64 : o.matvec;
      for (int q = 0; q < nsys; ++q) act[q] = res.done[q] ? 0 : 1;
      set_skip(act);
      ls_status s2 = apply_op(h, (const double *)x, (double *)t, nrhs, n, o.mode, pr, st);
      if (s2 != LS_OK) return s2;
      if (pr == LS_FP64) ++res.n_fp64; else ++res.n_mixed;
      axpy_kernel<<<gv, kBlock, 0, st>>>(n, b, n, -1.0, t, n, r, n);
      HIPTRY(hipGetLastError());
    }
    first_cycle = false;
    for (int q = 0; q < nsys; ++q) act[q] = res.done[q] ? 0 : 1;
    HIPTRY(G.set_active(act));
    HIPTRY(norms_of(r, rnorm));
    bool all = true;
    for (int q = 0; q < nsys; ++q) {
      if (res.done[q]) continue;
      est[q] = bnorm[q] > 0 ? rnorm[q] / bnorm[q] : 0.0;
      if (!std::isfinite(est[q])) return setup_fail(h, LS_ERR_NONFINITE, "non-finite residual");
      res.done[q] = est[q] <= o.tol;
      act[q] = res.done[q] ? 0 : 1;
      all = all && res.done[q];
    }
    if (all) {
      // the residual was taken with the FP64 operator unless this is the unapplied x = 0 start
      res.start_done = !(first_of_call && !o.x0_given) && (o.flexible || o.relax_eps > 0 || o.all_mixed ||
                                                           o.matvec == LS_FP64);
      res.rn0 = rnorm;
      res.bn0 = bnorm;
      break;
    }
    // the Arnoldi iteration's own target: tol, or for a refinement pass the reduction it is
    // asked for (its estimate follows the mixed-precision operator, so the pass stops where the
    // FP64 residual can still follow it)
    double tol_it = o.tol;
    if (o.pass_reduce > 0) {
      double w = 0.0;
      for (int q = 0; q < nsys; ++q)
        if (act[q]) w = std::max(w, est[q]);
      tol_it = std::max(0.3 * o.tol, o.pass_reduce * w);
    }
    HIPTRY(G.set_active(act));
    scale_kernel<<<gt, kBlock, 0, st>>>(nseg, G.tiles, G.active, G.beta, r, n, tbl[0], n);
    HIPTRY(hipGetLastError());
    const int m = cyc;
    for (auto &hc : H) hc.clear();
    cs.assign((size_t)nsys * m, cplx(0));
    sn.assign((size_t)nsys * m, cplx(0));
    g.assign((size_t)nsys * (m + 1), cplx(0));
    std::vector<int> mc(nsys, 0);
    std::vector<char> step_mixed(m, 0);   // step j applied the mixed operator (relaxed closing)
    const std::vector<int> part_in(act);   // systems that take part in this cycle
    for (int q = 0; q < nsys; ++q) g[(size_t)q * (m + 1)] = rnorm[q];
    int j = 0;
    for (; j < m && total_it < maxit; ++j, ++total_it) {
      HIPTRY(grow(j + 2));
      double2 *vj = tbl[j];
      double2 *w = tbl[j + 1];
      if (o.flexible && o.pc) {
        // z_j = P v_j = v_j + T_C^Q (S c - c), c = T_Q^C v_j (scatterer pc->s only), then w = L z_j
        HIPTRY(ensure_chunks(ws->Z, j + 1, n, nrhs));
        double2 *zj = ws->Z.vec(j, n, nrhs);
        const PrecondCb &pc = *o.pc;
        HIPTRY(hipMemcpyAsync(zj, vj, sizeof(double2) * (size_t)n * nrhs, hipMemcpyDeviceToDevice, st));
        if (pc.s >= 0) {
          const Scat &scp = h->sc[pc.s];
          HIPTRY(launch_quad_to_cart(scp, vj, n, pc.c, pc.ldc, nrhs, st));
          const ls_status sst = pc.S((const double *)pc.c, (double *)pc.sc, nrhs, pc.ldc, pc.user, st);
          if (sst < 0) return setup_fail(h, sst, "the preconditioner's S failed");
          HIPTRY(launch_precond_finish(scp, vj, n, pc.c, pc.sc, pc.ldc, zj, nrhs, st));
        } else {
          // the library's S^(C) per scatterer (P^H with D^-1 S^H D for adjoint solves); scatterers
          // none of whose systems is active keep z = v.  Each scatterer has its own grid buffers,
          // and with several live ones their chains run side by side on the auxiliary streams (a
          // sweep occupies one workgroup per right-hand side): each stream waits for z = v on st,
          // and st for every stream, before the operator application.  The chains write disjoint
          // node ranges of z.
          size_t need = 0;
          for (const Scat &scp : h->sc)
            if (scp.sp) need += 3 * sizeof(double2) * (size_t)scp.sp->nx * scp.sp->ny * nrhs;
          if (need > ws->grid_bytes) {
            HIPTRY(hipStreamSynchronize(st));
            HIPTRY(ensure(ws->grid, ws->grid_bytes, need));
          }
          int live_n = 0;
          for (int si = 0; si < nseg; ++si) {
            if (!h->sc[si].sp) continue;
            for (int c = 0; c < nrhs; ++c)
              if (act[c * nseg + si]) {
                ++live_n;
                break;
              }
          }
          const bool side = live_n > 1;
          if (side) {
            HIPTRY(aux_streams_ready(h));
            HIPTRY(hipEventRecord(h->aux_fork, st));
            for (hipStream_t q : h->aux_streams) HIPTRY(hipStreamWaitEvent(q, h->aux_fork, 0));
          }
          double2 *gbase = (double2 *)ws->grid;
          int used = 0;
          for (int si = 0; si < nseg; ++si) {
            const Scat &scp = h->sc[si];
            if (!scp.sp) continue;
            const int64_t nc = (int64_t)scp.sp->nx * scp.sp->ny;
            double2 *gc = gbase, *gs = gc + (size_t)nc * nrhs, *gt = gs + (size_t)nc * nrhs;
            gbase = gt + (size_t)nc * nrhs;
            bool live = false;
            for (int c = 0; c < nrhs && !live; ++c) live = act[c * nseg + si] != 0;
            if (!live) continue;
            const hipStream_t q = side ? h->aux_streams[used++ % h->aux_streams.size()] : st;
            HIPTRY(launch_quad_to_cart(scp, vj, n, gc, nc, nrhs, q));
            HIPTRY(launch_sparsify(*scp.sp, gc, nc, gs, nc, gt, nc, nrhs, o.mode == Mode::Adjoint, true, q));
            HIPTRY(launch_precond_finish(scp, vj, n, gc, gs, nc, zj, nrhs, q));
          }
          if (side)
            for (size_t a = 0; a < h->aux_streams.size(); ++a) {
              HIPTRY(hipEventRecord(h->aux_join[a], h->aux_streams[a]));
              HIPTRY(hipStreamWaitEvent(st, h->aux_join[a], 0));
            }
        }
        // relaxed: the mixed-precision operator once the residual allows it (as below)
        ls_precision pj = o.all_mixed ? LS_MIXED : LS_FP64;
        if (o.relax_eps > 0) {
          double worst = 0.0;
          for (int q = 0; q < nsys; ++q)
            if (act[q]) worst = std::max(worst, est[q]);
          pj = worst * o.relax_eps <= o.tol ? LS_MIXED : LS_FP64;
        }
        set_skip(act);
        ls_status s2 = apply_op(h, (const double *)zj, (double *)w, nrhs, n, o.mode, pj, st);
        if (s2 != LS_OK) return s2;
        if (pj == LS_FP64) ++res.n_fp64; else ++res.n_mixed;
        step_mixed[j] = pj == LS_MIXED ? 1 : 0;
      } else if (o.flexible) {
        // z_j ~ L^{-1} v_j by an inner GMRES with the mixed-precision operator (active systems
        // only), then w = L z_j
        HIPTRY(ensure_chunks(ws->Z, j + 1, n, nrhs));
        double2 *zj = ws->Z.vec(j, n, nrhs);
        CoreOpts io{o.inner_tol, o.inner_maxit, 0, o.mode, LS_MIXED, false, 0.0, 0, false, 0.0, 0};
        CoreResult ir;
        ls_status s2 = gmres_core(h, ws_inner, nullptr, vj, zj, nrhs, io, ir, st, &act);
        if (s2 < 0) return s2;
        res.n_mixed += ir.n_mixed;
        res.n_fp64 += ir.n_fp64;
        res.n_reorth += ir.n_reorth;
        // an inner solve that took no step (its tolerance already met by z = 0) leaves z_j = 0, a
        // useless direction: those systems take z_j = v_j (no preconditioning in this step)
        std::vector<int> idle(nsys, 0);
        bool any_idle = false;
        for (int q = 0; q < nsys; ++q)
          if (act[q] && ir.iters[q] == 0) idle[q] = any_idle = 1;
        if (any_idle) {
          const std::vector<double2> one(nsys, make_double2(1.0, 0.0));
          HIPTRY(hipMemcpyAsync(G.reorth, idle.data(), sizeof(int) * nsys, hipMemcpyHostToDevice, st));
          HIPTRY(hipMemcpyAsync(G.ybuf, one.data(), sizeof(double2) * nsys, hipMemcpyHostToDevice, st));
          update_kernel<<<gt, kBlock, 0, st>>>(1, nseg, G.tiles, G.reorth, G.ptrs + j, n, G.ybuf, 1, 1.0, zj, n);
          HIPTRY(hipGetLastError());
          HIPTRY(hipStreamSynchronize(st));   // idle and one go out of scope
        }
        set_skip(act);
        s2 = apply_op(h, (const double *)zj, (double *)w, nrhs, n, o.mode, LS_FP64, st);
        if (s2 != LS_OK) return s2;
        ++res.n_fp64;
      } else {
        // relaxed inexact Arnoldi: an application error of relative size eps perturbs the
        // residual by about eps times the current residual, so once the largest active residual
        // estimate is below tol / eps the cheaper mixed-precision operator is accurate enough
        ls_precision pj = o.all_mixed ? LS_MIXED : o.matvec;
        if (o.relax_eps > 0) {
          double worst = 0.0;
          for (int q = 0; q < nsys; ++q)
            if (act[q]) worst = std::max(worst, est[q]);
          pj = worst * o.relax_eps <= o.tol ? LS_MIXED : LS_FP64;
        }
        set_skip(act);
        ls_status s2 = apply_op(h, (const double *)vj, (double *)w, nrhs, n, o.mode, pj, st);
        if (s2 != LS_OK) return s2;
        if (pj == LS_FP64) ++res.n_fp64; else ++res.n_mixed;
      }
      // Gram-Schmidt against V[0..j]: one classical pass, whose dot products include ||w||^2 (w is
      // the table entry j + 1), and a second pass only for the systems reorth_flags_kernel flags
      const int nv = j + 1;
      double2 *h1 = G.hbuf, *h2 = G.ybuf;
      HIPTRY(G.dots(nv + 1, w, h1, nv + 1));
      update_kernel<<<gt, kBlock, 0, st>>>(nv, nseg, G.tiles, G.active, G.ptrs, n, h1, nv + 1, -1.0, w, n);
      reorth_flags_kernel<<<(unsigned)((nsys + 255) / 256), 256, 0, st>>>(nsys, nv, G.active, h1, nv + 1, G.reorth);
      HIPTRY(G.dots(nv, w, h2, nv, G.reorth));
      update_kernel<<<gt, kBlock, 0, st>>>(nv, nseg, G.tiles, G.reorth, G.ptrs, n, h2, nv, -1.0, w, n);
      HIPTRY(G.set_slot(w));
      HIPTRY(G.norms());
      scale_kernel<<<gt, kBlock, 0, st>>>(nseg, G.tiles, G.active, G.beta, w, n, w, n);
      HIPTRY(hipMemcpyAsync(hh.data(), h1, sizeof(double2) * nsys * (nv + 1), hipMemcpyDeviceToHost, st));
      HIPTRY(hipMemcpyAsync(hh.data() + (size_t)nsys * (nv + 1), h2, sizeof(double2) * nsys * nv,
                            hipMemcpyDeviceToHost, st));
      HIPTRY(hipMemcpyAsync(betah.data(), G.beta, sizeof(double) * nsys, hipMemcpyDeviceToHost, st));
      HIPTRY(hipMemcpyAsync(rflag.data(), G.reorth, sizeof(int) * nsys, hipMemcpyDeviceToHost, st));
      if (o.check_orth) {
        // <v_i, v_{j+1}> for i <= j and ||v_{j+1}||^2 of the normalized new vector: one more pass of
        // inner products (into h2, whose copy to the host is already enqueued before it)
        oc.resize((size_t)nsys * (nv + 1));
        HIPTRY(G.dots(nv + 1, w, h2, nv + 1));
        HIPTRY(hipMemcpyAsync(oc.data(), h2, sizeof(double2) * oc.size(), hipMemcpyDeviceToHost, st));
      }
      HIPTRY(hipStreamSynchronize(st));
      for (int q = 0; q < nsys; ++q) res.n_reorth += rflag[q];
      if (o.check_orth)
        for (int q = 0; q < nsys; ++q) {
          if (!act[q] || !(betah[q] > 0.0)) continue;   // no new vector for this system
          const double2 *c = &oc[(size_t)q * (nv + 1)];
          double l = std::hypot(c[nv].x - 1.0, c[nv].y);
          for (int i = 0; i < nv; ++i) l = std::max(l, std::hypot(c[i].x, c[i].y));
          res.orth_loss = std::max(res.orth_loss, l);
        }
      bool any = false, changed = false;
      double worst = 0.0;
      for (int q = 0; q < nsys; ++q) {
        if (!act[q]) continue;
        std::vector<cplx> &Hv = H[q];
        Hv.resize((size_t)(j + 1) * (j + 4) / 2, cplx(0));
        cplx *Hc = Hv.data();
        auto Hat = [&](int r_, int c_) -> cplx & { return Hc[(size_t)c_ * (c_ + 3) / 2 + r_]; };
        for (int i = 0; i < nv; ++i) {
          const double2 a = hh[(size_t)q * (nv + 1) + i], bq = hh[(size_t)nsys * (nv + 1) + (size_t)q * nv + i];
          Hat(i, j) = cplx(a.x + bq.x, a.y + bq.y);
        }
        Hat(j + 1, j) = betah[q];
        if (!std::isfinite(betah[q])) return setup_fail(h, LS_ERR_BREAKDOWN, "non-finite Arnoldi vector");
        cplx *csc = &cs[(size_t)q * m], *snc = &sn[(size_t)q * m], *gc = &g[(size_t)q * (m + 1)];
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
        mc[q] = j + 1;
        res.iters[q]++;
        est[q] = bnorm[q] > 0 ? std::abs(gc[j + 1]) / bnorm[q] : 0.0;
        if (est[q] <= tol_it || betah[q] == 0.0) {
          act[q] = 0;
          res.done[q] = 1;
          changed = true;
        } else {
          any = true;
          worst = std::max(worst, est[q]);
        }
      }
      // flexible outer steps each hold a whole inner solve, so every one of them is reported
      if (o.progress > 0 && (o.flexible || (total_it + 1) % o.progress == 0)) {
        int na = 0;
        for (int q = 0; q < nsys; ++q) na += act[q];
        std::fprintf(stderr, "[ls gmres] step %d: largest residual estimate %.3e, %d of %d systems active\n",
                     total_it + 1, worst, na, nsys);
        std::fflush(stderr);
      }
      if (!any) {
        ++j;
        ++total_it;
        break;
      }
      if (changed) HIPTRY(G.set_active(act));
    }
    // x += V y (or Z y for the flexible variant) per system that took part in the cycle
    std::vector<double2> yv((size_t)nsys * m, make_double2(0, 0));
    for (int q = 0; q < nsys; ++q) {
      const int mm = mc[q];
      if (mm == 0) continue;
      const cplx *Hc = H[q].data();
      auto Hat = [&](int r_, int c_) { return Hc[(size_t)c_ * (c_ + 3) / 2 + r_]; };
      std::vector<cplx> yc(mm);
      for (int i = mm - 1; i >= 0; --i) {
        cplx sacc = g[(size_t)q * (m + 1) + i];
        for (int k2 = i + 1; k2 < mm; ++k2) sacc -= Hat(i, k2) * yc[k2];
        yc[i] = sacc / Hat(i, i);
      }
      for (int i = 0; i < mm; ++i) yv[(size_t)q * m + i] = make_double2(yc[i].real(), yc[i].imag());
    }
    const int mmax = std::max(1, *std::max_element(mc.begin(), mc.end()));
    HIPTRY(hipMemcpyAsync(G.hbuf, yv.data(), sizeof(double2) * nsys * m, hipMemcpyHostToDevice, st));
    HIPTRY(G.set_active(part_in));
    // the residual update can close a refinement cycle when its starting residual is small enough,
    // and a relaxed cycle when its mixed steps' bound allows it
    bool closing_pass = o.close_update && o.x0_given;
    for (int q = 0; q < nsys && closing_pass; ++q)
      if (part_in[q] && kCloseEps * rnorm[q] > 0.5 * o.close_tol * bnorm[q]) closing_pass = false;
    const bool closing = closing_pass || o.close_relaxed;
    // dx = V y (or Z y) into t, then x += dx (or straight into x)
    double2 *upd = closing_pass ? t : x;
    if (closing_pass) HIPTRY(hipMemsetAsync(t, 0, vb, st));
    std::vector<double2 *> ztbl;
    if (o.flexible) {
      ztbl.resize(mmax);
      for (int i = 0; i < mmax; ++i) ztbl[i] = ws->Z.vec(i, n, nrhs);
      HIPTRY(hipMemcpyAsync(G.ptrs + G.max_vec + 4, ztbl.data(), sizeof(double2 *) * mmax, hipMemcpyHostToDevice,
                            st));
      update_kernel<<<gt, kBlock, 0, st>>>(mmax, nseg, G.tiles, G.active, G.ptrs + G.max_vec + 4, n, G.hbuf, m, 1.0,
                                           upd, n);
    } else {
      update_kernel<<<gt, kBlock, 0, st>>>(mmax, nseg, G.tiles, G.active, G.ptrs, n, G.hbuf, m, 1.0, upd, n);
    }
    HIPTRY(hipGetLastError());
    HIPTRY(hipStreamSynchronize(st));   // yv and ztbl go out of scope
    if (closing) {
      if (closing_pass) {
        axpy_kernel<<<gv, kBlock, 0, st>>>(n, x, n, 1.0, t, n, x, n);
        HIPTRY(hipGetLastError());
      }
      // r - L_mixed dx without another application: the Arnoldi relation L_mixed Z = V H (H the
      // (m + 1) x m Hessenberg matrix) gives r - L_mixed Z y = V (beta e_0 - H y) = V Q^H (g_m e_m),
      // Q the product of the cycle's Givens rotations and g_m the last entry of the rotated right-hand
      // side (|g_m| is the residual estimate).  Its coefficients u: from w = g_m, for i = m - 1 .. 0,
      // u_{i+1} = c_i w and w <- -s_i w; u_0 = w.
      std::vector<double2> uv((size_t)nsys * (m + 1), make_double2(0, 0));
      for (int q = 0; q < nsys; ++q) {
        if (!part_in[q]) continue;
        const int mm = mc[q];
        const cplx *csc = &cs[(size_t)q * m], *snc = &sn[(size_t)q * m];
        cplx w = g[(size_t)q * (m + 1) + mm];
        double2 *u = &uv[(size_t)q * (m + 1)];
        for (int i = mm - 1; i >= 0; --i) {
          const cplx ui = csc[i] * w;
          u[i + 1] = make_double2(ui.real(), ui.imag());
          w = -snc[i] * w;
        }
        u[0] = make_double2(w.real(), w.imag());
      }
      HIPTRY(hipMemcpyAsync(G.hbuf, uv.data(), sizeof(double2) * uv.size(), hipMemcpyHostToDevice, st));
      HIPTRY(hipMemsetAsync(d, 0, vb, st));
      update_kernel<<<gt, kBlock, 0, st>>>(mmax + 1, nseg, G.tiles, G.active, G.ptrs, n, G.hbuf, m + 1, 1.0, d, n);
      HIPTRY(hipGetLastError());
      HIPTRY(hipStreamSynchronize(st));   // uv goes out of scope
      std::vector<double> rn(nsys), extra(nsys, 0.0);
      HIPTRY(G.set_active(part_in));
      HIPTRY(norms_of(d, rn));
      if (closing_pass) {
        // ||L_mixed dx|| = ||r - r_new|| <= ||r|| + ||r_new||
        std::vector<double> dn(nsys);
        HIPTRY(norms_of(t, dn));
        for (int q = 0; q < nsys; ++q) extra[q] = rnorm[q] + rn[q] + dn[q];
      } else {
        // the mixed steps' part of the correction, dm = sum_{j mixed} y_j z_j, and L_mixed dm =
        // V sum_{j mixed} y_j h_j, h_j the unrotated Hessenberg column (rebuilt from the stored,
        // rotated one by the inverse rotations G_j^H .. G_0^H): (L - L_mixed) dm, the difference
        // between the basis residual and the FP64 one, is at most kCloseEps (||L_mixed dm|| + ||dm||)
        std::vector<double2> cv((size_t)nsys * (m + 1), make_double2(0, 0));
        std::vector<double2> ym((size_t)nsys * m, make_double2(0, 0));
        bool any_mixed = false;
        for (int q = 0; q < nsys; ++q) {
          if (!part_in[q]) continue;
          const int mm = mc[q];
          const cplx *Hc = H[q].data();
          const cplx *csc = &cs[(size_t)q * m], *snc = &sn[(size_t)q * m];
          std::vector<cplx> col(mm + 1), acc(mm + 1, cplx(0));
          for (int jj = 0; jj < mm; ++jj) {
            if (!step_mixed[jj]) continue;
            any_mixed = true;
            std::fill(col.begin(), col.end(), cplx(0));
            for (int i = 0; i <= jj; ++i) col[i] = Hc[(size_t)jj * (jj + 3) / 2 + i];
            for (int i = jj; i >= 0; --i) {
              const cplx a = col[i], b = col[i + 1];
              col[i] = std::conj(csc[i]) * a - snc[i] * b;
              col[i + 1] = std::conj(snc[i]) * a + csc[i] * b;
            }
            const double2 y2 = yv[(size_t)q * m + jj];
            const cplx yj(y2.x, y2.y);
            for (int i = 0; i <= jj + 1; ++i) acc[i] += yj * col[i];
            ym[(size_t)q * m + jj] = y2;
          }
          for (int i = 0; i <= mm; ++i) cv[(size_t)q * (m + 1) + i] = make_double2(acc[i].real(), acc[i].imag());
        }
        if (any_mixed) {
          HIPTRY(hipMemcpyAsync(G.hbuf, cv.data(), sizeof(double2) * cv.size(), hipMemcpyHostToDevice, st));
          HIPTRY(hipMemcpyAsync(G.ybuf, ym.data(), sizeof(double2) * ym.size(), hipMemcpyHostToDevice, st));
          HIPTRY(hipMemsetAsync(d, 0, vb, st));
          HIPTRY(hipMemsetAsync(t, 0, vb, st));
          update_kernel<<<gt, kBlock, 0, st>>>(mmax + 1, nseg, G.tiles, G.active, G.ptrs, n, G.hbuf, m + 1, 1.0, d,
                                               n);
          update_kernel<<<gt, kBlock, 0, st>>>(mmax, nseg, G.tiles, G.active, G.ptrs + G.max_vec + 4, n, G.ybuf, m,
                                               1.0, t, n);
          HIPTRY(hipGetLastError());
          HIPTRY(hipStreamSynchronize(st));   // cv and ym go out of scope
          std::vector<double> ln(nsys), dn(nsys);
          HIPTRY(norms_of(d, ln));
          HIPTRY(norms_of(t, dn));
          for (int q = 0; q < nsys; ++q) extra[q] = ln[q] + dn[q];
        }
      }
      bool all_closed = true;
      for (int q = 0; q < nsys; ++q) {
        if (!part_in[q]) continue;
        const double bq = bnorm[q] > 0 ? bnorm[q] : 1.0;
        const double e = rn[q] / bq, bound = kCloseEps * extra[q] / bq;
        if (!std::isfinite(e)) return setup_fail(h, LS_ERR_NONFINITE, "non-finite residual");
        all_closed = all_closed && e + bound <= o.close_tol;
      }
      if (all_closed) {
        for (int q = 0; q < nsys; ++q)
          if (part_in[q]) rnorm[q] = rn[q];
        res.closed = true;
        res.rn0 = rnorm;
        res.bn0 = bnorm;
        break;
      }
      // some system is not closed: the next pass starts from the FP64 residual of the updated x
    }
    bool all_done = true;
    for (int q = 0; q < nsys; ++q) all_done = all_done && res.done[q];
    if (all_done || cyc >= maxit) break;
  }
  return LS_OK;
#undef HIPTRY
}

ls_status solve_gmres(ls_ctx *h, const double *b_in, double *x_out, int nrhs, int64_t ld, const ls_solve_opts &o,
                      ls_solve_info *info, hipStream_t st, const PrecondCb *pc) {
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
  const char *pe = std::getenv("LS_PROGRESS");
  const int progress = pe ? std::max(0, std::atoi(pe)) : 0;
  // LS_MIXED: with inner_maxit > 0, flexible GMRES whose preconditioner is inner_maxit steps of
  // mixed-precision GMRES (to inner_tol); otherwise relaxed GMRES switching to the mixed operator
  // once the residual is below tol / inner_tol (inner_tol = relative accuracy granted to it,
  // default 1e-4: a later switch than the operator error alone would allow; see ls.h),
  // followed by FP64 refinement passes from the true residual if that missed tol
  // with the preconditioner P (pc): flexible GMRES with z_j = P v_j, its operator applications
  // relaxed to the mixed precision as above when LS_MIXED is asked for
  const bool mixed = o.prec == LS_MIXED;
  const bool flexible = (mixed && o.inner_maxit > 0 && !pc) || pc;
  const double relax = (mixed && (!flexible || pc)) ? (o.inner_tol > 0 ? o.inner_tol : 1e-4) : 0.0;
  // the relaxed iteration aims its residual estimate below 0.3 tol so that its FP64 residual,
  // perturbed by the mixed applications, still meets tol without a (Krylov-space-losing) restart
  CoreOpts co{relax > 0 ? 0.3 * o.tol : o.tol, o.maxit, o.restart, mode, LS_FP64, flexible,
              o.inner_tol > 0 ? o.inner_tol : 1e-12, o.inner_maxit, o.x0_given != 0, relax, progress, pc};
  co.close_tol = o.tol;
  co.check_orth = o.check_orth != 0;
  // a preconditioned relaxed solve keeps its z_j, so it can close on its basis residual
  co.close_relaxed = relax > 0 && pc != nullptr;
  // LS_MIXED with mixed_scheme = 1: refinement passes, each a GMRES cycle from the FP64 residual
  // whose applications are all mixed-precision, stopped once its estimate has fallen by inner_tol
  // (default 1e-5) or below 0.3 tol; the passes repeat until the FP64 residual meets tol
  const bool passes = mixed && o.mixed_scheme == 1;
  if (passes) {
    co.tol = o.tol;
    co.relax_eps = 0.0;
    co.all_mixed = true;
    co.matvec = LS_MIXED;
    co.flexible = pc != nullptr;
    co.pass_reduce = o.inner_tol > 0 ? o.inner_tol : 1e-5;
    co.close_update = true;
    co.close_relaxed = false;
  }
  CoreResult res;
  ls_status status = gmres_core(h, ws, wi, bb, xs, nrhs, co, res, st);
  if (status < 0) return status;
  const int nsys = (int)res.iters.size();
  // the last GMRES call's closing residual check, when it found every system done
  bool have_final = res.start_done || res.closed;
  std::vector<double> rn_final = res.rn0, bn_final = res.bn0;
  for (int pass = 0; pass < 30 && passes && !res.closed; ++pass) {
    int used = 0;
    for (int q = 0; q < nsys; ++q) used = std::max(used, res.iters[q]);
    if (used >= o.maxit) break;
    CoreOpts ro = co;
    ro.x0_given = true;
    ro.maxit = o.maxit - used;
    CoreResult rr;
    status = gmres_core(h, ws, wi, bb, xs, nrhs, ro, rr, st);
    if (status < 0) return status;
    int more = 0;
    for (int q = 0; q < nsys; ++q) {
      res.iters[q] += rr.iters[q];
      res.done[q] = rr.done[q];
      more += rr.iters[q];
    }
    res.n_fp64 += rr.n_fp64;
    res.n_mixed += rr.n_mixed;
    res.n_reorth += rr.n_reorth;
    res.orth_loss = std::max(res.orth_loss, rr.orth_loss);
    have_final = rr.start_done || rr.closed;
    rn_final = rr.rn0;
    bn_final = rr.bn0;
    if (more == 0 || rr.closed) break;   // every system met tol on its FP64 (or updated) residual
  }
  for (int pass = 0; pass < 3 && relax > 0 && !passes && !res.closed; ++pass) {
    // refinement from the FP64 residual for systems the relaxed iteration left above tol
    int used = 0;
    for (int q = 0; q < nsys; ++q) used = std::max(used, res.iters[q]);
    if (used >= o.maxit) break;
    CoreOpts ro = co;
    ro.x0_given = true;
    ro.tol = o.tol;
    ro.maxit = o.maxit - used;
    CoreResult rr;
    status = gmres_core(h, ws, wi, bb, xs, nrhs, ro, rr, st);
    if (status < 0) return status;
    int more = 0;
    for (int q = 0; q < nsys; ++q) {
      res.iters[q] += rr.iters[q];
      res.done[q] = rr.done[q];
      more += rr.iters[q];
    }
    res.n_fp64 += rr.n_fp64;
    res.n_mixed += rr.n_mixed;
    res.n_reorth += rr.n_reorth;
    res.orth_loss = std::max(res.orth_loss, rr.orth_loss);
    have_final = rr.start_done;
    rn_final = rr.rn0;
    bn_final = rr.bn0;
    if (more == 0) break;   // every system met tol on its FP64 residual
  }
  {
    Gmres G{h, st, n, nrhs, mode, ws};
    HIPTRY(G.init(1));
    const int nseg = G.nseg;
    std::vector<double> rn(nsys), bn(nsys);
    if (have_final) {
      // the last GMRES call closed on the FP64 residual of the current x: nothing to recompute
      rn = rn_final;
      bn = bn_final;
    } else {
      // true residuals with the FP64 apply
      ls_status s2 = apply_op(h, (const double *)xs, (double *)t, nrhs, n, mode, LS_FP64, st);
      if (s2 != LS_OK) return s2;
      ++res.n_fp64;
      const dim3 gv(blocks_of(n), nrhs);
      axpy_kernel<<<gv, kBlock, 0, st>>>(n, bb, n, -1.0, t, n, r, n);
      const std::vector<int> all(nsys, 1);
      HIPTRY(G.set_active(all));
      for (int pass = 0; pass < 2; ++pass) {
        HIPTRY(G.set_slot(pass == 0 ? r : bb));
        HIPTRY(G.norms());
        HIPTRY(hipMemcpyAsync((pass == 0 ? rn : bn).data(), G.beta, sizeof(double) * nsys, hipMemcpyDeviceToHost,
                              st));
        HIPTRY(hipStreamSynchronize(st));
      }
    }
    HIPTRY(hipMemcpy2DAsync(x_out, ld * sizeof(double2), xs, n * sizeof(double2), n * sizeof(double2), nrhs,
                            hipMemcpyDeviceToDevice, st));
    HIPTRY(hipStreamSynchronize(st));
    status = LS_OK;
    for (int c = 0; c < nrhs; ++c) {
      // a column's relative residual over all its scatterers; its iterations are the most any
      // of its systems took
      double r2 = 0.0, b2 = 0.0;
      int it = 0;
      bool done = true;
      for (int s = 0; s < nseg; ++s) {
        const int q = c * nseg + s;
        r2 += rn[q] * rn[q];
        b2 += bn[q] * bn[q];
        it = std::max(it, res.iters[q]);
        done = done && res.done[q];
      }
      const double rr = b2 > 0 ? std::sqrt(r2 / b2) : 0.0;
      if (info && info->relres) info->relres[c] = rr;
      if (info && info->iters) info->iters[c] = it;
      // refinement passes end on estimates only when maxit cut them short: check the FP64 residual
      if (passes && rr > o.tol) done = false;
      if (!done) status = LS_NOT_CONVERGED;
    }
  }
  if (info) {
    info->n_apply_fp64 = res.n_fp64 * nrhs;
    info->n_apply_mixed = res.n_mixed * nrhs;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    info->n_reorth = res.n_reorth;
    info->orth_loss = res.orth_loss;
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
    if (ws->meta) (void)hipFree(ws->meta);
    if (ws->vecs) (void)hipFree(ws->vecs);
    if (ws->grid) (void)hipFree(ws->grid);
  }
  delete[] all;
  h->ws_solve.ptr = nullptr;
}

}  // namespace lsk
