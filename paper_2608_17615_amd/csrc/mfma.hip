// Far-field Green's sum for a block of right-hand sides on the matrix cores.
//
// For a wavefront's 16*MT targets and 16*NT right-hand sides, each step over 4 sources forms
// the complex tile  Y[16 x 16] += G[16 x 4] X[4 x 16]  per (M-tile, N-tile) with three real
// 16x16x4 MFMAs (Gauss's three-product form).  The four-product form took 11-15% longer in FP64
// and FP32 alike: the matrix products compete with the Green's evaluation for SIMD cycles.  In
// the 16x16x4 operand layout lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16], so lane l
// evaluates G for exactly the pair (target l % 16 of the tile, source l / 16 of the step) it feeds
// to the matrix core: the Green's tile is built on the VALU in registers and never moves.  B
// operands are the densities of the 4 sources for 16 consecutive right-hand sides ([source][rhs]
// layout, coalesced 16-wide rows).
//   T = double : v_mfma_f64_16x16x4f64, FP64 everywhere (exact variant of the batched sum);
//   T = float  : v_mfma_f32_16x16x4f32 with FP32 Green's values (FP64 for z < 1) and FP32
//                accumulation within one source split; splits are summed in FP64 by the epilogue.
// Result rows: FP32 tiles return D[4 (l/16) + r][l % 16], FP64 tiles D[l/16 + 4 r][l % 16]
// (r = accumulator register), both verified on gfx950.  Green's values are G/K (hankel.h); the
// shared epilogue multiplies the summed partials by K.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "hankel.h"
#include "internal.h"

namespace lsk {

namespace {

constexpr int kBlock = 256;

__constant__ HankelTable m_hankel = kHankelTable;
__constant__ SinCosTable m_sincos = kSinCosTable;
typedef __attribute__((address_space(4))) const HankelTable ConstTab;

__device__ __forceinline__ ConstTab &mtab() {
  ConstTab *t = (ConstTab *)&m_hankel;
  asm volatile("" : "+s"(t));
  return *t;
}

template <class T>
constexpr bool kFP64 = std::is_same<T, double>::value;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <class T>
struct Tile;

template <>
struct Tile<double> {
  typedef v4d acc_t;
  typedef double2 cplx_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
  static __device__ __forceinline__ void green(double A, double &gr, double &gi, const PhaseLds &sct, bool) {
    lsk::green_unit<true>(A, gr, gi, mtab(), sct);
  }
  static __device__ __forceinline__ cplx_t make(double a, double b) { return make_double2(a, b); }
};

template <>
struct Tile<float> {
  typedef v4f acc_t;
  typedef float2 cplx_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
  static __device__ __forceinline__ void green(double A, float &gr, float &gi, const PhaseLds &, bool excl) {
    lsk::green32_unit(A, gr, gi, mtab(), excl);
  }
  static __device__ __forceinline__ cplx_t make(double a, double b) { return make_float2((float)a, (float)b); }
};

// X[i][b] (b < ldx, zero for b >= nrhs): w m x (forward) or x (adjoint) in precision T, plus the
// FP64 f[b][i] = m x (or x) for the sparse correction.
template <class T, Mode M>
__global__ __launch_bounds__(kBlock) void prologue_tile_kernel(int64_t n, int nrhs, int ldx,
                                                               const int32_t *__restrict__ perm,
                                                               const double *__restrict__ w,
                                                               const double2 *__restrict__ m,
                                                               const double2 *__restrict__ x, int64_t ld,
                                                               int64_t off, typename Tile<T>::cplx_t *__restrict__ X,
                                                               double2 *__restrict__ f) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n * ldx) return;
  const int64_t i = t / ldx;
  const int b = (int)(t - i * ldx);
  if (b >= nrhs) {
    X[t] = Tile<T>::make(0.0, 0.0);
    return;
  }
  const double2 xv = x[(int64_t)b * ld + off + perm[i]];
  if (M == Mode::Forward) {
    const double2 mi = m[i];
    const double2 fv = make_double2(mi.x * xv.x - mi.y * xv.y, mi.x * xv.y + mi.y * xv.x);
    f[(int64_t)b * n + i] = fv;
    X[t] = Tile<T>::make(w[i] * fv.x, w[i] * fv.y);
  } else {
    f[(int64_t)b * n + i] = xv;
    X[t] = Tile<T>::make(xv.x, xv.y);
  }
}

// One wavefront's work: targets [t0, t0 + 16 MT), right-hand sides [b0, b0 + 16 NT), sources
// [s0, s1) of one split; writes that split's FP64 partial sums part[(split * nrhs + b) * n + t].
// RI (at most 8 right-hand sides, NT = 1): the 16 columns of the N-tile carry Re X of the eight
// right-hand sides in columns 0-7 and Im X in columns 8-15, so two real MFMAs per step, one with
// Re G and one with Im G, give all four real products of the complex tile without padding columns
// (Gauss's form needs three MFMAs on 16 columns, half of them zero).  Column b and b + 8 of the
// results are then combined across lanes l and l ^ 8.
template <class T, int MT, int NT, bool CONJ, bool RI>
__device__ __forceinline__ void tile_body_ri(int n, const double2 *__restrict__ pos,
                                             const typename Tile<T>::cplx_t *__restrict__ X, int ldx, int nrhs,
                                             double k2, int s0, int s1, int t0, int b0, int split,
                                             double2 *__restrict__ part, const PhaseLds &sct, bool excl) {
  static_assert(NT == 1 && RI, "the split-column form has one N-tile");
  typedef Tile<T> TL;
  typedef typename TL::acc_t acc_t;
  const int lane = threadIdx.x & 63;
  const int kk = lane >> 4, col = lane & 15;
  const int bcol = col & 7;
  const bool im_col = col >= 8;
  int tm[MT];
  double xt[MT], yt[MT];
#pragma unroll
  for (int mi = 0; mi < MT; ++mi) {
    tm[mi] = t0 + 16 * mi + col;
    const double2 p = pos[tm[mi] < n ? tm[mi] : n - 1];
    xt[mi] = p.x;
    yt[mi] = p.y;
  }
  // d0 = Re G X_col, d1 = Im G X_col with X_col = Re X (columns 0-7) or Im X (columns 8-15)
  acc_t d0[MT], d1[MT];
#pragma unroll
  for (int mi = 0; mi < MT; ++mi) {
    d0[mi] = acc_t{0, 0, 0, 0};
    d1[mi] = acc_t{0, 0, 0, 0};
  }
  for (int s = s0; s < s1; s += 4) {
    const int src = s + kk;
    const bool ok = src < s1;
    const int sc = ok ? src : s0;
    const double2 p = pos[sc];
    // only a step that meets the wave's targets (the diagonal pair, G undefined there) or runs past
    // the split's last source has pairs to zero (the same for the whole wave); a zero G also
    // cancels the clamped source's density, so X needs no mask
    const bool edge = (s < t0 + 16 * MT && t0 < s + 4) || s + 4 > s1;
    T gr[MT], gi[MT];
#pragma unroll
    for (int mi = 0; mi < MT; ++mi) {
      const double dx = xt[mi] - p.x, dy = yt[mi] - p.y;
      const double A = k2 * std::fma(dx, dx, dy * dy);
      TL::green(A, gr[mi], gi[mi], sct, excl);
      if (edge) {
        const bool zero = !ok || src == tm[mi];
        gr[mi] = zero ? (T)0 : gr[mi];
        gi[mi] = zero ? (T)0 : gi[mi];
      }
      if (CONJ) gi[mi] = -gi[mi];
    }
    const typename TL::cplx_t xb = X[(int64_t)sc * ldx + b0 + bcol];
    const T xv = im_col ? xb.y : xb.x;
#pragma unroll
    for (int mi = 0; mi < MT; ++mi) {
      d0[mi] = TL::mma(gr[mi], xv, d0[mi]);
      d1[mi] = TL::mma(gi[mi], xv, d1[mi]);
    }
  }
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // lane col < 8 holds Re G Re X and Im G Re X of column col, its partner col + 8 the products
      // with Im X: Re Y = Re G Re X - Im G Im X, Im Y = Re G Im X + Im G Re X
      const double a = (double)d0[mi][r], c = (double)d1[mi][r];
      const double pa = __shfl_xor(a, 8), pc = __shfl_xor(c, 8);
      const int t = t0 + 16 * mi + TL::row(lane, r);
      const int b = b0 + bcol;
      if (!im_col && t < n && b < nrhs) part[((int64_t)split * nrhs + b) * n + t] = make_double2(a - pc, pa + c);
    }
}

template <class T, int MT, int NT, bool CONJ>
__device__ __forceinline__ void tile_body(int n, const double2 *__restrict__ pos,
                                          const typename Tile<T>::cplx_t *__restrict__ X, int ldx, int nrhs,
                                          double k2, int s0, int s1, int t0, int b0, int split,
                                          double2 *__restrict__ part, const PhaseLds &sct, bool excl) {
  typedef Tile<T> TL;
  typedef typename TL::acc_t acc_t;
  const int lane = threadIdx.x & 63;
  const int kk = lane >> 4, col = lane & 15;
  int tm[MT];
  double xt[MT], yt[MT];
#pragma unroll
  for (int mi = 0; mi < MT; ++mi) {
    tm[mi] = t0 + 16 * mi + col;
    const double2 p = pos[tm[mi] < n ? tm[mi] : n - 1];
    xt[mi] = p.x;
    yt[mi] = p.y;
  }
  // three real products per complex tile (Gauss): P0 = Re G Re X, P1 = Im G Im X and
  // P2 = (Re G + Im G)(Re X + Im X); Re = P0 - P1 and Im = P2 - P0 - P1 are formed once, at the end
  acc_t p0[MT][NT], p1[MT][NT], p2[MT][NT];
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
#pragma unroll
    for (int ni = 0; ni < NT; ++ni) {
      p0[mi][ni] = acc_t{0, 0, 0, 0};
      p1[mi][ni] = acc_t{0, 0, 0, 0};
      p2[mi][ni] = acc_t{0, 0, 0, 0};
    }
  for (int s = s0; s < s1; s += 4) {
    const int src = s + kk;
    const bool ok = src < s1;
    const int sc = ok ? src : s0;
    const double2 p = pos[sc];
    // only a step that meets the wave's targets (the diagonal pair, G undefined there) or runs past
    // the split's last source has pairs to zero (the same for the whole wave); a zero G also
    // cancels the clamped source's density, so X needs no mask
    const bool edge = (s < t0 + 16 * MT && t0 < s + 4) || s + 4 > s1;
    T gr[MT], gi[MT], g2[MT];
#pragma unroll
    for (int mi = 0; mi < MT; ++mi) {
      const double dx = xt[mi] - p.x, dy = yt[mi] - p.y;
      const double A = k2 * std::fma(dx, dx, dy * dy);
      TL::green(A, gr[mi], gi[mi], sct, excl);
      if (edge) {
        const bool zero = !ok || src == tm[mi];
        gr[mi] = zero ? (T)0 : gr[mi];
        gi[mi] = zero ? (T)0 : gi[mi];
      }
      if (CONJ) gi[mi] = -gi[mi];
      g2[mi] = gr[mi] + gi[mi];
    }
    typename TL::cplx_t xb[NT];
    T x2[NT];
#pragma unroll
    for (int ni = 0; ni < NT; ++ni) {
      xb[ni] = X[(int64_t)sc * ldx + b0 + 16 * ni + col];
      x2[ni] = xb[ni].x + xb[ni].y;
    }
#pragma unroll
    for (int mi = 0; mi < MT; ++mi)
#pragma unroll
      for (int ni = 0; ni < NT; ++ni) {
        p0[mi][ni] = TL::mma(gr[mi], xb[ni].x, p0[mi][ni]);
        p1[mi][ni] = TL::mma(gi[mi], xb[ni].y, p1[mi][ni]);
        p2[mi][ni] = TL::mma(g2[mi], x2[ni], p2[mi][ni]);
      }
  }
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
#pragma unroll
    for (int ni = 0; ni < NT; ++ni)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int t = t0 + 16 * mi + TL::row(lane, r);
        const int b = b0 + 16 * ni + col;
        if (t < n && b < nrhs) {
          const double a = (double)p0[mi][ni][r], c = (double)p1[mi][ni][r];
          part[((int64_t)split * nrhs + b) * n + t] = make_double2(a - c, (double)p2[mi][ni][r] - a - c);
        }
      }
}

// grid: (ceil(n / (4 * 16 * MT)), source splits, ldx / (16 * NT))
template <class T, int MT, int NT, bool CONJ, bool RI = false>
__global__ __launch_bounds__(kBlock) void far_tile_kernel(int n, const double2 *__restrict__ pos,
                                                          const typename Tile<T>::cplx_t *__restrict__ X, int ldx,
                                                          int nrhs, double k2, int split_len,
                                                          double2 *__restrict__ part, int excl) {
  // the FP64 Green's values take e^{i theta} from a table in LDS (hankel.h, phase_tail_table)
  __shared__ double2 sct_lds[kFP64<T> ? SINCOS_N : 1];
  PhaseLds sct{sct_lds, 0.0};
  if constexpr (kFP64<T>) sct = load_sincos(sct_lds, m_sincos);
  const int wave = threadIdx.x >> 6;
  const int s0 = blockIdx.y * split_len;
  if constexpr (RI)
    tile_body_ri<T, MT, NT, CONJ, RI>(n, pos, X, ldx, nrhs, k2, s0, min(n, s0 + split_len),
                                      (blockIdx.x * 4 + wave) * 16 * MT, blockIdx.z * 16 * NT, blockIdx.y, part, sct,
                                      excl != 0);
  else
    tile_body<T, MT, NT, CONJ>(n, pos, X, ldx, nrhs, k2, s0, min(n, s0 + split_len),
                               (blockIdx.x * 4 + wave) * 16 * MT, blockIdx.z * 16 * NT, blockIdx.y, part, sct,
                               excl != 0);
}

// Uneven batch of scatterers in one launch: each workgroup repeatedly takes the next work item
// (scatterer, block of 64 MT targets, source split, RHS group) from a global counter until the
// list, ordered longest first, is exhausted.  Every item writes its own partials, so the result
// does not depend on which workgroup took it.
template <class T, int MT, int NT, bool CONJ, bool RI = false>
__global__ __launch_bounds__(kBlock) void far_tile_persistent(const BatchDesc *__restrict__ desc,
                                                              const WorkItem *__restrict__ items, int n_items,
                                                              int *__restrict__ counter, int ldx, int nrhs) {
  __shared__ int next;
  __shared__ double2 sct_lds[kFP64<T> ? SINCOS_N : 1];
  PhaseLds sct{sct_lds, 0.0};
  if constexpr (kFP64<T>) sct = load_sincos(sct_lds, m_sincos);
  const int wave = threadIdx.x >> 6;
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int it = next;
    __syncthreads();
    if (it >= n_items) break;
    const WorkItem wi = items[it];
    const BatchDesc d = desc[wi.s];
    const int s0 = wi.split * d.split_len;
    if constexpr (RI)
      tile_body_ri<T, MT, NT, CONJ, RI>(d.n, d.pos, (const typename Tile<T>::cplx_t *)d.X, ldx, nrhs, d.k2, s0,
                                        min(d.n, s0 + d.split_len), (wi.tblock * 4 + wave) * 16 * MT,
                                        wi.bgroup * 16 * NT, wi.split, d.part, sct, d.excl != 0);
    else
      tile_body<T, MT, NT, CONJ>(d.n, d.pos, (const typename Tile<T>::cplx_t *)d.X, ldx, nrhs, d.k2, s0,
                                 min(d.n, s0 + d.split_len), (wi.tblock * 4 + wave) * 16 * MT, wi.bgroup * 16 * NT,
                                 wi.split, d.part, sct, d.excl != 0);
  }
}

template <class T, int MT, int NT, bool RI = false>
void launch_tile(const Scat &s, const void *X, int ldx, int nrhs, int split_len, int nsplit, double2 *part,
                 bool conj, hipStream_t st) {
  dim3 grid((unsigned)((s.n + 64 * MT - 1) / (64 * MT)), (unsigned)nsplit, (unsigned)(ldx / (16 * NT)));
  typedef typename Tile<T>::cplx_t C;
  // the FP32 tiles leave the pairs with z < 1 to the FP64 near part of the mixed correction
  const int excl = (!kFP64<T> && s.near_ok) ? 1 : 0;
  if (conj)
    far_tile_kernel<T, MT, NT, true, RI><<<grid, kBlock, 0, st>>>((int)s.n, s.pos, (const C *)X, ldx, nrhs,
                                                                 s.k * s.k, split_len, part, excl);
  else
    far_tile_kernel<T, MT, NT, false, RI><<<grid, kBlock, 0, st>>>((int)s.n, s.pos, (const C *)X, ldx, nrhs,
                                                                  s.k * s.k, split_len, part, excl);
}

// The pairs with z < 1 of a mixed-precision application, in FP64 (the mixed tiles leave them out):
// one wave per tile of 16 targets, over the tile's source intervals, keeping the pairs whose A =
// k^2 r^2 falls below 1 (the same test on the same positions as the tiles' exclusion).  G/K is the
// FP64 tiles' own evaluation and the densities come from f (w f forward, f adjoint); the result,
// one split of partial sums in G/K units, goes to part[b * n + t] for the epilogue.
// grid: (ceil(ntiles / 4), ldx / (16 NT))
template <int NT, bool CONJ>
__global__ __launch_bounds__(kBlock) void near_tile_kernel(int n, int ntiles, const double2 *__restrict__ pos,
                                                           const double *__restrict__ w,
                                                           const double2 *__restrict__ f, int nrhs, double k2,
                                                           const int32_t *__restrict__ tile_rp,
                                                           const int2 *__restrict__ iv, double2 *__restrict__ part) {
  __shared__ double2 sct_lds[SINCOS_N];
  const PhaseLds sct = load_sincos(sct_lds, m_sincos);
  const int lane = threadIdx.x & 63, kk = lane >> 4, col = lane & 15;
  const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntiles) return;
  const int t0 = tile * 16, tm = t0 + col;
  const int b0 = blockIdx.y * 16 * NT;
  const double2 pt = pos[tm < n ? tm : n - 1];
  v4d p0[NT], p1[NT], p2[NT];
#pragma unroll
  for (int ni = 0; ni < NT; ++ni) {
    p0[ni] = v4d{0, 0, 0, 0};
    p1[ni] = v4d{0, 0, 0, 0};
    p2[ni] = v4d{0, 0, 0, 0};
  }
  for (int q = tile_rp[tile]; q < tile_rp[tile + 1]; ++q) {
    const int2 r = iv[q];
    for (int s = r.x; s < r.y; s += 4) {
      const int src = s + kk;
      const bool ok = src < r.y;
      const int sc = ok ? src : r.x;
      const double2 p = pos[sc];
      const double dx = pt.x - p.x, dy = pt.y - p.y;
      const double A = k2 * std::fma(dx, dx, dy * dy);
      double gr = 0.0, gi = 0.0;
      if (ok && A < 1.0 && src != tm) lsk::green_unit<true>(A, gr, gi, mtab(), sct);
      if (CONJ) gi = -gi;
      const double g2 = gr + gi;
      const double ws = CONJ ? 1.0 : w[sc];
#pragma unroll
      for (int ni = 0; ni < NT; ++ni) {
        const int b = b0 + 16 * ni + col;
        double2 xv = make_double2(0.0, 0.0);
        if (ok && b < nrhs) xv = f[(int64_t)b * n + sc];
        const double xr = ws * xv.x, xi = ws * xv.y;
        p0[ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(gr, xr, p0[ni], 0, 0, 0);
        p1[ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(gi, xi, p1[ni], 0, 0, 0);
        p2[ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(g2, xr + xi, p2[ni], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int ni = 0; ni < NT; ++ni)
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int t = t0 + kk + 4 * rr;
      const int b = b0 + 16 * ni + col;
      if (t < n && b < nrhs) {
        const double a = p0[ni][rr], c = p1[ni][rr];
        part[(int64_t)b * n + t] = make_double2(a - c, p2[ni][rr] - a - c);
      }
    }
}

template <class T, int MT>
void launch_tile_nt(const Scat &s, const void *X, int ldx, int nrhs, int split_len, int nsplit, double2 *part,
                    bool conj, hipStream_t st) {
  const int groups = ldx / 16;
  if (nrhs <= 8)
    launch_tile<T, MT, 1, true>(s, X, ldx, nrhs, split_len, nsplit, part, conj, st);
  else if (groups % 4 == 0)
    launch_tile<T, MT, 4>(s, X, ldx, nrhs, split_len, nsplit, part, conj, st);
  else if (groups % 2 == 0)
    launch_tile<T, MT, 2>(s, X, ldx, nrhs, split_len, nsplit, part, conj, st);
  else
    launch_tile<T, MT, 1>(s, X, ldx, nrhs, split_len, nsplit, part, conj, st);
}

__global__ void zero_counter_kernel(int *c) { *c = 0; }

template <class T, int MT, int NT, bool RI = false>
void launch_persistent(const BatchDesc *desc, const WorkItem *items, int n_items, int *counter, int ldx, int nrhs,
                       bool conj, hipStream_t st) {
  // one full round of resident workgroups; each keeps taking items until none are left
  int dev = 0, cus = 256, per_cu = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (conj)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, far_tile_persistent<T, MT, NT, true>, kBlock, 0);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, far_tile_persistent<T, MT, NT, false>, kBlock, 0);
  const int grid = std::max(1, std::min(n_items, cus * std::max(per_cu, 1)));
  zero_counter_kernel<<<1, 1, 0, st>>>(counter);
  if (conj)
    far_tile_persistent<T, MT, NT, true, RI><<<grid, kBlock, 0, st>>>(desc, items, n_items, counter, ldx, nrhs);
  else
    far_tile_persistent<T, MT, NT, false, RI><<<grid, kBlock, 0, st>>>(desc, items, n_items, counter, ldx, nrhs);
}

template <class T, int MT>
void launch_persistent_nt(const BatchDesc *desc, const WorkItem *items, int n_items, int *counter, int ldx, int nrhs,
                          bool conj, hipStream_t st) {
  const int groups = ldx / 16;
  if (nrhs <= 8)
    launch_persistent<T, MT, 1, true>(desc, items, n_items, counter, ldx, nrhs, conj, st);
  else if (groups % 4 == 0)
    launch_persistent<T, MT, 4>(desc, items, n_items, counter, ldx, nrhs, conj, st);
  else if (groups % 2 == 0)
    launch_persistent<T, MT, 2>(desc, items, n_items, counter, ldx, nrhs, conj, st);
  else
    launch_persistent<T, MT, 1>(desc, items, n_items, counter, ldx, nrhs, conj, st);
}

int nt_of(int ldx) { return (ldx / 16) % 4 == 0 ? 4 : ((ldx / 16) % 2 == 0 ? 2 : 1); }

// the FP64 near launch of a mixed-precision application into the partial-sum slot `slot`
// ([nrhs][n]); nothing when the scatterer has no near lists
hipError_t launch_near(const Scat &s, const double2 *f, int nrhs, bool conj, double2 *slot, hipStream_t st) {
  if (!s.near_ok) return hipSuccess;
  const int ldx = tile_ldx(nrhs), nt = nt_of(ldx);
  const dim3 grid((unsigned)((s.near_ntiles + 3) / 4), (unsigned)(ldx / (16 * nt)));
  const int n = (int)s.n;
  const double k2 = s.k * s.k;
#define LSK_NEAR(NT, CJ)                                                                                          \
  near_tile_kernel<NT, CJ><<<grid, kBlock, 0, st>>>(n, s.near_ntiles, s.pos, s.w, f, nrhs, k2, s.near_rp, s.near_iv, \
                                                    slot)
  if (nt == 4) {
    if (conj) LSK_NEAR(4, true); else LSK_NEAR(4, false);
  } else if (nt == 2) {
    if (conj) LSK_NEAR(2, true); else LSK_NEAR(2, false);
  } else {
    if (conj) LSK_NEAR(1, true); else LSK_NEAR(1, false);
  }
#undef LSK_NEAR
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------------
// Split-FP16 tiles (mixed precision on the FP16 matrix cores).  Each real operand v is carried as
// v_hi + v_lo, two FP16 numbers (v_hi = fp16(v), v_lo = fp16(v - v_hi): about 22 significant bits),
// and a real product as A_hi B_hi + A_hi B_lo + A_lo B_hi, three v_mfma_f32_16x16x32_f16 with FP32
// accumulation (the dropped A_lo B_lo is below 2^-22 of the product).  A complex tile takes the four
// real products, accumulated straight into Re (Re G Re X - Im G Im X, the second with the FP16 sign
// bits of Im G flipped) and Im (Re G Im X + Im G Re X): twelve MFMAs per (M-tile, N-tile) and 32
// sources.  Gauss's three products need nine, but also a third accumulator, the split of Re G + Im G
// and two more density planes; at 64 columns the four-product form holds the wave in 162 VGPRs (three
// waves per SIMD instead of two) and the launch at N = 122 500 took 29.1 ms against 33.0.  FP16's range
// needs scales: the Green's values enter as 256 G (|G| < 0.8), the densities of right-hand side b
// as s_b 2^(13 - e_b) with 2^e_b <= max |Re s_b|, |Im s_b| < 2^(e_b + 1), so every hi part is far
// inside FP16's range and a lo part is normal for values above 2^-9 of the column's largest.  The
// partial sums are brought back to G/K units in FP64 per column (colinv).
//   Layout of the split densities: four planes (Re hi, Re lo, Im hi, Im lo), each
//   [source / 8][ldx][8] halves, sources padded with zeros to a multiple of 32: the eight
//   sources of one lane's MFMA operand are one 16-byte load.
//   Operand layout of the 16x16x32 MFMA: lane l supplies row l % 16 of A and column l % 16 of B at
//   eight contraction indices that depend on l / 16 only (the same eight for A and B), here the
//   sources s + 8 (l / 16) + j, j < 8.  Results are D[4 (l / 16) + r][l % 16], as for the FP32 tiles.
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
constexpr int kHPlanes = 4;

__host__ __device__ inline int64_t h_npad(int64_t n) { return (n + 31) / 32 * 32; }

__device__ __forceinline__ double2 density(int64_t i, int b, const int32_t *__restrict__ perm,
                                           const double *__restrict__ w, const double2 *__restrict__ m,
                                           const double2 *__restrict__ x, int64_t ld, int64_t off, bool fwd,
                                           double2 *fv) {
  const double2 xv = x[(int64_t)b * ld + off + perm[i]];
  if (!fwd) {
    *fv = xv;
    return xv;
  }
  const double2 mi = m[i];
  *fv = make_double2(mi.x * xv.x - mi.y * xv.y, mi.x * xv.y + mi.y * xv.x);
  return make_double2(w[i] * fv->x, w[i] * fv->y);
}

__global__ void zero_u32_kernel(unsigned *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// cmax[b] = max over the nodes of max(|Re s_b|, |Im s_b|) as the bits of a non-negative float
// (rounded up, so that the scale below never overflows); grid (ceil(n / kBlock), nrhs)
__global__ __launch_bounds__(kBlock) void colmax_kernel(int64_t n, const int32_t *__restrict__ perm,
                                                        const double *__restrict__ w, const double2 *__restrict__ m,
                                                        const double2 *__restrict__ x, int64_t ld, int64_t off,
                                                        int fwd, unsigned *__restrict__ cmax) {
  __shared__ float red[kBlock / 64];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int b = blockIdx.y;
  float v = 0.f;
  if (i < n) {
    double2 fv;
    const double2 sv = density(i, b, perm, w, m, x, ld, off, fwd != 0, &fv);
    const double a = fmax(fabs(sv.x), fabs(sv.y));
    v = __double2float_ru(a);
  }
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    float r = red[0];
    for (int k = 1; k < kBlock / 64; ++k) r = fmaxf(r, red[k]);
    atomicMax(cmax + b, __float_as_uint(r));
  }
}

__device__ __forceinline__ void split16(double v, _Float16 &hi, _Float16 &lo) {
  hi = (_Float16)(float)v;
  lo = (_Float16)(float)(v - (double)(float)hi);
}

// the same for an FP32 value: v - hi is exact in FP32 (hi is v rounded to 11 bits)
__device__ __forceinline__ void split16f(float v, _Float16 &hi, _Float16 &lo) {
  hi = (_Float16)v;
  lo = (_Float16)(v - (float)hi);
}

// the split densities (planes Xh), the FP64 f[b][i] for the sparse correction, and colinv[b] =
// 1 / (256 K cs_b) with cs_b the column's scale; grid over npad * ldx
__global__ __launch_bounds__(kBlock) void prologue_h_kernel(int64_t n, int nrhs, int ldx,
                                                            const int32_t *__restrict__ perm,
                                                            const double *__restrict__ w,
                                                            const double2 *__restrict__ m,
                                                            const double2 *__restrict__ x, int64_t ld, int64_t off,
                                                            int fwd, const unsigned *__restrict__ cmax,
                                                            _Float16 *__restrict__ Xh, double2 *__restrict__ f,
                                                            double *__restrict__ colinv) {
  const int64_t npad = h_npad(n);
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= npad * ldx) return;
  const int64_t i = t / ldx;
  const int b = (int)(t - i * ldx);
  const size_t plane = (size_t)npad * ldx;
  const size_t idx = ((size_t)(i >> 3) * ldx + b) * 8 + (i & 7);
  double sr = 0.0, si = 0.0, cs = 1.0;
  if (b < nrhs) {
    const float mx = __uint_as_float(cmax[b]);
    cs = mx > 0.f ? ldexp(1.0, 13 - ilogbf(mx)) : 1.0;
    if (i == 0) colinv[b] = 1.0 / (cs * 256.0 * G_SCALE);
    if (i < n) {
      double2 fv;
      const double2 sv = density(i, b, perm, w, m, x, ld, off, fwd != 0, &fv);
      f[(int64_t)b * n + i] = fv;
      sr = sv.x * cs;
      si = sv.y * cs;
    }
  }
  _Float16 h, l;
  split16(sr, h, l);
  Xh[idx] = h;
  Xh[plane + idx] = l;
  split16(si, h, l);
  Xh[2 * plane + idx] = h;
  Xh[3 * plane + idx] = l;
}

__device__ __forceinline__ v4f mma16(v8h a, v8h b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
union H8 {
  v8h v;
  h2 p[4];
};

// hi and lo parts of two FP32 values: hi by one packed conversion, each lo = v - hi by one
// mixed-precision FMA that reads hi as FP16 and rounds the (exact) FP32 difference to FP16 into
// its half of the register.  Two instructions fewer per value than converting hi back and
// subtracting; the result is the same.
__device__ __forceinline__ void split16x2(f2 v, h2 &hi, h2 &lo) {
  hi = __builtin_convertvector(v, h2);
  unsigned h, l;
  __builtin_memcpy(&h, &hi, 4);
  asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel:[0,0,0] op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixhi_f16 %0, %1, -1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
      : "=&v"(l)
      : "v"(h), "v"(v.x), "v"(v.y));
  __builtin_memcpy(&lo, &l, 4);
}

constexpr int kHChunk = kBlock;   // source positions staged in LDS per pass of a block

// grid: (ceil(n / (4 * 16 * MT)), source splits, ldx / (16 * NT)); split_len a multiple of 32.
// The four waves of a block take different targets and the same sources, whose positions pass
// through LDS kHChunk at a time.
template <int MT, int NT, bool CONJ>
__global__ __launch_bounds__(kBlock) void far_tile_h_kernel(int n, const double2 *__restrict__ pos,
                                                            const _Float16 *__restrict__ Xh, int ldx, int nrhs,
                                                            double k2, int split_len, float2 *__restrict__ part,
                                                            int excl) {
  __shared__ double2 spos[kHChunk];
  const int lane = threadIdx.x & 63;
  const int kq = lane >> 4, col = lane & 15;
  const int t0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16 * MT;
  const int b0 = blockIdx.z * 16 * NT;
  const int s0 = blockIdx.y * split_len;
  const int s1 = min(n, s0 + split_len);
  const size_t plane = (size_t)h_npad(n) * ldx;
  int tm[MT];
  double xt[MT], yt[MT];
#pragma unroll
  for (int mi = 0; mi < MT; ++mi) {
    tm[mi] = t0 + 16 * mi + col;
    const double2 p = pos[tm[mi] < n ? tm[mi] : n - 1];
    xt[mi] = p.x;
    yt[mi] = p.y;
  }
  v4f re[MT][NT], im[MT][NT];   // Re and Im of the 16 x 16 result tiles
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
#pragma unroll
    for (int ni = 0; ni < NT; ++ni) {
      re[mi][ni] = v4f{0, 0, 0, 0};
      im[mi][ni] = v4f{0, 0, 0, 0};
    }
  for (int c0 = s0; c0 < s1; c0 += kHChunk) {
    __syncthreads();   // every wave is done with the previous chunk
    {
      const int src = c0 + (int)threadIdx.x;
      spos[threadIdx.x] = pos[src < n ? src : n - 1];
    }
    __syncthreads();
    const int c1 = min(s1, c0 + kHChunk);
    for (int s = c0; s < c1; s += 32) {
      // 256 G for this lane's eight sources s + 8 kq + j and each of its M-tiles
      float gr[MT][8], gi[MT][8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double2 p = spos[s - c0 + 8 * kq + j];
#pragma unroll
        for (int mi = 0; mi < MT; ++mi) {
          const double dx = xt[mi] - p.x, dy = yt[mi] - p.y;
          lsk::green32_unit<true>(k2 * std::fma(dx, dx, dy * dy), gr[mi][j], gi[mi][j], mtab(), excl != 0);
          if (CONJ) gi[mi][j] = -gi[mi][j];
        }
      }
      // the wave's targets t0 .. t0 + 16 MT - 1 meet these sources (the diagonal pair, G undefined
      // there) or the step runs past the split's last source: zero those pairs
      if ((s < t0 + 16 * MT && t0 < s + 32) || s + 32 > c1) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int src = s + 8 * kq + j;
#pragma unroll
          for (int mi = 0; mi < MT; ++mi)
            if (src >= c1 || src == tm[mi]) {
              gr[mi][j] = 0.f;
              gi[mi][j] = 0.f;
            }
        }
      }
      H8 ar_h[MT], ar_l[MT], ai_h[MT], ai_l[MT], an_h[MT], an_l[MT];
#pragma unroll
      for (int mi = 0; mi < MT; ++mi)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const f2 vr = {gr[mi][2 * q], gr[mi][2 * q + 1]}, vi = {gi[mi][2 * q], gi[mi][2 * q + 1]};
          split16x2(vr, ar_h[mi].p[q], ar_l[mi].p[q]);
          split16x2(vi, ai_h[mi].p[q], ai_l[mi].p[q]);
          // -Im G for the real part: the sign bits of both halves flipped
          unsigned u, w;
          __builtin_memcpy(&u, &ai_h[mi].p[q], 4);
          __builtin_memcpy(&w, &ai_l[mi].p[q], 4);
          u ^= 0x80008000u;
          w ^= 0x80008000u;
          __builtin_memcpy(&an_h[mi].p[q], &u, 4);
          __builtin_memcpy(&an_l[mi].p[q], &w, 4);
        }
#pragma unroll
      for (int ni = 0; ni < NT; ++ni) {
        const size_t bi = ((size_t)(s / 8 + kq) * ldx + b0 + 16 * ni + col) * 8;
        const v8h br_h = *(const v8h *)(Xh + bi), br_l = *(const v8h *)(Xh + plane + bi);
        const v8h bi_h = *(const v8h *)(Xh + 2 * plane + bi), bi_l = *(const v8h *)(Xh + 3 * plane + bi);
#pragma unroll
        for (int mi = 0; mi < MT; ++mi) {
          re[mi][ni] = mma16(ar_h[mi].v, br_h, re[mi][ni]);
          re[mi][ni] = mma16(ar_h[mi].v, br_l, re[mi][ni]);
          re[mi][ni] = mma16(ar_l[mi].v, br_h, re[mi][ni]);
          re[mi][ni] = mma16(an_h[mi].v, bi_h, re[mi][ni]);
          re[mi][ni] = mma16(an_h[mi].v, bi_l, re[mi][ni]);
          re[mi][ni] = mma16(an_l[mi].v, bi_h, re[mi][ni]);
          im[mi][ni] = mma16(ar_h[mi].v, bi_h, im[mi][ni]);
          im[mi][ni] = mma16(ar_h[mi].v, bi_l, im[mi][ni]);
          im[mi][ni] = mma16(ar_l[mi].v, bi_h, im[mi][ni]);
          im[mi][ni] = mma16(ai_h[mi].v, br_h, im[mi][ni]);
          im[mi][ni] = mma16(ai_h[mi].v, br_l, im[mi][ni]);
          im[mi][ni] = mma16(ai_l[mi].v, br_h, im[mi][ni]);
        }
      }
    }
  }
  // the FP32 sums as they are: the epilogue applies the column scale in FP64
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
#pragma unroll
    for (int ni = 0; ni < NT; ++ni) {
      const int b = b0 + 16 * ni + col;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int t = t0 + 16 * mi + 4 * kq + r;
        if (t < n && b < nrhs) part[((int64_t)blockIdx.y * nrhs + b) * n + t] = make_float2(re[mi][ni][r], im[mi][ni][r]);
      }
    }
}

}  // namespace

int tile_ldx(int nrhs) { return (nrhs + 15) / 16 * 16; }

// 16-target M-tiles per wavefront.  FP32: two.  FP64: one, or two when a single 16-column N-tile
// covers the right-hand sides (B <= 16), where the wave otherwise has too little independent work
// per Green's evaluation.  Measured at N = 122 500 (disk) and N = 114 660 (two-material), k = 40:
// FP32 MT 4 -> 2 at B = 64, 77.4 -> 75.1 ms; FP64 at B = 64, MT 2 -> 1, 159.0 -> 150.3 ms; FP64 at
// B = 16, MT 1 -> 2, 54.6 -> 52.4 ms; sixteen scatterers at B = 8, 93.9 -> 90.1 ms.  Loading the
// next step's source ahead cost occupancy and was slower.
int tile_mt(int nrhs, bool single) {
  if (single) return 2;
  return (tile_ldx(nrhs) / 16) % 2 == 0 ? 1 : 2;
}

int batch_default_split_len(const ls_ctx *h, bool single) {
  (void)h;
  return 2048;   // FP32: bounds the accumulation error, as in tile_source_split
}

// per-scatterer layout of the batch workspace: X_s, f_s, part_s, each 256-byte aligned
static size_t batch_layout(const ls_ctx *h, int nrhs, bool single, int split_len, std::vector<size_t> *offs) {
  const int ldx = tile_ldx(nrhs);
  size_t o = 0;
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  for (const Scat &sc : h->sc) {
    // the mixed tiles' splits and, with near lists, the FP64 near launch's one
    const int64_t nsplit = (sc.n + split_len - 1) / split_len + ((single && sc.near_ok) ? 1 : 0);
    if (offs) offs->push_back(o);
    o = al(o + (single ? sizeof(float2) : sizeof(double2)) * (size_t)sc.n * ldx);
    if (offs) offs->push_back(o);
    o = al(o + sizeof(double2) * (size_t)sc.n * nrhs);
    if (offs) offs->push_back(o);
    o = al(o + sizeof(double2) * (size_t)sc.n * nrhs * nsplit);
  }
  return o + 256;
}

size_t batch_workspace_bytes(const ls_ctx *h, int nrhs, bool single, int split_len) {
  return batch_layout(h, nrhs, single, split_len, nullptr);
}

// bytes of the descriptor and work-item tables of the persistent launch when no scatterer is left out
static size_t batch_table_bytes(const ls_ctx *h, int nrhs, int mt, int split_len) {
  const int ldx = tile_ldx(nrhs);
  const int nt = nt_of(ldx);
  size_t items = 0;
  for (const Scat &sc : h->sc) {
    const int64_t nsplit = (sc.n + split_len - 1) / split_len;
    const int64_t tblocks = (sc.n + 64 * mt - 1) / (64 * mt);
    items += (size_t)(tblocks * nsplit * (ldx / (16 * nt)));
  }
  return sizeof(BatchDesc) * h->sc.size() + sizeof(WorkItem) * items + 512;
}

hipError_t reserve_batch_tables(ls_ctx *h, int nrhs, bool single, int mt, int split_len) {
  (void)single;
  const size_t tb = batch_table_bytes(h, nrhs, mt, split_len);
  if (tb <= h->batch_bytes) return hipSuccess;
  hipError_t e = hipDeviceSynchronize();   // an earlier launch may still read the old tables
  if (e != hipSuccess) return e;
  if (h->batch_tables) (void)hipFree(h->batch_tables);
  h->batch_tables = nullptr;
  h->batch_bytes = 0;
  e = lsk::dmalloc(&h->batch_tables, tb);
  if (e != hipSuccess) return e;
  h->batch_bytes = tb;
  h->batch_key = -1;
  return hipSuccess;
}

hipError_t launch_apply_batch(ls_ctx *h, const double *x, double *y, int nrhs, int64_t ld, Mode mode, bool single,
                              int mt, int split_len, void *ws, hipStream_t st, hipEvent_t far_start,
                              hipEvent_t far_stop, bool far_only, bool may_alloc) {
  const int ldx = tile_ldx(nrhs);
  const int nt = nt_of(ldx);
  const int ns = (int)h->sc.size();
  std::vector<size_t> offs;
  batch_layout(h, nrhs, single, split_len, &offs);
  char *base = (char *)ws;
  // descriptor and work-item tables, cached for this (layout, shape, skipped scatterers)
  // combination; skipped scatterers get no work items, prologue or epilogue
  const bool masked = !h->scat_skip.empty();
  auto skip = [&](int i) { return masked && h->scat_skip[i]; };
  long long mask_hash = 0;
  for (int i = 0; i < ns && masked; ++i) mask_hash = mask_hash * 1000003LL + (h->scat_skip[i] ? 7 : 3);
  const long long key = (((((long long)nrhs * 2 + single) * 8 + mt) << 24) ^ (long long)split_len ^
                         ((long long)(uintptr_t)ws << 1)) ^ (mask_hash * 0x9E3779B97F4A7C15LL);
  std::vector<BatchDesc> desc(ns);
  std::vector<WorkItem> items;
  for (int i = 0; i < ns; ++i) {
    const Scat &sc = h->sc[i];
    const int nsplit = (int)((sc.n + split_len - 1) / split_len);
    desc[i] = BatchDesc{(int)sc.n, split_len, (single && sc.near_ok) ? 1 : 0, sc.k * sc.k, sc.pos, base + offs[3 * i],
                        (double2 *)(base + offs[3 * i + 2])};
    if (skip(i)) continue;
    const int tblocks = (int)((sc.n + 64 * mt - 1) / (64 * mt));
    for (int tb = 0; tb < tblocks; ++tb)
      for (int sp = 0; sp < nsplit; ++sp)
        for (int g = 0; g < ldx / (16 * nt); ++g) items.push_back(WorkItem{i, tb, sp, g});
  }
  auto cost = [&](const WorkItem &w) {
    const int64_t n = h->sc[w.s].n;
    const int64_t t = std::min<int64_t>(64 * mt, n - (int64_t)w.tblock * 64 * mt);
    const int64_t src = std::min<int64_t>(split_len, n - (int64_t)w.split * split_len);
    return t * src;
  };
  std::stable_sort(items.begin(), items.end(), [&](const WorkItem &a, const WorkItem &b) { return cost(a) > cost(b); });
  const size_t tb = sizeof(BatchDesc) * ns + sizeof(WorkItem) * items.size() + 512;
  hipError_t e = hipSuccess;
  if (tb > h->batch_bytes) {
    if (!may_alloc) return hipErrorOutOfMemory;
    if (h->batch_tables) (void)hipFree(h->batch_tables);
    h->batch_tables = nullptr;
    h->batch_bytes = 0;
    e = lsk::dmalloc(&h->batch_tables, tb);
    if (e != hipSuccess) return e;
    h->batch_bytes = tb;
    h->batch_key = -1;
  }
  BatchDesc *ddesc = (BatchDesc *)h->batch_tables;
  WorkItem *ditems = (WorkItem *)(ddesc + ns);
  int *counter = (int *)(((uintptr_t)(ditems + items.size()) + 255) & ~(uintptr_t)255);
  if (h->batch_key != key) {
    e = hipMemcpyAsync(ddesc, desc.data(), sizeof(BatchDesc) * ns, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ditems, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);   // host vectors go out of scope
    if (e != hipSuccess) return e;
    h->batch_key = key;
  }
  const bool fwd = mode == Mode::Forward;
  const double2 *xc = (const double2 *)x;
  if (!far_only)
    for (int i = 0; i < ns; ++i) {
      if (skip(i)) continue;
      const Scat &sc = h->sc[i];
      const unsigned gp = (unsigned)((sc.n * ldx + kBlock - 1) / kBlock);
      double2 *f = (double2 *)(base + offs[3 * i + 1]);
      if (single) {
        if (fwd)
          prologue_tile_kernel<float, Mode::Forward><<<gp, kBlock, 0, st>>>(sc.n, nrhs, ldx, sc.perm, sc.w, sc.m, xc, ld,
                                                                            sc.off, (float2 *)desc[i].X, f);
        else
          prologue_tile_kernel<float, Mode::Adjoint><<<gp, kBlock, 0, st>>>(sc.n, nrhs, ldx, sc.perm, sc.w, sc.m, xc, ld,
                                                                            sc.off, (float2 *)desc[i].X, f);
      } else {
        if (fwd)
          prologue_tile_kernel<double, Mode::Forward><<<gp, kBlock, 0, st>>>(sc.n, nrhs, ldx, sc.perm, sc.w, sc.m, xc,
                                                                             ld, sc.off, (double2 *)desc[i].X, f);
        else
          prologue_tile_kernel<double, Mode::Adjoint><<<gp, kBlock, 0, st>>>(sc.n, nrhs, ldx, sc.perm, sc.w, sc.m, xc,
                                                                             ld, sc.off, (double2 *)desc[i].X, f);
      }
    }
  if (far_start) (void)hipEventRecord(far_start, st);
  const int n_items = (int)items.size();
  if (single) {
    if (mt == 2)
      launch_persistent_nt<float, 2>(ddesc, ditems, n_items, counter, ldx, nrhs, !fwd, st);
    else
      launch_persistent_nt<float, 4>(ddesc, ditems, n_items, counter, ldx, nrhs, !fwd, st);
  } else {
    if (mt == 1)
      launch_persistent_nt<double, 1>(ddesc, ditems, n_items, counter, ldx, nrhs, !fwd, st);
    else
      launch_persistent_nt<double, 2>(ddesc, ditems, n_items, counter, ldx, nrhs, !fwd, st);
  }
  if (far_stop) (void)hipEventRecord(far_stop, st);
  e = hipGetLastError();
  if (e != hipSuccess || far_only) return e;
  for (int i = 0; i < ns; ++i) {
    if (skip(i)) continue;
    const Scat &sc = h->sc[i];
    int nsplit = (int)((sc.n + split_len - 1) / split_len);
    const double2 *f = (const double2 *)(base + offs[3 * i + 1]);
    if (single && sc.near_ok) {
      e = launch_near(sc, f, nrhs, !fwd, desc[i].part + (size_t)nsplit * nrhs * sc.n, st);
      if (e != hipSuccess) return e;
      ++nsplit;
    }
    e = launch_epilogue(sc, desc[i].part, nsplit, f, x, y, nrhs, ld, mode, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

size_t tile_workspace_bytes(int64_t n, int nrhs, int nsplit) {
  // X [n][ldx] (double2 upper bound), f [nrhs][n], part [nsplit][nrhs][n]
  return sizeof(double2) * ((size_t)n * tile_ldx(nrhs) + (size_t)n * nrhs * (1 + (size_t)nsplit)) + 512;
}

int tile_source_split(int64_t n, int nrhs, bool single) {
  const int mt = tile_mt(nrhs, single);
  const int ldx = tile_ldx(nrhs);
  const int nt = (ldx / 16) % 4 == 0 ? 4 : ((ldx / 16) % 2 == 0 ? 2 : 1);
  const int64_t waves = ((n + 16 * mt - 1) / (16 * mt)) * (ldx / (16 * nt));
  int64_t s = (32768 + waves - 1) / waves;   // ~32 waves per SIMD over the launch
  int64_t cap = ((int64_t)1 << 30) / ((int64_t)16 * n * nrhs);   // FP64 partials <= 1 GiB
  if (single) {
    // The FP32 accumulation error grows with the number of sources one split sums, so aim at
    // about 2 048 per split, with up to 4 GiB of partials counted at 16 B per value (the FP32 tiles'
    // FP64 partials; the split-FP16 tiles store 8 B, half that).  At N = 122 500, B = 64 going from 9 to
    // 32 splits took the operator's relative error from 1.9e-6 to 6.7e-7 (2-norm; 5.9e-6 to 2.1e-6
    // entrywise) at the same launch time; 64 splits gave 4.1e-7.
    s = std::max<int64_t>(s, (n + 2047) / 2048);
    cap = ((int64_t)1 << 32) / ((int64_t)16 * n * nrhs);
  }
  if (s > cap) s = cap;
  if (s < 1) s = 1;
  if (s > 128) s = 128;
  if (s > n) s = n;
  return (int)s;
}

size_t tile_h_workspace_bytes(int64_t n, int nrhs, int nsplit) {
  // four FP16 planes [npad][ldx], column maxima and scales, f [nrhs][n], the FP32 partial sums
  // [nsplit][nrhs][n] and the near launch's FP64 partial [nrhs][n]
  const size_t ldx = (size_t)tile_ldx(nrhs);
  return 2 * kHPlanes * (size_t)h_npad(n) * ldx + 256 + 16 * ldx + 256 + sizeof(double2) * (size_t)n * nrhs +
         sizeof(float2) * (size_t)n * nrhs * (size_t)nsplit + 256 + sizeof(double2) * (size_t)n * nrhs + 512;
}

hipError_t launch_apply_tile_h(const Scat &s, const double *x, double *y, int nrhs, int64_t ld, Mode mode, int nsplit,
                               void *ws, hipStream_t st, hipEvent_t far_start, hipEvent_t far_stop) {
  const int64_t n = s.n, npad = h_npad(n);
  const int ldx = tile_ldx(nrhs);
  auto al = [](char *q) { return (char *)(((uintptr_t)q + 255) & ~(uintptr_t)255); };
  char *p = (char *)ws;
  _Float16 *Xh = (_Float16 *)p;
  p = al(p + 2 * kHPlanes * (size_t)npad * ldx);
  unsigned *cmax = (unsigned *)p;
  double *colinv = (double *)(p + 8 * (size_t)ldx);
  p = al(p + 16 * (size_t)ldx);
  double2 *f = (double2 *)p;
  // the tiles' FP32 partial sums [split][rhs][n], then the near launch's FP64 partial [rhs][n]
  float2 *part = (float2 *)(f + n * nrhs);
  const double2 *xc = (const double2 *)x;
  const int fwd = mode == Mode::Forward ? 1 : 0;
  zero_u32_kernel<<<(nrhs + 255) / 256, 256, 0, st>>>(cmax, nrhs);
  colmax_kernel<<<dim3((unsigned)((n + kBlock - 1) / kBlock), (unsigned)nrhs), kBlock, 0, st>>>(
      n, s.perm, s.w, s.m, xc, ld, s.off, fwd, cmax);
  prologue_h_kernel<<<(unsigned)((npad * ldx + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      n, nrhs, ldx, s.perm, s.w, s.m, xc, ld, s.off, fwd, cmax, Xh, f, colinv);
  // a multiple of 32 sources per split
  const int split_len = (int)(((n + nsplit - 1) / nsplit + 31) / 32 * 32);
  const int used = (int)((n + split_len - 1) / split_len);
  const int excl = s.near_ok ? 1 : 0;   // z < 1 pairs in FP64 through the mixed correction
  if (far_start) (void)hipEventRecord(far_start, st);
  // the kernel is bound by the Green's evaluation on the VALU, so a wave takes as many right-hand
  // sides as its registers hold: two M-tiles and four N-tiles (162 VGPRs, three waves per SIMD) at 64
  // columns.  Measured at N = 122 500, B = 64, k = 40: 29.1 ms (MT 2, NT 4), 35.0 (MT 1, NT 4), 40.9
  // (MT 2, NT 4 held to 128 VGPRs, four waves per SIMD, with spills); the FP32 tiles take 62.7 ms
  constexpr int MT = 2, NT = 2;
  const dim3 grid((unsigned)((n + 64 * MT - 1) / (64 * MT)), (unsigned)used, (unsigned)(ldx / 32 > 0 ? ldx / 32 : 1));
  if (ldx % 64 == 0) {
    const dim3 g4((unsigned)((n + 64 * MT - 1) / (64 * MT)), (unsigned)used, (unsigned)(ldx / 64));
    if (fwd)
      far_tile_h_kernel<MT, 4, false><<<g4, kBlock, 0, st>>>((int)n, s.pos, Xh, ldx, nrhs, s.k * s.k, split_len,
                                                              part, excl);
    else
      far_tile_h_kernel<MT, 4, true><<<g4, kBlock, 0, st>>>((int)n, s.pos, Xh, ldx, nrhs, s.k * s.k, split_len,
                                                             part, excl);
  } else if (ldx % 32 != 0) {
    // an odd number of 16-column groups: one N-tile per wave
    const dim3 g1((unsigned)((n + 64 * MT - 1) / (64 * MT)), (unsigned)used, (unsigned)(ldx / 16));
    if (fwd)
      far_tile_h_kernel<MT, 1, false><<<g1, kBlock, 0, st>>>((int)n, s.pos, Xh, ldx, nrhs, s.k * s.k, split_len,
                                                              part, excl);
    else
      far_tile_h_kernel<MT, 1, true><<<g1, kBlock, 0, st>>>((int)n, s.pos, Xh, ldx, nrhs, s.k * s.k, split_len,
                                                             part, excl);
  } else if (fwd) {
    far_tile_h_kernel<MT, NT, false><<<grid, kBlock, 0, st>>>((int)n, s.pos, Xh, ldx, nrhs, s.k * s.k, split_len,
                                                               part, excl);
  } else {
    far_tile_h_kernel<MT, NT, true><<<grid, kBlock, 0, st>>>((int)n, s.pos, Xh, ldx, nrhs, s.k * s.k, split_len,
                                                              part, excl);
  }
  if (far_stop) (void)hipEventRecord(far_stop, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double2 *near = (double2 *)al((char *)(part + (size_t)used * nrhs * n));
  e = launch_near(s, f, nrhs, !fwd, near, st);
  if (e != hipSuccess) return e;
  return launch_epilogue_h(s, part, used, colinv, s.near_ok ? near : nullptr, f, x, y, nrhs, ld, mode, st);
}

hipError_t launch_apply_tile(const Scat &s, const double *x, double *y, int nrhs, int64_t ld, Mode mode, bool single,
                             int nsplit, void *ws, hipStream_t st, hipEvent_t far_start, hipEvent_t far_stop) {
  const int64_t n = s.n;
  const int ldx = tile_ldx(nrhs);
  char *p = (char *)ws;
  void *X = p;
  p += (single ? sizeof(float2) : sizeof(double2)) * (size_t)n * ldx;
  p = (char *)(((uintptr_t)p + 255) & ~(uintptr_t)255);
  double2 *f = (double2 *)p;
  double2 *part = f + n * nrhs;
  const unsigned gp = (unsigned)((n * ldx + kBlock - 1) / kBlock);
  const double2 *xc = (const double2 *)x;
  const bool fwd = mode == Mode::Forward;
  if (single) {
    if (fwd)
      prologue_tile_kernel<float, Mode::Forward><<<gp, kBlock, 0, st>>>(n, nrhs, ldx, s.perm, s.w, s.m, xc, ld, s.off,
                                                                        (float2 *)X, f);
    else
      prologue_tile_kernel<float, Mode::Adjoint><<<gp, kBlock, 0, st>>>(n, nrhs, ldx, s.perm, s.w, s.m, xc, ld, s.off,
                                                                        (float2 *)X, f);
  } else {
    if (fwd)
      prologue_tile_kernel<double, Mode::Forward><<<gp, kBlock, 0, st>>>(n, nrhs, ldx, s.perm, s.w, s.m, xc, ld,
                                                                         s.off, (double2 *)X, f);
    else
      prologue_tile_kernel<double, Mode::Adjoint><<<gp, kBlock, 0, st>>>(n, nrhs, ldx, s.perm, s.w, s.m, xc, ld,
                                                                         s.off, (double2 *)X, f);
  }
  const int split_len = (int)((n + nsplit - 1) / nsplit);
  if (far_start) (void)hipEventRecord(far_start, st);
  // with four N-tiles of accumulators the larger M-tiles cost occupancy (tile_mt has the measurements)
  if (single)
    launch_tile_nt<float, 2>(s, X, ldx, nrhs, split_len, nsplit, part, !fwd, st);
  else if (tile_mt(nrhs, false) == 1)
    launch_tile_nt<double, 1>(s, X, ldx, nrhs, split_len, nsplit, part, !fwd, st);
  else
    launch_tile_nt<double, 2>(s, X, ldx, nrhs, split_len, nsplit, part, !fwd, st);
  if (far_stop) (void)hipEventRecord(far_stop, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (single && s.near_ok) {
    e = launch_near(s, f, nrhs, !fwd, part + (size_t)nsplit * nrhs * n, st);
    if (e != hipSuccess) return e;
    ++nsplit;
  }
  return launch_epilogue(s, part, nsplit, f, x, y, nrhs, ld, mode, st);
}

}  // namespace lsk
