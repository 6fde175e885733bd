// FP64 operator apply: y = L x = x + k^2 (G~ W + C)(m x)   (paper, Section 3,
// eqs. linear_system and linear_system_matrix), and its adjoint
// y = L^H x = x + k^2 conj(m) (W conj(G~) x + C^H x).
//
// Three kernels per apply, all stream-ordered:
//   prologue : gather each column from the caller's order into the internal order and form
//              the far-sum densities s = w m x (forward) or s = x (adjoint) in a [node][rhs]
//              layout, plus f = m x (or x) in [rhs][node] layout for the sparse correction;
//   far      : the punctured Green's sum t_j = sum_{n != j} G(y_j, y_n) s_n over a chunk of
//              sources.  One target per lane; every lane of a wavefront walks the same source,
//              whose position and densities are uniform across the wave and are read through the
//              scalar data path into SGPRs (no LDS staging or barriers needed); G/K is evaluated
//              in registers (hankel.h) once per pair and reused for the RHS of the chunk;
//   epilogue : sum the source-chunk partials in a fixed order (deterministic), scale by K, add
//              the CSR correction, apply the diagonal factors and scatter to the caller's order.
#include <vector>

#include "hankel.h"
#include "internal.h"

namespace lsk {

namespace {

constexpr int kBlock = 256;

__constant__ HankelTable d_hankel = kHankelTable;
__constant__ SinCosTable d_sincos = kSinCosTable;

typedef __attribute__((address_space(4))) const HankelTable ConstTab;

// The table's constant-address-space pointer, hidden from loop-invariant code motion: the
// coefficient loads stay inside the source loop as scalar loads feeding SGPR operands,
// instead of being hoisted into ~260 live vector registers.
__device__ __forceinline__ ConstTab &hankel_table() {
  ConstTab *t = (ConstTab *)&d_hankel;
  asm volatile("" : "+s"(t));
  return *t;
}

template <Mode M>
__global__ __launch_bounds__(kBlock) void prologue_kernel(int64_t n, int nrhs, const int32_t *__restrict__ perm,
                                                          const double *__restrict__ w,
                                                          const double2 *__restrict__ m,
                                                          const double2 *__restrict__ x, int64_t ld,
                                                          int64_t off, double2 *__restrict__ sd,
                                                          double2 *__restrict__ f) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n * nrhs) return;
  const int64_t i = t / nrhs;
  const int b = (int)(t - i * nrhs);
  const double2 xv = x[(int64_t)b * ld + off + perm[i]];
  if (M == Mode::Forward) {
    const double2 mi = m[i];
    const double2 fv = make_double2(mi.x * xv.x - mi.y * xv.y, mi.x * xv.y + mi.y * xv.x);
    f[(int64_t)b * n + i] = fv;
    sd[t] = make_double2(w[i] * fv.x, w[i] * fv.y);
  } else {
    f[(int64_t)b * n + i] = xv;
    sd[t] = xv;
  }
}

// One source against the TPL targets of this lane: positions and densities of the source are
// wave-uniform (scalar loads), G is evaluated once per pair and reused for the BC right-hand sides.
template <int TPL, int BC, bool CONJ, bool MASKED>
__device__ __forceinline__ void far_source(int j, const int (&it)[TPL], const double (&xt)[TPL],
                                           const double (&yt)[TPL], double k2, const double2 *__restrict__ pos,
                                           const double2 *__restrict__ d, const PhaseLds &sct,
                                           double (&ar)[TPL][BC], double (&ai)[TPL][BC]) {
  const double2 p = pos[j];
  double gr[TPL], gi[TPL];
#pragma unroll
  for (int q = 0; q < TPL; ++q) {
    const double dx = xt[q] - p.x;
    const double dy = yt[q] - p.y;
    const double A = k2 * std::fma(dx, dx, dy * dy);
    green_unit<true>(A, gr[q], gi[q], hankel_table(), sct);
    if (MASKED) {
      const bool self = (j == it[q]);
      gr[q] = self ? 0.0 : gr[q];
      gi[q] = self ? 0.0 : gi[q];
    }
    if (CONJ) gi[q] = -gi[q];
  }
#pragma unroll
  for (int b = 0; b < BC; ++b) {
    const double2 sv = d[b];
#pragma unroll
    for (int q = 0; q < TPL; ++q) {
      ar[q][b] = std::fma(gr[q], sv.x, std::fma(-gi[q], sv.y, ar[q][b]));
      ai[q][b] = std::fma(gr[q], sv.y, std::fma(gi[q], sv.x, ai[q][b]));
    }
  }
}

// grid: (ceil(n / (kBlock * TPL)), source splits, nrhs / BC).  Lane l of the wavefront starting at
// target w0 owns targets w0 + q*64 + l, q < TPL.
template <int TPL, int BC, bool CONJ>
__global__ __launch_bounds__(kBlock) void far_fp64_kernel(int n, const double *__restrict__ px,
                                                         const double *__restrict__ py,
                                                         const double2 *__restrict__ pos,
                                                         const double2 *__restrict__ sd, int nrhs,
                                                         double k2, int split_len,
                                                         double2 *__restrict__ part) {
  __shared__ double2 sct_lds[SINCOS_N];
  const PhaseLds sct = load_sincos(sct_lds, d_sincos);
  const int c0 = blockIdx.z * BC;
  const int w0 = __builtin_amdgcn_readfirstlane(blockIdx.x * kBlock * TPL + (threadIdx.x >> 6) * 64 * TPL);
  const int lane = threadIdx.x & 63;
  int it[TPL];
  double xt[TPL], yt[TPL];
#pragma unroll
  for (int q = 0; q < TPL; ++q) {
    it[q] = w0 + q * 64 + lane;
    const int ii = it[q] < n ? it[q] : n - 1;
    xt[q] = px[ii];
    yt[q] = py[ii];
  }
  const int s0 = blockIdx.y * split_len;
  const int s1 = min(n, s0 + split_len);
  double ar[TPL][BC], ai[TPL][BC];
#pragma unroll
  for (int q = 0; q < TPL; ++q)
#pragma unroll
    for (int b = 0; b < BC; ++b) ar[q][b] = ai[q][b] = 0.0;
  // sources before, inside and after this wavefront's own target range (only the middle
  // range can contain the self pair j == i, which the punctured sum drops)
  const int e0 = min(s1, max(s0, w0));
  const int e1 = min(s1, max(s0, w0 + 64 * TPL));
  for (int j = s0; j < e0; ++j)
    far_source<TPL, BC, CONJ, false>(j, it, xt, yt, k2, pos, sd + (int64_t)j * nrhs + c0, sct, ar, ai);
  for (int j = e0; j < e1; ++j)
    far_source<TPL, BC, CONJ, true>(j, it, xt, yt, k2, pos, sd + (int64_t)j * nrhs + c0, sct, ar, ai);
  for (int j = e1; j < s1; ++j)
    far_source<TPL, BC, CONJ, false>(j, it, xt, yt, k2, pos, sd + (int64_t)j * nrhs + c0, sct, ar, ai);
#pragma unroll
  for (int q = 0; q < TPL; ++q)
    if (it[q] < n) {
#pragma unroll
      for (int b = 0; b < BC; ++b)
        part[((int64_t)blockIdx.y * nrhs + c0 + b) * n + it[q]] = make_double2(ar[q][b], ai[q][b]);
    }
}

// The punctured far sum of one right-hand side with every unordered pair evaluated once (G is
// symmetric in its two points).  Workgroup (T, S), S >= T, takes the kBlock targets of block T
// against the kBlock sources of block S:
//   S > T : each lane adds G(t, j) d_j into its target t, and the wave's sum over its 64 targets
//           of G(t, j) d_t into source j (a butterfly across the lanes, the four waves through
//           LDS), so that the pair also serves row j;
//   S == T: every pair of the block in both orders, the self pair left out.
// Slot S of row i holds its sum over block S's sources: workgroup (blk(i), S) writes it for
// S >= blk(i), the transposed sums of workgroup (S, blk(i)) for S < blk(i), so every slot of every
// row is written exactly once and the epilogue adds the nb slots.
// grid: nb (nb + 1) / 2 workgroups in the order (0, 0), (0, 1), ..., (0, nb - 1), (1, 1), ...
template <bool CONJ>
__global__ __launch_bounds__(kBlock) void far_fp64_sym_kernel(int n, int nb, const double *__restrict__ px,
                                                             const double *__restrict__ py,
                                                             const double2 *__restrict__ pos,
                                                             const double2 *__restrict__ sd, double k2,
                                                             double2 *__restrict__ part) {
  __shared__ double2 sct_lds[SINCOS_N];
  __shared__ double2 red[kBlock / 64][kBlock];
  const PhaseLds sct = load_sincos(sct_lds, d_sincos);
  // (T, S) of this workgroup: T rows of nb, nb - 1, ... pairs precede row T
  const int64_t idx = blockIdx.x;
  const double b2 = 2.0 * nb + 1.0;
  int T = (int)((b2 - std::sqrt(b2 * b2 - 8.0 * (double)idx)) * 0.5);
  auto first = [&](int r) { return (int64_t)r * (2 * (int64_t)nb - r + 1) / 2; };
  while (T > 0 && first(T) > idx) --T;
  while (T + 1 < nb && first(T + 1) <= idx) ++T;
  const int S = T + (int)(idx - first(T));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int t = T * kBlock + threadIdx.x;
  const int ti = t < n ? t : n - 1;
  const double xt = px[ti], yt = py[ti];
  const double2 dt = t < n ? sd[t] : make_double2(0.0, 0.0);
  const int s0 = S * kBlock, s1 = min(n, s0 + kBlock);
  double ar[1][1] = {{0.0}}, ai[1][1] = {{0.0}};
  if (S == T) {
    const int it[1] = {t};
    const double xa[1] = {xt}, ya[1] = {yt};
    for (int j = s0; j < s1; ++j)
      far_source<1, 1, CONJ, true>(j, it, xa, ya, k2, pos, sd + j, sct, ar, ai);
  } else {
    // eight sources at a time: G d_t of each lane for the eight, then a reduce-scatter across the
    // lanes (lane bits 5, 4, 3 halve the set: 8 -> 4 -> 2 -> 1 values, then bits 2..0 add up), so
    // that lanes 8u .. 8u + 7 end with source u's wave sum; five exchanges per source
    const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
    for (int j0 = s0; j0 < s1; j0 += 8) {
      double vr[8], vi[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        vr[u] = vi[u] = 0.0;
        const int j = j0 + u;
        if (j < s1) {
          const double2 p = pos[j];
          const double dx = xt - p.x, dy = yt - p.y;
          const double A = k2 * std::fma(dx, dx, dy * dy);
          double gr, gi;
          green_unit<true>(A, gr, gi, hankel_table(), sct);
          if (CONJ) gi = -gi;
          const double2 sv = sd[j];
          ar[0][0] = std::fma(gr, sv.x, std::fma(-gi, sv.y, ar[0][0]));
          ai[0][0] = std::fma(gr, sv.y, std::fma(gi, sv.x, ai[0][0]));
          vr[u] = std::fma(gr, dt.x, -gi * dt.y);
          vi[u] = std::fma(gr, dt.y, gi * dt.x);
        }
      }
      double r4[4], i4[4], r2[2], i2[2];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        r4[q] = (h5 ? vr[4 + q] : vr[q]) + __shfl_xor(h5 ? vr[q] : vr[4 + q], 32);
        i4[q] = (h5 ? vi[4 + q] : vi[q]) + __shfl_xor(h5 ? vi[q] : vi[4 + q], 32);
      }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        r2[q] = (h4 ? r4[2 + q] : r4[q]) + __shfl_xor(h4 ? r4[q] : r4[2 + q], 16);
        i2[q] = (h4 ? i4[2 + q] : i4[q]) + __shfl_xor(h4 ? i4[q] : i4[2 + q], 16);
      }
      double r1 = (h3 ? r2[1] : r2[0]) + __shfl_xor(h3 ? r2[0] : r2[1], 8);
      double i1 = (h3 ? i2[1] : i2[0]) + __shfl_xor(h3 ? i2[0] : i2[1], 8);
#pragma unroll
      for (int off = 4; off > 0; off >>= 1) {
        r1 += __shfl_xor(r1, off);
        i1 += __shfl_xor(i1, off);
      }
      const int u = (h5 ? 4 : 0) + (h4 ? 2 : 0) + (h3 ? 1 : 0);
      if ((lane & 7) == 0 && j0 + u < s1) red[wave][j0 + u - s0] = make_double2(r1, i1);
    }
  }
  if (t < n) part[(int64_t)S * n + t] = make_double2(ar[0][0], ai[0][0]);
  if (S != T) {
    __syncthreads();
    const int j = s0 + threadIdx.x;
    if (j < s1) {
      double2 v = red[0][threadIdx.x];
#pragma unroll
      for (int w = 1; w < kBlock / 64; ++w) v = make_double2(v.x + red[w][threadIdx.x].x, v.y + red[w][threadIdx.x].y);
      part[(int64_t)T * n + j] = v;
    }
  }
}

// H: the partials are the split-FP16 tiles' FP32 sums (parth, [split][rhs][n]) times the column
// scale colinv[b], then the near launch's FP64 partial (part, [rhs][n], when given)
template <Mode M, bool H>
__global__ __launch_bounds__(kBlock) void epilogue_kernel(
    int64_t n, int nrhs, int nsplit, const double2 *__restrict__ part, const float2 *__restrict__ parth,
    const double *__restrict__ colinv, const double2 *__restrict__ f,
    const int64_t *__restrict__ rp, const int32_t *__restrict__ ci, const double2 *__restrict__ cv,
    const double *__restrict__ w, const double2 *__restrict__ m, const int32_t *__restrict__ perm,
    const double2 *__restrict__ x, double2 *__restrict__ y, int64_t ld, int64_t off, double k2) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= n) return;
  double ar = 0.0, ai = 0.0;
  // unrolled so that eight partial loads are in flight before the first add (the sum keeps its
  // order); one load per iteration waited for each round trip in turn
  if constexpr (H) {
    // each partial scaled, then added, without contraction into a fused multiply-add: the same
    // values as scaling in the tile kernel and summing FP64 partials
#pragma clang fp contract(off)
    const double cb = colinv[b];
#pragma unroll 8
    for (int sp = 0; sp < nsplit; ++sp) {
      const float2 p = parth[((int64_t)sp * nrhs + b) * n + i];
      ar += (double)p.x * cb;
      ai += (double)p.y * cb;
    }
    if (part) {
      const double2 p = part[(int64_t)b * n + i];
      ar += p.x;
      ai += p.y;
    }
  } else {
#pragma unroll 8
    for (int sp = 0; sp < nsplit; ++sp) {
      const double2 p = part[((int64_t)sp * nrhs + b) * n + i];
      ar += p.x;
      ai += p.y;
    }
  }
  // the far kernels sum G/K (hankel.h); K and, for the adjoint, the weight are applied here
  const double gs = M != Mode::Forward ? w[i] * G_SCALE : G_SCALE;
  ar *= gs;
  ai *= gs;
  const double2 *fb = f + (int64_t)b * n;
  double cr = 0.0, cim = 0.0;
#pragma unroll 4
  for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
    const double2 c = cv[q];
    const double2 v = fb[ci[q]];
    cr = std::fma(c.x, v.x, std::fma(-c.y, v.y, cr));
    cim = std::fma(c.x, v.y, std::fma(c.y, v.x, cim));
  }
  ar += cr;
  ai += cim;
  if (M == Mode::Adjoint) {
    const double2 mi = m[i];   // conj(m) * acc
    const double tr = mi.x * ar + mi.y * ai;
    const double ti = mi.x * ai - mi.y * ar;
    ar = tr;
    ai = ti;
  }
  const int64_t c = (int64_t)b * ld + off + perm[i];
  if (M == Mode::AdjointPotential) {
    y[c] = make_double2(ar, ai);
    return;
  }
  const double2 xv = x[c];
  y[c] = make_double2(std::fma(k2, ar, xv.x), std::fma(k2, ai, xv.y));
}

__global__ __launch_bounds__(kBlock) void eval_green_kernel(const double *__restrict__ z2, double2 *__restrict__ g,
                                                            int64_t n, int single) {
  __shared__ double2 sct_lds[SINCOS_N];
  const PhaseLds sct = load_sincos(sct_lds, d_sincos);
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  if (single) {
    float gr, gi;
    green32_unit(z2[i], gr, gi, d_hankel);
    g[i] = make_double2((double)gr * G_SCALE, (double)gi * G_SCALE);
  } else {
    double gr, gi;
    green<true>(z2[i], gr, gi, d_hankel, sct);
    g[i] = make_double2(gr, gi);
  }
}

template <int BC, bool CONJ>
void launch_far(const Scat &s, const double2 *pos, const double2 *sd, int nrhs, int split_len, int nsplit,
                double2 *part, int tpl, hipStream_t st) {
  const int per_block = kBlock * tpl;
  dim3 grid((unsigned)((s.n + per_block - 1) / per_block), (unsigned)nsplit, (unsigned)(nrhs / BC));
  if (tpl == 2)
    far_fp64_kernel<2, BC, CONJ><<<grid, kBlock, 0, st>>>((int)s.n, s.px, s.py, pos, sd, nrhs, s.k * s.k,
                                                          split_len, part);
  else
    far_fp64_kernel<1, BC, CONJ><<<grid, kBlock, 0, st>>>((int)s.n, s.px, s.py, pos, sd, nrhs, s.k * s.k,
                                                          split_len, part);
}

// Field recovery (paper, Section 3, eq. field_recovery): the far sum at nt targets that are
// not nodes, part[(split * nrhs + c0 + b) * nt + t] = sum over the split's sources of
// G/K(x_t, y_n) sd[n][c0 + b].  One target per lane; no pair is left out.
template <int BC>
__global__ __launch_bounds__(kBlock) void field_far_kernel(int nt, const double *__restrict__ tx,
                                                          const double *__restrict__ ty, int n,
                                                          const double2 *__restrict__ pos,
                                                          const double2 *__restrict__ sd, int nrhs, double k2,
                                                          int split_len, double2 *__restrict__ part) {
  __shared__ double2 sct_lds[SINCOS_N];
  const PhaseLds sct = load_sincos(sct_lds, d_sincos);
  const int c0 = blockIdx.z * BC;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int ti = t < nt ? t : nt - 1;
  const int it[1] = {-1};   // no source index matches
  const double xt[1] = {tx[ti]}, yt[1] = {ty[ti]};
  const int s0 = blockIdx.y * split_len;
  const int s1 = min(n, s0 + split_len);
  double ar[1][BC], ai[1][BC];
#pragma unroll
  for (int b = 0; b < BC; ++b) ar[0][b] = ai[0][b] = 0.0;
  for (int j = s0; j < s1; ++j)
    far_source<1, BC, false, false>(j, it, xt, yt, k2, pos, sd + (int64_t)j * nrhs + c0, sct, ar, ai);
  if (t < nt) {
#pragma unroll
    for (int b = 0; b < BC; ++b)
      part[((int64_t)blockIdx.y * nrhs + c0 + b) * nt + t] = make_double2(ar[0][b], ai[0][b]);
  }
}

// out[b * nt + t] = -k^2 (K sum_split part + sum_c C_tc f_b[c]): the scattered field
__global__ __launch_bounds__(kBlock) void field_epilogue_kernel(int64_t nt, int nrhs, int nsplit,
                                                               const double2 *__restrict__ part,
                                                               const int64_t *__restrict__ rp,
                                                               const int32_t *__restrict__ ci,
                                                               const double2 *__restrict__ cv,
                                                               const double2 *__restrict__ f, int64_t n, double k2,
                                                               double2 *__restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int b = blockIdx.y;
  if (t >= nt) return;
  double ar = 0.0, ai = 0.0;
#pragma unroll 8
  for (int sp = 0; sp < nsplit; ++sp) {
    const double2 p = part[((int64_t)sp * nrhs + b) * nt + t];
    ar += p.x;
    ai += p.y;
  }
  ar *= G_SCALE;
  ai *= G_SCALE;
  const double2 *fb = f + (int64_t)b * n;
#pragma unroll 4
  for (int64_t q = rp[t]; q < rp[t + 1]; ++q) {
    const double2 c = cv[q];
    const double2 v = fb[ci[q]];
    ar = std::fma(c.x, v.x, std::fma(-c.y, v.y, ar));
    ai = std::fma(c.x, v.y, std::fma(c.y, v.x, ai));
  }
  out[(int64_t)b * nt + t] = make_double2(-k2 * ar, -k2 * ai);
}

}  // namespace

int auto_source_split(int64_t n, int nrhs, int launches_per_split, int tpl) {
  // aim for about 128 waves per SIMD (256 CUs x 4 SIMDs) over the launch: many short rounds
  // of resident waves keep the CUs evenly loaded to the end (measured: 128 splits run the
  // N = 58 500 single-RHS sum 38% faster than 8); the partial sums are capped at 512 MiB
  const int64_t waves = ((n + 64 * tpl - 1) / (64 * tpl)) * (int64_t)launches_per_split;
  int64_t s = (131072 + waves - 1) / waves;
  const int64_t cap = ((int64_t)512 << 20) / ((int64_t)16 * n * nrhs);
  if (s > cap) s = cap;
  if (s < 1) s = 1;
  if (s > 256) s = 256;
  if (s > n) s = n;
  return (int)s;
}

int fp64_sym_splits(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

size_t apply_workspace_bytes(int64_t n, int nrhs, int nsplit) {
  // sd [n][nrhs], f [nrhs][n], part [nsplit][nrhs][n]  (double2 each)
  return sizeof(double2) * (size_t)n * nrhs * (2 + (size_t)nsplit) + 256;
}

hipError_t launch_apply_fp64(const Scat &s, const double *x, double *y, int nrhs, int64_t ld, Mode mode,
                             int nsplit, int rhs_chunk, int tpl, void *ws, hipStream_t st, hipEvent_t far_start,
                             hipEvent_t far_stop) {
  const int64_t n = s.n;
  double2 *sd = (double2 *)ws;
  double2 *f = sd + n * nrhs;
  double2 *part = f + n * nrhs;
  const double2 *pos = s.pos;
  const double2 *xc = (const double2 *)x;
  const unsigned gp = (unsigned)((n * nrhs + kBlock - 1) / kBlock);
  if (mode == Mode::Forward)
    prologue_kernel<Mode::Forward><<<gp, kBlock, 0, st>>>(n, nrhs, s.perm, s.w, s.m, xc, ld, s.off, sd, f);
  else
    prologue_kernel<Mode::Adjoint><<<gp, kBlock, 0, st>>>(n, nrhs, s.perm, s.w, s.m, xc, ld, s.off, sd, f);
  const int split_len = (int)((n + nsplit - 1) / nsplit);
  const bool conj = mode != Mode::Forward;
  if (nrhs == 1 && tpl == 1 && nsplit == fp64_sym_splits(n)) {
    // one right-hand side: each unordered pair once, one slot per source block
    const int nb = nsplit;
    const unsigned wg = (unsigned)((int64_t)nb * (nb + 1) / 2);
    if (far_start) (void)hipEventRecord(far_start, st);
    if (conj)
      far_fp64_sym_kernel<true><<<wg, kBlock, 0, st>>>((int)n, nb, s.px, s.py, pos, sd, s.k * s.k, part);
    else
      far_fp64_sym_kernel<false><<<wg, kBlock, 0, st>>>((int)n, nb, s.px, s.py, pos, sd, s.k * s.k, part);
    if (far_stop) (void)hipEventRecord(far_stop, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_epilogue(s, part, nsplit, f, x, y, nrhs, ld, mode, st);
  }
  // RHS per pass: the largest of 16, 8, 4, 1 that is <= rhs_chunk and divides nrhs
  int bc = 1;
  for (int c : {16, 8, 4})
    if (c <= rhs_chunk && nrhs % c == 0) {
      bc = c;
      break;
    }
  if (far_start) (void)hipEventRecord(far_start, st);
  switch (bc * 2 + (conj ? 1 : 0)) {
    case 2: launch_far<1, false>(s, pos, sd, nrhs, split_len, nsplit, part, tpl, st); break;
    case 3: launch_far<1, true>(s, pos, sd, nrhs, split_len, nsplit, part, tpl, st); break;
    case 8: launch_far<4, false>(s, pos, sd, nrhs, split_len, nsplit, part, tpl, st); break;
    case 9: launch_far<4, true>(s, pos, sd, nrhs, split_len, nsplit, part, tpl, st); break;
    case 16: launch_far<8, false>(s, pos, sd, nrhs, split_len, nsplit, part, tpl, st); break;
    case 17: launch_far<8, true>(s, pos, sd, nrhs, split_len, nsplit, part, tpl, st); break;
    case 32: launch_far<16, false>(s, pos, sd, nrhs, split_len, nsplit, part, tpl, st); break;
    case 33: launch_far<16, true>(s, pos, sd, nrhs, split_len, nsplit, part, tpl, st); break;
    default: return hipErrorInvalidValue;
  }
  if (far_stop) (void)hipEventRecord(far_stop, st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_epilogue(s, part, nsplit, f, x, y, nrhs, ld, mode, st);
}

hipError_t launch_epilogue(const Scat &s, const double2 *part, int nsplit, const double2 *f, const double *x,
                           double *y, int nrhs, int64_t ld, Mode mode, hipStream_t st) {
  const int64_t n = s.n;
  const double2 *xc = (const double2 *)x;
  double2 *yc = (double2 *)y;
  dim3 ge((unsigned)((n + kBlock - 1) / kBlock), (unsigned)nrhs);
  const double k2 = s.k * s.k;
  const int64_t *rp = s.rp, *rpH = s.rpH;
  const int32_t *ci = s.ci, *ciH = s.ciH;
  const double2 *cv = s.cv, *cvH = s.cvH;
  if (mode == Mode::Forward)
    epilogue_kernel<Mode::Forward, false><<<ge, kBlock, 0, st>>>(n, nrhs, nsplit, part, nullptr, nullptr, f, rp, ci,
                                                                cv, s.w, s.m, s.perm, xc, yc, ld, s.off, k2);
  else if (mode == Mode::Adjoint)
    epilogue_kernel<Mode::Adjoint, false><<<ge, kBlock, 0, st>>>(n, nrhs, nsplit, part, nullptr, nullptr, f, rpH, ciH,
                                                                cvH, s.w, s.m, s.perm, xc, yc, ld, s.off, k2);
  else
    epilogue_kernel<Mode::AdjointPotential, false><<<ge, kBlock, 0, st>>>(n, nrhs, nsplit, part, nullptr, nullptr, f,
                                                                         rpH, ciH, cvH, s.w, s.m, s.perm, xc, yc, ld,
                                                                         s.off, k2);
  return hipGetLastError();
}

hipError_t launch_epilogue_h(const Scat &s, const float2 *parth, int nsplit, const double *colinv,
                             const double2 *near, const double2 *f, const double *x, double *y, int nrhs, int64_t ld,
                             Mode mode, hipStream_t st) {
  const int64_t n = s.n;
  const double2 *xc = (const double2 *)x;
  double2 *yc = (double2 *)y;
  dim3 ge((unsigned)((n + kBlock - 1) / kBlock), (unsigned)nrhs);
  const double k2 = s.k * s.k;
  if (mode == Mode::Forward)
    epilogue_kernel<Mode::Forward, true><<<ge, kBlock, 0, st>>>(n, nrhs, nsplit, near, parth, colinv, f, s.rp, s.ci,
                                                               s.cv, s.w, s.m, s.perm, xc, yc, ld, s.off, k2);
  else if (mode == Mode::Adjoint)
    epilogue_kernel<Mode::Adjoint, true><<<ge, kBlock, 0, st>>>(n, nrhs, nsplit, near, parth, colinv, f, s.rpH,
                                                               s.ciH, s.cvH, s.w, s.m, s.perm, xc, yc, ld, s.off, k2);
  else
    epilogue_kernel<Mode::AdjointPotential, true><<<ge, kBlock, 0, st>>>(n, nrhs, nsplit, near, parth, colinv, f,
                                                                        s.rpH, s.ciH, s.cvH, s.w, s.m, s.perm, xc, yc,
                                                                        ld, s.off, k2);
  return hipGetLastError();
}

// The kernels' arithmetic on the host, table tail included (for checks on a CPU).
void eval_green_host(const double *z2, double *g, int64_t n) {
  static const std::vector<double2> sct = [] {
    std::vector<double2> t(SINCOS_N);
    for (int i = 0; i < SINCOS_N; ++i) t[i] = make_double2(kSinCosTable.v[2 * i], kSinCosTable.v[2 * i + 1]);
    return t;
  }();
  const PhaseLds ph = host_phase_lds(sct.data());
  for (int64_t i = 0; i < n; ++i) green<true>(z2[i], g[2 * i], g[2 * i + 1], kHankelTable, ph);
}

hipError_t launch_eval_green(const double *z2, double *g, int64_t n, int single, hipStream_t st) {
  if (n == 0) return hipSuccess;
  eval_green_kernel<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(z2, (double2 *)g, n, single);
  return hipGetLastError();
}

}  // namespace lsk

namespace lsk {

int field_source_split(int64_t n, int64_t nt, int nrhs) {
  // about 128 waves per SIMD over the launch, partials capped at 512 MiB
  const int64_t waves = (nt + 63) / 64;
  int64_t s = (131072 + waves - 1) / waves;
  const int64_t cap = ((int64_t)512 << 20) / ((int64_t)16 * nt * nrhs);
  if (s > cap) s = cap;
  if (s < 1) s = 1;
  if (s > 256) s = 256;
  if (s > n) s = n;
  return (int)s;
}

size_t field_workspace_bytes(int64_t n, int nrhs, int64_t nt, int nsplit) {
  // sd [n][nrhs], f [nrhs][n], part [nsplit][nrhs][nt]  (double2 each), 256-byte aligned
  return sizeof(double2) * ((size_t)2 * n * nrhs + (size_t)nsplit * nrhs * nt) + 1024;
}

hipError_t launch_field(const Scat &s, const double *u, int nrhs, int64_t ld, int64_t nt, const double *tx,
                        const double *ty, const int64_t *rp, const int32_t *ci, const double2 *cv, int nsplit,
                        double *out, void *ws, hipStream_t st, hipEvent_t far_start, hipEvent_t far_stop) {
  const int64_t n = s.n;
  auto al = [](char *p) { return (char *)(((uintptr_t)p + 255) & ~(uintptr_t)255); };
  char *p = al((char *)ws);
  double2 *sd = (double2 *)p;
  p = al(p + sizeof(double2) * n * nrhs);
  double2 *f = (double2 *)p;
  p = al(p + sizeof(double2) * n * nrhs);
  double2 *part = (double2 *)p;
  prologue_kernel<Mode::Forward><<<(unsigned)((n * nrhs + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      n, nrhs, s.perm, s.w, s.m, (const double2 *)u, ld, s.off, sd, f);
  const int split_len = (int)((n + nsplit - 1) / nsplit);
  const int bc = nrhs % 16 == 0 ? 16 : (nrhs % 8 == 0 ? 8 : (nrhs % 4 == 0 ? 4 : 1));
  dim3 grid((unsigned)((nt + kBlock - 1) / kBlock), (unsigned)nsplit, (unsigned)(nrhs / bc));
  if (far_start) (void)hipEventRecord(far_start, st);
  const double k2 = s.k * s.k;
  switch (bc) {
    case 16: field_far_kernel<16><<<grid, kBlock, 0, st>>>((int)nt, tx, ty, (int)n, s.pos, sd, nrhs, k2, split_len, part); break;
    case 8: field_far_kernel<8><<<grid, kBlock, 0, st>>>((int)nt, tx, ty, (int)n, s.pos, sd, nrhs, k2, split_len, part); break;
    case 4: field_far_kernel<4><<<grid, kBlock, 0, st>>>((int)nt, tx, ty, (int)n, s.pos, sd, nrhs, k2, split_len, part); break;
    default: field_far_kernel<1><<<grid, kBlock, 0, st>>>((int)nt, tx, ty, (int)n, s.pos, sd, nrhs, k2, split_len, part);
  }
  if (far_stop) (void)hipEventRecord(far_stop, st);
  dim3 ge((unsigned)((nt + kBlock - 1) / kBlock), (unsigned)nrhs);
  field_epilogue_kernel<<<ge, kBlock, 0, st>>>(nt, nrhs, nsplit, part, rp, ci, cv, f, n, k2, (double2 *)out);
  return hipGetLastError();
}

}  // namespace lsk
