// Far-field pattern, its adjoint and the contrast update, for misfit gradients.
//
// With G(x,y) ~ e^{i pi/4} / sqrt(8 pi k |x|) e^{ik|x|} e^{-ik x^.y} (the large-argument form of
// (i/4) H0^(1), paper Section 2), the scattered part of the representation formula
// (eq. representation_formula) has the far-field pattern
//     u_inf(x^_r) = -k^2 gamma sum_q w_q e^{-ik x^_r.y_q} m_q u_q,   gamma = e^{i pi/4}/sqrt(8 pi k),
// the normalisation under which the energy balance of Section 5 (eq. dissipativity_identity)
// holds.  A_rq denotes the matrix of that map; the adjoint kernel forms a = A^H r and the
// right-hand side conj(m) a of the adjoint solve.  All sums are fixed-order (deterministic).
#include <cmath>

#include "internal.h"

namespace lsk {

namespace {

constexpr int kBlock = 256;
constexpr int kQT = 4096;   // nodes per far-field partial

// part[(tile * R + r) * nrhs + d] = sum_{q in tile} A_rq m_q u_qd   (one block per (r, tile))
__global__ __launch_bounds__(kBlock) void farfield_kernel(int64_t n, int64_t off, int R, int nrhs,
                                                          const double *__restrict__ th, double k,
                                                          const double *__restrict__ px,
                                                          const double *__restrict__ py,
                                                          const double *__restrict__ w, const double2 *__restrict__ m,
                                                          const int32_t *__restrict__ perm,
                                                          const double2 *__restrict__ u, int64_t ld,
                                                          double2 *__restrict__ part) {
  __shared__ double2 lds[kBlock / 64];
  const int r = blockIdx.x, tile = blockIdx.y;
  const double cr = std::cos(th[r]), sr = std::sin(th[r]);
  const double g = k * k / std::sqrt(8.0 * M_PI * k);
  // -k^2 gamma = -(k^2 / sqrt(8 pi k)) e^{i pi/4}
  const double cre = -g * M_SQRT1_2, cim = -g * M_SQRT1_2;
  const int64_t q0 = (int64_t)tile * kQT, q1 = q0 + kQT < n ? q0 + kQT : n;
  for (int d = 0; d < nrhs; ++d) {
    double ar = 0.0, ai = 0.0;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += kBlock) {
      double s, c;
      sincos(-k * (cr * px[q] + sr * py[q]), &s, &c);
      const double2 mq = m[q];
      const double2 uq = u[(int64_t)d * ld + off + perm[q]];
      const double fr = (mq.x * uq.x - mq.y * uq.y) * w[q], fi = (mq.x * uq.y + mq.y * uq.x) * w[q];
      ar += c * fr - s * fi;
      ai += c * fi + s * fr;
    }
    for (int o = 32; o > 0; o >>= 1) {
      ar += __shfl_xor(ar, o);
      ai += __shfl_xor(ai, o);
    }
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = make_double2(ar, ai);
    __syncthreads();
    if (threadIdx.x == 0) {
      double tr = 0.0, ti = 0.0;
      for (int k2 = 0; k2 < kBlock / 64; ++k2) {
        tr += lds[k2].x;
        ti += lds[k2].y;
      }
      part[((int64_t)tile * R + r) * nrhs + d] = make_double2(cre * tr - cim * ti, cre * ti + cim * tr);
    }
    __syncthreads();
  }
}

// uinf[d * R + r] = sum_tile part[...]; res = uinf - data (if data)
__global__ void farfield_reduce_kernel(int ntiles, int R, int nrhs, const double2 *__restrict__ part,
                                       double2 *__restrict__ uinf, const double2 *__restrict__ data,
                                       double2 *__restrict__ res) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R * nrhs) return;
  const int d = t / R, r = t - d * R;
  double ar = 0.0, ai = 0.0;
  for (int k = 0; k < ntiles; ++k) {
    const double2 p = part[((int64_t)k * R + r) * nrhs + d];
    ar += p.x;
    ai += p.y;
  }
  uinf[t] = make_double2(ar, ai);
  if (res) res[t] = data ? make_double2(ar - data[t].x, ai - data[t].y) : make_double2(ar, ai);
}

// a_q = sum_r conj(A_rq) res_r; rhs_q = conj(m_q) a_q  (caller order, scatterer segment only)
__global__ __launch_bounds__(kBlock) void farfield_adjoint_kernel(int64_t n, int64_t off, int R, int nrhs,
                                                                  const double *__restrict__ th, double k,
                                                                  const double *__restrict__ px,
                                                                  const double *__restrict__ py,
                                                                  const double *__restrict__ w,
                                                                  const double2 *__restrict__ m,
                                                                  const int32_t *__restrict__ perm,
                                                                  const double2 *__restrict__ res, double2 *a,
                                                                  double2 *rhs, int64_t ld) {
  const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int d = blockIdx.y;
  if (q >= n) return;
  const double g = k * k / std::sqrt(8.0 * M_PI * k);
  // conj(-k^2 gamma) w_q = -(k^2/sqrt(8 pi k)) e^{-i pi/4} w_q
  const double cre = -g * M_SQRT1_2 * w[q], cim = g * M_SQRT1_2 * w[q];
  double ar = 0.0, ai = 0.0;
  for (int r = 0; r < R; ++r) {
    double s, c;
    sincos(k * (std::cos(th[r]) * px[q] + std::sin(th[r]) * py[q]), &s, &c);
    const double2 v = res[(int64_t)d * R + r];
    ar += c * v.x - s * v.y;
    ai += c * v.y + s * v.x;
  }
  const double2 av = make_double2(cre * ar - cim * ai, cre * ai + cim * ar);
  const int64_t idx = (int64_t)d * ld + off + perm[q];
  if (a) a[idx] = av;
  if (rhs) {
    const double2 mq = m[q];
    rhs[idx] = make_double2(mq.x * av.x + mq.y * av.y, mq.x * av.y - mq.y * av.x);
  }
}

__global__ void set_contrast_kernel(int64_t n, int64_t off, const int32_t *__restrict__ perm,
                                    const double2 *__restrict__ mc, double2 *__restrict__ m) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) m[i] = mc[off + perm[i]];
}

}  // namespace

size_t farfield_workspace_bytes(int64_t n, int R, int nrhs) {
  const int64_t tiles = (n + kQT - 1) / kQT;
  // partials, then (256-byte aligned, from the end) a residual buffer and the angles
  return sizeof(double2) * ((size_t)tiles * R * nrhs + 2 * (size_t)R * nrhs) + sizeof(double) * R + 2048;
}

hipError_t launch_farfield(const Scat &s, const double *u, int nrhs, int64_t ld, const double *th_dev, int R,
                           const double *data, double *uinf, double *res, void *ws, hipStream_t st) {
  const int64_t tiles = (s.n + kQT - 1) / kQT;
  double2 *part = (double2 *)ws;
  farfield_kernel<<<dim3((unsigned)R, (unsigned)tiles), kBlock, 0, st>>>(s.n, s.off, R, nrhs, th_dev, s.k, s.px, s.py,
                                                                        s.w, s.m, s.perm, (const double2 *)u, ld,
                                                                        part);
  farfield_reduce_kernel<<<(unsigned)((R * nrhs + 255) / 256), 256, 0, st>>>(
      (int)tiles, R, nrhs, part, (double2 *)uinf, (const double2 *)data, (double2 *)res);
  return hipGetLastError();
}

hipError_t launch_farfield_adjoint(const Scat &s, const double *res, int nrhs, int64_t ld, const double *th_dev,
                                   int R, double *a, double *rhs, hipStream_t st) {
  dim3 g((unsigned)((s.n + kBlock - 1) / kBlock), (unsigned)nrhs);
  farfield_adjoint_kernel<<<g, kBlock, 0, st>>>(s.n, s.off, R, nrhs, th_dev, s.k, s.px, s.py, s.w, s.m, s.perm,
                                               (const double2 *)res, (double2 *)a, (double2 *)rhs, ld);
  return hipGetLastError();
}

hipError_t launch_set_contrast(const Scat &s, const double *m_caller, hipStream_t st) {
  set_contrast_kernel<<<(unsigned)((s.n + kBlock - 1) / kBlock), kBlock, 0, st>>>(
      s.n, s.off, s.perm, (const double2 *)m_caller, s.m);
  return hipGetLastError();
}

}  // namespace lsk
