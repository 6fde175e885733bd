// In-register evaluation of the 2-D Helmholtz Green's function G = (i/4) H0^(1)(z).
//
// The Green's function is the one of the paper's Section 2 (after eq. Lippmann-Schwinger).
// Inputs are z^2 = k^2 |x - y|^2 (never z itself: the small-argument branch needs no square
// root and the others get z, 1/z and z^(-1/2) from one inverse fourth root).  Branches:
//   z <  ZS : power series of J0 and of Y0 - (2/pi) ln(z/2) J0 in u = z^2/4, own ln;
//   ZS <= z < ZF : modulus-phase form H0 = M e^{i theta} with two fitted intervals in 1/z;
//   z >= ZF : modulus-phase form from the even/odd Hankel asymptotic structure in 1/z.
// e^{i theta} uses a reduction modulo pi (two-constant Cody-Waite with FMA) and minimax
// sine/cosine on [-pi/2, pi/2], the parity of the multiple of pi flipping the sign; or, in the
// kernels that keep a 512-entry table of e^{i j pi/256} in LDS, a reduction modulo pi/256, one
// table entry and short series of the remainder.
// All coefficients are produced by gen_hankel_tables.py and passed in as one HankelTable, so a
// kernel can keep them in memory read through the scalar data path instead of pinning ~130
// doubles in vector registers.  Functions are host+device so the same arithmetic can be
// checked on a CPU; on the device the initial inverse fourth root comes from the
// single-precision hardware approximations and one Halley step.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "hankel_tables.h"

namespace lsk {

// r * x + c with c a wave-uniform coefficient.  On the device the coefficient stays in its
// SGPR pair as the third operand of a VOP3 FMA; left to itself the compiler prefers the
// two-address FMAC form, which first copies every coefficient into a vector register.
__host__ __device__ __forceinline__ double fma_uniform(double r, double x, double c) {
#ifdef __HIP_DEVICE_COMPILE__
  double out;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(out) : "v"(r), "v"(x), "s"(c));
  return out;
#else
  return std::fma(r, x, c);
#endif
}

// x + c (or c - x with NEG) with c wave-uniform, kept as a separate add so the compiler does not
// contract it with the product that formed x (that FMA would need c copied into a VGPR).
template <bool NEG = false>
__host__ __device__ __forceinline__ double add_uniform(double x, double c) {
#ifdef __HIP_DEVICE_COMPILE__
  double out;
  if (NEG)
    asm("v_add_f64 %0, %2, -%1" : "=v"(out) : "v"(x), "s"(c));
  else
    asm("v_add_f64 %0, %1, %2" : "=v"(out) : "v"(x), "s"(c));
  return out;
#else
  return NEG ? c - x : x + c;
#endif
}

// Horner evaluation, constant term first.  Arr is a double[N] member of a table that may live
// in any address space (the kernels read it from the constant address space).
template <class Arr>
__host__ __device__ __forceinline__ double horner(const Arr &c, double x) {
  constexpr int N = (int)(sizeof(Arr) / sizeof(double));
  double r = c[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) r = fma_uniform(r, x, c[i]);
  return r;
}

// Horner evaluation of q[0] + q[1] x + ... + q[N-1] x^(N-1) + (+-1) x^N: the leading
// coefficient is +1 (or -1 with NEG), so the chain starts with one add of a scalar operand.
template <bool NEG = false, class Arr>
__host__ __device__ __forceinline__ double horner_lead1(const Arr &q, double x) {
  constexpr int N = (int)(sizeof(Arr) / sizeof(double));
  double r = add_uniform<NEG>(x, q[N - 1]);
#pragma unroll
  for (int i = N - 2; i >= 0; --i) r = fma_uniform(r, x, q[i]);
  return r;
}

// s = A^(-1/4), accurate to about one rounding.
template <class Tab>
__host__ __device__ __forceinline__ double inv_fourth_root(double A, const Tab &T) {
#ifdef __HIP_DEVICE_COMPILE__
  const float af = (float)A;
  double s = (double)__builtin_amdgcn_rsqf(__builtin_amdgcn_sqrtf(af));
#else
  double s = 1.0 / std::sqrt(std::sqrt(A));
#endif
  // Halley-type step for (1 - e)^(-1/4) with e = 1 - A s^4: s (1 + e/4 + 5 e^2/32)
  const double s2 = s * s;
  const double e = std::fma(-A, s2 * s2, 1.0);
  const double p = std::fma(e, T.consts[6], 0.25);
  return std::fma(s * e, p, s);
}

__host__ __device__ __forceinline__ double rint_d(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_rint(x);
#else
  return std::nearbyint(x);
#endif
}

__host__ __device__ __forceinline__ double fract_d(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_fract(x);
#else
  return x - std::floor(x);
#endif
}

__host__ __device__ __forceinline__ double rcp_d(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  double y = __builtin_amdgcn_rcp(x);
  double e = std::fma(-x, y, 1.0);
  y = std::fma(y, e, y);
  e = std::fma(-x, y, 1.0);
  return std::fma(y, e, y);
#else
  return 1.0 / x;
#endif
}

// natural logarithm of a positive normal double
template <class Tab>
__host__ __device__ __forceinline__ double log_d(double u, const Tab &T) {
#ifdef __HIP_DEVICE_COMPILE__
  double m = __builtin_amdgcn_frexp_mant(u);   // [0.5, 1)
  int e = __builtin_amdgcn_frexp_exp(u);
#else
  int e;
  double m = std::frexp(u, &e);
#endif
  const bool lo = m < T.consts[4];
  m = lo ? m + m : m;
  e = lo ? e - 1 : e;
  const double s = (m - 1.0) * rcp_d(m + 1.0);
  const double s2 = s * s;
  const double lm = 2.0 * s * horner(T.log_p, s2);
  return std::fma((double)e, T.consts[3], lm);
}

// m with its sign flipped when the integer j = jm - RND_MAGIC is odd.  jm = x + RND_MAGIC is
// x rounded to an integer (|x| < 2^51) sitting in the low mantissa bits, so its lowest bit is
// the parity of j (RND_MAGIC = 1.5 * 2^52 is even).
__host__ __device__ __forceinline__ double flip_if_odd(double m, double jm) {
#ifdef __HIP_DEVICE_COMPILE__
  const unsigned lo = (unsigned)__double_as_longlong(jm);
  const long long b = __double_as_longlong(m) ^ ((long long)(lo << 31) << 32);
  return __longlong_as_double(b);
#else
  long long bj, bm;
  std::memcpy(&bj, &jm, 8);
  std::memcpy(&bm, &m, 8);
  bm ^= (long long)((unsigned long long)(bj & 1) << 63);
  double out;
  std::memcpy(&out, &bm, 8);
  return out;
#endif
}

constexpr double RND_MAGIC = 6755399441055744.0;   // 1.5 * 2^52

// (gre, gim) = Mu e^{i theta} rotated by i, theta = zp = z + ph, Mu = |H0| / (4K).  The
// multiple j of pi nearest to theta is removed with a two-constant Cody-Waite reduction (exact
// products in the FMAs); (-1)^j flips the sign of the modulus.
template <class Tab>
__host__ __device__ __forceinline__ void phase_tail(double zp, double Mu, double &gre, double &gim,
                                                    const Tab &T) {
  const double jm = std::fma(zp, T.consts[2], RND_MAGIC);
  const double jf = jm - RND_MAGIC;
  double r = std::fma(-jf, T.consts[0], zp);
  r = std::fma(-jf, T.consts[1], r);
  const double Ms = flip_if_odd(Mu, jm);
  const double r2 = r * r;
  // sin r = c8 (sigma r) q_s(r^2), cos r = c8 q_c(r^2); c8 is part of K
  const double sn = (r * T.consts[9]) * horner_lead1(T.sin_q, r2);
  const double cs = horner_lead1(T.cos_q, r2);
  // G/K = i Mu (cos + i sin) = -Mu sin + i Mu cos
  gre = -(Ms * sn);
  gim = Ms * cs;
}

// x c + v with c wave-uniform (an SGPR pair) and v a loop-invariant vector register: a VOP3 FMA
// may read one scalar operand only.
__host__ __device__ __forceinline__ double fma_uniform_v(double x, double c, double v) {
#ifdef __HIP_DEVICE_COMPILE__
  double out;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(out) : "v"(x), "s"(c), "v"(v));
  return out;
#else
  return std::fma(x, c, v);
#endif
}

// x c - 1/2 with c wave-uniform: -0.5 is an inline constant of the instruction encoding, so the
// FMA needs no register for it.
__host__ __device__ __forceinline__ double fma_uniform_mhalf(double x, double c) {
#ifdef __HIP_DEVICE_COMPILE__
  double out;
  asm("v_fma_f64 %0, %1, %2, -0.5" : "=v"(out) : "v"(x), "s"(c));
  return out;
#else
  return std::fma(x, c, -0.5);
#endif
}

// The LDS copy of kSinCosTable, and -1/6 (the cubic coefficient of sin r below) in a vector
// register: a VOP3 FMA may read only one scalar operand, and a value the compiler knows to be a
// constant it copies from its SGPR again inside every loop.
struct PhaseLds {
  const double2 *e;
  double m6;
};

// The same result by a table: theta = j pi/256 + r with |r| <= pi/512, SC[j mod 512] =
// e^{i j pi/256}/c8 (kSinCosTable, copied by the kernels into LDS with load_sincos) rotated by
// e^{i r} - 1: sin r = r + r^3 (r^2/120 - 1/6) and cos r - 1 = r^2 (c4 r^2 - 1/2), c4 the minimax
// coefficient on |r| <= pi/512 (tail_k; truncation below 1e-17).  jm's low mantissa bits hold j
// (RND_MAGIC has none set).
template <class Tab>
__host__ __device__ __forceinline__ void phase_tail_table(double zp, double Mu, double &gre, double &gim,
                                                          const Tab &T, const PhaseLds &SC) {
  const double jm = std::fma(zp, T.tail_k[0], RND_MAGIC);
  const double jf = jm - RND_MAGIC;
  double r = std::fma(-jf, T.tail_k[1], zp);
  r = std::fma(-jf, T.tail_k[2], r);
  unsigned long long bits;
  std::memcpy(&bits, &jm, sizeof bits);
  const double2 e = SC.e[(unsigned)bits & (SINCOS_N - 1)];
  const double r2 = r * r;
  const double sr = std::fma(r2 * r, fma_uniform_v(r2, T.tail_k[3], SC.m6), r);   // sin r
  const double cm = r2 * fma_uniform_mhalf(r2, T.tail_k[5]);                   // cos r - 1
  const double C = std::fma(e.x, cm, std::fma(-e.y, sr, e.x));
  const double S = std::fma(e.y, cm, std::fma(e.x, sr, e.y));
  // G/K = i Mu (C + i S)
  gre = -(Mu * S);
  gim = Mu * C;
}

// Copies the table of phase_tail_table into the workgroup's LDS array lds[SINCOS_N] (all threads
// of the block take part; the barrier makes it visible to every wavefront) and returns it with
// -1/6 placed in a vector register once per kernel (the empty asm hides the value from the
// compiler, so it stays in that register).
__device__ __forceinline__ PhaseLds load_sincos(double2 *lds, const SinCosTable &t) {
  for (int i = threadIdx.x; i < SINCOS_N; i += blockDim.x) lds[i] = make_double2(t.v[2 * i], t.v[2 * i + 1]);
  __syncthreads();
  double m6 = kHankelTable.tail_k[4];
  asm volatile("" : "+v"(m6));
  return PhaseLds{lds, m6};
}

// The same object over a host copy of the table (host evaluation of the same arithmetic).
inline PhaseLds host_phase_lds(const double2 *table) { return PhaseLds{table, kHankelTable.tail_k[4]}; }

// ZS <= z: modulus-phase form.  Only the two polynomials depend on the argument range; the
// inverse fourth root, the reduction and the sine/cosine are shared, so a wavefront whose lanes
// straddle a range boundary repeats only the polynomial evaluation.  Returns G/K.
template <bool TBL = false, class Tab>
__host__ __device__ __forceinline__ void green_modphase(double A, double &gre, double &gim, const Tab &T,
                                                        const PhaseLds &SC = PhaseLds{}) {
  const double s = inv_fourth_root(A, T);  // z^(-1/2)
  const double t = s * s;                  // 1/z
  double mod, ph;                          // M sqrt(z) / (4 m8), theta - z
  if (A >= ZF2) {
    const double t2 = t * t;
    mod = horner_lead1(T.far_mod_q, t2);
    ph = std::fma(t * T.consts[8], horner_lead1(T.far_ph_q, t2), T.consts[5]);
  } else if (A >= ZM2) {
    const double x = t - MID2_TA;
    mod = horner_lead1<MID2_MOD_NEG>(T.mid2_mod_q, x * MID2_SM);
    ph = horner_lead1<MID2_PH_NEG>(T.mid2_ph_q, x * MID2_SP);
  } else {
    const double x = t - MID1_TA;
    mod = horner_lead1<MID1_MOD_NEG>(T.mid1_mod_q, x * MID1_SM);
    ph = horner_lead1<MID1_PH_NEG>(T.mid1_ph_q, x * MID1_SP);
  }
  // z + ph = A t + ph in one rounding, the same error as z = A t alone
  if constexpr (TBL)
    phase_tail_table(std::fma(A, t, ph), mod * s, gre, gim, T, SC);
  else
    phase_tail(std::fma(A, t, ph), mod * s, gre, gim, T);
}

// 0 < z < ZS; returns G/K
template <class Tab>
__host__ __device__ __forceinline__ void green_small(double A, double &gre, double &gim, const Tab &T) {
  const double u = 0.25 * A;
  const double j4 = horner(T.small_j_k, u);  // J0/(4K)
  const double r4 = horner(T.small_r_k, u);  // (Y0 - ln(u) J0 / pi)/(4K)
  const double L = log_d(u, T);
  // G = (i/4)(J0 + i Y0) = -Y0/4 + i J0/4
  gre = -std::fma(T.consts[2] * L, j4, r4);
  gim = j4;
}

// G/K for z^2 = A > 0 (any branch), K = G_SCALE.  The far sums accumulate G/K and multiply
// the total by K once.
// TBL: e^{i theta} from the table SC (phase_tail_table) instead of the polynomials.
template <bool TBL = false, class Tab>
__host__ __device__ __forceinline__ void green_unit(double A, double &gre, double &gim, const Tab &T,
                                                    const PhaseLds &SC = PhaseLds{}) {
  if (A >= ZS2) {
    green_modphase<TBL>(A, gre, gim, T, SC);
  } else {
    green_small(A, gre, gim, T);
  }
}

// G = (i/4) H0^(1)(z) for z^2 = A > 0
template <bool TBL = false, class Tab>
__host__ __device__ __forceinline__ void green(double A, double &gre, double &gim, const Tab &T,
                                               const PhaseLds &SC = PhaseLds{}) {
  green_unit<TBL>(A, gre, gim, T, SC);
  gre *= T.consts[7];
  gim *= T.consts[7];
}

// ---------------------------------------------------------------- single precision
// For the mixed-precision tiles: G/K with z >= 1 in FP32 (far form for z >= F32_ZF, one
// fitted modulus-phase interval below), e^{i theta} from the hardware sine/cosine of the
// fractional number of turns; z < 1 falls back to the FP64 series (its logarithm needs the
// precision).  The phase is reduced in FP64 (z refined by one Newton step), so the relative
// accuracy stays at the FP32 level (a few 1e-7) for every z.
template <class Arr>
__host__ __device__ __forceinline__ float hornerf(const Arr &c, float x) {
  constexpr int N = (int)(sizeof(Arr) / sizeof(float));
  float r = c[N - 1];
#pragma unroll
  for (int i = N - 2; i >= 0; --i) r = std::fma(r, x, c[i]);
  return r;
}

// A polynomial's coefficients times a constant factor, rounded to FP32 at compile time.
template <int N>
struct F32Poly {
  float c[N];
  __host__ __device__ constexpr float operator[](int i) const { return c[i]; }
};
template <int N>
constexpr F32Poly<N> f32_scaled(const float (&a)[N], double f) {
  F32Poly<N> r{};
  for (int i = 0; i < N; ++i) r.c[i] = (float)((double)a[i] * f);
  return r;
}
// H16: return 256 G instead of G/K (the split-FP16 tiles' scale), by modulus polynomials that carry
// the factor 256 K; the extra rounding of the coefficients is 2^-24 relative.
constexpr double H16_GSCALE = 256.0 * G_SCALE;
constexpr F32Poly<4> F32_FAR_MOD_H16 = f32_scaled(F32_FAR_MOD, H16_GSCALE);
constexpr F32Poly<11> F32_MID_MOD_H16 = f32_scaled(F32_MID_MOD, H16_GSCALE);
// The phase polynomials in turns (radians / 2 pi), so that the phase joins the FP64 number of turns
// without a multiplication; the far form's constant -pi/4 is -1/8 turn.
constexpr double F32_INV_2PI = 0.15915494309189535;
constexpr F32Poly<4> F32_FAR_PH_TURNS = f32_scaled(F32_FAR_PH, F32_INV_2PI);
constexpr F32Poly<9> F32_MID_PH_TURNS = f32_scaled(F32_MID_PH, F32_INV_2PI);

// excl_small: pairs with z < 1 give 0 (the caller adds them in FP64 through a sparse near part)
template <bool H16 = false, class Tab>
__host__ __device__ __forceinline__ void green32_unit(double A, float &gre, float &gim, const Tab &T,
                                                      bool excl_small = false) {
  if (A < 1.0) {
    if (excl_small) {
      gre = 0.f;
      gim = 0.f;
      return;
    }
    double r, i;
    green_small(A, r, i, T);
    if (H16) {
      r *= H16_GSCALE;
      i *= H16_GSCALE;
    }
    gre = (float)r;
    gim = (float)i;
    return;
  }
  const float a = (float)A;
#ifdef __HIP_DEVICE_COMPILE__
  const float s = __builtin_amdgcn_rsqf(__builtin_amdgcn_sqrtf(a));  // z^(-1/2)
#else
  const float s = 1.0f / std::sqrt(std::sqrt(a));
#endif
  const float t = s * s, z = a * t;
  float mod, ph;   // ph in turns
  if (a >= F32_ZF * F32_ZF) {
    const float t2 = t * t;
    if constexpr (H16)
      mod = hornerf(F32_FAR_MOD_H16, t2);
    else
      mod = hornerf(F32_FAR_MOD, t2);
    ph = std::fma(t, hornerf(F32_FAR_PH_TURNS, t2), -0.125f);
  } else {
    const float x = (t - F32_MID_TA) * F32_MID_SCALE;
    if constexpr (H16)
      mod = hornerf(F32_MID_MOD_H16, x);
    else
      mod = hornerf(F32_MID_MOD, x);
    ph = hornerf(F32_MID_PH_TURNS, x);
  }
  const float m4 = mod * s;
  // Phase in FP64: z in FP32 carries a relative error ~2^-24, i.e. ~z 2^-24 radians of phase.
  // One Newton step for sqrt(A) from the FP32 z restores z to ~1e-14 relative, and the number of
  // turns (z + ph)/(2 pi) is reduced in FP64; only the fraction goes to the FP32 sine/cosine.
  const double zd = (double)z;
  const double z64 = std::fma(std::fma(-zd, zd, A), (double)(0.5f * t), zd);
  const double rev = std::fma(z64, F32_INV_2PI, (double)ph);   // turns
#ifdef __HIP_DEVICE_COMPILE__
  const float f = (float)__builtin_amdgcn_fract(rev);
  const float sn = __builtin_amdgcn_sinf(f), cs = __builtin_amdgcn_cosf(f);
#else
  const float f = (float)(rev - std::floor(rev));
  const float sn = std::sin(6.283185307f * f), cs = std::cos(6.283185307f * f);
#endif
  gre = -m4 * sn;
  gim = m4 * cs;
}

}  // namespace lsk
