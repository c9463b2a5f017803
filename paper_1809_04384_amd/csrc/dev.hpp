// Device-side helpers shared by the HIP kernels (complex arithmetic, Chebyshev
// tables, kernel function).  gfx950, wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace dh2 {

template <typename R>
struct cpx {
  R x, y;
};
using z64 = cpx<double>;
using z32 = cpx<float>;

template <typename R>
__host__ __device__ inline cpx<R> mk(R a, R b) {
  return cpx<R>{a, b};
}
template <typename R>
__host__ __device__ inline cpx<R> operator+(cpx<R> a, cpx<R> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename R>
__host__ __device__ inline cpx<R> operator-(cpx<R> a, cpx<R> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename R>
__host__ __device__ inline cpx<R> operator*(cpx<R> a, cpx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__host__ __device__ inline cpx<R> operator*(R s, cpx<R> a) {
  return {s * a.x, s * a.y};
}
template <typename R>
__host__ __device__ inline cpx<R> conj(cpx<R> a) {
  return {a.x, -a.y};
}
// a += b * c
template <typename R>
__host__ __device__ inline void cfma(cpx<R>& a, cpx<R> b, cpx<R> c) {
  a.x += b.x * c.x - b.y * c.y;
  a.y += b.x * c.y + b.y * c.x;
}
// a += conj(b) * c
template <typename R>
__host__ __device__ inline void cfmac(cpx<R>& a, cpx<R> b, cpx<R> c) {
  a.x += b.x * c.x + b.y * c.y;
  a.y += b.x * c.y - b.y * c.x;
}
template <typename R>
__host__ __device__ inline R abs2(cpx<R> a) {
  return a.x * a.x + a.y * a.y;
}

constexpr int kMaxOrder = 8;  // Chebyshev points per axis (k = m^3 <= 512)

// Chebyshev nodes of the first kind on [-1,1] and Lagrange normalisation
// factors: L_j(x) = prod_{l != j} (x - node_l) * inv_den[j].
struct ChebTab {
  int m;
  double node[kMaxOrder];
  double inv_den[kMaxOrder];
};

// L_j(xh) for j < m at a reference coordinate xh.
template <typename R>
__device__ inline void lagrange(const ChebTab& ct, R xh, R* out) {
  for (int j = 0; j < ct.m; ++j) {
    R p = (R)ct.inv_den[j];
    for (int l = 0; l < ct.m; ++l)
      if (l != j) p *= (xh - (R)ct.node[l]);
    out[j] = p;
  }
}

// physical -> reference coordinate of one box axis; zero width -> 0
template <typename R>
__device__ inline R to_ref(R x, R lo, R hi) {
  const R half = (R)0.5 * (hi - lo);
  if (half == (R)0) return (R)0;
  return (x - (R)0.5 * (lo + hi)) / half;
}

template <typename R>
__device__ inline R axis_point(const ChebTab& ct, R lo, R hi, int j) {
  return (R)0.5 * (lo + hi) + (R)0.5 * (hi - lo) * (R)ct.node[j];
}

// sin and cos of x for |x| < 2^20: x = n pi/2 + y with n = rint(2x/pi) and pi/2
// in three parts (the first two with 33-bit significands, so n times either is
// exact for n < 2^20 and the first subtraction is exact as well); on
// |y| <= pi/4 the Taylor series of sin y to y^17 and of cos y to y^16, whose
// first omitted terms stay below 2^-56 of the value; the quadrant n mod 4
// then swaps and negates.  Outside that range: the library routine.
__device__ inline void sincos_fast(double x, double* s, double* c) {
  if (!(fabs(x) < 1048576.0)) {
    sincos(x, s, c);
    return;
  }
  constexpr double kPio2Hi = 0x1.921fb544p+0, kPio2Mid = 0x1.0b4611a6p-34, kPio2Lo = 0x1.3198a2e037073p-69;
  const double n = rint(x * 0.63661977236758134);
  double y = fma(-n, kPio2Hi, x);
  y = fma(-n, kPio2Mid, y);
  y = fma(-n, kPio2Lo, y);
  const double z = y * y;
  // sin y = y + y z (-1/3! + z (1/5! - z (1/7! - ...)))
  double ps = 2.8114572543455206e-15;            //  1/17!
  ps = fma(ps, z, -7.647163731819816e-13);       // -1/15!
  ps = fma(ps, z, 1.6059043836821613e-10);       //  1/13!
  ps = fma(ps, z, -2.505210838544172e-08);       // -1/11!
  ps = fma(ps, z, 2.7557319223985893e-06);       //  1/9!
  ps = fma(ps, z, -0.0001984126984126984);       // -1/7!
  ps = fma(ps, z, 0.008333333333333333);         //  1/5!
  ps = fma(ps, z, -0.16666666666666666);         // -1/3!
  const double sn = fma(y * z, ps, y);
  // cos y = 1 + z (-1/2! + z (1/4! - ...))
  double pc = 4.779477332387385e-14;             //  1/16!
  pc = fma(pc, z, -1.1470745597729725e-11);      // -1/14!
  pc = fma(pc, z, 2.08767569878681e-09);         //  1/12!
  pc = fma(pc, z, -2.755731922398589e-07);       // -1/10!
  pc = fma(pc, z, 2.48015873015873e-05);         //  1/8!
  pc = fma(pc, z, -0.001388888888888889);        // -1/6!
  pc = fma(pc, z, 0.041666666666666664);         //  1/4!
  pc = fma(pc, z, -0.5);                         // -1/2!
  const double cs = fma(z, pc, 1.0);
  const int q = (int)((long long)n & 3);
  const double ss = (q & 1) ? cs : sn, cc = (q & 1) ? sn : cs;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

__device__ inline void sincos_r(double a, double* s, double* c) { sincos_fast(a, s, c); }

// 1 / sqrt(a) for a > 0: the hardware estimate refined by two Newton steps
// y <- y + y (1 - a y^2) / 2 (each squares the relative error), so r = a y and
// 1 / r = y come without a square root and a division.
__device__ inline double rsqrt_r(double a) {
#if defined(__HIP_DEVICE_COMPILE__)
  double y = __builtin_amdgcn_rsq(a);
#else
  double y = 1.0 / sqrt(a);   // host compilation of this header (never called there)
#endif
  double e = fma(-a * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-a * y, y, 1.0);
  return fma(0.5 * y, e, y);
}
__device__ inline float rsqrt_r(float a) { return 1.0f / sqrtf(a); }
__device__ inline void sincos_r(float a, float* s, float* c) { sincosf(a, s, c); }
__device__ inline double sqrt_r(double a) { return sqrt(a); }
__device__ inline float sqrt_r(float a) { return sqrtf(a); }

}  // namespace dh2
