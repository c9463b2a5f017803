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

__device__ inline void sincos_r(double a, double* s, double* c) { sincos(a, s, c); }
__device__ inline void sincos_r(float a, float* s, float* c) { sincosf(a, s, c); }
__device__ inline double sqrt_r(double a) { return sqrt(a); }
__device__ inline float sqrt_r(float a) { return sqrtf(a); }

}  // namespace dh2
