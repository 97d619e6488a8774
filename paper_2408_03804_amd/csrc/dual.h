// Forward-mode automatic differentiation with dual numbers, usable in HIP kernels.
//
// The paper (section 2) differentiates energy densities by automatic
// differentiation: the stress is the gradient of psi (section 3.1) and the
// incremental stress K : d_eps is a Jacobian-vector product of the stress
// (section 3.2).  Here both come from forward mode:
//
//   Dual<double, C>               value + C partials: one pass gives psi and the
//                                 full gradient (stress) of psi(e_1..e_C);
//   Dual<Dual<double, 1>, C>      forward over forward: seeding the inner level
//                                 with the direction d_eps gives, in the partials'
//                                 inner tangents, the directional derivative of
//                                 the gradient, i.e. K : d_eps, without forming K.
//
// Arithmetic is the plain chain rule; nothing is approximated.
#pragma once

#include <hip/hip_runtime.h>

namespace fh {

template <class T, int K>
struct Dual {
  T v;
  T d[K];
};

// Lifting a double into a (possibly nested) dual: zero partials at every level.
template <class S>
struct Lift;

template <>
struct Lift<double> {
  __host__ __device__ static double from(double a) { return a; }
};

template <class T, int K>
struct Lift<Dual<T, K>> {
  __host__ __device__ static Dual<T, K> from(double a) {
    Dual<T, K> r;
    r.v = Lift<T>::from(a);
    for (int k = 0; k < K; ++k) r.d[k] = Lift<T>::from(0.0);
    return r;
  }
};

template <class S>
__host__ __device__ inline S lift(double a) { return Lift<S>::from(a); }

// ---- arithmetic -------------------------------------------------------------
template <class T, int K>
__host__ __device__ inline Dual<T, K> operator+(const Dual<T, K>& a, const Dual<T, K>& b) {
  Dual<T, K> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}

template <class T, int K>
__host__ __device__ inline Dual<T, K> operator-(const Dual<T, K>& a, const Dual<T, K>& b) {
  Dual<T, K> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}

template <class T, int K>
__host__ __device__ inline Dual<T, K> operator-(const Dual<T, K>& a) {
  Dual<T, K> r;
  r.v = -a.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}

template <class T, int K>
__host__ __device__ inline Dual<T, K> operator*(const Dual<T, K>& a, const Dual<T, K>& b) {
  Dual<T, K> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.v * b.d[k] + a.d[k] * b.v;
  return r;
}

template <class T, int K>
__host__ __device__ inline Dual<T, K> operator/(const Dual<T, K>& a, const Dual<T, K>& b) {
  Dual<T, K> r;
  const T inv = lift<T>(1.0) / b.v;
  r.v = a.v * inv;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * inv;
  return r;
}

// mixed with plain doubles
template <class T, int K>
__host__ __device__ inline Dual<T, K> operator*(double s, const Dual<T, K>& a) {
  Dual<T, K> r;
  r.v = s * a.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = s * a.d[k];
  return r;
}

template <class T, int K>
__host__ __device__ inline Dual<T, K> operator*(const Dual<T, K>& a, double s) { return s * a; }

template <class T, int K>
__host__ __device__ inline Dual<T, K> operator+(const Dual<T, K>& a, double s) {
  Dual<T, K> r = a;
  r.v = a.v + s;
  return r;
}

template <class T, int K>
__host__ __device__ inline Dual<T, K> operator+(double s, const Dual<T, K>& a) { return a + s; }

template <class T, int K>
__host__ __device__ inline Dual<T, K> operator-(const Dual<T, K>& a, double s) {
  Dual<T, K> r = a;
  r.v = a.v - s;
  return r;
}

template <class T, int K>
__host__ __device__ inline Dual<T, K> operator-(double s, const Dual<T, K>& a) {
  Dual<T, K> r;
  r.v = s - a.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}

// ---- elementary functions ---------------------------------------------------
// value part at the innermost level (branch decisions are taken on it)
__host__ __device__ inline double val(double a) { return a; }
template <class T, int K>
__host__ __device__ inline double val(const Dual<T, K>& a) { return val(a.v); }

__host__ __device__ inline double dsqrt(double a) { return sqrt(a); }

template <class T, int K>
__host__ __device__ inline Dual<T, K> dsqrt(const Dual<T, K>& a) {
  Dual<T, K> r;
  r.v = dsqrt(a.v);
  const T h = lift<T>(0.5) / r.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * h;
  return r;
}

__host__ __device__ inline double dexp(double a) { return exp(a); }

template <class T, int K>
__host__ __device__ inline Dual<T, K> dexp(const Dual<T, K>& a) {
  Dual<T, K> r;
  r.v = dexp(a.v);
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * r.v;
  return r;
}

__host__ __device__ inline double dlog(double a) { return log(a); }

template <class T, int K>
__host__ __device__ inline Dual<T, K> dlog(const Dual<T, K>& a) {
  Dual<T, K> r;
  r.v = dlog(a.v);
  const T inv = lift<T>(1.0) / a.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * inv;
  return r;
}

}  // namespace fh
