// Energy densities psi(e) written once, generically in the scalar type, so the
// same source gives psi (S = double), the stress (S = Dual<double, C>) and the
// incremental stress K : d_e (S = Dual<Dual<double, 1>, C>).
//
// Packed strain e (C components):
//   small strain, Mandel: 3D [e11, e22, e33, sqrt2 e23, sqrt2 e13, sqrt2 e12],
//                          2D [e11, e22, sqrt2 e12]  (plane strain, e33 = 0);
//     with this packing the tensor product e:s is the plain dot product, so
//     d psi / d e_k is the Mandel-packed stress.
//   finite strain: deformation gradient F row-major (2D: 2x2, plane strain F33 = 1);
//     d psi / d F_k is the first Piola-Kirchhoff stress P.
//
// Energies (the paper's section 3.1 / 4.1.1 forms; the Neo-Hookean law is the
// standard compressible one, not written out in the paper):
//   linear elastic      psi = lam/2 tr(eps)^2 + mu eps:eps
//   Neo-Hookean         psi = mu/2 (tr(F^T F) - 3) - mu ln J + lam/2 (ln J)^2
//   St.Venant-Kirchhoff psi = lam/2 tr(E)^2 + mu E:E,  E = (F^T F - I)/2
#pragma once

#include "dual.h"

namespace fh {

enum { MAT_LE = 0, MAT_NH = 1, MAT_STVK = 2 };

template <int MAT, int NDIM>
struct MatTraits;
template <> struct MatTraits<MAT_LE, 2> { static constexpr int C = 3; };
template <> struct MatTraits<MAT_LE, 3> { static constexpr int C = 6; };
template <> struct MatTraits<MAT_NH, 2> { static constexpr int C = 4; };
template <> struct MatTraits<MAT_NH, 3> { static constexpr int C = 9; };
template <> struct MatTraits<MAT_STVK, 2> { static constexpr int C = 4; };
template <> struct MatTraits<MAT_STVK, 3> { static constexpr int C = 9; };

template <int MAT, int NDIM, class S>
struct Energy;

// ---- small strain, linear elastic -------------------------------------------
template <class S>
struct Energy<MAT_LE, 3, S> {
  __device__ static S psi(const S* e, double lam, double mu) {
    S tr = e[0] + e[1] + e[2];
    S ee = e[0] * e[0] + e[1] * e[1] + e[2] * e[2] + e[3] * e[3] + e[4] * e[4] + e[5] * e[5];
    return (0.5 * lam) * (tr * tr) + mu * ee;
  }
};

template <class S>
struct Energy<MAT_LE, 2, S> {
  __device__ static S psi(const S* e, double lam, double mu) {
    S tr = e[0] + e[1];
    S ee = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
    return (0.5 * lam) * (tr * tr) + mu * ee;
  }
};

// ---- finite strain, compressible Neo-Hookean ---------------------------------
template <class S>
struct Energy<MAT_NH, 3, S> {
  __device__ static S psi(const S* F, double lam, double mu) {
    S J = F[0] * (F[4] * F[8] - F[5] * F[7]) + F[1] * (F[5] * F[6] - F[3] * F[8]) +
          F[2] * (F[3] * F[7] - F[4] * F[6]);
    S I1 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2] + F[3] * F[3] + F[4] * F[4] + F[5] * F[5] +
           F[6] * F[6] + F[7] * F[7] + F[8] * F[8];
    S lnJ = dlog(J);
    return (0.5 * mu) * (I1 - 3.0) - mu * lnJ + (0.5 * lam) * (lnJ * lnJ);
  }
};

template <class S>
struct Energy<MAT_NH, 2, S> {
  __device__ static S psi(const S* F, double lam, double mu) {
    S J = F[0] * F[3] - F[1] * F[2];
    S I1 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2] + F[3] * F[3];  // + F33^2 = 1
    S lnJ = dlog(J);
    return (0.5 * mu) * (I1 - 2.0) - mu * lnJ + (0.5 * lam) * (lnJ * lnJ);
  }
};

// ---- finite strain, St. Venant-Kirchhoff --------------------------------------
template <class S>
struct Energy<MAT_STVK, 3, S> {
  __device__ static S psi(const S* F, double lam, double mu) {
    // E = (F^T F - I)/2 ; F row-major: F[3*i + J]
    S E00 = 0.5 * (F[0] * F[0] + F[3] * F[3] + F[6] * F[6] - 1.0);
    S E11 = 0.5 * (F[1] * F[1] + F[4] * F[4] + F[7] * F[7] - 1.0);
    S E22 = 0.5 * (F[2] * F[2] + F[5] * F[5] + F[8] * F[8] - 1.0);
    S E01 = 0.5 * (F[0] * F[1] + F[3] * F[4] + F[6] * F[7]);
    S E02 = 0.5 * (F[0] * F[2] + F[3] * F[5] + F[6] * F[8]);
    S E12 = 0.5 * (F[1] * F[2] + F[4] * F[5] + F[7] * F[8]);
    S tr = E00 + E11 + E22;
    S EE = E00 * E00 + E11 * E11 + E22 * E22 + 2.0 * (E01 * E01 + E02 * E02 + E12 * E12);
    return (0.5 * lam) * (tr * tr) + mu * EE;
  }
};

template <class S>
struct Energy<MAT_STVK, 2, S> {
  __device__ static S psi(const S* F, double lam, double mu) {
    S E00 = 0.5 * (F[0] * F[0] + F[2] * F[2] - 1.0);
    S E11 = 0.5 * (F[1] * F[1] + F[3] * F[3] - 1.0);
    S E01 = 0.5 * (F[0] * F[1] + F[2] * F[3]);
    S tr = E00 + E11;
    S EE = E00 * E00 + E11 * E11 + 2.0 * (E01 * E01);
    return (0.5 * lam) * (tr * tr) + mu * EE;
  }
};

// ---- derivatives by forward-mode AD -------------------------------------------

// psi and its gradient (the stress) at e: one vector-dual pass.
template <int MAT, int NDIM>
__device__ inline double stress_ad(const double* e, double lam, double mu, double* P) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  Dual<double, C> x[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    x[k].v = e[k];
#pragma unroll
    for (int j = 0; j < C; ++j) x[k].d[j] = (j == k) ? 1.0 : 0.0;
  }
  Dual<double, C> r = Energy<MAT, NDIM, Dual<double, C>>::psi(x, lam, mu);
#pragma unroll
  for (int k = 0; k < C; ++k) P[k] = r.d[k];
  return r.v;
}

// K(e) : de, the Jacobian-vector product of the stress, by forward over forward.
template <int MAT, int NDIM>
__device__ inline void tangent_jvp_ad(const double* e, const double* de, double lam, double mu,
                                      double* out) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  typedef Dual<double, 1> T;
  Dual<T, C> x[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    x[k].v.v = e[k];
    x[k].v.d[0] = de[k];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      x[k].d[j].v = (j == k) ? 1.0 : 0.0;
      x[k].d[j].d[0] = 0.0;
    }
  }
  Dual<T, C> r = Energy<MAT, NDIM, Dual<T, C>>::psi(x, lam, mu);
#pragma unroll
  for (int k = 0; k < C; ++k) out[k] = r.d[k].d[0];
}

// Same product, one input direction at a time: for each k, a hyper-dual pass
// seeded with e_k (outer level) and de (inner level) gives (K : de)_k as the
// mixed second derivative of psi.  C cheap passes over 4-double numbers
// instead of one pass over 2(C+1)-double numbers: fewer live registers.
template <int MAT, int NDIM>
__device__ inline void tangent_jvp_ad_dirs(const double* e, const double* de, double lam, double mu,
                                           double* out) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  typedef Dual<double, 1> T;
  typedef Dual<T, 1> S;
#pragma unroll
  for (int k = 0; k < C; ++k) out[k] = 0.0;
#pragma unroll 1
  for (int k = 0; k < C; ++k) {
    S x[C];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      x[j].v.v = e[j];
      x[j].v.d[0] = de[j];
      x[j].d[0].v = (j == k) ? 1.0 : 0.0;
      x[j].d[0].d[0] = 0.0;
    }
    const S r = Energy<MAT, NDIM, S>::psi(x, lam, mu);
    const double val = r.d[0].d[0];
#pragma unroll
    for (int j = 0; j < C; ++j)
      if (j == k) out[j] = val;
  }
}

// Stress and K : de together (same nested pass; the stress is in the partials' values).
template <int MAT, int NDIM>
__device__ inline double stress_and_jvp_ad(const double* e, const double* de, double lam, double mu,
                                           double* P, double* KdE) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  typedef Dual<double, 1> T;
  Dual<T, C> x[C];
#pragma unroll
  for (int k = 0; k < C; ++k) {
    x[k].v.v = e[k];
    x[k].v.d[0] = de[k];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      x[k].d[j].v = (j == k) ? 1.0 : 0.0;
      x[k].d[j].d[0] = 0.0;
    }
  }
  Dual<T, C> r = Energy<MAT, NDIM, Dual<T, C>>::psi(x, lam, mu);
#pragma unroll
  for (int k = 0; k < C; ++k) {
    P[k] = r.d[k].v;
    KdE[k] = r.d[k].d[0];
  }
  return r.v.v;
}

// Determinant of the packed deformation gradient (finite strain domain check).
template <int NDIM>
__device__ inline double det_packed(const double* F);
template <>
__device__ inline double det_packed<3>(const double* F) {
  return F[0] * (F[4] * F[8] - F[5] * F[7]) + F[1] * (F[5] * F[6] - F[3] * F[8]) +
         F[2] * (F[3] * F[7] - F[4] * F[6]);
}
template <>
__device__ inline double det_packed<2>(const double* F) { return F[0] * F[3] - F[1] * F[2]; }

}  // namespace fh
