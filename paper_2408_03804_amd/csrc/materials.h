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
//
// J2 plasticity (small strain, linear isotropic hardening) has no energy whose
// derivative is the stress: its stress is the predictor-corrector return mapping
// of the paper's Appendix B, written once generically in the scalar type, and
// K : d_e is the forward-mode derivative of that function along d_e (the paper's
// jvp of its stress update).
#pragma once

#include "dual.h"

namespace fh {

// MAT_NH_PS, MAT_J2_PS: Neo-Hookean and J2 plasticity under plane stress (2D only)
enum { MAT_LE = 0, MAT_NH = 1, MAT_STVK = 2, MAT_J2 = 3, MAT_NH_PS = 4, MAT_J2_PS = 5 };

// J2 plasticity: per-voxel yield parameters and plastic history
constexpr bool j2_mat(int mat) { return mat == MAT_J2 || mat == MAT_J2_PS; }

// finite strain: the packed strain is a deformation gradient, whose determinant must stay positive
constexpr bool finite_mat(int mat) { return mat == MAT_NH || mat == MAT_STVK || mat == MAT_NH_PS; }

// Parameters and state of one voxel: Lame parameters, and for J2 the yield stress,
// hardening modulus and plastic history (packed plastic strain, cumulative plastic strain)
// of the last committed load step.
struct Local {
  double lam, mu;
  double sy, H;
  double hist[7];
};

template <int MAT, int NDIM>
struct MatTraits;
template <> struct MatTraits<MAT_J2, 2> { static constexpr int C = 3; };
template <> struct MatTraits<MAT_J2, 3> { static constexpr int C = 6; };
template <> struct MatTraits<MAT_LE, 2> { static constexpr int C = 3; };
template <> struct MatTraits<MAT_LE, 3> { static constexpr int C = 6; };
template <> struct MatTraits<MAT_NH, 2> { static constexpr int C = 4; };
template <> struct MatTraits<MAT_NH, 3> { static constexpr int C = 9; };
template <> struct MatTraits<MAT_STVK, 2> { static constexpr int C = 4; };
template <> struct MatTraits<MAT_STVK, 3> { static constexpr int C = 9; };
template <> struct MatTraits<MAT_NH_PS, 2> { static constexpr int C = 4; };
template <> struct MatTraits<MAT_J2_PS, 2> { static constexpr int C = 3; };

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

// ---- finite strain, Neo-Hookean under plane stress (2D) ------------------------
// The 2D gradient F2 is completed to F = [[F2, 0], [0, F33]] with F33 = e^t chosen so that P33 of
// the 3D law vanishes (the out-of-plane shear stresses vanish by isotropy).  With J2 = det F2,
//   g(t) = F33 P33 = mu e^{2t} + lam (ln J2 + t) - mu,
// which for lam >= 0, mu > 0 is increasing and convex in t: Newton's method from t = 0 converges
// from either side of the root (after the first step the iterates fall monotonically onto it).
// Stress and energy are the 3D law's at that F.  The energy is stationary in F33, so P needs only
// the value of t; its derivative along dF2 needs dt = -lam (dJ2 / J2) / g'(t), which one Newton
// step taken in the dual type from the converged root gives exactly (g = 0 there).  Returns psi.
template <class T>
__device__ inline T nh_plane_stress(const T* F, double lam, double mu, T* P) {
  const T J2 = F[0] * F[3] - F[1] * F[2];
  const T lnJ2 = dlog(J2);
  const double l2 = val(lnJ2);
  double t = 0.0;
  for (int it = 0; it < 64; ++it) {
    const double e2 = exp(2.0 * t);
    const double dt = (mu * e2 + lam * (l2 + t) - mu) / (2.0 * mu * e2 + lam);
    t -= dt;
    if (!(fabs(dt) > 1e-15 * (1.0 + fabs(t)))) break;  // converged (or not finite: no more steps)
  }
  const double e2 = exp(2.0 * t);
  const T tt = t - ((lnJ2 + t) * lam + (mu * e2 - mu)) * (1.0 / (2.0 * mu * e2 + lam));
  const T lnJ = lnJ2 + tt;
  const T F33 = dexp(tt);
  const T c = (lnJ * lam - mu) / J2;  // (lam ln J - mu) / J2: F2^-T = [[F3, -F2], [-F1, F0]] / J2
  P[0] = mu * F[0] + c * F[3];
  P[1] = mu * F[1] - c * F[2];
  P[2] = mu * F[2] - c * F[1];
  P[3] = mu * F[3] + c * F[0];
  const T I1 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2] + F[3] * F[3] + F33 * F33;
  return (0.5 * mu) * (I1 - 3.0) - mu * lnJ + (0.5 * lam) * (lnJ * lnJ);
}

// ---- J2 return mapping (generic in the scalar type) ---------------------------
// Packed Mandel strain e (C components; 2D plane strain: [e11, e22, sqrt2 e12], e33 = 0).
// Internally full 3D Mandel [11, 22, 33, sqrt2 23, sqrt2 13, sqrt2 12]; the plastic strain
// is deviatoric, so in 2D its out-of-plane entry is -(ep11 + ep22).
//   trial: ee = e - ep, sig = lam tr(ee) I + 2 mu ee, s = dev(sig), seq = sqrt(3/2 s:s)
//   Phi = seq - (sy + H p); if Phi > 0: dp = Phi / (3 mu + H), N = 3/2 s / seq,
//   sig -= 2 mu dp N  (N = 3/2 s / seq returns the stress onto the hardened yield surface)
// The elastic / plastic branch is decided on the value; derivatives follow the branch.
template <int NDIM, class T>
__device__ inline void j2_return(const T* e, const Local& L, T* sig6, T& dp, T* N6, bool& plastic) {
  T ee[6];
  if (NDIM == 3) {
#pragma unroll
    for (int k = 0; k < 6; ++k) ee[k] = e[k] - L.hist[k];
  } else {
    ee[0] = e[0] - L.hist[0];
    ee[1] = e[1] - L.hist[1];
    ee[2] = lift<T>(L.hist[0] + L.hist[1]);  // 0 - ep33
    ee[3] = lift<T>(0.0);
    ee[4] = lift<T>(0.0);
    ee[5] = e[2] - L.hist[2];
  }
  const double p = L.hist[NDIM == 3 ? 6 : 3];
  const T tr = ee[0] + ee[1] + ee[2];
#pragma unroll
  for (int k = 0; k < 6; ++k) sig6[k] = (2.0 * L.mu) * ee[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) sig6[k] = sig6[k] + L.lam * tr;
  const T m = (sig6[0] + sig6[1] + sig6[2]) * (1.0 / 3.0);
  T s[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) s[k] = (k < 3) ? sig6[k] - m : sig6[k];
  T ss = s[0] * s[0];
#pragma unroll
  for (int k = 1; k < 6; ++k) ss = ss + s[k] * s[k];
  const double phi_v = sqrt(1.5 * val(ss)) - (L.sy + L.H * p);
  plastic = phi_v > 0.0;
  if (!plastic) {
    dp = lift<T>(0.0);
#pragma unroll
    for (int k = 0; k < 6; ++k) N6[k] = lift<T>(0.0);
    return;
  }
  const T seq = dsqrt(1.5 * ss);
  dp = (seq - (L.sy + L.H * p)) * (1.0 / (3.0 * L.mu + L.H));
  const T f = lift<T>(1.5) / seq;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    N6[k] = f * s[k];
    sig6[k] = sig6[k] - (2.0 * L.mu) * (dp * N6[k]);
  }
}

template <int NDIM, class T>
__device__ inline void j2_pack(const T* sig6, T* out) {
  if (NDIM == 3) {
#pragma unroll
    for (int k = 0; k < 6; ++k) out[k] = sig6[k];
  } else {
    out[0] = sig6[0];
    out[1] = sig6[1];
    out[2] = sig6[5];
  }
}

// stored elastic energy 1/2 ee : C : ee of the returned state (the J2 "energy" output)
template <int NDIM>
__device__ inline double j2_energy(const double* e, const Local& L, const double* sig6) {
  // ee = C^-1 sig: tr(ee) = tr(sig) / (3 lam + 2 mu), dev(ee) = dev(sig) / (2 mu)
  const double trs = sig6[0] + sig6[1] + sig6[2];
  const double tre = trs / (3.0 * L.lam + 2.0 * L.mu);
  double w = 0.5 * trs * tre / 3.0;  // volumetric part 1/2 (tr sig / 3)(tr ee)
  const double m = trs / 3.0;
  double dd = 0.0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double s = (k < 3) ? sig6[k] - m : sig6[k];
    dd += s * s;
  }
  return w + 0.25 * dd / L.mu;
}

// ---- J2 under plane stress (2D) -------------------------------------------------
// The packed 2D strain [e11, e22, sqrt2 e12] is completed to the 3D Mandel strain
// [e11, e22, z, 0, 0, sqrt2 e12] and the history to [ep11, ep22, -(ep11 + ep22), 0, 0, sqrt2 ep12; p]
// (the plastic strain stays deviatoric, with no out-of-plane shear), and the 3D return mapping
// runs on them.  z = eps_33 makes sigma_33 vanish.  sigma_33(z) is continuous and increasing (its
// slope, the 3333 entry of the consistent tangent, is positive for mu > 0, H >= 0,
// 3 lam + 2 mu > 0): Newton's method from the elastic-trial root, kept inside a bracket that each
// step narrows and bisecting when a step leaves it (the slope jumps where the elastic and plastic
// branches meet), converges.  K : de is condensed on eps_33 from a second dual direction along z.
__device__ inline void j2_ps_local(const Local& L, Local& L3) {
  L3 = L;
  L3.hist[2] = -(L.hist[0] + L.hist[1]);
  L3.hist[3] = 0.0;
  L3.hist[4] = 0.0;
  L3.hist[5] = L.hist[2];
  L3.hist[6] = L.hist[3];
}

template <class T>
__device__ inline void j2_ps_strain(const T* e, const T& z, T* e3) {
  e3[0] = e[0];
  e3[1] = e[1];
  e3[2] = z;
  e3[3] = lift<T>(0.0);
  e3[4] = lift<T>(0.0);
  e3[5] = e[2];
}

__device__ inline double j2_ps_e33(const double* e, const Local& L3) {
  typedef Dual<double, 1> T;
  // trial sigma_33 = lam (e11 + e22 + z) + 2 mu (z - ep33) vanishes here
  double z = (2.0 * L3.mu * L3.hist[2] - L3.lam * (e[0] + e[1])) / (L3.lam + 2.0 * L3.mu);
  const double scale = fabs(e[0]) + fabs(e[1]) + fabs(e[2]) + fabs(z);
  double lo = -1e300, hi = 1e300;
  for (int it = 0; it < 100; ++it) {
    T x[3], zz, e3[6], sig6[6], N6[6], dp;
    bool pl;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      x[k].v = e[k];
      x[k].d[0] = 0.0;
    }
    zz.v = z;
    zz.d[0] = 1.0;
    j2_ps_strain<T>(x, zz, e3);
    j2_return<3, T>(e3, L3, sig6, dp, N6, pl);
    const double f = sig6[2].v, df = sig6[2].d[0];
    const double step = f / df;
    // converged: take the last step, which may be below half an ulp of z (also stops on a
    // non-finite step; the stress then carries it to the domain checks)
    if (!(fabs(step) > 1e-15 * scale)) {
      if (f != 0.0) z -= step;
      break;
    }
    if (f < 0.0) lo = z;
    else hi = z;
    double zn = z - step;
    // bisect only inside a finite bracket: with a positive slope a step above the tolerance moves
    // away from the bracket side it came from, so it can leave the bracket only past a finite side
    if (!(zn > lo && zn < hi) && lo > -1e300 && hi < 1e300) zn = 0.5 * (lo + hi);
    z = zn;
  }
  return z;
}

// stress (in-plane Mandel) and stored elastic energy
__device__ inline double j2_ps_stress(const double* e, const Local& L, double* P) {
  Local L3;
  j2_ps_local(L, L3);
  const double z = j2_ps_e33(e, L3);
  double e3[6], sig6[6], N6[6], dp;
  bool pl;
  j2_ps_strain<double>(e, z, e3);
  j2_return<3, double>(e3, L3, sig6, dp, N6, pl);
  P[0] = sig6[0];
  P[1] = sig6[1];
  P[2] = sig6[5];
  return j2_energy<3>(e3, L3, sig6);
}

// stress, K : de (condensed on eps_33) and stored elastic energy
__device__ inline double j2_ps_stress_jvp(const double* e, const double* de, const Local& L, double* P,
                                          double* KdE) {
  typedef Dual<double, 2> T;
  Local L3;
  j2_ps_local(L, L3);
  const double z = j2_ps_e33(e, L3);
  T x[3], zz, e3[6], sig6[6], N6[6], dp;
  bool pl;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    x[k].v = e[k];
    x[k].d[0] = de[k];
    x[k].d[1] = 0.0;
  }
  zz.v = z;
  zz.d[0] = 0.0;
  zz.d[1] = 1.0;
  j2_ps_strain<T>(x, zz, e3);
  j2_return<3, T>(e3, L3, sig6, dp, N6, pl);
  const double dz = -sig6[2].d[0] / sig6[2].d[1];
  const int idx[3] = {0, 1, 5};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P[k] = sig6[idx[k]].v;
    KdE[k] = sig6[idx[k]].d[0] + sig6[idx[k]].d[1] * dz;
  }
  double ev[6], s6[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    ev[k] = e3[k].v;
    s6[k] = sig6[k].v;
  }
  return j2_energy<3>(ev, L3, s6);
}

// history of the converged plane-stress state
__device__ inline void j2_ps_commit(const double* e, const Local& L, double* hist_out) {
  Local L3;
  j2_ps_local(L, L3);
  const double z = j2_ps_e33(e, L3);
  double e3[6], sig6[6], N6[6], dp;
  bool pl;
  j2_ps_strain<double>(e, z, e3);
  j2_return<3, double>(e3, L3, sig6, dp, N6, pl);
  hist_out[0] = L.hist[0] + dp * N6[0];
  hist_out[1] = L.hist[1] + dp * N6[1];
  hist_out[2] = L.hist[2] + dp * N6[5];
  hist_out[3] = L.hist[3] + dp;
}

// ---- derivatives by forward-mode AD -------------------------------------------

// psi and its gradient (the stress) at e: one vector-dual pass.  J2: the return-mapped
// stress, and the stored elastic energy.
template <int MAT, int NDIM>
__device__ inline double stress_ad(const double* e, const Local& L, double* P) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  if constexpr (MAT == MAT_J2) {
    double sig6[6], N6[6], dp;
    bool pl;
    j2_return<NDIM, double>(e, L, sig6, dp, N6, pl);
    j2_pack<NDIM, double>(sig6, P);
    return j2_energy<NDIM>(e, L, sig6);
  } else if constexpr (MAT == MAT_NH_PS) {
    return nh_plane_stress<double>(e, L.lam, L.mu, P);
  } else if constexpr (MAT == MAT_J2_PS) {
    return j2_ps_stress(e, L, P);
  } else {
    Dual<double, C> x[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      x[k].v = e[k];
#pragma unroll
      for (int j = 0; j < C; ++j) x[k].d[j] = (j == k) ? 1.0 : 0.0;
    }
    Dual<double, C> r = Energy<MAT, NDIM, Dual<double, C>>::psi(x, L.lam, L.mu);
#pragma unroll
    for (int k = 0; k < C; ++k) P[k] = r.d[k];
    return r.v;
  }
}

// K(e) : de, the Jacobian-vector product of the stress, by forward over forward (J2:
// one forward pass of the return mapping along de).
template <int MAT, int NDIM>
__device__ inline void tangent_jvp_ad(const double* e, const double* de, const Local& L, double* out) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  typedef Dual<double, 1> T;
  if constexpr (MAT == MAT_J2) {
    T x[C], sig6[6], N6[6], dp, o[C];
    bool pl;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      x[k].v = e[k];
      x[k].d[0] = de[k];
    }
    j2_return<NDIM, T>(x, L, sig6, dp, N6, pl);
    j2_pack<NDIM, T>(sig6, o);
#pragma unroll
    for (int k = 0; k < C; ++k) out[k] = o[k].d[0];
  } else if constexpr (MAT == MAT_NH_PS) {
    T x[C], o[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      x[k].v = e[k];
      x[k].d[0] = de[k];
    }
    nh_plane_stress<T>(x, L.lam, L.mu, o);
#pragma unroll
    for (int k = 0; k < C; ++k) out[k] = o[k].d[0];
  } else if constexpr (MAT == MAT_J2_PS) {
    double P[C];
    j2_ps_stress_jvp(e, de, L, P, out);
  } else {
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
    Dual<T, C> r = Energy<MAT, NDIM, Dual<T, C>>::psi(x, L.lam, L.mu);
#pragma unroll
    for (int k = 0; k < C; ++k) out[k] = r.d[k].d[0];
  }
}

// Stress and K : de together (same nested pass; the stress is in the partials' values).
template <int MAT, int NDIM>
__device__ inline double stress_and_jvp_ad(const double* e, const double* de, const Local& L, double* P,
                                           double* KdE) {
  constexpr int C = MatTraits<MAT, NDIM>::C;
  typedef Dual<double, 1> T;
  if constexpr (MAT == MAT_J2) {
    T x[C], sig6[6], N6[6], dp, o[C];
    bool pl;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      x[k].v = e[k];
      x[k].d[0] = de[k];
    }
    j2_return<NDIM, T>(x, L, sig6, dp, N6, pl);
    j2_pack<NDIM, T>(sig6, o);
    double s6[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) s6[k] = sig6[k].v;
#pragma unroll
    for (int k = 0; k < C; ++k) {
      P[k] = o[k].v;
      KdE[k] = o[k].d[0];
    }
    return j2_energy<NDIM>(e, L, s6);
  } else if constexpr (MAT == MAT_NH_PS) {
    T x[C], o[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
      x[k].v = e[k];
      x[k].d[0] = de[k];
    }
    const T psi = nh_plane_stress<T>(x, L.lam, L.mu, o);
#pragma unroll
    for (int k = 0; k < C; ++k) {
      P[k] = o[k].v;
      KdE[k] = o[k].d[0];
    }
    return psi.v;
  } else if constexpr (MAT == MAT_J2_PS) {
    return j2_ps_stress_jvp(e, de, L, P, KdE);
  } else {
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
    Dual<T, C> r = Energy<MAT, NDIM, Dual<T, C>>::psi(x, L.lam, L.mu);
#pragma unroll
    for (int k = 0; k < C; ++k) {
      P[k] = r.d[k].v;
      KdE[k] = r.d[k].d[0];
    }
    return r.v.v;
  }
}

// J2 history of the converged state at e: packed plastic strain and cumulative plastic strain
template <int NDIM>
__device__ inline void j2_commit(const double* e, const Local& L, double* hist_out) {
  constexpr int C = MatTraits<MAT_J2, NDIM>::C;
  double sig6[6], N6[6], dp;
  bool pl;
  j2_return<NDIM, double>(e, L, sig6, dp, N6, pl);
  double n[C];
  j2_pack<NDIM, double>(N6, n);
#pragma unroll
  for (int k = 0; k < C; ++k) hist_out[k] = L.hist[k] + dp * n[k];
  hist_out[C] = L.hist[C] + dp;
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
