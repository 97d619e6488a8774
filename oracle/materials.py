"""Energy density, stress and tangent in closed form (oracle).

These are the paper's "analytical implementation" counterparts of the
automatic-differentiation path (section 3.1: stress is the derivative of the
energy density; section 3.2: the incremental stress is the tangent applied to a
strain increment).  Every function accepts real or complex arrays so that the
CPU tests can pin them with complex-step derivatives.

Arguments: strain-like tensors ``E`` of shape (*grid, d, d); Lame parameters
``lam``, ``mu`` broadcastable to the grid.  d = 2 means plane strain: the
out-of-plane strain is zero (F33 = 1 for finite strain).

Readings of the paper used here:
* linear elastic energy  psi = lam/2 tr(eps)^2 + mu eps:eps.  The paper prints
  it without the 1/2 and with a trace on the scalar; its Table 1 values
  (C_xxxx about 4.04 for a lam=2, mu=1 matrix, i.e. lam + 2 mu) fix the 1/2.
* St. Venant-Kirchhoff (section 4.1.1, hyperelastic energy): Green-Lagrange
  strain E = (F^T F - I)/2, psi = lam/2 tr(E)^2 + mu E:E.
* compressible Neo-Hookean (not written out in the paper):
  psi = mu/2 (I1 - 3) - mu ln J + lam/2 (ln J)^2, I1 = tr(F^T F).
* plane stress (named with the 2D examples of section 4.4, not written out):
  the 3D law with the out-of-plane entry chosen so that the out-of-plane
  normal stress vanishes at each point, for every law here.
"""

import numpy as np


def _eye(d):
    return np.eye(d)


def _tr(A):
    return np.einsum("...ii->...", A)


def _lm(lam, mu):
    lam = np.asarray(lam)
    mu = np.asarray(mu)
    return lam[..., None, None], mu[..., None, None]


# ----------------------------------------------------------------------------
# small strain, linear elastic
# ----------------------------------------------------------------------------
class LinearElastic:
    kinematics = "small"

    @staticmethod
    def psi(eps, lam, mu):
        lam = np.asarray(lam)
        mu = np.asarray(mu)
        tr = _tr(eps)
        return 0.5 * lam * tr * tr + mu * np.einsum("...ij,...ij->...", eps, eps)

    @staticmethod
    def stress(eps, lam, mu):
        d = eps.shape[-1]
        L, M = _lm(lam, mu)
        return L * _tr(eps)[..., None, None] * _eye(d) + 2.0 * M * eps

    @staticmethod
    def tangent_apply(eps, deps, lam, mu):
        d = deps.shape[-1]
        L, M = _lm(lam, mu)
        return L * _tr(deps)[..., None, None] * _eye(d) + 2.0 * M * deps

    @staticmethod
    def tangent_tensor(eps, lam, mu):
        d = eps.shape[-1]
        I = _eye(d)
        lam = np.asarray(lam)[..., None, None, None, None]
        mu = np.asarray(mu)[..., None, None, None, None]
        base = (
            lam * np.einsum("ij,kl->ijkl", I, I)
            + mu * (np.einsum("ik,jl->ijkl", I, I) + np.einsum("il,jk->ijkl", I, I))
        )
        return np.broadcast_to(base, eps.shape[:-2] + (d, d, d, d)).copy()


class LinearElasticPlaneStress:
    """2D linear elasticity under plane stress: the out-of-plane strain eps_33 takes the value that
    makes sigma_33 of the 3D law vanish, eps_33 = -lam tr(eps) / (lam + 2 mu); stress, tangent and
    energy are those of the 3D law at that strain (the in-plane block of the stress)."""

    kinematics = "small"

    @staticmethod
    def _full(eps, lam, mu):
        lam = np.asarray(lam, dtype=np.float64)
        mu = np.asarray(mu, dtype=np.float64)
        e3 = np.zeros(eps.shape[:-2] + (3, 3), dtype=eps.dtype)
        e3[..., :2, :2] = eps
        e3[..., 2, 2] = -lam * _tr(eps) / (lam + 2.0 * mu)
        return e3

    @staticmethod
    def stress(eps, lam, mu):
        e3 = LinearElasticPlaneStress._full(eps, lam, mu)
        return LinearElastic.stress(e3, lam, mu)[..., :2, :2]

    @staticmethod
    def tangent_apply(eps, deps, lam, mu):
        return LinearElasticPlaneStress.stress(deps, lam, mu)

    @staticmethod
    def psi(eps, lam, mu):
        return LinearElastic.psi(LinearElasticPlaneStress._full(eps, lam, mu), lam, mu)


# ----------------------------------------------------------------------------
# finite strain, compressible Neo-Hookean
# ----------------------------------------------------------------------------
class NeoHookean:
    kinematics = "finite"

    @staticmethod
    def _invariants(F):
        d = F.shape[-1]
        J = np.linalg.det(F)
        I1 = np.einsum("...ij,...ij->...", F, F) + (3 - d)
        return J, I1

    @staticmethod
    def psi(F, lam, mu):
        lam = np.asarray(lam)
        mu = np.asarray(mu)
        J, I1 = NeoHookean._invariants(F)
        lnJ = np.log(J)
        return 0.5 * mu * (I1 - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ

    @staticmethod
    def stress(F, lam, mu):
        L, M = _lm(lam, mu)
        J = np.linalg.det(F)
        FinvT = np.swapaxes(np.linalg.inv(F), -1, -2)
        lnJ = np.log(J)[..., None, None]
        return M * F + (L * lnJ - M) * FinvT

    @staticmethod
    def tangent_apply(F, dF, lam, mu):
        L, M = _lm(lam, mu)
        Finv = np.linalg.inv(F)
        FinvT = np.swapaxes(Finv, -1, -2)
        lnJ = np.log(np.linalg.det(F))[..., None, None]
        tr = np.einsum("...ij,...ji->...", Finv, dF)[..., None, None]  # tr(F^-1 dF)
        dFT = np.swapaxes(dF, -1, -2)
        return M * dF + L * tr * FinvT - (L * lnJ - M) * (FinvT @ dFT @ FinvT)

    @staticmethod
    def tangent_tensor(F, lam, mu):
        d = F.shape[-1]
        I = _eye(d)
        Finv = np.linalg.inv(F)
        lnJ = np.log(np.linalg.det(F))[..., None, None, None, None]
        lam = np.asarray(lam)[..., None, None, None, None]
        mu = np.asarray(mu)[..., None, None, None, None]
        t1 = np.einsum("ik,jl->ijkl", I, I)
        t2 = np.einsum("...ji,...lk->...ijkl", Finv, Finv)
        t3 = np.einsum("...jk,...li->...ijkl", Finv, Finv)
        return mu * t1 + lam * t2 - (lam * lnJ - mu) * t3


# ----------------------------------------------------------------------------
# finite strain, St. Venant-Kirchhoff
# ----------------------------------------------------------------------------
class StVenantKirchhoff:
    kinematics = "finite"

    @staticmethod
    def _green(F):
        d = F.shape[-1]
        return 0.5 * (np.swapaxes(F, -1, -2) @ F - _eye(d))

    @staticmethod
    def psi(F, lam, mu):
        lam = np.asarray(lam)
        mu = np.asarray(mu)
        E = StVenantKirchhoff._green(F)
        tr = _tr(E)
        return 0.5 * lam * tr * tr + mu * np.einsum("...ij,...ij->...", E, E)

    @staticmethod
    def _S(E, L, M):
        d = E.shape[-1]
        return L * _tr(E)[..., None, None] * _eye(d) + 2.0 * M * E

    @staticmethod
    def stress(F, lam, mu):
        L, M = _lm(lam, mu)
        return F @ StVenantKirchhoff._S(StVenantKirchhoff._green(F), L, M)

    @staticmethod
    def tangent_apply(F, dF, lam, mu):
        L, M = _lm(lam, mu)
        S = StVenantKirchhoff._S(StVenantKirchhoff._green(F), L, M)
        FT = np.swapaxes(F, -1, -2)
        dE = 0.5 * (np.swapaxes(dF, -1, -2) @ F + FT @ dF)
        return dF @ S + F @ StVenantKirchhoff._S(dE, L, M)

    @staticmethod
    def tangent_tensor(F, lam, mu):
        d = F.shape[-1]
        out = np.zeros(F.shape[:-2] + (d, d, d, d), dtype=np.result_type(F, 1.0))
        for k in range(d):
            for l in range(d):
                dF = np.zeros(F.shape, dtype=out.dtype)
                dF[..., k, l] = 1.0
                out[..., :, :, k, l] = StVenantKirchhoff.tangent_apply(F, dF, lam, mu)
        return out


# ----------------------------------------------------------------------------
# finite strain under plane stress
# ----------------------------------------------------------------------------
# A 2D deformation gradient F2 is completed to F = [[F2, 0], [0, F33]]; the out-of-plane stretch F33
# takes the value at which the 3D law's P33 vanishes.  For an isotropic law the out-of-plane shear
# stresses vanish with the shear entries of F.  Stress and energy are those of the 3D law at that F
# (the in-plane block of P).  The tangent is the 3D tangent condensed on dF33, the textbook static
# condensation:  K_ps : dF2 = K_ab:dF - K_ab33 (K_33:dF) / K_3333.


def _embed(F, F33):
    out = np.zeros(F.shape[:-2] + (3, 3), dtype=np.result_type(F, F33))
    out[..., :2, :2] = F
    out[..., 2, 2] = F33
    return out


def _condensed_apply(K3, dF):
    dF3 = _embed(dF, np.zeros(dF.shape[:-2]))
    q = np.einsum("...ijkl,...kl->...ij", K3, dF3)
    dF33 = -q[..., 2, 2] / K3[..., 2, 2, 2, 2]
    return q[..., :2, :2] + K3[..., :2, :2, 2, 2] * dF33[..., None, None]


class NeoHookeanPlaneStress:
    """Neo-Hookean under plane stress.  With J = det(F2) F33, P33 F33 = mu F33^2 + lam ln J - mu is
    increasing in F33 > 0 for lam >= 0, mu > 0 and runs from -inf to +inf, so its root is found by
    bisection on a bracket grown from 1."""

    kinematics = "finite"

    @staticmethod
    def stretch(F, lam, mu):
        J2 = np.linalg.det(F)
        lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), J2.shape)
        mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), J2.shape)

        def h(s):
            return mu * s * s + lam * np.log(J2 * s) - mu

        lo = np.ones(J2.shape)
        hi = np.ones(J2.shape)
        for _ in range(2000):
            m = h(lo) > 0
            if not m.any():
                break
            lo = np.where(m, 0.5 * lo, lo)
        for _ in range(2000):
            m = h(hi) < 0
            if not m.any():
                break
            hi = np.where(m, 2.0 * hi, hi)
        for _ in range(4000):
            mid = 0.5 * (lo + hi)
            done = (mid <= lo) | (mid >= hi)
            if done.all():
                break
            up = h(mid) > 0
            hi = np.where(up & ~done, mid, hi)
            lo = np.where(~up & ~done, mid, lo)
        return 0.5 * (lo + hi)

    @staticmethod
    def full(F, lam, mu):
        return _embed(F, NeoHookeanPlaneStress.stretch(F, lam, mu))

    @staticmethod
    def stress(F, lam, mu):
        return NeoHookean.stress(NeoHookeanPlaneStress.full(F, lam, mu), lam, mu)[..., :2, :2]

    @staticmethod
    def psi(F, lam, mu):
        return NeoHookean.psi(NeoHookeanPlaneStress.full(F, lam, mu), lam, mu)

    @staticmethod
    def tangent_apply(F, dF, lam, mu):
        K3 = NeoHookean.tangent_tensor(NeoHookeanPlaneStress.full(F, lam, mu), lam, mu)
        return _condensed_apply(K3, dF)


class StVenantKirchhoffPlaneStress:
    """St. Venant-Kirchhoff under plane stress.  P33 = F33 S33 and S33 = lam (E11 + E22) +
    (lam + 2 mu) E33, so P33 = 0 fixes E33 = -lam (E11 + E22) / (lam + 2 mu) and
    F33 = sqrt(1 + 2 E33)."""

    kinematics = "finite"

    @staticmethod
    def full(F, lam, mu):
        lam = np.asarray(lam, dtype=np.float64)
        mu = np.asarray(mu, dtype=np.float64)
        E = StVenantKirchhoff._green(F)
        E33 = -lam * (E[..., 0, 0] + E[..., 1, 1]) / (lam + 2.0 * mu)
        return _embed(F, np.sqrt(1.0 + 2.0 * E33))

    @staticmethod
    def stress(F, lam, mu):
        return StVenantKirchhoff.stress(StVenantKirchhoffPlaneStress.full(F, lam, mu), lam, mu)[..., :2, :2]

    @staticmethod
    def psi(F, lam, mu):
        return StVenantKirchhoff.psi(StVenantKirchhoffPlaneStress.full(F, lam, mu), lam, mu)

    @staticmethod
    def tangent_apply(F, dF, lam, mu):
        K3 = StVenantKirchhoff.tangent_tensor(StVenantKirchhoffPlaneStress.full(F, lam, mu), lam, mu)
        return _condensed_apply(K3, dF)


MATERIALS = {
    "linear_elastic": LinearElastic,
    "linear_elastic_plane_stress": LinearElasticPlaneStress,
    "neo_hookean": NeoHookean,
    "stvk": StVenantKirchhoff,
    "neo_hookean_plane_stress": NeoHookeanPlaneStress,
    "stvk_plane_stress": StVenantKirchhoffPlaneStress,
}


def lame_from_young(E, nu):
    """Lame parameters from Young's modulus and Poisson ratio (3D / plane strain)."""
    E = np.asarray(E, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu
