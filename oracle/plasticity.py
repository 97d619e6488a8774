"""J2 (von Mises) small-strain plasticity with linear isotropic hardening (oracle).

TEST INFRASTRUCTURE ONLY (see the package header).

Follows the predictor-corrector of the paper's Appendix B (elastoplastic
material) with the consistent tangent of its section 4.1.2 example:

    trial:      eps_e = eps - eps_p(t),  sig_tr = C_elas : eps_e,  s = dev(sig_tr)
                sig_eq = sqrt(3/2 s:s),  Phi = sig_eq - (sig_y + H p(t))
    corrector:  dp = <Phi>_+ / (3 mu + H),  N = (3/2) s / sig_eq
                sig = sig_tr - 2 mu dp N
    history:    eps_p(t+dt) = eps_p(t) + dp N,  p(t+dt) = p(t) + dp
    tangent:    K = C_elas                                             (dp = 0)
                K = C_elas - (6 mu^2 dp / sig_eq) I_dev
                    + 4 mu^2 (dp / sig_eq - 1 / (3 mu + H)) N (x) N     (dp > 0)

Reading: the appendix prints the corrector with the unit-free direction
s / sig_eq; only N = (3/2) s / sig_eq returns the stress onto the yield surface
(sig_eq(sig) = sig_y + H (p + dp)) with dp = Phi / (3 mu + H), and it is the N
for which the printed tangent is the derivative of the update.  The pins in
tests/test_oracle_plasticity.py check both facts.

Tensors are full 3x3 (plane strain in 2D: eps_33 = 0, the plastic strain keeps
its out-of-plane component eps_p33 = -(eps_p11 + eps_p22)).  The elastic part is
the isotropic linear elastic law of materials.LinearElastic.  Plane stress
(PlasticPlaneStressProblem) chooses eps_33 per point so that sigma_33 vanishes;
the paper names plane stress with its 2D examples without writing it out.
"""

import numpy as np

from . import newton_cg
from .spectral import apply_G


def _tr(A):
    return np.einsum("...ii->...", A)


def _dev(A):
    return A - _tr(A)[..., None, None] / 3.0 * np.eye(3)


def embed(E):
    """(..., d, d) in-plane strain -> (..., 3, 3) with zero out-of-plane entries (d = 2 or 3)."""
    d = E.shape[-1]
    if d == 3:
        return E
    out = np.zeros(E.shape[:-2] + (3, 3), dtype=E.dtype)
    out[..., :2, :2] = E
    return out


def _elastic(E3, lam, mu):
    return lam[..., None, None] * _tr(E3)[..., None, None] * np.eye(3) + 2.0 * mu[..., None, None] * E3


def return_map(E, ep, p, lam, mu, sy, H):
    """Trial state and radial return at total strain E (..., d, d) from history (ep (..., 3, 3), p).

    Returns (sigma (..., 3, 3), dp (...), N (..., 3, 3)); N is zero where dp = 0.
    """
    lam, mu, sy, H = (np.asarray(a, dtype=np.float64) for a in (lam, mu, sy, H))
    ee = embed(E) - ep
    sig_tr = _elastic(ee, lam, mu)
    s = _dev(sig_tr)
    seq = np.sqrt(1.5 * np.einsum("...ij,...ij->...", s, s))
    phi = seq - (sy + H * p)
    dp = np.maximum(phi, 0.0) / (3.0 * mu + H)
    safe = np.where(seq > 0.0, seq, 1.0)
    N = np.where((dp > 0.0)[..., None, None], 1.5 * s / safe[..., None, None], 0.0)
    sigma = sig_tr - 2.0 * mu[..., None, None] * dp[..., None, None] * N
    return sigma, dp, N


def tangent_apply(E, dE, ep, p, lam, mu, sy, H):
    """Consistent tangent applied to dE (..., d, d), in closed form; returns (..., 3, 3)."""
    lam, mu, sy, H = (np.asarray(a, dtype=np.float64) for a in (lam, mu, sy, H))
    sigma, dp, N = return_map(E, ep, p, lam, mu, sy, H)
    ee = embed(E) - ep
    s = _dev(_elastic(ee, lam, mu))
    seq = np.sqrt(1.5 * np.einsum("...ij,...ij->...", s, s))
    safe = np.where(seq > 0.0, seq, 1.0)
    dE3 = embed(dE)
    out = _elastic(dE3, lam, mu)
    plastic = dp > 0.0
    a = np.where(plastic, 6.0 * mu * mu * dp / safe, 0.0)
    b = np.where(plastic, 4.0 * mu * mu * (dp / safe - 1.0 / (3.0 * mu + H)), 0.0)
    NdE = np.einsum("...ij,...ij->...", N, dE3)
    return out - a[..., None, None] * _dev(dE3) + b[..., None, None] * NdE[..., None, None] * N


class PlasticProblem(newton_cg.Problem):
    """A periodic RVE of J2 phases: per-voxel (lam, mu, sig_y, H) and the plastic history.

    The history (eps_p, p) belongs to the last committed load step.  ``commit`` moves it
    to the converged state of the current step; the solver commits at the start of the
    next load increment, so stresses and tangents after a solve are those of the step
    that produced them.
    """

    def __init__(self, shape, lam, mu, sy, H, lengths=None):
        super().__init__(shape, "linear_elastic", lam, mu, lengths)
        self.material = "j2_plastic"
        self.sy = np.broadcast_to(np.asarray(sy, dtype=np.float64), self.shape).copy()
        self.H = np.broadcast_to(np.asarray(H, dtype=np.float64), self.shape).copy()
        self.ep = np.zeros(self.shape + (3, 3))
        self.p = np.zeros(self.shape)
        self.pending = False

    def _inplane(self, S3):
        d = self.d
        return S3[..., :d, :d]

    def stress(self, E):
        sigma, _, _ = return_map(E, self.ep, self.p, self.lam, self.mu, self.sy, self.H)
        return self._inplane(sigma)

    def stress3(self, E):
        return return_map(E, self.ep, self.p, self.lam, self.mu, self.sy, self.H)[0]

    def energy_density(self, E):
        """Stored elastic energy of the returned state, 1/2 eps_e : C : eps_e."""
        _, dp, N = return_map(E, self.ep, self.p, self.lam, self.mu, self.sy, self.H)
        ee = embed(E) - self.ep - dp[..., None, None] * N
        return 0.5 * self.lam * _tr(ee) ** 2 + self.mu * np.einsum("...ij,...ij->...", ee, ee)

    def tangent_apply(self, E, dE):
        return self._inplane(tangent_apply(E, dE, self.ep, self.p, self.lam, self.mu, self.sy, self.H))

    def operator(self, E, v):
        return apply_G(self.tangent_apply(E, v), "small", self.lengths)

    def plastic_strain_now(self, E):
        """Cumulative plastic strain of the state at E (history plus this step's increment)."""
        _, dp, _ = return_map(E, self.ep, self.p, self.lam, self.mu, self.sy, self.H)
        return self.p + dp

    def commit(self, E):
        _, dp, N = return_map(E, self.ep, self.p, self.lam, self.mu, self.sy, self.H)
        self.ep = self.ep + dp[..., None, None] * N
        self.p = self.p + dp
        self.pending = False


class PlasticPlaneStressProblem(PlasticProblem):
    """2D J2 cell under plane stress: at each voxel the out-of-plane strain eps_33 takes the value at
    which sigma_33 of the 3D return mapping (from that voxel's history) vanishes; eps_13 = eps_23 = 0
    and the out-of-plane shear stresses vanish with them.  sigma_33 is continuous and increasing in
    eps_33 (its slope is the consistent tangent's 3333 entry), so bisection on a bracket grown about
    the elastic-trial root finds it.  The tangent is the consistent tangent condensed on eps_33."""

    def __init__(self, shape, lam, mu, sy, H, lengths=None):
        super().__init__(shape, lam, mu, sy, H, lengths)
        if self.d != 2:
            raise ValueError("plane stress is a 2D setting")
        self._last = None

    def _s33(self, E, z):
        E3 = embed(E).copy()
        E3[..., 2, 2] = z
        return return_map(E3, self.ep, self.p, self.lam, self.mu, self.sy, self.H)[0][..., 2, 2]

    def full(self, E):
        """The 3D strain of the plane-stress state at in-plane strain E."""
        if self._last is not None and self._last[0].shape == E.shape and np.array_equal(self._last[0], E) \
                and self._last[1] is self.ep:
            return self._last[2]
        # elastic trial root: lam (e11 + e22 + z) + 2 mu (z - ep33) = 0
        z0 = (2.0 * self.mu * self.ep[..., 2, 2] - self.lam * (E[..., 0, 0] + E[..., 1, 1])) / (self.lam + 2.0 * self.mu)
        w = np.abs(E).max(axis=(-2, -1)) + np.abs(z0) + 1e-12
        lo, hi = z0 - w, z0 + w
        for _ in range(200):
            bad = self._s33(E, lo) > 0
            if not bad.any():
                break
            lo = np.where(bad, lo - 2 * w, lo)
            w = np.where(bad, 2 * w, w)
        for _ in range(200):
            bad = self._s33(E, hi) < 0
            if not bad.any():
                break
            hi = np.where(bad, hi + 2 * w, hi)
            w = np.where(bad, 2 * w, w)
        for _ in range(2000):
            mid = 0.5 * (lo + hi)
            done = (mid <= lo) | (mid >= hi)
            if done.all():
                break
            up = self._s33(E, mid) > 0
            hi = np.where(up & ~done, mid, hi)
            lo = np.where(~up & ~done, mid, lo)
        E3 = embed(E).copy()
        E3[..., 2, 2] = 0.5 * (lo + hi)
        self._last = (E.copy(), self.ep, E3)
        return E3

    def stress(self, E):
        return super().stress3(self.full(E))[..., :2, :2]

    def stress3(self, E):
        return super().stress3(self.full(E))

    def energy_density(self, E):
        return super().energy_density(self.full(E))

    def tangent_apply(self, E, dE):
        E3 = self.full(E)
        q = tangent_apply(E3, embed(dE), self.ep, self.p, self.lam, self.mu, self.sy, self.H)
        u = np.zeros(E3.shape)
        u[..., 2, 2] = 1.0
        k = tangent_apply(E3, u, self.ep, self.p, self.lam, self.mu, self.sy, self.H)
        dz = -q[..., 2, 2] / k[..., 2, 2]
        return (q + dz[..., None, None] * k)[..., :2, :2]

    def plastic_strain_now(self, E):
        return super().plastic_strain_now(self.full(E))

    def commit(self, E):
        super().commit(self.full(E))


def homogenized_tangent(problem, state, tol_cg=1e-10, max_cg=100000, zero_rhs_rel=1e-13):
    """Implicit homogenized tangent of the current (uncommitted) step: the linear-elastic
    machinery of newton_cg with the consistent tangent in place of the elastic one."""
    d = problem.d
    field = state.field
    basis = newton_cg.macro_basis("small", d)
    K = problem.tangent_apply
    totals, counts = [], []
    for E in basis:
        EI = problem.uniform(E)
        KE = K(field, EI)
        b = -problem.G(KE)
        if np.sqrt(newton_cg.inner(b, b)) <= zero_rhs_rel * np.sqrt(newton_cg.inner(KE, KE)):
            x, k = np.zeros_like(b), 0
        else:
            x, k, st = newton_cg.conjugate_gradient(lambda v: problem.operator(field, v), b, tol_cg, max_cg)
            if st != "ok":
                raise RuntimeError("tangent CG: " + st)
        counts.append(k)
        totals.append(EI + x)
    m = len(basis)
    C = np.zeros((m, m))
    for J in range(m):
        KJ = K(field, totals[J])
        for I in range(m):
            C[I, J] = newton_cg.inner(totals[I], KJ) / problem.N
    return C, counts
