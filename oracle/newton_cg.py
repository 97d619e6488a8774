"""Newton-CG solve of the Fourier-Galerkin equilibrium problem (oracle).

Follows the paper's Appendix A, Algorithm 1 (Newton-Krylov solver) with
textbook conjugate gradients as the inner linear solver (section 3), the
homogenized stress as the voxel average of the local stress (section 3.3), and
the homogenized tangent as the derivative of that average with respect to the
macroscopic strain (section 3.3, the homogenized-stiffness equation and the
macro-tangent listing).

Readings where the paper is silent or garbled:
* Newton stop test: the paper prints "delta eps / ||eps-bar|| < tol".  Read as
  the RMS ratio ||delta eps||_2 / (sqrt(N) ||eps-bar||_F) < tol_newton, where
  for finite strain eps-bar is the full macro F-bar (identity included).  The
  paper never loads to a zero macro strain; there (small strain unloaded to
  zero, where plasticity leaves residual stresses) the scale is the norm of the
  updated field ||eps||_2 instead, and a zero field counts as converged.
* A right-hand side that is already zero to rounding (homogeneous medium) is
  not handed to CG: if ||b|| <= 1e-13 ||sigma|| the Newton loop stops.
* Load increments: increment n starts from the previous converged field plus
  the uniform macro increment (the paper restarts from the uniform macro field
  and states no increment scheme).
* Homogenized tangent: the derivative of the converged solve with respect to
  the macro load equals, at convergence, the implicit linearisation: for each
  unit load E_I solve G*(K:x_I) = -G*(K:E_I) and set
  C_IJ = < (E_I + x_I) : K : (E_J + x_J) >.
* Index convention of macro quantities: small strain in Voigt order
  [11,22,33,23,13,12] with engineering shear (2D: [11,22,12]); finite strain
  row-major F-bar.  Stress components use the same order without factors.
"""

import math

import numpy as np

from .materials import MATERIALS
from .spectral import apply_G, inner

VOIGT_PAIRS = {
    2: [(0, 0), (1, 1), (0, 1)],
    3: [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)],
}


def macro_basis(kinematics, d):
    """Unit tensors E_I such that macro tensor = sum_I v_I E_I and stress_I = S:E_I."""
    out = []
    if kinematics == "small":
        for i, j in VOIGT_PAIRS[d]:
            E = np.zeros((d, d))
            if i == j:
                E[i, i] = 1.0
            else:
                E[i, j] = 0.5
                E[j, i] = 0.5
            out.append(E)
    else:
        for i in range(d):
            for j in range(d):
                E = np.zeros((d, d))
                E[i, j] = 1.0
                out.append(E)
    return out


def macro_to_tensor(macro, kinematics, d):
    basis = macro_basis(kinematics, d)
    macro = np.asarray(macro, dtype=np.float64)
    assert macro.shape == (len(basis),)
    return sum(v * E for v, E in zip(macro, basis))


def tensor_to_components(S, kinematics, d):
    """Voigt (small) or row-major (finite) components of the last two axes of S."""
    return np.stack([np.einsum("...ij,ij->...", S, E) for E in macro_basis(kinematics, d)], axis=-1)


class Problem:
    """A periodic voxel RVE: grid, constitutive law and per-voxel Lame parameters."""

    def __init__(self, shape, material, lam, mu, lengths=None):
        self.shape = tuple(int(s) for s in shape)
        self.d = len(self.shape)
        assert self.d in (2, 3)
        self.mat = MATERIALS[material]
        self.material = material
        self.kinematics = self.mat.kinematics
        self.lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), self.shape).copy()
        self.mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), self.shape).copy()
        self.lengths = lengths
        self.N = int(np.prod(self.shape))

    def reference_macro(self):
        d = self.d
        return np.eye(d) if self.kinematics == "finite" else np.zeros((d, d))

    def uniform(self, T):
        return np.broadcast_to(T, self.shape + (self.d, self.d)).copy()

    # --- operators of the method ------------------------------------------------
    def stress(self, E):
        return self.mat.stress(E, self.lam, self.mu)

    def energy_density(self, E):
        return self.mat.psi(E, self.lam, self.mu)

    def G(self, A):
        return apply_G(A, self.kinematics, self.lengths)

    def operator(self, E, p):
        """The linearised Fourier-Galerkin operator  p -> G*(K(E) : p)."""
        return self.G(self.mat.tangent_apply(E, p, self.lam, self.mu))

    def rhs(self, E):
        return -self.G(self.stress(E))


def conjugate_gradient(apply_A, b, tol, max_iter):
    """Textbook (Hestenes-Stiefel) CG from x0 = 0; stops when ||r|| <= tol ||b||.

    Returns (x, iterations, status) with status in {"ok", "not_converged",
    "breakdown"}.
    """
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = inner(r, r)
    stop = tol * math.sqrt(rr)
    k = 0
    while math.sqrt(rr) > stop:
        if k >= max_iter:
            return x, k, "not_converged"
        q = apply_A(p)
        pq = inner(p, q)
        if not pq > 0.0:
            return x, k, "breakdown"
        alpha = rr / pq
        x += alpha * p
        r -= alpha * q
        rr_new = inner(r, r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        k += 1
    return x, k, "ok"


class State:
    """Converged local field and the macro tensor it belongs to."""

    def __init__(self, field, macro):
        self.field = field
        self.macro = macro


def initial_state(problem):
    ref = problem.reference_macro()
    return State(problem.uniform(ref), ref.copy())


def solve(problem, macro, n_increments=1, tol_newton=1e-10, tol_cg=1e-10, max_newton=50,
          max_cg=100000, state=None, zero_rhs_rel=1e-13):
    """Newton-CG (Algorithm 1) with linear load increments.

    Returns a dict with the converged ``state``, ``macro_stress`` (Voigt or
    row-major components), ``energy`` (volume-averaged energy density) and
    ``stats`` (Newton iterations, CG iterations per Newton iteration, status).
    """
    d = problem.d
    if state is None:
        state = initial_state(problem)
    field = state.field.copy()
    start = state.macro.copy()
    target = macro_to_tensor(macro, problem.kinematics, d)
    sqrtN = math.sqrt(problem.N)

    newton_total = 0
    cg_counts = []
    status = "ok"
    prev = start
    for n in range(1, n_increments + 1):
        # history-dependent laws (J2 plasticity) carry the converged state of the previous
        # load step into this one (Appendix B: the trial state starts from eps_elas(t))
        if getattr(problem, "pending", False):
            problem.commit(field)
        current = start + (float(n) / float(n_increments)) * (target - start)
        field += current - prev
        prev = current
        macro_norm = math.sqrt(float(np.sum(current * current)))
        it = 0
        while True:
            if problem.kinematics == "finite" and np.any(np.linalg.det(field) <= 0.0):
                status = "domain"
                break
            sigma = problem.stress(field)
            b = -problem.G(sigma)
            if math.sqrt(inner(b, b)) <= zero_rhs_rel * math.sqrt(inner(sigma, sigma)):
                break
            if it >= max_newton:
                status = "not_converged"
                break
            x, k, st = conjugate_gradient(lambda v: problem.operator(field, v), b, tol_cg, max_cg)
            cg_counts.append(k)
            if st != "ok":
                status = st
                break
            field += x
            it += 1
            scale = sqrtN * macro_norm if macro_norm > 0.0 else math.sqrt(inner(field, field))
            dn = math.sqrt(inner(x, x))
            res = dn / scale if scale > 0.0 else (math.inf if dn > 0.0 else 0.0)
            if res < tol_newton:
                break
        newton_total += it
        if status != "ok":
            break
        if hasattr(problem, "commit"):
            problem.pending = True

    out_state = State(field, prev)
    result = {
        "state": out_state,
        "stats": {"newton": newton_total, "cg": cg_counts, "cg_total": int(sum(cg_counts)),
                  "status": status},
    }
    if status != "domain":
        result["macro_stress"] = tensor_to_components(
            homogenized(problem.stress(field)), problem.kinematics, d)
        result["energy"] = float(np.mean(problem.energy_density(field)))
    return result


def homogenized(S):
    """Voxel average of a tensor field (section 3.3)."""
    d = S.shape[-1]
    return np.mean(S.reshape(-1, d, d), axis=0)


def homogenized_tangent(problem, state, tol_cg=1e-10, max_cg=100000, zero_rhs_rel=1e-13):
    """Homogenized tangent at a converged state by the implicit linearisation.

    Returns (C, C_direct, cg_counts): C_IJ = <(E_I + x_I):K:(E_J + x_J)> (the
    energy form, symmetric), C_direct_IJ = <E_I : K : (E_J + x_J)>.  A load
    whose right-hand side is zero to rounding (||b|| <= 1e-13 ||K:E_I||) gets
    x_I = 0 without CG, as in the Newton loop.
    """
    d = problem.d
    field = state.field
    basis = macro_basis(problem.kinematics, d)
    K = lambda v: problem.mat.tangent_apply(field, v, problem.lam, problem.mu)  # noqa: E731
    totals = []
    counts = []
    for E in basis:
        EI = problem.uniform(E)
        KE = K(EI)
        b = -problem.G(KE)
        if math.sqrt(inner(b, b)) <= zero_rhs_rel * math.sqrt(inner(KE, KE)):
            x, k = np.zeros_like(b), 0
        else:
            x, k, st = conjugate_gradient(lambda v: problem.operator(field, v), b, tol_cg, max_cg)
            if st != "ok":
                raise RuntimeError("tangent CG: " + st)
        counts.append(k)
        totals.append(EI + x)
    m = len(basis)
    C = np.zeros((m, m))
    Cd = np.zeros((m, m))
    for J in range(m):
        KJ = K(totals[J])
        for I in range(m):
            C[I, J] = inner(totals[I], KJ) / problem.N
            Cd[I, J] = inner(problem.uniform(basis[I]), KJ) / problem.N
    return C, Cd, counts
