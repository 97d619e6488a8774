"""Gradient of homogenized energy / stress with respect to a per-voxel density (oracle).

The paper's section 4.4.2 (microstructure optimisation) needs the sensitivity of
homogenized quantities to a density field rho(x) whose SIMP interpolation
scales the stiffness; it obtains them by reverse-mode AD through the solver.
Here the same derivative is written as the adjoint of the converged
Fourier-Galerkin problem (the macro load is prescribed):

  J(rho) = w_e * Psi-bar + W : P-bar,     W = sum_I w_I E_I (macro index convention)
  g      = w_e P + K : W                  (dJ/dF per voxel, times N)
  solve    G*(K : x) = -G*(g)             (same operator as the Newton-CG solve)
  dJ/drho_v = (p / (N rho_v)) [ w_e psi_v + (W + x_v) : P_v ]

using lam_v = lam0_v rho_v^p, mu_v = mu0_v rho_v^p, so that d psi_v / d rho_v =
(p / rho_v) psi_v and d P_v / d rho_v = (p / rho_v) P_v at fixed strain.  For a
pure energy objective the right-hand side vanishes at equilibrium and the
gradient is the envelope form p psi_v / (N rho_v).
"""

import math

import numpy as np

from .newton_cg import conjugate_gradient, macro_basis
from .spectral import inner


def simp_gradient(problem, state, density, p, w_stress, w_energy, tol_cg=1e-12, max_cg=100000,
                  zero_rhs_rel=1e-13):
    """Returns (grad, cg_iterations); `problem` must already carry lam0 rho^p, mu0 rho^p."""
    F = state.field
    d = problem.d
    W = sum(w * E for w, E in zip(np.asarray(w_stress, dtype=np.float64), macro_basis(problem.kinematics, d)))
    P = problem.stress(F)
    psi = problem.energy_density(F)
    g = w_energy * P + problem.mat.tangent_apply(F, problem.uniform(W), problem.lam, problem.mu)
    b = -problem.G(g)
    if math.sqrt(inner(b, b)) <= zero_rhs_rel * math.sqrt(inner(g, g)):
        x, k = np.zeros_like(b), 0
    else:
        x, k, st = conjugate_gradient(lambda v: problem.operator(F, v), b, tol_cg, max_cg)
        if st != "ok":
            raise RuntimeError("adjoint CG: " + st)
    WP = np.einsum("...ij,...ij->...", W + x, P)
    grad = p / (problem.N * np.asarray(density)) * (w_energy * psi + WP)
    return grad, k


def objective(problem, state, w_stress, w_energy):
    """J = w_e Psi-bar + sum_I w_I P-bar_I at a converged state."""
    from .newton_cg import homogenized, tensor_to_components
    F = state.field
    Pbar = tensor_to_components(homogenized(problem.stress(F)), problem.kinematics, problem.d)
    return float(w_energy * np.mean(problem.energy_density(F)) + np.dot(np.asarray(w_stress), Pbar))
