"""torch.autograd.Function around the solve and its hand-written adjoint.

Forward: set the per-voxel density (SIMP scaling of lam, mu by rho^p), restart
from the undeformed state, run fft_homog_solve and return
J = w_energy * psi-bar + w_stress . out.  Backward: fft_homog_adjoint (one
extra CG solve with the same operator) gives dJ/drho per voxel.  Both run in
the HIP library; the handle keeps the converged state between the two calls,
so a backward must follow its own forward on the same handle.
"""

import numpy as np
import torch


class HomogenizedObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, density, solver, phase, table, simp_p, macro, n_increments, w_stress, w_energy):
        solver.set_material(phase, table, density.detach(), simp_p)
        solver.reset()
        out, psi, st = solver.solve(macro, n_increments)
        ws = np.asarray(w_stress, dtype=np.float64)
        ctx.solver = solver
        ctx.w = (ws, float(w_energy))
        ctx.stats = st
        return torch.tensor(float(w_energy) * psi + float(np.dot(ws, out)), dtype=torch.float64,
                            device=density.device)

    @staticmethod
    def backward(ctx, grad_out):
        ws, we = ctx.w
        g, _ = ctx.solver.adjoint(ws, we)
        return grad_out * g.reshape(ctx.solver.shape), None, None, None, None, None, None, None, None


def homogenized_objective(density, solver, phase, table, simp_p, macro, n_increments, w_stress, w_energy):
    return HomogenizedObjective.apply(density, solver, phase, table, simp_p, macro, n_increments, w_stress,
                                      w_energy)
