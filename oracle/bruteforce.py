"""Dense displacement-formulation solve for tiny grids (oracle cross-check).

Independent of the projection operator and of CG: the fluctuating strain is
written as the discrete gradient of a periodic displacement u, built from
explicit DFT matrices (spectral derivative, Nyquist component zeroed on even
axes), and the total energy  sum_v psi_v(E-bar + grad u)  is minimised by a
dense Newton method with numpy.linalg.lstsq.  On the Fourier-Galerkin
discretisation (section 3) the compatible fields are exactly these gradients,
so the minimiser equals the Newton-CG solution.
"""

import numpy as np


def derivative_matrix(n, length):
    """Real n x n spectral derivative matrix  Re(W^-1 diag(i k) W)."""
    j = np.arange(n)
    W = np.exp(-2j * np.pi * np.outer(j, j) / n)
    k = np.array([m if 2 * m < n else (0 if 2 * m == n else m - n) for m in range(n)],
                 dtype=np.float64) * (2.0 * np.pi / length)
    D = (W.conj().T @ np.diag(1j * k) @ W) / n
    return D.real


def gradient_operators(shape, lengths=None):
    """Stack D[a] (N x N) differentiating a flattened C-order field along direction a."""
    d = len(shape)
    if lengths is None:
        lengths = (1.0,) * d
    ops = []
    for a in range(d):
        axis = d - 1 - a
        M = np.ones((1, 1))
        for ax in range(d):
            if ax == axis:
                M = np.kron(M, derivative_matrix(shape[ax], lengths[a]))
            else:
                M = np.kron(M, np.eye(shape[ax]))
        ops.append(M)
    return np.stack(ops)


def solve_displacement(problem, macro_tensor, max_iter=50, tol=1e-13):
    """Minimise the RVE energy over periodic displacements; returns the strain field."""
    d = problem.d
    N = problem.N
    D = gradient_operators(problem.shape, problem.lengths)
    lam = problem.lam.reshape(N)
    mu = problem.mu.reshape(N)
    mat = problem.mat
    small = problem.kinematics == "small"
    u = np.zeros((d, N))

    def field_of(u):
        H = np.einsum("jvw,iw->vij", D, u)
        if small:
            H = 0.5 * (H + np.swapaxes(H, -1, -2))
        return macro_tensor[None, :, :] + H

    step0 = None
    for _ in range(max_iter):
        E = field_of(u)
        S = mat.stress(E, lam, mu)
        K = mat.tangent_tensor(E, lam, mu)
        g = np.einsum("jvw,vaj->aw", D, S).reshape(d * N)
        Hs = np.einsum("jvw,vajbl,lvx->awbx", D, K, D).reshape(d * N, d * N)
        du = np.linalg.lstsq(Hs, -g, rcond=1e-12)[0].reshape(d, N)
        u += du
        step = np.linalg.norm(du)
        if step0 is None:
            step0 = max(step, 1e-300)
        if step <= tol * max(step0, np.linalg.norm(u)):
            break
    return field_of(u).reshape(problem.shape + (d, d))
