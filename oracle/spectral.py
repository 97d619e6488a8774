"""Wavevectors and the Fourier-Galerkin projection operator (oracle).

The paper (section 3, Fourier-Galerkin equilibrium equation) writes static
equilibrium on the periodic cell as  IFFT( G-hat(xi) : FFT(sigma) ) = 0  and
describes G only by its role: it maps an arbitrary strain field onto a
compatible one (periodic, curl-free), identically for small and finite strain;
its explicit form is left to the cited Fourier-Galerkin literature.  The
oracle therefore uses the orthogonal projection onto the discrete compatible
fields, mode by mode:

* finite strain (gradients of a periodic displacement):  A-hat -> (A-hat n) (x) n
* small strain (symmetrised gradients):
      A-hat -> n (x) (A-hat n) + (A-hat n) (x) n - (n . A-hat . n) n (x) n

with n = xi/|xi| and G-hat(0) = 0.  On an even axis the Nyquist index gets a
zero wavevector component (the spectral derivative of the real trigonometric
interpolant has no Nyquist part); the paper only uses odd grids.

Conventions: grid shape is (Ny, Nx) in 2D and (Nz, Ny, Nx) in 3D, x fastest.
Tensor index a = 0, 1, 2 is the x, y, z direction, i.e. spatial array axis
ndim-1-a.  Fields have shape (*grid, d, d).
"""

import numpy as np
from scipy import fft as _fft

# Threads of the library FFT (scipy.fft's pocketfft); the element-wise NumPy work is
# single-threaded either way.  Changed only to time the oracle on several host cores.
FFT_WORKERS = 1


def axis_wavenumbers(n, length):
    """Angular wavenumbers 2*pi*k/L of one axis in numpy.fft order, Nyquist -> 0."""
    k = np.arange(n, dtype=np.float64)
    signed = np.where(k < n / 2.0, k, k - n)
    if n % 2 == 0:
        signed[n // 2] = 0.0
    return 2.0 * np.pi * signed / float(length)


def wavevectors(shape, lengths=None):
    """xi[..., a] on the full complex spectrum grid, a = direction x, y, (z)."""
    d = len(shape)
    if lengths is None:
        lengths = (1.0,) * d
    xi = np.zeros(tuple(shape) + (d,))
    for a in range(d):
        axis = d - 1 - a
        k = axis_wavenumbers(shape[axis], lengths[a])
        bshape = [1] * d
        bshape[axis] = shape[axis]
        xi[..., a] = k.reshape(bshape)
    return xi


def unit_wavevectors(shape, lengths=None):
    xi = wavevectors(shape, lengths)
    norm = np.sqrt(np.sum(xi * xi, axis=-1))
    n = np.zeros_like(xi)
    nz = norm > 0.0
    n[nz] = xi[nz] / norm[nz][:, None]
    return n


def project_modes(Ahat, n, kinematics):
    """Apply G-hat(xi) mode by mode to complex tensor modes Ahat (*grid, d, d)."""
    An = np.einsum("...ij,...j->...i", Ahat, n)
    if kinematics == "finite":
        return An[..., :, None] * n[..., None, :]
    if kinematics == "small":
        s = np.einsum("...i,...i->...", n, An)
        out = An[..., :, None] * n[..., None, :] + n[..., :, None] * An[..., None, :]
        out -= s[..., None, None] * (n[..., :, None] * n[..., None, :])
        return out
    raise ValueError(kinematics)


def apply_G(A, kinematics, lengths=None):
    """G*A = IFFT(G-hat : FFT(A)) for a real tensor field A of shape (*grid, d, d)."""
    d = A.shape[-1]
    shape = A.shape[:-2]
    axes = tuple(range(d))
    n = unit_wavevectors(shape, lengths)
    Ahat = _fft.fftn(A, axes=axes, workers=FFT_WORKERS)
    return _fft.ifftn(project_modes(Ahat, n, kinematics), axes=axes, workers=FFT_WORKERS).real


def inner(A, B):
    """Frobenius inner product summed over all voxels (and load cases)."""
    return float(np.sum(A * B))
