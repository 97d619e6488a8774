"""Plain CPU FP64 oracle for the Fourier-Galerkin Newton-CG homogenization solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this package.
The product path (the HIP library and its Python binding) never imports it, and
this package never imports the product package: the two share no code.

Everything here is written for a reader who checks it against the paper
(Pundir & Kammer, "Simplifying FFT-based methods for solid mechanics with
automatic differentiation", arXiv:2408.03804) by eye:

* full d x d tensors everywhere (no Voigt or Mandel packing inside the solver),
* ``scipy.fft.fftn``/``ifftn`` on the full complex spectrum (one thread unless a timing run sets
  ``spectral.FFT_WORKERS``),
* closed-form stress and tangent (the paper's "analytical implementation"),
* textbook conjugate gradients and the Newton loop of Appendix A, Algorithm 1.

Modules
-------
spectral     wavevectors, the projection operator G-hat, G*A = IFFT(G-hat : FFT(A))
materials    energy density, stress and tangent in closed form
newton_cg    Newton-CG solve, homogenized stress/energy and homogenized tangent
bruteforce   dense displacement-formulation solve for tiny grids (independent of G and CG)
closed_forms isotropic stiffness, exact laminate, Voigt/Reuss bounds
adjoint      gradient of homogenized energy/stress w.r.t. a per-voxel SIMP density
plasticity   J2 return mapping, consistent tangent and history (Appendix B), the RVE problem
surrogate    forward pass, loss gradient and Adam step of the stiffness surrogate network

Parity status: every function above is pinned by the CPU tests in
``tests/test_oracle_pins.py``, ``tests/test_oracle_plasticity.py`` and
``tests/test_oracle_surrogate.py``; none is "parity unpinned".
"""

from . import spectral, materials, newton_cg, bruteforce, closed_forms, adjoint, plasticity, surrogate  # noqa: F401
