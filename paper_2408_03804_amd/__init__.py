"""MI355X-native Fourier-Galerkin Newton-CG homogenization (arXiv:2408.03804).

The compute path is the HIP shared library ``libfft_homog.so`` built from
``csrc/``; ``binding`` wraps its C ABI with ctypes.  Importing this package
does not load the library; the first use of the binding does, and raises if
the library has not been built.
"""

__all__ = ["binding", "workloads"]
