"""ctypes binding of the C ABI in include/fft_homog.h.

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch provides the device workspace (a uint8 tensor owned by the handle's
Python object) and the stream (torch.cuda.current_stream()).  The functions
below carry the C names; ``FFTHomog`` bundles a handle with its workspace.

Grid arrays use numpy order (Ny, Nx) / (Nz, Ny, Nx), x fastest; the C
descriptor takes n = (Nx, Ny, Nz).
"""

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfft_homog.so")

SMALL_STRAIN, FINITE_STRAIN = 0, 1
LINEAR_ELASTIC, NEO_HOOKEAN, STVK, J2_PLASTIC = 0, 1, 2, 3
K_RECOMPUTE, K_STORED = 0, 1
FLAG_TANGENT, FLAG_DENSITY, FLAG_GRAPH, FLAG_PLANE_STRESS = 1, 2, 4, 8
FIELD_STRAIN, FIELD_STRESS, FIELD_ENERGY, FIELD_PLASTIC = 0, 1, 2, 3
MAX_RECORDED = 256

STATUS = {0: "ok", 1: "einval", 2: "enotconv", 3: "edomain", 4: "ebreakdown", 5: "estate",
          6: "eunsupported", 7: "edevice", 8: "eworkspace"}
MATERIALS = {"linear_elastic": LINEAR_ELASTIC, "neo_hookean": NEO_HOOKEAN, "stvk": STVK, "j2_plastic": J2_PLASTIC}


class Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("n", ctypes.c_int * 3),
        ("len", ctypes.c_double * 3),
        ("kinematics", ctypes.c_int),
        ("material", ctypes.c_int),
        ("nphase", ctypes.c_int),
        ("tol_newton", ctypes.c_double),
        ("tol_cg", ctypes.c_double),
        ("max_newton", ctypes.c_int),
        ("max_cg", ctypes.c_int),
        ("k_mode", ctypes.c_int),
        ("flags", ctypes.c_uint),
        ("batch", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("increments", ctypes.c_int),
        ("newton_iterations", ctypes.c_int),
        ("cg_iterations", ctypes.c_int),
        ("newton_residual", ctypes.c_double),
        ("cg_residual", ctypes.c_double),
        ("seconds", ctypes.c_double),
        ("n_recorded", ctypes.c_int),
        ("cg_per_newton", ctypes.c_int * MAX_RECORDED),
        ("host_checks", ctypes.c_int),
    ]

    def as_dict(self):
        return {
            "status": STATUS.get(self.status, str(self.status)),
            "increments": self.increments,
            "newton": self.newton_iterations,
            "cg_total": self.cg_iterations,
            "cg": list(self.cg_per_newton[: self.n_recorded]),
            "newton_residual": self.newton_residual,
            "cg_residual": self.cg_residual,
            "seconds": self.seconds,
            "host_checks": self.host_checks,
        }


EXPORTS = [
    "fft_homog_workspace_size", "fft_homog_create", "fft_homog_set_material", "fft_homog_solve",
    "fft_homog_tangent", "fft_homog_adjoint", "fft_homog_get_field", "fft_homog_set_field",
    "fft_homog_destroy", "fft_homog_strerror", "fft_homog_last_error",
    "fft_homog_debug_constitutive", "fft_homog_debug_rfft", "fft_homog_debug_irfft",
    "fft_homog_debug_project", "fft_homog_debug_apply_operator", "fft_homog_debug_cg",
    "fft_homog_debug_cg_chunk", "fft_homog_debug_time_cg",
    "fft_homog_set_kernel_timing", "fft_homog_get_kernel_timing",
    "fft_homog_get_launch_shape", "fft_homog_set_launch_shape", "fft_homog_autotune", "fft_homog_tune_placement",
    "fft_homog_set_placement",
    "fft_homog_project_noalloc",
]

_lib = None


def load_library(path=LIB_PATH):
    """Load libfft_homog.so; raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libfft_homog.so is not built (expected at %s); run "
                           "`python -m paper_2408_03804_amd.build`" % path)
    # torch ships its own HIP runtime; load it first so that the library binds to
    # the same runtime instance as the tensors and streams it is given
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    DP = ctypes.POINTER(ctypes.c_double)
    sig = {
        "fft_homog_workspace_size": (I, [ctypes.POINTER(Desc), ctypes.POINTER(S)]),
        "fft_homog_create": (I, [ctypes.POINTER(Desc), P, S, P, ctypes.POINTER(P)]),
        "fft_homog_set_material": (I, [P, P, DP, P, D]),
        "fft_homog_solve": (I, [P, DP, I, DP, DP, ctypes.POINTER(Stats)]),
        "fft_homog_tangent": (I, [P, DP, ctypes.POINTER(Stats)]),
        "fft_homog_adjoint": (I, [P, DP, D, P, ctypes.POINTER(Stats)]),
        "fft_homog_get_field": (I, [P, I, P]),
        "fft_homog_set_field": (I, [P, P, DP]),
        "fft_homog_destroy": (None, [P]),
        "fft_homog_strerror": (ctypes.c_char_p, [I]),
        "fft_homog_last_error": (ctypes.c_char_p, [P]),
        "fft_homog_debug_constitutive": (I, [P, P, P, P, P, P]),
        "fft_homog_debug_rfft": (I, [P, P, P, I]),
        "fft_homog_debug_irfft": (I, [P, P, P, I]),
        "fft_homog_debug_project": (I, [P, P, P, I]),
        "fft_homog_debug_apply_operator": (I, [P, P, P, I]),
        "fft_homog_debug_cg": (I, [P, I, P, P]),
        "fft_homog_debug_cg_chunk": (I, [I, D, D, D, I, D]),
        "fft_homog_debug_time_cg": (I, [P, I, DP]),
        "fft_homog_set_kernel_timing": (I, [P, I]),
        "fft_homog_get_kernel_timing": (I, [P, DP, ctypes.POINTER(ctypes.c_longlong)]),
        "fft_homog_get_launch_shape": (I, [P, ctypes.POINTER(I)]),
        "fft_homog_set_launch_shape": (I, [P, ctypes.POINTER(I)]),
        "fft_homog_autotune": (I, [P, I, ctypes.POINTER(I)]),
        "fft_homog_tune_placement": (I, [P, I, ctypes.POINTER(S)]),
        "fft_homog_set_placement": (I, [P, S]),
        "fft_homog_project_noalloc": (I, [ctypes.POINTER(Desc), P, P, I, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class FFTHomogError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS.get(code, code), msg))
        self.code = code
        self.status = STATUS.get(code, str(code))


def _shape_dict(s):
    return {"x_rows": s[0], "y_bins": s[1], "outer_bins": s[2], "x_regs": s[3], "y_regs": s[4], "outer_regs": s[5],
            "spectrum_pitch": s[6]}


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _tptr(t):
    return ctypes.c_void_p(t.data_ptr())


def make_desc(shape, kinematics, material, nphase, tol_newton=1e-10, tol_cg=1e-10, max_newton=50,
              max_cg=10000, k_mode=K_RECOMPUTE, tangent=False, density=False, lengths=None, graph=False,
              batch=1, plane_stress=False):
    d = Desc()
    shape = tuple(int(s) for s in shape)
    d.ndim = len(shape)
    n = list(reversed(shape)) + [1] * (3 - len(shape))
    for a in range(3):
        d.n[a] = n[a]
        d.len[a] = 1.0 if lengths is None or a >= len(lengths) else float(lengths[a])
    d.kinematics = SMALL_STRAIN if kinematics == "small" else FINITE_STRAIN
    d.material = MATERIALS[material] if isinstance(material, str) else int(material)
    d.nphase = int(nphase)
    d.tol_newton = float(tol_newton)
    d.tol_cg = float(tol_cg)
    d.max_newton = int(max_newton)
    d.max_cg = int(max_cg)
    d.k_mode = int(k_mode)
    d.flags = (FLAG_TANGENT if tangent else 0) | (FLAG_DENSITY if density else 0) | (FLAG_GRAPH if graph else 0) \
        | (FLAG_PLANE_STRESS if plane_stress else 0)
    d.batch = int(batch)
    return d


def fft_homog_workspace_size(desc):
    L = load_library()
    nbytes = ctypes.c_size_t(0)
    rc = L.fft_homog_workspace_size(ctypes.byref(desc), ctypes.byref(nbytes))
    if rc:
        raise FFTHomogError(rc, L.fft_homog_strerror(rc).decode())
    return nbytes.value


class FFTHomog:
    """One solver handle (fft_homog_create) plus its torch-owned device workspace."""

    def __init__(self, shape, kinematics, material, nphase, device=None, stream=None, **kw):
        import torch

        self.torch = torch
        self.L = load_library()
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.kinematics = kinematics
        self.c = (3 if self.ndim == 2 else 6) if kinematics == "small" else self.ndim * self.ndim
        self.N = int(np.prod(self.shape))
        self.desc = make_desc(shape, kinematics, material, nphase, **kw)
        self.cells = max(1, int(kw.get("batch", 1)))
        self.batch_max = self.c * self.cells if kw.get("tangent") else 1
        self.device = torch.device(device if device is not None else "cuda")
        nbytes = fft_homog_workspace_size(self.desc)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        rc = self.L.fft_homog_create(ctypes.byref(self.desc), ctypes.c_void_p(self._ws_ptr), nbytes,
                                     ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if rc:
            msg = self.L.fft_homog_last_error(None)
            raise FFTHomogError(rc, "fft_homog_create: " + (msg.decode() if msg else ""))
        self.h = h

    # ------------------------------------------------------------------ helpers
    def _check(self, rc, allow=()):
        if rc and rc not in allow:
            msg = self.L.fft_homog_last_error(self.h)
            raise FFTHomogError(rc, msg.decode() if msg else "")
        return rc

    def _dev(self, a, dtype):
        """A device copy (or view) of `a` that the handle's stream may read: made on the handle's
        stream, after the work already queued on the caller's current stream."""
        t = self.torch
        cur = t.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)
        with t.cuda.stream(self.stream):
            if isinstance(a, t.Tensor):
                return a.to(device=self.device, dtype=dtype).contiguous()
            return t.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=self.device)

    def close(self):
        if getattr(self, "h", None):
            self.L.fft_homog_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ C ABI
    def set_material(self, phase, table, density=None, simp_p=3.0):
        ph = self._dev(phase, self.torch.uint8)
        assert ph.numel() == self.N * self.cells
        tab = np.ascontiguousarray(table, dtype=np.float64)
        assert tab.size == (4 if self.desc.material == J2_PLASTIC else 2) * self.desc.nphase * self.cells
        den = None if density is None else self._dev(density, self.torch.float64)
        self._keep = (ph, den)
        rc = self.L.fft_homog_set_material(self.h, _tptr(ph), _dptr(tab),
                                           None if den is None else _tptr(den), float(simp_p))
        self._check(rc)

    def solve(self, macro, n_increments=1, allow=()):
        m = np.ascontiguousarray(macro, dtype=np.float64)
        assert m.shape == (self.c,)
        out = np.zeros(self.c)
        en = ctypes.c_double(0.0)
        st = Stats()
        rc = self.L.fft_homog_solve(self.h, _dptr(m), int(n_increments), _dptr(out), ctypes.byref(en),
                                    ctypes.byref(st))
        self._check(rc, allow)
        return out, en.value, st.as_dict()

    def tangent(self, allow=()):
        """(c, c) tangent; (batch, c, c) on a multi-cell handle."""
        C = np.zeros((self.cells, self.c, self.c))
        st = Stats()
        rc = self.L.fft_homog_tangent(self.h, _dptr(C), ctypes.byref(st))
        self._check(rc, allow)
        return (C[0] if self.cells == 1 else C), st.as_dict()

    def launch_shape(self):
        s = (ctypes.c_int * 7)()
        self._check(self.L.fft_homog_get_launch_shape(self.h, s))
        return _shape_dict(s)

    def set_launch_shape(self, shape):
        keys = ["x_rows", "y_bins", "outer_bins", "x_regs", "y_regs", "outer_regs", "spectrum_pitch"]
        s = (ctypes.c_int * 7)(*[int(shape[k]) for k in keys])
        self._check(self.L.fft_homog_set_launch_shape(self.h, s))

    def autotune(self, reps=10):
        s = (ctypes.c_int * 7)()
        self._check(self.L.fft_homog_autotune(self.h, int(reps), s))
        return _shape_dict(s)

    def tune_placement(self, reps=10):
        """Time the work-vector placements and keep the fastest; returns the chosen stagger (bytes)."""
        s = ctypes.c_size_t(0)
        self._check(self.L.fft_homog_tune_placement(self.h, int(reps), ctypes.byref(s)))
        return int(s.value)

    def set_placement(self, stagger):
        self._check(self.L.fft_homog_set_placement(self.h, int(stagger)))

    def reset(self):
        """Back to the undeformed reference state (eps = 0 / F = I) with zero macro load."""
        d = self.ndim
        with self.torch.cuda.stream(self.stream):
            # made on the stream that set_field's kernels run on
            ref = self.torch.zeros((d * d,) + self.shape, dtype=self.torch.float64, device=self.device)
            if self.kinematics != "small":
                for i in range(d):
                    ref[i * d + i] = 1.0
        macro = np.eye(d).reshape(-1) if self.kinematics != "small" else np.zeros(self.c)
        self.set_field(ref, macro)

    def adjoint(self, w_stress, w_energy):
        w = np.ascontiguousarray(w_stress, dtype=np.float64)
        g = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        st = Stats()
        rc = self.L.fft_homog_adjoint(self.h, _dptr(w), float(w_energy), _tptr(g), ctypes.byref(st))
        self._check(rc)
        return g, st.as_dict()

    def get_field(self, which):
        d = self.ndim
        shape = self.shape if which in (FIELD_ENERGY, FIELD_PLASTIC) else (d, d) + self.shape
        out = self.torch.empty(shape, dtype=self.torch.float64, device=self.device)
        self._check(self.L.fft_homog_get_field(self.h, int(which), _tptr(out)))
        return out

    def set_field(self, full, macro):
        f = self._dev(full, self.torch.float64)
        m = np.ascontiguousarray(macro, dtype=np.float64)
        self._check(self.L.fft_homog_set_field(self.h, _tptr(f), _dptr(m)))

    # ------------------------------------------------------------------ stages (tests)
    def debug_constitutive(self, e, de):
        e = self._dev(e, self.torch.float64)
        de = self._dev(de, self.torch.float64)
        P = self.torch.empty_like(e)
        K = self.torch.empty_like(e)
        psi = self.torch.empty(self.shape, dtype=self.torch.float64, device=self.device)
        self._check(self.L.fft_homog_debug_constitutive(self.h, _tptr(e), _tptr(de), _tptr(P), _tptr(K), _tptr(psi)))
        return P, K, psi

    def debug_rfft(self, x):
        x = self._dev(x, self.torch.float64)
        batch = x.numel() // (self.c * self.N)
        hs = self.shape[:-1] + (self.shape[-1] // 2 + 1,)
        spec = self.torch.empty((batch, self.c) + hs, dtype=self.torch.complex128, device=self.device)
        self._check(self.L.fft_homog_debug_rfft(self.h, _tptr(x), _tptr(spec), batch))
        return spec

    def debug_irfft(self, spec):
        spec = self._dev(spec, self.torch.complex128)
        hs = self.shape[:-1] + (self.shape[-1] // 2 + 1,)
        batch = spec.numel() // (self.c * int(np.prod(hs)))
        out = self.torch.empty((batch, self.c) + self.shape, dtype=self.torch.float64, device=self.device)
        self._check(self.L.fft_homog_debug_irfft(self.h, _tptr(spec), _tptr(out), batch))
        return out

    def debug_project(self, x):
        x = self._dev(x, self.torch.float64)
        batch = x.numel() // (self.c * self.N)
        out = self.torch.empty_like(x)
        self._check(self.L.fft_homog_debug_project(self.h, _tptr(x), _tptr(out), batch))
        return out

    def debug_apply_operator(self, p):
        p = self._dev(p, self.torch.float64)
        batch = p.numel() // (self.c * self.N)
        q = self.torch.empty_like(p)
        self._check(self.L.fft_homog_debug_apply_operator(self.h, _tptr(p), _tptr(q), batch))
        return q

    def debug_cg(self, iters):
        """(x, r) after exactly `iters` CG iterations on the Newton system at the current state
        (packed layout (c, *grid))."""
        x = self.torch.empty((self.c,) + self.shape, dtype=self.torch.float64, device=self.device)
        r = self.torch.empty_like(x)
        self._check(self.L.fft_homog_debug_cg(self.h, int(iters), _tptr(x), _tptr(r)))
        return x, r

    def debug_time_cg(self, iters):
        ms = np.zeros(7)
        self._check(self.L.fft_homog_debug_time_cg(self.h, int(iters), _dptr(ms)))
        return ms

    def set_kernel_timing(self, every):
        """Sample every `every`-th CG iteration of later solves with HIP events (0: off)."""
        self._check(self.L.fft_homog_set_kernel_timing(self.h, int(every)))

    def kernel_timing(self):
        """(ms[7] per launch of a CG iteration averaged over the samples, number of samples)."""
        ms = np.zeros(7)
        n = ctypes.c_longlong(0)
        self._check(self.L.fft_homog_get_kernel_timing(self.h, _dptr(ms), ctypes.byref(n)))
        return ms, int(n.value)


# module-level functions with the C names (thin pass-throughs on a handle object)
def fft_homog_create(shape, kinematics, material, nphase, **kw):
    return FFTHomog(shape, kinematics, material, nphase, **kw)


def fft_homog_set_material(h, phase, table, density=None, simp_p=3.0):
    return h.set_material(phase, table, density, simp_p)


def fft_homog_solve(h, macro, n_increments=1):
    return h.solve(macro, n_increments)


def fft_homog_tangent(h):
    return h.tangent()


def fft_homog_adjoint(h, w_stress, w_energy):
    return h.adjoint(w_stress, w_energy)


def fft_homog_get_field(h, which):
    return h.get_field(which)


def fft_homog_set_field(h, full, macro):
    return h.set_field(full, macro)


def fft_homog_project_noalloc(desc, x, out, stream=None):
    """out = G*x through the allocation-free entry point: x and out are device float64 tensors of
    shape (batch, c, *grid) (packed layout), enqueued on `stream` (default: the current stream)
    with no synchronisation; raises FFTHomogError on a non-zero status."""
    import torch

    L = load_library()
    assert x.dtype == torch.float64 and out.dtype == torch.float64 and x.is_contiguous() and out.is_contiguous()
    assert x.shape == out.shape and x.dim() >= 2
    s = stream if stream is not None else torch.cuda.current_stream(x.device)
    rc = L.fft_homog_project_noalloc(ctypes.byref(desc), _tptr(x), _tptr(out), int(x.shape[0]),
                                     ctypes.c_void_p(s.cuda_stream))
    if rc:
        msg = L.fft_homog_last_error(None)
        raise FFTHomogError(rc, "fft_homog_project_noalloc: " + (msg.decode() if msg else ""))
    return out


def fft_homog_get_launch_shape(h):
    return h.launch_shape()


def fft_homog_autotune(h, reps=10):
    return h.autotune(reps)


def fft_homog_destroy(h):
    h.close()
