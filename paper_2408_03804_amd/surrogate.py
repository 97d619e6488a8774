"""ctypes binding of include/fft_homog_cnn.h and the stiffness-surrogate workflow around it.

``CNN`` marshals arguments to the C ABI (every layer, the backward pass and the
optimizer run in the HIP library).  ``StiffnessSurrogate`` holds the data
conventions: input = phase indicator of an n^3 cell plus log(E2/E1); output =
the position of the 6x6 homogenized stiffness between the cell's Reuss and
Voigt bounds, y = (C - C_Reuss) / |C_Voigt - C_Reuss|_F on the 21 upper-triangle
components (C lies between the bounds, so y is O(1); the prediction's error in C
is that of y times the bounds' gap, which vanishes as the phase contrast goes to
one), standardised per component during training and un-standardised by folding
the scales into the last layer afterwards; the forward pass then returns
C = C_Reuss + gap * y.  Samples that fft_homog_cnn_check rejects go to the
FP64 solver (multi-cell tangent handles).
"""

import ctypes
import math

import numpy as np

from . import binding

CHANNELS = (1, 32, 64, 128, 256)
UPPER = [(i, j) for i in range(6) for j in range(i, 6)]


class CnnDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("channels", ctypes.c_int * 5), ("hidden", ctypes.c_int),
                ("n_feat", ctypes.c_int), ("n_out", ctypes.c_int), ("max_batch", ctypes.c_int)]


CNN_EXPORTS = ["fft_homog_cnn_param_count", "fft_homog_cnn_workspace_size", "fft_homog_cnn_create",
               "fft_homog_cnn_set_params", "fft_homog_cnn_get_params", "fft_homog_cnn_forward",
               "fft_homog_cnn_loss_grad", "fft_homog_cnn_adam_step", "fft_homog_cnn_check",
               "fft_homog_cnn_last_ms", "fft_homog_cnn_destroy", "fft_homog_cnn_debug_gemm"]

_lib = None


def load_library():
    global _lib
    if _lib is not None:
        return _lib
    L = binding.load_library()
    P, I, F, S, LL = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_size_t, ctypes.c_longlong
    D = ctypes.POINTER(CnnDesc)
    sig = {
        "fft_homog_cnn_param_count": (I, [D, ctypes.POINTER(S)]),
        "fft_homog_cnn_workspace_size": (I, [D, ctypes.POINTER(S)]),
        "fft_homog_cnn_create": (I, [D, P, S, P, ctypes.POINTER(P)]),
        "fft_homog_cnn_set_params": (I, [P, P]),
        "fft_homog_cnn_get_params": (I, [P, P]),
        "fft_homog_cnn_forward": (I, [P, P, P, P, P, P, I]),
        "fft_homog_cnn_loss_grad": (I, [P, P, P, P, I, ctypes.POINTER(F), P]),
        "fft_homog_cnn_adam_step": (I, [P, F, F, F, F]),
        "fft_homog_cnn_check": (I, [P, P, P, P, P, P, I, F, F, F, F, P, P]),
        "fft_homog_cnn_last_ms": (I, [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
        "fft_homog_cnn_destroy": (None, [P]),
        "fft_homog_cnn_debug_gemm": (I, [P, I, I, I, P, LL, LL, P, LL, LL, P, I]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def make_desc(n=32, channels=CHANNELS, hidden=256, n_feat=1, n_out=21, max_batch=256):
    d = CnnDesc()
    d.n = int(n)
    for i in range(5):
        d.channels[i] = int(channels[i])
    d.hidden, d.n_feat, d.n_out, d.max_batch = int(hidden), int(n_feat), int(n_out), int(max_batch)
    return d


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class CNN:
    """One surrogate network handle with its torch-owned device workspace."""

    def __init__(self, n=32, channels=CHANNELS, hidden=256, n_feat=1, n_out=21, max_batch=256, device=None,
                 stream=None):
        import torch

        self.torch = torch
        self.L = load_library()
        self.desc = make_desc(n, channels, hidden, n_feat, n_out, max_batch)
        self.n, self.channels, self.hidden, self.n_feat, self.n_out = n, tuple(channels), hidden, n_feat, n_out
        self.max_batch = max_batch
        self.device = torch.device(device if device is not None else "cuda")
        cnt, nbytes = ctypes.c_size_t(0), ctypes.c_size_t(0)
        self._check(self.L.fft_homog_cnn_param_count(ctypes.byref(self.desc), ctypes.byref(cnt)))
        self._check(self.L.fft_homog_cnn_workspace_size(ctypes.byref(self.desc), ctypes.byref(nbytes)))
        self.n_params = cnt.value
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        self._check(self.L.fft_homog_cnn_create(ctypes.byref(self.desc), ctypes.c_void_p(ptr), nbytes.value,
                                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h

    def _check(self, rc):
        if rc:
            raise binding.FFTHomogError(rc, "surrogate call failed")

    def close(self):
        if getattr(self, "h", None):
            self.L.fft_homog_cnn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f32(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=t.float32).contiguous()
        return t.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=self.device)

    def _u8(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=t.uint8).contiguous()
        return t.as_tensor(np.ascontiguousarray(a, dtype=np.uint8), device=self.device)

    def set_params(self, theta):
        th = self._f32(theta)
        assert th.numel() == self.n_params
        self._check(self.L.fft_homog_cnn_set_params(self.h, _p(th)))

    def get_params(self):
        out = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.device)
        self._check(self.L.fft_homog_cnn_get_params(self.h, _p(out)))
        return out

    def forward(self, phase, feat, out_scale=None, out_offset=None):
        ph = self._u8(phase)
        B = ph.shape[0]
        ft = self._f32(feat).reshape(B, self.n_feat) if self.n_feat else None
        sc = None if out_scale is None else self._f32(out_scale).reshape(B)
        of = None if out_offset is None else self._f32(out_offset).reshape(B, self.n_out)
        out = self.torch.empty((B, self.n_out), dtype=self.torch.float32, device=self.device)
        self._check(self.L.fft_homog_cnn_forward(self.h, _p(ph), _p(ft), _p(sc), _p(of), _p(out), B))
        return out

    def loss_grad(self, phase, feat, target, want_grad=True):
        ph = self._u8(phase)
        B = ph.shape[0]
        ft = self._f32(feat).reshape(B, self.n_feat) if self.n_feat else None
        tg = self._f32(target).reshape(B, self.n_out)
        g = self.torch.empty(self.n_params, dtype=self.torch.float32, device=self.device) if want_grad else None
        loss = ctypes.c_float(0.0)
        self._check(self.L.fft_homog_cnn_loss_grad(self.h, _p(ph), _p(ft), _p(tg), B, ctypes.byref(loss), _p(g)))
        return loss.value, g

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.L.fft_homog_cnn_adam_step(self.h, float(lr), float(beta1), float(beta2), float(eps)))

    def check(self, phase, lam_mu, feat, C21, tol=0.0, feat_lo=-1e30, feat_hi=1e30, C2=None, max_spread=1e30,
              want_spread=False):
        """Indicator per sample (and, with want_spread, the members' spread per sample); with C2, C21
        (a device f32 tensor) is replaced by the ensemble mean."""
        ph = self._u8(phase)
        B = ph.shape[0]
        lm = self._f32(lam_mu).reshape(B, 4)
        ft = self._f32(feat).reshape(B, self.n_feat) if self.n_feat else None
        C = C21 if isinstance(C21, self.torch.Tensor) and C21.dtype == self.torch.float32 and C21.is_cuda \
            and C21.is_contiguous() else self._f32(C21).reshape(B, 21)
        C2t = None if C2 is None else self._f32(C2).reshape(B, 21)
        ok = self.torch.empty(B, dtype=self.torch.int32, device=self.device)
        sp = self.torch.empty(B, dtype=self.torch.float32, device=self.device) if want_spread else None
        self._check(self.L.fft_homog_cnn_check(self.h, _p(ph), _p(lm), _p(ft), _p(C), _p(C2t), B, float(tol),
                                               float(feat_lo), float(feat_hi), float(max_spread), _p(ok), _p(sp)))
        return (ok, sp) if want_spread else ok

    def last_ms(self):
        f, t = ctypes.c_double(0), ctypes.c_double(0)
        self._check(self.L.fft_homog_cnn_last_ms(self.h, ctypes.byref(f), ctypes.byref(t)))
        return f.value, t.value

    def debug_gemm(self, M, N, K, A, sam, sak, B, sbn, sbk, splits=1):
        """A, B: torch bfloat16 device tensors addressed with the given element strides."""
        C = self.torch.empty((splits, M, N), dtype=self.torch.float32, device=self.device)
        self._check(self.L.fft_homog_cnn_debug_gemm(self.h, M, N, K, _p(A), sam, sak, _p(B), sbn, sbk, _p(C), splits))
        return C


def init_params(n_params_shapes, seed=0):
    """He-uniform weights (fan-in), zero biases; n_params_shapes: ordered (name, shape) list."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shape in n_params_shapes:
        if name.startswith("W"):
            fan_in = int(np.prod(shape[1:]))
            lim = math.sqrt(6.0 / fan_in)
            out.append(rng.uniform(-lim, lim, size=int(np.prod(shape))))
        else:
            out.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(out).astype(np.float32)


def param_shapes(channels=CHANNELS, hidden=256, n_feat=1, n_out=21):
    shapes = []
    for l in range(1, 5):
        shapes.append(("W%d" % l, (channels[l], 27, channels[l - 1])))
        shapes.append(("b%d" % l, (channels[l],)))
    shapes += [("W5", (hidden, channels[4] + n_feat)), ("b5", (hidden,)), ("W6", (n_out, hidden)), ("b6", (n_out,))]
    return shapes


def upper21(C):
    C = np.asarray(C)
    return np.stack([C[..., i, j] for i, j in UPPER], axis=-1)


def full6(v):
    v = np.asarray(v)
    C = np.zeros(v.shape[:-1] + (6, 6))
    for k, (i, j) in enumerate(UPPER):
        C[..., i, j] = C[..., j, i] = v[..., k]
    return C


class StiffnessSurrogate:
    """Train on solver tangents, predict with the CNN ensemble, fall back to the solver when the check trips.

    ``members`` networks are trained from different initialisations and batch orders; the
    prediction is their mean, and with two members their disagreement is part of the
    error indicator (fft_homog_cnn_check).
    """

    def __init__(self, n=32, max_batch=256, device=None, seed=0, channels=CHANNELS, hidden=256, members=1):
        assert members in (1, 2)
        self.nets = [CNN(n=n, channels=channels, hidden=hidden, n_feat=1, n_out=21, max_batch=max_batch, device=device)
                     for _ in range(members)]
        self.net = self.nets[0]
        self.n = n
        self.seed = seed
        self.shapes = param_shapes(channels, hidden, 1, 21)
        for i, net in enumerate(self.nets):
            net.set_params(init_params(self.shapes, seed + 1000 * i))
        self.mean = np.zeros(21)
        self.std = np.ones(21)
        self.feat_range = (-np.inf, np.inf)
        self.folded = False
        # indicator settings: bounds slack and members' spread limit (calibrate() sets the latter)
        self.tol = 0.02
        self.max_spread = 0.03

    @staticmethod
    def features(tables):
        """log(E2/E1) from per-cell (lam, mu) tables [S, 2, 2]; E from mu (nu fixed): E2/E1 = mu2/mu1."""
        t = np.asarray(tables, dtype=np.float64)
        return np.log(t[:, 1, 1] / t[:, 0, 1])[:, None]

    @staticmethod
    def bounds(tables, fractions):
        """Voigt and Reuss bounds (6x6 Voigt matrices, engineering shear) of two-phase cells with
        isotropic phases (lam, mu) and stiff volume fraction f: arithmetic means of lam and mu, and
        harmonic means of the bulk and shear moduli."""
        t = np.asarray(tables, dtype=np.float64)
        f = np.asarray(fractions, dtype=np.float64)
        f0 = 1.0 - f
        l0, m0, l1, m1 = t[:, 0, 0], t[:, 0, 1], t[:, 1, 0], t[:, 1, 1]
        lv, mv = f0 * l0 + f * l1, f0 * m0 + f * m1
        k0, k1 = l0 + 2.0 * m0 / 3.0, l1 + 2.0 * m1 / 3.0
        kr, mr = 1.0 / (f0 / k0 + f / k1), 1.0 / (f0 / m0 + f / m1)
        lr = kr - 2.0 * mr / 3.0

        def iso(lam, mu):
            C = np.zeros(lam.shape + (6, 6))
            C[:, :3, :3] = lam[:, None, None]
            for i in range(3):
                C[:, i, i] += 2.0 * mu
                C[:, 3 + i, 3 + i] = mu
            return C
        return iso(lv, mv), iso(lr, mr)

    @classmethod
    def reference(cls, tables, fractions):
        """(C_Reuss upper triangle [S, 21], |C_Voigt - C_Reuss|_F [S]) of each cell: the output offset
        and scale of the network."""
        CV, CR = cls.bounds(tables, fractions)
        gap = np.linalg.norm((CV - CR).reshape(len(CV), -1), axis=1)
        gap = np.maximum(gap, 1e-12 * np.linalg.norm(CV.reshape(len(CV), -1), axis=1))
        return upper21(CR), gap

    @staticmethod
    def fractions(phase):
        """Stiff volume fraction of each cell (phase maps on the device)."""
        return phase.reshape(phase.shape[0], -1).float().mean(dim=1).double().cpu().numpy()

    def fit(self, phase, tables, C, epochs=30, batch=256, lr=1e-3, lr_end=1e-5, log=None):
        """phase: device uint8 [S, n, n, n]; tables [S, 2, 2] (lam, mu); C [S, 6, 6] solver tangents."""
        torch = self.net.torch
        feat = self.features(tables)
        ref, gap = self.reference(tables, self.fractions(phase))
        y = (upper21(C) - ref) / gap[:, None]
        self.mean = y.mean(axis=0)
        self.std = y.std(axis=0) + 1e-12
        # inputs are trusted where the training data is dense: the central 95 % of its contrasts
        self.feat_range = (float(np.percentile(feat, 2.5)), float(np.percentile(feat, 97.5)))
        yt = torch.as_tensor(((y - self.mean) / self.std).astype(np.float32), device=self.net.device)
        ft = torch.as_tensor(feat.astype(np.float32), device=self.net.device)
        S = phase.shape[0]
        steps = epochs * (S // batch)
        hist = []
        for i, net in enumerate(self.nets):
            rng = np.random.default_rng(self.seed + 1000 * i)
            k = 0
            h = []
            for ep in range(epochs):
                perm = torch.as_tensor(rng.permutation(S), device=self.net.device)
                tot = 0.0
                for s in range(0, S - batch + 1, batch):
                    idx = perm[s:s + batch]
                    loss, _ = net.loss_grad(phase[idx], ft[idx], yt[idx], want_grad=False)
                    # cosine decay of the learning rate
                    lr_k = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * k / max(1, steps)))
                    net.adam_step(lr_k)
                    tot += loss
                    k += 1
                h.append(tot / max(1, S // batch))
                if log:
                    log("member %d epoch %d loss %.4e" % (i, ep, h[-1]))
            hist.append(h)
        return hist

    def fold(self):
        """Fold the target standardisation into the last layer: the networks then output C21 / scale."""
        if self.folded:
            return
        for net in self.nets:
            th = net.get_params().cpu().numpy().astype(np.float64)
            off = 0
            offs = {}
            for name, shape in self.shapes:
                offs[name] = (off, int(np.prod(shape)), shape)
                off += int(np.prod(shape))
            o, m, shp = offs["W6"]
            th[o:o + m] = (th[o:o + m].reshape(shp) * self.std[:, None]).reshape(-1)
            o, m, _ = offs["b6"]
            th[o:o + m] = th[o:o + m] * self.std + self.mean
            net.set_params(th.astype(np.float32))
        self.folded = True

    def predict_checked(self, phase, tables, tol=None, max_spread=None, want_spread=False):
        """C21 (absolute units; the ensemble mean) of a batch of cells and the per-sample indicator
        (by default with the bounds slack and the calibrated spread limit of this surrogate)."""
        self.fold()
        torch = self.net.torch
        tol = self.tol if tol is None else tol
        max_spread = self.max_spread if max_spread is None else max_spread
        ft = torch.as_tensor(self.features(tables).astype(np.float32), device=self.net.device)
        ref, gap = self.reference(tables, self.fractions(phase))
        sc = torch.as_tensor(gap.astype(np.float32), device=self.net.device)
        of = torch.as_tensor(ref.astype(np.float32), device=self.net.device)
        C = self.nets[0].forward(phase, ft, sc, of)
        C2 = self.nets[1].forward(phase, ft, sc, of) if len(self.nets) > 1 else None
        lm = torch.as_tensor(np.asarray(tables, dtype=np.float32).reshape(-1, 4), device=self.net.device)
        res = self.net.check(phase, lm, ft, C, tol, self.feat_range[0], self.feat_range[1], C2=C2,
                             max_spread=max_spread, want_spread=want_spread)
        if want_spread:
            return C, res[0], res[1]
        return C, res

    def calibrate(self, phase, tables, C_true, target=0.02, safety=0.8):
        """Set the members' spread limit from held-out cells with known tangents (cells used neither
        for training nor for reporting): the largest limit at which every calibration cell the
        indicator accepts has a relative Frobenius error of at most safety * target.  The other
        tests (positive definiteness, bounds, contrast range) keep their settings.  Returns the
        calibration statistics."""
        assert len(self.nets) == 2, "the spread test needs two members"
        C, ok, sp = self.predict_checked(phase, tables, max_spread=1e30, want_spread=True)
        Cp = full6(C.cpu().numpy().astype(np.float64))
        Ct = np.asarray(C_true, dtype=np.float64)
        n = Ct.shape[0]
        err = np.linalg.norm((Cp - Ct).reshape(n, -1), axis=1) / np.linalg.norm(Ct.reshape(n, -1), axis=1)
        ok = ok.cpu().numpy().astype(bool)
        sp = sp.cpu().numpy().astype(np.float32)
        bound = safety * target
        cand = np.nonzero(ok)[0]
        order = cand[np.argsort(sp[cand], kind="stable")]
        runmax = np.maximum.accumulate(err[order]) if order.size else np.zeros(0)
        # the last position whose running maximum is within the bound and whose spread differs from
        # the next one (a tie would admit the next cell too); the limit is that spread, which the
        # kernel compares in double, so a borderline cell may only be rejected, never admitted
        ssorted = sp[order]
        distinct = np.append(ssorted[1:] > ssorted[:-1], True) if order.size else np.zeros(0, bool)
        good = np.nonzero((runmax <= bound) & distinct)[0]
        self.max_spread = float(ssorted[good[-1]]) if good.size else 0.0
        acc = ok & (sp <= np.float32(self.max_spread))
        return {"max_spread": self.max_spread, "target": target, "safety": safety, "cells": int(n),
                "accepted": int(acc.sum()),
                "accepted_max_error": float(err[acc].max()) if acc.any() else None,
                "all_max_error": float(err.max())}

    def indicator_parts(self, phase, tables, tol=None, max_spread=None):
        """Diagnostics: the indicator's three tests evaluated one at a time (bounds, spread, contrast range)."""
        self.fold()
        torch = self.net.torch
        ft = torch.as_tensor(self.features(tables).astype(np.float32), device=self.net.device)
        ref, gap = self.reference(tables, self.fractions(phase))
        sc = torch.as_tensor(gap.astype(np.float32), device=self.net.device)
        of = torch.as_tensor(ref.astype(np.float32), device=self.net.device)
        lm = torch.as_tensor(np.asarray(tables, dtype=np.float32).reshape(-1, 4), device=self.net.device)
        outs = [net.forward(phase, ft, sc, of) for net in self.nets]
        C2 = outs[1] if len(outs) > 1 else None
        mean = outs[0].clone() if C2 is None else 0.5 * (outs[0] + C2)
        tol = self.tol if tol is None else tol
        bounds = self.net.check(phase, lm, ft, mean, tol).cpu().numpy()
        spread = np.ones_like(bounds)
        max_spread = self.max_spread if max_spread is None else max_spread
        if C2 is not None:
            # a slack of 10 |C_Voigt| leaves only the positive definiteness of C and the spread
            spread = self.net.check(phase, lm, ft, outs[0].clone(), 10.0, C2=C2, max_spread=max_spread).cpu().numpy()
        f = self.features(tables)[:, 0]
        contrast = ((f >= self.feat_range[0]) & (f <= self.feat_range[1])).astype(int)
        return {"bounds": bounds.astype(bool), "spread": spread.astype(bool), "contrast": contrast.astype(bool)}

    def close(self):
        for net in self.nets:
            net.close()
