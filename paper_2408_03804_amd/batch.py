"""Homogenized tangents of many cells of uneven grid size.

Cells are grouped by grid shape.  Each group runs on multi-cell handles
(``desc.batch`` > 1): the ncomp unit-load tangent solves of every cell in a
chunk share each launch of the CG passes, so small grids still fill the GPU.
A group is split into chunks whose workspace fits ``max_bytes``.  Handles are
cached per (shape, chunk size); with ``graph`` the CG iterations replay a
captured HIP graph and with ``autotune`` each new handle picks its launch shape
by timing the candidates once.  Argument marshalling only: all arithmetic runs
in the HIP library.
"""

from collections import OrderedDict

import numpy as np

from . import binding

MAX_CELLS_PER_LAUNCH = 65535


class TangentBatcher:
    """With ``concurrent``, the grid-size groups run at the same time, each on its own stream
    (default priority) driven by its own host thread, so that one group's convergence tail
    overlaps the others' work.  Launch shapes are tuned beforehand, one group at a time."""

    def __init__(self, kinematics="small", material="linear_elastic", nphase=2, tol_cg=1e-10, max_cg=20000,
                 max_bytes=64 << 30, graph=True, autotune=True, device=None, stream=None, concurrent=False):
        self.kinematics = kinematics
        self.material = material
        self.nphase = int(nphase)
        self.kw = dict(tol_cg=tol_cg, max_cg=max_cg, tangent=True, graph=graph)
        self.max_bytes = int(max_bytes)
        self.autotune = autotune
        self.device = device
        self.stream = stream
        self.handles = OrderedDict()
        self.shapes = {}
        self.concurrent = concurrent
        self.streams = {}

    def _ncomp(self, shape):
        d = len(shape)
        return (3 if d == 2 else 6) if self.kinematics == "small" else d * d

    def chunk_size(self, shape, n):
        """Largest number of cells (<= n) of this shape whose workspace fits max_bytes."""
        c = self._ncomp(shape)
        hi = max(1, min(n, MAX_CELLS_PER_LAUNCH // (c * c)))

        def size(k):
            d = binding.make_desc(shape, self.kinematics, self.material, self.nphase, batch=k, **self.kw)
            return binding.fft_homog_workspace_size(d)

        if size(1) > self.max_bytes:
            raise ValueError("one cell of shape %s needs more than max_bytes" % (shape,))
        lo = 1
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if size(mid) <= self.max_bytes:
                lo = mid
            else:
                hi = mid - 1
        return lo

    def _stream(self, shape):
        if not self.concurrent:
            return self.stream
        import torch
        st = self.streams.get(shape)
        if st is None:
            st = torch.cuda.Stream(device=self.device)
            self.streams[shape] = st
        return st

    def handle(self, shape, k):
        key = (tuple(shape), int(k))
        h = self.handles.get(key)
        if h is None:
            h = binding.FFTHomog(shape, self.kinematics, self.material, self.nphase, device=self.device,
                                 stream=self._stream(tuple(shape)), batch=k, **self.kw)
            self.handles[key] = h
            self._tune = key if self.autotune else None
        return h

    def tangents(self, cells):
        """cells: sequence of dicts with 'phase' (grid array, numpy or torch, host or device) and
        'table' ((nphase, 2) lam, mu).

        Returns (C, info): C is an array (len(cells), c, c) when every cell has the same c
        (otherwise a list), info a list of per-chunk records (shape, cells, cg total, seconds).
        """
        import torch

        groups = OrderedDict()
        for i, cell in enumerate(cells):
            groups.setdefault(tuple(cell["phase"].shape), []).append(i)
        out = [None] * len(cells)
        jobs = OrderedDict()
        for shape, idx in groups.items():
            k = self.chunk_size(shape, len(idx))
            jobs[shape] = [idx[s:s + k] for s in range(0, len(idx), k)]

        def stack_phase(h, chunk):
            # on the handle's stream, which the library then uses: no cross-stream dependency
            with torch.cuda.stream(h.stream):
                return torch.stack([torch.as_tensor(cells[i]["phase"]).to(device=h.device, dtype=torch.uint8)
                                    for i in chunk])

        def run_chunk(shape, chunk, allow_tune):
            self._tune = None
            h = self.handle(shape, len(chunk))
            tune = self._tune if allow_tune else None
            phase = stack_phase(h, chunk)
            table = np.stack([np.asarray(cells[i]["table"], dtype=np.float64) for i in chunk])
            h.set_material(phase, table)
            if tune is not None:
                # one tuning per grid shape; later chunk sizes of that grid reuse it
                known = [v for kk, v in self.shapes.items() if kk[0] == tune[0]]
                if known:
                    h.set_launch_shape(known[0])
                else:
                    self.shapes[tune] = h.autotune()
            if h.cells == 1:
                # a one-cell handle takes its tangent at a converged state: the reference
                # state is one (zero load, no CG)
                d = len(shape)
                h.reset()
                h.solve(np.eye(d).reshape(-1) if self.kinematics == "finite" else np.zeros(h.c), 1)
            C, st = h.tangent()
            C = C.reshape(len(chunk), h.c, h.c)
            for j, i in enumerate(chunk):
                out[i] = C[j]
            return dict(shape=shape, cells=len(chunk), cg_total=st["cg_total"], seconds=st["seconds"],
                        status=st["status"])

        if not self.concurrent:
            info = [run_chunk(shape, chunk, self.autotune) for shape, chs in jobs.items() for chunk in chs]
        else:
            import threading

            # handles are created and tuned one group at a time, so that tuning timings do not overlap
            for shape, chs in jobs.items():
                for chunk in chs:
                    key = (shape, len(chunk))
                    if key not in self.handles:
                        self._tune = None
                        h = self.handle(shape, len(chunk))
                        if self._tune is not None:
                            phase = stack_phase(h, chunk)
                            h.set_material(phase, np.stack([np.asarray(cells[i]["table"], dtype=np.float64)
                                                            for i in chunk]))
                            known = [v for kk, v in self.shapes.items() if kk[0] == shape]
                            if known:
                                h.set_launch_shape(known[0])
                            else:
                                self.shapes[self._tune] = h.autotune()
            results = {}
            errors = []

            def worker(shape, chs):
                try:
                    results[shape] = [run_chunk(shape, chunk, False) for chunk in chs]
                except Exception as e:  # re-raised in the calling thread
                    errors.append(e)

            threads = [threading.Thread(target=worker, args=(shape, chs)) for shape, chs in jobs.items()]
            for t in threads:
                t.start()
            for t in threads:
                t.join()
            if errors:
                raise errors[0]
            info = [r for shape in jobs for r in results[shape]]
        if len({o.shape for o in out}) == 1:
            out = np.stack(out)
        return out, info

    def close(self):
        for h in self.handles.values():
            h.close()
        self.handles.clear()
