"""Write the oracle goldens of the full-size workloads (test infrastructure).

Every stored value is computed here by the CPU oracle (``oracle/``) on the seeded
inputs of ``paper_2408_03804_amd.workloads`` (input generation only); nothing is
taken from the HIP path.  The GPU parity tests compare against these files.

    python tests/golden/make_goldens.py spheres64   # 64^3 RSA spheres: 6x6 tangent
    python tests/golden/make_goldens.py nh64        # 64^3 Neo-Hookean GRF, 10 increments
    python tests/golden/make_goldens.py nh128       # the same at 128^3 (hours of CPU time)
    python tests/golden/make_goldens.py uq256       # a 32^3 and a 96^3 cell of the 256-cell workload

Each run writes ``<name>.json`` (homogenized values, iteration counts, settings and
the command) and, for the Neo-Hookean solves, ``<name>_samples.npz`` with the
converged deformation gradient at 4096 seeded voxels.

Tolerances follow the parity reading: CG 1e-12 so that field differences between
two converged solves reflect rounding, Newton 1e-10.
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import newton_cg  # noqa: E402
from paper_2408_03804_amd import workloads  # noqa: E402

TOL_CG = 1e-12
TOL_NEWTON = 1e-10
N_SAMPLES = 4096
SAMPLE_SEED = 20240803


def sample_indices(N):
    """Seeded voxel indices (flat, x fastest) of the stored field samples."""
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(N, size=min(N_SAMPLES, N), replace=False))


def spheres(n):
    w = workloads.workload_spheres3d(n=n)
    tab = np.asarray(w["table"])
    prob = newton_cg.Problem(w["shape"], "linear_elastic", tab[w["phase"], 0], tab[w["phase"], 1])
    t0 = time.time()
    C, Cd, counts = newton_cg.homogenized_tangent(prob, newton_cg.initial_state(prob), tol_cg=TOL_CG)
    out = {
        "workload": w["name"],
        "what": "6x6 homogenized tangent (Voigt, engineering shear) of the 3D small-strain linear elastic "
                "RSA-sphere cell at the reference state, implicit linearisation, energy form",
        "grid": list(w["shape"]), "stiff_fraction": float(w["phase"].mean()),
        "table": tab.tolist(), "tol_cg": TOL_CG,
        "C": C.tolist(), "C_direct": Cd.tolist(), "cg_per_load": [int(k) for k in counts],
        "oracle_seconds": time.time() - t0,
    }
    return w["name"] + "_tangent", out, None


def uq_cells():
    """6x6 tangents of the first 32^3 and the first 96^3 cell of the 256-cell uneven-size workload."""
    cells = workloads.workload_uq_cells(256)
    sizes = [c["shape"][0] for c in cells]
    out = {"workload": "uq256", "what": "6x6 homogenized tangents (Voigt, engineering shear) of single cells of the "
           "256-cell small-strain linear elastic workload of uneven size, at the reference state, implicit "
           "linearisation, energy form", "tol_cg": TOL_CG, "cells": []}
    t0 = time.time()
    for n in (32, 96):
        i = sizes.index(n)
        c = cells[i]
        tab = np.asarray(c["table"])
        prob = newton_cg.Problem(c["shape"], "linear_elastic", tab[c["phase"], 0], tab[c["phase"], 1])
        C, Cd, counts = newton_cg.homogenized_tangent(prob, newton_cg.initial_state(prob), tol_cg=TOL_CG)
        out["cells"].append({"index": i, "grid": list(c["shape"]), "stiff_fraction": float(c["phase"].mean()),
                             "table": tab.tolist(), "C": C.tolist(), "cg_per_load": [int(k) for k in counts]})
    out["oracle_seconds"] = time.time() - t0
    return "uq256_cells", out, None


def neohookean(n):
    w = workloads.workload_neohookean3d(n=n)
    tab = np.asarray(w["table"])
    prob = newton_cg.Problem(w["shape"], "neo_hookean", tab[w["phase"], 0], tab[w["phase"], 1])
    t0 = time.time()
    ref = newton_cg.solve(prob, w["macro"], n_increments=w["n_increments"], tol_newton=TOL_NEWTON,
                          tol_cg=TOL_CG, max_cg=100000)
    secs = time.time() - t0
    if ref["stats"]["status"] != "ok":
        raise RuntimeError("oracle solve failed: %s" % ref["stats"]["status"])
    F = ref["state"].field.reshape(-1, 3, 3)
    idx = sample_indices(F.shape[0])
    out = {
        "workload": w["name"],
        "what": "3D finite-strain compressible Neo-Hookean Gaussian-random-field cell, F-bar = diag(1.05,1,1) "
                "in 10 increments: homogenized first Piola-Kirchhoff stress (row-major), mean energy density, "
                "Newton and CG counts; converged F at seeded voxels in the companion .npz",
        "grid": list(w["shape"]), "stiff_fraction": float(w["phase"].mean()), "table": tab.tolist(),
        "macro": w["macro"].tolist(), "n_increments": w["n_increments"],
        "tol_cg": TOL_CG, "tol_newton": TOL_NEWTON,
        "macro_stress": [float(v) for v in ref["macro_stress"]], "energy": ref["energy"],
        "newton": ref["stats"]["newton"], "cg": ref["stats"]["cg"], "cg_total": ref["stats"]["cg_total"],
        "sample_seed": SAMPLE_SEED, "n_samples": int(idx.size),
        "oracle_seconds": secs,
    }
    samples = {"index": idx.astype(np.int64), "F": F[idx].reshape(-1, 9)}
    return w["name"], out, samples


def main(argv):
    jobs = {"spheres64": lambda: spheres(64), "nh64": lambda: neohookean(64), "nh128": lambda: neohookean(128),
            "uq256": uq_cells}
    for name in argv[1:]:
        stem, out, samples = jobs[name]()
        out["command"] = "python tests/golden/make_goldens.py " + name
        with open(os.path.join(HERE, stem + ".json"), "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")
        if samples is not None:
            np.savez_compressed(os.path.join(HERE, stem + "_samples.npz"), **samples)
        print("%s: written (%.0f s of oracle time)" % (stem, out["oracle_seconds"]), flush=True)


if __name__ == "__main__":
    main(sys.argv)
