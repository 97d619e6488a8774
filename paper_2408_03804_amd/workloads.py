"""Seeded synthetic microstructures and load cases.

Input generation only: nothing in this module computes any part of the
homogenization method.  Both the HIP path (through tests and the benchmark) and
the CPU oracle (through the tests) receive the arrays produced here.

All generators are deterministic functions of their arguments and a
``numpy.random.default_rng(seed)`` stream.  Voxel centres sit at (i + 1/2) h.
Phase id 0 is the matrix / soft phase, phase id 1 the inclusion / stiff phase.
Arrays use the grid order (Ny, Nx) or (Nz, Ny, Nx) with x fastest.
"""

import math

import numpy as np


def lame(E, nu):
    """(lambda, mu) from Young's modulus and Poisson ratio."""
    E = float(E)
    return E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), E / (2.0 * (1.0 + nu))


# ---------------------------------------------------------------------------
# microstructures
# ---------------------------------------------------------------------------
def centered_disk(n, radius_fraction):
    """2D disk centred on the centre of voxel (n//2, n//2); inside if centre distance <= r."""
    c = n // 2 + 0.5
    r = radius_fraction * n
    x = np.arange(n) + 0.5
    d2 = (x[None, :] - c) ** 2 + (x[:, None] - c) ** 2
    return (d2 <= r * r).astype(np.uint8)


def disk_of_area_fraction(n, fraction):
    """2D centred disk whose radius gives the requested area fraction of the cell."""
    return centered_disk(n, math.sqrt(fraction / math.pi))


def _periodic_dist2(a, b, n):
    d = np.abs(a - b)
    d = np.minimum(d, n - d)
    return np.sum(d * d, axis=-1)


def rsa_spheres(n, radius, min_center_distance, volume_fraction, seed, max_attempts=100000):
    """Random sequential addition of non-overlapping periodic spheres on an n^3 grid.

    Centres are uniform in [0, n)^3 (voxel units).  A voxel belongs to a sphere
    if the periodic distance between its centre and the sphere centre is
    <= radius.  A candidate closer than ``min_center_distance`` to an accepted
    centre is rejected; spheres are added while the voxel volume fraction stays
    <= ``volume_fraction``.
    """
    rng = np.random.default_rng(seed)
    phase = np.zeros((n, n, n), dtype=np.uint8)
    coords = np.arange(n) + 0.5
    centres = []
    count = 0
    limit = volume_fraction * n ** 3
    for _ in range(max_attempts):
        c = rng.uniform(0.0, n, size=3)
        if centres and np.min(_periodic_dist2(np.array(centres), c[None, :], n)) < min_center_distance ** 2:
            continue
        dz = np.abs(coords - c[2]); dz = np.minimum(dz, n - dz)
        dy = np.abs(coords - c[1]); dy = np.minimum(dy, n - dy)
        dx = np.abs(coords - c[0]); dx = np.minimum(dx, n - dx)
        inside = (dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2) <= radius * radius
        add = int(np.count_nonzero(inside & (phase == 0)))
        if count + add > limit:
            break
        phase[inside] = 1
        count += add
        centres.append(c)
    return phase


def gaussian_random_field(shape, correlation_length, seed):
    """Standardised Gaussian random field with covariance exp(-r^2 / (2 l^2)).

    White N(0,1) noise filtered in Fourier space by sqrt(S(k)),
    S(k) = exp(-l^2 |k|^2 / 2) with k in radians per voxel.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    what = np.fft.rfftn(w)
    ks = [2.0 * np.pi * np.fft.fftfreq(s) for s in shape[:-1]] + [2.0 * np.pi * np.fft.rfftfreq(shape[-1])]
    k2 = np.zeros(what.shape)
    for ax, k in enumerate(ks):
        bs = [1] * len(shape)
        bs[ax] = k.shape[0]
        k2 = k2 + (k.reshape(bs)) ** 2
    g = np.fft.irfftn(what * np.exp(-0.25 * correlation_length ** 2 * k2), s=shape, axes=tuple(range(len(shape))))
    g -= g.mean()
    g /= g.std()
    return g


def threshold_top(field, fraction):
    """Phase 1 on exactly round(fraction*N) voxels with the largest values (ties: flat index)."""
    flat = field.reshape(-1)
    m = int(round(fraction * flat.size))
    phase = np.zeros(flat.size, dtype=np.uint8)
    if 0 < m < flat.size:
        # the m largest values; equal to the stable descending sort's first m unless the
        # value at the cut is shared, which then decides by flat index
        top = np.argpartition(-flat, m - 1)[:m]
        cut = flat[top].min()
        if np.count_nonzero(flat >= cut) == m and np.count_nonzero(flat == cut) == 1:
            phase[top] = 1
            return phase.reshape(field.shape)
    order = np.argsort(-flat, kind="stable")
    phase[order[:m]] = 1
    return phase.reshape(field.shape)


def grf_two_phase(shape, correlation_length, stiff_fraction, seed):
    return threshold_top(gaussian_random_field(shape, correlation_length, seed), stiff_fraction)


def simp_density(shape, correlation_length, seed, rho_min=0.01):
    """rho = rho_min + (1 - rho_min) Phi(g), g a standardised Gaussian random field."""
    from scipy.special import ndtr
    g = gaussian_random_field(shape, correlation_length, seed)
    return rho_min + (1.0 - rho_min) * ndtr(g)


def laminate(shape, axis, layer_ids):
    """Layered phase map: ``layer_ids[i]`` is the phase of index i along spatial ``axis``."""
    ids = np.asarray(layer_ids, dtype=np.uint8)
    assert ids.shape[0] == shape[axis]
    bs = [1] * len(shape)
    bs[axis] = shape[axis]
    return np.broadcast_to(ids.reshape(bs), shape).copy()


def random_phases(shape, nphase, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, nphase, size=shape).astype(np.uint8)


def random_field(shape, ncomp, seed, scale=1.0):
    """Seeded N(0, scale^2) real field of shape (ncomp, *shape)."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((ncomp,) + tuple(shape))


# ---------------------------------------------------------------------------
# the benchmark workloads
# ---------------------------------------------------------------------------
def workload_disk2d(n=31):
    """2D plane-strain linear elastic disk inclusion (E=10 in E=1, nu=0.3), eps_xx = 0.01."""
    lm0 = lame(1.0, 0.3)
    lm1 = lame(10.0, 0.3)
    return dict(name="le2d_disk_%d" % n, ndim=2, shape=(n, n), kinematics="small",
                material="linear_elastic", phase=centered_disk(n, 0.25),
                table=np.array([lm0, lm1]), macro=np.array([0.01, 0.0, 0.0]),
                n_increments=1)


def workload_spheres3d(n=64, seed=0):
    """3D small-strain linear elastic RSA spheres, r=6, 20 % stiff, contrast 100."""
    lm0 = lame(1.0, 0.3)
    lm1 = lame(100.0, 0.3)
    return dict(name="le3d_spheres_%d" % n, ndim=3, shape=(n, n, n), kinematics="small",
                material="linear_elastic",
                phase=rsa_spheres(n, 6.0 * n / 64.0, 12.0 * n / 64.0, 0.20, seed),
                table=np.array([lm0, lm1]),
                macro=np.array([1.0, 0.0, 0.0, 0.0, 0.0, 0.0]), n_increments=1)


def workload_neohookean3d(n=128, seed=0, correlation_length=8.0):
    """3D finite-strain Neo-Hookean GRF two-phase, mu 1 vs 20, lam = 2 mu, F = diag(1.05,1,1)."""
    table = np.array([[2.0, 1.0], [40.0, 20.0]])
    F = np.eye(3)
    F[0, 0] = 1.05
    return dict(name="nh3d_grf_%d" % n, ndim=3, shape=(n, n, n), kinematics="finite",
                material="neo_hookean",
                phase=grf_two_phase((n, n, n), correlation_length, 0.30, seed),
                table=table, macro=F.reshape(-1), n_increments=10)


def workload_uq_cells(n_cells=256, sizes=(32, 48, 64, 96), seed=0, stiff_ratio=10.0):
    """Many small-strain linear elastic cells of uneven size (uncertainty quantification).

    Per cell, from one seeded stream: edge n uniform over ``sizes``; a thresholded
    Gaussian random field with correlation length ~ U[4, 12] voxels and stiff
    fraction ~ U[0.1, 0.5]; matrix Young's modulus ~ lognormal(0, 0.2); the stiff
    phase ``stiff_ratio`` times stiffer; nu = 0.3 in both.  The stiff modulus is
    not fixed by the workload statement; 10 x the matrix is the reading used.
    Returns a list of dicts with keys shape, phase, table, seed.
    """
    rng = np.random.default_rng(seed)
    cells = []
    for i in range(n_cells):
        n = int(sizes[int(rng.integers(0, len(sizes)))])
        ell = float(rng.uniform(4.0, 12.0))
        frac = float(rng.uniform(0.1, 0.5))
        E0 = float(rng.lognormal(0.0, 0.2))
        cell_seed = int(rng.integers(0, 2 ** 31 - 1))
        phase = grf_two_phase((n, n, n), ell, frac, cell_seed)
        table = np.array([lame(E0, 0.3), lame(stiff_ratio * E0, 0.3)])
        cells.append(dict(shape=(n, n, n), phase=phase, table=table, seed=cell_seed,
                          correlation_length=ell, stiff_fraction=frac))
    return cells


def _grf_filter(w, correlation_length, axes):
    """Filter white noise w over `axes` by sqrt(S(k)), S(k) = exp(-l^2 |k|^2 / 2), and standardise
    each field (the other axes index independent fields)."""
    import scipy.fft

    shape = [w.shape[a] for a in axes]
    what = scipy.fft.rfftn(w, axes=axes, workers=-1)
    ks = [2.0 * np.pi * np.fft.fftfreq(s) for s in shape[:-1]] + [2.0 * np.pi * np.fft.rfftfreq(shape[-1])]
    k2 = np.zeros([what.shape[a] for a in axes])
    for ax, k in enumerate(ks):
        bs = [1] * len(axes)
        bs[ax] = k.shape[0]
        k2 = k2 + k.reshape(bs) ** 2
    g = scipy.fft.irfftn(what * np.exp(-0.25 * correlation_length ** 2 * k2), s=shape, axes=axes, workers=-1)
    g -= g.mean(axis=axes, keepdims=True)
    g /= g.std(axis=axes, keepdims=True)
    return g


def workload_tangent_cells(n_cells=1024, n=32, seed=0, correlation_length=8.0, stiff_fraction=0.30, chunk=256):
    """Training-style cells for a stiffness surrogate: the 3D Gaussian-random-field recipe of
    the finite-strain workload (l = 8 voxels, top 30 % stiff) at n^3, small-strain linear
    elastic with Young's moduli E1 (phase 0) and E2 (phase 1, the thresholded top) drawn
    independently from lognormal(0, 0.5), nu = 0.3 (the spread of the moduli is a reading:
    the workload statement does not fix it).  The moduli come from the stream
    default_rng([seed, 0]); the white noise of cell i is the i-th n^3 block of
    default_rng([seed, 1]).standard_normal, drawn in chunks of `chunk` cells.
    Returns a list of dicts like workload_uq_cells.
    """
    E = np.random.default_rng([seed, 0]).lognormal(0.0, 0.5, size=(n_cells, 2))
    rng = np.random.default_rng([seed, 1])
    cells = []
    for c0 in range(0, n_cells, chunk):
        k = min(chunk, n_cells - c0)
        g = _grf_filter(rng.standard_normal((k, n, n, n)), correlation_length, (1, 2, 3))
        for j in range(k):
            i = c0 + j
            phase = threshold_top(g[j], stiff_fraction)
            cells.append(dict(shape=(n, n, n), phase=phase,
                              table=np.array([lame(E[i, 0], 0.3), lame(E[i, 1], 0.3)]), seed=i,
                              correlation_length=correlation_length, stiff_fraction=stiff_fraction))
    return cells


def corner_square(n, fraction):
    """2D square inclusion of edge fraction * n at the (0, 0) corner: voxel centres inside [0, f L)^2."""
    x = np.arange(n) + 0.5
    inside = x < fraction * n
    return (inside[:, None] & inside[None, :]).astype(np.uint8)


def workload_e2_stvk(n=299, contrast=10.0):
    """The paper's hyperelastic example: 2D St. Venant-Kirchhoff cell with a stiff square inclusion of
    edge L/3 at a corner, simple shear F-bar = [[1, 0.1], [0, 1]] in one increment, Newton tolerance
    1e-5, CG tolerance 1e-8.  The stiffness contrast is not stated; 10 (both Lame parameters) is the
    reading used, with matrix E = 1, nu = 0.3."""
    lm0 = lame(1.0, 0.3)
    lm1 = lame(contrast, 0.3)
    F = np.eye(2)
    F[0, 1] = 0.1
    return dict(name="e2_stvk_%d" % n, ndim=2, shape=(n, n), kinematics="finite", material="stvk",
                phase=corner_square(n, 1.0 / 3.0), table=np.array([lm0, lm1]), macro=F.reshape(-1),
                n_increments=1, tol_newton=1e-5, tol_cg=1e-8)


def workload_e3_j2(n=199, n_increments=10):
    """The paper's elastoplastic example: 2D plane-strain J2 cell with a hard circular inclusion (twice
    the matrix yield stress and hardening modulus), biaxial macro strain [1e-2, 1e-2, 0].  Not stated,
    and read here: inclusion radius L/4, E = 1, nu = 0.3 in both phases, matrix sig_y = 5e-3,
    H = 0.1, and the load applied in 10 increments."""
    lm = lame(1.0, 0.3)
    table = np.array([[lm[0], lm[1], 5e-3, 0.1], [lm[0], lm[1], 1e-2, 0.2]])
    return dict(name="e3_j2_%d" % n, ndim=2, shape=(n, n), kinematics="small", material="j2_plastic",
                phase=centered_disk(n, 0.25), table=table, macro=np.array([1e-2, 1e-2, 0.0]),
                n_increments=n_increments, tol_newton=1e-10, tol_cg=1e-10)
