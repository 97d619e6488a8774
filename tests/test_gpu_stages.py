"""Stage-level parity of the HIP path against the CPU oracle (and numpy's FFT).

Each stage is called through its C-ABI entry point: constitutive law (dual
numbers vs closed form), real 3D/2D FFT, projection G*, and the CG operator
G*(K:p).  Grids cover odd, even, prime and ragged sizes and several LDS tiles.
"""

import numpy as np
import pytest

from helpers import field_err, lame_fields, ncomp, pack, unpack
from oracle import materials, spectral
from paper_2408_03804_amd import workloads

pytestmark = pytest.mark.gpu

MATS = [("linear_elastic", "small"), ("neo_hookean", "finite"), ("stvk", "finite")]
FFT_SHAPES = [(7, 5), (31, 31), (8, 12), (1, 9), (6, 10, 12), (9, 16, 15), (5, 6, 7), (3, 4, 1), (13, 11, 17),
              # lengths with compiled-in radix schedules (16, 8, 8.4, 16.3, 8.8, 16.5, 8.4.3, 16.8, 16.5.2,
              # 16.4.3, 16.16) on every axis
              (2, 4, 128), (128, 3, 2), (3, 256, 2), (16, 32, 64), (64, 16, 32), (256, 6), (5, 256),
              (2, 4, 96), (96, 3, 2), (3, 48, 2), (48, 96, 4), (48, 5),
              (2, 3, 80), (80, 4), (3, 160, 2), (160, 2, 3), (2, 192, 3), (192, 5),
              # lengths with large prime factors on each axis: chirp-z transforms (199, 257 and, on the
              # outer axis, 97) and direct prime stages (299 = 13 * 23, and 97 on the x axis)
              (199, 6), (3, 257), (4, 199, 5), (299, 4), (2, 3, 199), (3, 97), (97, 3), (2, 5, 97), (4, 3, 257),
              # the longest axes (1024 points; 1021 is prime: a 2048-point chirp-z convolution)
              (1021, 2), (2, 1021), (1024, 3)]


def make(shape, kin, mat, nphase=2, **kw):
    from paper_2408_03804_amd.binding import FFTHomog
    return FFTHomog(shape, kin, mat, nphase, **kw)


def random_state(shape, kin, seed, scale):
    d = len(shape)
    rng = np.random.default_rng(seed)
    A = scale * rng.standard_normal(tuple(shape) + (d, d))
    if kin == "small":
        return 0.5 * (A + np.swapaxes(A, -1, -2))
    return np.eye(d) + A


@pytest.mark.parametrize("mat,kin", MATS)
@pytest.mark.parametrize("shape", [(5, 7), (3, 4, 5)])
def test_constitutive_dual_numbers_match_closed_form(mat, kin, shape):
    d = len(shape)
    h = make(shape, kin, mat)
    phase = workloads.random_phases(shape, 2, 1)
    table = [[1.3, 0.7], [4.0, 2.5]]
    h.set_material(phase, table)
    E = random_state(shape, kin, 2, 0.1)
    dE = random_state(shape, kin, 3, 1.0) - (np.eye(d) if kin == "finite" else 0.0)
    small = kin == "small"
    P, K, psi = h.debug_constitutive(pack(E, small), pack(dE, small))
    lam, mu = lame_fields(phase, table)
    M = materials.MATERIALS[mat]
    assert field_err(P.cpu().numpy(), pack(M.stress(E, lam, mu), small)) < 1e-13
    assert field_err(K.cpu().numpy(), pack(M.tangent_apply(E, dE, lam, mu), small)) < 1e-13
    assert field_err(psi.cpu().numpy(), M.psi(E, lam, mu)) < 1e-13


@pytest.mark.parametrize("shape", FFT_SHAPES)
def test_rfft_and_irfft_match_numpy(shape):
    kin = "small"
    c = ncomp(kin, len(shape))
    h = make(shape, kin, "linear_elastic", tangent=True)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, c) + tuple(shape))
    spec = h.debug_rfft(x).cpu().numpy()
    ref = np.fft.rfftn(x, axes=tuple(range(2, 2 + len(shape))))
    assert np.abs(spec - ref).max() < 1e-13 * np.abs(ref).max()
    back = h.debug_irfft(ref).cpu().numpy()
    assert np.abs(back - x).max() < 1e-14 * np.abs(x).max() * 10


@pytest.mark.parametrize("kin,mat", [("small", "linear_elastic"), ("finite", "neo_hookean")])
@pytest.mark.parametrize("shape,lengths", [((7, 9), (1.0, 1.3)), ((31, 31), None), ((6, 8), None),
                                           ((5, 6, 7), (1.0, 0.8, 1.2)), ((8, 12, 10), None), ((9, 16, 15), None),
                                           ((128, 4, 6), None), ((6, 128, 32), None),
                                           # chirp-z transforms on the x, y and outer axes
                                           ((199, 3, 4), None), ((4, 199, 3), None), ((5, 4, 97), (1.0, 0.9, 1.1)),
                                           ((199, 8), None), ((6, 257), None)])
def test_projection_matches_oracle(kin, mat, shape, lengths):
    d = len(shape)
    h = make(shape, kin, mat, lengths=lengths)
    rng = np.random.default_rng(5)
    A = rng.standard_normal(tuple(shape) + (d, d))
    if kin == "small":
        A = 0.5 * (A + np.swapaxes(A, -1, -2))
    small = kin == "small"
    out = h.debug_project(pack(A, small)[None]).cpu().numpy()[0]
    ref = pack(spectral.apply_G(A, kin, lengths), small)
    assert field_err(out, ref) < 1e-13


@pytest.mark.parametrize("mat,kin", MATS)
@pytest.mark.parametrize("shape", [(9, 8), (6, 5, 7), (199, 5), (3, 4, 97)])  # the last two: chirp-z axes
@pytest.mark.parametrize("k_mode", [0, 1])
def test_cg_operator_matches_oracle(mat, kin, shape, k_mode):
    d = len(shape)
    small = kin == "small"
    h = make(shape, kin, mat, k_mode=k_mode)
    phase = workloads.random_phases(shape, 2, 6)
    table = [[1.0, 1.0], [6.0, 3.0]]
    h.set_material(phase, table)
    E = random_state(shape, kin, 7, 0.08)
    macro = E.reshape(-1, d, d).mean(axis=0)
    if small:
        macro_v = np.array([macro[i, j] * (1 if i == j else 2) for i, j in
                            ([(0, 0), (1, 1), (0, 1)] if d == 2 else [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)])])
    else:
        macro_v = macro.reshape(-1)
    h.set_field(np.moveaxis(E.reshape(tuple(shape) + (d * d,)), -1, 0), macro_v)
    rng = np.random.default_rng(8)
    p = rng.standard_normal(tuple(shape) + (d, d))
    if small:
        p = 0.5 * (p + np.swapaxes(p, -1, -2))
    q = h.debug_apply_operator(pack(p, small)[None]).cpu().numpy()[0]
    lam, mu = lame_fields(phase, table)
    M = materials.MATERIALS[mat]
    ref = pack(spectral.apply_G(M.tangent_apply(E, p, lam, mu), kin), small)
    assert field_err(q, ref) < 1e-13


def test_get_field_expands_packed_storage():
    shape = (4, 5, 6)
    h = make(shape, "small", "linear_elastic")
    E = random_state(shape, "small", 9, 0.1)
    full = np.moveaxis(E.reshape(shape + (9,)), -1, 0)
    h.set_field(full, np.zeros(6))
    back = h.get_field(0).cpu().numpy().reshape(9, *shape)
    assert np.abs(back - full).max() < 1e-15
