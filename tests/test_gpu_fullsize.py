"""Parity at the full workload sizes, in the launch configuration bench.py times.

The oracle cannot solve 128^3 in seconds, so these tests check outputs it can
compute one by one (the constitutive law at sampled voxels) and properties
that hold at any size: the mean of the strain field equals the macro load, the
converged stress is in equilibrium (G* applied by the oracle's own FFT), the
fluctuation is compatible, the homogenized stress is the voxel average, and the
homogenized tangent is symmetric, inside the Voigt-Reuss bounds and equal to
the macro response of independent solves.
"""

import numpy as np
import pytest

from helpers import field_err, lame_fields, pack, rel, relmax, unpack
from oracle import closed_forms, materials, newton_cg, spectral
from paper_2408_03804_amd import workloads

pytestmark = pytest.mark.gpu


def make(shape, kin, mat, nphase=2, **kw):
    from paper_2408_03804_amd.binding import FFTHomog
    return FFTHomog(shape, kin, mat, nphase, **kw)


def to_full(field, shape):
    """(d, d, *grid) device tensor -> (*grid, d, d) numpy."""
    d = len(shape)
    a = field.cpu().numpy().reshape((d, d) + tuple(shape))
    return np.moveaxis(a, (0, 1), (-2, -1))


# launch shape that bench.py times at 128^3 (the default of a one-cell 128^3 finite-strain handle):
# rows per x-pass block, kx bins per y / outer block, register-staged FFTs, padded spectrum pitch
BENCH_SHAPE_128 = {"x_rows": 2, "y_bins": 16, "outer_bins": 8, "x_regs": 1, "y_regs": 1, "outer_regs": 1,
                   "spectrum_pitch": 72}


@pytest.fixture(scope="module")
def nh128():
    """The 128^3 Neo-Hookean workload solved exactly as bench.py solves it."""
    w = workloads.workload_neohookean3d(n=128)
    shape = w["shape"]
    h = make(shape, "finite", "neo_hookean", tol_newton=1e-10, tol_cg=1e-10, max_newton=50, max_cg=20000)
    h.set_material(w["phase"], w["table"])
    stagger = h.tune_placement(reps=10)  # as bench.py does before its timed solves
    S, psi, st = h.solve(w["macro"], w["n_increments"])
    return dict(w=w, h=h, S=S, psi=psi, st=st, stagger=stagger)


def test_neohookean_128_bench_configuration(nh128):
    w, h, S, psi, st = nh128["w"], nh128["h"], nh128["S"], nh128["psi"], nh128["st"]
    shape = w["shape"]
    assert st["status"] == "ok" and st["increments"] == 10
    assert 10 <= st["newton"] <= 80 and st["cg_total"] > 0
    F = to_full(h.get_field(0), shape)
    P = to_full(h.get_field(1), shape)
    E = h.get_field(2).cpu().numpy()
    Fbar = w["macro"].reshape(3, 3)
    lam, mu = lame_fields(w["phase"], w["table"])

    # mean strain is the macro load
    assert np.abs(F.reshape(-1, 3, 3).mean(axis=0) - Fbar).max() < 1e-13
    # homogenized outputs are the voxel averages of the returned fields
    assert rel(S, P.reshape(-1, 9).mean(axis=0)) < 1e-13
    assert abs(psi - E.mean()) < 1e-13 * abs(psi)
    # constitutive law at 4096 sampled voxels against the closed form
    rng = np.random.default_rng(0)
    idx = rng.integers(0, F.reshape(-1, 3, 3).shape[0], 4096)
    Fs = F.reshape(-1, 3, 3)[idx]
    ls, ms = lam.reshape(-1)[idx], mu.reshape(-1)[idx]
    assert field_err(P.reshape(-1, 3, 3)[idx], materials.NeoHookean.stress(Fs, ls, ms)) < 1e-13
    # psi is O(strain^2) assembled from O(1) terms: its relative rounding is larger than P's
    assert field_err(E.reshape(-1)[idx], materials.NeoHookean.psi(Fs, ls, ms)) < 1e-12
    # equilibrium and compatibility, with the oracle's projection
    GP = spectral.apply_G(P, "finite")
    assert np.linalg.norm(GP) <= 1e-8 * np.linalg.norm(P)
    fl = F - Fbar
    assert field_err(spectral.apply_G(fl, "finite"), fl) < 1e-12


def test_neohookean_128_operator_and_rhs_elementwise_at_bench_shape(nh128):
    """The CG operator q = G*(K(F):p) at the converged 128^3 state, and the Newton right-hand side
    -G*(P(F)) of the next load step, element by element against the oracle, through the kernels and
    the launch shape the benchmark times."""
    w, h = nh128["w"], nh128["h"]
    shape = w["shape"]
    assert h.launch_shape() == BENCH_SHAPE_128, h.launch_shape()
    F = to_full(h.get_field(0), shape)
    lam, mu = lame_fields(w["phase"], w["table"])
    prob = newton_cg.Problem(shape, "neo_hookean", lam, mu)
    rng = np.random.default_rng(11)
    p = 1e-2 * rng.standard_normal(shape + (3, 3))
    q = unpack(h.debug_apply_operator(pack(p, False)).cpu().numpy(), False, 3)
    qref = prob.operator(F, p)
    assert relmax(q, qref) < 1e-12 and rel(q, qref) < 1e-12
    # stress everywhere, and the right-hand side of the first Newton step of a further increment
    P = to_full(h.get_field(1), shape)
    assert relmax(P, prob.stress(F)) < 1e-13
    Fs = F.copy()
    Fs[..., 0, 0] += 0.005
    macro = w["macro"].copy()
    macro[0] += 0.005
    h.set_field(np.ascontiguousarray(np.moveaxis(Fs, (-2, -1), (0, 1)).reshape((9,) + shape)), macro)
    Ps = to_full(h.get_field(1), shape)
    b = h.debug_project(pack(-Ps, False)).cpu().numpy()
    bref = prob.rhs(Fs)
    assert relmax(unpack(b, False, 3), bref) < 1e-12
    nh128["shifted"] = (Fs, macro, bref)


def test_neohookean_128_first_cg_iterates_elementwise(nh128):
    """The first CG iterates x_k and residuals r_k (k = 1, 3) of that Newton step, run by the
    solver's own CG kernels at the benchmark's launch shape, against the oracle's textbook CG."""
    w, h = nh128["w"], nh128["h"]
    shape = w["shape"]
    assert "shifted" in nh128, "runs after the operator test, which sets the shifted state"
    Fs, macro, bref = nh128["shifted"]
    lam, mu = lame_fields(w["phase"], w["table"])
    prob = newton_cg.Problem(shape, "neo_hookean", lam, mu)
    op = lambda v: prob.operator(Fs, v)  # noqa: E731
    for k in (1, 3):
        x, r = h.debug_cg(k)
        xref, kk, status = newton_cg.conjugate_gradient(op, bref, 0.0, k)
        assert kk == k and status == "not_converged"
        rref = bref - op(xref)
        assert field_err(unpack(x.cpu().numpy(), False, 3), xref) < 1e-11, k
        assert field_err(unpack(r.cpu().numpy(), False, 3), rref) < 1e-11, k


def test_spheres_64_tangent_properties():
    w = workloads.workload_spheres3d(n=64)
    shape = w["shape"]
    h = make(shape, "small", "linear_elastic", tangent=True, tol_newton=1e-10, tol_cg=1e-10, max_cg=20000)
    h.set_material(w["phase"], w["table"])
    S, psi, st = h.solve(np.zeros(6), 1)
    assert st["status"] == "ok"
    C, st = h.tangent()
    assert st["status"] == "ok" and len(st["cg"]) == 6
    scale = np.abs(C).max()
    assert np.abs(C - C.T).max() < 1e-12 * scale
    f1 = float(w["phase"].mean())
    tab = w["table"]
    CV, CR = closed_forms.voigt_reuss([closed_forms.isotropic_matrix(*tab[0], 3),
                                       closed_forms.isotropic_matrix(*tab[1], 3)], [1 - f1, f1])
    assert np.linalg.eigvalsh(CV - C).min() > -1e-12 * scale
    assert np.linalg.eigvalsh(C - CR).min() > -1e-12 * scale
    # linear elasticity: the macro stress of a unit load is the tangent's column
    for J in (0, 3):
        g = make(shape, "small", "linear_elastic", tol_newton=1e-10, tol_cg=1e-10, max_cg=20000)
        g.set_material(w["phase"], w["table"])
        e = np.zeros(6)
        e[J] = 1.0
        SJ, _, stJ = g.solve(e, 1)
        assert stJ["status"] == "ok"
        assert np.abs(SJ - C[:, J]).max() < 1e-8 * scale


def test_disk_31_grid_is_config_of_small_workload():
    w = workloads.workload_disk2d(31)
    assert int(w["phase"].sum()) == 185 and w["shape"] == (31, 31)


def test_work_vector_placement_changes_no_result():
    """The work vectors' placement (fft_homog_set_placement / tune_placement) moves pointers only:
    a 100^3 Neo-Hookean solve is bitwise the same at every stagger candidate the tuner may pick."""
    w = workloads.workload_neohookean3d(n=100)
    shape = w["shape"]
    out = []
    for s in (0, 256, 4 << 20, None):
        h = make(shape, "finite", "neo_hookean", tol_newton=1e-10, tol_cg=1e-10, max_newton=50, max_cg=20000)
        h.set_material(w["phase"], w["table"])
        if s is None:
            s = h.tune_placement(reps=3)
            assert s in (0, 256, 16 << 10, 256 << 10, 2 << 20, 4 << 20)
        else:
            h.set_placement(s)
        S, psi, st = h.solve(w["macro"], 2)
        assert st["status"] == "ok"
        out.append((S, psi, st["cg"], h.get_field(0).cpu().numpy()))
        del h
    for S, psi, cg, F in out[1:]:
        assert np.array_equal(S, out[0][0]) and psi == out[0][1] and cg == out[0][2]
        assert np.array_equal(F, out[0][3])
    # small grids keep no slack: only stagger 0 is valid
    from paper_2408_03804_amd.binding import FFTHomogError
    g = make((16, 16, 16), "finite", "neo_hookean")
    g.set_material(np.zeros((16, 16, 16), dtype=np.uint8), [[2.0, 1.0], [4.0, 2.0]])
    assert g.tune_placement(reps=1) == 0
    with pytest.raises(FFTHomogError):
        g.set_placement(256)
