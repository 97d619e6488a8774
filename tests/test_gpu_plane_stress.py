"""Finite-strain plane stress on the GPU against the oracle.

Neo-Hookean runs a law of its own (the out-of-plane stretch solved per voxel by Newton's method in
the kernel, its derivative by one dual-number Newton step); St. Venant-Kirchhoff runs the 2D law
with the reduced first Lame parameter; J2 solves for eps_33 per voxel through the 3D return mapping
(bracketed Newton) and condenses K on it with a second dual direction.  The oracle completes the
strain with the out-of-plane entry at which the 3D law's out-of-plane normal stress vanishes
(bisection for Neo-Hookean and J2, closed form for St. Venant-Kirchhoff) and condenses the 3D
tangent on it.
"""

import numpy as np
import pytest

from helpers import field_err, lame_fields, pack
from oracle import materials, newton_cg
from paper_2408_03804_amd import workloads

pytestmark = pytest.mark.gpu

TOL_FIELD = 1e-10
TOL_HOMOG = 1e-11
LAWS = [("neo_hookean", "neo_hookean_plane_stress"), ("stvk", "stvk_plane_stress")]


def make(shape, kin, mat, nphase=2, **kw):
    from paper_2408_03804_amd.binding import FFTHomog
    return FFTHomog(shape, kin, mat, nphase, **kw)


@pytest.mark.parametrize("mat,oracle_mat", LAWS)
@pytest.mark.parametrize("shape", [(5, 7), (16, 9)])
def test_finite_plane_stress_constitutive_matches_oracle(mat, oracle_mat, shape):
    h = make(shape, "finite", mat, plane_stress=True)
    phase = workloads.random_phases(shape, 2, 1)
    table = [[1.3, 0.7], [4.0, 2.5]]
    h.set_material(phase, table)
    rng = np.random.default_rng(5)
    F = np.eye(2) + 0.15 * rng.standard_normal(shape + (2, 2))
    dF = rng.standard_normal(shape + (2, 2))
    P, K, psi = h.debug_constitutive(pack(F, False), pack(dF, False))
    lam, mu = lame_fields(phase, table)
    M = materials.MATERIALS[oracle_mat]
    assert field_err(P.cpu().numpy(), pack(M.stress(F, lam, mu), False)) < 1e-13
    assert field_err(K.cpu().numpy(), pack(M.tangent_apply(F, dF, lam, mu), False)) < 1e-13
    assert field_err(psi.cpu().numpy(), M.psi(F, lam, mu)) < 1e-13


@pytest.mark.parametrize("mat,oracle_mat", LAWS)
def test_finite_plane_stress_disk_matches_oracle(mat, oracle_mat):
    """The 31 x 31 disk cell in finite strain under plane stress, two load increments: fields,
    homogenized stress, energy, CG counts and the homogenized tangent dP/dF against the oracle."""
    w = workloads.workload_disk2d(31)
    shape = w["shape"]
    Fbar = np.array([[1.06, 0.03], [-0.01, 0.97]]).reshape(-1)
    h = make(shape, "finite", mat, tol_cg=1e-12, tol_newton=1e-10, tangent=True, plane_stress=True)
    h.set_material(w["phase"], w["table"])
    S, psi, st = h.solve(Fbar, 2)
    lam, mu = lame_fields(w["phase"], w["table"])
    prob = newton_cg.Problem(shape, oracle_mat, lam, mu)
    ref = newton_cg.solve(prob, Fbar, n_increments=2, tol_newton=1e-10, tol_cg=1e-12)
    rs = ref["stats"]
    assert st["status"] == "ok" and rs["status"] == "ok"
    assert abs(st["newton"] - rs["newton"]) <= 1
    if st["newton"] == rs["newton"]:
        for a, b in zip(st["cg"], rs["cg"]):
            assert abs(a - b) <= 1, (st["cg"], rs["cg"])
    F = np.moveaxis(h.get_field(0).cpu().numpy().reshape((2, 2) + shape), (0, 1), (-2, -1))
    P = np.moveaxis(h.get_field(1).cpu().numpy().reshape((2, 2) + shape), (0, 1), (-2, -1))
    Fm = ref["state"].macro
    assert field_err(F - Fm, ref["state"].field - Fm) < TOL_FIELD
    assert field_err(P, prob.stress(ref["state"].field)) < TOL_FIELD
    assert np.abs(S - ref["macro_stress"]).max() < TOL_HOMOG * np.abs(ref["macro_stress"]).max()
    assert abs(psi - ref["energy"]) < TOL_HOMOG * abs(ref["energy"])
    C, _ = h.tangent()
    Cref, _, _ = newton_cg.homogenized_tangent(prob, ref["state"], tol_cg=1e-12)
    assert np.abs(C - Cref).max() < TOL_HOMOG * np.abs(Cref).max()
    # plane stress is softer than plane strain under the in-plane stretch
    g = make(shape, "finite", mat, tol_cg=1e-12, tol_newton=1e-10)
    g.set_material(w["phase"], w["table"])
    S2, _, _ = g.solve(Fbar, 2)
    assert S[0] < S2[0]


def test_neo_hookean_plane_stress_stored_tangent_matches_recomputed():
    """K stored per voxel (the condensed tangent is symmetric) gives the solve that recomputes K:p."""
    shape = (12, 10)
    phase = workloads.random_phases(shape, 2, 7)
    table = [[2.0, 1.0], [10.0, 5.0]]
    Fbar = np.array([[1.04, 0.02], [-0.01, 0.98]]).reshape(-1)
    out = []
    for k_mode in (0, 1):
        h = make(shape, "finite", "neo_hookean", tol_cg=1e-12, tol_newton=1e-10, k_mode=k_mode, plane_stress=True)
        h.set_material(phase, table)
        out.append(h.solve(Fbar, 2))
    assert np.abs(out[0][0] - out[1][0]).max() < 1e-12 * np.abs(out[0][0]).max()
    assert out[0][2]["cg"] == out[1][2]["cg"] or all(abs(a - b) <= 1 for a, b in zip(out[0][2]["cg"], out[1][2]["cg"]))


def test_plane_stress_argument_checks():
    from paper_2408_03804_amd.binding import FFTHomogError
    shape = (8, 9)
    phase = workloads.random_phases(shape, 2, 1)
    h = make(shape, "finite", "neo_hookean", plane_stress=True)
    with pytest.raises(FFTHomogError) as ei:
        h.set_material(phase, [[-0.5, 1.0], [2.0, 2.0]])
    assert ei.value.status == "einval"
    g = make(shape, "small", "j2_plastic", plane_stress=True)
    with pytest.raises(FFTHomogError) as ei:
        g.set_material(phase, [[1.0, 0.0, 0.01, 0.1], [2.0, 1.0, 0.01, 0.1]])
    assert ei.value.status == "einval"
    with pytest.raises(FFTHomogError):
        make((4, 5, 6), "finite", "neo_hookean", plane_stress=True)


def j2_table(E=(1.0, 2.0), sy=(0.005, 0.01), H=(0.1, 0.2)):
    return np.array([[*workloads.lame(E[i], 0.3), sy[i], H[i]] for i in range(2)])


@pytest.mark.parametrize("shape", [(5, 7), (16, 9)])
def test_j2_plane_stress_return_mapping_matches_oracle(shape):
    """J2 under plane stress from a virgin history: P, the condensed K : dE and the stored elastic
    energy at every voxel against the oracle (eps_33 by bisection there, by bracketed Newton here)."""
    from oracle import plasticity as OP
    tab = j2_table()
    phase = workloads.random_phases(shape, 2, 2)
    h = make(shape, "small", "j2_plastic", plane_stress=True)
    h.set_material(phase, tab)
    rng = np.random.default_rng(6)
    A = 0.02 * rng.standard_normal(shape + (2, 2))
    E = 0.5 * (A + np.swapaxes(A, -1, -2))
    B = rng.standard_normal(shape + (2, 2))
    dE = 0.5 * (B + np.swapaxes(B, -1, -2))
    P, K, psi = h.debug_constitutive(pack(E, True), pack(dE, True))
    lam, mu, sy, H = [tab[phase, k] for k in range(4)]
    pr = OP.PlasticPlaneStressProblem(shape, lam, mu, sy, H)
    _, dp, _ = OP.return_map(pr.full(E), pr.ep, pr.p, lam, mu, sy, H)
    assert (dp > 0).mean() > 0.5
    assert field_err(P.cpu().numpy(), pack(pr.stress(E), True)) < 1e-13
    assert field_err(K.cpu().numpy(), pack(pr.tangent_apply(E, dE), True)) < 1e-12
    assert field_err(psi.cpu().numpy(), pr.energy_density(E)) < 1e-12


def test_j2_plane_stress_disk_loading_unloading_path_matches_oracle():
    """Hard disk in a soft matrix under plane stress: biaxial loading in 4 increments, unloading in 2,
    then a sheared reload in 3; after each solve the fields, stress, cumulative plastic strain,
    homogenized stress and energy, and the homogenized consistent tangent against the oracle."""
    from oracle import plasticity as OP
    n = 24
    shape = (n, n)
    phase = workloads.centered_disk(n, 0.25)
    tab = j2_table()
    h = make(shape, "small", "j2_plastic", tangent=True, tol_cg=1e-12, plane_stress=True)
    h.set_material(phase, tab)
    lam, mu, sy, H = [tab[phase, k] for k in range(4)]
    prob = OP.PlasticPlaneStressProblem(shape, lam, mu, sy, H)
    state = None
    first = None
    for macro, n_inc in [(np.array([1e-2, 1e-2, 0.0]), 4), (np.array([5e-3, 5e-3, 0.0]), 2),
                         (np.array([1e-2, 1.5e-2, 4e-3]), 3)]:
        S, psi, st = h.solve(macro, n_inc)
        ref = newton_cg.solve(prob, macro, n_increments=n_inc, tol_cg=1e-12, state=state)
        state = ref["state"]
        assert st["status"] == "ok" and ref["stats"]["status"] == "ok"
        assert abs(st["newton"] - ref["stats"]["newton"]) <= 1
        first = S if first is None else first
        Fg = np.moveaxis(h.get_field(0).cpu().numpy().reshape((2, 2) + shape), (0, 1), (-2, -1))
        Pg = np.moveaxis(h.get_field(1).cpu().numpy().reshape((2, 2) + shape), (0, 1), (-2, -1))
        assert field_err(Fg - state.macro, state.field - state.macro) < TOL_FIELD
        assert field_err(Pg, prob.stress(state.field)) < TOL_FIELD
        pl = h.get_field(3).cpu().numpy()
        plref = prob.plastic_strain_now(state.field)
        assert np.abs(pl - plref).max() < TOL_FIELD * np.abs(plref).max()
        assert np.abs(S - ref["macro_stress"]).max() < TOL_HOMOG * np.abs(ref["macro_stress"]).max()
        assert abs(psi - ref["energy"]) < TOL_HOMOG * abs(ref["energy"])
        C, _ = h.tangent()
        Cref, _ = OP.homogenized_tangent(prob, state, tol_cg=1e-12)
        assert np.abs(C - Cref).max() < TOL_HOMOG * np.abs(Cref).max()
    assert float(pl.max()) > 1e-3
    # plane stress is softer than plane strain under the first (biaxial) load
    g = make(shape, "small", "j2_plastic", tol_cg=1e-12)
    g.set_material(phase, tab)
    S2, _, _ = g.solve(np.array([1e-2, 1e-2, 0.0]), 4)
    assert first[0] < S2[0]
