"""Pins of the J2 plasticity oracle (oracle/plasticity.py): closed forms, finite differences, invariants."""

import numpy as np
import pytest

from oracle import materials, newton_cg
from oracle import plasticity as P

LAM, MU, SY, H = 1.2, 0.8, 0.01, 0.3


def scal(x, shape=()):
    return np.full(shape, x, dtype=np.float64)


def random_sym(rng, shape, d, scale):
    A = scale * rng.standard_normal(shape + (d, d))
    return 0.5 * (A + np.swapaxes(A, -1, -2))


def test_below_yield_is_linear_elastic():
    rng = np.random.default_rng(0)
    E = random_sym(rng, (20,), 3, 1e-4)
    sig = P.return_map(E, np.zeros((20, 3, 3)), np.zeros(20), scal(LAM, (20,)), scal(MU, (20,)), scal(SY, (20,)),
                       scal(H, (20,)))[0]
    assert np.abs(sig - materials.LinearElastic.stress(E, LAM, MU)).max() < 1e-15
    dE = random_sym(rng, (20,), 3, 1.0)
    K = P.tangent_apply(E, dE, np.zeros((20, 3, 3)), np.zeros(20), LAM, MU, SY, H)
    assert np.abs(K - materials.LinearElastic.tangent_apply(E, dE, LAM, MU)).max() < 1e-14


def test_returned_stress_is_on_the_hardened_yield_surface():
    rng = np.random.default_rng(1)
    E = random_sym(rng, (50,), 3, 0.05)
    ep = np.zeros((50, 3, 3))
    p = rng.uniform(0, 0.01, 50)
    sig, dp, N = P.return_map(E, ep, p, LAM, MU, SY, H)
    s = sig - np.einsum("...ii->...", sig)[:, None, None] / 3 * np.eye(3)
    seq = np.sqrt(1.5 * np.einsum("...ij,...ij->...", s, s))
    plastic = dp > 0
    assert plastic.sum() > 40
    assert np.abs(seq[plastic] - (SY + H * (p[plastic] + dp[plastic]))).max() < 1e-13
    # the flow direction is deviatoric with N:N = 3/2
    assert np.abs(np.einsum("...ii->...", N)).max() < 1e-14
    assert np.abs(np.einsum("...ij,...ij->...", N[plastic], N[plastic]) - 1.5).max() < 1e-13


def test_printed_unit_direction_would_miss_the_yield_surface():
    """The appendix's corrector without the 3/2 factor leaves sig_eq above sig_y + H p: the pin above
    would fail for it, which is why the reading N = 3/2 s / sig_eq is used."""
    rng = np.random.default_rng(2)
    E = random_sym(rng, (10,), 3, 0.05)
    ee = E
    sig_tr = LAM * np.einsum("...ii->...", ee)[:, None, None] * np.eye(3) + 2 * MU * ee
    s = sig_tr - np.einsum("...ii->...", sig_tr)[:, None, None] / 3 * np.eye(3)
    seq = np.sqrt(1.5 * np.einsum("...ij,...ij->...", s, s))
    dp = np.maximum(seq - SY, 0) / (3 * MU + H)
    sig_printed = sig_tr - 2 * MU * dp[:, None, None] * s / seq[:, None, None]
    sp = sig_printed - np.einsum("...ii->...", sig_printed)[:, None, None] / 3 * np.eye(3)
    seq_p = np.sqrt(1.5 * np.einsum("...ij,...ij->...", sp, sp))
    assert np.min(seq_p - (SY + H * dp)) > 1e-4


def test_consistent_tangent_matches_central_differences():
    rng = np.random.default_rng(3)
    for d in (3, 2):
        E = random_sym(rng, (30,), d, 0.05)
        ep = P._dev(random_sym(rng, (30,), 3, 0.003))
        if d == 2:
            ep[:, :2, 2] = ep[:, 2, :2] = 0.0
        p = rng.uniform(0, 0.02, 30)
        dE = random_sym(rng, (30,), d, 1.0)
        h = 1e-7
        sp = P.return_map(E + h * dE, ep, p, LAM, MU, SY, H)[0]
        sm = P.return_map(E - h * dE, ep, p, LAM, MU, SY, H)[0]
        fd = (sp - sm) / (2 * h)
        K = P.tangent_apply(E, dE, ep, p, LAM, MU, SY, H)
        assert np.abs(K - fd).max() < 1e-6 * np.abs(K).max(), d


def test_consistent_tangent_is_symmetric():
    rng = np.random.default_rng(4)
    E = random_sym(rng, (30,), 3, 0.05)
    A = random_sym(rng, (30,), 3, 1.0)
    B = random_sym(rng, (30,), 3, 1.0)
    z, zp = np.zeros((30, 3, 3)), np.zeros(30)
    KA = P.tangent_apply(E, A, z, zp, LAM, MU, SY, H)
    KB = P.tangent_apply(E, B, z, zp, LAM, MU, SY, H)
    assert np.abs(np.einsum("...ij,...ij->...", B, KA) - np.einsum("...ij,...ij->...", A, KB)).max() < 1e-13


def test_proportional_loading_of_a_homogeneous_cell_has_the_closed_form():
    """A homogeneous cell under a deviatoric macro strain path t D: the radial return is exact
    for proportional loading, so the increments do not matter and sig_eq = (3 mu sig_y + H sig_eq_tr) / (3 mu + H)."""
    shape = (3, 4, 2)
    D = np.array([[1.0, 0.3, 0.0], [0.3, -0.4, 0.2], [0.0, 0.2, -0.6]]) * 0.02
    macro = np.array([D[0, 0], D[1, 1], D[2, 2], 2 * D[1, 2], 2 * D[0, 2], 2 * D[0, 1]])
    for n_inc in (1, 4):
        prob = P.PlasticProblem(shape, LAM, MU, SY, H)
        res = newton_cg.solve(prob, macro, n_increments=n_inc)
        assert res["stats"]["status"] == "ok" and res["stats"]["cg_total"] == 0
        sig = prob.stress3(res["state"].field)[0, 0, 0]
        s = sig - np.trace(sig) / 3 * np.eye(3)
        seq = np.sqrt(1.5 * np.sum(s * s))
        seq_tr = 2 * MU * np.sqrt(1.5 * np.sum(D * D))
        assert abs(seq - (3 * MU * SY + H * seq_tr) / (3 * MU + H)) < 1e-12


def test_history_commit_keeps_stress_and_lands_on_the_surface():
    rng = np.random.default_rng(5)
    shape = (4, 3, 5)
    prob = P.PlasticProblem(shape, LAM, MU, SY, H)
    E = random_sym(rng, shape, 3, 0.03)
    s_before = prob.stress(E)
    prob.commit(E)
    assert np.abs(prob.stress(E) - s_before).max() < 1e-14
    # after the commit the state is on (or inside) the yield surface: no further return
    _, dp, _ = P.return_map(E, prob.ep, prob.p, LAM, MU, SY, H)
    assert dp.max() < 1e-14
    assert np.abs(np.einsum("...ii->...", prob.ep)).max() < 1e-15


def test_two_phase_plane_strain_solve_and_unloading():
    """Heterogeneous plane-strain cell, biaxial loading then partial unloading: equilibrium at
    convergence, plastic strain only where the trial state yielded, and elastic unloading (no new
    plastic strain, stress change given by the consistent elastic tangent)."""
    from paper_2408_03804_amd import workloads
    n = 12
    phase = workloads.centered_disk(n, 0.3)
    sy = np.where(phase == 1, 2 * SY, SY)
    Hh = np.where(phase == 1, 2 * H, H)
    prob = P.PlasticProblem((n, n), LAM, MU, sy, Hh)
    load = np.array([0.02, 0.02, 0.0])
    r1 = newton_cg.solve(prob, load, n_increments=4, tol_cg=1e-12)
    assert r1["stats"]["status"] == "ok"
    F1 = r1["state"].field
    assert np.linalg.norm(prob.G(prob.stress(F1))) < 1e-8 * np.linalg.norm(prob.stress(F1))
    p1 = prob.plastic_strain_now(F1)
    assert p1.max() > 0
    r2 = newton_cg.solve(prob, 0.9 * load, n_increments=1, state=r1["state"], tol_cg=1e-12)
    assert r2["stats"]["status"] == "ok"
    p2 = prob.plastic_strain_now(r2["state"].field)
    assert np.abs(p2 - p1).max() < 1e-14  # unloading is elastic


def test_unloading_to_zero_macro_strain_converges_with_residual_stresses():
    """Unloading a yielded cell to exactly zero macro strain leaves residual stresses; the Newton
    test then scales the update by the field's own norm (the macro norm is zero) and converges,
    with a finite residual and an equilibrated residual stress field."""
    from paper_2408_03804_amd import workloads
    n = 12
    phase = workloads.centered_disk(n, 0.3)
    prob = P.PlasticProblem((n, n), LAM, MU, np.where(phase == 1, 2 * SY, SY), np.where(phase == 1, 2 * H, H))
    r1 = newton_cg.solve(prob, np.array([0.02, 0.02, 0.0]), n_increments=4, tol_cg=1e-12)
    r2 = newton_cg.solve(prob, np.zeros(3), n_increments=2, state=r1["state"], tol_cg=1e-12)
    assert r2["stats"]["status"] == "ok" and r2["stats"]["newton"] >= 1
    F = r2["state"].field
    assert np.abs(F.reshape(-1, 2, 2).mean(axis=0)).max() < 1e-15
    sig = prob.stress(F)
    assert np.linalg.norm(sig) > 1e-4 * np.linalg.norm(prob.stress(r1["state"].field))  # residual stresses
    assert np.linalg.norm(prob.G(sig)) < 1e-8 * np.linalg.norm(sig)  # in equilibrium
    # under strain control the mean plastic strain leaves a macro stress at zero macro strain
    assert np.all(np.isfinite(r2["macro_stress"])) and np.abs(r2["macro_stress"]).max() > 0


def _ps_problem(shape, lam, mu, sy, H, rng=None):
    pr = P.PlasticPlaneStressProblem(shape, lam, mu, sy, H)
    if rng is not None:  # a committed plastic history: deviatoric eps_p, p >= |eps_p|
        A = 2e-3 * rng.standard_normal(shape + (3, 3))
        ep = 0.5 * (A + np.swapaxes(A, -1, -2))
        ep[..., 0, 2] = ep[..., 2, 0] = ep[..., 1, 2] = ep[..., 2, 1] = 0.0
        ep[..., 2, 2] = -(ep[..., 0, 0] + ep[..., 1, 1])
        pr.ep = ep
        pr.p = np.sqrt(2.0 / 3.0 * np.einsum("...ij,...ij->...", ep, ep)) + 1e-3
    return pr


@pytest.mark.parametrize("history", [False, True])
def test_plane_stress_j2_has_no_out_of_plane_stress_and_stays_on_the_surface(history):
    """Pins the J2 plane-stress oracle: the 3D stress at the completed strain has no out-of-plane
    entries, and where the step is plastic its von Mises stress is sig_y + H (p + dp)."""
    rng = np.random.default_rng(50)
    shape = (5, 8)
    lam, mu = scal(1.3, shape), scal(0.8, shape)
    sy, H = scal(4e-3, shape), scal(0.1, shape)
    pr = _ps_problem(shape, lam, mu, sy, H, rng if history else None)
    E = random_sym(rng, shape, 2, 1e-2)
    s3 = pr.stress3(E)
    scale = np.abs(s3).max()
    assert np.abs(s3[..., 2, :]).max() < 1e-13 * scale and np.abs(s3[..., :, 2]).max() < 1e-13 * scale
    _, dp, _ = P.return_map(pr.full(E), pr.ep, pr.p, lam, mu, sy, H)
    assert (dp > 0).mean() > 0.5
    dev = s3 - np.einsum("...ii->...", s3)[..., None, None] / 3.0 * np.eye(3)
    seq = np.sqrt(1.5 * np.einsum("...ij,...ij->...", dev, dev))
    pl = dp > 0
    assert np.abs(seq[pl] - (sy + H * (pr.p + dp))[pl]).max() < 1e-12 * scale


def test_plane_stress_j2_equibiaxial_closed_form():
    """Equibiaxial in-plane strain e from a virgin state: sigma_11 = sigma_22 = sig_y + H dp with
    dp = (2 mu (3 lam + 2 mu) e / (lam + 2 mu) - sig_y) / (mu (3 lam + 2 mu) / (lam + 2 mu) + H) and
    eps_33 = -(2 lam e + 2 mu dp) / (lam + 2 mu), worked out by hand from sigma_33 = 0 and the radial
    return (N = diag(1/2, 1/2, -1) for this stress)."""
    lam, mu, sy, H = 1.7, 0.9, 3e-3, 0.15
    e = np.array([[5e-4, 4e-3], [1e-2, 5e-2]])
    shape = e.shape
    pr = P.PlasticPlaneStressProblem(shape, lam, mu, sy, H)
    E = e[..., None, None] * np.eye(2)
    k = lam + 2 * mu
    dp = np.maximum(2 * mu * (3 * lam + 2 * mu) * e / k - sy, 0.0) / (mu * (3 * lam + 2 * mu) / k + H)
    elastic = dp == 0
    assert elastic[0, 0] and elastic.sum() == 1
    sig = np.where(elastic, 2 * mu * (3 * lam + 2 * mu) * e / k, sy + H * dp)
    s = pr.stress(E)
    assert np.abs(s[..., 0, 0] - sig).max() < 1e-14 and np.abs(s[..., 1, 1] - sig).max() < 1e-14
    assert np.abs(s[..., 0, 1]).max() < 1e-16
    e33 = -(2 * lam * e + 2 * mu * dp) / k
    assert np.abs(pr.full(E)[..., 2, 2] - e33).max() < 1e-15


def test_plane_stress_j2_below_yield_is_linear_plane_stress():
    rng = np.random.default_rng(51)
    shape = (4, 5)
    lam, mu = rng.uniform(0.5, 2.0, shape), rng.uniform(0.3, 1.5, shape)
    pr = P.PlasticPlaneStressProblem(shape, lam, mu, scal(1e3, shape), scal(0.1, shape))
    E = random_sym(rng, shape, 2, 1e-2)
    ref = materials.LinearElasticPlaneStress.stress(E, lam, mu)
    assert np.abs(pr.stress(E) - ref).max() < 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("history", [False, True])
def test_plane_stress_j2_condensed_tangent_is_the_stress_derivative_and_symmetric(history):
    rng = np.random.default_rng(52)
    shape = (5, 6)
    lam, mu = scal(1.3, shape), scal(0.8, shape)
    sy, H = scal(4e-3, shape), scal(0.1, shape)
    pr = _ps_problem(shape, lam, mu, sy, H, rng if history else None)
    E = random_sym(rng, shape, 2, 1e-2)
    dE = random_sym(rng, shape, 2, 1.0)
    dG = random_sym(rng, shape, 2, 1.0)
    h = 1e-8
    fd = (pr.stress(E + h * dE) - pr.stress(E - h * dE)) / (2 * h)
    K = pr.tangent_apply(E, dE)
    assert np.abs(K - fd).max() < 1e-6 * np.abs(K).max()
    KG = pr.tangent_apply(E, dG)
    a = np.einsum("...ij,...ij->...", dG, K)
    b = np.einsum("...ij,...ij->...", dE, KG)
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()
    # plane stress is softer than plane strain along the in-plane normal strain
    one = np.zeros(shape + (2, 2))
    one[..., 0, 0] = 1.0
    ps = pr.tangent_apply(E, one)[..., 0, 0]
    pe = P.tangent_apply(pr.full(E), P.embed(one), pr.ep, pr.p, lam, mu, sy, H)[..., 0, 0]
    assert (ps < pe).all()
