"""Adjoint density gradient (SIMP) of the HIP path: oracle parity, envelope form,
finite differences of full solves, and the torch.autograd.Function wrapper."""

import numpy as np
import pytest

from helpers import field_err, lame_fields, rel
from oracle import adjoint, newton_cg
from paper_2408_03804_amd import workloads

pytestmark = pytest.mark.gpu


def make(shape, kin, mat, nphase=2, **kw):
    from paper_2408_03804_amd.binding import FFTHomog
    return FFTHomog(shape, kin, mat, nphase, density=True, **kw)


def oracle_problem(shape, mat, phase, table, rho, p):
    lam, mu = lame_fields(phase, table, rho, p)
    return newton_cg.Problem(shape, mat, lam, mu)


@pytest.mark.parametrize("mat,kin,shape", [("neo_hookean", "finite", (6, 5, 7)), ("linear_elastic", "small", (9, 8)),
                                           ("stvk", "finite", (5, 6))])
def test_adjoint_gradient_matches_oracle(mat, kin, shape):
    d = len(shape)
    rng = np.random.default_rng(31)
    phase = workloads.random_phases(shape, 2, 32)
    table = [[1.0, 1.0], [4.0, 3.0]]
    rho = rng.uniform(0.05, 1.0, shape)
    p = 3.0
    if kin == "small":
        macro = 0.01 * rng.standard_normal(3 if d == 2 else 6)
    else:
        macro = (np.eye(d) + 0.03 * rng.standard_normal((d, d))).reshape(-1)
    ws = rng.standard_normal(len(macro))
    we = 0.4
    h = make(shape, kin, mat, tol_cg=1e-13, tol_newton=1e-12)
    h.set_material(phase, table, rho, p)
    h.solve(macro, 2)
    g, st = h.adjoint(ws, we)
    assert st["status"] == "ok" and st["cg_total"] > 0
    prob = oracle_problem(shape, mat, phase, table, rho, p)
    ref = newton_cg.solve(prob, macro, n_increments=2, tol_newton=1e-12, tol_cg=1e-13)
    gref, k = adjoint.simp_gradient(prob, ref["state"], rho, p, ws, we, tol_cg=1e-13)
    assert field_err(g.cpu().numpy(), gref) < 1e-10
    # counts at tol 1e-13 sit in CG's stagnation regime, where rounding moves them by a few
    assert abs(st["cg_total"] - k) <= max(2, 0.03 * k)


def test_energy_gradient_is_envelope_form_without_cg():
    w = workloads.workload_neohookean3d(n=16, correlation_length=4.0)
    rho = workloads.simp_density(w["shape"], 4.0, 7)
    h = make(w["shape"], "finite", "neo_hookean")
    h.set_material(w["phase"], w["table"], rho, 3.0)
    h.solve(w["macro"], 4)
    g, st = h.adjoint(np.zeros(9), 1.0)
    assert st["cg_total"] == 0
    psi = h.get_field(2).cpu().numpy()
    assert field_err(g.cpu().numpy(), 3.0 * psi / (psi.size * rho)) < 1e-14


def _fd_check(w, rho, ws, we, nvox, seed, tol, tol_cg=1e-10, tol_newton=1e-10, max_cg=20000):
    """Central differences of full solves (restarted from the converged base state) on random voxels.

    The energy part of J(rho + h) - J(rho - h) is summed voxel by voxel.  Away from the perturbed
    voxel the energy difference is taken by the trapezoid rule, psi(F+) - psi(F-) =
    (P(F+) + P(F-)) : (F+ - F-) / 2 up to O(|F+ - F-|^3), because the energies themselves are
    O(strain^2) values assembled from O(mu |F|^2) terms whose rounding, different in the two
    solves, would swamp an O(h) change summed over N voxels.  At the perturbed voxel, whose
    parameters differ, the energies are differenced directly.

    Besides the relative tolerance, each comparison allows the rounding floor of the quotient.  The
    two solves add different Newton updates to the same base field, so every entry of their
    fields carries an independent rounding error of about u |F| per update (u = 2^-53), an error
    that is not a compatible field, so equilibrium does not cancel it.  Through P : dF (and K : dF
    for the stress part) it adds a random term of size sqrt(2 n N) u |P| |F| to the voxel sum,
    which the quotient divides by 2 h N; the stress part also differences P itself, an O(strain)
    value assembled from O((lam + 2 mu) |F|) terms.  The bound takes four times those sizes.
    """
    shape = w["shape"]
    h = make(shape, "finite", "neo_hookean", tol_cg=tol_cg, tol_newton=tol_newton, max_cg=max_cg)
    h.set_material(w["phase"], w["table"], rho, 3.0)
    out, psi, st = h.solve(w["macro"], w["n_increments"])
    assert st["status"] == "ok"
    g, sa = h.adjoint(ws, we)
    assert sa["status"] == "ok"
    g = g.cpu().numpy()
    base = h.get_field(0).clone()
    N = rho.size
    u = 2.0 ** -53
    Fb = base.cpu().numpy().reshape(9, -1)
    Pb = h.get_field(1).cpu().numpy().reshape(9, -1)
    rmsF = np.sqrt(np.mean(np.sum(Fb * Fb, axis=0)))
    rmsP = np.sqrt(np.mean(np.sum(Pb * Pb, axis=0)))
    lam_v, mu_v = lame_fields(w["phase"], w["table"], rho, 3.0)
    kmod = (lam_v + 2.0 * mu_v).reshape(-1)
    kmax = 2.0 * kmod.max()
    rms_pterm = np.sqrt(np.mean((kmod * np.sqrt(np.sum(Fb * Fb, axis=0))) ** 2))
    rng = np.random.default_rng(seed)
    flat = rng.choice(rho.size, nvox, replace=False)
    for f in flat:
        v = np.unravel_index(f, shape)
        hstep = 1e-3 * rho[v]
        fields = []
        n_upd = 0
        for sgn in (1.0, -1.0):
            r2 = rho.copy()
            r2[v] += sgn * hstep
            h.set_material(w["phase"], w["table"], r2, 3.0)
            h.set_field(base, w["macro"])
            o2, _, st2 = h.solve(w["macro"], 1)
            assert st2["status"] == "ok"
            n_upd = max(n_upd, st2["newton"])
            fields.append((h.get_field(2).cpu().numpy().reshape(-1), h.get_field(1).cpu().numpy().reshape(9, -1),
                           h.get_field(0).cpu().numpy().reshape(9, -1)))
        (psi_p, P_p, F_p), (psi_m, P_m, F_m) = fields
        dpsi_vox = 0.5 * np.sum((P_p + P_m) * (F_p - F_m), axis=0)
        dpsi_vox[f] = psi_p[f] - psi_m[f]
        dpsi = np.sum(dpsi_vox) / N
        dP = np.sum(P_p - P_m, axis=1) / N
        fd = (we * dpsi + np.dot(ws, dP)) / (2 * hstep)
        root = np.sqrt(2.0 * max(n_upd, 1) * N)
        noise = 4.0 * u * root * (rmsF * (abs(we) * rmsP + np.linalg.norm(ws) * kmax)
                                  + 2.0 * np.linalg.norm(ws) * rms_pterm)
        floor = noise / (2 * hstep * N)
        assert abs(fd - g[v]) <= tol * abs(g[v]) + floor, (v, fd, g[v], floor)
    return st, sa


# Densities down to 0.2 at the larger grids: with rho down to 0.01 and p = 3 the stiffness spans
# ~2e7, and the unpreconditioned CG of the method needs ~2e4 iterations per Newton step already at
# 16^3 (test_full_density_range_finite_differences covers that range there).
RHO_MIN = 0.2


def test_full_density_range_finite_differences():
    """The SIMP range rho in [0.01, 1] of the workload (E = rho^3 E0, phase contrast 20: stiffness
    spanning ~2e7) at 16^3, where the unpreconditioned CG is affordable: an objective with both an
    energy and a stress part (the adjoint CG runs) against central differences of full solves on
    20 random voxels.  CG: about 16,000-22,000 iterations per Newton step at tolerance 1e-11, near
    the floor that rounding leaves at this conditioning (at 1e-12 some solves stagnate just above
    the tolerance)."""
    w = workloads.workload_neohookean3d(n=16, correlation_length=4.0)
    w["n_increments"] = 2
    rho = workloads.simp_density(w["shape"], 4.0, 2, rho_min=0.01)
    assert rho.min() < 0.02 and rho.max() > 0.98
    ws = np.zeros(9)
    ws[0] = 1.0
    ws[1] = 0.5
    st, sa = _fd_check(w, rho, ws, 0.3, 20, 5, 1e-5, tol_cg=1e-11, tol_newton=1e-12, max_cg=100000)
    assert min(st["cg"]) > 10000 and sa["cg_total"] > 10000


def test_energy_gradient_finite_differences_128_bench_configuration():
    """The 128^3 workload with a SIMP density: d psi-bar / d rho on 20 random voxels."""
    w = workloads.workload_neohookean3d(n=128)
    rho = workloads.simp_density(w["shape"], 8.0, 1, rho_min=RHO_MIN)
    # each voxel's gradient is O(1/N) ~ 3e-11: the equilibrium residual left by the solver
    # tolerance enters as (1/N) <r, dF/drho_v>, ~2e-5 relative at 1e-10, ~2e-7 at 1e-12; the
    # rounding floor of the quotient (see _fd_check) is ~2e-6 relative at this size
    _fd_check(w, rho, np.zeros(9), 1.0, 20, 3, 1e-5, tol_cg=1e-12, tol_newton=1e-12)


def test_stress_gradient_finite_differences_adjoint_cg():
    """A non-energy objective (P-bar_11 + P-bar_12) exercises the adjoint CG solve."""
    w = workloads.workload_neohookean3d(n=24, correlation_length=6.0)
    w["n_increments"] = 3
    rho = workloads.simp_density(w["shape"], 6.0, 2, rho_min=RHO_MIN)
    ws = np.zeros(9)
    ws[0] = 1.0
    ws[1] = 0.5
    _fd_check(w, rho, ws, 0.0, 20, 4, 1e-5, tol_cg=1e-13, tol_newton=1e-12)


def test_autograd_function_backward_is_the_adjoint():
    import torch

    from paper_2408_03804_amd.autograd import homogenized_objective
    w = workloads.workload_neohookean3d(n=12, correlation_length=3.0)
    rho = torch.tensor(workloads.simp_density(w["shape"], 3.0, 5), dtype=torch.float64, device="cuda",
                       requires_grad=True)
    h = make(w["shape"], "finite", "neo_hookean", tol_cg=1e-12, tol_newton=1e-12)
    ws = np.zeros(9)
    ws[4] = 1.0
    J = homogenized_objective(rho, h, w["phase"], w["table"], 3.0, w["macro"], 2, ws, 0.3)
    J.backward()
    g_auto = rho.grad.cpu().numpy()
    g_adj, _ = h.adjoint(ws, 0.3)
    assert np.array_equal(g_auto, g_adj.cpu().numpy())
    # J equals the oracle's objective at the same density
    prob = oracle_problem(w["shape"], "neo_hookean", w["phase"], w["table"], rho.detach().cpu().numpy(), 3.0)
    ref = newton_cg.solve(prob, w["macro"], n_increments=2, tol_newton=1e-12, tol_cg=1e-12)
    # homogenized values are compared relative to the size of the homogenized quantities (the stress
    # norm and the weighted energy), as everywhere else: J's stress part is a small component of P-bar
    scale = abs(0.3 * ref["energy"]) + np.abs(ref["macro_stress"]).max()
    assert abs(float(J) - adjoint.objective(prob, ref["state"], ws, 0.3)) < 1e-11 * scale
