"""The seeded input generators produce the microstructures their docstrings state."""

import numpy as np

from paper_2408_03804_amd import workloads


def test_disk_31_has_185_voxels():
    assert int(workloads.centered_disk(31, 0.25).sum()) == 185


def test_grf_threshold_exact_fraction_and_seeded():
    a = workloads.grf_two_phase((16, 16, 16), 4.0, 0.3, 5)
    b = workloads.grf_two_phase((16, 16, 16), 4.0, 0.3, 5)
    assert int(a.sum()) == round(0.3 * 16 ** 3)
    assert np.array_equal(a, b)


def test_rsa_spheres_fraction_and_separation():
    ph = workloads.rsa_spheres(32, 3.0, 6.0, 0.2, 1)
    assert 0.1 < ph.mean() <= 0.2


def test_simp_density_range():
    rho = workloads.simp_density((8, 8, 8), 2.0, 3)
    assert rho.min() >= 0.01 and rho.max() <= 1.0


def test_workload_tables():
    w = workloads.workload_neohookean3d(n=8, correlation_length=2.0)
    assert w["table"][1, 1] == 20.0 and w["table"][1, 0] == 40.0
    assert w["macro"][0] == 1.05 and w["n_increments"] == 10


def test_uq_cells_follow_their_recipe():
    cells = workloads.workload_uq_cells(n_cells=12, sizes=(8, 12), seed=3)
    again = workloads.workload_uq_cells(n_cells=12, sizes=(8, 12), seed=3)
    assert {c["shape"] for c in cells} <= {(8, 8, 8), (12, 12, 12)}
    assert len({c["shape"] for c in cells}) == 2
    for c, d in zip(cells, again):
        assert np.array_equal(c["phase"], d["phase"]) and np.array_equal(c["table"], d["table"])
        assert 4.0 <= c["correlation_length"] <= 12.0 and 0.1 <= c["stiff_fraction"] <= 0.5
        n = c["phase"].size
        assert int(c["phase"].sum()) == int(round(c["stiff_fraction"] * n))
        lam0, mu0 = c["table"][0]
        lam1, mu1 = c["table"][1]
        assert abs(mu1 / mu0 - 10.0) < 1e-12 and abs(lam1 / lam0 - 10.0) < 1e-12
        assert abs(lam0 / mu0 - 2 * 0.3 / (1 - 2 * 0.3)) < 1e-12
