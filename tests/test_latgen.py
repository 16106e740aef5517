"""Seeded input generators: group properties of the links and the statistics of
the Haar measure, the exp(i eps H) recipe against scipy's matrix exponential,
determinism of the seeds, and the point-source layout."""
import numpy as np
import scipy.linalg

import latgen


def _su3_check(u):
    eye = np.eye(3)
    assert np.abs(u @ np.conj(np.swapaxes(u, -1, -2)) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-14


def test_haar_group_and_moments():
    g = latgen.rng(5, 0, 0)
    u = latgen.haar_su3(g, 20000)
    _su3_check(u)
    # E|U_ab|^2 = 1/3 and E tr U = 0 for Haar SU(3)
    assert abs(np.mean(np.abs(u) ** 2) - 1 / 3) < 5e-3
    assert abs(np.mean(np.trace(u, axis1=1, axis2=2))) < 2e-2
    # E|tr U|^2 = 1 for Haar SU(3)
    assert abs(np.mean(np.abs(np.trace(u, axis1=1, axis2=2)) ** 2) - 1) < 5e-2


def test_expih_against_expm():
    n, eps = 50, 0.4
    u = latgen.expih_su3(latgen.rng(6, 0, 0), n, eps)
    _su3_check(u)
    a = latgen.complex_gaussian(latgen.rng(6, 0, 0), (n, 3, 3))
    for k in range(n):
        h = 0.5 * (a[k] + np.conj(a[k].T))
        h -= np.trace(h).real / 3 * np.eye(3)
        assert np.abs(u[k] - scipy.linalg.expm(1j * eps * h)).max() < 1e-13


def test_deterministic_and_distinct():
    a = latgen.make_config(0)
    b = latgen.make_config(0)
    assert np.array_equal(a["U"], b["U"]) and np.array_equal(a["b"], b["b"])
    c = latgen.make_config(3, sys=1, with_source=False)
    d = latgen.make_config(3, sys=2, with_source=False)
    assert c["dims"] == d["dims"] == (8, 8, 8, 8)
    assert not np.array_equal(c["U"], d["U"])
    assert 0.2 <= c["eps"] <= 0.5 and 0.10 <= c["kappa"] <= 0.12


def test_config_shapes():
    cfg = latgen.make_config(0)
    assert cfg["U"].shape == (4, 4, 4, 4, 4, 3, 3)
    assert cfg["b"].shape == (1, 4, 4, 4, 4, 3, 4)
    _su3_check(cfg["U"].reshape(-1, 3, 3))


def test_point_sources():
    dims = (4, 2, 2, 6)
    b = latgen.point_sources(2, 0, dims)
    x, y, z, t = latgen.point_site(2, 0, dims)
    assert b.shape == (12, 6, 2, 2, 4, 3, 4)
    for k in range(12):
        c, s = divmod(k, 4)
        assert b[k, t, z, y, x, c, s] == 1 and np.count_nonzero(b[k]) == 1
