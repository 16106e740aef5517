"""The average plaquette (a summary of how rough a gauge field is), pinned by
closed forms: 1 for unit links, (5 + cos B) / 6 for a U(1) field with flux B
through every xy plaquette, invariance under a gauge transformation, and the
Haar average 0."""
import numpy as np

import latgen
from oracle import wilson


def _unit(dims):
    lx, ly, lz, lt = dims
    U = np.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    return U


def _haar_links(seed, dims):
    n = int(np.prod(dims)) * 4
    return latgen.haar_su3(latgen.rng(78, seed, 0), n).reshape(tuple(dims[::-1]) + (4, 3, 3))


def test_unit_links():
    assert abs(wilson.plaquette(_unit((4, 4, 2, 2))) - 1.0) < 1e-15


def test_constant_flux_closed_form():
    # U_x(x, y, z, t) = exp(-i B y) 1, other links 1: the xy plaquette at every site is
    # U_x(n) U_y(n + x) U_x(n + y)^+ U_y(n)^+ = exp(i B) (periodic in y for B = 2 pi k / Ly);
    # the other five planes have plaquette 1, so the average is (5 + cos B) / 6.
    dims = (4, 6, 2, 4)
    for k in (1, 2):
        B = 2 * np.pi * k / dims[1]
        U = _unit(dims)
        y = np.arange(dims[1])
        U[:, :, :, :, 0] = np.exp(-1j * B * y)[None, None, :, None, None, None] * np.eye(3)
        assert abs(wilson.plaquette(U) - (5 + np.cos(B)) / 6) < 1e-14


def test_gauge_invariance():
    dims = (4, 4, 2, 2)
    U = _haar_links(3, dims)
    Om = latgen.random_su3_field(3, dims)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = Om @ U[..., mu, :, :] @ wilson.dagger3(wilson.shift_fwd(Om, mu))
    assert abs(wilson.plaquette(Ug) - wilson.plaquette(U)) < 1e-14


def test_haar_average_is_zero():
    # independent Haar links: E[tr P] = 0, and the average over 6 V plaquettes has
    # standard deviation about sqrt(1 / (9 * 6 V)) per real trace / 3
    dims = (8, 8, 8, 8)
    U = _haar_links(5, dims)
    assert abs(wilson.plaquette(U)) < 5 * np.sqrt(1.0 / (9 * 6 * np.prod(dims)))
