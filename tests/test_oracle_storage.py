"""Reduced-precision storage classes: the F16S round-trip error bound, zero sites,
and reconstruct-12 exactness for special unitary links."""
import numpy as np

import latgen
from oracle import storage


def test_f16s_bound():
    rng = np.random.default_rng(0)
    psi = (rng.standard_normal((50, 3, 4)) + 1j * rng.standard_normal((50, 3, 4))) * rng.uniform(1e-3, 1e3, (50, 1, 1))
    q, s = storage.f16s_quantize(psi)
    back = storage.f16s_dequantize(q, s)
    # |stored / scale| <= 1 and FP16 keeps 11 significant bits: error <= 2^-11 scale (+ FP32 rounding)
    err = np.abs(back - psi).reshape(50, -1).max(axis=1)
    assert np.all(err <= (2.0 ** -11 + 2.0 ** -22) * s * np.sqrt(2))
    assert np.all(np.abs(q.astype(np.float32)) <= 1)


def test_f16s_zero_site():
    psi = np.zeros((2, 3, 4), dtype=complex)
    psi[1, 0, 0] = 2 - 1j
    q, s = storage.f16s_quantize(psi)
    assert s[0] == 0 and np.all(q[0] == 0) and s[1] == 2
    assert np.array_equal(storage.f16s_dequantize(q, s), psi)


def test_reconstruct12_exact():
    u = latgen.haar_su3(latgen.rng(9, 0, 0), 1000)
    assert np.abs(storage.reconstruct12(u[:, :2, :]) - u).max() < 1e-14
    u2 = latgen.expih_su3(latgen.rng(9, 0, 0), 1000, 0.4)
    assert np.abs(storage.reconstruct12(u2[:, :2, :]) - u2).max() < 1e-14
