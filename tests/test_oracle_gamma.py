"""Pins of the spin matrices against the identities of Fig. "id" (hermiticity,
gamma_5 diagonal, squaring to one, anticommuting) and the sparsity statement
of Sec. 4.2 (two non-zeros per row in {1,-1,i,-i} for the hop spin factors),
plus the Clifford algebra that any Euclidean basis must satisfy."""
import numpy as np

from oracle.gamma import GAMMA, GAMMA5, P_MINUS, P_PLUS, ID4


def test_hermitian():
    for g in list(GAMMA) + [GAMMA5]:
        assert np.array_equal(g, np.conj(g.T))


def test_clifford():
    for m in range(4):
        for n in range(4):
            ac = GAMMA[m] @ GAMMA[n] + GAMMA[n] @ GAMMA[m]
            assert np.array_equal(ac, 2 * ID4 * (m == n))


def test_gamma5():
    assert np.array_equal(GAMMA5, np.diag([1, 1, -1, -1]).astype(complex))
    assert np.array_equal(GAMMA5 @ GAMMA5, ID4)
    for g in GAMMA:
        assert np.array_equal(GAMMA5 @ g, -g @ GAMMA5)


def test_projector_sparsity():
    allowed = {1, -1, 1j, -1j}
    for P in list(P_MINUS) + list(P_PLUS):
        for row in P:
            nz = [v for v in row if v != 0]
            assert len(nz) == 2
            assert all(complex(v) in allowed for v in nz)


def test_projectors_rank2():
    for m in range(4):
        assert np.allclose(P_MINUS[m] @ P_MINUS[m], 2 * P_MINUS[m])
        assert np.allclose(P_MINUS[m] @ P_PLUS[m], 0)
        assert np.linalg.matrix_rank(P_MINUS[m]) == 2
