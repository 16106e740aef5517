"""Euclidean gamma matrices in a chiral basis.

The paper gives only identities for the spin matrices (Fig. "id"): each
gamma[d] is Hermitian, gamma_5 is Hermitian, diagonal and squares to one, and
gamma_5 anticommutes with every gamma[d]; Sec. 4.2 adds that the spin factors
of the hopping terms have exactly two non-zeros per row, each in {1,-1,i,-i}.
Those identities do not fix a basis.  The basis used here satisfies all of
them: gamma_mu = [[0, B_mu], [B_mu^dagger, 0]] in 2x2 blocks with
B_k = -i sigma_k (k = x, y, z) and B_t = 1, so that
gamma_5 = gamma_x gamma_y gamma_z gamma_t = diag(1, 1, -1, -1).
Spin index order is 0..3, direction order mu = 0..3 = x, y, z, t.
"""
import numpy as np

SIGMA = [
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]
BLOCK = [-1j * SIGMA[0], -1j * SIGMA[1], -1j * SIGMA[2], np.eye(2, dtype=np.complex128)]


def _gamma(b):
    g = np.zeros((4, 4), dtype=np.complex128)
    g[0:2, 2:4] = b
    g[2:4, 0:2] = np.conj(b.T)
    return g


GAMMA = np.array([_gamma(b) for b in BLOCK])          # shape (4, 4, 4): GAMMA[mu]
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ID4 = np.eye(4, dtype=np.complex128)
P_MINUS = np.array([ID4 - GAMMA[mu] for mu in range(4)])   # 1 - gamma_mu (forward hop)
P_PLUS = np.array([ID4 + GAMMA[mu] for mu in range(4)])    # 1 + gamma_mu (backward hop)
