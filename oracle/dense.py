"""Dense assembly of small operators (a lattice of at most a few hundred sites):
column k of the matrix is the operator applied to the k-th unit vector of the
canonical [t][z][y][x][colour][spin] ordering."""
import numpy as np


def assemble(apply, dims):
    lx, ly, lz, lt = dims
    shape = (lt, lz, ly, lx, 3, 4)
    n = int(np.prod(shape))
    M = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        e[k] = 1.0
        M[:, k] = apply(e.reshape(shape)).reshape(n)
        e[k] = 0.0
    return M
