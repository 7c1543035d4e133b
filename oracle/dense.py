"""Dense matrices of the lattice operators for tiny lattices (test infrastructure only).

Column ``c`` of the dense matrix is the operator applied to the unit vector
``e_c``; the dense forms feed ``numpy.linalg`` eigendecompositions and solves
that pin the iterative oracle on lattices up to 4^4 (n = 3072).
"""

from __future__ import annotations

import numpy as np


def dense_matrix(apply, n):
    out = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for c in range(n):
        e[c] = 1.0
        out[:, c] = apply(e)
        e[c] = 0.0
    return out


def dense_A(op):
    """``A = M^H M`` as an explicit matrix, built from the dense M."""
    M = dense_matrix(op.M, op.n)
    return M.conj().T @ M, M
