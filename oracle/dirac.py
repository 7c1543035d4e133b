"""Wilson-Dirac operator, plain NumPy FP64 (test infrastructure only).

The paper (Section 1) writes the lattice Dirac operator as ``M = m_q I - D``,
gamma5-Hermitian (``gamma5 M = M^H gamma5`` with gamma5 diagonal with entries
+1 and -1), and solves with CG on the Hermitian positive definite ``A = M^H M``.
The paper does not print D; the Wilson form used throughout this project is

    (M psi)(x) = (4 + m_q) psi(x)
                 - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x)            psi(x + mu)
                              + (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu) ]

on a periodic 4D lattice, i.e. ``D`` is the Wilson hopping term and the
diagonal shift is ``4 + m_q``.

Gamma matrices: Euclidean, Hermitian, chiral basis (the paper only asks that
gamma5 be diagonal):

    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]   k = 1, 2, 3 (x, y, z)
    gamma_4 = [[0, I], [I, 0]]                    (t)
    gamma5  = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1)

The adjoint ``M^H`` is implemented here as its own stencil (the adjoint of each
hopping term), *not* through gamma5, so that gamma5-Hermiticity is something
the tests check rather than something assumed.

Array conventions come from ``synthetic``: spinors are
``(Lt, Lz, Ly, Lx, 4, 3)`` complex128, links ``(Lt, Lz, Ly, Lx, 4, 3, 3)``;
direction mu = 0, 1, 2, 3 is x, y, z, t, i.e. array axis 3, 2, 1, 0.
"""

from __future__ import annotations

import numpy as np

_SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)
_I2 = np.eye(2, dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)


def _block(a, b, c, d):
    return np.block([[a, b], [c, d]])


GAMMA = (
    _block(_Z2, -1j * _SIGMA[0], 1j * _SIGMA[0], _Z2),  # x
    _block(_Z2, -1j * _SIGMA[1], 1j * _SIGMA[1], _Z2),  # y
    _block(_Z2, -1j * _SIGMA[2], 1j * _SIGMA[2], _Z2),  # z
    _block(_Z2, _I2, _I2, _Z2),                         # t
)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
IDENTITY4 = np.eye(4, dtype=np.complex128)

# array axis of lattice direction mu in a (Lt, Lz, Ly, Lx, ...) array
_AXIS = (3, 2, 1, 0)


def _spin(mat, psi):
    """Apply a 4x4 spin matrix to every site of ``psi`` (..., 4, 3)."""
    return np.einsum("st,...ta->...sa", mat, psi)


def _colour(links, psi):
    """Apply per-site 3x3 colour matrices ``links`` (..., 3, 3) to ``psi``."""
    return np.einsum("...ab,...sb->...sa", links, psi)


def _dagger(links):
    return np.conj(np.swapaxes(links, -1, -2))


def shift_forward(field, mu):
    """``out(x) = field(x + mu)`` with periodic wrap."""
    return np.roll(field, -1, axis=_AXIS[mu])


def shift_backward(field, mu):
    """``out(x) = field(x - mu)`` with periodic wrap."""
    return np.roll(field, 1, axis=_AXIS[mu])


def hopping(U, psi, sign_forward):
    """Wilson hopping sum for M (``sign_forward = -1``) or M^H (``+1``).

    Returns ``sum_mu [(1 + s gamma_mu) U_mu(x) psi(x+mu)
                     + (1 - s gamma_mu) U_mu(x-mu)^dagger psi(x-mu)]``
    with ``s = sign_forward``.
    """
    out = np.zeros_like(psi)
    for mu in range(4):
        u = U[..., mu, :, :]
        fwd = _colour(u, shift_forward(psi, mu))
        bwd = _colour(_dagger(shift_backward(u, mu)), shift_backward(psi, mu))
        out += _spin(IDENTITY4 + sign_forward * GAMMA[mu], fwd)
        out += _spin(IDENTITY4 - sign_forward * GAMMA[mu], bwd)
    return out


def apply_M(U, mass, psi):
    """``M psi`` for a spinor field shaped (Lt, Lz, Ly, Lx, 4, 3)."""
    return (4.0 + mass) * psi - 0.5 * hopping(U, psi, -1.0)


def apply_Mdag(U, mass, psi):
    """``M^H psi``: the adjoint of every hopping term (forward and backward
    terms swap their ``1 -/+ gamma_mu`` projectors)."""
    return (4.0 + mass) * psi - 0.5 * hopping(U, psi, +1.0)


def apply_gamma5(psi):
    return _spin(GAMMA5, psi)


class WilsonOperator:
    """M, M^H and A = M^H M acting on flat complex128 vectors of length n = 12 V."""

    def __init__(self, U, mass):
        U = np.asarray(U, dtype=np.complex128)
        if U.ndim != 7 or U.shape[4:] != (4, 3, 3):
            raise ValueError("gauge field must be (Lt, Lz, Ly, Lx, 4, 3, 3)")
        self.U = U
        self.mass = float(mass)
        self.site_shape = U.shape[:4]
        self.dims = (U.shape[3], U.shape[2], U.shape[1], U.shape[0])
        self.n = 12 * int(np.prod(self.site_shape))

    def _field(self, v):
        return np.asarray(v, dtype=np.complex128).reshape(self.site_shape + (4, 3))

    def M(self, v):
        return apply_M(self.U, self.mass, self._field(v)).reshape(-1)

    def Mdag(self, v):
        return apply_Mdag(self.U, self.mass, self._field(v)).reshape(-1)

    def A(self, v):
        """``A v = M^H (M v)`` (Section 1: CG is applied to A = M^H M)."""
        return self.Mdag(self.M(v))

    def gamma5(self, v):
        return apply_gamma5(self._field(v)).reshape(-1)

    def A_block(self, V):
        """A applied to every column of an (n, k) block."""
        V = np.asarray(V, dtype=np.complex128)
        return np.stack([self.A(V[:, c]) for c in range(V.shape[1])], axis=1)
