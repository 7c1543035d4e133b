"""Spectral preconditioning with a bank of approximate eigenvectors, plain
NumPy FP64 (test infrastructure only).

Section 2.1 names the use of a deflation space U as a spectral
preconditioner as the alternative to init-CG that keeps deflation effective
below the accuracy of U, at a higher cost per iteration; Section 4 reports
that the window V of one eigCG run used that way speeds the next solve more
than init-CG deflation does.  The paper does not write the preconditioner
out.  The reading used here is the standard one for an orthonormal basis of
Ritz vectors ``U`` with Ritz values ``theta`` (``U^H A U = diag(theta)``):

    P^{-1} = I + U (sigma diag(theta)^{-1} - I) U^H ,

which maps the Ritz directions' eigenvalues to ``sigma`` (exactly, for exact
eigenvectors) and leaves the orthogonal complement unchanged, so with
``sigma`` at the top of the spectrum the condition number becomes
``lambda_max / lambda_{l+1}``.  ``P^{-1}`` is Hermitian positive definite for
``sigma > 0`` and ``theta > 0``.  A bank ``(U, H)`` whose ``H = U^H A U`` is
not diagonal is first rotated to its Ritz basis (``H Y = Y Theta``,
``U <- U Y``), which is what ``ritz_basis`` does.
"""

from __future__ import annotations

import numpy as np


def ritz_basis(U, H):
    """Rayleigh-Ritz on a bank: ``(U Y, theta)`` with ``H Y = Y diag(theta)``."""
    theta, Y = np.linalg.eigh(0.5 * (H + H.conj().T))
    return U @ Y, theta


def spectral_preconditioner(U, theta, sigma):
    """``z = P^{-1} r = r + U ((sigma / theta - 1) * (U^H r))`` for orthonormal
    Ritz vectors ``U`` (n x l) and their values ``theta`` (l)."""
    U = np.asarray(U, dtype=np.complex128)
    d = sigma / np.asarray(theta, dtype=np.float64) - 1.0
    if not (sigma > 0 and np.all(np.asarray(theta) > 0)):
        raise ValueError("the spectral preconditioner needs sigma > 0 and theta > 0")

    def apply_Pinv(r):
        r = np.asarray(r, dtype=np.complex128)
        return r + U @ (d * (U.conj().T @ r))

    return apply_Pinv
