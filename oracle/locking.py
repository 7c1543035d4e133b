"""Locking accurate eigenvectors out of the bank (test infrastructure only).

Section 4 discusses two ways of lowering the cost of growing ``U``; the second
is to lock eigenvectors that are already accurate so that they no longer take
part in building ``H``.  Reading taken here (the paper does not spell it out):

* ``lock_bank``: Rayleigh-Ritz on the unlocked columns, ``H_u Y = Y Theta``
  with ``H_u`` the block of ``H`` on the unlocked columns (its coupling with
  the locked block is zero by construction), ``U_u <- U_u Y``; the Ritz
  vectors whose residual ``||A u - theta u||`` is at most ``tol`` are locked.
  Locked columns come first (previously locked ones, then the new ones in
  ascending Ritz value), the unlocked Ritz vectors follow in ascending order,
  and ``H`` becomes ``diag(theta)`` on every rotated column.
* ``extend_bank_locked``: the Section 4 update of ``H`` with the rows of the
  locked columns left at zero.  The entries skipped are ``u^H A v = r^H v``
  for a locked ``u`` with residual ``r`` and a new ``v`` orthogonal to ``u``,
  so each is at most ``||r|| <= tol`` in modulus: ``H`` stays within ``tol``
  of ``U^H A U`` entry by entry.

The new vectors are still orthonormalised against every column of ``U``,
locked or not, so ``U`` keeps full rank.
"""

from __future__ import annotations

import numpy as np


def lock_bank(apply_A, U, H, nlock, tol):
    """Returns ``(U, H, nlock, theta, res)``: the bank with its unlocked
    columns rotated to Ritz vectors, the accurate ones locked, and the Ritz
    values and residual norms of the rotated columns (in their new order)."""
    l = U.shape[1]
    if nlock >= l:
        return U, H, nlock, np.zeros(0), np.zeros(0)
    theta, Y = np.linalg.eigh(H[nlock:, nlock:])
    X = U[:, nlock:] @ Y
    res = np.array([np.linalg.norm(apply_A(X[:, j]) - theta[j] * X[:, j])
                    for j in range(X.shape[1])])
    new = [j for j in range(len(theta)) if res[j] <= tol]
    rest = [j for j in range(len(theta)) if res[j] > tol]
    order = new + rest
    Un = np.hstack([U[:, :nlock], X[:, order]])
    Hn = np.zeros_like(H)
    Hn[:nlock, :nlock] = H[:nlock, :nlock]
    Hn[nlock:, nlock:] = np.diag(theta[order]).astype(np.complex128)
    return Un, Hn, nlock + len(new), theta[order], res[order]


def extend_bank_locked(apply_A, U, H, Vbar, nlock):
    """Section 4's bank update with the first ``nlock`` columns locked: their
    rows of ``U^H A Vbar`` are not formed (left at zero)."""
    W = np.stack([apply_A(Vbar[:, c]) for c in range(Vbar.shape[1])], axis=1)
    UW = np.zeros((U.shape[1], Vbar.shape[1]), dtype=np.complex128)
    UW[nlock:, :] = U[:, nlock:].conj().T @ W
    VW = Vbar.conj().T @ W
    VW = 0.5 * (VW + VW.conj().T)
    Hn = np.block([[H, UW], [UW.conj().T, VW]])
    return np.hstack([U, Vbar]), Hn
