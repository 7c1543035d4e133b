"""Incremental eigCG, plain FP64 (test infrastructure only).

Section 4 algorithm box: for each of the first ``s1`` right-hand sides

    x_0 = U H^{-1} U^H b_i                      (init-CG part, eq. (2.1))
    [x_i, V, M] = eigCG(nev, m, A, x_0, b_i)
    Vbar = V orthonormalised against U
    W = A Vbar
    H = [[H, U^H W], [W^H U, Vbar^H W]]         (nev new rows and columns)
    U = [U, Vbar]

Readings: the paper treats the orthonormalisation as optional;
here it is always done, by classical Gram-Schmidt applied twice against ``U``
and then inside ``Vbar`` (column by column, again twice).  A column whose norm
after projection falls below ``drop_tol`` times its norm before is dropped, so
``H`` stays well conditioned.  The convergence target is ``||r|| / ||b||``.
"""

from __future__ import annotations

import numpy as np

from .eigcg import eigcg
from .initcg import galerkin_guess


def orthonormalize_against(U, V, drop_tol=1e-10):
    """CGS2 of the columns of ``V`` against ``U`` and then among themselves.

    Returns the kept orthonormal columns (n, k' <= k).
    """
    V = np.array(V, dtype=np.complex128)
    norms_in = np.linalg.norm(V, axis=0)
    if U is not None and U.shape[1] > 0:
        for _ in range(2):
            V = V - U @ (U.conj().T @ V)
    kept = []
    for c in range(V.shape[1]):
        v = V[:, c].copy()
        before = norms_in[c]
        if before == 0.0:
            continue
        if kept:
            Q = np.stack(kept, axis=1)
            for _ in range(2):
                v = v - Q @ (Q.conj().T @ v)
        after = np.linalg.norm(v)
        if after <= drop_tol * before:
            continue
        kept.append(v / after)
    if not kept:
        return np.zeros((V.shape[0], 0), dtype=np.complex128)
    return np.stack(kept, axis=1)


def extend_bank(apply_A, U, H, Vbar):
    """Add the columns of ``Vbar`` (orthonormal, orthogonal to U) to the bank."""
    W = np.stack([apply_A(Vbar[:, c]) for c in range(Vbar.shape[1])], axis=1)
    if U is None or U.shape[1] == 0:
        Hn = Vbar.conj().T @ W
        Hn = 0.5 * (Hn + Hn.conj().T)
        return Vbar.copy(), Hn
    UW = U.conj().T @ W
    VW = Vbar.conj().T @ W
    VW = 0.5 * (VW + VW.conj().T)
    Hn = np.block([[H, UW], [UW.conj().T, VW]])
    return np.hstack([U, Vbar]), Hn


def incremental_eigcg(apply_A, rhs_list, nev, m, tol=1e-10, max_iter=100000,
                      max_bank=None, drop_tol=1e-10):
    """Run the Section 4 outer loop over ``rhs_list``; returns
    ``(xs, U, H, infos)``."""
    n = np.asarray(rhs_list[0]).size
    U = np.zeros((n, 0), dtype=np.complex128)
    H = np.zeros((0, 0), dtype=np.complex128)
    xs, infos = [], []
    for b in rhs_list:
        b = np.asarray(b, dtype=np.complex128).reshape(-1)
        x0 = galerkin_guess(apply_A, U, H, b)
        x, V, theta, info = eigcg(apply_A, b, nev, m, x0=x0, tol=tol, max_iter=max_iter)
        room = V.shape[1] if max_bank is None else max(0, min(V.shape[1], max_bank - U.shape[1]))
        Vbar = orthonormalize_against(U, V[:, :room], drop_tol=drop_tol)
        if Vbar.shape[1] > 0:
            U, H = extend_bank(apply_A, U, H, Vbar)
        info["ritz_values"] = theta
        info["bank_size"] = U.shape[1]
        xs.append(x)
        infos.append(info)
    return xs, U, H, infos


def bank_ritz(apply_A, U, H, residuals=True):
    """Rayleigh-Ritz on the bank (Section 5.2): eigenpairs of ``H`` lifted by U,
    with explicit residual norms ``||A u - theta u||`` when asked."""
    theta, Y = np.linalg.eigh(H)
    if not residuals:
        return theta, None
    X = U @ Y
    res = np.array([np.linalg.norm(apply_A(X[:, c]) - theta[c] * X[:, c])
                    for c in range(X.shape[1])])
    return theta, res
