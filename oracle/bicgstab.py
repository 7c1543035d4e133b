"""Deflated BiCGSTAB on the Wilson operator M, plain FP64 (test infrastructure only).

Section 1: the paper solves with CG on ``A = M^H M`` and observes that the
eigenvectors of ``A`` are also eigenvectors of the Hermitian ``Q = gamma5 M``
(``Q^2 = A``), so once an eigCG phase has built a bank ``U`` it can deflate a
nonsymmetric solver, BiCGSTAB, on ``M x = b`` for the remaining right-hand
sides.  The paper does not spell out either part.  Readings taken here:

* BiCGSTAB is van der Vorst's method (SIAM J. Sci. Stat. Comput. 13 (1992)
  631-644) in complex arithmetic, inner products ``(a, b) = a^H b``, shadow
  residual ``rh = r_0``.  Each iteration applies ``M`` twice; when the half-step
  residual ``s`` already meets the tolerance the half step is taken and the
  iteration ends there.  When the recursive residual meets the tolerance the
  true residual ``b - M x`` is formed; if it does not meet the tolerance the
  method restarts from the current iterate (a new ``r_0`` and ``rh``).
* BiCGSTAB runs on ``Q x = gamma5 b`` (reading of "BiCGSTAB on gamma5 M"; the
  bank approximates eigenvectors of ``Q``, not of ``M``), or on ``M x = b``.
* The deflated starting guess minimises ``||b - M x||`` over
  ``x in xt + span(U)``.  Its normal equations have the matrix
  ``(M U)^H (M U) = U^H A U = H``, the bank's own matrix, so the guess is
  init-CG's eq. (2.1) applied to ``A x = M^H b``:
  ``x_0 = xt + U H^{-1} U^H M^H (b - M xt)``.  For exact eigenvectors of ``A``
  (hence of ``gamma5 M``, eigenvalues ``mu``, ``mu^2 = lambda``) it equals the
  Galerkin projection of ``gamma5 M x = gamma5 b`` onto ``span(U)``; unlike that
  projection it never raises the residual when ``U`` is approximate (the
  Galerkin matrix ``U^H gamma5 M U`` is indefinite and can be nearly singular).

Only tests/, the smoke check and the bench's CPU baseline use this module.
"""

from __future__ import annotations

import numpy as np

from .initcg import galerkin_guess


def _dot(a, b):
    return np.vdot(a, b)


def bicgstab(apply_M, b, x0=None, tol=1e-10, max_iter=10000, max_restarts=8):
    """Solve ``M x = b``; returns ``(x, info)``.

    ``info``: ``iterations`` (over all restarts), ``restarts``, ``status``
    ("ok", "max_iter" or "breakdown"), ``true_rel_res`` and the history
    ``rel_res`` of ``||r|| / ||b||`` after each iteration.
    """
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128).reshape(-1)
    bnorm = np.linalg.norm(b)
    info = {"iterations": 0, "restarts": 0, "status": "ok", "rel_res": []}
    if bnorm == 0.0:
        info["true_rel_res"] = 0.0
        return np.zeros_like(b), info
    stop = tol * bnorm
    it = 0
    while True:
        r = b - apply_M(x)
        if np.linalg.norm(r) <= stop:
            break
        if info["restarts"] > max_restarts:
            break
        rh = r.copy()
        rho_old = alpha = omega = 1.0 + 0.0j
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        converged = False
        while it < max_iter:
            rho = _dot(rh, r)
            if rho == 0.0 or omega == 0.0:
                info["status"] = "breakdown"
                break
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
            v = apply_M(p)
            rv = _dot(rh, v)
            if rv == 0.0:
                info["status"] = "breakdown"
                break
            alpha = rho / rv
            s = r - alpha * v
            it += 1
            if np.linalg.norm(s) <= stop:
                x = x + alpha * p
                r = s
                info["rel_res"].append(np.linalg.norm(s) / bnorm)
                converged = True
                break
            t = apply_M(s)
            tt = _dot(t, t)
            if tt == 0.0:
                info["status"] = "breakdown"
                break
            omega = _dot(t, s) / tt
            x = x + alpha * p + omega * s
            r = s - omega * t
            rho_old = rho
            info["rel_res"].append(np.linalg.norm(r) / bnorm)
            if np.linalg.norm(r) <= stop:
                converged = True
                break
        if not converged:
            if info["status"] == "ok":
                info["status"] = "max_iter"
            break
        # the recursion met the tolerance: check the true residual
        if np.linalg.norm(b - apply_M(x)) <= stop:
            break
        info["restarts"] += 1
    info["iterations"] = it
    info["true_rel_res"] = np.linalg.norm(b - apply_M(x)) / bnorm
    if info["status"] == "ok" and info["true_rel_res"] > tol:
        info["status"] = "max_iter"
    return x, info


def deflated_guess(apply_M, apply_Mdag, U, b, x_tilde=None):
    """``x0 = xt + U H^{-1} U^H M^H (b - M xt)``, ``H = U^H M^H M U`` formed
    here column by column (``xt = 0`` if omitted)."""
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    base = np.zeros_like(b) if x_tilde is None else np.array(x_tilde, dtype=np.complex128)
    if U is None or U.shape[1] == 0:
        return base
    apply_A = lambda v: apply_Mdag(apply_M(v))
    AU = np.stack([apply_A(U[:, j]) for j in range(U.shape[1])], axis=1)
    H = U.conj().T @ AU
    return galerkin_guess(apply_A, U, H, apply_Mdag(b), x_tilde=x_tilde)


def deflated_bicgstab(apply_M, apply_Mdag, gamma5, U, b, x0=None, tol=1e-10, max_iter=10000,
                      on_gamma5=True):
    """Deflated guess from the bank ``U``, then BiCGSTAB.

    ``on_gamma5``: iterate on ``gamma5 M x = gamma5 b`` (the Hermitian
    operator whose eigenvectors ``U`` approximates, the form Section 1 names);
    otherwise on ``M x = b``.  Both have the same solution and the same
    residual norm (gamma5 is unitary).
    """
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    xg = deflated_guess(apply_M, apply_Mdag, U, b, x_tilde=x0)
    if on_gamma5:
        x, info = bicgstab(lambda v: gamma5(apply_M(v)), gamma5(b), x0=xg, tol=tol,
                           max_iter=max_iter)
    else:
        x, info = bicgstab(apply_M, b, x0=xg, tol=tol, max_iter=max_iter)
    bnorm = np.linalg.norm(b)
    info["guess_rel_res"] = np.linalg.norm(b - apply_M(xg)) / bnorm if bnorm else 0.0
    return x, info
