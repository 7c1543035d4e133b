"""init-CG, plain FP64 (test infrastructure only).

Section 2.1, eq. (2.1): given a basis ``U`` of approximate eigenvectors and
``H = U^H A U``, the Galerkin (oblique) projection of an initial guess is

    x_0 = xt_0 + U H^{-1} U^H (b - A xt_0)

and CG is then started from ``x_0``.  ``H`` is Hermitian positive definite when
``U`` has full rank, so the solve uses a Cholesky factorisation (reading: the
paper writes ``H^{-1}``).

Section 5.3 restarts init-CG once, when the residual norm comes within an
order of magnitude of machine precision scaled by the norm of the matrix,
deflating the current iterate again (the deflation cost is paid twice,
Section 5.5).  Reading: the restart fires when ``||r|| / ||b||`` first falls
to ``restart_tol``; the caller chooses ``restart_tol`` (``10 u ||A||`` with the
single-precision unit roundoff ``u = 2^-24`` of the paper's runs, Section 5.1, and
``||A||`` estimated by the largest known Ritz value; or 0 for no restart).
"""

from __future__ import annotations

import numpy as np

from .cg import cg


def galerkin_guess(apply_A, U, H, b, x_tilde=None):
    """eq. (2.1): ``x0 = xt + U H^{-1} U^H (b - A xt)`` (``xt = 0`` if omitted)."""
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    if U is None or U.shape[1] == 0:
        return np.zeros_like(b) if x_tilde is None else np.array(x_tilde, dtype=np.complex128)
    if x_tilde is None:
        res = b
        base = np.zeros_like(b)
    else:
        base = np.asarray(x_tilde, dtype=np.complex128).reshape(-1)
        res = b - apply_A(base)
    L = np.linalg.cholesky(H)
    c = U.conj().T @ res
    y = np.linalg.solve(L, c)
    y = np.linalg.solve(L.conj().T, y)
    return base + U @ y


def init_cg(apply_A, U, H, b, tol=1e-10, restart_tol=0.0, max_iter=100000,
            first_leg_iters=None, second_leg_iters=None):
    """Deflated solve: Galerkin guess, CG, optionally one restart (Section 5.3).

    Returns ``(x, info)`` with ``iterations`` summed over both CG runs and
    ``restarted`` telling whether the restart happened.

    ``first_leg_iters`` / ``second_leg_iters`` (test support) run exactly that
    many iterations in the leg before / after the restart instead of stopping
    at its tolerance.  Stop tests compare a recursively updated residual with a
    tolerance, so an implementation with different rounding may stop one
    iteration apart; these give the oracle's own iterates either side of its
    stop without changing any arithmetic.
    """
    x0 = galerkin_guess(apply_A, U, H, b)
    if restart_tol > tol or first_leg_iters is not None:
        if first_leg_iters is None:
            x1, info1 = cg(apply_A, b, x0=x0, tol=restart_tol, max_iter=max_iter)
        else:
            x1, info1 = cg(apply_A, b, x0=x0, tol=0.0, max_iter=first_leg_iters,
                           true_residual_restarts=0)
        x0 = galerkin_guess(apply_A, U, H, b, x_tilde=x1)
        if second_leg_iters is None:
            x, info2 = cg(apply_A, b, x0=x0, tol=tol,
                          max_iter=max(0, max_iter - info1["iterations"]))
        else:
            x, info2 = cg(apply_A, b, x0=x0, tol=0.0, max_iter=second_leg_iters,
                          true_residual_restarts=0)
        info = dict(info2)
        info["iterations"] = info1["iterations"] + info2["iterations"]
        info["first_leg_iterations"] = info1["iterations"]
        info["restarted"] = True
        return x, info
    if second_leg_iters is None:
        x, info = cg(apply_A, b, x0=x0, tol=tol, max_iter=max_iter)
    else:
        x, info = cg(apply_A, b, x0=x0, tol=0.0, max_iter=second_leg_iters,
                     true_residual_restarts=0)
    info["restarted"] = False
    info["first_leg_iterations"] = info["iterations"]
    return x, info
