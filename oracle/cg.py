"""Conjugate Gradient, plain FP64 (test infrastructure only).

Follows the CG algorithm in the left box of Figure 3.1 of the paper.  With
the preconditioner ``P = I`` (the default) ``z = r`` and ``rho = r^H r``;
with an SPD preconditioner given as ``apply_Pinv`` (``z = P^{-1} r``) the
same box reads

    r = b - A x;  j = 0
    while not converged:
        j += 1;  rho_prev = rho;  z = P^{-1} r;  rho = r^H z
        p = z                      (j == 1)
        p = z + beta_j p,  beta_j = rho / rho_prev   (j > 1)
        t = A p;  alpha_j = rho / (p^H t)
        x += alpha_j p;  r -= alpha_j t

Stopping rule (a reading; the paper's box tests ``||r|| / ||r_0||``): the
iteration stops when the recursive residual satisfies ``||r|| / ||b|| <= tol``.
The true residual ``||b - A x|| / ||b||`` is then recomputed; if it does not
meet ``tol`` the iteration restarts from the current ``x`` with ``r = b - A x``.
Measuring against ``||b||`` keeps the target fixed when ``x_0`` is a deflated
guess (init-CG), where ``||r_0||`` would already be small.
"""

from __future__ import annotations

import numpy as np


def _dot(a, b):
    """``a^H b``."""
    return np.vdot(a, b)


def _real_positive(val, what):
    if abs(val.imag) > 1e-10 * max(abs(val.real), 1e-300):
        raise FloatingPointError(f"{what} has a large imaginary part: {val}")
    return float(val.real)


def cg(apply_A, b, x0=None, tol=1e-10, max_iter=100000, true_residual_restarts=3,
       apply_Pinv=None):
    """Solve ``A x = b``; returns ``(x, info)``.

    ``info`` holds ``iterations``, ``alpha`` and ``beta`` (per iteration,
    ``beta[0] = 0``), ``rho`` (``r_{j-1}^H z_{j-1}`` seen at iteration j,
    ``||r_{j-1}||^2`` without a preconditioner),
    ``true_rel_res`` and ``converged``.
    """
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128).reshape(-1)
    bnorm = np.linalg.norm(b)
    info = {"alpha": [], "beta": [], "rho": [], "iterations": 0, "cg_restarts": 0}
    if bnorm == 0.0:
        x[:] = 0.0
        info.update(true_rel_res=0.0, converged=True)
        return x, info

    j = 0
    restarts = 0
    while True:
        r = b - apply_A(x)
        rho = None
        p = None
        first = True
        while np.linalg.norm(r) / bnorm > tol and j < max_iter:
            j += 1
            rho_prev = rho
            z = r if apply_Pinv is None else apply_Pinv(r)
            rho = _real_positive(_dot(r, z), "r^H z")
            if first:
                beta = 0.0
                p = z.copy()
                first = False
            else:
                beta = rho / rho_prev
                p = z + beta * p
            t = apply_A(p)
            pt = _real_positive(_dot(p, t), "p^H A p")
            if pt <= 0.0:
                raise FloatingPointError("p^H A p <= 0: A is not positive definite")
            alpha = rho / pt
            x = x + alpha * p
            r = r - alpha * t
            info["alpha"].append(alpha)
            info["beta"].append(beta)
            info["rho"].append(rho)
        true_res = np.linalg.norm(b - apply_A(x)) / bnorm
        if true_res <= tol or j >= max_iter or restarts >= true_residual_restarts:
            break
        restarts += 1
    info.update(iterations=j, true_rel_res=float(true_res),
                converged=bool(true_res <= tol), cg_restarts=restarts)
    return x, info
