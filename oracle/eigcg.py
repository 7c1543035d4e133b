"""eigCG(nev, m), plain FP64 (test infrastructure only).

Follows Figure 3.1 of the paper: the CG of ``oracle.cg`` (P = I) with the
eigCG additions of the right box, which keep a window ``V`` of at most ``m``
normalised residuals and the projection ``T = V^H A V`` built from the CG
scalars, and restart the window with the locally optimal thick restart of
eq. (2.3) using the lowest ``nev`` Ritz vectors of ``T_m`` and of ``T_{m-1}``.

Lanczos/CG relation (Section 3, eq. (3.1)): with ``v_k = r_{k-1} / sqrt(rho_k)``,

    T[k, k]     = 1/alpha_k + beta_k / alpha_{k-1}     (beta_1 / alpha_0 := 0)
    T[k, k + 1] = -sqrt(beta_{k+1}) / alpha_k

The off-diagonal sign is negative (as the figure's tridiagonal update has
it); eq. (3.1) prints it positive, which corresponds to sign-alternated
Lanczos vectors.  With the normalised residuals themselves as basis the
negative sign is the one that makes ``T = V^H A V`` (pinned by a test).

Readings where the figure is terse (each one is listed in the design notes):

* the diagonal entry filled after each new ``A p`` belongs to the *window*
  column appended in the previous iteration (window index ``i``), using
  ``alpha`` (the figure's ``a_{j-2}`` is ``alpha_{j-2}``);
* the off-diagonal update is skipped while the window is empty (j = 1);
* ``orth([Y, Ybar])`` is a thin Householder QR, so the restarted window always
  holds ``2 nev`` columns;
* ``T`` is kept complex Hermitian, since the arrow row ``w^H V`` of the
  restart is complex in floating point;
* the output (the figure returns ``[x, V, M]``) is a final Rayleigh-Ritz on
  the current ``T_i`` after filling its last diagonal entry, returning the
  ``min(nev, i)`` lowest Ritz pairs, eigenvalues ascending;
* convergence is tested on ``||r|| / ||b||`` (see ``oracle.cg``).
"""

from __future__ import annotations

import numpy as np

from .cg import _dot, _real_positive


def _lowest_eigvecs(T, k):
    """Eigenvectors of the Hermitian ``T`` for its ``k`` smallest eigenvalues."""
    w, v = np.linalg.eigh(T)
    return w[:k], v[:, :k]


def restart_coefficients(Tm, nev):
    """Restart coefficients of Figure 3.1 (eq. (2.3)) from the full window matrix ``T_m``:
    lowest Ritz vectors of ``T_m`` and ``T_{m-1}``, their orthonormal basis, and
    the Rayleigh-Ritz of ``T_m`` on it.

    Returns ``(QZ, Mvals, Q, Z, Y, Ybar)`` where ``V (QZ)`` is the restarted
    window and ``diag(Mvals)`` its projection.
    """
    m = Tm.shape[0]
    _, Y = _lowest_eigvecs(Tm, nev)                       # T_m Y = Y M
    _, Yb = _lowest_eigvecs(Tm[: m - 1, : m - 1], nev)    # T_{m-1} Ybar = Ybar Mbar
    Ybar = np.vstack([Yb, np.zeros((1, nev), dtype=Tm.dtype)])  # pad Ybar to m rows
    Q, _ = np.linalg.qr(np.hstack([Y, Ybar]), mode="reduced")   # orth([Y, Ybar])
    Hs = Q.conj().T @ Tm @ Q
    Hs = 0.5 * (Hs + Hs.conj().T)
    Mvals, Z = np.linalg.eigh(Hs)                          # Q^H T_m Q = Z M Z^H
    return Q @ Z, Mvals, Q, Z, Y, Ybar


def eigcg(apply_A, b, nev, m, x0=None, tol=1e-10, max_iter=100000, record=False,
          apply_Pinv=None):
    """Solve ``A x = b`` while computing ``nev`` Ritz pairs; returns
    ``(x, ritz_vectors (n, k), ritz_values (k,), info)``.

    ``apply_Pinv`` (``z = P^{-1} r`` for an SPD preconditioner P; default
    P = I): the preconditioned form of Section 3.  CG then runs with
    ``z = P^{-1} r``, ``rho = r^H z`` and ``p = z + beta p``, and the window
    holds ``V = P^{-1} R`` normalised, ``v = z / sqrt(rho)``, so that
    ``V^H P V = I`` and ``T = V^H A V`` is the Lanczos matrix of
    ``P^{-1/2} A P^{-1/2}`` built from the same CG scalars.  The Ritz pairs
    approximate the pencil ``A y = lambda P y``; their vectors ``V Y`` deflate
    later systems through eq. (2.1) unchanged (the derivation of Section 3
    with a general P).  The arrow row of a restart uses
    ``w = t - beta t_prev = A z``.

    ``info`` holds ``iterations``, ``alpha``, ``beta``, ``rho``,
    ``restart_iterations`` (the CG iteration j at which each restart ran) and
    ``true_rel_res``; with ``record=True`` also ``restarts`` (per restart:
    ``Tm``, ``QZ``, ``M``, ``arrow``, ``Q``, ``Z``) and the final ``T``.
    """
    if not (m > 2 * nev >= 2):
        raise ValueError("eigCG needs m > 2 nev >= 2")
    b = np.asarray(b, dtype=np.complex128).reshape(-1)
    n = b.shape[0]
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128).reshape(-1)
    bnorm = np.linalg.norm(b)
    info = {"alpha": [], "beta": [], "rho": [], "restart_iterations": [],
            "iterations": 0}
    if record:
        info["restarts"] = []
    if bnorm == 0.0:
        info.update(true_rel_res=0.0, converged=True)
        return np.zeros_like(b), np.zeros((n, 0), complex), np.zeros(0), info

    V = np.zeros((n, m), dtype=np.complex128)
    T = np.zeros((m, m), dtype=np.complex128)
    i = 0                       # columns currently in the window V
    r = b - apply_A(x)
    j = 0
    rho = None
    alpha_1 = alpha_2 = None    # alpha_{j-1}, alpha_{j-2}
    beta_1 = 0.0                # beta_{j-1}
    p = t = None

    while np.linalg.norm(r) / bnorm > tol and j < max_iter:
        j += 1
        rho_prev = rho
        z = r if apply_Pinv is None else apply_Pinv(r)     # z = P^{-1} r (z = r for P = I)
        rho = _real_positive(_dot(r, z), "r^H z")
        if j == 1:
            beta = 0.0
            p = z.copy()
        else:
            beta = rho / rho_prev
            p = z + beta * p
        if i == m:
            t_prev = t                                     # A p of the previous iteration
        t = apply_A(p)
        if j > 1:  # diagonal of the window column appended last iteration
            T[i - 1, i - 1] = 1.0 / alpha_1 + (beta_1 / alpha_2 if j > 2 else 0.0)
        if i == m:                                         # full window: restart
            QZ, Mvals, Q, Z, _, _ = restart_coefficients(T.copy(), nev)
            Tm = T.copy() if record else None
            V[:, : 2 * nev] = V[:, :m] @ QZ                # V <- V (QZ)
            V[:, 2 * nev:] = 0.0
            T[:, :] = 0.0
            T[: 2 * nev, : 2 * nev] = np.diag(Mvals)
            i = 2 * nev
            w = t - beta * t_prev                          # w = A z
            arrow = (w.conj() @ V[:, :i]) / np.sqrt(rho)   # z^H A V / sqrt(rho)
            T[i, :i] = arrow
            T[:i, i] = np.conj(arrow)
            info["restart_iterations"].append(j)
            if record:
                info["restarts"].append({"Tm": Tm, "QZ": QZ, "M": Mvals,
                                         "arrow": arrow, "Q": Q, "Z": Z, "j": j})
        elif i >= 1:                                       # off-diagonal of T
            T[i, i - 1] = T[i - 1, i] = -np.sqrt(beta) / alpha_1
        i += 1                                             # append z / sqrt(rho) to V
        V[:, i - 1] = z / np.sqrt(rho)
        pt = _real_positive(_dot(p, t), "p^H A p")
        if pt <= 0.0:
            raise FloatingPointError("p^H A p <= 0: A is not positive definite")
        alpha = rho / pt
        x = x + alpha * p
        r = r - alpha * t
        info["alpha"].append(alpha)
        info["beta"].append(beta)
        info["rho"].append(rho)
        alpha_2, alpha_1, beta_1 = alpha_1, alpha, beta

    # finalisation: last diagonal entry, then Rayleigh-Ritz on T_i
    if i >= 1:
        T[i - 1, i - 1] = 1.0 / alpha_1 + (beta_1 / alpha_2 if j > 1 else 0.0)
        theta, Yf = np.linalg.eigh(T[:i, :i])
        k = min(nev, i)
        ritz_vecs = V[:, :i] @ Yf[:, :k]
        ritz_vals = theta[:k]
    else:
        ritz_vecs = np.zeros((n, 0), dtype=np.complex128)
        ritz_vals = np.zeros(0)
    true_res = np.linalg.norm(b - apply_A(x)) / bnorm
    info.update(iterations=j, true_rel_res=float(true_res),
                converged=bool(true_res <= tol), window=i,
                rho_final=float(np.vdot(r, r).real))
    if record:
        info["T"] = T[:i, :i].copy()
        info["V"] = V[:, :i].copy()
    return x, ritz_vecs, ritz_vals, info
