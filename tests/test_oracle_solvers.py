"""Pins of the oracle's CG, eigCG, init-CG and Incremental eigCG (CPU only).

Each solver is checked against something other than itself: dense solves and
eigendecompositions of the 4^4 operator, exact-arithmetic properties (finite
termination on the free field, Galerkin orthogonality, T = V^H A V before loss
of orthogonality), and closed forms for the restart (the arrow row).
"""

import numpy as np
import pytest

from oracle.cg import cg
from oracle.dirac import WilsonOperator
from oracle.eigcg import eigcg, restart_coefficients
from oracle.incremental import bank_ritz, incremental_eigcg, orthonormalize_against
from oracle.initcg import galerkin_guess, init_cg
from synthetic import gaussian_rhs, unit_gauge_field


def test_cg_matches_dense_solve(cfg0_op, cfg0_dense, cfg0_rhs):
    b = cfg0_rhs
    x, info = cg(cfg0_op.A, b, tol=1e-10)
    lam = cfg0_dense["lam"]
    xs = np.linalg.solve(cfg0_dense["A"], b)
    kappa = lam[-1] / lam[0]
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    assert info["converged"] and info["true_rel_res"] <= 1e-10
    assert err <= kappa * 1e-10
    assert err < 1e-7


def test_cg_free_field_finite_termination():
    """Unit links: A has 15 distinct eigenvalues on 4^4, so exact CG terminates
    within 15 steps; in FP64 the residual collapses right after."""
    op = WilsonOperator(unit_gauge_field((4, 4, 4, 4)), -0.2)
    b = gaussian_rhs((4, 4, 4, 4), 1000).reshape(-1)
    x, info = cg(op.A, b, tol=1e-13)
    assert info["iterations"] <= 18
    rel = np.sqrt(np.array(info["rho"]) / info["rho"][0])
    # no gradual convergence before step 15, then the residual collapses
    assert rel[14] > 1e-2
    assert rel[15] < 1e-7
    assert info["true_rel_res"] <= 1e-13


def _explicit_T(info):
    a = np.array(info["alpha"])
    bt = np.array(info["beta"])
    k = len(a)
    T = np.zeros((k, k))
    for i in range(k):
        T[i, i] = 1 / a[i] + (bt[i] / a[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            T[i, i + 1] = T[i + 1, i] = -np.sqrt(bt[i + 1]) / a[i]
    return T


def test_eigcg_x_identical_to_cg(cfg0_op, cfg0_rhs):
    """eigCG leaves the CG iteration untouched (Section 3)."""
    x1, i1 = cg(cfg0_op.A, cfg0_rhs, tol=1e-8)
    x2, _, _, i2 = eigcg(cfg0_op.A, cfg0_rhs, 10, 40, tol=1e-8)
    assert i1["iterations"] == i2["iterations"]
    assert np.array_equal(x1, x2)
    assert np.array_equal(np.array(i1["alpha"]), np.array(i2["alpha"]))


def test_window_T_equals_VhAV_before_restart(cfg0_op, cfg0_dense, cfg0_rhs):
    """eq. (3.1) with the negative off-diagonal (as Figure 3.1 updates T): T = V^H A V for
    V = normalised residuals, while orthogonality holds."""
    A = cfg0_dense["A"]
    _, _, _, info = eigcg(cfg0_op.A, cfg0_rhs, 2, 60, tol=1e-14, max_iter=25, record=True)
    V = info["V"]
    T = info["T"]
    assert V.shape[1] == 25
    assert np.max(np.abs(V.conj().T @ V - np.eye(25))) < 1e-12
    assert np.max(np.abs(V.conj().T @ A @ V - T)) < 1e-11 * cfg0_dense["lam"][-1]
    # the same T follows from the CG scalars alone
    assert np.max(np.abs(_explicit_T(info) - T)) < 1e-13 * cfg0_dense["lam"][-1]
    # a positive off-diagonal (the printed eq. (3.1) sign) would not match
    Tpos = T.copy()
    idx = np.arange(24)
    Tpos[idx, idx + 1] *= -1
    Tpos[idx + 1, idx] *= -1
    assert np.max(np.abs(V.conj().T @ A @ V - Tpos)) > 1e-3


def test_lanczos_residual_identity(cfg0_op, cfg0_dense, cfg0_rhs):
    """||A V y - theta V y|| = |T_{i+1,i}| |y_i| (Section 3.1) before any restart."""
    x, Vr, th, info = eigcg(cfg0_op.A, cfg0_rhs, 3, 60, tol=1e-14, max_iter=30, record=True)
    T = info["T"]
    V = info["V"]
    theta, Y = np.linalg.eigh(T)
    j = info["iterations"]
    beta_next = info["rho_final"] / info["rho"][-1]
    t_next = np.sqrt(beta_next) / info["alpha"][-1]
    A = cfg0_dense["A"]
    for c in range(3):
        u = V @ Y[:, c]
        explicit = np.linalg.norm(A @ u - theta[c] * u)
        assert abs(explicit - t_next * abs(Y[-1, c])) < 1e-9 * cfg0_dense["lam"][-1]
    assert j == 30


def test_restart_invariants(cfg0_op, cfg0_dense, cfg0_rhs):
    """Restart (Figure 3.1, eq. (2.3)): span Q contains Y, so the lowest nev
    eigenvalues of H equal those of T_m; the arrow row equals its closed form
    (-sqrt(beta_j)/alpha_{j-1}) (QZ)_{m,:} in exact arithmetic; afterwards
    V^H V = I and V^H A V = T."""
    nev, m = 4, 12
    A = cfg0_dense["A"]
    _, _, _, info = eigcg(cfg0_op.A, cfg0_rhs, nev, m, tol=1e-14, max_iter=20, record=True)
    rs = info["restarts"]
    assert [r["j"] for r in rs] == [13, 17]  # m + 1 + k (m - 2 nev)
    r0 = rs[0]
    lam_T = np.linalg.eigvalsh(r0["Tm"])
    assert np.max(np.abs(r0["M"][:nev] - lam_T[:nev])) < 1e-13 * lam_T[-1]
    j = r0["j"]
    alpha_prev = info["alpha"][j - 2]
    beta_j = info["beta"][j - 1]
    closed = (-np.sqrt(beta_j) / alpha_prev) * r0["QZ"][m - 1, :]
    assert np.max(np.abs(r0["arrow"] - closed)) < 1e-10 * cfg0_dense["lam"][-1]
    V = info["V"]
    T = info["T"]
    assert np.max(np.abs(V.conj().T @ V - np.eye(V.shape[1]))) < 1e-12
    assert np.max(np.abs(V.conj().T @ A @ V - T)) < 1e-10 * cfg0_dense["lam"][-1]
    # restart coefficients on a random symmetric tridiagonal: Q orthonormal
    rng = np.random.default_rng(3)
    d = rng.uniform(1, 5, 9)
    e = rng.uniform(-1, 1, 8)
    Tt = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    QZ, Mv, Q, Z, Y, Yb = restart_coefficients(Tt.astype(complex), 3)
    assert np.allclose(Q.conj().T @ Q, np.eye(6), atol=1e-14)
    assert np.allclose(QZ.conj().T @ Tt @ QZ, np.diag(Mv), atol=1e-13)


def test_free_field_eigcg_finds_lowest_distinct_eigenvalues():
    """Free 4^4 field: the Krylov space of b sees one vector per distinct
    eigenvalue (closed form: lowest two are 0.04 and 1.64), so eigCG with a
    window larger than that count returns them exactly."""
    op = WilsonOperator(unit_gauge_field((4, 4, 4, 4)), -0.2)
    b = gaussian_rhs((4, 4, 4, 4), 1000).reshape(-1)
    _, V, th, info = eigcg(op.A, b, 2, 20, tol=1e-12)
    assert abs(th[0] - 0.04) < 1e-10
    assert abs(th[1] - 1.64) < 1e-9


def test_eigcg_ritz_pairs_vs_dense(cfg0_op, cfg0_dense, cfg0_rhs):
    """Ritz pairs of eigCG(4, 40) at tol 1e-8 lie within their residual norm
    of the dense spectrum (and within res^2/gap); the lowest four converge."""
    lam = cfg0_dense["lam"]
    A = cfg0_dense["A"]
    x, V, th, info = eigcg(cfg0_op.A, cfg0_rhs, 4, 40, tol=1e-8)
    for c in range(V.shape[1]):
        u = V[:, c] / np.linalg.norm(V[:, c])
        res = np.linalg.norm(A @ u - th[c] * u)
        k = np.argmin(np.abs(lam - th[c]))
        assert abs(th[c] - lam[k]) <= res + 1e-13
        gap = np.min(np.abs(np.delete(lam, k) - th[c]))
        assert abs(th[c] - lam[k]) <= res * res / gap + 1e-13
    assert np.max(np.abs(th - lam[:4])) < 1e-9  # absolute; ~1e-11 relative to the norm of A


def test_galerkin_condition(cfg0_op, cfg0_rhs):
    """eq. (2.1): U^H (b - A x0) = 0 for any full-rank U."""
    rng = np.random.default_rng(8)
    n = cfg0_op.n
    U, _ = np.linalg.qr(rng.standard_normal((n, 12)) + 1j * rng.standard_normal((n, 12)))
    AU = cfg0_op.A_block(U)
    H = U.conj().T @ AU
    x0 = galerkin_guess(cfg0_op.A, U, H, cfg0_rhs)
    r = cfg0_rhs - cfg0_op.A(x0)
    assert np.linalg.norm(U.conj().T @ r) < 1e-12 * np.linalg.norm(cfg0_rhs)
    xt = rng.standard_normal(n) + 0j
    x1 = galerkin_guess(cfg0_op.A, U, H, cfg0_rhs, x_tilde=xt)
    r1 = cfg0_rhs - cfg0_op.A(x1)
    assert np.linalg.norm(U.conj().T @ r1) < 1e-11 * np.linalg.norm(cfg0_rhs)


def test_initcg_with_exact_eigenvectors(cfg0_op, cfg0_dense):
    """b in span(U) with U exact eigenvectors: x0 = x*, zero CG iterations;
    for a general b deflation of the lowest 40 eigenvectors cuts iterations."""
    X = cfg0_dense["X"][:, :40]
    lam = cfg0_dense["lam"][:40]
    H = np.diag(lam).astype(complex)
    rng = np.random.default_rng(2)
    c = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    b = X @ c
    x, info = init_cg(cfg0_op.A, X, H, b, tol=1e-10)
    assert info["iterations"] == 0
    assert np.linalg.norm(x - X @ (c / lam)) < 1e-10 * np.linalg.norm(x)
    b2 = rng.standard_normal(cfg0_op.n) + 0j
    _, i_plain = cg(cfg0_op.A, b2, tol=1e-10)
    xd, i_defl = init_cg(cfg0_op.A, X, H, b2, tol=1e-10)
    assert i_defl["converged"]
    assert i_defl["iterations"] < 0.6 * i_plain["iterations"]


def test_initcg_restart(cfg0_op, cfg0_dense, cfg0_rhs):
    X = cfg0_dense["X"][:, :20]
    H = np.diag(cfg0_dense["lam"][:20]).astype(complex)
    x, info = init_cg(cfg0_op.A, X, H, cfg0_rhs, tol=1e-10, restart_tol=1e-6)
    assert info["restarted"] and info["converged"]
    assert 0 < info["first_leg_iterations"] < info["iterations"]
    xs = np.linalg.solve(cfg0_dense["A"], cfg0_rhs)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-6
    # forcing each leg to the oracle's own counts replays the same arithmetic
    k1 = info["first_leg_iterations"]
    k2 = info["iterations"] - k1
    xf, infof = init_cg(cfg0_op.A, X, H, cfg0_rhs, tol=1e-10, restart_tol=1e-6,
                        first_leg_iters=k1, second_leg_iters=k2)
    assert np.array_equal(xf, x) and infof["iterations"] == info["iterations"]
    # one iteration more in the second leg moves x by less than the residual allows
    x1, _ = init_cg(cfg0_op.A, X, H, cfg0_rhs, tol=1e-10, restart_tol=1e-6,
                    first_leg_iters=k1, second_leg_iters=k2 + 1)
    assert 0 < np.linalg.norm(x1 - x) / np.linalg.norm(x) < 1e-6


def test_incremental_bank_invariants(cfg0_op, cfg0_dense):
    """Section 4: the incrementally built H equals U^H A U and U is orthonormal;
    later right-hand sides need fewer iterations."""
    from synthetic import gaussian_rhs_block
    bs = gaussian_rhs_block((4, 4, 4, 4), [1000, 1001, 1002, 1003]).reshape(4, -1)
    xs, U, H, infos = incremental_eigcg(cfg0_op.A, list(bs), 4, 30, tol=1e-8)
    A = cfg0_dense["A"]
    assert U.shape[1] == 16
    assert np.max(np.abs(U.conj().T @ U - np.eye(16))) < 1e-12
    assert np.max(np.abs(U.conj().T @ A @ U - H)) < 1e-11 * cfg0_dense["lam"][-1]
    its = [inf["iterations"] for inf in infos]
    assert its[-1] < its[0]
    for b, x in zip(bs, xs):
        assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-8
    theta, res = bank_ritz(cfg0_op.A, U, H)
    lam = cfg0_dense["lam"]
    for t_, r_ in zip(theta, res):
        assert np.min(np.abs(lam - t_)) <= r_ + 1e-12


def test_orthonormalize_drops_dependent_columns():
    rng = np.random.default_rng(4)
    U, _ = np.linalg.qr(rng.standard_normal((50, 5)) + 0j)
    V = np.hstack([U[:, :2] @ rng.standard_normal((2, 2)), rng.standard_normal((50, 3)) + 0j])
    V[:, 4] = V[:, 3]
    out = orthonormalize_against(U, V)
    assert out.shape[1] == 2
    assert np.max(np.abs(U.conj().T @ out)) < 1e-14
    assert np.allclose(out.conj().T @ out, np.eye(2), atol=1e-14)


def test_zero_rhs_and_validation(cfg0_op):
    z = np.zeros(cfg0_op.n, dtype=complex)
    x, info = cg(cfg0_op.A, z)
    assert np.all(x == 0) and info["iterations"] == 0
    x, V, th, info = eigcg(cfg0_op.A, z, 2, 6)
    assert np.all(x == 0) and V.shape[1] == 0
    with pytest.raises(ValueError):
        eigcg(cfg0_op.A, z + 1, 3, 6)
