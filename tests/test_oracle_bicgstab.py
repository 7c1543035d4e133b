"""Pins of the oracle's deflated BiCGSTAB on M (CPU only).

What fixes it independently of its own code:
* every iterate equals SciPy's BiCGSTAB (an independent implementation of the
  same published method) on a random complex nonsymmetric matrix;
* finite termination: with k distinct eigenvalues BiCGSTAB ends within k
  iterations (the residual is a product of polynomials that vanish on the
  spectrum), also for a non-normal similarity transform;
* a scalar matrix is solved by the half step of the first iteration;
* the Wilson solve equals the dense solve of M;
* the paper's premise that eigenvectors of A = M^H M are eigenvectors of
  gamma5 M, with eigenvalue +-sqrt(lambda), on the dense 4^4 operator;
* the deflated guess is the dense least-squares solution of M (U y) = b
  (minimal residual over span(U)) for an approximate U; with exact
  eigenvectors it equals the dense Galerkin projection of gamma5 M and the
  orthogonal projection of the exact solution;
* deflation with the lowest eigenvectors of A cuts BiCGSTAB's iterations on
  gamma5 M by more than half.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle.bicgstab import bicgstab, deflated_bicgstab, deflated_guess
from oracle.dirac import apply_gamma5


def _random_system(n, seed):
    rng = np.random.default_rng(seed)
    M = 3.0 * np.eye(n) + 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return M, b


def test_iterates_equal_scipy_bicgstab():
    M, b = _random_system(60, 1)
    ref = []
    sla.bicgstab(M, b, rtol=1e-30, atol=0.0, maxiter=8, callback=lambda x: ref.append(x.copy()))
    assert len(ref) == 8
    for k in range(1, 9):
        x, info = bicgstab(lambda v: M @ v, b, tol=1e-30, max_iter=k, max_restarts=0)
        assert info["iterations"] == k and info["status"] == "max_iter"
        assert np.linalg.norm(x - ref[k - 1]) <= 1e-10 * np.linalg.norm(ref[k - 1])
    # with a starting guess
    x0 = np.full(60, 0.1 - 0.2j)
    ref = []
    sla.bicgstab(M, b, x0=x0, rtol=1e-30, atol=0.0, maxiter=4,
                 callback=lambda x: ref.append(x.copy()))
    x, _ = bicgstab(lambda v: M @ v, b, x0=x0, tol=1e-30, max_iter=4, max_restarts=0)
    assert np.linalg.norm(x - ref[-1]) <= 1e-12 * np.linalg.norm(ref[-1])


@pytest.mark.parametrize("normal", [True, False])
def test_finite_termination_with_k_distinct_eigenvalues(normal):
    rng = np.random.default_rng(4)
    n, k = 48, 4
    eigs = np.array([1.0 + 0.5j, 2.0 - 0.3j, 3.5 + 0.1j, 5.0 + 1.0j])
    D = np.diag(np.repeat(eigs, n // k))
    if normal:
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        M = Q @ D @ Q.conj().T
    else:
        S = np.eye(n) + 0.2 * rng.standard_normal((n, n))
        M = S @ D @ np.linalg.inv(S)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, info = bicgstab(lambda v: M @ v, b, tol=1e-10, max_iter=50)
    assert info["status"] == "ok"
    assert info["iterations"] <= k
    assert np.linalg.norm(M @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_scalar_matrix_is_one_half_step():
    rng = np.random.default_rng(5)
    c = 2.5 - 1.25j
    b = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    x, info = bicgstab(lambda v: c * v, b, tol=1e-12)
    assert info["iterations"] == 1 and info["status"] == "ok"
    assert np.max(np.abs(x - b / c)) < 1e-14


def test_zero_rhs():
    x, info = bicgstab(lambda v: 2.0 * v, np.zeros(12, np.complex128))
    assert info["iterations"] == 0 and not np.any(x)


def test_wilson_solve_equals_dense(cfg0_op, cfg0_dense, cfg0_rhs):
    b = cfg0_rhs
    x, info = bicgstab(cfg0_op.M, b, tol=1e-11)
    assert info["status"] == "ok"
    assert info["true_rel_res"] <= 1e-11
    x_ref = np.linalg.solve(cfg0_dense["M"], b)
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)


def _q_matrix(op, dense_M):
    g5 = np.array([op.gamma5(e) for e in np.eye(op.n, dtype=np.complex128)]).T
    return g5 @ dense_M


def test_eigenvectors_of_A_are_eigenvectors_of_gamma5_M(cfg0_op, cfg0_dense):
    Q = _q_matrix(cfg0_op, cfg0_dense["M"])
    assert np.max(np.abs(Q - Q.conj().T)) < 1e-13          # gamma5 M is Hermitian
    lam, X = cfg0_dense["lam"], cfg0_dense["X"]
    for j in range(12):
        u = X[:, j]
        mu = np.vdot(u, Q @ u).real
        assert abs(mu * mu - lam[j]) < 1e-10 * lam[-1]
        assert np.linalg.norm(Q @ u - mu * u) < 1e-9


def test_guess_is_least_squares_and_galerkin_for_exact_eigenvectors(cfg0_op, cfg0_dense,
                                                                     cfg0_rhs):
    b = cfg0_rhs
    Md = cfg0_dense["M"]
    X = cfg0_dense["X"][:, :16]
    # approximate basis: least squares over span(U), from the dense matrix
    rng = np.random.default_rng(3)
    Un, _ = np.linalg.qr(X + 1e-2 * (rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape)))
    y, *_ = np.linalg.lstsq(Md @ Un, b, rcond=None)
    xg = deflated_guess(cfg0_op.M, cfg0_op.Mdag, Un, b)
    assert np.linalg.norm(xg - Un @ y) <= 1e-9 * np.linalg.norm(Un @ y)
    assert np.linalg.norm(b - cfg0_op.M(xg)) < np.linalg.norm(b)
    # from a starting point: least squares for the correction
    xt = 0.1 * b
    y, *_ = np.linalg.lstsq(Md @ Un, b - Md @ xt, rcond=None)
    x1 = deflated_guess(cfg0_op.M, cfg0_op.Mdag, Un, b, x_tilde=xt)
    assert np.linalg.norm(x1 - xt - Un @ y) <= 1e-9 * np.linalg.norm(Un @ y)
    # exact eigenvectors: the Galerkin projection of Q = gamma5 M on span(X) ...
    Q = _q_matrix(cfg0_op, Md)
    HQ = X.conj().T @ Q @ X
    x_gal = X @ np.linalg.solve(HQ, X.conj().T @ cfg0_op.gamma5(b))
    xg = deflated_guess(cfg0_op.M, cfg0_op.Mdag, X, b)
    assert np.linalg.norm(xg - x_gal) <= 1e-9 * np.linalg.norm(x_gal)
    # ... which is the orthogonal projection of the exact solution
    x_star = np.linalg.solve(Md, b)
    proj = X @ (X.conj().T @ x_star)
    assert np.linalg.norm(xg - proj) <= 1e-9 * np.linalg.norm(proj)
    # the boundary gamma5 agrees with the dense one
    assert np.allclose(cfg0_op.gamma5(b), apply_gamma5(b.reshape(4, 4, 4, 4, 4, 3)).reshape(-1))


def test_deflation_cuts_iterations_on_gamma5_M(cfg0_op, cfg0_dense, cfg0_rhs):
    """Deflating the lowest eigenvectors of Q = gamma5 M (those of A) takes the
    small-magnitude part of Q's indefinite spectrum out of the initial residual."""
    b = cfg0_rhs
    U = cfg0_dense["X"][:, :24]
    _, plain = deflated_bicgstab(cfg0_op.M, cfg0_op.Mdag, cfg0_op.gamma5, None, b, tol=1e-10)
    x, defl = deflated_bicgstab(cfg0_op.M, cfg0_op.Mdag, cfg0_op.gamma5, U, b, tol=1e-10)
    assert plain["status"] == "ok" and defl["status"] == "ok"
    assert plain["guess_rel_res"] == 1.0 and defl["guess_rel_res"] < 1.0
    assert 2 * defl["iterations"] < plain["iterations"]
    x_ref = np.linalg.solve(cfg0_dense["M"], b)
    assert np.linalg.norm(x - x_ref) <= 1e-8 * np.linalg.norm(x_ref)
    # the iteration on gamma5 M is BiCGSTAB on the matrix Q itself
    xq, q = bicgstab(lambda v: cfg0_op.gamma5(cfg0_op.M(v)), cfg0_op.gamma5(b), tol=1e-10)
    assert q["iterations"] == plain["iterations"] and np.array_equal(xq, np.asarray(
        deflated_bicgstab(cfg0_op.M, cfg0_op.Mdag, cfg0_op.gamma5, None, b, tol=1e-10)[0]))
