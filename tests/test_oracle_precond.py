"""Pins of the preconditioned forms of the oracle (test infrastructure):
preconditioned CG and eigCG with a general SPD P (the derivation of
Section 3) and the spectral preconditioner built from a bank of approximate
eigenvectors (Section 2.1; Section 4's example), against dense linear
algebra on the 4^4 lattice."""

import numpy as np
import pytest
import scipy.linalg

from oracle.cg import cg
from oracle.eigcg import eigcg
from oracle.initcg import init_cg
from oracle.spectral import ritz_basis, spectral_preconditioner
from synthetic import gaussian_rhs


@pytest.fixture(scope="module")
def diag_P(cfg0_op):
    """A site- and component-dependent SPD diagonal P, entries in [0.5, 2]."""
    rng = np.random.default_rng(99)
    n = 12 * 256
    return 0.5 + 1.5 * rng.random(n)


def test_identity_preconditioner_reproduces_plain_cg_and_eigcg(cfg0_op, cfg0_rhs):
    x0, i0 = cg(cfg0_op.A, cfg0_rhs, tol=1e-10)
    x1, i1 = cg(cfg0_op.A, cfg0_rhs, tol=1e-10, apply_Pinv=lambda r: r)
    assert np.array_equal(x0, x1) and i0["iterations"] == i1["iterations"]
    e0 = eigcg(cfg0_op.A, cfg0_rhs, 4, 12, tol=1e-8, max_iter=60)
    e1 = eigcg(cfg0_op.A, cfg0_rhs, 4, 12, tol=1e-8, max_iter=60, apply_Pinv=lambda r: r)
    assert np.array_equal(e0[0], e1[0]) and np.array_equal(e0[2], e1[2])


def test_preconditioned_cg_solves_the_system(cfg0_op, cfg0_dense, cfg0_rhs, diag_P):
    x, info = cg(cfg0_op.A, cfg0_rhs, tol=1e-10, apply_Pinv=lambda r: r / diag_P)
    xs = np.linalg.solve(cfg0_dense["A"], cfg0_rhs)
    assert info["converged"]
    lam = cfg0_dense["lam"]
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= lam[-1] / lam[0] * 1e-10


def test_preconditioned_window_is_P_orthonormal_and_projects_A(cfg0_op, cfg0_dense, cfg0_rhs,
                                                              diag_P):
    """Before the first restart the window V = P^{-1} R (normalised) satisfies
    V^H P V = I and the tridiagonal T built from the CG scalars equals
    V^H A V (the Lanczos relation of P^{-1/2} A P^{-1/2}, Section 3): a
    dropped P^{-1} in the window or in rho fails both."""
    A = cfg0_dense["A"]
    _, V, _, info = eigcg(cfg0_op.A, cfg0_rhs, 4, 30, tol=1e-14, max_iter=25, record=True,
                          apply_Pinv=lambda r: r / diag_P)
    V = info["V"]
    T = info["T"]
    G = V.conj().T @ (diag_P[:, None] * V)
    assert np.max(np.abs(G - np.eye(V.shape[1]))) < 1e-9
    assert np.max(np.abs(V.conj().T @ A @ V - T)) < 1e-9 * cfg0_dense["lam"][-1]


def test_preconditioned_eigcg_ritz_pairs_of_the_pencil(cfg0_op, cfg0_dense, cfg0_rhs, diag_P):
    """Ritz pairs of preconditioned eigCG approximate the pencil
    A y = lambda P y: each Ritz value lies within the P^{-1}-norm of its
    residual of an eigenvalue of the pencil (dense generalised eigh)."""
    A = cfg0_dense["A"]
    x, Y, th, info = eigcg(cfg0_op.A, cfg0_rhs, 10, 40, tol=1e-8,
                           apply_Pinv=lambda r: r / diag_P)
    lam_p = scipy.linalg.eigh(A, np.diag(diag_P), eigvals_only=True)
    for k in range(len(th)):
        y = Y[:, k]
        ny = np.sqrt(np.real(np.vdot(y, diag_P * y)))
        y = y / ny
        res = A @ y - th[k] * (diag_P * y)
        bound = np.sqrt(np.real(np.vdot(res, res / diag_P)))
        assert np.min(np.abs(lam_p - th[k])) <= bound + 1e-12
    assert th[0] < 1.5 * lam_p[0]   # the lowest pencil eigenvalue is found
    xs = np.linalg.solve(A, cfg0_rhs)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-4


def test_spectral_preconditioner_maps_ritz_eigenvalues_to_sigma(cfg0_dense):
    """With exact eigenvectors, P^{-1} A has eigenvalue sigma on them and
    keeps the rest of the spectrum (dense check)."""
    A, lam, X = cfg0_dense["A"], cfg0_dense["lam"], cfg0_dense["X"]
    l, sigma = 20, lam[-1]
    Pinv = spectral_preconditioner(X[:, :l], lam[:l], sigma)
    n = A.shape[0]
    PA = np.stack([Pinv(A[:, c]) for c in range(n)], axis=1)
    ev = np.sort(np.linalg.eigvals(PA).real)
    expect = np.sort(np.concatenate([np.full(l, sigma), lam[l:]]))
    assert np.max(np.abs(ev - expect)) < 1e-9 * lam[-1]
    # Hermitian positive definite
    Pd = np.stack([Pinv(np.eye(n)[:, c]) for c in range(n)], axis=1)
    assert np.allclose(Pd, Pd.conj().T) and np.min(np.linalg.eigvalsh(Pd)) > 0


def test_spectral_pcg_converges_like_the_deflated_spectrum(cfg0_op, cfg0_dense, cfg0_rhs):
    A, lam, X = cfg0_dense["A"], cfg0_dense["lam"], cfg0_dense["X"]
    l = 24
    Pinv = spectral_preconditioner(X[:, :l], lam[:l], lam[-1])
    xp, ip = cg(cfg0_op.A, cfg0_rhs, tol=1e-10, apply_Pinv=Pinv)
    xc, ic = cg(cfg0_op.A, cfg0_rhs, tol=1e-10)
    xs = np.linalg.solve(A, cfg0_rhs)
    assert np.linalg.norm(xp - xs) / np.linalg.norm(xs) <= lam[-1] / lam[0] * 1e-10
    # CG iterations scale with sqrt(kappa): lambda_max / lambda_{l+1} against lambda_max / lambda_1
    assert ip["iterations"] < 0.7 * ic["iterations"]


def test_ritz_basis_of_a_bank(cfg0_dense):
    A = cfg0_dense["A"]
    rng = np.random.default_rng(3)
    U, _ = np.linalg.qr(rng.standard_normal((A.shape[0], 8)) + 1j * rng.standard_normal((A.shape[0], 8)))
    H = U.conj().T @ A @ U
    UR, th = ritz_basis(U, H)
    assert np.allclose(UR.conj().T @ UR, np.eye(8), atol=1e-12)
    assert np.allclose(UR.conj().T @ A @ UR, np.diag(th), atol=1e-10 * np.max(th))


def test_window_as_spectral_preconditioner_beats_init_cg(cfg0_op, cfg0_dense):
    """Section 4's example: the nev Ritz vectors from one eigCG solve, used as
    a spectral preconditioner for the next right-hand side, cut its
    iterations more than init-CG deflation with the same vectors."""
    A = cfg0_dense["A"]
    b1 = gaussian_rhs((4, 4, 4, 4), 1000).reshape(-1)
    b2 = gaussian_rhs((4, 4, 4, 4), 1001).reshape(-1)
    _, Y, th, _ = eigcg(cfg0_op.A, b1, 10, 40, tol=1e-8)
    U, _ = np.linalg.qr(Y)
    UR, th = ritz_basis(U, U.conj().T @ A @ U)
    _, i_plain = cg(cfg0_op.A, b2, tol=1e-8)
    _, i_init = init_cg(cfg0_op.A, UR, np.diag(th).astype(complex), b2, tol=1e-8)
    lmax = np.linalg.eigvalsh(A)[-1]
    _, i_spec = cg(cfg0_op.A, b2, tol=1e-8, apply_Pinv=spectral_preconditioner(UR, th, lmax))
    # on this field one solve gives Ritz vectors with residuals above their
    # values (loss of orthogonality past ~100 iterations): init-CG gains
    # nothing, while the spectral preconditioner still cuts the iterations
    assert i_spec["iterations"] < 0.7 * min(i_init["iterations"], i_plain["iterations"])
