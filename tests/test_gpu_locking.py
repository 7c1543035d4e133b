"""GPU parity of bank locking (Section 4's discussion of limiting the cost of
growing U) against the oracle, through the C ABI.

A bank grown by the oracle's Incremental eigCG on the 4^4 test lattice is
loaded into the context and into the oracle; both lock their accurate Ritz
vectors, then take eight more vectors.  Ritz vectors are
defined up to a phase per column, so U and H are compared after aligning those
phases; the deflated guess of eq. (2.1) does not depend on them and is
compared directly.  The bank is extended by perturbed eigenvectors of A
nearly orthogonal to it (see the fixture).
"""

import numpy as np
import pytest

from gpu_common import dev, host, make_ctx, rel
from oracle.dirac import WilsonOperator
from oracle.incremental import incremental_eigcg, orthonormalize_against
from oracle.initcg import galerkin_guess
from oracle.locking import extend_bank_locked, lock_bank
from synthetic import gaussian_rhs

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 4)
SHAPE = (4, 4, 4, 4, 4, 3)
MASS = -0.2
TOL_LOCK = 1e-6


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0707_0131_amd import binding
    return binding


@pytest.fixture(scope="module")
def grown(cfg0_field, cfg0_dense):
    """The bank of three Incremental eigCG(8, 24) solves, and as the vectors
    that extend it eigenvectors 200..207 of A with 1e-3 noise: nearly
    orthogonal to the bank, so that orthonormalising them against it does not
    amplify rounding (eigCG's own Ritz vectors overlap the bank closely and
    turn rounding-level differences of U into 1e-9 differences of H)."""
    op = WilsonOperator(cfg0_field, MASS)
    rhs = [gaussian_rhs(DIMS, 2000 + i).reshape(-1) for i in range(3)]
    _, U, H, _ = incremental_eigcg(op.A, rhs, 8, 24, tol=1e-7)
    rng = np.random.default_rng(31)
    Z = cfg0_dense["X"][:, 200:208]
    V = Z + 1e-3 * (rng.standard_normal(Z.shape) + 1j * rng.standard_normal(Z.shape))
    return op, U, H, V


def _vecs(X):
    return dev(np.ascontiguousarray(X.T).reshape((X.shape[1],) + SHAPE))


def _bank_vectors(B, ctx, l):
    import torch
    out = torch.empty((l,) + SHAPE, dtype=torch.complex128, device="cuda:0")
    B.eigcg_bank_vectors(ctx, 0, l, out)
    return host(out).reshape(l, -1).T


def test_lock_then_extend_matches_oracle(B, cfg0_field, grown):
    op, U, H, V = grown
    l = U.shape[1]
    Ul, Hl, nl, theta, res = lock_bank(op.A, U, H, 0, TOL_LOCK)
    # the choice is decided away from the tolerance
    assert 0 < nl < l and np.min(np.abs(res - TOL_LOCK)) > 1e-2 * TOL_LOCK
    Vbar = orthonormalize_against(Ul, V)
    Ue, He = extend_bank_locked(op.A, Ul, Hl, Vbar, nl)
    k = Ue.shape[1] - l
    ctx, _ = make_ctx(cfg0_field, MASS, nev=8, m=24, max_bank=40, max_batch=4)
    try:
        assert B.eigcg_bank_load(ctx, _vecs(U)) == l
        assert np.max(np.abs(B.eigcg_bank_matrix(ctx, l) - H)) <= 1e-12 * np.max(theta)
        assert B.eigcg_bank_lock(ctx, TOL_LOCK) == nl
        assert B.eigcg_bank_locked(ctx) == nl
        Hg = B.eigcg_bank_matrix(ctx, l)
        np.testing.assert_allclose(np.real(np.diag(Hg)), theta, rtol=1e-10)
        assert np.all(Hg - np.diag(np.diag(Hg)) == 0.0)
        Ug = _bank_vectors(B, ctx, l)
        ph = np.einsum("ij,ij->j", Ul.conj(), Ug)  # u_gpu = ph * u_oracle
        assert np.max(np.abs(np.abs(ph) - 1.0)) < 1e-9
        ph = ph / np.abs(ph)
        assert np.max(np.abs(Ug - Ul * ph)) < 1e-9
        # extension with the locked rows left at zero
        assert B.eigcg_bank_load(ctx, _vecs(V)) == k
        He_g = B.eigcg_bank_matrix(ctx, l + k)
        P = np.concatenate([ph, np.ones(k)])
        aligned = P.conj()[:, None] * He * P[None, :]
        assert np.max(np.abs(He_g - aligned)) <= 1e-11 * np.max(theta)
        assert np.all(He_g[:nl, l:] == 0.0) and np.all(He_g[l:, :nl] == 0.0)
        # the deflated guess, eq. (2.1), is independent of the phases
        b = gaussian_rhs(DIMS, 3100)
        x0 = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        B.eigcg_deflate_init(ctx, dev(b[None]), x0)
        ref = galerkin_guess(op.A, Ue, He, b.reshape(-1))
        assert rel(host(x0)[0].reshape(-1), ref) <= 1e-10
        # a second lock call locks among the unlocked columns only
        n2 = B.eigcg_bank_lock(ctx, TOL_LOCK)
        U2, H2, nl2, _, _ = lock_bank(op.A, Ue, He, nl, TOL_LOCK)
        assert n2 == nl2 >= nl
        B.eigcg_bank_truncate(ctx, l + k)  # no-op size: keeps every column and the locks
        assert B.eigcg_bank_locked(ctx) == n2
        B.eigcg_bank_truncate(ctx, l)
        assert B.eigcg_bank_locked(ctx) == 0
    finally:
        B.eigcg_destroy(ctx)


def test_lock_tolerance_zero_locks_nothing(B, cfg0_field, grown):
    """tol = 0 rotates the bank to its Ritz vectors and locks nothing; later
    updates are the plain Section 4 update (H = U^H A U)."""
    op, U, H, V = grown
    l = U.shape[1]
    ctx, _ = make_ctx(cfg0_field, MASS, nev=8, m=24, max_bank=40, max_batch=4)
    try:
        B.eigcg_bank_load(ctx, _vecs(U))
        assert B.eigcg_bank_lock(ctx, 0.0) == 0
        k = B.eigcg_bank_load(ctx, _vecs(V))
        Ug = _bank_vectors(B, ctx, l + k)
        AU = np.stack([op.A(Ug[:, j]) for j in range(l + k)], axis=1)
        Hx = Ug.conj().T @ AU
        assert np.max(np.abs(B.eigcg_bank_matrix(ctx, l + k) - Hx)) <= 1e-11 * np.max(np.abs(Hx))
        with pytest.raises(B.EigcgError):
            B.eigcg_bank_lock(ctx, -1.0)
    finally:
        B.eigcg_destroy(ctx)
