"""GPU parity of the deflated BiCGSTAB path (eigcg_solve_bicgstab) against
the oracle's ``oracle.bicgstab``, through the C ABI.

Tolerances: a fixed number of iterations from the same start reproduces the
oracle's iterate to 1e-10 relative (FP64, only the order of rounding differs);
converged solutions agree with the dense solve to 1e-8; the deflated guess's
residual norm agrees to 1e-9 relative.

On M the iterates are stable (a 1e-15 relative change of b moves the 25th
iterate by 1e-11), so trajectories are compared over 25 iterations and the
iteration counts to within eight.  On the indefinite gamma5 M the method meets
near-breakdowns (r_0^H gamma5 M p close to zero) that amplify rounding: the same
1e-15 change of b moves the third iterate by 4e-6 and the sixth by O(1) in the
oracle itself, and its iteration count ranges over 966..1555.  There
trajectories are compared over the first two iterations, and converged runs by
their solution and their iteration count within 50 %.
"""

import numpy as np
import pytest

from gpu_common import dev, host, make_ctx, rel
from oracle.bicgstab import deflated_bicgstab, deflated_guess
from oracle.schur import SchurOperator
from synthetic import gaussian_half_rhs, gaussian_rhs

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 4)
MASS = -0.2


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0707_0131_amd import binding
    return binding


def _solve(B, ctx, b, x0, tol, gamma5, deflate, max_iter=0, guess_only=False):
    x = dev(x0.copy())
    rc, st = B.eigcg_solve_bicgstab(ctx, dev(b), x, tol, gamma5=gamma5, deflate=deflate,
                                    max_iter=max_iter, guess_only=guess_only)
    return rc, st, host(x)


def _oracle(op, b, x0, tol, gamma5, max_iter, U=None):
    if U is None and x0 is not None and not np.any(x0):
        x0 = None
    return deflated_bicgstab(op.M, op.Mdag, op.gamma5, U, b, x0=x0, tol=tol,
                             max_iter=max_iter, on_gamma5=gamma5)


@pytest.mark.parametrize("gamma5,k", [(False, 1), (False, 6), (False, 25), (True, 1),
                                     (True, 2)])
def test_iterates_match_oracle(B, cfg0_field, cfg0_op, gamma5, k):
    b = gaussian_rhs(DIMS, 3100)
    x0 = np.zeros((1,) + b.shape, np.complex128)
    ctx, _ = make_ctx(cfg0_field, MASS)
    try:
        rc, st, x = _solve(B, ctx, b[None], x0, 1e-14, gamma5, False, max_iter=k)
        assert rc == B.EIGCG_ENOTCONV and st[0]["iters"] == k
        xo, info = _oracle(cfg0_op, b.reshape(-1), None, 1e-14, gamma5, k)
        assert info["iterations"] == k
        assert rel(x[0].reshape(-1), xo) <= 1e-10
        assert abs(st[0]["true_rel_res"] - info["true_rel_res"]) <= 1e-9 * info["true_rel_res"]
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("gamma5", [False, True])
def test_converged_solution(B, cfg0_field, cfg0_op, cfg0_dense, gamma5):
    b = gaussian_rhs(DIMS, 3101)
    x_ref = np.linalg.solve(cfg0_dense["M"], b.reshape(-1))
    ctx, _ = make_ctx(cfg0_field, MASS, max_iter=4000)
    try:
        rc, st, x = _solve(B, ctx, b[None], np.zeros((1,) + b.shape, np.complex128), 1e-10,
                           gamma5, False)
        assert rc == B.EIGCG_OK and st[0]["true_rel_res"] <= 1e-10
        _, info = _oracle(cfg0_op, b.reshape(-1), None, 1e-10, gamma5, 4000)
        assert info["status"] == "ok"
        assert abs(st[0]["iters"] - info["iterations"]) <= _iters_band(info["iterations"], gamma5)
        assert rel(x[0].reshape(-1), x_ref) <= 1e-8
        assert st[0]["bank_used"] == 0 and st[0]["guess_rel_res"] == pytest.approx(1.0)
    finally:
        B.eigcg_destroy(ctx)


def _iters_band(n, gamma5):
    # spread of the oracle's own counts under 1e-15 relative changes of b (six
    # draws, 4^4 lattice): 186..194 on M, 966..1555 on gamma5 M
    return int(0.5 * n) + 5 if gamma5 else 8


def _bank(X, l):
    return dev(X[:, :l].T.reshape((l,) + DIMS[::-1] + (4, 3)).copy())


def test_deflated_guess_and_iterates_with_loaded_bank(B, cfg0_field, cfg0_op, cfg0_dense):
    """Bank = 24 lowest eigenvectors of A: the guess's residual and the
    iterates after it equal the oracle's; deflation cuts the iterations on
    gamma5 M by more than half; a start x0 != 0 is deflated from there."""
    X = cfg0_dense["X"]
    b = gaussian_rhs(DIMS, 3102)
    ctx, _ = make_ctx(cfg0_field, MASS, max_bank=40, max_iter=4000)
    try:
        assert B.eigcg_bank_load(ctx, _bank(X, 24)) == 24
        Ub = X[:, :24]  # the oracle deflates with the dense eigenvectors themselves
        x0 = np.zeros((1,) + b.shape, np.complex128)
        for gamma5, k in ((False, 6), (False, 25), (True, 2)):
            rc, st, x = _solve(B, ctx, b[None], x0, 1e-14, gamma5, True, max_iter=k)
            xo, info = _oracle(cfg0_op, b.reshape(-1), None, 1e-14, gamma5, k, U=Ub)
            assert st[0]["bank_used"] == 24
            assert abs(st[0]["guess_rel_res"] - info["guess_rel_res"]) <= \
                1e-9 * info["guess_rel_res"]
            assert rel(x[0].reshape(-1), xo) <= 1e-10
        # converged, against the undeflated solve
        rc, sd, x = _solve(B, ctx, b[None], x0, 1e-10, True, True)
        rc2, sp, _ = _solve(B, ctx, b[None], x0, 1e-10, True, False, max_iter=20000)
        assert rc == B.EIGCG_OK and rc2 == B.EIGCG_OK
        assert 2 * sd[0]["iters"] < sp[0]["iters"]
        _, infod = _oracle(cfg0_op, b.reshape(-1), None, 1e-10, True, 4000, U=Ub)
        assert abs(sd[0]["iters"] - infod["iterations"]) <= _iters_band(infod["iterations"], True)
        assert rel(x[0].reshape(-1), np.linalg.solve(cfg0_dense["M"], b.reshape(-1))) <= 1e-8
        # non-zero start: x0 + projected correction
        xs = 0.05 * b[None]
        rc, st, x = _solve(B, ctx, b[None], xs, 1e-14, False, True, max_iter=3)
        xo, info = _oracle(cfg0_op, b.reshape(-1), xs[0].reshape(-1), 1e-14, False, 3, U=Ub)
        assert abs(st[0]["guess_rel_res"] - info["guess_rel_res"]) <= 1e-9 * info["guess_rel_res"]
        assert rel(x[0].reshape(-1), xo) <= 1e-10
    finally:
        B.eigcg_destroy(ctx)


def test_guess_follows_bank_changes(B, cfg0_field, cfg0_op, cfg0_dense):
    """The guess follows the bank as it grows, is truncated or reset."""
    X = cfg0_dense["X"]
    b = gaussian_rhs(DIMS, 3103).reshape(-1)
    bb = b.reshape((1,) + DIMS[::-1] + (4, 3))
    x0 = np.zeros_like(bb)
    ctx, _ = make_ctx(cfg0_field, MASS, max_bank=40, max_iter=4000)

    def guess_res(l):
        # the bank spans the l lowest eigenvectors in every state below (loaded
        # 8, then 12 more; truncated to its 10 lowest Ritz vectors), and the
        # guess depends on the span only
        xg = deflated_guess(cfg0_op.M, cfg0_op.Mdag, X[:, :l], b)
        return np.linalg.norm(b - cfg0_op.M(xg)) / np.linalg.norm(b)

    try:
        B.eigcg_bank_load(ctx, _bank(X, 8))
        _, s8, _ = _solve(B, ctx, bb, x0, 1e-14, True, True, max_iter=1)
        assert s8[0]["bank_used"] == 8
        assert abs(s8[0]["guess_rel_res"] - guess_res(8)) <= 1e-9
        B.eigcg_bank_load(ctx, dev(X[:, 8:20].T.reshape((12,) + DIMS[::-1] + (4, 3)).copy()))
        _, s20, _ = _solve(B, ctx, bb, x0, 1e-14, True, True, max_iter=1)
        assert s20[0]["bank_used"] == 20
        assert abs(s20[0]["guess_rel_res"] - guess_res(20)) <= 1e-9
        assert s20[0]["guess_rel_res"] < s8[0]["guess_rel_res"]
        B.eigcg_bank_truncate(ctx, 10)
        _, s10, _ = _solve(B, ctx, bb, x0, 1e-14, True, True, max_iter=1)
        assert s10[0]["bank_used"] == 10
        assert abs(s10[0]["guess_rel_res"] - guess_res(10)) <= 1e-9
        B.eigcg_bank_reset(ctx)
        _, s0, _ = _solve(B, ctx, bb, x0, 1e-14, True, True, max_iter=1)
        assert s0[0]["bank_used"] == 0 and s0[0]["guess_rel_res"] == pytest.approx(1.0)
    finally:
        B.eigcg_destroy(ctx)


def test_columns_match_single_solves(B, cfg0_field, cfg0_dense):
    X = cfg0_dense["X"]
    bs = np.stack([gaussian_rhs(DIMS, s) for s in (3110, 3111, 3112)])
    ctx, _ = make_ctx(cfg0_field, MASS, max_bank=40, max_iter=4000)
    try:
        B.eigcg_bank_load(ctx, _bank(X, 16))
        rc, st, x = _solve(B, ctx, bs, np.zeros_like(bs), 1e-10, True, True)
        assert rc == B.EIGCG_OK and len(st) == 3
        for j in range(3):
            _, sj, xj = _solve(B, ctx, bs[j:j + 1], np.zeros_like(bs[j:j + 1]), 1e-10, True, True)
            assert sj[0]["iters"] == st[j]["iters"]
            assert np.array_equal(xj[0], x[j])
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("gamma5,k", [(False, 8), (True, 2)])
def test_odd_even_context(B, cfg0_field, gamma5, k):
    """In an odd-even context the operator is Mhat on even-site fields."""
    op = SchurOperator(cfg0_field, MASS)
    b = gaussian_half_rhs(DIMS, 3120)
    ctx, _ = make_ctx(cfg0_field, MASS, schur=1, max_iter=4000)
    try:
        x0 = np.zeros((1,) + b.shape, np.complex128)
        rc, st, x = _solve(B, ctx, b[None], x0, 1e-14, gamma5, False, max_iter=k)
        xo, info = deflated_bicgstab(op.Mhat, op.Mhat_dag, op.gamma5, None, b.reshape(-1),
                                     tol=1e-14, max_iter=k, on_gamma5=gamma5)
        assert rel(x[0].reshape(-1), xo) <= 1e-10
        rc, st, x = _solve(B, ctx, b[None], x0, 1e-10, gamma5, False, max_iter=20000)
        assert rc == B.EIGCG_OK
        r = b.reshape(-1) - op.Mhat(x[0].reshape(-1))
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
    finally:
        B.eigcg_destroy(ctx)


def _normal_equations_ratio(op, Um, b, x0):
    """||(M U)^H (b - M x0)|| / ||(M U)^H b||: zero for the least-squares guess."""
    MU = np.stack([op.M(Um[:, j]) for j in range(Um.shape[1])], axis=1)
    r0 = b - op.M(x0)
    return np.linalg.norm(MU.conj().T @ r0) / np.linalg.norm(MU.conj().T @ b)


def test_mixed_context_fp32_bank(B, cfg0_field, cfg0_op):
    """A bank grown by Incremental eigCG in an FP32 context (FP32 storage).
    The guess alone (FP32 products, FP64 correction) lies in span(U) and meets
    the least-squares normal equations (M U)^H (b - M x0) = 0 to FP32 accuracy,
    checked with the oracle's M on the library's bank; the FP64 BiCGSTAB after
    it converges."""
    ctx, _ = make_ctx(cfg0_field, MASS, precision=1, nev=8, m=40, max_bank=48, max_iter=20000)
    try:
        for s in (3130, 3131, 3132, 3133):
            b = gaussian_rhs(DIMS, s)
            x = dev(np.zeros((1,) + b.shape, np.complex128))
            rc, _ = B.eigcg_solve(ctx, dev(b[None]), x, 1e-8, B.EIGCG_MODE_EIGCG)
            assert rc == B.EIGCG_OK
        vals, _ = B.eigcg_bank_info(ctx)
        l = len(vals)
        assert l >= 16
        Ut = dev(np.zeros((l,) + DIMS[::-1] + (4, 3), np.complex128))
        B.eigcg_bank_vectors(ctx, 0, l, Ut)
        Um = host(Ut).reshape(l, -1).T
        b = gaussian_rhs(DIMS, 3140)
        x0 = np.zeros((1,) + b.shape, np.complex128)
        rc, sg, xg = _solve(B, ctx, b[None], x0, 1e-10, False, True, guess_only=True)
        assert rc == B.EIGCG_ENOTCONV and sg[0]["iters"] == 0 and sg[0]["bank_used"] == l
        xg = xg[0].reshape(-1)
        assert np.linalg.norm(xg - Um @ (Um.conj().T @ xg)) <= 1e-5 * np.linalg.norm(xg)
        assert _normal_equations_ratio(cfg0_op, Um, b.reshape(-1), xg) <= 1e-3
        g = np.linalg.norm(b.reshape(-1) - cfg0_op.M(xg)) / np.linalg.norm(b)
        assert abs(sg[0]["guess_rel_res"] - g) <= 1e-12 and g < 1.0
        for gamma5 in (True, False):
            rc, sd, x = _solve(B, ctx, b[None], x0, 1e-10, gamma5, True)
            assert rc == B.EIGCG_OK, sd
            assert sd[0]["guess_rel_res"] == pytest.approx(g, rel=1e-9)
            r = b.reshape(-1) - cfg0_op.M(x[0].reshape(-1))
            assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
    finally:
        B.eigcg_destroy(ctx)


def test_errors_and_zero_rhs(B, cfg0_field):
    ctx, _ = make_ctx(cfg0_field, MASS)
    try:
        b = gaussian_rhs(DIMS, 3150)[None]
        x = dev(np.zeros_like(b))
        assert B.LIB.eigcg_solve_bicgstab(ctx, 1, None, None, 1e-10, 0, 0, None) == B.EIGCG_EINVAL
        assert B.LIB.eigcg_solve_bicgstab(ctx, 1, B._ptr(dev(b)), B._ptr(x), 1e-10, 8, 0,
                                          None) == B.EIGCG_EINVAL
        assert B.LIB.eigcg_solve_bicgstab(ctx, 1, B._ptr(dev(b)), B._ptr(x), 0.0, 0, 0,
                                          None) == B.EIGCG_EINVAL
        bn = b.copy()
        bn[0, 0, 0, 0, 0, 0, 0] = np.nan
        with pytest.raises(B.EigcgError):
            B.eigcg_solve_bicgstab(ctx, dev(bn), x, 1e-10)
        xz = dev(np.ones_like(b))
        rc, st = B.eigcg_solve_bicgstab(ctx, dev(np.zeros_like(b)), xz, 1e-10)
        assert rc == B.EIGCG_OK and st[0]["iters"] == 0 and not np.any(host(xz))
        # a deflation request with an empty bank is the plain solve
        x1 = dev(np.zeros_like(b))
        x2 = dev(np.zeros_like(b))
        _, s1 = B.eigcg_solve_bicgstab(ctx, dev(b), x1, 1e-10, deflate=True)
        _, s2 = B.eigcg_solve_bicgstab(ctx, dev(b), x2, 1e-10, deflate=False)
        assert s1[0]["bank_used"] == 0 and s1[0]["iters"] == s2[0]["iters"]
        assert np.array_equal(host(x1), host(x2))
    finally:
        B.eigcg_destroy(ctx)
