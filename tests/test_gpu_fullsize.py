"""GPU parity at the bench's full size (16^3 x 32, eps 0.5, seed 1, m_q -0.58)
in the launch configuration the bench times (autotuned stencil variant,
single-RHS FP64 contexts).

The oracle cannot run CG or eigCG to convergence at this size in seconds, so
the checks are element-wise where the oracle is cheap (one stencil
application) and otherwise properties that hold at any size, evaluated with
the oracle's operator: the FP64 true residual of every returned solution, the
orthonormality of the bank, H = U^H A U column by column, the Ritz residual
bounds, and the Galerkin condition U^H (b - A x0) = 0 of eq. (2.1) for the
deflated initial guess.
"""

import numpy as np
import pytest

from gpu_common import dev, host, make_ctx
from oracle.bicgstab import bicgstab
from oracle.dirac import WilsonOperator
from synthetic import gauge_field, gaussian_rhs

pytestmark = pytest.mark.gpu

DIMS = (16, 16, 16, 32)
MASS = -0.58


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0707_0131_amd import binding
    return binding


@pytest.fixture(scope="module")
def field():
    U = gauge_field(DIMS, 0.5, 1)
    return U, WilsonOperator(U, MASS)


def _true_rel_res(op, b, x):
    b = b.reshape(-1)
    return float(np.linalg.norm(b - op.A(x.reshape(-1))) / np.linalg.norm(b))


def test_fullsize_stencil_matches_oracle(B, field):
    U, op = field
    ctx, _ = make_ctx(U, MASS)
    try:
        psi = gaussian_rhs(DIMS, 4242)[None]
        out = dev(np.zeros_like(psi))
        for code, fn in [(B.EIGCG_OP_M, op.M), (B.EIGCG_OP_MDAG, op.Mdag), (B.EIGCG_OP_A, op.A)]:
            B.eigcg_apply(ctx, code, dev(psi), out)
            ref = fn(psi.reshape(-1))
            got = host(out).reshape(-1)
            assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)), code
    finally:
        B.eigcg_destroy(ctx)


def test_kernel_samples_count_the_launches_that_ran(B, field):
    """Every 4th CG iteration timed, segments of 64 iterations: the segment in
    which the column converges runs on with launches that exit at once, and
    the samples count exactly the timed iterations that ran (iterations 1, 5,
    9, ... of the solve, the context's first)."""
    U, op = field
    ctx, _ = make_ctx(U, MASS, max_iter=20000, check_every=64, sample_every=4)
    try:
        b = gaussian_rhs(DIMS, 4243)[None]
        x = dev(np.zeros_like(b))
        rc, st = B.eigcg_solve(ctx, dev(b), x, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK
        iters = st[0]["iters"]
        # timed launches after the stop: iterations iters + 1 .. the segment's end
        seg_end = -(-iters // 64) * 64
        assert len(range(((iters + 3) // 4) * 4 + 1, seg_end + 1, 4)) >= 2
        s = B.eigcg_kernel_samples(ctx, reset=True)["f64"]
        assert s["n"] == (iters + 3) // 4
        assert 0.0 < s["pass1_ms"] < 1.0 and 0.0 < s["pass2_ms"] < 1.0 and s["cols"] == 1.0
        assert B.eigcg_kernel_samples(ctx)["f64"]["n"] == 0
    finally:
        B.eigcg_destroy(ctx)


def test_fullsize_cg_and_eigcg_bank(B, field):
    """Plain CG, then two Incremental eigCG(10, 100) solves and a deflated
    solve, as in the bench's phases; every solution and the bank are checked
    with the oracle's A."""
    U, op = field
    ctx, _ = make_ctx(U, MASS, nev=10, m=100, max_bank=40, max_iter=20000, check_every=16)
    try:
        b0 = gaussian_rhs(DIMS, 1000)
        x = dev(np.zeros((1,) + b0.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b0[None]), x, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK
        assert _true_rel_res(op, b0, host(x)) <= 1.01e-10
        assert abs(_true_rel_res(op, b0, host(x)) - st[0]["true_rel_res"]) <= 1e-12

        for seed in (1001, 1002):
            b = gaussian_rhs(DIMS, seed)
            x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
            rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_EIGCG)
            assert rc == B.EIGCG_OK
            assert _true_rel_res(op, b, host(x)) <= 1.01e-10
        vals, res = B.eigcg_bank_info(ctx, residuals=True)
        l = len(vals)
        assert l >= 15
        Ut = dev(np.zeros((l,) + b0.shape, dtype=np.complex128))
        B.eigcg_bank_vectors(ctx, 0, l, Ut)
        Um = host(Ut).reshape(l, -1).T
        del Ut
        assert np.max(np.abs(Um.conj().T @ Um - np.eye(l))) < 1e-12
        H = B.eigcg_bank_matrix(ctx, l)
        for j in (0, l // 2, l - 1):  # H = U^H A U, column by column with the oracle's A
            col = Um.conj().T @ op.A(Um[:, j])
            assert np.max(np.abs(col - H[:, j])) <= 1e-12 * 64.0
        # Ritz pairs of the bank: residual of the lowest three with the oracle's A
        theta, Y = np.linalg.eigh(H)
        assert np.allclose(theta, vals, rtol=1e-10, atol=1e-14)
        for i in range(3):
            u = Um @ Y[:, i]
            r = np.linalg.norm(op.A(u) - theta[i] * u)
            assert theta[i] > 0
            assert abs(r - res[i]) <= 1e-8 + 1e-6 * r

        # deflated initial guess (eq. (2.1)): its residual is orthogonal to U
        b = gaussian_rhs(DIMS, 1003)
        x0 = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        B.eigcg_deflate_init(ctx, dev(b[None]), x0)
        r0 = b.reshape(-1) - op.A(host(x0).reshape(-1))
        assert np.max(np.abs(Um.conj().T @ r0)) <= 1e-12 * np.linalg.norm(b)
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_INITCG)
        assert rc == B.EIGCG_OK
        assert _true_rel_res(op, b, host(x)) <= 1.01e-10
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("precision", [1, 2])
def test_fullsize_batched_mixed_precision(B, field, precision):
    """The batching form at full size: 4 right-hand sides per launch, FP32
    inner iteration with FP64 reliable updates (precision 1) or 16-bit
    storage with rescaled inner solves and FP64 refinement (precision 2);
    every column's FP64 true residual (oracle's A) is below 1e-10."""
    U, op = field
    ctx, _ = make_ctx(U, MASS, precision=precision, max_batch=4, reliable_every=50,
                      max_iter=20000, max_bank=0)
    try:
        bs = np.stack([gaussian_rhs(DIMS, 1100 + i) for i in range(4)])
        x = dev(np.zeros_like(bs))
        rc, st = B.eigcg_solve(ctx, dev(bs), x, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK
        xs = host(x)
        for i in range(4):
            assert _true_rel_res(op, bs[i], xs[i]) <= 1.01e-10
    finally:
        B.eigcg_destroy(ctx)


def test_fullsize_schur_stencil_and_solve(B, field):
    """Odd-even preconditioning at full size (the bench's odd-even leg):
    Mhat, Mhat^H element-wise against the oracle, then M x = b through the
    even-site system (rhs, CG, reconstruction) checked with the oracle's full
    M and its Ahat."""
    from oracle.schur import SchurOperator
    from synthetic import gaussian_half_rhs
    U, op = field
    sop = SchurOperator(U, MASS)
    ctx, _ = make_ctx(U, MASS, max_iter=20000, check_every=32, schur=1)
    try:
        psi = gaussian_half_rhs(DIMS, 4343)[None]
        out = dev(np.zeros_like(psi))
        for code, fn in [(B.EIGCG_OP_M, sop.Mhat), (B.EIGCG_OP_MDAG, sop.Mhat_dag)]:
            B.eigcg_apply(ctx, code, dev(psi), out)
            ref = fn(psi.reshape(-1))
            got = host(out).reshape(-1)
            assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)), code
        b = gaussian_rhs(DIMS, 1200)[None]
        bd = dev(b)
        rhs = dev(np.zeros_like(psi))
        B.eigcg_schur_rhs(ctx, bd, rhs)
        ref = sop.rhs(b.reshape(-1))
        assert np.max(np.abs(host(rhs).reshape(-1) - ref)) <= 1e-13 * np.max(np.abs(ref))
        xe = dev(np.zeros_like(psi))
        rc, st = B.eigcg_solve(ctx, rhs, xe, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK
        xe_h = host(xe).reshape(-1)
        assert np.linalg.norm(ref - sop.A(xe_h)) <= 1.01e-10 * np.linalg.norm(ref)
        xf = dev(np.zeros_like(b))
        B.eigcg_schur_reconstruct(ctx, bd, xe, xf)
        xf_h = host(xf).reshape(-1)
        # the odd half from the oracle's reconstruction, the full system with its M
        assert np.max(np.abs(xf_h - sop.reconstruct(b.reshape(-1), xe_h))) <= \
            1e-13 * np.max(np.abs(xf_h))
        assert np.linalg.norm(op.M(xf_h) - b.reshape(-1)) <= 1e-8 * np.linalg.norm(b)
    finally:
        B.eigcg_destroy(ctx)


def test_fullsize_bicgstab(B, field):
    """Deflated BiCGSTAB on M at full size: the first iterates against the
    oracle's BiCGSTAB; the deflated guess alone lies in span(U) and meets the
    least-squares normal equations (M U)^H (b - M x0) = 0 on sampled bank
    columns (oracle's M); the converged solution checked with the oracle's M."""
    U, op = field
    ctx, _ = make_ctx(U, MASS, nev=10, m=100, max_bank=40, max_iter=20000, check_every=16)
    try:
        b = gaussian_rhs(DIMS, 1010)
        z = np.zeros((1,) + b.shape, dtype=np.complex128)
        x = dev(z)
        rc, st = B.eigcg_solve_bicgstab(ctx, dev(b[None]), x, 1e-10, gamma5=False,
                                        deflate=False, max_iter=3)
        assert rc == B.EIGCG_ENOTCONV and st[0]["iters"] == 3
        xo, info = bicgstab(op.M, b.reshape(-1), tol=1e-10, max_iter=3)
        assert info["iterations"] == 3
        assert np.linalg.norm(host(x).reshape(-1) - xo) <= 1e-10 * np.linalg.norm(xo)

        for seed in (1001, 1002):  # a bank from two Incremental eigCG solves
            bs = gaussian_rhs(DIMS, seed)
            xs = dev(np.zeros((1,) + bs.shape, dtype=np.complex128))
            assert B.eigcg_solve(ctx, dev(bs[None]), xs, 1e-10, B.EIGCG_MODE_EIGCG)[0] == B.EIGCG_OK
        vals, _ = B.eigcg_bank_info(ctx)
        l = len(vals)
        Ut = dev(np.zeros((l,) + b.shape, dtype=np.complex128))
        B.eigcg_bank_vectors(ctx, 0, l, Ut)
        Um = host(Ut).reshape(l, -1).T
        del Ut
        x = dev(z)
        rc, sg = B.eigcg_solve_bicgstab(ctx, dev(b[None]), x, 1e-10, gamma5=False, deflate=True,
                                        guess_only=True)
        assert sg[0]["bank_used"] == l and sg[0]["iters"] == 0
        xg = host(x).reshape(-1)
        assert np.linalg.norm(xg - Um @ (Um.conj().T @ xg)) <= 1e-12 * np.linalg.norm(xg)
        r0 = b.reshape(-1) - op.M(xg)
        assert abs(np.linalg.norm(r0) / np.linalg.norm(b) - sg[0]["guess_rel_res"]) <= 1e-12
        for j in (0, l // 2, l - 1):
            mu = op.M(Um[:, j])
            assert abs(np.vdot(mu, r0)) <= 1e-8 * abs(np.vdot(mu, b.reshape(-1)))
        x = dev(z)
        rc, st = B.eigcg_solve_bicgstab(ctx, dev(b[None]), x, 1e-10, gamma5=False, deflate=True)
        assert rc == B.EIGCG_OK
        r = b.reshape(-1) - op.M(host(x).reshape(-1))
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("dims,seed,precision,tol", [
    ((32, 32, 32, 64), 4, 2, 4e-3),   # the largest configuration: 16-bit inner storage
    ((24, 24, 24, 48), 3, 1, 5e-6),   # the serving field above the MALL: FP32 inner
])
def test_fullsize_largest_lattice_operators(B, dims, seed, precision, tol):
    """Lattices of the larger configurations (eps 0.5): the FP64 stencil M and
    M^H of the autotuned launch element-wise against the oracle (<= 1e-13), and
    the inner operator that their deflated solves iterate with (16-bit or FP32
    storage, two-row SU(3) links, 12 columns per launch) within its storage
    rounding of the largest entry of the oracle's M."""
    U = gauge_field(dims, 0.5, seed)
    op = WilsonOperator(U, MASS)
    psi = gaussian_rhs(dims, 4242)[None]
    ref_m = op.M(psi.reshape(-1)).reshape(psi.shape)
    ctx, g = make_ctx(U, MASS)
    try:
        inp = dev(psi)
        out = dev(np.zeros_like(psi))
        B.eigcg_apply(ctx, B.EIGCG_OP_M, inp, out)
        assert np.max(np.abs(host(out) - ref_m)) <= 1e-13 * np.max(np.abs(ref_m))
        ref_d = op.Mdag(psi.reshape(-1)).reshape(psi.shape)
        B.eigcg_apply(ctx, B.EIGCG_OP_MDAG, inp, out)
        assert np.max(np.abs(host(out) - ref_d)) <= 1e-13 * np.max(np.abs(ref_d))
    finally:
        B.eigcg_destroy(ctx)
    del g
    ctx, g = make_ctx(U, MASS, precision=precision, compress_links=1, max_batch=12)
    try:
        B.eigcg_apply(ctx, B.EIGCG_OP_INNER + B.EIGCG_OP_M, inp, out)
        assert np.max(np.abs(host(out) - ref_m)) <= tol * np.max(np.abs(ref_m))
    finally:
        B.eigcg_destroy(ctx)
