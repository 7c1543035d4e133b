"""GPU parity of the odd-even (Schur complement) preconditioned path against
the oracle's SchurOperator, through the C ABI.

Tolerances as for the unpreconditioned operator: stencil entries to 1e-13
relative (rounding order only); FP64 solutions to 1e-10 relative on the same
trajectory; Ritz values to 1e-8 on the same trajectory.  The right-hand side
of the even-site system is computed by each side from the same full-lattice
field (the library with eigcg_schur_rhs, the oracle with SchurOperator.rhs).
"""

import numpy as np
import pytest

from gpu_common import dev, host, make_ctx, rel
from oracle.cg import cg
from oracle.dirac import WilsonOperator
from oracle.eigcg import eigcg
from oracle.schur import SchurOperator
from synthetic import gauge_field, gaussian_half_rhs, gaussian_rhs, gaussian_rhs_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0707_0131_amd import binding
    return binding


CASES = [
    ("cfg0_4444", (4, 4, 4, 4), 0.3, 0, -0.2),
    ("ragged_4628", (4, 6, 2, 8), 0.5, 5, -0.1),      # half xy-plane of 12 sites
    ("L8", (8, 8, 8, 8), 0.5, 2, -0.3),
    ("slab_16_8_2_8", (16, 8, 2, 8), 0.5, 4, -0.15),  # whole 64-site tiles per half xy-plane
]


def _half_block(dims, seeds):
    return np.stack([gaussian_half_rhs(dims, s) for s in seeds])


@pytest.mark.parametrize("name,dims,eps,seed,mass", CASES)
@pytest.mark.parametrize("compress,variant", [(0, 3), (1, 1), (1, 3), (1, 4), (1, 5), (1, 6),
                                              (1, 7), (1, 8), (1, 9), (0, 9), (1, 10),
                                              (1, 14), (1, 15)])
def test_schur_apply_matches_oracle(B, name, dims, eps, seed, mass, compress, variant):
    U = gauge_field(dims, eps, seed)
    op = SchurOperator(U, mass)
    ctx, _ = make_ctx(U, mass, compress_links=compress, max_batch=2, stencil_variant=variant,
                      schur=1)
    try:
        psi = _half_block(dims, [11, 12])
        inp = dev(psi)
        out = dev(np.zeros_like(psi))
        for code, fn in [(B.EIGCG_OP_M, op.Mhat), (B.EIGCG_OP_MDAG, op.Mhat_dag),
                         (B.EIGCG_OP_A, op.A)]:
            B.eigcg_apply(ctx, code, inp, out)
            got = host(out)
            for c in range(2):
                ref = fn(psi[c].reshape(-1)).reshape(psi[c].shape)
                assert np.max(np.abs(got[c] - ref)) <= 1e-13 * np.max(np.abs(ref)), (name, code)
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("name,dims,eps,seed,mass", CASES[:2])
def test_schur_rhs_and_reconstruct(B, name, dims, eps, seed, mass):
    U = gauge_field(dims, eps, seed)
    op = SchurOperator(U, mass)
    ctx, _ = make_ctx(U, mass, max_batch=2, schur=1)
    try:
        b = gaussian_rhs_block(dims, [21, 22, 23])  # three columns: a batch of 2, then 1
        rhs = dev(np.zeros((3,) + (op.n // 12, 4, 3), dtype=np.complex128))
        B.eigcg_schur_rhs(ctx, dev(b), rhs)
        xe = _half_block(dims, [31, 32, 33])
        xf = dev(np.zeros_like(b))
        B.eigcg_schur_reconstruct(ctx, dev(b), dev(xe), xf)
        got_rhs, got_x = host(rhs), host(xf)
        for c in range(3):
            ref = op.rhs(b[c].reshape(-1))
            assert np.max(np.abs(got_rhs[c].reshape(-1) - ref)) <= 1e-13 * np.max(np.abs(ref))
            ref = op.reconstruct(b[c].reshape(-1), xe[c].reshape(-1))
            assert np.max(np.abs(got_x[c].reshape(-1) - ref)) <= 1e-13 * np.max(np.abs(ref))
    finally:
        B.eigcg_destroy(ctx)


def _solve_full(B, ctx, b_full, tol, mode):
    """M x = b through the even-site system: rhs, solve, reconstruct."""
    nh = b_full.shape[1] * b_full.shape[2] * b_full.shape[3] * b_full.shape[4] // 2
    bd = dev(b_full)
    rhs = dev(np.zeros((b_full.shape[0], nh, 4, 3), dtype=np.complex128))
    B.eigcg_schur_rhs(ctx, bd, rhs)
    xe = dev(np.zeros((b_full.shape[0], nh, 4, 3), dtype=np.complex128))
    rc, st = B.eigcg_solve(ctx, rhs, xe, tol, mode)
    xf = dev(np.zeros_like(b_full))
    B.eigcg_schur_reconstruct(ctx, bd, xe, xf)
    return rc, st, host(xe), host(xf)


@pytest.mark.parametrize("variant", [3, 6, 10])
def test_schur_cg_parity(B, cfg0_field, variant):
    """CG on the even-site system: the GPU stops within one iteration of the
    oracle's CG on Ahat (both test a recursive residual), x_e equals the
    oracle's iterate after the same number of iterations to 1e-10, and so
    does the reconstructed full solution."""
    U = cfg0_field
    op = SchurOperator(U, -0.2)
    full = WilsonOperator(U, -0.2)
    b = gaussian_rhs((4, 4, 4, 4), 1000)
    rhs = op.rhs(b.reshape(-1))
    xo_e, io = cg(op.A, rhs, tol=1e-10)
    k = io["iterations"]
    cands = {k: xo_e}
    for kk in (k - 1, k + 1):
        cands[kk] = cg(op.A, rhs, tol=0.0, max_iter=kk, true_residual_restarts=0)[0]
    ctx, _ = make_ctx(U, -0.2, max_iter=5000, stencil_variant=variant, schur=1)
    try:
        rc, st, xe, xf = _solve_full(B, ctx, b[None], 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK, B.eigcg_last_error(ctx)
        assert st[0]["iters"] in cands, (st[0]["iters"], k)
        assert st[0]["true_rel_res"] <= 1e-10
        ref_e = cands[st[0]["iters"]]
        assert rel(xe[0].reshape(-1), ref_e) <= 1e-10
        assert rel(xf[0].reshape(-1), op.reconstruct(b.reshape(-1), ref_e)) <= 1e-10
        # the reconstructed field solves the full system M x = b
        r = full.M(xf[0].reshape(-1)) - b.reshape(-1)
        assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b)
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("nev,m,iters", [(4, 12, 40), (10, 40, 70)])
def test_schur_eigcg_same_trajectory(B, cfg0_field, nev, m, iters):
    U = cfg0_field
    op = SchurOperator(U, -0.2)
    b = gaussian_rhs((4, 4, 4, 4), 1000)
    xo, Vo, tho, io = eigcg(op.A, op.rhs(b.reshape(-1)), nev, m, tol=1e-14, max_iter=iters)
    ctx, _ = make_ctx(U, -0.2, nev=nev, m=m, max_iter=iters, max_bank=64, schur=1)
    try:
        rc, st, xe, _ = _solve_full(B, ctx, b[None], 1e-14, B.EIGCG_MODE_EIGCG)
        assert rc == B.EIGCG_ENOTCONV
        assert st[0]["iters"] == iters
        assert st[0]["restarts"] == len(io["restart_iterations"])
        th = B.eigcg_last_ritz(ctx)
        assert len(th) == len(tho)
        assert np.max(np.abs(th - tho) / np.abs(tho)) <= 1e-8
        assert rel(xe[0].reshape(-1), xo) <= 1e-10
    finally:
        B.eigcg_destroy(ctx)


def test_schur_incremental_bank_and_initcg(B, cfg0_field):
    """Three Incremental eigCG(6, 30) solves, then init-CG: every solution's
    FP64 residual in the even-site system (oracle's Ahat), the bank's
    orthonormality and H = U^H Ahat U, and fewer iterations once deflated."""
    U = cfg0_field
    op = SchurOperator(U, -0.2)
    ctx, _ = make_ctx(U, -0.2, nev=6, m=30, max_bank=36, max_iter=5000, schur=1)
    try:
        iters = []
        for seed, mode in [(2000, B.EIGCG_MODE_EIGCG), (2001, B.EIGCG_MODE_EIGCG),
                           (2002, B.EIGCG_MODE_EIGCG), (2003, B.EIGCG_MODE_INITCG)]:
            b = gaussian_rhs((4, 4, 4, 4), seed)
            rc, st, xe, _ = _solve_full(B, ctx, b[None], 1e-10, mode)
            assert rc == B.EIGCG_OK, B.eigcg_last_error(ctx)
            rhs = op.rhs(b.reshape(-1))
            assert np.linalg.norm(rhs - op.A(xe[0].reshape(-1))) <= 1.01e-10 * np.linalg.norm(rhs)
            iters.append(st[0]["iters"])
        assert iters[-1] < iters[0]
        vals, _ = B.eigcg_bank_info(ctx)
        l = len(vals)
        assert 12 <= l <= 18
        Ut = dev(np.zeros((l, op.n // 12, 4, 3), dtype=np.complex128))
        B.eigcg_bank_vectors(ctx, 0, l, Ut)
        Um = host(Ut).reshape(l, -1).T
        assert np.max(np.abs(Um.conj().T @ Um - np.eye(l))) < 1e-12
        H = B.eigcg_bank_matrix(ctx, l)
        AU = np.stack([op.A(Um[:, j]) for j in range(l)], axis=1)
        assert np.max(np.abs(Um.conj().T @ AU - H)) <= 1e-12 * np.max(np.abs(H))
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("precision", [1, 2])
def test_schur_mixed_precision_batched(B, precision):
    """FP32 (reliable updates) and 16-bit (rescaled inner solves with FP64
    refinement) iterations on the even-site system, 3 right-hand sides in a
    batch of 4: FP64 residual below 1e-10 with the oracle's Ahat."""
    dims = (8, 8, 4, 8)
    U = gauge_field(dims, 0.5, 7)
    op = SchurOperator(U, -0.3)
    ctx, _ = make_ctx(U, -0.3, precision=precision, max_batch=4, reliable_every=50,
                      max_iter=20000, max_bank=0, schur=1)
    try:
        b = gaussian_rhs_block(dims, [41, 42, 43])
        rc, st, xe, _ = _solve_full(B, ctx, b, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK, B.eigcg_last_error(ctx)
        for c in range(3):
            rhs = op.rhs(b[c].reshape(-1))
            assert np.linalg.norm(rhs - op.A(xe[c].reshape(-1))) <= 1.01e-10 * np.linalg.norm(rhs)
    finally:
        B.eigcg_destroy(ctx)


def test_schur_batched_columns_match_single(B):
    """Columns of a 4-wide batch give the bits of single-column solves (same
    stencil variant; columns per workgroup do not change any column's
    arithmetic)."""
    dims = (8, 8, 4, 8)
    U = gauge_field(dims, 0.5, 7)
    b = gaussian_rhs_block(dims, [51, 52, 53, 54])
    out = []
    for K in (4, 1):
        ctx, _ = make_ctx(U, -0.3, max_batch=K, max_iter=5000, stencil_variant=6, schur=1)
        try:
            rc, st, xe, _ = _solve_full(B, ctx, b, 1e-10, B.EIGCG_MODE_CG)
            assert rc == B.EIGCG_OK
            out.append((xe, [s["iters"] for s in st]))
        finally:
            B.eigcg_destroy(ctx)
    assert out[0][1] == out[1][1]
    assert np.array_equal(out[0][0], out[1][0])


def test_schur_batched_initcg_guesses_match_single_solves(B, cfg0_field):
    """FP64 init-CG in a one-column odd-even context forms the deflated guesses
    of 18 right-hand sides in groups of 16 and 2 (the odd-even operator's
    intermediate then needs 16 odd-site fields, not one); each solve is
    bitwise the one of a single-right-hand-side call, with the restart."""
    U = cfg0_field
    op = SchurOperator(U, -0.2)
    ctx, _ = make_ctx(U, -0.2, nev=6, m=30, max_bank=12, max_iter=5000, schur=1,
                      restart_tol=1e-6)
    try:
        for seed in (2100, 2101):  # a bank of two Incremental eigCG solves
            b = gaussian_rhs((4, 4, 4, 4), seed)
            rc, _, _, _ = _solve_full(B, ctx, b[None], 1e-10, B.EIGCG_MODE_EIGCG)
            assert rc == B.EIGCG_OK
        assert len(B.eigcg_bank_info(ctx)[0]) >= 6
        nh = op.n // 12
        rhs = np.stack([gaussian_half_rhs((4, 4, 4, 4), 2200 + i) for i in range(18)])
        xall = dev(np.zeros_like(rhs))
        rc, st_all = B.eigcg_solve(ctx, dev(rhs), xall, 1e-10, B.EIGCG_MODE_INITCG)
        assert rc == B.EIGCG_OK
        got = host(xall)
        for i in range(18):
            x1 = dev(np.zeros((1, nh, 4, 3), dtype=np.complex128))
            rc, st1 = B.eigcg_solve(ctx, dev(rhs[i:i + 1].copy()), x1, 1e-10,
                                    B.EIGCG_MODE_INITCG)
            assert rc == B.EIGCG_OK
            assert st1[0]["iters"] == st_all[i]["iters"]
            assert np.array_equal(host(x1)[0], got[i]), i
            r = rhs[i].reshape(-1) - op.A(got[i].reshape(-1))
            assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(rhs[i])
    finally:
        B.eigcg_destroy(ctx)


def test_schur_errors(B, cfg0_field):
    U = gauge_field((4, 4, 3, 4), 0.3, 1)
    lt, lz, ly, lx = U.shape[:4]
    p = B.eigcg_default_params(dims=(lx, ly, lz, lt), mass=-0.2, schur=1)
    with pytest.raises(B.EigcgError):
        B.eigcg_create(p, dev(U))
    ctx, _ = make_ctx(cfg0_field, -0.2)
    try:
        b = dev(gaussian_rhs((4, 4, 4, 4), 1)[None])
        with pytest.raises(B.EigcgError):
            B.eigcg_schur_rhs(ctx, b, dev(np.zeros((1, 128, 4, 3), dtype=np.complex128)))
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("schur", [0, 1])
@pytest.mark.parametrize("precision,tol,compress", [(1, 5e-6, 1), (1, 5e-6, 0), (2, 4e-3, 1)])
def test_inner_precision_operator(B, schur, precision, tol, compress):
    """The inner-precision stencil kernels (FP32, 16-bit storage) applied
    alone (EIGCG_OP_INNER + op) against the FP64 oracle: entries within the
    storage precision's rounding (FP32: 5e-6, 16-bit: 4e-3 of the largest
    entry), full and odd-even geometry, two columns per launch."""
    dims = (8, 8, 4, 8)
    U = gauge_field(dims, 0.5, 7)
    op = SchurOperator(U, -0.3) if schur else WilsonOperator(U, -0.3)
    fns = [op.Mhat, op.Mhat_dag, op.A] if schur else [op.M, op.Mdag, op.A]
    ctx, _ = make_ctx(U, -0.3, precision=precision, max_batch=2, schur=schur,
                      compress_links=compress)
    try:
        psi = _half_block(dims, [61, 62]) if schur else gaussian_rhs_block(dims, [61, 62])
        inp = dev(psi)
        out = dev(np.zeros_like(psi))
        for code, fn in zip((B.EIGCG_OP_M, B.EIGCG_OP_MDAG, B.EIGCG_OP_A), fns):
            B.eigcg_apply(ctx, B.EIGCG_OP_INNER + code, inp, out)
            got = host(out)
            for c in range(2):
                ref = fn(psi[c].reshape(-1)).reshape(psi[c].shape)
                assert np.max(np.abs(got[c] - ref)) <= tol * np.max(np.abs(ref)), code
    finally:
        B.eigcg_destroy(ctx)


def test_schur_auto_mode_fp32(B):
    """EIGCG_MODE_AUTO on the even-site system with FP32 iterations (eigCG
    groups with FP64 reliable updates, then init-CG with FP64 refinement):
    a prefix of eigCG solves, every right-hand side to 1e-10 in FP64 with the
    oracle's Ahat."""
    dims = (8, 8, 4, 8)
    U = gauge_field(dims, 0.5, 7)
    op = SchurOperator(U, -0.3)
    ctx, _ = make_ctx(U, -0.3, precision=1, nev=4, m=24, max_bank=32, max_iter=20000,
                      reliable_every=50, schur=1)
    try:
        b = gaussian_rhs_block(dims, [71 + i for i in range(6)])
        rc, st, xe, _ = _solve_full(B, ctx, b, 1e-10, B.EIGCG_MODE_AUTO)
        assert rc == B.EIGCG_OK, B.eigcg_last_error(ctx)
        modes = [s["mode_used"] for s in st]
        keig = modes.count(B.EIGCG_MODE_EIGCG)
        assert keig >= 3 and modes == [B.EIGCG_MODE_EIGCG] * keig + [B.EIGCG_MODE_INITCG] * (6 - keig)
        assert len(B.eigcg_bank_info(ctx)[0]) > 0
        for c in range(6):
            rhs = op.rhs(b[c].reshape(-1))
            assert np.linalg.norm(rhs - op.A(xe[c].reshape(-1))) <= 1.01e-10 * np.linalg.norm(rhs)
    finally:
        B.eigcg_destroy(ctx)


def test_half_precision_needs_two_row_links(B):
    dims = (4, 4, 4, 4)
    U = gauge_field(dims, 0.3, 0)
    with pytest.raises(B.EigcgError) as e:
        make_ctx(U, -0.2, precision=2, compress_links=0)
    assert e.value.code == B.EIGCG_EINVAL
