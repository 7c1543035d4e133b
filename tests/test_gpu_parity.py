"""GPU parity of the HIP library against the FP64 oracle (through the C ABI).

Tolerances: stencil entries to 1e-13 relative (rounding-order differences
only); FP64 solutions to 1e-10 relative on the same trajectory; Ritz values
to 1e-8 on the same trajectory before loss of orthogonality; afterwards Ritz
pairs are checked against the dense spectrum with their residual bound.
"""

import numpy as np
import pytest

from gpu_common import dev, host, make_ctx, rel
from oracle.cg import cg
from oracle.dirac import WilsonOperator
from oracle.eigcg import eigcg
from oracle.incremental import bank_ritz
from oracle.initcg import galerkin_guess, init_cg
from oracle.restart_model import choose_restart
from oracle.spectral import ritz_basis, spectral_preconditioner
from synthetic import gauge_field, gaussian_rhs, gaussian_rhs_block, unit_gauge_field

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
    ("ragged_4628", (4, 6, 2, 8), 0.5, 5, -0.1),
    ("L8", (8, 8, 8, 8), 0.5, 2, -0.3),
    ("odd_3535", (3, 5, 3, 5), 0.4, 9, 0.2),
    ("slab_8_8_3_16", (8, 8, 3, 16), 0.5, 4, -0.15),  # whole 64-site tiles per xy-plane
]


@pytest.mark.parametrize("name,dims,eps,seed,mass", CASES)
@pytest.mark.parametrize("compress,variant", [(0, 1), (1, 1), (1, 2), (1, 3), (0, 3), (1, 4),
                                              (1, 5), (1, 6), (1, 7), (1, 8), (1, 9), (0, 9),
                                              (1, 10), (1, 11), (0, 11), (1, 12), (1, 13),
                                              (1, 14), (0, 14), (1, 15)])
def test_apply_matches_oracle(B, name, dims, eps, seed, mass, compress, variant):
    U = gauge_field(dims, eps, seed)
    op = WilsonOperator(U, mass)
    ctx, _ = make_ctx(U, mass, compress_links=compress, max_batch=2, stencil_variant=variant)
    try:
        psi = gaussian_rhs_block(dims, [11, 12])
        inp = dev(psi)
        out = dev(np.zeros_like(psi))
        for code, fn in [(B.EIGCG_OP_M, op.M), (B.EIGCG_OP_MDAG, op.Mdag), (B.EIGCG_OP_A, op.A)]:
            B.eigcg_apply(ctx, code, inp, out)
            got = host(out)
            for c in range(2):
                ref = fn(psi[c].reshape(-1)).reshape(psi[c].shape)
                assert np.max(np.abs(got[c] - ref)) <= 1e-13 * np.max(np.abs(ref)), (name, code)
    finally:
        B.eigcg_destroy(ctx)


def test_apply_free_field_plane_wave_8888(B):
    """Unit links, single momentum: the GPU stencil reproduces the closed form
    (4 + m - sum cos p) + i sum gamma sin p at every site."""
    from oracle import dirac
    dims = (8, 8, 8, 8)
    U = unit_gauge_field(dims)
    mass = -0.25
    k = (1, 2, 3, 5)
    p = [2 * np.pi * k[i] / dims[i] for i in range(4)]
    t, z, y, x = np.meshgrid(*(np.arange(8),) * 4, indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    chi = np.arange(12).reshape(4, 3) + 1j
    psi = (phase[..., None, None] * chi)[None]
    sym = (4 + mass - sum(np.cos(p))) * np.eye(4) + 1j * sum(
        np.sin(p[m]) * dirac.GAMMA[m] for m in range(4))
    ctx, _ = make_ctx(U, mass)
    try:
        out = dev(np.zeros_like(psi))
        B.eigcg_apply(ctx, B.EIGCG_OP_M, dev(psi), out)
        expect = phase[..., None, None] * (sym @ chi)
        assert np.max(np.abs(host(out)[0] - expect)) < 1e-12
    finally:
        B.eigcg_destroy(ctx)


@pytest.fixture(scope="module")
def cfg0():
    U = gauge_field((4, 4, 4, 4), 0.3, 0)
    op = WilsonOperator(U, -0.2)
    b = gaussian_rhs((4, 4, 4, 4), 1000)
    return U, op, b


def _cg_candidates(apply_A, b, tol, x0=None):
    """The oracle's CG solution and its iterates one step either side of its
    own stop (both sides stop on a recursively updated residual, whose
    rounding differs), keyed by iteration count."""
    xo, io = cg(apply_A, b, x0=x0, tol=tol)
    k = io["iterations"]
    cands = {k: xo}
    for kk in (k - 1, k + 1):
        if kk >= 0:
            cands[kk] = cg(apply_A, b, x0=x0, tol=0.0, max_iter=kk, true_residual_restarts=0)[0]
    return cands, io


@pytest.mark.parametrize("variant", list(range(1, 16)))
def test_cg_parity_cfg0(B, cfg0, variant):
    """Single-column FP64 CG with every stencil variant: x matches the
    oracle's iterate after the same number of iterations to 1e-10."""
    U, op, b = cfg0
    cands, io = _cg_candidates(op.A, b.reshape(-1), 1e-10)
    ctx, _ = make_ctx(U, -0.2, max_iter=5000, stencil_variant=variant)
    try:
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK, B.eigcg_last_error(ctx)
        assert st[0]["iters"] in cands, (st[0]["iters"], io["iterations"])
        assert st[0]["true_rel_res"] <= 1e-10
        assert rel(host(x)[0].reshape(-1), cands[st[0]["iters"]]) <= 1e-10
    finally:
        B.eigcg_destroy(ctx)


ZMARCH_LATTICES = [((8, 8, 3, 16), 0.5, 4, -0.15), ((8, 8, 8, 8), 0.5, 2, -0.3)]


@pytest.mark.parametrize("dims,eps,seed,mass", ZMARCH_LATTICES)
@pytest.mark.parametrize("compress", [0, 1])
def test_zmarch_equals_variant1_bitwise(B, dims, eps, seed, mass, compress):
    """The z-march kernels (variants 11-13: z-hops carried in registers, the
    z-range in 1, 2 or 4 chunks; Lz = 3 gives chunks of one plane) form every
    site's output with variant 1's operations in variant 1's order: M and
    M^H agree bit for bit."""
    U = gauge_field(dims, eps, seed)
    psi = gaussian_rhs_block(dims, [31, 32])
    outs = {}
    for v in (1, 11, 12, 13):
        ctx, _ = make_ctx(U, mass, compress_links=compress, max_batch=2, stencil_variant=v)
        try:
            assert B.eigcg_layout_info(ctx)["variant64"] == v
            res = []
            for code in (B.EIGCG_OP_M, B.EIGCG_OP_MDAG, B.EIGCG_OP_A):
                out = dev(np.zeros_like(psi))
                B.eigcg_apply(ctx, code, dev(psi), out)
                res.append(host(out))
            outs[v] = res
        finally:
            B.eigcg_destroy(ctx)
    for v in (11, 12, 13):
        for k in range(3):
            assert np.array_equal(outs[v][k], outs[1][k]), (v, k)


@pytest.mark.parametrize("variant", [11, 12, 13])
def test_zmarch_cg_parity(B, variant):
    """FP64 CG with the z-march stencil on a lattice it runs on (whole 64-site
    tiles per xy-plane, Lt divisible by 8): x equals the oracle's iterate
    after the same number of iterations to 1e-10."""
    dims, eps, seed, mass = ZMARCH_LATTICES[0]
    U = gauge_field(dims, eps, seed)
    op = WilsonOperator(U, mass)
    b = gaussian_rhs(dims, 1000)
    cands, io = _cg_candidates(op.A, b.reshape(-1), 1e-10)
    ctx, _ = make_ctx(U, mass, max_iter=5000, stencil_variant=variant)
    try:
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK, B.eigcg_last_error(ctx)
        assert st[0]["iters"] in cands, (st[0]["iters"], io["iterations"])
        assert rel(host(x)[0].reshape(-1), cands[st[0]["iters"]]) <= 1e-10
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("nev,m,iters", [(4, 12, 40), (10, 40, 90), (2, 20, 60), (16, 40, 70)])
def test_eigcg_same_trajectory(B, cfg0, nev, m, iters):
    """Forced iteration count (max_iter) before loss of orthogonality: Ritz
    values to 1e-8 and x to 1e-10 against the oracle's eigCG."""
    U, op, b = cfg0
    xo, Vo, tho, io = eigcg(op.A, b.reshape(-1), nev, m, tol=1e-14, max_iter=iters)
    ctx, _ = make_ctx(U, -0.2, nev=nev, m=m, max_iter=iters, max_bank=64)
    try:
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-14, B.EIGCG_MODE_EIGCG)
        assert rc == B.EIGCG_ENOTCONV
        assert st[0]["iters"] == iters
        assert st[0]["restarts"] == len(io["restart_iterations"])
        th = B.eigcg_last_ritz(ctx)
        assert len(th) == len(tho)
        assert np.max(np.abs(th - tho) / np.abs(tho)) <= 1e-8
        assert rel(host(x)[0].reshape(-1), xo) <= 1e-10
    finally:
        B.eigcg_destroy(ctx)


def test_eigcg_full_run_cfg0(B, cfg0):
    """eigCG(10, 40) to 1e-8 on 4^4: the iteration count matches the oracle's
    (to one iteration: both stop tests compare a recursively updated residual
    with the tolerance, and their rounding differs), x matches the oracle's
    iterate after the same number of iterations to 1e-10; every Ritz pair of
    the resulting bank lies within its residual of the spectrum of A (dense
    eigendecomposition)."""
    from oracle.dense import dense_A
    U, op, b = cfg0
    xo, _, _, io = eigcg(op.A, b.reshape(-1), 10, 40, tol=1e-8)
    # the oracle's iterates one step either side of its own stop
    k = io["iterations"]
    cands = {k: xo}
    for kk in (k - 1, k + 1):
        cands[kk] = eigcg(op.A, b.reshape(-1), 10, 40, tol=0.0, max_iter=kk)[0]
    ctx, _ = make_ctx(U, -0.2, nev=10, m=40, max_bank=40)
    try:
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-8, B.EIGCG_MODE_EIGCG)
        assert rc == B.EIGCG_OK
        assert st[0]["iters"] in cands
        assert rel(host(x)[0].reshape(-1), cands[st[0]["iters"]]) <= 1e-10
        vals, res = B.eigcg_bank_info(ctx, residuals=True)
        A, _ = dense_A(op)
        lam = np.linalg.eigvalsh(A)
        for t_, r_ in zip(vals, res):
            assert np.min(np.abs(lam - t_)) <= r_ + 1e-12
        l = len(vals)
        Uv = dev(np.zeros((l, 4, 4, 4, 4, 4, 3), dtype=np.complex128))
        B.eigcg_bank_vectors(ctx, 0, l, Uv)
        Um = host(Uv).reshape(l, -1).T
        assert np.max(np.abs(Um.conj().T @ Um - np.eye(l))) < 1e-12
        H = B.eigcg_bank_matrix(ctx, l)
        assert np.max(np.abs(Um.conj().T @ (A @ Um) - H)) < 1e-11 * lam[-1]
    finally:
        B.eigcg_destroy(ctx)


def _dense_lowest(op, k):
    from oracle.dense import dense_A
    A, _ = dense_A(op)
    lam, X = np.linalg.eigh(A)
    return A, lam, X[:, :k]


def test_initcg_and_deflate_with_loaded_bank(B, cfg0):
    U, op, b = cfg0
    A, lam, X = _dense_lowest(op, 20)
    H = X.conj().T @ A @ X
    bf = b.reshape(-1)
    x0o = galerkin_guess(op.A, X, H, bf)
    xo, io = init_cg(op.A, X, H, bf, tol=1e-10)
    ctx, _ = make_ctx(U, -0.2, nev=10, m=40, max_bank=40, restart_tol=-1.0)
    try:
        vecs = dev(X.T.reshape((20, 4, 4, 4, 4, 4, 3)).copy())
        assert B.eigcg_bank_load(ctx, vecs) == 20
        x0 = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        B.eigcg_deflate_init(ctx, dev(b[None]), x0)
        assert rel(host(x0)[0].reshape(-1), x0o) <= 1e-12
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_INITCG)
        assert rc == B.EIGCG_OK
        assert st[0]["iters"] == io["iterations"]
        assert rel(host(x)[0].reshape(-1), xo) <= 1e-10
        vals, _ = B.eigcg_bank_info(ctx)
        assert np.max(np.abs(vals - lam[:20]) / lam[:20]) < 1e-10
    finally:
        B.eigcg_destroy(ctx)


def _restart_parity(B, ctx, op, X, H, b, rtol):
    """FP64 init-CG with one restart (Section 5.3) against the oracle's
    restarted init-CG: the first leg and the whole solve each stop within one
    iteration of the oracle's own stops, and x equals the oracle's iterate on
    that trajectory (restart after the same first leg, same total) to 1e-10."""
    bf = b.reshape(-1)
    _, io = init_cg(op.A, X, H, bf, tol=1e-10, restart_tol=rtol)
    assert io["restarted"]
    x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
    rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_INITCG)
    assert rc == B.EIGCG_OK, B.eigcg_last_error(ctx)
    assert st[0]["outer_steps"] == 1
    assert st[0]["true_rel_res"] <= 1e-10
    g1 = st[0]["first_leg_iters"]
    g2 = st[0]["iters"] - g1
    assert abs(g1 - io["first_leg_iterations"]) <= 1
    # the oracle's own second-leg stop after a first leg of that length
    _, io1 = init_cg(op.A, X, H, bf, tol=1e-10, restart_tol=rtol, first_leg_iters=g1)
    assert abs(g2 - (io1["iterations"] - g1)) <= 1
    xref, _ = init_cg(op.A, X, H, bf, tol=1e-10, restart_tol=rtol, first_leg_iters=g1,
                      second_leg_iters=g2)
    assert rel(host(x)[0].reshape(-1), xref) <= 1e-10
    return st[0]


def test_initcg_restart_parity(B, cfg0):
    """init-CG restarted once at ||r||/||b|| = 1e-6 (Section 5.3)."""
    U, op, b = cfg0
    A, lam, X = _dense_lowest(op, 12)
    H = X.conj().T @ A @ X
    ctx, _ = make_ctx(U, -0.2, nev=6, m=20, max_bank=12, restart_tol=1e-6)
    try:
        B.eigcg_bank_load(ctx, dev(X.T.reshape((12, 4, 4, 4, 4, 4, 3)).copy()))
        _restart_parity(B, ctx, op, X, H, b, 1e-6)
    finally:
        B.eigcg_destroy(ctx)


def _noisy_bank(op, noise_low=(-9.0, -7.0), seed=23):
    """The 20 lowest eigenvectors of the 4^4 operator, the lowest 12 with
    complex Gaussian noise of 10^-9 .. 10^-7 per entry (Ritz residuals of
    1e-6 .. 1e-4) and the next 8 with 1e-3, orthonormalised."""
    A, lam, Z = _dense_lowest(op, 20)
    rng = np.random.default_rng(seed)
    scale = np.concatenate([10.0 ** np.linspace(*noise_low, 12), np.full(8, 1e-3)])
    Xn = Z + scale * (rng.standard_normal(Z.shape) + 1j * rng.standard_normal(Z.shape))
    Xn, _ = np.linalg.qr(Xn)
    return A, lam, Xn, Xn.conj().T @ A @ Xn


def test_initcg_dynamic_restart_parity(B, cfg0):
    """The dynamic init-CG restart threshold (the open choice at the end of
    Section 5.3) on a loaded bank of approximate eigenvectors.  The context
    computes the bank's Ritz values and residual norms (blocks of 8 Ritz
    vectors per pass, a ragged last block of 4) and picks tau with the cost
    model; the oracle does the same from its own bank.  Ritz pairs, tau and
    the restarted solve agree (x to 1e-10 on the same trajectory)."""
    U, op, b = cfg0
    A, lam, Xn, H = _noisy_bank(op)
    theta, res = bank_ritz(op.A, Xn, H)
    tau_o, c0, c1 = choose_restart(theta, res, (8 + 0.2) ** 2, 1e-10, 6.0)
    assert tau_o > 0 and c1 < c0
    ctx, _ = make_ctx(U, -0.2, nev=10, m=40, max_bank=20, max_batch=8,
                      restart_rule=B.EIGCG_RESTART_DYNAMIC, restart_cost=6.0)
    try:
        assert B.eigcg_bank_load(ctx, dev(Xn.T.reshape((20, 4, 4, 4, 4, 4, 3)).copy())) == 20
        assert np.max(np.abs(B.eigcg_bank_matrix(ctx, 20) - H)) <= 1e-12 * lam[-1]
        vals, resg = B.eigcg_bank_info(ctx, residuals=True)
        np.testing.assert_allclose(vals, theta, rtol=1e-10)
        np.testing.assert_allclose(resg, res, rtol=1e-6, atol=1e-12 * lam[-1])
        st = _restart_parity(B, ctx, op, Xn, H, b, tau_o)
        assert st["restart_tau"] == pytest.approx(tau_o, rel=1e-9)
        # a second solve reuses the cached Ritz pairs: the same threshold
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st2 = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_INITCG)
        assert rc == B.EIGCG_OK and st2[0]["restart_tau"] == st["restart_tau"]
    finally:
        B.eigcg_destroy(ctx)


def test_initcg_dynamic_restart_declines_when_exact(B, cfg0):
    """With the exact eigenvectors (residuals at rounding level) nothing comes
    back after the projection: the dynamic rule plans no restart, and the
    solve is the oracle's unrestarted init-CG."""
    U, op, b = cfg0
    A, lam, X = _dense_lowest(op, 12)
    H = X.conj().T @ A @ X
    bf = b.reshape(-1)
    _, io = init_cg(op.A, X, H, bf, tol=1e-10)
    ctx, _ = make_ctx(U, -0.2, nev=6, m=20, max_bank=12,
                      restart_rule=B.EIGCG_RESTART_DYNAMIC)
    try:
        B.eigcg_bank_load(ctx, dev(X.T.reshape((12, 4, 4, 4, 4, 4, 3)).copy()))
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_INITCG)
        assert rc == B.EIGCG_OK
        assert st[0]["restart_tau"] == 0.0 and st[0]["first_leg_iters"] == st[0]["iters"]
        its = st[0]["iters"]
        assert abs(its - io["iterations"]) <= 1
        ref = init_cg(op.A, X, H, bf, tol=1e-10, second_leg_iters=its)[0]
        assert rel(host(x)[0].reshape(-1), ref) <= 1e-10
    finally:
        B.eigcg_destroy(ctx)


def test_initcg_default_restart_threshold_parity(B, cfg0):
    """The default init-CG restart threshold of an FP64 context (restart_tol
    = 0): 10 u ||A|| with the single-precision unit roundoff u = 2^-24 (the
    paper's runs are single precision, Section 5.1; Section 5.3 restarts
    within an order of magnitude of machine precision scaled by ||A||).  With
    a loaded bank no Ritz value has been seen yet, so ||A|| is estimated by
    the bound (8 + |m|)^2 of the Wilson normal operator.  The oracle runs
    init-CG with that threshold; a bank of approximate eigenvectors (the
    exact lowest 12 with 1e-7 noise) makes the restart matter."""
    U, op, b = cfg0
    A, lam, X = _dense_lowest(op, 12)
    rng = np.random.default_rng(17)
    Xn = X + 1e-7 * (rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape))
    Xn, _ = np.linalg.qr(Xn)
    H = Xn.conj().T @ A @ Xn
    rtol = 10 * 2.0 ** -24 * (8 + 0.2) ** 2
    ctx, _ = make_ctx(U, -0.2, nev=6, m=20, max_bank=12, restart_tol=0.0)
    try:
        B.eigcg_bank_load(ctx, dev(Xn.T.reshape((12, 4, 4, 4, 4, 4, 3)).copy()))
        # the bank as loaded (CGS2 keeps an orthonormal input up to rounding)
        Hg = B.eigcg_bank_matrix(ctx, 12)
        assert np.max(np.abs(Hg - H)) <= 1e-12 * lam[-1]
        _restart_parity(B, ctx, op, Xn, H, b, rtol)
    finally:
        B.eigcg_destroy(ctx)


def test_eigcg_same_trajectory_10_100(B):
    """eigCG(10, 100), the bench's window, past two restarts (iterations 101
    and 181) on the 8^4 field (eps 0.5, seed 2) at m = -0.3, forced to 200
    iterations: still before loss of orthogonality there (the oracle's Ritz
    values move by 2e-13 under a 1e-15 relative change of b).  Same restart
    count, Ritz values to 1e-8, x to 1e-10; this pins the tall product with
    K = 100 inputs and 20 outputs that the restart runs."""
    dims = (8, 8, 8, 8)
    U = gauge_field(dims, 0.5, 2)
    op = WilsonOperator(U, -0.3)
    b = gaussian_rhs(dims, 1000)
    xo, _, tho, io = eigcg(op.A, b.reshape(-1), 10, 100, tol=1e-14, max_iter=200)
    assert len(io["restart_iterations"]) == 2
    ctx, _ = make_ctx(U, -0.3, nev=10, m=100, max_iter=200, max_bank=16)
    try:
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-14, B.EIGCG_MODE_EIGCG)
        assert rc == B.EIGCG_ENOTCONV
        assert st[0]["iters"] == 200
        assert st[0]["restarts"] == 2
        th = B.eigcg_last_ritz(ctx)
        assert len(th) == len(tho) == 10
        assert np.max(np.abs(th - tho) / np.abs(tho)) <= 1e-8
        assert rel(host(x)[0].reshape(-1), xo) <= 1e-10
    finally:
        B.eigcg_destroy(ctx)


def test_batched_initcg_guesses_match_single_solves(B, cfg0):
    """FP64 init-CG over many right-hand sides forms the deflated guesses
    (eq. (2.1)) in groups of up to 16 columns, one pass over the bank per
    group; each solve is bitwise the one of a single-right-hand-side call
    (18 right-hand sides: groups of 16 and 2; with the init-CG restart)."""
    U, op, _ = cfg0
    A, lam, X = _dense_lowest(op, 12)
    rng = np.random.default_rng(23)
    Xn, _ = np.linalg.qr(X + 1e-6 * (rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape)))
    bs = gaussian_rhs_block((4, 4, 4, 4), [2400 + i for i in range(18)])
    x0 = 0.01 * gaussian_rhs_block((4, 4, 4, 4), [2500 + i for i in range(18)])
    ctx, _ = make_ctx(U, -0.2, nev=6, m=20, max_bank=12, restart_tol=1e-6)
    try:
        assert B.eigcg_bank_load(ctx, dev(Xn.T.reshape((12, 4, 4, 4, 4, 4, 3)).copy())) == 12
        xall = dev(x0)
        rc, st_all = B.eigcg_solve(ctx, dev(bs), xall, 1e-10, B.EIGCG_MODE_INITCG)
        assert rc == B.EIGCG_OK
        got = host(xall)
        for i in range(18):
            x1 = dev(x0[i:i + 1].copy())
            rc, st1 = B.eigcg_solve(ctx, dev(bs[i:i + 1]), x1, 1e-10, B.EIGCG_MODE_INITCG)
            assert rc == B.EIGCG_OK
            assert st1[0]["iters"] == st_all[i]["iters"]
            assert st1[0]["first_leg_iters"] == st_all[i]["first_leg_iters"]
            assert np.array_equal(host(x1)[0], got[i]), i
            assert st_all[i]["true_rel_res"] <= 1e-10
    finally:
        B.eigcg_destroy(ctx)


def test_lockstep_initcg_batches_match_single_solves(B, cfg0):
    """init-CG over a fixed bank (eq. (2.1), with the Section 5.3 restart) in
    lockstep batches of 4 right-hand sides: each column restarts on its own
    at its own iteration, and every solve is bitwise the single-right-hand-side
    solve run with the same stencil variant (6 right-hand sides: batches of 4
    and 2, guesses formed for all of them in one group)."""
    U, op, _ = cfg0
    A, lam, X = _dense_lowest(op, 12)
    rng = np.random.default_rng(29)
    Xn, _ = np.linalg.qr(X + 1e-6 * (rng.standard_normal(X.shape) + 1j * rng.standard_normal(X.shape)))
    bank = Xn.T.reshape((12, 4, 4, 4, 4, 4, 3)).copy()
    bs = gaussian_rhs_block((4, 4, 4, 4), [2600 + i for i in range(6)])
    kw = dict(nev=6, m=20, max_bank=12, restart_tol=1e-6)
    ctx4, _ = make_ctx(U, -0.2, max_batch=4, **kw)
    ctx1, _ = make_ctx(U, -0.2, max_batch=1, stencil_variant=B.eigcg_layout_info(ctx4)["variant64"],
                       **kw)
    try:
        assert B.eigcg_bank_load(ctx4, dev(bank)) == 12
        assert B.eigcg_bank_load(ctx1, dev(bank)) == 12
        x4 = dev(np.zeros_like(bs))
        rc, st4 = B.eigcg_solve(ctx4, dev(bs), x4, 1e-10, B.EIGCG_MODE_INITCG)
        assert rc == B.EIGCG_OK
        got = host(x4)
        assert sum(s["outer_steps"] for s in st4) >= 6  # every column restarted
        for i in range(6):
            x1 = dev(np.zeros_like(bs[i:i + 1]))
            rc, st1 = B.eigcg_solve(ctx1, dev(bs[i:i + 1]), x1, 1e-10, B.EIGCG_MODE_INITCG)
            assert rc == B.EIGCG_OK
            assert st1[0]["iters"] == st4[i]["iters"]
            assert st1[0]["first_leg_iters"] == st4[i]["first_leg_iters"]
            assert np.array_equal(host(x1)[0], got[i]), i
            assert st4[i]["true_rel_res"] <= 1e-10
    finally:
        B.eigcg_destroy(ctx1)
        B.eigcg_destroy(ctx4)


def _spectral_setup(op, nbank=12, sigma=40.0):
    """The lowest nbank eigenvectors of the 4^4 A (dense) as the bank, and the
    oracle's spectral preconditioner built from them (Ritz basis of H = X^H A X)."""
    A, lam, X = _dense_lowest(op, nbank)
    H = X.conj().T @ A @ X
    UR, th = ritz_basis(X, H)
    return A, X, H, spectral_preconditioner(UR, th, sigma)


def test_spectral_preconditioned_cg_parity(B, cfg0):
    """CG preconditioned by the bank as a spectral preconditioner (sigma = 40;
    the 12 near-zero modes of this field move to 40, CG needs ~5x fewer
    iterations): same stop within one iteration of the oracle's
    preconditioned CG, x equal to its iterate at the GPU's count to 1e-10."""
    U, op, b = cfg0
    A, X, H, Pinv = _spectral_setup(op)
    bf = b.reshape(-1)
    xo, io = cg(op.A, bf, tol=1e-10, apply_Pinv=Pinv)
    k = io["iterations"]
    cands = {k: xo}
    for kk in (k - 1, k + 1):
        cands[kk] = cg(op.A, bf, tol=0.0, max_iter=kk, true_residual_restarts=0, apply_Pinv=Pinv)[0]
    _, iplain = cg(op.A, bf, tol=1e-10)
    assert k < 0.3 * iplain["iterations"]
    ctx, _ = make_ctx(U, -0.2, nev=6, m=20, max_bank=12, max_iter=5000, precond=1,
                      precond_sigma=40.0)
    try:
        assert B.eigcg_bank_load(ctx, dev(X.T.reshape((12, 4, 4, 4, 4, 4, 3)).copy())) == 12
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK, B.eigcg_last_error(ctx)
        assert st[0]["iters"] in cands, (st[0]["iters"], k)
        assert st[0]["true_rel_res"] <= 1e-10
        assert rel(host(x)[0].reshape(-1), cands[st[0]["iters"]]) <= 1e-10
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("nev,m,iters", [(4, 12, 40), (10, 40, 80)])
def test_spectral_preconditioned_eigcg_same_trajectory(B, cfg0, nev, m, iters):
    """eigCG in the preconditioned form of Section 3 (window V = P^{-1} R,
    Ritz pairs of the pencil A y = lambda P y) with the spectral
    preconditioner, after the init-CG guess from the same bank, forced to a
    fixed iteration count: same restarts, Ritz values to 1e-8, x to 1e-10."""
    U, op, b = cfg0
    A, X, H, Pinv = _spectral_setup(op)
    bf = b.reshape(-1)
    x0 = galerkin_guess(op.A, X, H, bf)
    xo, _, tho, io = eigcg(op.A, bf, nev, m, x0=x0, tol=1e-14, max_iter=iters, apply_Pinv=Pinv)
    ctx, _ = make_ctx(U, -0.2, nev=nev, m=m, max_bank=64, max_iter=iters, precond=1,
                      precond_sigma=40.0)
    try:
        assert B.eigcg_bank_load(ctx, dev(X.T.reshape((12, 4, 4, 4, 4, 4, 3)).copy())) == 12
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-14, B.EIGCG_MODE_EIGCG)
        assert rc == B.EIGCG_ENOTCONV
        assert st[0]["iters"] == iters
        assert st[0]["restarts"] == len(io["restart_iterations"])
        th = B.eigcg_last_ritz(ctx)
        assert len(th) == len(tho)
        assert np.max(np.abs(th - tho) / np.abs(tho)) <= 1e-8
        assert rel(host(x)[0].reshape(-1), xo) <= 1e-10
        # the bank grew by the preconditioned Ritz vectors and stays orthonormal
        l = len(B.eigcg_bank_info(ctx)[0])
        assert l > 12
        Uv = dev(np.zeros((l, 4, 4, 4, 4, 4, 3), dtype=np.complex128))
        B.eigcg_bank_vectors(ctx, 0, l, Uv)
        Um = host(Uv).reshape(l, -1).T
        assert np.max(np.abs(Um.conj().T @ Um - np.eye(l))) < 1e-12
    finally:
        B.eigcg_destroy(ctx)


def test_spectral_preconditioner_with_batches_and_empty_bank(B, cfg0):
    """Preconditioned CG over a batch of 3 columns equals single-column solves
    bitwise; with an empty bank the preconditioner is the identity (the same
    bits as plain CG)."""
    U, op, _ = cfg0
    A, X, H, Pinv = _spectral_setup(op)
    bs = gaussian_rhs_block((4, 4, 4, 4), [2600, 2601, 2602])
    kw = dict(nev=6, m=20, max_bank=12, max_iter=5000, precond=1, precond_sigma=40.0)
    ctx3, _ = make_ctx(U, -0.2, max_batch=3, stencil_variant=3, **kw)
    ctx1, _ = make_ctx(U, -0.2, max_batch=1, stencil_variant=3, **kw)
    plain, _ = make_ctx(U, -0.2, max_batch=1, stencil_variant=3, max_iter=5000)
    try:
        # empty bank: P = I
        x_e = dev(np.zeros_like(bs[:1]))
        x_p = dev(np.zeros_like(bs[:1]))
        rc, st_e = B.eigcg_solve(ctx1, dev(bs[:1]), x_e, 1e-10, B.EIGCG_MODE_CG)
        rc, st_p = B.eigcg_solve(plain, dev(bs[:1]), x_p, 1e-10, B.EIGCG_MODE_CG)
        assert st_e[0]["iters"] == st_p[0]["iters"] and np.array_equal(host(x_e), host(x_p))
        vecs = dev(X.T.reshape((12, 4, 4, 4, 4, 4, 3)).copy())
        B.eigcg_bank_load(ctx1, vecs)
        B.eigcg_bank_load(ctx3, vecs)
        x3 = dev(np.zeros_like(bs))
        rc, st3 = B.eigcg_solve(ctx3, dev(bs), x3, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK
        for i in range(3):
            x1 = dev(np.zeros_like(bs[i:i + 1]))
            rc, st1 = B.eigcg_solve(ctx1, dev(bs[i:i + 1]), x1, 1e-10, B.EIGCG_MODE_CG)
            assert st1[0]["iters"] == st3[i]["iters"]
            assert np.array_equal(host(x1)[0], host(x3)[i])
    finally:
        for c in (ctx3, ctx1, plain):
            B.eigcg_destroy(c)


def test_incremental_eigcg_bank(B, cfg0):
    """Three Incremental eigCG steps: bank orthonormal, H = U^H A U, later
    right-hand sides converge faster, x matches the oracle's incremental run."""
    from oracle.incremental import incremental_eigcg
    U, op, _ = cfg0
    bs = gaussian_rhs_block((4, 4, 4, 4), [1000, 1001, 1002])
    xs, Uo, Ho, infos = incremental_eigcg(op.A, list(bs.reshape(3, -1)), 4, 30, tol=1e-8)
    # the oracle's first-solve iterates one step either side of its own stop
    k0 = infos[0]["iterations"]
    first = {k0: xs[0]}
    for kk in (k0 - 1, k0 + 1):
        first[kk] = eigcg(op.A, bs[0].reshape(-1), 4, 30, tol=0.0, max_iter=kk)[0]
    ctx, _ = make_ctx(U, -0.2, nev=4, m=30, max_bank=12)
    try:
        its = []
        for i in range(3):
            x = dev(np.zeros((1,) + bs[i].shape, dtype=np.complex128))
            rc, st = B.eigcg_solve(ctx, dev(bs[i][None]), x, 1e-8, B.EIGCG_MODE_EIGCG)
            assert rc == B.EIGCG_OK
            its.append(st[0]["iters"])
            # the first solve is the oracle's trajectory (its stop test may fire
            # one iteration apart: both test a recursive residual against the
            # tolerance with different rounding; then compare after the same
            # number of iterations); later ones start from banks built past
            # loss of orthogonality, whose rounding-level differences change
            # the init-CG guess: both solutions then only agree to the accuracy
            # their 1e-8 residuals fix
            ref = xs[i]
            if i == 0:
                assert its[0] in first
                ref = first[its[0]]
            assert rel(host(x)[0].reshape(-1), ref) <= (1e-10 if i == 0 else 1e-6)
        assert its[2] < its[0]
        vals, _ = B.eigcg_bank_info(ctx)
        vo = np.linalg.eigvalsh(Ho)
        assert len(vals) == len(vo)
        assert np.max(np.abs(vals[:4] - vo[:4]) / vo[:4]) < 1e-6
    finally:
        B.eigcg_destroy(ctx)


def test_batched_columns_match_single(B, cfg0):
    """Each column of a batched solve is bitwise the single-RHS solve run with
    the same stencil variant (the autotuner may pick different variants for
    different batch widths; each variant's results do not depend on the
    width)."""
    U, op, _ = cfg0
    bs = gaussian_rhs_block((4, 4, 4, 4), [2000, 2001, 2002, 2003])
    ctx4, _ = make_ctx(U, -0.2, max_batch=4)
    ctx1, _ = make_ctx(U, -0.2, max_batch=1,
                       stencil_variant=B.eigcg_layout_info(ctx4)["variant64"])
    try:
        x4 = dev(np.zeros_like(bs))
        rc, st4 = B.eigcg_solve(ctx4, dev(bs), x4, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK
        for i in range(4):
            x1 = dev(np.zeros_like(bs[i:i + 1]))
            rc, st1 = B.eigcg_solve(ctx1, dev(bs[i:i + 1]), x1, 1e-10, B.EIGCG_MODE_CG)
            assert st1[0]["iters"] == st4[i]["iters"]
            assert np.array_equal(host(x1)[0], host(x4)[i])
    finally:
        B.eigcg_destroy(ctx1)
        B.eigcg_destroy(ctx4)


@pytest.mark.parametrize("dims,variant", [((4, 4, 4, 4), 9), ((4, 4, 4, 4), 3),
                                          ((8, 8, 2, 8), 9), ((8, 8, 2, 8), 5), ((8, 8, 2, 8), 10),
                                          ((8, 8, 4, 8), 14), ((8, 8, 4, 8), 15)])
@pytest.mark.parametrize("precision", [0, 1])
def test_batched_multicolumn_kernels_match_single(B, dims, variant, precision):
    """Batches of 5 columns run the stencil with several right-hand sides per
    workgroup (links loaded once for all of them); every column is bitwise
    the single-RHS solve, in FP64 and in mixed precision (FP32 inner
    iteration, lockstep FP64 reliable updates)."""
    U = gauge_field(dims, 0.4, 3)
    bs = gaussian_rhs_block(dims, [2200 + i for i in range(5)])
    kw = dict(precision=precision, reliable_every=20, stencil_variant=variant, max_iter=3000)
    ctx1, _ = make_ctx(U, -0.1, max_batch=1, **kw)
    ctx5, _ = make_ctx(U, -0.1, max_batch=5, **kw)
    try:
        x5 = dev(np.zeros_like(bs))
        rc, st5 = B.eigcg_solve(ctx5, dev(bs), x5, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK
        for i in range(5):
            x1 = dev(np.zeros_like(bs[i:i + 1]))
            rc, st1 = B.eigcg_solve(ctx1, dev(bs[i:i + 1]), x1, 1e-10, B.EIGCG_MODE_CG)
            assert st1[0]["iters"] == st5[i]["iters"]
            assert np.array_equal(host(x1)[0], host(x5)[i])
            assert st5[i]["true_rel_res"] <= 1e-10
    finally:
        B.eigcg_destroy(ctx1)
        B.eigcg_destroy(ctx5)


def test_edge_cases(B, cfg0):
    U, op, b = cfg0
    ctx, _ = make_ctx(U, -0.2, max_iter=7, max_batch=2)
    try:
        bb = np.stack([np.zeros_like(b), b])
        x = dev(np.ones_like(bb))
        rc, st = B.eigcg_solve(ctx, dev(bb), x, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_ENOTCONV
        assert st[0]["iters"] == 0 and np.all(host(x)[0] == 0)
        assert st[1]["iters"] == 7 and st[1]["status"] == B.EIGCG_ENOTCONV
        bad = b.copy()
        bad[0, 0, 0, 0, 0, 0] = np.nan
        with pytest.raises(B.EigcgError):
            B.eigcg_solve(ctx, dev(bad[None]), dev(np.zeros_like(b[None])), 1e-10)
    finally:
        B.eigcg_destroy(ctx)
    with pytest.raises(B.EigcgError):
        make_ctx(U, -0.2, nev=10, m=20)  # m must exceed 2 nev


def test_mixed_precision_cg(B, cfg0):
    """FP32 inner CG with FP64 reliable updates reaches the FP64 tolerance;
    error against the FP64 oracle solution is stated: <= 1e-6 relative."""
    U, op, b = cfg0
    xo, io = cg(op.A, b.reshape(-1), tol=1e-10)
    ctx, _ = make_ctx(U, -0.2, precision=B.EIGCG_MIXED_FP32, reliable_every=25, max_iter=5000)
    try:
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK, B.eigcg_last_error(ctx)
        assert st[0]["true_rel_res"] <= 1e-10
        assert rel(host(x)[0].reshape(-1), xo) <= 1e-6
    finally:
        B.eigcg_destroy(ctx)


def test_mixed_precision_eigcg_bank(B, cfg0):
    """Mixed-precision Incremental eigCG: FP32 window and bank, FP64 reliable
    updates.  The bank stays a valid Rayleigh-Ritz space of the HPD A: its
    Ritz values lie in the spectrum's range (up to FP32 rounding of the
    stored vectors), the lowest approximates the smallest eigenvalue, and
    deflated solves converge to 1e-10.  Error against the dense spectrum is
    stated in the assertions."""
    from oracle.dense import dense_A
    U, op, b = cfg0
    A, _ = dense_A(op)
    lam = np.linalg.eigvalsh(A)
    ctx, _ = make_ctx(U, -0.2, precision=B.EIGCG_MIXED_FP32, reliable_every=50, max_iter=5000,
                      nev=6, m=24, max_bank=24)
    try:
        rhs = gaussian_rhs_block((4, 4, 4, 4), [2100 + i for i in range(4)])
        for i in range(4):
            x = dev(np.zeros((1,) + rhs[i].shape, dtype=np.complex128))
            rc, st = B.eigcg_solve(ctx, dev(rhs[i][None].copy()), x, 1e-10, B.EIGCG_MODE_EIGCG)
            assert rc == B.EIGCG_OK and st[0]["true_rel_res"] <= 1e-10
        vals, _ = B.eigcg_bank_info(ctx)
        assert len(vals) >= 6
        assert vals[0] >= lam[0] * (1 - 1e-3) - 1e-5 * lam[-1]
        assert vals[-1] <= lam[-1] * (1 + 1e-5)
        assert abs(vals[0] - lam[0]) <= 1e-2 * lam[0]
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_INITCG)
        assert rc == B.EIGCG_OK and st[0]["true_rel_res"] <= 1e-10
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replay_matches_eager(B, cfg0, precision):
    """CG segments replayed from captured HIP graphs give bitwise the eager
    result, over several solves in a row (each replays its graphs many times,
    with the solver's own copies and host synchronisations in between)."""
    U, op, _ = cfg0
    bs = gaussian_rhs_block((4, 4, 4, 4), [2300 + i for i in range(3)])
    kw = dict(precision=precision, max_batch=3, reliable_every=20, max_iter=3000, check_every=8)
    ctx_e, _ = make_ctx(U, -0.2, **kw)
    ctx_g, _ = make_ctx(U, -0.2, use_graphs=1, **kw)
    try:
        for rep in range(3):
            xe = dev(np.zeros_like(bs))
            xg = dev(np.zeros_like(bs))
            rc_e, st_e = B.eigcg_solve(ctx_e, dev(bs), xe, 1e-10, B.EIGCG_MODE_CG)
            rc_g, st_g = B.eigcg_solve(ctx_g, dev(bs), xg, 1e-10, B.EIGCG_MODE_CG)
            assert rc_e == rc_g == B.EIGCG_OK
            assert [s["iters"] for s in st_e] == [s["iters"] for s in st_g]
            assert np.array_equal(host(xe), host(xg)), rep
    finally:
        B.eigcg_destroy(ctx_e)
        B.eigcg_destroy(ctx_g)


def test_graph_replay_with_sampling_matches_eager(B, cfg0):
    """The bench's launch path: Incremental eigCG then init-CG in one context,
    segments replayed from graphs kept across solves while every 7th
    iteration is launched on its own with timing events.  Bitwise the eager
    result and the same iterations; the graph path still times launches."""
    U, op, _ = cfg0
    bs = gaussian_rhs_block((4, 4, 4, 4), [2400 + i for i in range(5)])
    kw = dict(nev=4, m=16, max_bank=16, max_iter=3000, check_every=8, sample_every=7)
    ctx_e, _ = make_ctx(U, -0.2, **kw)
    ctx_g, _ = make_ctx(U, -0.2, use_graphs=1, **kw)
    try:
        out = []
        for ctx in (ctx_e, ctx_g):
            x = dev(np.zeros_like(bs))
            its = []
            for i in range(2):  # one right-hand side per call: the bank grows in between
                rc, st = B.eigcg_solve(ctx, dev(bs[i:i + 1]), x[i:i + 1], 1e-10, B.EIGCG_MODE_EIGCG)
                assert rc == B.EIGCG_OK
                its.append(st[0]["iters"])
            rc, st = B.eigcg_solve(ctx, dev(bs[2:]), x[2:], 1e-10, B.EIGCG_MODE_INITCG)
            assert rc == B.EIGCG_OK
            its += [s["iters"] for s in st]
            out.append((host(x), its, B.eigcg_kernel_samples(ctx)["f64"]["n"]))
        (xe, ie, ne), (xg, ig, ng) = out
        assert ie == ig
        assert np.array_equal(xe, xg)
        assert ne > 0 and ng > 0
    finally:
        B.eigcg_destroy(ctx_e)
        B.eigcg_destroy(ctx_g)


def test_half_precision_cg_and_initcg(B, cfg0):
    """16-bit links and vectors with FP32 arithmetic (FP32 iterate), each inner
    solve rescaled, FP64 refinement: CG and init-CG reach the FP64 tolerance;
    error against the FP64 oracle solution stated: <= 1e-6 relative.  A batch
    of three columns is bitwise the three single solves (per-column
    refinement schedule), and eigCG mode is refused."""
    from oracle.dense import dense_A
    U, op, b = cfg0
    xo, _ = cg(op.A, b.reshape(-1), tol=1e-10)
    ctx, _ = make_ctx(U, -0.2, precision=B.EIGCG_MIXED_HALF, max_iter=20000, max_bank=12)
    # batch invariance holds for one stencil variant (FP64 outer passes and
    # 16-bit inner passes alike), so both contexts force the same one
    ctx1, _ = make_ctx(U, -0.2, precision=B.EIGCG_MIXED_HALF, max_iter=20000, stencil_variant=6)
    ctx3, _ = make_ctx(U, -0.2, precision=B.EIGCG_MIXED_HALF, max_iter=20000, max_batch=3,
                       stencil_variant=6)
    try:
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK, B.eigcg_last_error(ctx)
        assert st[0]["true_rel_res"] <= 1e-10 and st[0]["outer_steps"] >= 2
        assert rel(host(x)[0].reshape(-1), xo) <= 1e-6
        bs = gaussian_rhs_block((4, 4, 4, 4), [2400, 2401, 2402])
        x3 = dev(np.zeros_like(bs))
        rc, st3 = B.eigcg_solve(ctx3, dev(bs), x3, 1e-10, B.EIGCG_MODE_CG)
        assert rc == B.EIGCG_OK
        for i in range(3):
            x1 = dev(np.zeros_like(bs[i:i + 1]))
            rc, st1 = B.eigcg_solve(ctx1, dev(bs[i:i + 1]), x1, 1e-10, B.EIGCG_MODE_CG)
            assert st1[0]["iters"] == st3[i]["iters"]
            assert np.array_equal(host(x1)[0], host(x3)[i])
        # init-CG with a bank of exact low eigenvectors
        A, _ = dense_A(op)
        lam, X = np.linalg.eigh(A)
        B.eigcg_bank_load(ctx, dev(X[:, :12].T.reshape((12, 4, 4, 4, 4, 4, 3)).copy()))
        Xb = X[:, :12]
        xi, _ = init_cg(op.A, Xb, Xb.conj().T @ A @ Xb, b.reshape(-1), tol=1e-10)
        x = dev(np.zeros((1,) + b.shape, dtype=np.complex128))
        rc, st2 = B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_INITCG)
        assert rc == B.EIGCG_OK and st2[0]["true_rel_res"] <= 1e-10
        assert rel(host(x)[0].reshape(-1), xi) <= 1e-6
        assert st2[0]["iters"] < st[0]["iters"]
        with pytest.raises(B.EigcgError):
            B.eigcg_solve(ctx, dev(b[None]), x, 1e-10, B.EIGCG_MODE_EIGCG)
    finally:
        B.eigcg_destroy(ctx)
        B.eigcg_destroy(ctx1)
        B.eigcg_destroy(ctx3)


def test_auto_mode_matches_explicit_modes(B, cfg0):
    """EIGCG_MODE_AUTO over eight right-hand sides: a prefix solved with
    Incremental eigCG (at least three), the rest with init-CG, every solve to
    1e-10; the same right-hand sides through explicit EIGCG then INITCG calls
    on a fresh context give the same bits."""
    import torch
    U, op, _ = cfg0
    bs = gaussian_rhs_block((4, 4, 4, 4), [4000 + i for i in range(8)])
    kw = dict(nev=4, m=20, max_bank=40, max_iter=5000, stencil_variant=6)
    ctx, _ = make_ctx(U, -0.2, **kw)
    try:
        x = dev(np.zeros_like(bs))
        rc, st = B.eigcg_solve(ctx, dev(bs), x, 1e-10, B.EIGCG_MODE_AUTO)
        assert rc == B.EIGCG_OK
        modes = [s["mode_used"] for s in st]
        keig = modes.count(B.EIGCG_MODE_EIGCG)
        assert keig >= 3 and modes == [B.EIGCG_MODE_EIGCG] * keig + [B.EIGCG_MODE_INITCG] * (8 - keig)
        xa = host(x)
        for j in range(8):  # FP64 residual with the oracle's A
            r = bs[j].reshape(-1) - op.A(xa[j].reshape(-1))
            assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(bs[j])
        l_auto = len(B.eigcg_bank_info(ctx)[0])
    finally:
        B.eigcg_destroy(ctx)
    ctx, _ = make_ctx(U, -0.2, **kw)
    try:
        x = dev(np.zeros_like(bs))
        rc1, _ = B.eigcg_solve(ctx, dev(bs[:keig]), x[:keig], 1e-10, B.EIGCG_MODE_EIGCG)
        xr = torch.zeros_like(x[keig:])
        rc2, _ = B.eigcg_solve(ctx, dev(bs[keig:]), xr, 1e-10, B.EIGCG_MODE_INITCG) \
            if keig < 8 else (B.EIGCG_OK, [])
        assert rc1 == B.EIGCG_OK and rc2 == B.EIGCG_OK
        assert np.array_equal(host(x)[:keig], xa[:keig])
        if keig < 8:
            assert np.array_equal(host(xr), xa[keig:])
        assert len(B.eigcg_bank_info(ctx)[0]) == l_auto
    finally:
        B.eigcg_destroy(ctx)



def test_bank_truncate_and_restore(B, cfg0):
    """A bank from three Incremental eigCG(6, 30) solves: saved with
    eigcg_bank_vectors / eigcg_bank_matrix and restored into a fresh context,
    init-CG gives the same bits; truncated to its 8 lowest Ritz vectors, the
    bank holds the 8 lowest Ritz values of before, stays orthonormal with
    H = U^H A U diagonal (oracle's A), and still deflates init-CG to 1e-10."""
    import torch
    U, op, _ = cfg0
    kw = dict(nev=6, m=30, max_bank=36, max_iter=5000, stencil_variant=6)
    bs = gaussian_rhs_block((4, 4, 4, 4), [4100, 4101, 4102, 4103])
    ctx, _ = make_ctx(U, -0.2, **kw)
    ctx2, _ = make_ctx(U, -0.2, **kw)
    try:
        x = dev(np.zeros_like(bs))
        rc, _ = B.eigcg_solve(ctx, dev(bs[:3]), x[:3], 1e-10, B.EIGCG_MODE_EIGCG)
        assert rc == B.EIGCG_OK
        vals, _ = B.eigcg_bank_info(ctx)
        l = len(vals)
        Ut = dev(np.zeros((l,) + bs.shape[1:], dtype=np.complex128))
        B.eigcg_bank_vectors(ctx, 0, l, Ut)
        H = B.eigcg_bank_matrix(ctx, l)
        B.eigcg_bank_restore(ctx2, Ut, H)
        assert np.array_equal(B.eigcg_bank_matrix(ctx2, l), H)
        xa, xb = torch.zeros_like(x[3:]), torch.zeros_like(x[3:])
        B.eigcg_solve(ctx, dev(bs[3:]), xa, 1e-10, B.EIGCG_MODE_INITCG)
        B.eigcg_solve(ctx2, dev(bs[3:]), xb, 1e-10, B.EIGCG_MODE_INITCG)
        assert torch.equal(xa, xb)
        # truncation
        B.eigcg_bank_truncate(ctx, 8)
        tvals, _ = B.eigcg_bank_info(ctx)
        assert len(tvals) == 8
        assert np.max(np.abs(tvals - vals[:8]) / vals[:8]) <= 1e-10
        Ut8 = dev(np.zeros((8,) + bs.shape[1:], dtype=np.complex128))
        B.eigcg_bank_vectors(ctx, 0, 8, Ut8)
        Um = host(Ut8).reshape(8, -1).T
        assert np.max(np.abs(Um.conj().T @ Um - np.eye(8))) < 1e-12
        AU = np.stack([op.A(Um[:, j]) for j in range(8)], axis=1)
        G = Um.conj().T @ AU
        assert np.max(np.abs(G - np.diag(tvals))) <= 1e-10 * tvals[-1]
        xt = torch.zeros_like(x[3:])
        rc, st = B.eigcg_solve(ctx, dev(bs[3:]), xt, 1e-10, B.EIGCG_MODE_INITCG)
        assert rc == B.EIGCG_OK and st[0]["true_rel_res"] <= 1e-10
        with pytest.raises(B.EigcgError):
            B.eigcg_bank_restore(ctx2, Ut[:2], -np.eye(2))  # not positive definite
    finally:
        B.eigcg_destroy(ctx)
        B.eigcg_destroy(ctx2)


def test_bank_truncate_large(B, cfg0):
    """Truncation of a full 240-vector bank to 200 and 30 (the product U Y_k
    then runs in several column groups): the lowest Ritz values of H are
    kept, U stays orthonormal and H = U^H A U is the diagonal of them."""
    U, op, _ = cfg0
    ctx, _ = make_ctx(U, -0.2, nev=10, m=40, max_bank=240, max_iter=5000)
    try:
        vecs = gaussian_rhs_block((4, 4, 4, 4), [5000 + i for i in range(240)])
        added = B.eigcg_bank_load(ctx, dev(vecs))
        assert added == 240
        vals, _ = B.eigcg_bank_info(ctx)
        for k in (200, 30):
            B.eigcg_bank_truncate(ctx, k)
            tv, _ = B.eigcg_bank_info(ctx)
            assert len(tv) == k
            assert np.max(np.abs(tv - vals[:k]) / vals[:k]) <= 1e-10
            Ut = dev(np.zeros((k,) + vecs.shape[1:], dtype=np.complex128))
            B.eigcg_bank_vectors(ctx, 0, k, Ut)
            Um = host(Ut).reshape(k, -1).T
            assert np.max(np.abs(Um.conj().T @ Um - np.eye(k))) < 1e-11
            G = Um.conj().T @ np.stack([op.A(Um[:, j]) for j in range(k)], axis=1)
            assert np.max(np.abs(G - np.diag(tv))) <= 1e-10 * tv[-1]
    finally:
        B.eigcg_destroy(ctx)


def test_auto_mode_with_16bit_inner_solves_is_initcg(B, cfg0):
    """16-bit inner solves cannot run eigCG: EIGCG_MODE_AUTO solves every
    right-hand side with init-CG (FP64 refinement) and leaves the bank alone."""
    U, op, _ = cfg0
    ctx, _ = make_ctx(U, -0.2, precision=2, nev=4, m=20, max_bank=40, max_iter=20000)
    try:
        bs = gaussian_rhs_block((4, 4, 4, 4), [4200, 4201, 4202, 4203])
        x = dev(np.zeros_like(bs))
        rc, st = B.eigcg_solve(ctx, dev(bs), x, 1e-10, B.EIGCG_MODE_AUTO)
        assert rc == B.EIGCG_OK
        assert all(s["mode_used"] == B.EIGCG_MODE_INITCG for s in st)
        assert len(B.eigcg_bank_info(ctx)[0]) == 0
        xa = host(x)
        for j in range(4):
            r = bs[j].reshape(-1) - op.A(xa[j].reshape(-1))
            assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(bs[j])
    finally:
        B.eigcg_destroy(ctx)


@pytest.mark.parametrize("precision,tol", [(1, 1e-6), (2, 1e-6)])
def test_deflate_init_mixed_bank(B, cfg0, precision, tol):
    """eq. (2.1) with the FP32 bank of a mixed context (FP32 or 16-bit inner
    solves): the deflated guess matches the oracle's Galerkin guess to FP32
    accuracy, for two right-hand sides in one call."""
    U, op, b = cfg0
    A, lam, X = _dense_lowest(op, 20)
    H = X.conj().T @ A @ X
    bs = gaussian_rhs_block((4, 4, 4, 4), [4300, 4301])
    ctx, _ = make_ctx(U, -0.2, precision=precision, nev=10, m=40, max_bank=40, max_batch=2)
    try:
        vecs = dev(X.T.reshape((20, 4, 4, 4, 4, 4, 3)).copy())
        assert B.eigcg_bank_load(ctx, vecs) == 20
        x0 = dev(np.zeros_like(bs))
        B.eigcg_deflate_init(ctx, dev(bs), x0)
        for j in range(2):
            x0o = galerkin_guess(op.A, X, H, bs[j].reshape(-1))
            assert rel(host(x0)[j].reshape(-1), x0o) <= tol
    finally:
        B.eigcg_destroy(ctx)
