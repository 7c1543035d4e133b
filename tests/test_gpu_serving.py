"""GPU tests of the serving loop (continuous batching over several fields).

Every request's result must be the same alone and in the mix: each column of
the batched iteration is reduced in a fixed order of its own and refined on
its own schedule, so the comparison is bitwise.  Results are also checked
against the FP64 oracle's deflated solve (same bank).
"""

import time

import numpy as np
import pytest

from gpu_common import dev, host, make_ctx, rel
from oracle.dense import dense_A
from oracle.dirac import WilsonOperator
from oracle.initcg import init_cg
from synthetic import gauge_field, gaussian_rhs_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0707_0131_amd import binding
    return binding


FIELDS = [((4, 4, 4, 4), 0.3, 0, -0.2), ((4, 4, 2, 8), 0.4, 6, -0.1)]


def _setup(B, precision, max_batch, nbank=12):
    ctxs, keep, ops, banks = [], [], [], []
    for dims, eps, seed, mass in FIELDS:
        U = gauge_field(dims, eps, seed)
        op = WilsonOperator(U, mass)
        A, _ = dense_A(op)
        lam, X = np.linalg.eigh(A)
        # no init-CG restart: the comparison below is with the oracle's init-CG
        # without one (mixed contexts refine instead and ignore it)
        ctx, g = make_ctx(U, mass, precision=precision, max_batch=max_batch, max_bank=nbank,
                          nev=6, m=20, max_iter=4000, restart_tol=-1.0)
        shape = (dims[3], dims[2], dims[1], dims[0], 4, 3)
        B.eigcg_bank_load(ctx, dev(X[:, :nbank].T.reshape((nbank,) + shape).copy()))
        ctxs.append(ctx)
        keep.append(g)
        ops.append((op, shape))
        banks.append((X[:, :nbank], A))
    return ctxs, keep, ops, banks


def _serve(B, ctxs, jobs, budget=0, one_by_one=False):
    srv = B.eigcg_server_create(budget)
    fids = [B.eigcg_server_add(srv, c) for c in ctxs]
    try:
        tickets = []
        for f, b, x in jobs:
            tickets.append(B.eigcg_submit(srv, fids[f], b, x, 1e-10))
            if one_by_one:
                B.eigcg_server_drain(srv)
        B.eigcg_server_drain(srv)
        out = [B.eigcg_poll(srv, t) for t in tickets]
    finally:
        B.eigcg_server_destroy(srv)
    return out


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_alone_equals_mixed(B, precision):
    import torch
    ctxs, keep, ops, banks = _setup(B, precision, max_batch=3)
    try:
        rhs = []
        for f, (op, shape) in enumerate(ops):
            bs = gaussian_rhs_block(tuple(reversed(shape[:4])), [3000 + 10 * f + i for i in range(5)])
            rhs.append(bs)
        jobs_alone, jobs_mix = [], []
        for f in range(2):
            for i in range(5):
                b = dev(rhs[f][i][None].copy())
                jobs_alone.append((f, b, torch.zeros_like(b)))
                jobs_mix.append((f, b, torch.zeros_like(b)))
        res_alone = _serve(B, ctxs, jobs_alone, one_by_one=True)
        # interleave fields and submit everything at once (more requests than slots)
        order = [0, 5, 1, 6, 2, 7, 3, 8, 4, 9]
        jobs_mix2 = [jobs_mix[k] for k in order]
        res_mix = _serve(B, ctxs, jobs_mix2)
        for k, (f, b, x) in enumerate(jobs_alone):
            rc, st = res_alone[k]
            assert rc == B.EIGCG_OK and st["true_rel_res"] <= 1e-10
        for pos, k in enumerate(order):
            rc, st = res_mix[pos]
            assert rc == B.EIGCG_OK
            assert res_alone[k][1]["iters"] == st["iters"]
            assert torch.equal(jobs_alone[k][2], jobs_mix[k][2])
        # against the oracle's init-CG with the same bank: FP64 results equal
        # the oracle's iterate after the same number of iterations (the
        # oracle's stop either side of its own count) to 1e-10; mixed
        # precision has its stated error against the FP64 solution
        for k, (f, b, x) in enumerate(jobs_alone):
            op, shape = ops[f]
            X, A = banks[f]
            H = X.conj().T @ A @ X
            bf = host(b).reshape(-1)
            xo, io = init_cg(op.A, X, H, bf, tol=1e-10)
            if precision == 0:
                its = res_alone[k][1]["iters"]
                assert abs(its - io["iterations"]) <= 1
                ref = init_cg(op.A, X, H, bf, tol=1e-10, second_leg_iters=its)[0]
                assert rel(host(x).reshape(-1), ref) <= 1e-10
            else:
                assert rel(host(x).reshape(-1), xo) <= 1e-6
    finally:
        for c in ctxs:
            B.eigcg_destroy(c)


def test_small_budget_still_completes(B):
    import torch
    ctxs, keep, ops, banks = _setup(B, 0, max_batch=4)
    try:
        jobs = []
        for f, (op, shape) in enumerate(ops):
            bs = gaussian_rhs_block(tuple(reversed(shape[:4])), [5000 + i for i in range(4)])
            for i in range(4):
                b = dev(bs[i][None].copy())
                jobs.append((f, b, torch.zeros_like(b)))
        mem = sum(B.eigcg_memory(c) for c in ctxs)
        res = _serve(B, ctxs, jobs, budget=mem + 1)  # room for no extra working set
        for rc, st in res:
            assert rc == B.EIGCG_OK and st["true_rel_res"] <= 1e-10
            assert st["seconds"] > 0
    finally:
        for c in ctxs:
            B.eigcg_destroy(c)


def test_schur_field_alone_equals_mixed(B):
    """An odd-even preconditioned context served beside an unpreconditioned
    one (FP32 inner solves, FP64 refinement): each even-site request gives the
    same bits alone and in the mix and matches the oracle's init-CG on Ahat
    with the same bank."""
    import torch
    from oracle.dense import dense_matrix
    from oracle.schur import SchurOperator
    from synthetic import gaussian_half_rhs
    dims, eps, seed, mass = (4, 4, 4, 4), 0.3, 0, -0.2
    U = gauge_field(dims, eps, seed)
    sop = SchurOperator(U, mass)
    A = dense_matrix(sop.A, sop.n)
    lam, X = np.linalg.eigh(A)
    nbank = 12
    sctx, g1 = make_ctx(U, mass, precision=1, max_batch=3, max_bank=nbank, nev=6, m=20,
                        max_iter=4000, schur=1)
    ctxs, keep, ops, banks = _setup(B, 1, max_batch=3)
    try:
        B.eigcg_bank_load(sctx, dev(X[:, :nbank].T.reshape((nbank, sop.n // 12, 4, 3)).copy()))
        allc = [sctx, ctxs[1]]
        jobs_alone, jobs_mix = [], []
        for i in range(4):
            b = dev(gaussian_half_rhs(dims, 3100 + i)[None].copy())
            jobs_alone.append((0, b, torch.zeros_like(b)))
            jobs_mix.append((0, b, torch.zeros_like(b)))
        op1, shape1 = ops[1]
        bs = gaussian_rhs_block(tuple(reversed(shape1[:4])), [3200 + i for i in range(4)])
        for i in range(4):
            b = dev(bs[i][None].copy())
            jobs_alone.append((1, b, torch.zeros_like(b)))
            jobs_mix.append((1, b, torch.zeros_like(b)))
        res_alone = _serve(B, allc, jobs_alone, one_by_one=True)
        order = [0, 4, 1, 5, 2, 6, 3, 7]
        res_mix = _serve(B, allc, [jobs_mix[k] for k in order])
        for pos, k in enumerate(order):
            assert res_alone[k][0] == B.EIGCG_OK and res_mix[pos][0] == B.EIGCG_OK
            assert res_alone[k][1]["iters"] == res_mix[pos][1]["iters"]
            assert torch.equal(jobs_alone[k][2], jobs_mix[k][2])
        H = X[:, :nbank].conj().T @ A @ X[:, :nbank]
        for k in range(4):
            _, b, x = jobs_alone[k]
            xo, _ = init_cg(sop.A, X[:, :nbank], H, host(b).reshape(-1), tol=1e-10)
            assert rel(host(x).reshape(-1), xo) <= 1e-6
    finally:
        B.eigcg_destroy(sctx)
        for c in ctxs:
            B.eigcg_destroy(c)
