"""CPU tests of the C-ABI library: it loads, exports every function that
include/eigcg.h declares, validates arguments without touching a GPU, and its
host FP64 linear algebra (window eigensolver, thin QR, Cholesky) agrees with
numpy.linalg."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eigcg.h")


@pytest.fixture(scope="module")
def B():
    lib = os.path.join(ROOT, "paper_0707_0131_amd", "libeigcg.so")
    if not os.path.exists(lib):
        from paper_0707_0131_amd.build import build
        build()
    from paper_0707_0131_amd import binding
    return binding


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(eigcg_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported(B):
    names = _declared()
    assert len(names) >= 25
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps each one under the same name
    assert set(names) <= set(B.SIGNATURES)


def test_default_params_and_validation(B):
    p = B.eigcg_default_params()
    assert (p.nev, p.m, p.max_bank, p.precision, p.max_batch) == (10, 100, 240, 0, 1)
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    for bad in [dict(nev=10, m=20), dict(dims=(1, 4, 4, 4)), dict(max_batch=13),
                dict(max_bank=300), dict(precision=7), dict(max_iter=0),
                dict(mass=float("nan")), dict(nev=0), dict(schur=2),
                dict(schur=1, dims=(4, 4, 3, 4)), dict(stencil_variant=16),
                dict(sample_every=-1), dict(nev=16, m=257), dict(precond=2),
                dict(precond=1, precision=1), dict(precond_sigma=float("inf")),
                dict(restart_rule=2), dict(restart_cost=float("nan"))]:
        q = B.eigcg_default_params(**bad)
        rc = B.LIB.eigcg_create(ctypes.byref(q), fake, None, ctypes.byref(ctx))
        assert rc == B.EIGCG_EINVAL, bad
        assert B.eigcg_last_error(None), bad  # the thread's create error says why
    assert B.LIB.eigcg_create(ctypes.byref(p), None, None, ctypes.byref(ctx)) == B.EIGCG_EINVAL
    assert B.LIB.eigcg_solve(None, 1, None, None, 1e-10, 0, None) == B.EIGCG_EINVAL
    assert B.LIB.eigcg_destroy(None) == B.EIGCG_EINVAL
    for fn, args in [("eigcg_schur_rhs", (None, 1, None, None)),
                     ("eigcg_schur_reconstruct", (None, 1, None, None, None)),
                     ("eigcg_bank_truncate", (None, 1)),
                     ("eigcg_bank_lock", (None, 1e-6, None)),
                     ("eigcg_bank_locked", (None,)),
                     ("eigcg_bank_restore", (None, 1, None, None)),
                     ("eigcg_solve_bicgstab", (None, 1, None, None, 1e-10, 0, 0, None))]:
        assert getattr(B.LIB, fn)(*args) == B.EIGCG_EINVAL, fn
    with pytest.raises(KeyError):
        B.eigcg_default_params(no_such_field=1)


def test_server_validation_without_gpu(B):
    srv = B.eigcg_server_create(0)
    t = ctypes.c_uint64()
    assert B.LIB.eigcg_submit(srv, 0, ctypes.c_void_p(8), ctypes.c_void_p(8), 1e-10,
                              ctypes.byref(t)) == B.EIGCG_EINVAL
    assert B.LIB.eigcg_poll(srv, 12345, None) == B.EIGCG_EINVAL
    assert B.eigcg_server_destroy(srv) == B.EIGCG_OK


def _herm(rng, n):
    a = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return a + a.conj().T


def _check_eig(B, a, k, tol=1e-12):
    w, z = B.eigcg_host_eig_lowest(a, k)
    w0 = np.linalg.eigvalsh(a)
    scale = max(1.0, np.max(np.abs(w0)))
    assert np.max(np.abs(w - w0)) <= tol * scale
    assert np.max(np.abs(a @ z - z * w[:k])) <= 10 * tol * scale
    assert np.max(np.abs(z.conj().T @ z - np.eye(k))) <= 1e-12


def test_host_eig_dense_tridiagonal_arrowhead_clustered(B):
    rng = np.random.default_rng(0)
    _check_eig(B, _herm(rng, 60), 10)
    _check_eig(B, _herm(rng, 7), 7)
    # real symmetric tridiagonal (a window before its first restart)
    d = rng.uniform(0.1, 60, 100)
    e = -rng.uniform(0.01, 5, 99)
    _check_eig(B, (np.diag(d) + np.diag(e, 1) + np.diag(e, -1)).astype(complex), 10)
    # restarted window: diagonal block, complex arrow row, tridiagonal tail
    m, b = 100, 20
    T = np.zeros((m, m), dtype=complex)
    T[np.arange(b), np.arange(b)] = np.sort(rng.uniform(0.001, 1, b))
    T[b, :b] = rng.standard_normal(b) + 1j * rng.standard_normal(b)
    T[:b, b] = T[b, :b].conj()
    for i in range(b, m):
        T[i, i] = rng.uniform(0.5, 50)
        if i + 1 < m:
            T[i, i + 1] = T[i + 1, i] = -rng.uniform(0.1, 3)
    _check_eig(B, T, 10)
    # clustered and exactly repeated eigenvalues
    Q, _ = np.linalg.qr(rng.standard_normal((9, 9)) + 1j * rng.standard_normal((9, 9)))
    lam = np.array([1.0, 1.0, 1.0 + 1e-14, 2.0, 2.0, 3.0, 4.0, 4.0 + 1e-9, 5.0])
    a = Q @ np.diag(lam) @ Q.conj().T
    _check_eig(B, 0.5 * (a + a.conj().T), 9)


def test_host_qr_and_cholesky(B):
    rng = np.random.default_rng(1)
    a = rng.standard_normal((50, 20)) + 1j * rng.standard_normal((50, 20))
    q, r = B.eigcg_host_qr(a)
    assert np.max(np.abs(q @ r - a)) < 1e-13
    assert np.max(np.abs(q.conj().T @ q - np.eye(20))) < 1e-14
    assert np.allclose(np.tril(r, -1), 0)
    h = a.conj().T @ a + np.eye(20)
    bb = rng.standard_normal((20, 3)) + 1j * rng.standard_normal((20, 3))
    x = B.eigcg_host_chol_solve(h, bb)
    assert np.max(np.abs(h @ x - bb)) < 1e-12
    with pytest.raises(B.EigcgError):
        B.eigcg_host_chol_solve(-np.eye(3, dtype=complex), np.ones(3, dtype=complex))


def test_auto_switch_rule_cases(B):
    f = B.eigcg_host_auto_continue
    # no bank room, or nothing left to gain from: init-CG
    assert not f([], [], 5, 1.0, 0)
    assert not f([900.0, 800.0, 700.0], [1.5, 1.3, 1.2], 1, 1.0, 10)
    # fewer than three eigCG groups: the drop is not measured yet, keep growing
    assert f([], [], 5, 1.0, 10)
    assert f([900.0, 950.0], [1.5, 1.5], 5, 1.0, 10)
    # no mean drop over the last groups: stop
    assert not f([700.0, 720.0, 700.0], [1.0, 1.0, 1.0], 20, 1.0, 10)
    # mean drop 100 iterations; overhead 0.2 s against (left - 1) * 0.1 s saved
    assert f([1000.0, 900.0, 800.0], [1.0, 1.0, 1.0], 4, 1.0, 10)      # 0.2 < 0.3
    assert not f([1000.0, 900.0, 800.0], [1.0, 1.0, 1.0], 2, 1.0, 10)  # 0.2 > 0.1
    # the drop is the mean over the last three groups: one noisy pair does not end it
    assert f([1000.0, 850.0, 700.0, 710.0], [1.0, 1.0, 1.0, 0.9], 20, 1.0, 10)
    # a history without times is refused
    rc = B.LIB.eigcg_host_auto_continue(1, 3, None, None, 1.0, 1)
    assert rc == B.EIGCG_EINVAL


def _model(k, n1=1000.0, ninf=160.0, tau=4.0):
    """Iterations of the k-th right-hand side (1-based) after k - 1 eigCG solves."""
    return ninf + (n1 - ninf) * np.exp(-(k - 1) / tau)


def test_auto_switch_grows_with_the_number_of_rhs(B):
    """Section 5.5's observation, on a model of its shape: iterations decay
    with each eigCG solve towards a floor, an eigCG solve costs its
    iterations plus a 30 % overhead plus a bank update growing with the bank.
    The rule's plan (decided one right-hand side at a time from the measured
    history) never runs eigCG for every right-hand side, runs more of them for
    longer sequences, and costs within 5 % of the best fixed number of eigCG
    solves of the same model, also with a 4 % spread of iteration counts
    between right-hand sides."""
    iter_ms = 1.0

    def eig_secs(k):
        return (1.3 * _model(k) + 20.0 * k) * iter_ms * 1e-3

    def total(s, keig):
        t = sum(eig_secs(k) for k in range(1, keig + 1))
        return t + (s - keig) * _model(keig + 1) * iter_ms * 1e-3

    chosen = []
    for s in (6, 12, 24, 32, 48):
        iters, secs = [], []
        for k in range(1, s + 1):
            if not B.eigcg_host_auto_continue(iters, secs, s - k + 1, iter_ms, 100):
                break
            iters.append(_model(k))
            secs.append(eig_secs(k))
        keig = len(iters)
        best = min(total(s, q) for q in range(0, s + 1))
        assert 3 <= keig < s
        assert total(s, keig) <= 1.05 * best, (s, keig)
        chosen.append(keig)
    assert chosen == sorted(chosen) and chosen[-1] > chosen[0], chosen
    rng = np.random.default_rng(1)
    for s in (24, 48):
        best = min(total(s, q) for q in range(0, s + 1))
        for rep in range(10):
            iters, secs = [], []
            for k in range(1, s + 1):
                if not B.eigcg_host_auto_continue(iters, secs, s - k + 1, iter_ms, 100):
                    break
                n = _model(k) * (1.0 + 0.04 * rng.standard_normal())
                iters.append(n)
                secs.append((1.3 * n + 20.0 * k) * iter_ms * 1e-3)
            assert total(s, len(iters)) <= 1.05 * best, (s, len(iters))


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus N > 1 exits with a message before
    touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_auto_switch_against_the_papers_table(B):
    """Section 5.5 tabulates the best number of Incremental eigCG solves for
    6 to 48 right-hand sides (tests/golden).  The rule, run on the model of the
    paper's iteration decay used above, picks counts within a factor of two of
    the table's and growing with the number of right-hand sides like it."""
    import json
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "golden", "optimal_incremental_eigcg_rhs.json")) as f:
        table = json.load(f)
    iter_ms = 1.0

    def eig_secs(k):
        return (1.3 * _model(k) + 20.0 * k) * iter_ms * 1e-3

    chosen = []
    for s in table["total_rhs"]:
        iters, secs = [], []
        for k in range(1, s + 1):
            if not B.eigcg_host_auto_continue(iters, secs, s - k + 1, iter_ms, 100):
                break
            iters.append(_model(k))
            secs.append(eig_secs(k))
        chosen.append(len(iters))
    for got, paper in zip(chosen, table["optimal_incremental_rhs"]):
        assert paper / 2 <= got <= 2 * paper, (chosen, table)
    assert chosen == sorted(chosen) and chosen[-1] > chosen[0]


class _FakeDeviceTensor:
    """Stands in for a complex128 device tensor in the binding's argument
    checks; the checks must refuse it before any library call reads its
    (invalid) data pointer."""

    def __init__(self, *shape):
        import torch
        self.shape = tuple(shape)
        self.is_cuda = True
        self.dtype = torch.complex128

    def is_contiguous(self):
        return True

    def dim(self):
        return len(self.shape)

    def numel(self):
        return int(np.prod(self.shape))

    def data_ptr(self):
        raise AssertionError("a mis-sized tensor reached the library")


def test_binding_refuses_mis_sized_tensors(B):
    """Every entry point taking device fields checks their sizes against the
    context's lattice before calling the C ABI (which takes raw pointers)."""
    F = _FakeDeviceTensor
    full = ctypes.c_void_p(0x7e57)      # 4^4 lattice, full geometry
    eo = ctypes.c_void_p(0x7e58)        # 4^4 lattice, odd-even (128 even sites)
    B._GEOM[full.value] = (256, 256)
    B._GEOM[eo.value] = (128, 256)
    try:
        good = (1, 4, 4, 4, 4, 4, 3)
        bad_cases = [
            (B.eigcg_solve, (full, F(*good), F(1, 4, 4, 4, 4, 4, 2), 1e-10)),   # x too small
            (B.eigcg_solve, (full, F(2, 4, 4, 4, 4, 4, 3), F(*good), 1e-10)),   # x misses a column
            (B.eigcg_solve, (full, F(1, 4, 4, 4, 2, 4, 3), F(1, 4, 4, 4, 2, 4, 3), 1e-10)),
            (B.eigcg_solve, (eo, F(*good), F(*good), 1e-10)),                   # full fields, even system
            (B.eigcg_deflate_init, (full, F(*good), F(1, 3072 - 1))),
            (B.eigcg_solve_bicgstab, (full, F(*good), F(1, 4, 4, 4, 4, 4, 4), 1e-10)),
            (B.eigcg_apply, (full, 0, F(*good), F(1, 4, 4, 4, 4, 3, 3))),
            (B.eigcg_schur_rhs, (eo, F(*good), F(*good))),                      # rhs is half size
            (B.eigcg_schur_rhs, (eo, F(1, 128, 4, 3), F(1, 128, 4, 3))),        # b_full is full size
            (B.eigcg_schur_reconstruct, (eo, F(*good), F(1, 128, 4, 3), F(1, 128, 4, 3))),
            (B.eigcg_bank_load, (full, F(3, 255, 4, 3))),
            (B.eigcg_bank_vectors, (full, 0, 2, F(*good))),
            (B.eigcg_bank_restore, (full, F(2, 256, 4, 3), np.eye(3))),
            (B.eigcg_solve, (ctypes.c_void_p(0x7e59), F(*good), F(*good), 1e-10)),  # unknown ctx
        ]
        for fn, args in bad_cases:
            with pytest.raises(ValueError):
                fn(*args)
        # a gauge field of the wrong lattice is refused before create
        p = B.eigcg_default_params(dims=(4, 4, 4, 4))
        with pytest.raises(ValueError):
            B.eigcg_create(p, F(4, 4, 4, 4, 4, 3, 2))
        # a server request for a field it does not hold, or of the wrong size
        srv = B.eigcg_server_create(0)
        try:
            B._SERVERS[srv.value] = {0: (256, 256)}
            with pytest.raises(ValueError):
                B.eigcg_submit(srv, 1, F(*good), F(*good), 1e-10)
            with pytest.raises(ValueError):
                B.eigcg_submit(srv, 0, F(1, 4, 4, 4, 4, 4, 2), F(*good), 1e-10)
        finally:
            B.eigcg_server_destroy(srv)
    finally:
        B._GEOM.pop(full.value, None)
        B._GEOM.pop(eo.value, None)


def test_bounds_layer_refuses_accesses_past_an_allocation(B):
    """The library's host-side bounds layer (every device allocation
    registered with its size; column pointers and the fields of a launch
    checked before enqueueing): an access must end inside the allocation it
    starts in.  Fake addresses, never dereferenced."""
    base, size = 0x5e0000000000, 12 * 4096
    nxt = base + size + 256                      # the next allocation
    assert B.eigcg_debug_span(0, base, size) == B.EIGCG_OK
    assert B.eigcg_debug_span(0, nxt, size) == B.EIGCG_OK
    try:
        field = 4096
        for k in range(1, 13):                   # fields 0..11 of 12 fit
            assert B.eigcg_debug_span(2, base, k * field) == B.EIGCG_OK
        assert B.eigcg_debug_span(2, base, 13 * field) == B.EIGCG_EINVAL
        # a column pointer inside the allocation, checked from where it starts
        assert B.eigcg_debug_span(2, base + 11 * field, field) == B.EIGCG_OK
        assert B.eigcg_debug_span(2, base + 11 * field, field + 1) == B.EIGCG_EINVAL
        # 16 columns in a 1-column workspace: refused, although the overrun
        # would land in the next allocation
        assert B.eigcg_debug_span(2, nxt, 16 * size) == B.EIGCG_EINVAL
        # memory the library did not allocate (the caller's tensors) is not checked
        assert B.eigcg_debug_span(2, nxt + 2 * size, 1 << 40) == B.EIGCG_OK
        assert B.eigcg_debug_span(2, base - 64, 128) == B.EIGCG_OK
    finally:
        assert B.eigcg_debug_span(1, base) == B.EIGCG_OK
        assert B.eigcg_debug_span(1, nxt) == B.EIGCG_OK
    assert B.eigcg_debug_span(1, base) == B.EIGCG_EINVAL  # already removed


def _restart_inputs(seed):
    rng = np.random.default_rng(seed)
    l = int(rng.integers(2, 40))
    theta = np.sort(np.concatenate([10.0 ** rng.uniform(-4, -2, l // 3),
                                    10.0 ** rng.uniform(-1, 0.5, l - l // 3)]))
    res = 10.0 ** rng.uniform(-10, -1, l)
    return theta, res, float(rng.uniform(20, 80)), 10.0 ** -rng.uniform(6, 12), float(rng.uniform(0, 60))


@pytest.mark.parametrize("seed", range(24))
def test_restart_model_matches_oracle(B, seed):
    """The library's dynamic restart threshold (host logic) against the
    oracle's cost model on seeded inputs: same threshold and predicted
    iteration counts to rounding."""
    from oracle.restart_model import choose_restart
    theta, res, lam_max, tol, cost = _restart_inputs(seed)
    want = choose_restart(theta, res, lam_max, tol, cost)
    got = B.eigcg_restart_model(theta, res, lam_max, tol, cost)
    assert (got[0] == 0.0) == (want[0] == 0.0)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=0.0)


def test_restart_model_closed_forms_and_errors(B):
    """One separated cluster of three accurate Ritz pairs: tau = sqrt(tol);
    exact eigenvectors or a prohibitive restart cost: no restart; unsorted,
    non-positive or non-finite inputs: EINVAL."""
    theta = np.array([1e-3, 2e-3, 3e-3, 1.0, 1.1, 1.2])
    res = np.array([1e-7] * 3 + [0.3] * 3)
    tau, c0, c1 = B.eigcg_restart_model(theta, res, 60.0, 1e-10, 7.0)
    assert tau == pytest.approx(1e-5, rel=1e-12) and c1 < c0
    assert B.eigcg_restart_model(theta, np.zeros(6), 60.0, 1e-10, 7.0)[0] == 0.0
    assert B.eigcg_restart_model(theta, res, 60.0, 1e-10, 1e6)[0] == 0.0
    assert B.eigcg_restart_model(theta[:0], res[:0], 60.0, 1e-10, 7.0) == (0.0, 0.0, 0.0)
    for th, rs, lm, tl in [(theta[::-1], res, 60.0, 1e-10), (theta - 1.0, res, 60.0, 1e-10),
                           (theta, -res, 60.0, 1e-10), (theta, res, float("nan"), 1e-10),
                           (theta, res, 60.0, 0.0), (theta, res, 60.0, 1.0)]:
        with pytest.raises(B.EigcgError):
            B.eigcg_restart_model(th, rs, lm, tl, 7.0)
