"""GPU unit tests of the MFMA products against plain numpy products.

The complex tall-skinny products of the library (restart V (QZ), Ritz vectors,
U C, U^H R) run on the 16x16x4 matrix-core instructions; the lane-layout probe
pins the register layout they rely on, the products are then compared element
by element with numpy in FP64 (1e-13) and FP32 (1e-5, relative to the norms),
including the shapes of the bench's eigCG(10, 100) restart (K = 100 inputs,
2 nev = 20 outputs) and of deflation with a 240-vector bank (the tall product
splits its outputs into groups whose K x N coefficients fit 64 KB of LDS).
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0707_0131_amd import binding
    return binding


def test_mfma_lane_layout(B):
    out = B.eigcg_debug_mfma_probe()
    for base, name in [(0, "f64"), (512, "f32")]:
        got = {}
        for lane in range(64):
            for r in range(4):
                row = int(round(out[base + (lane * 4 + r) * 2])) - 1
                col = int(round(out[base + (lane * 4 + r) * 2 + 1])) - 1
                got[(lane, r)] = (row, col)
        if name == "f32":
            expect = {(l, r): (4 * (l // 16) + r, l % 16) for l in range(64) for r in range(4)}
        else:
            expect = {(l, r): (l // 16 + 4 * r, l % 16) for l in range(64) for r in range(4)}
        bad = [(k, got[k], expect[k]) for k in expect if got[k] != expect[k]]
        assert not bad, f"{name} layout differs, first: {bad[:6]}"


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,K,N", [(1000, 1, 1), (3072, 7, 5), (1024, 40, 20), (777, 33, 24),
                                   (6144, 100, 20), (5000, 240, 17), (4099, 240, 1)])
def test_gemm_tall(B, dt, n, K, N):
    import torch
    rng = np.random.default_rng(K * 100 + N)
    cdt = np.complex128 if dt == "c128" else np.complex64
    A = (rng.standard_normal((K, n)) + 1j * rng.standard_normal((K, n))).astype(cdt)
    S = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    out = B.eigcg_debug_gemm(0, torch.from_numpy(A).to("cuda:0"),
                             s=torch.from_numpy(S).to("cuda:0"))
    ref = (A.astype(np.complex128).T @ S).T
    tol = 1e-13 if dt == "c128" else 2e-6
    assert np.max(np.abs(out - ref)) <= tol * np.max(np.abs(ref)) * np.sqrt(K)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("kind", [2, 3])
@pytest.mark.parametrize("n,K,N", [(1000, 1, 1), (777, 33, 24), (6144, 100, 20), (4099, 240, 1),
                                   (5000, 9, 17)])
def test_gemm_tall_accumulate(B, dt, kind, n, K, N):
    """The beta = 1 epilogue: out += in S (kind 2, the init-CG lift of
    eq. (2.1)) and out -= in S (kind 3, the Gram-Schmidt update of Section 4),
    every old output value read before the tile's stores."""
    import torch
    rng = np.random.default_rng(K * 31 + N + kind)
    cdt = np.complex128 if dt == "c128" else np.complex64
    A = (rng.standard_normal((K, n)) + 1j * rng.standard_normal((K, n))).astype(cdt)
    S = rng.standard_normal((K, N)) + 1j * rng.standard_normal((K, N))
    O = (rng.standard_normal((N, n)) + 1j * rng.standard_normal((N, n))).astype(cdt)
    out = torch.from_numpy(O.copy()).to("cuda:0")
    got = B.eigcg_debug_gemm(kind, torch.from_numpy(A).to("cuda:0"),
                             s=torch.from_numpy(S).to("cuda:0"), out=out)
    prod = (A.astype(np.complex128).T @ S).T
    ref = O.astype(np.complex128) + (prod if kind == 2 else -prod)
    tol = 1e-13 if dt == "c128" else 2e-6
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)) * np.sqrt(K)


@pytest.mark.parametrize("dt", ["c128", "c64"])
@pytest.mark.parametrize("n,K,N", [(1000, 1, 1), (3072, 20, 1), (1024, 40, 12), (4097, 17, 16),
                                   (6144, 100, 1), (5000, 240, 16), (4099, 240, 1)])
def test_gemm_reduce(B, dt, n, K, N):
    import torch
    rng = np.random.default_rng(K * 7 + N)
    cdt = np.complex128 if dt == "c128" else np.complex64
    A = (rng.standard_normal((K, n)) + 1j * rng.standard_normal((K, n))).astype(cdt)
    R = (rng.standard_normal((N, n)) + 1j * rng.standard_normal((N, n))).astype(cdt)
    out = B.eigcg_debug_gemm(1, torch.from_numpy(A).to("cuda:0"),
                             r=torch.from_numpy(R).to("cuda:0"))
    ref = A.astype(np.complex128).conj() @ R.astype(np.complex128).T
    tol = 1e-13 if dt == "c128" else 2e-6
    assert np.max(np.abs(out - ref)) <= tol * np.sqrt(n) * 2


def test_tuning_choices_are_persisted(B, tmp_path, monkeypatch):
    """The stencil tuner writes its choice to the file named by
    EIGCG_TUNE_CACHE; a later process (here: after dropping this process's
    choices) takes the choice from the file instead of timing again."""
    import torch
    from synthetic import gauge_field
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("EIGCG_TUNE_CACHE", str(path))
    B.eigcg_tune_cache_reset()
    dims = (8, 8, 4, 8)
    U = torch.from_numpy(gauge_field(dims, 0.5, 11)).to("cuda:0")
    try:
        p = B.eigcg_default_params(dims=dims, mass=-0.2, max_bank=0, max_batch=3)
        ctx = B.eigcg_create(p, U)
        info = B.eigcg_layout_info(ctx)
        B.eigcg_destroy(ctx)
        lines = path.read_text().splitlines()
        assert len(lines) == 1
        key, val = lines[0].split(" : ")
        fields = val.split()
        assert int(fields[0]) == info["variant64"]
        assert len(fields) == 2 + B.STENCIL_VARIANTS
        # another choice in the file (variant 3, one column per workgroup) is
        # what a fresh process takes
        forced = [3, 1] + [float(v) for v in fields[2:]]
        path.write_text(key + " : " + " ".join(str(v) for v in forced) + "\n")
        B.eigcg_tune_cache_reset()
        ctx = B.eigcg_create(p, U)
        info2 = B.eigcg_layout_info(ctx)
        B.eigcg_destroy(ctx)
        assert info2["variant64"] == 3 and info2["cols_per_group64"] == 1
        assert info2["tune_ms64"] == pytest.approx([float(v) for v in fields[2:]], rel=1e-5)
        assert len(path.read_text().splitlines()) == 1  # nothing re-timed
    finally:
        B.eigcg_tune_cache_reset()
