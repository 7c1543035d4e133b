"""Pins of the oracle's Wilson operator (CPU only).

What fixes the operator independently of the oracle's code:
gamma-matrix algebra, the free-field plane-wave closed form, a brute-force
site-loop matrix, gamma5-Hermiticity (Section 1), positivity of A = M^H M,
gauge covariance, and the closed-form free spectrum of A.
"""

import itertools

import numpy as np
import pytest

from oracle import dirac
from oracle.dense import dense_matrix
from oracle.dirac import WilsonOperator
from synthetic import gauge_field, gaussian_rhs, random_su3_sites, unit_gauge_field

from _bruteforce import wilson_dense


def test_gamma_algebra():
    g = dirac.GAMMA
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            anti = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(anti, 2.0 * (mu == nu) * np.eye(4))
    # gamma5 is diagonal with entries +1, +1, -1, -1 and anticommutes with gamma_mu
    assert np.allclose(dirac.GAMMA5, np.diag([1, 1, -1, -1]))
    for mu in range(4):
        assert np.allclose(dirac.GAMMA5 @ g[mu], -g[mu] @ dirac.GAMMA5)


def _free_symbol(p, mass):
    """Closed form (derived): with unit links, M e^{ipx} chi =
    [(4 + m - sum cos p_mu) + i sum gamma_mu sin p_mu] e^{ipx} chi."""
    out = (4.0 + mass - sum(np.cos(p))) * np.eye(4, dtype=complex)
    for mu in range(4):
        out = out + 1j * np.sin(p[mu]) * dirac.GAMMA[mu]
    return out


@pytest.mark.parametrize("k", [(0, 0, 0, 0), (1, 0, 2, 3), (3, 5, 1, 7), (2, 3, 2, 4)])
def test_plane_wave(k):
    dims = (4, 6, 3, 8)
    mass = -0.37
    lx, ly, lz, lt = dims
    p = np.array([2 * np.pi * k[0] / lx, 2 * np.pi * k[1] / ly,
                  2 * np.pi * k[2] / lz, 2 * np.pi * k[3] / lt])
    rng = np.random.default_rng(5)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx),
                             indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    psi = phase[..., None, None] * chi
    U = unit_gauge_field(dims)
    out = dirac.apply_M(U, mass, psi)
    expect = phase[..., None, None] * (_free_symbol(p, mass) @ chi)
    assert np.max(np.abs(out - expect)) < 1e-12
    # the adjoint's symbol is the Hermitian conjugate
    outd = dirac.apply_Mdag(U, mass, psi)
    expectd = phase[..., None, None] * (_free_symbol(p, mass).conj().T @ chi)
    assert np.max(np.abs(outd - expectd)) < 1e-12


def test_stencil_equals_bruteforce_matrix():
    dims = (3, 2, 4, 3)
    U = gauge_field(dims, 0.7, 11)
    mass = 0.13
    op = WilsonOperator(U, mass)
    M_stencil = dense_matrix(op.M, op.n)
    M_brute = wilson_dense(U, mass, dirac.GAMMA, dims)
    assert np.max(np.abs(M_stencil - M_brute)) < 1e-13
    Mdag_stencil = dense_matrix(op.Mdag, op.n)
    assert np.max(np.abs(Mdag_stencil - M_brute.conj().T)) < 1e-13


def test_gamma5_hermiticity_and_positivity():
    dims = (4, 4, 4, 6)
    U = gauge_field(dims, 0.5, 3)
    op = WilsonOperator(U, -0.3)
    x = gaussian_rhs(dims, 1).reshape(-1)
    y = gaussian_rhs(dims, 2).reshape(-1)
    lhs = np.vdot(y, op.gamma5(op.M(op.gamma5(x))))
    rhs = np.vdot(op.M(y), x)
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)
    assert np.allclose(op.gamma5(op.M(op.gamma5(x))), op.Mdag(x), atol=1e-13)
    vav = np.vdot(x, op.A(x))
    mx = np.linalg.norm(op.M(x)) ** 2
    assert abs(vav.imag) < 1e-10 * mx
    assert abs(vav.real - mx) < 1e-11 * mx
    assert vav.real > 0


def test_gauge_covariance():
    """U_mu(x) -> G(x) U_mu(x) G(x+mu)^dag and psi -> G psi give M -> G M G^dag."""
    dims = (4, 4, 2, 6)
    U = gauge_field(dims, 0.5, 4)
    G = random_su3_sites(dims, 99)
    Ug = np.empty_like(U)
    for mu in range(4):
        Gfwd = dirac.shift_forward(G, mu)
        Ug[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(Gfwd, -1, -2))
    psi = gaussian_rhs(dims, 7)
    gpsi = np.einsum("...ab,...sb->...sa", G, psi)
    lhs = dirac.apply_M(Ug, -0.1, gpsi)
    rhs = np.einsum("...ab,...sb->...sa", G, dirac.apply_M(U, -0.1, psi))
    assert np.max(np.abs(lhs - rhs)) < 1e-12


def _free_spectrum(dims, mass):
    """Closed form (derived): lambda(p) = (m + sum(1 - cos p))^2 + sum sin^2 p,
    each with multiplicity 12."""
    lams = []
    for k in itertools.product(*(range(L) for L in dims)):
        p = [2 * np.pi * k[mu] / dims[mu] for mu in range(4)]
        a = mass + sum(1 - np.cos(pm) for pm in p)
        s = sum(np.sin(pm) ** 2 for pm in p)
        lams.extend([a * a + s] * 12)
    return np.sort(np.array(lams))


def test_free_spectrum_4444():
    dims = (4, 4, 4, 4)
    op = WilsonOperator(unit_gauge_field(dims), -0.2)
    M = dense_matrix(op.M, op.n)
    lam = np.linalg.eigvalsh(M.conj().T @ M)
    expect = _free_spectrum(dims, -0.2)
    assert np.max(np.abs(lam - expect)) < 1e-11
    distinct = np.unique(np.round(expect, 9))
    assert len(distinct) == 15
    assert abs(expect[0] - 0.04) < 1e-14 and abs(expect[-1] - 60.84) < 1e-12
    assert abs(expect[-1] / expect[0] - 1521.0) < 1e-8


def test_pure_gauge_has_free_spectrum():
    dims = (4, 2, 2, 4)
    G = random_su3_sites(dims, 21)
    U = np.empty(G.shape[:4] + (4, 3, 3), dtype=np.complex128)
    for mu in range(4):
        U[..., mu, :, :] = G @ np.conj(np.swapaxes(dirac.shift_forward(G, mu), -1, -2))
    op = WilsonOperator(U, -0.2)
    M = dense_matrix(op.M, op.n)
    lam = np.linalg.eigvalsh(M.conj().T @ M)
    assert np.max(np.abs(lam - _free_spectrum(dims, -0.2))) < 1e-11


def test_cfg0_spectrum_gauge_invariant_and_gamma5M(cfg0_field, cfg0_dense):
    """Random gauge transform leaves spec(A) unchanged; eig(A) = eig(gamma5 M)^2
    (the eigenvectors of A are those of gamma5 M, Section 1)."""
    U = cfg0_field
    G = random_su3_sites((4, 4, 4, 4), 77)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(
            np.swapaxes(dirac.shift_forward(G, mu), -1, -2))
    op_g = WilsonOperator(Ug, -0.2)
    Mg = dense_matrix(op_g.M, op_g.n)
    lam_g = np.linalg.eigvalsh(Mg.conj().T @ Mg)
    lam = cfg0_dense["lam"]
    assert np.max(np.abs(lam - lam_g)) < 1e-11 * lam[-1]
    g5 = np.kron(np.eye(256), np.kron(dirac.GAMMA5, np.eye(3)))
    h = g5 @ cfg0_dense["M"]
    assert np.max(np.abs(h - h.conj().T)) < 1e-13
    mu2 = np.sort(np.linalg.eigvalsh(h) ** 2)
    assert np.max(np.abs(mu2 - lam)) < 1e-11 * lam[-1]
    assert lam[0] > 0  # Hermitian positive definite
