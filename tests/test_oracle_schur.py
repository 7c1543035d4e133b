"""Pins of the oracle's odd-even (Schur complement) operator (CPU only).

What fixes it independently of its own code:
* block elimination of the brute-force site-loop Wilson matrix (numpy.linalg
  on the dense even/odd blocks, no stencil involved);
* the closed-form free-field spectrum of Ahat = Mhat^H Mhat;
* the full system: the reconstructed solution solves M x = b and equals the
  dense solve of M;
* adjointness, gamma5-Hermiticity and positivity; gauge invariance of the
  spectrum;
* CG on the halved system reaches the full system's solution in fewer
  iterations (the reason the paper's runs use it).
"""

import itertools

import numpy as np
import pytest

from oracle import dirac
from oracle.cg import cg
from oracle.dense import dense_matrix
from oracle.dirac import WilsonOperator
from oracle.schur import SchurOperator
from synthetic import gauge_field, gaussian_half_rhs, gaussian_rhs, random_su3_sites, \
    unit_gauge_field

from _bruteforce import site_index, wilson_dense


def _parity_dofs(dims, parity):
    """Row indices (12 per site) of the sites of one parity, lexicographic."""
    sites = [site_index(c, dims) for c in itertools.product(*(range(L) for L in dims))
             if sum(c) % 2 == parity]
    sites.sort()
    return np.array([12 * s + k for s in sites for k in range(12)])


def test_schur_equals_block_elimination_of_bruteforce_matrix():
    dims = (4, 2, 2, 4)
    mass = -0.3
    U = gauge_field(dims, 0.6, 31)
    M = wilson_dense(U, mass, dirac.GAMMA, dims)
    e, o = _parity_dofs(dims, 0), _parity_dofs(dims, 1)
    # the hopping term couples opposite parities only: diagonal blocks are (4 + m) I
    assert np.max(np.abs(M[np.ix_(o, o)] - (4.0 + mass) * np.eye(len(o)))) == 0.0
    schur = M[np.ix_(e, e)] - M[np.ix_(e, o)] @ np.linalg.solve(M[np.ix_(o, o)], M[np.ix_(o, e)])
    op = SchurOperator(U, mass)
    Mhat = dense_matrix(op.Mhat, op.n)
    assert np.max(np.abs(Mhat - schur)) < 1e-13
    Mhat_dag = dense_matrix(op.Mhat_dag, op.n)
    assert np.max(np.abs(Mhat_dag - schur.conj().T)) < 1e-13


def _free_schur_spectrum(dims, mass):
    """Closed form (derived): with unit links D e^{ipx} chi = 2 (C - i g.s) e^{ipx} chi,
    C = sum cos p_mu, g.s = sum gamma_mu sin p_mu, (g.s)^2 = s^2.  D_eo D_oe is D^2
    restricted to the even sites, so Mhat(p) = a + b g.s with
    a = d - (C^2 - s^2) / d, b = 2 i C / d, a normal matrix whose Mhat^H Mhat has
    the eigenvalue a^2 + 4 C^2 s^2 / d^2.  On the even sites p and p + (pi, pi, pi, pi)
    are the same mode, so each of the V momenta carries multiplicity 12 / 2."""
    d = 4.0 + mass
    lams = []
    for k in itertools.product(*(range(L) for L in dims)):
        p = [2 * np.pi * k[mu] / dims[mu] for mu in range(4)]
        C = sum(np.cos(pm) for pm in p)
        s2 = sum(np.sin(pm) ** 2 for pm in p)
        a = d - (C * C - s2) / d
        lams.extend([a * a + 4.0 * C * C * s2 / (d * d)] * 6)
    return np.sort(np.array(lams))


def test_free_schur_spectrum():
    dims = (4, 4, 2, 4)
    mass = -0.2
    op = SchurOperator(unit_gauge_field(dims), mass)
    Mhat = dense_matrix(op.Mhat, op.n)
    lam = np.linalg.eigvalsh(Mhat.conj().T @ Mhat)
    expect = _free_schur_spectrum(dims, mass)
    assert np.max(np.abs(lam - expect)) < 1e-11
    # the same values follow from the full operator: |lambda(p)|^2 |lambda(p+pi)|^2 / d^2
    d = 4.0 + mass
    full = []
    for k in itertools.product(*(range(L) for L in dims)):
        p = np.array([2 * np.pi * k[mu] / dims[mu] for mu in range(4)])
        l1 = (d - np.cos(p).sum()) ** 2 + (np.sin(p) ** 2).sum()
        l2 = (d + np.cos(p).sum()) ** 2 + (np.sin(p) ** 2).sum()
        full.extend([l1 * l2 / (d * d)] * 6)
    assert np.max(np.abs(np.sort(full) - expect)) < 1e-11


def test_reconstructed_solution_solves_full_system(cfg0_field):
    mass = -0.2
    op = SchurOperator(cfg0_field, mass)
    full = WilsonOperator(cfg0_field, mass)
    b = gaussian_rhs((4, 4, 4, 4), 77).reshape(-1)
    Mhat = dense_matrix(op.Mhat, op.n)
    x_e = np.linalg.solve(Mhat, op.bhat(b))
    x = op.reconstruct(b, x_e)
    assert np.linalg.norm(full.M(x) - b) / np.linalg.norm(b) < 1e-13
    Mfull = dense_matrix(full.M, full.n)
    x_dense = np.linalg.solve(Mfull, b)
    assert np.max(np.abs(x - x_dense)) < 1e-12 * np.max(np.abs(x_dense))
    # x_e also solves the normal equations Ahat x_e = Mhat^H bhat
    r = op.A(x_e) - op.rhs(b)
    assert np.linalg.norm(r) < 1e-12 * np.linalg.norm(op.rhs(b))
    # split / join are inverse maps
    b_e, b_o = op.split(b)
    assert np.array_equal(op.join(b_e, b_o), b)


def test_adjoint_gamma5_and_positivity():
    dims = (4, 4, 2, 6)
    op = SchurOperator(gauge_field(dims, 0.5, 8), -0.45)
    u = gaussian_half_rhs(dims, 1).reshape(-1)
    v = gaussian_half_rhs(dims, 2).reshape(-1)
    lhs = np.vdot(u, op.Mhat(v))
    rhs = np.vdot(op.Mhat_dag(u), v)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    g5 = op.gamma5(op.Mhat(op.gamma5(v)))
    assert np.max(np.abs(g5 - op.Mhat_dag(v))) < 1e-12
    q = np.vdot(v, op.A(v))
    assert abs(q.imag) < 1e-10 * q.real and q.real > 0
    with pytest.raises(ValueError):
        SchurOperator(gauge_field((4, 4, 3, 4), 0.5, 8), -0.45)


def test_spectrum_gauge_invariant():
    dims = (4, 2, 2, 4)
    U = gauge_field(dims, 0.5, 12)
    G = random_su3_sites(dims, 5)
    Ug = np.empty_like(U)
    for mu in range(4):
        Gf = dirac.shift_forward(G, mu)
        Ug[..., mu, :, :] = G @ U[..., mu, :, :] @ np.conj(np.swapaxes(Gf, -1, -2))
    lam = []
    for links in (U, Ug):
        op = SchurOperator(links, -0.25)
        A = dense_matrix(op.A, op.n)
        lam.append(np.linalg.eigvalsh(A))
    assert np.max(np.abs(lam[0] - lam[1])) < 1e-11 * lam[0][-1]


def test_cg_on_halved_system_matches_full_solve():
    dims = (4, 4, 4, 8)
    mass = -0.35
    U = gauge_field(dims, 0.5, 3)
    op = SchurOperator(U, mass)
    full = WilsonOperator(U, mass)
    b = gaussian_rhs(dims, 9).reshape(-1)
    x_e, info = cg(op.A, op.rhs(b), tol=1e-11)
    x = op.reconstruct(b, x_e)
    assert np.linalg.norm(full.M(x) - b) / np.linalg.norm(b) < 1e-8
    x_f, info_f = cg(full.A, full.Mdag(b), tol=1e-11)
    assert np.max(np.abs(x - x_f)) < 1e-8 * np.max(np.abs(x_f))
    assert info["iterations"] < info_f["iterations"]
