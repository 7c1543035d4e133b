"""Pins of the oracle's bank locking (Section 4's discussion; CPU only).

Checked against what locking must preserve: the Ritz values of the bank, an
orthonormal U, H equal to U^H A U except in the skipped entries, which stay
within the locked vectors' residual norms (Cauchy-Schwarz), and the deflation
the bank gives.
"""

import numpy as np
import pytest

from oracle.dirac import WilsonOperator
from oracle.eigcg import eigcg
from oracle.incremental import extend_bank, incremental_eigcg, orthonormalize_against
from oracle.initcg import init_cg
from oracle.locking import extend_bank_locked, lock_bank
from synthetic import gaussian_rhs

DIMS = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def grown(cfg0_field):
    op = WilsonOperator(cfg0_field, -0.2)
    rhs = [gaussian_rhs(DIMS, 2000 + i).reshape(-1) for i in range(3)]
    _, U, H, _ = incremental_eigcg(op.A, rhs, 8, 24, tol=1e-7)
    # Ritz vectors of one more eigCG solve, for the extensions below
    _, V, _, _ = eigcg(op.A, gaussian_rhs(DIMS, 2100).reshape(-1), 8, 24, tol=1e-7)
    return op, U, H, V


def _explicit_H(op, U):
    AU = np.stack([op.A(U[:, j]) for j in range(U.shape[1])], axis=1)
    return U.conj().T @ AU


def test_lock_rotates_and_locks(grown):
    op, U, H, _ = grown
    tol = 1e-6
    Ul, Hl, nl, theta, res = lock_bank(op.A, U, H, 0, tol)
    assert 0 < nl < U.shape[1]
    assert np.all(res[:nl] <= tol) and np.all(res[nl:] > tol)
    np.testing.assert_allclose(np.sort(theta), np.linalg.eigvalsh(H), rtol=1e-10, atol=1e-14)
    assert np.max(np.abs(Ul.conj().T @ Ul - np.eye(U.shape[1]))) < 1e-12
    assert np.max(np.abs(Hl - np.diag(theta))) == 0.0
    assert np.max(np.abs(_explicit_H(op, Ul) - Hl)) < 1e-12 * np.max(theta)
    # locking again locks nothing new and keeps the locked block
    U2, H2, nl2, _, res2 = lock_bank(op.A, Ul, Hl, nl, tol)
    assert nl2 == nl and np.all(res2 > tol)
    np.testing.assert_array_equal(U2[:, :nl], Ul[:, :nl])


def test_extension_skips_only_locked_entries_within_their_residuals(grown):
    op, U, H, V = grown
    tol = 1e-6
    Ul, Hl, nl, theta, res = lock_bank(op.A, U, H, 0, tol)
    Vbar = orthonormalize_against(Ul, V)
    Ue, He = extend_bank_locked(op.A, Ul, Hl, Vbar, nl)
    exact = _explicit_H(op, Ue)
    l = Ul.shape[1]
    diff = np.abs(He - exact)
    skipped = np.abs(exact[:nl, l:])
    assert np.all(He[:nl, l:] == 0.0) and np.all(He[l:, :nl] == 0.0)
    # the skipped entries are u^H A v = r^H v, at most ||r|| each, and not all zero
    assert np.all(skipped <= res[:nl, None] * (1 + 1e-8) + 1e-15)
    assert np.max(skipped) > 1e-3 * np.max(res[:nl])
    mask = np.ones_like(diff, dtype=bool)
    mask[:nl, l:] = False
    mask[l:, :nl] = False
    assert np.max(diff[mask]) < 1e-12 * np.max(theta)


def test_nothing_locked_is_the_plain_update(grown):
    op, U, H, V = grown
    Vbar = orthonormalize_against(U, V)
    Ua, Ha = extend_bank(op.A, U, H, Vbar)
    Ub, Hb = extend_bank_locked(op.A, U, H, Vbar, 0)
    np.testing.assert_array_equal(Ua, Ub)
    np.testing.assert_array_equal(Ha, Hb)
    _, _, nl, _, _ = lock_bank(op.A, U, H, 0, 0.0)
    assert nl == 0


def test_locked_bank_deflates_alike(grown):
    """Restarted init-CG (Section 5.3, restart at 1e-5) with the locked and
    extended bank needs the iterations of the same vectors with the exact H,
    within two."""
    op, U, H, V = grown
    Ul, Hl, nl, _, _ = lock_bank(op.A, U, H, 0, 1e-6)
    Vbar = orthonormalize_against(Ul, V)
    Ue, He = extend_bank_locked(op.A, Ul, Hl, Vbar, nl)
    exact = _explicit_H(op, Ue)
    exact = 0.5 * (exact + exact.conj().T)
    b = gaussian_rhs(DIMS, 3000).reshape(-1)
    _, ia = init_cg(op.A, Ue, He, b, tol=1e-10, restart_tol=1e-5)
    _, ib = init_cg(op.A, Ue, exact, b, tol=1e-10, restart_tol=1e-5)
    assert ia["converged"] and ib["converged"]
    assert abs(ia["iterations"] - ib["iterations"]) <= 2
