"""Pins of the oracle's dynamic init-CG restart threshold (CPU only).

The rule is a cost model (the paper leaves a dynamic threshold open at the end
of Section 5.3).  It is pinned by what does not depend on it: the CG bound with
outlying eigenvalues against CG on diagonal matrices, closed-form choices, a
brute-force minimisation of the stated cost, and on the 4^4 test lattice the
iteration counts of restarted init-CG over a sweep of thresholds.
"""

import math

import numpy as np
import pytest

from oracle.cg import cg
from oracle.dirac import WilsonOperator
from oracle.incremental import bank_ritz, incremental_eigcg
from oracle.initcg import init_cg
from oracle.restart_model import (bulk_start, choose_restart, contamination_levels, leg_cost,
                                  outlier_bound)
from synthetic import gaussian_rhs


def _energy_reduction(d, b, k):
    """||e_k||_A / ||e_0||_A of CG on diag(d) after k iterations from x = 0."""
    x, _ = cg(lambda v: d * v, b, tol=0.0, max_iter=k, true_residual_restarts=0)
    xs = b / d
    e0, ek = xs, xs - x
    return math.sqrt(np.real(np.vdot(ek * d, ek)) / np.real(np.vdot(e0 * d, e0)))


@pytest.mark.parametrize("outliers", [(), (1e-4,), (1e-4, 3e-3)])
def test_outlier_bound_holds_for_cg(outliers):
    """After the bound's iteration count, CG on a diagonal matrix with a bulk
    in [1, 100] and the given outliers has reduced the energy norm of the
    error by at least f."""
    rng = np.random.default_rng(5)
    d = np.concatenate([np.linspace(1.0, 100.0, 300), np.array(outliers)])
    b = rng.standard_normal(d.size) + 1j * rng.standard_normal(d.size)
    for f in (1e-3, 1e-8):
        k = math.ceil(outlier_bound(f, 100.0, 1.0, outliers))
        assert _energy_reduction(d, b, k) <= f


def test_outlier_term_is_needed():
    """Two outliers at 1e-4 and 3e-3 cost CG more iterations than the bulk
    alone: the bound without its outlier terms would be violated."""
    rng = np.random.default_rng(6)
    d = np.concatenate([np.linspace(1.0, 100.0, 300), [1e-4, 3e-3]])
    b = rng.standard_normal(d.size) + 1j * rng.standard_normal(d.size)
    k0 = math.ceil(outlier_bound(1e-8, 100.0, 1.0, ()))
    assert _energy_reduction(d, b, k0) > 1e-8


def _cluster(res_low):
    theta = np.array([1e-3, 2e-3, 3e-3, 1.0, 1.1, 1.2])
    res = np.array([res_low] * 3 + [0.3] * 3)
    return theta, res


def test_contamination_levels_closed_form():
    theta, res = _cluster(1e-7)
    s = contamination_levels(theta, res, 60.0)
    assert s[0] == 0.0
    assert s[1] == pytest.approx(1e-7 / 60.0, rel=1e-14)
    assert s[3] == pytest.approx(math.sqrt(3) * 1e-7 / 60.0, rel=1e-14)
    assert s[5] == pytest.approx(math.sqrt(3 * 1e-14 + 2 * 0.09) / 60.0, rel=1e-14)
    # the three low pairs are resolved (Davis-Kahan bound below one), the
    # bulk pairs with residual 0.3 and gaps 0.1 are not
    assert bulk_start(theta, res) == 4
    assert bulk_start(theta, np.full(6, 0.9)) == 1


def test_exact_eigenvectors_never_restart():
    theta, res = _cluster(0.0)
    res[3:] = 0.0
    tau, c0, c1 = choose_restart(theta, res, 60.0, 1e-10, 5.0)
    assert tau == 0.0 and c1 == c0
    # nothing is contaminated: the whole bank is deflated, kappa = 60 / 1.2
    assert c0 == pytest.approx(0.5 * math.sqrt(60.0 / 1.2) * math.log(2e10), rel=1e-14)


def test_separated_cluster_restarts_at_sqrt_tol():
    """Three accurate low Ritz pairs well below an unresolved bulk: one restart
    anywhere in [s_3, tol/s_3] keeps both legs clean, so tau is the midpoint
    sqrt(tol) and the cost is R plus the clean two-leg cost."""
    theta, res = _cluster(1e-7)
    lam_max, tol, R = 60.0, 1e-10, 7.0
    tau, c0, c1 = choose_restart(theta, res, lam_max, tol, R)
    assert tau == pytest.approx(1e-5, rel=1e-12)
    assert c1 == pytest.approx(R + 0.5 * math.sqrt(lam_max / 1.0) * math.log(4.0 / tol), rel=1e-13)
    # no restart: the three directions resurface (tol < s_3)
    extra = sum(math.log(lam_max / t - 1.0) for t in theta[:3])
    assert c0 == pytest.approx(3 + 0.5 * math.sqrt(lam_max) * (math.log(2.0 / tol) + extra),
                               rel=1e-13)


def test_large_restart_cost_never_restarts():
    theta, res = _cluster(1e-7)
    tau, c0, c1 = choose_restart(theta, res, 60.0, 1e-10, 1e6)
    assert tau == 0.0 and c1 == c0


@pytest.mark.parametrize("seed", range(6))
def test_choice_minimises_the_stated_cost(seed):
    """Brute force over a fine grid of tau: no grid point beats the choice,
    and the chosen tau attains the reported cost."""
    rng = np.random.default_rng(seed)
    l = int(rng.integers(2, 12))
    theta = np.sort(np.concatenate([10.0 ** rng.uniform(-4, -2, l // 2),
                                    10.0 ** rng.uniform(-0.5, 0.5, l - l // 2)]))
    res = 10.0 ** rng.uniform(-9, -2, l)
    lam_max, tol, R = 60.0, 1e-10, float(rng.uniform(0, 40))
    tau, c0, c1 = choose_restart(theta, res, lam_max, tol, R)
    s = contamination_levels(theta, res, lam_max)
    b = bulk_start(theta, res)

    def cost(t):
        return leg_cost(t, theta, s, b, lam_max) + R + leg_cost(tol / t, theta, s, b, lam_max)

    grid = np.exp(np.linspace(math.log(tol), 0.0, 2001))[1:-1]
    best = min(min(cost(t) for t in grid), c0)
    assert c1 <= best + 1e-9 * best
    if tau > 0:
        assert cost(tau) == pytest.approx(c1, rel=1e-12)
        assert c1 < c0


@pytest.mark.slow
def test_model_threshold_on_lattice(cfg0_field):
    """4^4 lattice (kappa about 1.2e5, twelve near-zero modes): a bank grown by
    Incremental eigCG(8, 24) on four right-hand sides to 1e-7, then init-CG on
    a fifth to 1e-10.  The model's threshold is within three iterations of the
    best of a sweep and needs less than half the iterations of no restart."""
    op = WilsonOperator(cfg0_field, -0.2)
    rhs = [gaussian_rhs((4, 4, 4, 4), 2000 + i).reshape(-1) for i in range(4)]
    _, U, H, _ = incremental_eigcg(op.A, rhs, 8, 24, tol=1e-7)
    theta, res = bank_ritz(op.A, U, H)
    tau, _, _ = choose_restart(theta, res, (8.0 + 0.2) ** 2, 1e-10, 6.0)
    assert 0.0 < tau < 1.0
    b = gaussian_rhs((4, 4, 4, 4), 3000).reshape(-1)
    _, i_none = init_cg(op.A, U, H, b, tol=1e-10)
    _, i_tau = init_cg(op.A, U, H, b, tol=1e-10, restart_tol=tau)
    sweep = [init_cg(op.A, U, H, b, tol=1e-10, restart_tol=t)[1]["iterations"]
             for t in (1e-2, 1e-3, 1e-4, 1e-6, 1e-7, 1e-8)]
    assert i_tau["converged"] and i_tau["restarted"]
    assert i_tau["iterations"] <= min(sweep) + 3
    assert i_tau["iterations"] < 0.5 * i_none["iterations"]
