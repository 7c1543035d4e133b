"""A dynamic init-CG restart threshold (test infrastructure only).

Section 5.3 restarts init-CG once, near machine precision scaled by the norm
of A, and remarks that the threshold could instead be chosen at run time from
the computed eigenvalues and their residual norms, trading the lower
condition number that re-deflation restores against the cost of restarting;
the paper leaves the rule open.  This module writes out the rule the library
takes, as a cost model in four steps.

1. Contamination.  For the ``k`` lowest Ritz pairs ``(theta_j, u_j)`` of the
   bank, with residuals ``R_k = [A u_j - theta_j u_j]``, the sine of the angle
   between ``span(u_1..u_k)`` and the true invariant subspace lies between
   ``||R_k|| / lambda_max`` and ``||R_k|| / gap_k`` (the second is the
   Davis-Kahan sin-Theta bound, the gap to the rest of the spectrum estimated
   by ``theta_{k+1} - theta_k``).  After a Galerkin projection (eq. (2.1))
   the residual keeps components along those eigenvectors of at most that
   angle relative to the projected residual, usually far less because the
   error of a Ritz vector spreads over the whole spectrum; they reappear once
   CG has reduced the residual that far.  Reading: the model takes the lower
   end, ``s_k = ||R_k||_F / lambda_max`` (``s_0 = 0``), which is also Section
   5.3's observation that Ritz vectors keep deflating until the linear
   residual reaches their own residual norm scaled by the norm of A.
2. Bulk.  The span of the ``k`` lowest is resolved when its Davis-Kahan
   bound ``d_k = ||R_k||_F / gap_k`` is below one; the bank separates its
   lowest ``b-1`` Ritz values from the rest, ``b = 1 + max{k : d_k < 1}``
   (``b = 1`` if none), so deflation leaves the condition number
   ``kappa = lambda_max / theta_b``.
3. Leg cost.  A CG leg that starts right after a projection and reduces the
   residual by ``f`` keeps the lowest ``k'(f) = max{k < b : s_k <= f}``
   directions deflated; the others, ``O(f) = {k'+1 .. b-1}``, are outlying
   small eigenvalues, and the CG bound with outliers (each adds one iteration
   and a factor ``lambda_max/theta_j - 1``) gives
   ``n(f) = |O(f)| + sqrt(kappa)/2 * (ln(2/f) + sum_{j in O(f)} ln(lambda_max/theta_j - 1))``.
4. Choice.  Without a restart a solve to ``tol`` costs ``n(tol)``; one restart
   at ``tau`` costs ``n(tau) + R + n(tol/tau)`` with ``R`` the restart's cost in
   iterations.  The linear terms of the two legs add up to
   ``sqrt(kappa)/2 * ln(4/tol)`` whatever ``tau`` is, so the restarted cost is
   constant between the break points ``{s_k, tol/s_k}``.  Adjacent intervals
   of equal cost are merged; the cheapest merged interval wins (ties: the
   wider in ``ln tau``, then the larger ``tau``), and ``tau`` is its geometric
   midpoint.  The restart is taken only if it is strictly cheaper than none.

Parity pins (``tests/test_oracle_restart_model.py``): the outlier bound
against CG on diagonal matrices, closed-form choices (exact eigenvectors, one
separated cluster, a large restart cost) and, on the 4^4 test lattice with a
bank grown by the oracle's Incremental eigCG, that the chosen threshold is
within a few iterations of the best of a sweep and far better than no restart.
"""

from __future__ import annotations

import math

import numpy as np


def _frobenius(res, k):
    return math.sqrt(sum(float(r) * float(r) for r in res[:k]))


def contamination_levels(theta, res, lam_max):
    """Step 1: ``s_0 .. s_{l-1}`` (``s_0 = 0``; ``s_k`` for the span of the
    ``k`` lowest of the ascending Ritz values)."""
    l = len(theta)
    s = np.zeros(max(l, 1))
    for k in range(1, l):
        s[k] = _frobenius(res, k) / lam_max
    return s


def bulk_start(theta, res):
    """Step 2: ``b``, the 1-based index of the first Ritz value of the bulk."""
    b = 1
    for k in range(1, len(theta)):
        gap = theta[k] - theta[k - 1]
        if gap > 0.0 and _frobenius(res, k) / gap < 1.0:
            b = k + 1
    return b


def outlier_bound(f, lam_max, lam_bulk, outliers):
    """CG iterations after which the bound with outlying small eigenvalues
    guarantees an error reduction by ``f`` in the energy norm: the polynomial
    that vanishes at each outlier times the shifted Chebyshev polynomial of the
    bulk ``[lam_bulk, lam_max]``, with ``(sqrt(k)-1)/(sqrt(k)+1) <= exp(-2/sqrt(k))``."""
    kappa = lam_max / lam_bulk
    extra = sum(math.log(max(lam_max / o - 1.0, 1.0)) for o in outliers)
    return len(outliers) + 0.5 * math.sqrt(kappa) * (math.log(2.0 / f) + extra)


def leg_cost(f, theta, s, b, lam_max):
    """Step 3: predicted iterations of a leg that reduces the residual by ``f``."""
    kp = max([k for k in range(0, b) if s[k] <= f], default=0)
    return outlier_bound(f, lam_max, theta[b - 1], [theta[j - 1] for j in range(kp + 1, b)])


def choose_restart(theta, res, lam_max, tol, restart_cost):
    """Step 4 for ascending Ritz values ``theta`` with residual norms ``res``.
    Returns ``(tau, cost_without, cost_with)``; ``tau = 0`` means no restart
    (then ``cost_with == cost_without``)."""
    theta = np.asarray(theta, dtype=np.float64)
    res = np.asarray(res, dtype=np.float64)
    if theta.size == 0:
        return 0.0, 0.0, 0.0
    if res.shape != theta.shape or np.any(np.diff(theta) < 0) or theta[0] <= 0.0:
        raise ValueError("need ascending positive Ritz values and one residual each")
    s = contamination_levels(theta, res, lam_max)
    b = bulk_start(theta, res)
    none = leg_cost(tol, theta, s, b, lam_max)
    pts = {tol, 1.0}
    for k in range(1, theta.size):
        for p in (s[k], tol / s[k] if s[k] > 0 else 0.0):
            if tol < p < 1.0:
                pts.add(p)
    pts = sorted(pts)
    merged = []  # [lo, hi, cost]
    for lo, hi in zip(pts[:-1], pts[1:]):
        mid = math.sqrt(lo * hi)
        c = (leg_cost(mid, theta, s, b, lam_max) + restart_cost
             + leg_cost(tol / mid, theta, s, b, lam_max))
        if merged and abs(merged[-1][2] - c) <= 1e-12 * max(1.0, abs(c)):
            merged[-1][1] = hi
        else:
            merged.append([lo, hi, c])
    best = None
    for lo, hi, c in merged:
        key = (c, -math.log(hi / lo), -hi)
        if best is None or key < best[0]:
            best = (key, lo, hi, c)
    _, lo, hi, c = best
    if c < none:
        return math.sqrt(lo * hi), none, c
    return 0.0, none, none
