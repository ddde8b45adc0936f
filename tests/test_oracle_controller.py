"""Pins of the oracle's PI step-size controller (beta term included).

The single-size problem M = 1 has S_1 = -K n^2 (K = U_11 V_11; the shattering
sums of Eq. (4) are empty), so n(t) = n0 / (1 + K n0 t) in closed form.  It is
scale invariant: every stage of an RK attempt from n with step h is n times a
function of x = K h n, so with atol = 0 the weighted-RMS norm of an attempt is
a function of x alone.  A PI controller h_{j+1} = h_j * safety *
err_j^-alpha * err_{j-1}^beta then settles at a fixed x*, where the step
factor equals the observed step growth rho = h_{j+1} / h_j; with
err_j = err_{j-1} = err* there,
    err* = (safety / rho)^(1 / (alpha - beta)).
The mathematics fixes this value from alpha - beta alone, independently of
how the oracle's code is written: a flipped sign of beta settles at
(safety / rho)^(1 / (alpha + beta)), and an err_prev that is never updated
(stuck at its initial 1) at (safety / rho)^(1 / alpha); both fail the check.
"""
import numpy as np
import pytest

import oracle

K = 2.5
N0 = 1.0


def _m1(k=K):
    return np.array([[1.0]]), np.array([[k]]), np.array([N0])


def _settled(log, tail=3):
    """(err_j, rho_j) for consecutive accepted attempts j, j+1 after the
    controller has settled (no rejections in between, the clipped last steps
    left out)."""
    rows = []
    for j in range(len(log) // 2, len(log) - 1 - tail):
        if log[j, 3] == 1 and log[j + 1, 3] == 1 and (j == 0 or log[j - 1, 3] == 1):
            rows.append((log[j, 2], log[j + 1, 1] / log[j, 1]))
    return np.array(rows)


def _fixed_point_err(log, alpha, beta, safety=0.9):
    """max relative deviation of the accepted norms from the fixed point
    predicted by the observed step growth, and the settled norm itself"""
    r = _settled(log)
    assert len(r) > 20, len(r)
    pred = (safety / r[:, 1]) ** (1.0 / (alpha - beta))
    return float(np.max(np.abs(r[:, 0] / pred - 1.0))), float(np.median(r[:, 0]))


@pytest.mark.parametrize("method,k", [(oracle.BS32, 3), (oracle.DP54, 5)])
def test_closed_form_single_size(method, k):
    """M = 1: n(T) = n0 / (1 + K n0 T) (both pairs, tight tolerance)."""
    U, V, n0 = _m1()
    T = 100.0
    out, st, _ = oracle.integrate(U, V, 0.01, n0, T, 1e-10, 1e-16, method=method)
    exact = N0 / (1.0 + K * N0 * T)
    assert st["status"] == oracle.OK and st["t"] == T
    assert abs(out[0] / exact - 1.0) < 1e-8


@pytest.mark.parametrize("method,k", [(oracle.BS32, 3), (oracle.DP54, 5)])
def test_pi_fixed_point_default_constants(method, k):
    """Default exponents (alpha, beta) = (0.7/k, 0.4/k): the accepted norm
    settles at (0.9/rho)^(1/(alpha-beta)).  Near rho = 1 this is about 0.17
    for DP5(4) and 0.35 for BS3(2); a flipped beta would sit near 0.6."""
    U, V, n0 = _m1()
    _, st, log = oracle.integrate(U, V, 0.0, n0, 1e9, 1e-6, 0.0, method=method,
                                  log_cap=100000)
    assert st["status"] == oracle.OK and st["n_reject"] == 0
    dev, err_star = _fixed_point_err(log, 0.7 / k, 0.4 / k)
    assert dev < 1e-6, (dev, err_star)
    # and the defaults are exactly the explicit (0.7/k, 0.4/k)
    _, st2, log2 = oracle.integrate(U, V, 0.0, n0, 1e9, 1e-6, 0.0, method=method,
                                    alpha=0.7 / k, beta=0.4 / k, log_cap=100000)
    assert st2 == st and np.array_equal(log2, log)


@pytest.mark.parametrize("alpha,beta", [(0.2, 0.05), (0.15, 0.1), (0.25, 0.0)])
def test_pi_fixed_point_given_exponents(alpha, beta):
    U, V, n0 = _m1(0.7)
    _, st, log = oracle.integrate(U, V, 0.0, n0, 1e9, 1e-7, 0.0, method=oracle.DP54,
                                  alpha=alpha, beta=beta, log_cap=100000)
    assert st["status"] == oracle.OK
    dev, _ = _fixed_point_err(log, alpha, beta)
    assert dev < 1e-6, dev


@pytest.mark.parametrize("method,k", [(oracle.BS32, 3), (oracle.DP54, 5)])
def test_planted_controller_mistakes_fail_the_pin(method, k):
    """Plant mistakes in the oracle's controller through its exponents: a
    flipped sign of beta (err_prev^-beta) and an err_prev that never changes
    from 1 (equivalent to beta = 0).  Each run settles where the check with
    the true (alpha, beta) fails by a wide margin."""
    U, V, n0 = _m1()
    alpha, beta = 0.7 / k, 0.4 / k
    for planted in (-beta, 0.0):
        _, st, log = oracle.integrate(U, V, 0.0, n0, 1e9, 1e-6, 0.0, method=method,
                                      alpha=alpha, beta=planted, log_cap=100000)
        assert st["status"] == oracle.OK
        dev, err_star = _fixed_point_err(log, alpha, beta)
        assert dev > 0.5, (planted, dev, err_star)
        # ... while the planted run does satisfy its own fixed point
        dev_own, _ = _fixed_point_err(log, alpha, planted)
        assert dev_own < 1e-6
