"""Pins of the oracle's version of the paper's own schemes (Sec. 2): RKF45
with Fehlberg's step rule, RK2 / RK4 with step doubling and the step update of
Eq. (6) or the halve / double rule, with the Euclidean error norm.

Checked against: Butcher order conditions, local error orders and the
Richardson ratio of step doubling on the K == 1 closed form, whole runs
against the closed form, the worked examples the paper gives for Fehlberg's
rule and the RKF45 coefficients it prints (both stored under tests/golden/
with their citation)."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle import _order_conditions, closed_form

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_rkf45_tableau_orders():
    """As printed: the propagated weights are fourth order, the error
    estimate's fifth order, and neither is one order higher."""
    A, b, bh = oracle.tableau(oracle.RKF45)
    assert A.shape == (6, 6) and np.all(np.triu(A) == 0)
    assert max(_order_conditions(A, b, 4)) < 1e-14
    assert max(_order_conditions(A, bh, 5)) < 1e-14
    assert max(_order_conditions(A, b, 5)) > 1e-6


@pytest.mark.parametrize("scheme,p", [(oracle.RKF45, 4), (oracle.RK2_DBL, 2), (oracle.RK4_DBL, 4)])
def test_local_error_orders(scheme, p):
    """One attempt from n(0) = e_1 on the K == 1 closed form.  RKF45: the
    fourth- and fifth-order solutions have local errors ~ tau^5 and tau^6.
    Step doubling: the single step's local error ~ tau^(p+1), and the two
    half steps are 2^p times closer (Richardson)."""
    M = 64
    U, V = W.constant_kernel(M)
    n0 = W.monodisperse(M)
    # small enough to be asymptotic, large enough to stay above round-off
    taus = [0.05, 0.025, 0.0125] if scheme == oracle.RKF45 else [0.2, 0.1, 0.05]
    e_a, e_b = [], []
    for tau in taus:
        a, b = oracle.paper_attempt(U, V, 0.0, n0, tau, scheme)
        ref = closed_form(M, tau)
        e_a.append(np.abs(a - ref).max())
        e_b.append(np.abs(b - ref).max())
    slope_a = np.log2(e_a[1] / e_a[2])
    slope_b = np.log2(e_b[1] / e_b[2])
    if scheme == oracle.RKF45:
        assert abs(slope_a - 5) < 0.15 and abs(slope_b - 6) < 0.4, (slope_a, slope_b)
    else:
        assert abs(slope_a - (p + 1)) < 0.3, slope_a
        assert abs(slope_b - (p + 1)) < 0.3, slope_b
        assert abs(e_a[2] / e_b[2] / 2 ** p - 1) < 0.05, e_a[2] / e_b[2]


CASES = [(oracle.RKF45, oracle.RULE_FEHLBERG), (oracle.RK2_DBL, oracle.RULE_EQ6),
         (oracle.RK2_DBL, oracle.RULE_HALVE_DOUBLE), (oracle.RK4_DBL, oracle.RULE_EQ6),
         (oracle.RKF45, oracle.RULE_EQ6)]


@pytest.mark.parametrize("scheme,rule", CASES)
def test_runs_follow_closed_form(scheme, rule):
    """Whole runs to t = 5 on the closed form: accurate, and more accurate at
    a tighter tolerance."""
    M = 96
    U, V = W.constant_kernel(M)
    n0 = W.monodisperse(M)
    ref = closed_form(M, 5.0)
    errs = []
    for tol in (1e-6, 1e-9):
        out, st, _ = oracle.integrate_paper(U, V, 0.0, n0, 5.0, tol, scheme, rule)
        assert st["status"] == oracle.OK and st["t"] == 5.0
        errs.append(np.abs(out - ref).max())
    assert errs[0] < 1e-4 and errs[1] < errs[0] / 10, errs


def _ratios(log, t_end):
    """h_{j+1} / h_j and err_j over the attempts whose successor was not
    clipped to land on t_end."""
    t, h, err = log[:, 0], log[:, 1], log[:, 2]
    free = t[1:] + h[1:] < t_end
    return (h[1:] / h[:-1])[free], err[:-1][free]


def test_fehlberg_rule_matches_worked_examples():
    """The paper's examples for Fehlberg's rule: err = 2 tol shrinks the step
    by about 20 %, err = tol / 2 grows it by about 3 %, err = tol shrinks it by
    10 %.  Every step change in a run follows one function of err/tol that
    passes through those points."""
    M = 48
    U, V = W.brownian_rank3(M, 0.4)
    # a too-large first step forces rejections as well as growth
    _, st, log = oracle.integrate_paper(U, V, 0.02, W.monodisperse(M), 40.0, 1e-7,
                                        oracle.RKF45, oracle.RULE_FEHLBERG, h0=4.0,
                                        log_cap=100000)
    r, e = _ratios(log, 40.0)
    f = lambda x: np.clip(0.9 * x ** (-0.2), 0.2, 10.0)  # noqa: E731
    np.testing.assert_allclose(r, f(e), rtol=1e-12)
    for x, fac, tol in np.loadtxt(os.path.join(GOLDEN, "fehlberg_rule_examples.txt"), ndmin=2):
        assert abs(f(x) - fac) < tol, (x, fac)
    assert st["n_reject"] > 0 and (e < 0.59).any()  # shrinking and growing both exercised


def test_step_doubling_rules():
    """Eq. (6) with s = 1/4 and p = 2 for RK2; the halve / double rule
    changes the step by exactly 2 or 1/2."""
    M = 48
    U, V = W.brownian_rank3(M, 0.4)
    n0 = W.monodisperse(M)
    _, _, log = oracle.integrate_paper(U, V, 0.02, n0, 40.0, 1e-6, oracle.RK2_DBL,
                                       oracle.RULE_EQ6, log_cap=100000)
    r, e = _ratios(log, 40.0)
    np.testing.assert_allclose(r, np.clip(0.25 * e ** -0.5, 0.2, 10.0), rtol=1e-12)
    _, _, log = oracle.integrate_paper(U, V, 0.02, n0, 40.0, 1e-6, oracle.RK2_DBL,
                                       oracle.RULE_HALVE_DOUBLE, log_cap=100000)
    r, e = _ratios(log, 40.0)
    # (h is re-derived as (t + h) - t each attempt: equal up to rounding)
    np.testing.assert_allclose(r, np.where(e <= 1.0, 2.0, 0.5), rtol=1e-12)


@pytest.mark.parametrize("scheme,per_attempt", [(oracle.RKF45, 5), (oracle.RK2_DBL, 4),
                                                (oracle.RK4_DBL, 10)])
def test_rhs_counts(scheme, per_attempt):
    """S at a state is evaluated once: 1 (start) + 1 (starting-step probe) +
    per attempt (RKF45: k_2..k_6; RK2 doubling: 1 + 1 + 1 + 1; RK4 doubling:
    3 + 3 + 1 + 3) + 1 per accepted state before t_end."""
    M = 32
    U, V = W.brownian_rank3(M, 0.4)
    _, st, _ = oracle.integrate_paper(U, V, 0.02, W.monodisperse(M), 20.0, 1e-6, scheme,
                                      oracle.RULE_EQ6 if scheme != oracle.RKF45 else
                                      oracle.RULE_FEHLBERG)
    att = st["n_accept"] + st["n_reject"]
    assert st["n_rhs"] == 2 + per_attempt * att + st["n_accept"] - 1


def test_rkf45_tableau_is_the_printed_one():
    """The oracle's RKF45 coefficients are exactly the rationals the paper
    prints (tests/golden/rkf45_sec2.txt), converted to FP64."""
    from fractions import Fraction
    a, b, bh = oracle.tableau(oracle.RKF45)
    A = np.zeros((6, 6))
    B4, B5 = np.zeros(6), np.zeros(6)
    for line in open(os.path.join(GOLDEN, "rkf45_sec2.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        kind, i, j, num, den = line.split()
        v = float(Fraction(int(num), int(den)))
        if kind == "a":
            A[int(i) - 1, int(j) - 1] = v
        elif kind == "b4":
            B4[int(j) - 1] = v
        else:
            B5[int(j) - 1] = v
    np.testing.assert_array_equal(a[:6, :6], A)
    np.testing.assert_array_equal(b[:6], B4)      # propagated: fourth order
    np.testing.assert_array_equal(bh[:6], B5)     # error estimate: fifth order
