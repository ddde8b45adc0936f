"""Pins of the oracle's source term, Eq. (3): constant sources P_s added to
the right-hand side (the printed P_k read as P_s)."""
import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle import _K, _trunc_flux


def two_sources(M, p):
    """The paper's two constant sources: P_1 = 1, P_100 = p (Sec. 3.1)."""
    P = np.zeros(M)
    P[0] = 1.0
    P[99] = p
    return P


def test_source_mass_balance():
    """sum_s s (S + P)_s = sum_s s P_s - F_trunc, with F_trunc the mass the
    truncated aggregation pushes beyond M (lam = 0, Eq. (3))."""
    M = 150
    U, V = W.brownian_rank3(M, 0.45)
    n = W.random_state(M, seed=6, s0=30.0)
    P = two_sources(M, 0.3)
    S = oracle.rhs_source(U, V, 0.0, n, P)
    s = np.arange(1, M + 1)
    F = _trunc_flux(_K(U, V), n)
    scale = np.sum(s * np.abs(S)) + F + np.dot(s, P)
    assert abs(np.dot(s, S) - (np.dot(s, P) - F)) <= 1e-13 * scale


@pytest.mark.parametrize("kind", ["embedded", "paper"])
def test_sources_without_kernel_grow_linearly(kind):
    """K == 0: dn/dt = P, so n(t) = n0 + P t for any scheme."""
    M = 120
    U, V = np.zeros((1, M)), np.zeros((1, M))
    n0 = W.random_state(M, seed=2)
    P = two_sources(M, 0.25)
    if kind == "embedded":
        out, st, _ = oracle.integrate(U, V, 0.0, n0, 7.0, 1e-8, 1e-12, method=oracle.DP54,
                                      source=P)
    else:
        out, st, _ = oracle.integrate_paper(U, V, 0.0, n0, 7.0, 1e-8, oracle.RKF45,
                                            oracle.RULE_FEHLBERG, source=P)
    assert st["status"] == oracle.OK
    np.testing.assert_allclose(out, n0 + 7.0 * P, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("p", [0.0, 0.1])
def test_constant_kernel_number_density_with_sources(p):
    """K == 1, no shattering, n(0) = e_1, sources P_1 = 1 and P_100 = p: the
    number density obeys N' = J - N^2 / 2 with J = 1 + p, so
    N(t) = sqrt(2J) tanh(sqrt(J/2) t + artanh(N(0) / sqrt(2J)))."""
    # sizes stay far below M up to t_end (the tail holds < 1e-10)
    M, t_end = 1200, 3.0
    U, V = W.constant_kernel(M)
    out, st, _ = oracle.integrate(U, V, 0.0, W.monodisperse(M), t_end, 1e-10, 1e-14,
                                  method=oracle.DP54, source=two_sources(M, p))
    assert st["status"] == oracle.OK
    J = 1.0 + p
    a = np.sqrt(2.0 * J)
    N = a * np.tanh(np.sqrt(J / 2.0) * t_end + np.arctanh(1.0 / a))
    assert abs(out.sum() - N) < 1e-8, (out.sum(), N)
