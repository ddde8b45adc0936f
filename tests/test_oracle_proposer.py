"""Pins of the oracle's learned-proposer functions (CPU only): the training
rows built from a run log and the learned controller's step factors.

What fixes them besides their own code:
  * on the log of a PI-controlled run of the oracle integrator, the next step
    is the PI step, so the dataset's PI term cancels and the target reduces to
    (1/k) log(err_target / err_{j+1}) on every unclamped row;
  * if the error of an attempt is C h^k, the hindsight step the target
    encodes meets err_target exactly;
  * a network with constant output b gives the factor clamp(PI e^b), b = 0
    the integrator's own PI steps, large |b| the clamp limits; where the
    attempt's err exceeds 0.5 the factor is at most PI's."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

K_DP5 = 5


def _pi_run_log():
    M = 200
    U, V = W.brownian_rank3(M, 0.4)
    n0 = W.monodisperse(M)
    _, st, log5 = oracle.integrate(U, V, 0.02, n0, 20.0, 1e-5, 1e-10, method=oracle.DP54,
                                   h0=2.0, log_cap=4000)
    assert st["n_reject"] > 0 and st["status"] == 0
    log = np.zeros((log5.shape[0], 9))
    log[:, :5] = log5
    log[:, 5:] = np.array([1.0, 2.0, 5.0, 20.0])  # moments (any positive values)
    return log


def _decisions(log):
    """Accepted attempts that did not follow a rejection and have a successor."""
    acc = log[:, 3] == 1.0
    return [j for j in range(len(log) - 1) if acc[j] and (j == 0 or acc[j - 1])]


def zero_net(b3=0.0):
    p = np.zeros(oracle.mlp_nparams())
    p[-1] = b3  # the output bias: the network's output is b3 for every input
    return p


def test_dataset_pi_term_cancels_on_pi_run():
    log = _pi_run_log()
    X, tg = oracle.proposer_dataset(log, K_DP5, err_target=0.8)
    js = _decisions(log)
    assert len(js) == len(tg) and len(js) > 20
    checked = 0
    for row, j in enumerate(js):
        c = math.log(0.8 / log[j + 1, 2]) / K_DP5
        d = math.log(log[j + 1, 1] / log[j, 1]) + c
        last = j + 1 == len(log) - 1  # the final attempt is clipped to t_end
        if math.log(0.2) < d < math.log(10.0) and not last:
            assert abs(tg[row] - c) < 1e-12, (j, tg[row], c)
            checked += 1
        # features: moments of row j, h_j, the error history
        hist = log[max(0, j - 3):j + 1, 2][::-1]
        np.testing.assert_array_equal(X[row], oracle.proposer_features(log[j, 5:], log[j, 1], hist))
    assert checked > 20


def test_dataset_target_meets_err_target_under_power_law():
    """err_j = C h_j^k (below 0.5) on an all-accepted log: the step
    exp(target + log PI) h_j has model error err_target (the learned factor
    with output = target is that step)."""
    g = W.SplitMix64(3)
    rows, C, k = 40, 3.0e9, K_DP5
    h = 1e-2 * np.exp(0.1 * (g.uniforms(rows) - 0.5))  # err_j within 0.3 e^(+-0.25)
    log = np.zeros((rows, 9))
    log[:, 0] = np.concatenate([[0.0], np.cumsum(h)[:-1]])
    log[:, 1] = h
    log[:, 2] = C * h ** k
    log[:, 3] = 1.0
    log[:, 4] = log[:, 0] + h
    log[:, 5:] = np.array([1.0, 1.5, 4.0, 9.0])
    X, tg = oracle.proposer_dataset(log, k, err_target=0.3)
    assert len(tg) == rows - 1
    for j in range(rows - 1):
        hist = log[max(0, j - 3):j + 1, 2][::-1]
        err_prev = 1.0 if j == 0 else max(log[j - 1, 2], 1e-4)
        f = oracle.learned_factor(zero_net(tg[j]), log[j, 5:], log[j, 1], hist, err_prev, k)
        assert abs(C * (h[j] * f) ** k / 0.3 - 1.0) < 1e-10


def test_learned_steps_zero_network_is_pi_run():
    log = _pi_run_log()
    r = oracle.learned_steps(zero_net(), log, K_DP5)
    js = _decisions(log)
    assert np.isnan(np.delete(r, js)).all()
    for j in js[:-1]:  # the last decision's successor is clipped to t_end
        assert abs(r[j] / (log[j + 1, 1] / log[j, 1]) - 1.0) < 1e-12


def test_learned_factor_clamps_and_scales():
    log = _pi_run_log()
    # accepted norms spread over (0.05, 0.95), so that some decisions are
    # taken near the acceptance limit
    g = W.SplitMix64(17)
    acc = log[:, 3] == 1.0
    log[acc, 2] = 0.05 + 0.9 * g.uniforms(int(acc.sum()))
    r0 = oracle.learned_steps(zero_net(), log, K_DP5)
    rb = oracle.learned_steps(zero_net(0.25), log, K_DP5)
    hi = oracle.learned_steps(zero_net(9.0), log, K_DP5)
    lo = oracle.learned_steps(zero_net(-9.0), log, K_DP5)
    capped = 0
    for j in _decisions(log):
        near_limit = log[j, 2] > 0.5  # the step may not grow beyond PI's there
        capped += near_limit
        expect = min(10.0, max(0.2, r0[j] * math.exp(0.25)))
        assert abs(rb[j] / (r0[j] if near_limit else expect) - 1.0) < 1e-12
        if near_limit:
            assert abs(hi[j] / r0[j] - 1.0) < 1e-12
        else:
            assert hi[j] == pytest.approx(10.0, rel=1e-14)
        assert lo[j] == pytest.approx(0.2, rel=1e-14)
    assert capped > 0


def test_proposer_features_from_moments_match_state_features():
    M = 300
    n = W.random_state(M, seed=9)
    hist = np.array([0.3, 0.9, 0.05])
    np.testing.assert_allclose(oracle.proposer_features(oracle.moments(n), 0.01, hist),
                               oracle.features(n, 0.01, hist), rtol=0, atol=0)
