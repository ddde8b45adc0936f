"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own formula: each checks it against a hand
expansion, a different derivation (the reaction mechanism behind Eq. (4)),
a conservation identity, a closed-form solution, order conditions, or a library
routine (scipy's RK23 / RK45, torch's CPU MLP and Adam).
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W


# ---------------------------------------------------------------------------
# Right-hand side, Eq. (2) and Eq. (4)
# ---------------------------------------------------------------------------

def _K(U, V):
    return U.T @ V  # K[i-1, j-1] = sum_a U[a, i-1] V[a, j-1]


def test_rhs_m2_hand_expanded():
    """M = 2 worked out by hand from Eq. (4) (general, non-symmetric K):
    S1 = -n1 (K11 n1 + K12 n2) + 2 lam K22 n2^2 + 2 lam K12 n1 n2,
    S2 = K11 n1^2 / 2 - (1 + lam) n2 (K21 n1 + K22 n2)."""
    U, V = W.random_factors(2, 2, seed=7)
    n = np.array([0.7, 0.35])
    lam = 0.3
    K = _K(U, V)
    n1, n2 = n
    S1 = -n1 * (K[0, 0] * n1 + K[0, 1] * n2) + 2 * lam * K[1, 1] * n2 ** 2 \
        + 2 * lam * K[0, 1] * n1 * n2
    S2 = 0.5 * K[0, 0] * n1 ** 2 - (1 + lam) * n2 * (K[1, 0] * n1 + K[1, 1] * n2)
    got = oracle.rhs(U, V, lam, n)
    np.testing.assert_allclose(got, [S1, S2], rtol=1e-14)


@pytest.mark.parametrize("lam", [0.0, 0.2])
def test_rhs_point_state(lam):
    """n = e_1: only monomer-monomer collisions happen, so S_1 = -K_11,
    S_2 = K_11 / 2 and every other entry vanishes."""
    M = 9
    U, V = W.random_factors(M, 3, seed=3)
    K11 = _K(U, V)[0, 0]
    got = oracle.rhs(U, V, lam, W.monodisperse(M))
    want = np.zeros(M)
    want[0], want[1] = -K11, 0.5 * K11
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=1e-300)


def _reaction_rates(M, K, n, lam):
    """dn/dt built from the collision mechanism, in exact rationals.

    Every ordered pair (i, j) collides at rate K_ij n_i n_j / 2.  With rate 1
    it aggregates: one i and one j are lost and one (i+j)-mer appears when
    i + j <= M (otherwise the product leaves the truncated system).  With
    rate lam it shatters: one i and one j are lost and i + j monomers appear.
    """
    d = [Fraction(0)] * M
    for i in range(1, M + 1):
        for j in range(1, M + 1):
            r = Fraction(1, 2) * K[i - 1][j - 1] * n[i - 1] * n[j - 1]
            d[i - 1] -= r
            d[j - 1] -= r
            if i + j <= M:
                d[i + j - 1] += r
            rs = lam * r
            d[i - 1] -= rs
            d[j - 1] -= rs
            d[0] += (i + j) * rs
    return d


@pytest.mark.parametrize("M", [1, 2, 3, 5, 7])
def test_rhs_matches_reaction_mechanism_exactly(M):
    """Eq. (4) with the n_1 factor on the monomer-j shattering gain is exactly
    the rate equation of the collision mechanism (symmetric rational kernel)."""
    g = W.SplitMix64(100 + M)
    R = 2
    Uq = [[Fraction(1 + int(7 * g.uniform()), 1 + int(5 * g.uniform())) for _ in range(M)]
          for _ in range(R)]
    dq = [Fraction(1, 2), Fraction(3, 1)]
    Vq = [[dq[a] * Uq[a][j] for j in range(M)] for a in range(R)]  # K = U^T diag(d) U
    K = [[sum(Uq[a][i] * Vq[a][j] for a in range(R)) for j in range(M)] for i in range(M)]
    n = [Fraction(1 + int(9 * g.uniform()), 7 + s) for s in range(M)]
    lam = Fraction(1, 10)
    exact = _reaction_rates(M, K, n, lam)
    U = np.array([[float(x) for x in row] for row in Uq])
    V = np.array([[float(x) for x in row] for row in Vq])
    got = oracle.rhs(U, V, float(lam), np.array([float(x) for x in n]))
    scale = max(abs(float(x)) for x in exact)
    np.testing.assert_allclose(got, [float(x) for x in exact], rtol=0, atol=1e-14 * scale)


def _trunc_flux(K, n):
    """(1/2) sum_{i,j<=M, i+j>M} (i+j) K_ij n_i n_j: mass carried out of the
    truncated system by aggregates larger than M."""
    M = n.size
    s = np.arange(1, M + 1)
    I, J = np.meshgrid(s, s, indexing="ij")
    mask = (I + J) > M
    return 0.5 * np.sum(((I + J) * K * np.outer(n, n))[mask])


@pytest.mark.parametrize("lam", [0.0, 0.01, 0.3])
def test_rhs_mass_balance(lam):
    """Aggregation and shattering conserve mass; only the truncation flux
    leaves: sum_s s S_s = -F_trunc (symmetric kernel)."""
    M = 96
    U, V = W.brownian_rank3(M, 0.45)
    n = W.random_state(M, seed=11, s0=30.0)
    S = oracle.rhs(U, V, lam, n)
    s = np.arange(1, M + 1)
    F = _trunc_flux(_K(U, V), n)
    scale = np.sum(s * np.abs(S)) + F
    assert abs(np.sum(s * S) + F) <= 1e-13 * scale


def test_rhs_number_balance_no_shattering():
    """lam = 0: every collision inside the system removes one cluster and
    every collision leaving it removes two: dN/dt = -C_in - 2 C_out, with C
    the collision rates (1/2) sum K_ij n_i n_j over pairs with i+j <= M or > M."""
    M = 80
    U, V = W.brownian_rank3(M, 1.0 / 3.0)
    n = W.random_state(M, seed=5, s0=20.0)
    K = _K(U, V)
    s = np.arange(1, M + 1)
    I, J = np.meshgrid(s, s, indexing="ij")
    P = K * np.outer(n, n)
    C_in = 0.5 * np.sum(P[(I + J) <= M])
    C_out = 0.5 * np.sum(P[(I + J) > M])
    S = oracle.rhs(U, V, 0.0, n)
    np.testing.assert_allclose(np.sum(S), -C_in - 2 * C_out, rtol=1e-13)


def test_rhs_rank_split_invariance():
    """Splitting every rank-one term into two halves leaves K, hence S, unchanged."""
    M = 40
    U, V = W.random_factors(M, 2, seed=9)
    n = W.random_state(M, seed=10)
    a = oracle.rhs(U, V, 0.07, n)
    b = oracle.rhs(np.concatenate([U / 2, U / 2]), np.concatenate([V, V]), 0.07, n)
    np.testing.assert_allclose(b, a, rtol=1e-13, atol=1e-16 * np.abs(a).max())


def test_rank4_product_kernel_equals_rank3():
    """(i^a+j^a)(i^-a+j^-a) = (i/j)^a + (j/i)^a + 2, so the rank-4 and rank-3
    factorizations give the same right-hand side."""
    M = 50
    n = W.random_state(M, seed=12)
    a = oracle.rhs(*W.product_rank4(M, 0.3), 0.02, n)
    b = oracle.rhs(*W.brownian_rank3(M, 0.3), 0.02, n)
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-15 * np.abs(b).max())


def test_rhs_zero_kernel():
    M = 17
    n = W.random_state(M, seed=1)
    assert np.all(oracle.rhs(np.zeros((1, M)), np.zeros((1, M)), 0.5, n) == 0.0)


def test_rhs_entries_match_full():
    M = 64
    U, V = W.brownian_rank3(M, 0.4)
    n = W.random_state(M, seed=2)
    full = oracle.rhs(U, V, 0.01, n)
    idx = np.array([0, 1, 2, 31, 62, 63])
    np.testing.assert_array_equal(oracle.rhs_entries(U, V, 0.01, n, idx), full[idx])


def test_rhs_thread_count_invariant():
    M = 128
    U, V = W.brownian_rank3(M, 0.4)
    n = W.random_state(M, seed=4)
    np.testing.assert_array_equal(oracle.rhs(U, V, 0.01, n, threads=1),
                                  oracle.rhs(U, V, 0.01, n, threads=4))


# ---------------------------------------------------------------------------
# Tableaux: order conditions (Butcher trees up to order 5)
# ---------------------------------------------------------------------------

def _order_conditions(A, b, p):
    c = A.sum(axis=1)
    conds = [(b.sum(), 1.0)]
    if p >= 2:
        conds += [(b @ c, 1 / 2)]
    if p >= 3:
        conds += [(b @ c ** 2, 1 / 3), (b @ A @ c, 1 / 6)]
    if p >= 4:
        conds += [(b @ c ** 3, 1 / 4), (b @ (c * (A @ c)), 1 / 8), (b @ A @ c ** 2, 1 / 12),
                  (b @ A @ A @ c, 1 / 24)]
    if p >= 5:
        Ac = A @ c
        conds += [(b @ c ** 4, 1 / 5), (b @ (c ** 2 * Ac), 1 / 10), (b @ (c * (A @ c ** 2)), 1 / 15),
                  (b @ (c * (A @ Ac)), 1 / 30), (b @ Ac ** 2, 1 / 20), (b @ A @ c ** 3, 1 / 20),
                  (b @ A @ (c * Ac), 1 / 40), (b @ A @ A @ c ** 2, 1 / 60),
                  (b @ A @ A @ A @ c, 1 / 120)]
    return [abs(x - y) for x, y in conds]


@pytest.mark.parametrize("method,p,q", [(oracle.BS32, 3, 2), (oracle.DP54, 5, 4)])
def test_tableau_order_conditions(method, p, q):
    A, b, bh = oracle.tableau(method)
    assert np.all(np.triu(A) == 0)  # explicit
    assert max(_order_conditions(A, b, p)) < 1e-14
    assert max(_order_conditions(A, bh, q)) < 1e-14
    # and not one order higher: the propagated and embedded weights are not swapped
    if p + 1 <= 5:
        assert max(_order_conditions(A, b, p + 1)) > 1e-6
    assert max(_order_conditions(A, bh, q + 1)) > 1e-6
    # FSAL: the last stage is evaluated at the propagated solution
    np.testing.assert_array_equal(A[-1, :-1], b[:-1])
    assert b[-1] == 0.0


# ---------------------------------------------------------------------------
# Trajectories: the K == 1 closed form
# ---------------------------------------------------------------------------

def closed_form(M, t):
    """K == 1, lam = 0, n(0) = e_1: n_s(t) = (t/2)^(s-1) / (1+t/2)^(s+1)."""
    s = np.arange(1, M + 1, dtype=np.float64)
    x = t / 2.0
    return np.exp((s - 1) * np.log(x) - (s + 1) * np.log1p(x)) if t > 0 else W.monodisperse(M)


@pytest.mark.parametrize("method", [oracle.BS32, oracle.DP54])
def test_closed_form_trajectory(method):
    M, t_end = 128, 5.0
    U, V = W.constant_kernel(M)
    out, st, _ = oracle.integrate(U, V, 0.0, W.monodisperse(M), t_end, rtol=1e-10,
                                  atol=1e-14, method=method)
    assert st["status"] == oracle.OK and st["t"] == t_end
    ref = closed_form(M, t_end)
    assert np.abs(out - ref).max() / ref.max() < 2e-8
    m = oracle.moments(out)
    assert abs(m[0] - 1.0 / (1.0 + t_end / 2)) < 1e-8   # number density N(t)
    assert abs(m[1] - 1.0) < 1e-12                       # mass (tail ~ 1e-19 at M=128)


@pytest.mark.parametrize("method,embedded,order", [
    (oracle.BS32, False, 3), (oracle.BS32, True, 2),
    (oracle.DP54, False, 5), (oracle.DP54, True, 4)])
def test_fixed_step_convergence_order(method, embedded, order):
    """Self-convergence of the fixed-step propagated / embedded solutions on a
    nonlinear aggregation-shattering problem: |y_h - y_{h/2}| ~ h^order."""
    M, T = 32, 1.0
    U, V = W.brownian_rank3(M, 0.4)
    n0 = 0.05 * W.random_state(M, seed=3, s0=4.0)
    ys = [oracle.rk_fixed(U, V, 0.05, n0, method, T / n, n, embedded) for n in (4, 8, 16, 32)]
    d = [np.abs(ys[i] - ys[i + 1]).max() for i in range(3)]
    slope = np.log2(d[1] / d[2])
    assert abs(slope - order) < 0.3, (slope, d)


# ---------------------------------------------------------------------------
# Controller: with beta = 0 it is scipy's RK23 / RK45 I-controller
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("h0", [0.0, 3.0])
@pytest.mark.parametrize("method,name", [(oracle.BS32, "RK23"), (oracle.DP54, "RK45")])
def test_controller_reduces_to_scipy(method, name, h0):
    """alpha = 1/k, beta = 0 turns the PI controller into scipy's I controller;
    starting step (h0 = 0: Hairer's procedure), accept/reject decisions, step
    factors, the cap after a rejection and the final clipping must all agree."""
    from scipy.integrate import RK23, RK45
    M, lam, t_end, rtol, atol = 24, 0.02, 30.0, 1e-5, 1e-10
    U, V = W.brownian_rank3(M, 0.4)
    n0 = W.monodisperse(M)
    k = 3 if method == oracle.BS32 else 5
    out, st, log = oracle.integrate(U, V, lam, n0, t_end, rtol, atol, method=method, h0=h0,
                                    alpha=1.0 / k, beta=0.0, log_cap=100000)
    cls = RK23 if name == "RK23" else RK45
    sol = cls(lambda t, y: oracle.rhs(U, V, lam, y), 0.0, n0.copy(), t_end, rtol=rtol, atol=atol,
              first_step=h0 if h0 > 0 else None)
    ts = []
    while sol.status == "running":
        sol.step()
        ts.append(sol.t)
    acc_t = log[log[:, 3] == 1][:, 4]
    assert st["n_accept"] == len(ts)
    assert st["n_rhs"] == sol.nfev
    np.testing.assert_allclose(acc_t, ts, rtol=1e-9)
    np.testing.assert_allclose(out, sol.y, rtol=1e-8, atol=1e-13)
    if h0 > 0:
        assert st["n_reject"] > 0  # the comparison exercised the reject path too


def test_integrate_status_codes():
    M = 8
    U, V = W.brownian_rank3(M, 0.3)
    n0 = W.monodisperse(M)
    out, st, _ = oracle.integrate(U, V, 0.01, n0, 0.0, 1e-6, 1e-12)
    assert st["status"] == oracle.OK and st["n_accept"] == 0 and np.array_equal(out, n0)
    bad = n0.copy()
    bad[3] = np.nan
    _, st, _ = oracle.integrate(U, V, 0.01, bad, 1.0, 1e-6, 1e-12)
    assert st["status"] == oracle.ENONFINITE
    _, st, _ = oracle.integrate(U, V, 0.01, n0, 100.0, 1e-6, 1e-12, max_steps=3)
    assert st["status"] == oracle.EMAXSTEPS and st["n_accept"] + st["n_reject"] == 3
    # a tolerance that needs steps below the smallest allowed one
    _, st, _ = oracle.integrate(U, V, 0.01, n0, 1.0, 1e-14, 1e-20, h0=0.1, h_min=0.01,
                                max_steps=10000)
    assert st["status"] == oracle.ESTEPSIZE and st["t"] < 1.0 and st["n_reject"] > 0


def test_integrate_ends_exactly_at_t_end():
    M = 16
    U, V = W.brownian_rank3(M, 0.3)
    _, st, log = oracle.integrate(U, V, 0.01, W.monodisperse(M), 7.25, 1e-6, 1e-12,
                                  log_cap=10000)
    assert st["t"] == 7.25 and log[-1, 4] == 7.25


# ---------------------------------------------------------------------------
# Proposer features and MLP
# ---------------------------------------------------------------------------

def test_features_on_closed_form():
    """Moments of the closed-form state: M0 = 1/(1+t/2), M1 = 1, and
    M2 = 1 + t (second moment of the K == 1 solution from e_1); features
    are the logs scaled by 1/40 (moments) and 1/10 (step, errors)."""
    t = 3.0
    n = closed_form(512, t)
    x = oracle.features(n, 0.25, [0.5, 0.25])
    np.testing.assert_allclose(40 * x[0], -np.log1p(t / 2), rtol=1e-12)
    assert abs(x[1]) < 1e-12
    np.testing.assert_allclose(40 * x[2], np.log1p(t), rtol=1e-10)
    np.testing.assert_allclose(10 * x[4:7], np.log([0.25, 0.5, 0.25]), rtol=1e-14)
    assert x[7] == 0.0 and x[8] == 0.0


def _rand_params(seed, scale=0.3):
    g = np.random.default_rng(seed)
    return g.normal(0, scale, oracle.mlp_nparams())


def test_mlp_forward_matches_torch():
    import torch
    p = _rand_params(0)
    X = np.random.default_rng(1).normal(size=(32, 9))
    net = torch.nn.Sequential(torch.nn.Linear(9, 64), torch.nn.Tanh(), torch.nn.Linear(64, 64),
                              torch.nn.Tanh(), torch.nn.Linear(64, 1)).double()
    o = 0
    with torch.no_grad():
        for layer, (r, c) in zip([net[0], net[2], net[4]], [(64, 9), (64, 64), (1, 64)]):
            layer.weight.copy_(torch.from_numpy(p[o:o + r * c].reshape(r, c)))
            o += r * c
            layer.bias.copy_(torch.from_numpy(p[o:o + r]))
            o += r
        want = net(torch.from_numpy(X)).numpy()[:, 0]
    assert o == p.size
    np.testing.assert_allclose(oracle.mlp_forward(p, X), want, rtol=1e-12, atol=1e-14)


def test_mlp_gradient_central_differences():
    p = _rand_params(2)
    g = np.random.default_rng(3)
    X = g.normal(size=(16, 9))
    tgt = g.normal(size=16)
    _, grad = oracle.mlp_loss_grad(p, X, tgt, 4.0)
    idx = np.random.default_rng(4).choice(p.size, 60, replace=False)
    idx = np.concatenate([idx, [p.size - 1, 0, 640, 704, 4800]])
    for i in idx:
        e = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += e
        pm[i] -= e
        fd = (oracle.mlp_loss_grad(pp, X, tgt, 4.0)[0] - oracle.mlp_loss_grad(pm, X, tgt, 4.0)[0]) / (2 * e)
        assert abs(fd - grad[i]) <= 1e-7 * max(1.0, abs(grad[i])) + 1e-9, (i, fd, grad[i])


def test_mlp_overshoot_weight():
    """Over-prediction costs over_w times as much as the same under-prediction."""
    p = np.zeros(oracle.mlp_nparams())
    X = np.zeros((1, 9))
    lo, _ = oracle.mlp_loss_grad(p, X, np.array([0.5]), 4.0)   # y = 0 < target
    hi, _ = oracle.mlp_loss_grad(p, X, np.array([-0.5]), 4.0)  # y = 0 > target
    assert lo == pytest.approx(0.25) and hi == pytest.approx(1.0)


def test_adam_matches_torch():
    import torch
    g = np.random.default_rng(5)
    p = g.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.nn.Parameter(torch.from_numpy(p.copy()))
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        grad = g.normal(size=50)
        oracle.adam(p, grad, m, v, step)
        tp.grad = torch.from_numpy(grad.copy())
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-15)
