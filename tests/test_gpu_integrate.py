"""smol_integrate (HIP) against the FP64 oracle's integrator.

Bars: trajectory max-norm relative error <= 1e-6 at t_end; with the same
controller the step sequence matches the oracle's (times to 1e-9)."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import normwise, say, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smol():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_16559_amd as smol
    return smol


def test_config1_full_trajectory(smol):
    """Plain method, small: M = 512, rank-3 kernel a = 1/3, lam = 0.01,
    monodisperse start, BS3 with PI control, rtol 1e-6, atol 1e-12, t_end 50."""
    c = W.WORKLOADS["plain-small"]
    U, V, lam, n0 = W.workload_instance("plain-small")
    say("config 1 trajectory")
    out, st = smol.integrate(t(U), t(V), lam, t(n0), c["t_end"], c["rtol"], c["atol"], method="bs3")
    ref, rst, _ = oracle.integrate(U, V, lam, n0, c["t_end"], c["rtol"], c["atol"],
                                   method=oracle.BS32)
    say("gpu", st, "oracle", rst)
    assert st["status"] == 0 and st["t"] == c["t_end"]
    assert normwise(out.cpu().numpy(), ref) < 1e-6
    assert abs(st["n_accept"] - rst["n_accept"]) <= 2
    assert abs(st["n_rhs"] - rst["n_rhs"]) <= 8


@pytest.mark.parametrize("method,name", [("bs3", oracle.BS32), ("dp5", oracle.DP54)])
def test_step_sequence_matches_oracle(smol, method, name):
    """Same tableau, norm, starting step and controller: the accepted times,
    step sizes and accept/reject decisions agree with the oracle's."""
    M = 200
    U, V = W.brownian_rank3(M, 0.4)
    n0 = W.monodisperse(M)
    import torch
    log = torch.zeros((4000, 9), dtype=torch.float64, device="cuda:0")
    out, st = smol.integrate(t(U), t(V), 0.02, t(n0), 20.0, 1e-5, 1e-10, method=method,
                             h0=2.0, log=log)
    ref, rst, rlog = oracle.integrate(U, V, 0.02, n0, 20.0, 1e-5, 1e-10, method=name, h0=2.0,
                                      log_cap=4000)
    g = log.cpu().numpy()[: st["n_accept"] + st["n_reject"]]
    assert st["n_reject"] > 0
    assert len(g) == len(rlog)
    np.testing.assert_array_equal(g[:, 3], rlog[:, 3])        # decisions
    np.testing.assert_allclose(g[:, 0], rlog[:, 0], rtol=1e-9)  # t
    np.testing.assert_allclose(g[:, 1], rlog[:, 1], rtol=1e-9)  # h
    # the norm itself only where the attempt is not wildly off (an err of
    # 1e40 is where the FFT's normwise accuracy meets atol-sized scales; both
    # sides still reject with the same factor)
    ok = rlog[:, 2] < 1e3
    np.testing.assert_allclose(g[ok, 2], rlog[ok, 2], rtol=1e-6)
    assert normwise(out.cpu().numpy(), ref) < 1e-9
    m = oracle.moments(out.cpu().numpy())
    np.testing.assert_allclose(g[-1, 5:9], m, rtol=1e-9)


def test_i_controller_option(smol):
    """alpha = 1/k, beta = 0 gives the I controller (as in the oracle pin)."""
    M = 64
    U, V = W.brownian_rank3(M, 0.4)
    n0 = W.monodisperse(M)
    out, st = smol.integrate(t(U), t(V), 0.02, t(n0), 30.0, 1e-5, 1e-10, method="dp5",
                             alpha=0.2, beta=0.0)
    ref, rst, _ = oracle.integrate(U, V, 0.02, n0, 30.0, 1e-5, 1e-10, method=oracle.DP54,
                                   alpha=0.2, beta=0.0)
    assert st["n_accept"] == rst["n_accept"] and st["n_rhs"] == rst["n_rhs"]
    assert normwise(out.cpu().numpy(), ref) < 1e-9


@pytest.mark.parametrize("method", ["bs3", "dp5"])
def test_closed_form(smol, method):
    """K == 1, lam = 0, n(0) = e_1: n_s(t) = (t/2)^(s-1) / (1+t/2)^(s+1)."""
    M, T = 1024, 5.0
    U, V = W.constant_kernel(M)
    out, st = smol.integrate(t(U), t(V), 0.0, t(W.monodisperse(M)), T, 1e-10, 1e-16,
                             method=method)
    s = np.arange(1, M + 1)
    ref = np.exp((s - 1) * np.log(T / 2) - (s + 1) * np.log1p(T / 2))
    assert st["status"] == 0
    assert normwise(out.cpu().numpy(), ref) < 1e-8


def test_mid_size_dp5_trajectory(smol):
    """M = 4096 (several FFT tiles, L = 8192), DP5 to t = 30 against the oracle."""
    M = 4096
    U, V = W.brownian_rank3(M, 0.45)
    n0 = W.exponential_start(M, 5.0)
    say("mid-size trajectory")
    out, st = smol.integrate(t(U), t(V), 0.005, t(n0), 30.0, 1e-6, 1e-12, method="dp5")
    ref, rst, _ = oracle.integrate(U, V, 0.005, n0, 30.0, 1e-6, 1e-12, method=oracle.DP54)
    say("gpu", st, "oracle", rst)
    assert st["status"] == 0
    assert normwise(out.cpu().numpy(), ref) < 1e-6


def test_status_codes(smol):
    M = 16
    U, V = W.brownian_rank3(M, 0.3)
    n0 = W.monodisperse(M)
    out, st = smol.integrate(t(U), t(V), 0.01, t(n0), 0.0, 1e-6, 1e-12)
    assert st["status"] == 0 and st["n_accept"] == 0 and np.array_equal(out.cpu().numpy(), n0)
    bad = n0.copy()
    bad[5] = np.nan
    _, st = smol.integrate(t(U), t(V), 0.01, t(bad), 1.0, 1e-6, 1e-12)
    assert st["status"] == smol.ENONFINITE
    out, st = smol.integrate(t(U), t(V), 0.01, t(n0), 100.0, 1e-6, 1e-12, max_steps=3)
    assert st["status"] == smol.EMAXSTEPS and st["n_accept"] + st["n_reject"] == 3
    assert st["t"] < 100.0
    _, st = smol.integrate(t(U), t(V), 0.01, t(n0), 1.0, 1e-14, 1e-20, h0=0.1, h_min=0.01,
                           max_steps=10000)
    assert st["status"] == smol.ESTEPSIZE and st["t"] < 1.0
    _, rst, _ = oracle.integrate(U, V, 0.01, n0, 1.0, 1e-14, 1e-20, h0=0.1, h_min=0.01,
                                 max_steps=10000)
    assert rst["status"] == oracle.ESTEPSIZE and rst["n_reject"] == st["n_reject"]


def test_invalid_arguments(smol):
    M = 8
    U, V = W.brownian_rank3(M, 0.3)
    n0 = t(W.monodisperse(M))
    for kw in (dict(rtol=0.0), dict(atol=-1.0), dict(t_end=-1.0)):
        args = dict(t_end=1.0, rtol=1e-6, atol=1e-12)
        args.update(kw)
        with pytest.raises(smol.SmolError):
            smol.integrate(t(U), t(V), 0.01, n0, args["t_end"], args["rtol"], args["atol"])


def test_output_aliases_input(smol):
    M = 300
    U, V = W.brownian_rank3(M, 0.3)
    n0 = W.monodisperse(M)
    x = t(n0)
    a, _ = smol.integrate(t(U), t(V), 0.01, t(n0), 3.0, 1e-6, 1e-12)
    b, _ = smol.integrate(t(U), t(V), 0.01, x, 3.0, 1e-6, 1e-12, out=x)
    assert b.data_ptr() == x.data_ptr()
    assert np.array_equal(a.cpu().numpy(), x.cpu().numpy())


def test_repeatable(smol):
    """Deterministic reductions: two runs are bitwise identical."""
    U, V, lam, n0 = W.workload_instance("plain-small")
    a, sa = smol.integrate(t(U), t(V), lam, t(n0), 20.0, 1e-6, 1e-12, method="bs3")
    b, sb = smol.integrate(t(U), t(V), lam, t(n0), 20.0, 1e-6, 1e-12, method="bs3")
    assert sa == sb and np.array_equal(a.cpu().numpy(), b.cpu().numpy())


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def window_against_oracle(smol, U, V, lam, t_end, fixture, precision):
    """The first 16 DP5 attempts (rtol 1e-6, atol 1e-12, monodisperse start)
    against an oracle window stored by tests/golden/make_oracle_windows.py:
    identical accept / reject decisions, t and h to 1e-6, the error norms to
    1e-5 where they exceed round-off level (1e-6), the end state to 1e-7
    (max-norm relative).  From the monodisperse
    start almost every entry is far below atol, where the weighted norm
    weighs the transform's round-off (relative to the largest entries) by
    1 / atol: err differs from the direct sums' by ~1e-8 (FP64) to ~1e-7
    (float-float) relative, and the controller carries that into h."""
    import torch
    ref = np.load(os.path.join(GOLDEN, fixture))
    rlog = ref["log"]
    M = U.shape[1]
    log = torch.zeros((64, 9), dtype=torch.float64, device="cuda:0")
    out, st = smol.integrate(t(U), t(V), lam, t(W.monodisperse(M)), t_end, 1e-6, 1e-12,
                             method="dp5", precision=precision, max_steps=16, log=log)
    say("gpu", st, "oracle counts", ref["counts"])
    assert st["status"] == smol.EMAXSTEPS
    assert [st["n_rhs"], st["n_accept"], st["n_reject"]] == list(ref["counts"])
    g = log.cpu().numpy()[:16]
    np.testing.assert_array_equal(g[:, 3], rlog[:, 3])
    np.testing.assert_allclose(g[:, 0], rlog[:, 0], rtol=1e-6)
    np.testing.assert_allclose(g[:, 1], rlog[:, 1], rtol=1e-6)
    # the norm itself where it is not at round-off level (the first steps
    # from the monodisperse start have err ~ 1e-13)
    ok = rlog[:, 2] > 1e-6
    np.testing.assert_allclose(g[ok, 2], rlog[ok, 2], rtol=1e-5)
    err = normwise(out.cpu().numpy(), ref["n"])
    say(f"{fixture} ({precision}): t = {st['t']:.4e}, end state error {err:.2e}")
    assert err < 1e-7
    return err


@pytest.mark.parametrize("precision", ["fp64", "fp32x2"])
def test_single_large_window_matches_oracle(smol, precision):
    """The single-large instance (M = 65536, a = 0.45, lam = 0.005) and the
    precision workload's first instance: the first 16 attempts against the
    oracle's integrator (about 100 direct O(M^2 R) right-hand sides)."""
    c = W.WORKLOADS["single-large"]
    U, V, lam, _ = W.workload_instance("single-large")
    window_against_oracle(smol, U, V, lam, c["t_end"], "single_large_dp5_w16.npz", precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32x2"])
def test_precision_rank4_window_matches_oracle(smol, precision):
    """The precision workload's rank-4 product kernel (a = 0.3, lam = 0.02)."""
    p = W.WORKLOADS["precision"]
    U, V = W.product_rank4(p["M"], p["a"])
    window_against_oracle(smol, U, V, p["lam"], p["t_eval"], "precision_rank4_dp5_w16.npz",
                          precision)


def test_config2_full_run_properties(smol):
    """Config 2 (M = 65536, a = 0.45, lam = 0.005, DP5, t_end = 1e4): the
    oracle cannot run this trajectory, so check what holds at any size: the
    run ends at t_end, mass is conserved while the distribution stays far
    from M, and the final state's RHS matches the oracle at sampled sizes."""
    c = W.WORKLOADS["single-large"]
    U, V, lam, n0 = W.workload_instance("single-large")
    say("config 2 full run")
    out, st = smol.integrate(t(U), t(V), lam, t(n0), c["t_end"], c["rtol"], c["atol"],
                             method="dp5")
    say("config 2 stats", st)
    assert st["status"] == 0 and st["t"] == c["t_end"]
    n = out.cpu().numpy()
    s = np.arange(1, n.size + 1)
    assert abs(np.sum(s * n) - 1.0) < 1e-5
    S = smol.rhs(t(U), t(V), lam, out).cpu().numpy()
    idx = np.array([0, 1, 2, 10, 100, 1000, 20000, n.size - 1])
    ref = oracle.rhs_entries(U, V, lam, n, idx)
    # near a stationary state S is a small difference of the gain and loss
    # terms; round-off is relative to those terms, so scale by the loss term
    loss = (1 + lam) * np.abs(n) * np.abs(U.T @ (V @ n))
    assert np.abs(S[idx] - ref).max() / loss.max() < 1e-10


def test_largest_size_run(smol):
    """M = 2^19 + 1 (transform length 2^20, the largest): DP5 from the
    monodisperse start to t = 5 ends with status OK and t = t_end; mass is
    conserved up to the transform's round-off in the long, nearly empty tail
    (weighted by the size there); the leading sizes follow the same run at
    M = 4096 (the norms average over different M, so the step sizes differ:
    compared loosely); the end state's right-hand side matches the oracle's
    direct sums at sampled sizes >= 2."""
    res = {}
    for M in (4096, 2 ** 19 + 1):
        U, V = W.brownian_rank3(M, 0.4)
        out, st = smol.integrate(t(U), t(V), 0.01, t(W.monodisperse(M)), 5.0, 1e-6, 1e-12,
                                 method="dp5")
        n = out.cpu().numpy()
        mass = np.sum(np.arange(1, M + 1) * n)
        say(f"M={M}: {st}, mass - 1 = {mass - 1.0:.2e}")
        assert st["status"] == 0 and st["t"] == 5.0
        assert abs(mass - 1.0) < 1e-6, mass
        res[M] = (n, U, V, out)
    a, (b, U, V, out) = res[4096][0], res[2 ** 19 + 1]
    d = normwise(b[:200], a[:200])
    say(f"leading 200 sizes against the M = 4096 run: {d:.2e}")
    assert d < 1e-4
    S = smol.rhs(t(U), t(V), 0.01, out).cpu().numpy()
    idx = np.array([1, 2, 10, 100, 1000, 2 ** 18, 2 ** 19])
    ref = oracle.rhs_entries(U, V, 0.01, b, idx)
    err = np.abs(S[idx] - ref).max() / np.abs(S).max()
    say(f"end-state RHS, sampled sizes >= 2 against the oracle: {err:.2e}")
    assert err < 1e-10
