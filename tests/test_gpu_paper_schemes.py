"""The paper's own schemes on the GPU (Sec. 2): RKF45 with Fehlberg's rule,
RK2 and RK4 with step doubling and Eq. (6) or the halve / double rule,
Euclidean norm.  Each run must take the oracle's decisions (accept / reject, step
sizes) and end on its state; the GPU evaluates S at every attempt's new
state (the next attempt's first stage), so it counts one evaluation more per
rejection than the oracle, which reuses S(n) across retries, and one for the
final state, which the oracle does not evaluate."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import normwise, say, t

pytestmark = pytest.mark.gpu

CASES = [("rkf45", "fehlberg", oracle.RKF45, oracle.RULE_FEHLBERG),
         ("rk2_dbl", "step_doubling", oracle.RK2_DBL, oracle.RULE_EQ6),
         ("rk2_dbl", "halve_double", oracle.RK2_DBL, oracle.RULE_HALVE_DOUBLE),
         ("rkf45", "step_doubling", oracle.RKF45, oracle.RULE_EQ6),
         ("rk4_dbl", "step_doubling", oracle.RK4_DBL, oracle.RULE_EQ6),
         ("rk4_dbl", "halve_double", oracle.RK4_DBL, oracle.RULE_HALVE_DOUBLE)]


@pytest.fixture(scope="module")
def smol():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_16559_amd as smol
    return smol


@pytest.mark.parametrize("method,ctrl,scheme,rule", CASES)
@pytest.mark.parametrize("M,h0", [(300, 0.0), (130, 3.0)])
def test_paper_scheme_matches_oracle(smol, method, ctrl, scheme, rule, M, h0):
    import torch
    U, V = W.brownian_rank3(M, 0.4)
    n0 = W.monodisperse(M)
    tol, t_end, lam = 1e-7, 30.0, 0.02
    ref, ost, olog = oracle.integrate_paper(U, V, lam, n0, t_end, tol, scheme, rule, h0=h0,
                                            log_cap=100000)
    log = torch.zeros((100000, 9), dtype=torch.float64, device="cuda:0")
    out, st = smol.integrate(t(U), t(V), lam, t(n0), t_end, tol, 0.0, method=method,
                             controller=ctrl, h0=h0, log=log)
    say(f"{method}/{ctrl} M={M} h0={h0}: gpu {st['n_accept']}/{st['n_reject']} rhs {st['n_rhs']}, "
        f"oracle {ost['n_accept']}/{ost['n_reject']} rhs {ost['n_rhs']}")
    assert st["status"] == 0 and ost["status"] == 0
    assert (st["n_accept"], st["n_reject"]) == (ost["n_accept"], ost["n_reject"])
    assert st["n_rhs"] == ost["n_rhs"] + ost["n_reject"] + 1
    g = log.cpu().numpy()[:len(olog)]
    np.testing.assert_array_equal(g[:, 3], olog[:, 3])                   # decisions
    # t and h: each step factor depends on err, a difference of two close
    # solutions (relative rounding ~1e-16 / tol per attempt), so over ~10^3
    # attempts the sequences drift apart at the 1e-8 level
    np.testing.assert_allclose(g[:, [0, 1, 4]], olog[:, [0, 1, 4]], rtol=1e-6)
    # err / tol: the estimate is a difference of close solutions, accurate to
    # ~1e-16 / tol absolute per component (decisions are compared exactly above)
    np.testing.assert_allclose(g[:, 2], olog[:, 2], rtol=1e-6, atol=1e-6)
    assert normwise(out.cpu().numpy(), ref) < 1e-9


@pytest.mark.parametrize("M", [1, 2, 3, 64])
def test_rk4_doubling_small_sizes(smol, M):
    """Degenerate sizes (a single size class, the smallest transforms): the
    same decisions as the oracle and the same end state."""
    U, V = W.brownian_rank3(M, 0.3)
    n0 = W.exponential_start(M, 2.0)
    ref, ost, _ = oracle.integrate_paper(U, V, 0.05, n0, 5.0, 1e-8, oracle.RK4_DBL,
                                         oracle.RULE_EQ6)
    out, st = smol.integrate(t(U), t(V), 0.05, t(n0), 5.0, 1e-8, 0.0, method="rk4_dbl",
                             controller="step_doubling")
    say(f"rk4_dbl M={M}: gpu {st['n_accept']}/{st['n_reject']}, "
        f"oracle {ost['n_accept']}/{ost['n_reject']}")
    assert st["status"] == 0 and (st["n_accept"], st["n_reject"]) == (ost["n_accept"], ost["n_reject"])
    assert normwise(out.cpu().numpy(), ref) < 1e-12


def test_rk4_doubling_closed_form(smol):
    """K == 1, lam = 0, n(0) = e_1: n_s(t) = (t/2)^(s-1) / (1+t/2)^(s+1),
    reached by RK4 with step doubling at a tight tolerance."""
    M, T = 1024, 5.0
    U, V = W.constant_kernel(M)
    out, st = smol.integrate(t(U), t(V), 0.0, t(W.monodisperse(M)), T, 1e-11, 0.0,
                             method="rk4_dbl", controller="step_doubling")
    s = np.arange(1, M + 1)
    ref = np.exp((s - 1) * np.log(T / 2) - (s + 1) * np.log1p(T / 2))
    assert st["status"] == 0
    assert normwise(out.cpu().numpy(), ref) < 1e-8


def test_paper_schemes_in_batch(smol):
    """Batched runs take the same paths: bitwise equal to single runs."""
    insts = []
    for M, a, lam in ((200, 0.3, 0.01), (3000, 0.45, 0.005), (5000, 0.2, 0.05)):
        U, V = W.brownian_rank3(M, a)
        insts.append(dict(U=t(U), V=t(V), lam=lam, n0=t(W.exponential_start(M, 4.0)), t_end=10.0,
                          rtol=1e-7, atol=0.0))
    for method, ctrl in (("rkf45", "fehlberg"), ("rk2_dbl", "step_doubling"),
                         ("rk4_dbl", "step_doubling")):
        outs, stats = smol.integrate_batch(insts, method=method, controller=ctrl)
        for d, o, st in zip(insts, outs, stats):
            r, rs = smol.integrate(d["U"], d["V"], d["lam"], d["n0"], 10.0, 1e-7, 0.0,
                                   method=method, controller=ctrl)
            assert st == rs and np.array_equal(o.cpu().numpy(), r.cpu().numpy())


def test_rhs_counts_versus_tolerance(smol):
    """The paper's observation (Tables 1-3): RKF45's evaluations grow slowly as
    the tolerance tightens, RK2 with step doubling's grow steeply.  Reported
    (M = 32768, Brownian a = 1/3, lam = 0.01, monodisperse, t = 0 -> 100);
    the ordering at the tightest tolerance is asserted."""
    M = 32768
    U, V = W.brownian_rank3(M, 1.0 / 3.0)
    n0 = t(W.monodisperse(M))
    rows = {}
    for tol in (1e-4, 1e-6, 1e-8):
        for method, ctrl in (("rk2_dbl", "step_doubling"), ("rk4_dbl", "step_doubling"),
                             ("rkf45", "fehlberg"), ("dp5", "pi")):
            rtol, atol = (tol, 0.0) if ctrl != "pi" else (tol, tol * 1e-6)
            _, st = smol.integrate(t(U), t(V), 0.01, n0, 100.0, rtol, atol, method=method,
                                   controller=ctrl)
            assert st["status"] == 0
            rows[(method, tol)] = st["n_rhs"]
    for method in ("rk2_dbl", "rk4_dbl", "rkf45", "dp5"):
        say(f"{method}: RHS evaluations at tol 1e-4 / 1e-6 / 1e-8: "
            f"{rows[(method, 1e-4)]} / {rows[(method, 1e-6)]} / {rows[(method, 1e-8)]}")
    assert rows[("rkf45", 1e-8)] < rows[("rk2_dbl", 1e-8)]
