"""Checkpoint and resume (smol_options.state): a run stopped after K attempts
and resumed from its checkpoint equals the uninterrupted run bitwise, state
and statistics, for each scheme and controller; the split may fall after an
accepted or a rejected attempt."""
import ctypes

import numpy as np
import pytest

import workloads as W
from gpu_util import say, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smol():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_16559_amd as smol
    return smol


CASES = [("bs3", "pi"), ("dp5", "pi"), ("dp5", "learned"), ("rkf45", "fehlberg"),
         ("rk4_dbl", "step_doubling"), ("rk2_dbl", "halve_double")]


def _problem(M=3000):
    U, V = W.brownian_rank3(M, 0.4)
    return t(U), t(V), 0.01, t(W.exponential_start(M, 4.0))


@pytest.mark.parametrize("method,controller", CASES)
def test_split_runs_equal_unsplit(smol, method, controller):
    import torch
    if controller == "learned":
        p = W.mlp_init(31)
        smol.proposer_set(torch.from_numpy(p.astype(np.float32)).to("cuda:0"))
    U, V, lam, n0 = _problem()
    M = n0.numel()
    kw = dict(method=method, controller=controller, h0=0.8)  # h0 large: early rejections
    log = torch.zeros((20000, 9), dtype=torch.float64, device="cuda:0")
    full, sf = smol.integrate(U, V, lam, n0, 40.0, 1e-6, 1e-12, log=log, **kw)
    n_att = sf["n_accept"] + sf["n_reject"]
    acc = log.cpu().numpy()[:n_att, 3]
    say(f"{method}/{controller}: {sf}")
    assert sf["status"] == 0 and sf["n_reject"] > 0 and n_att > 12
    j_rej = int(np.argmin(acc))          # first rejected attempt
    j_acc = n_att // 2 + int(acc[n_att // 2] == 0)
    for splits in ([j_rej + 1], [j_acc + 1], [3, j_acc + 1, n_att - 2]):
        st = smol.State(M)
        n = n0
        done = 0
        for k in splits:
            n, s1 = smol.integrate(U, V, lam, n, 40.0, 1e-6, 1e-12, max_steps=k - done,
                                   state=st, **kw)
            assert s1["status"] == smol.EMAXSTEPS and st.valid
            assert s1["n_accept"] + s1["n_reject"] == k
            done = k
        assert st.c.rejected == (acc[done - 1] == 0)
        out, s2 = smol.integrate(U, V, lam, n, 40.0, 1e-6, 1e-12, state=st, **kw)
        assert s2 == sf, (splits, s2, sf)
        assert np.array_equal(out.cpu().numpy(), full.cpu().numpy()), splits
        assert st.valid and st.c.t == 40.0


def test_resume_past_t_end_and_continue(smol):
    """A finished run's checkpoint continues to a later t_end (counters carry
    on); resuming at t >= t_end returns n0 unchanged after 0 attempts."""
    U, V, lam, n0 = _problem(1000)
    st = smol.State(1000)
    a, s1 = smol.integrate(U, V, lam, n0, 5.0, 1e-6, 1e-12, method="dp5", state=st)
    assert s1["status"] == 0 and st.valid and st.c.t == 5.0
    b, s2 = smol.integrate(U, V, lam, a, 5.0, 1e-6, 1e-12, method="dp5", state=st)
    assert s2["n_accept"] == s1["n_accept"] and np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    c, s3 = smol.integrate(U, V, lam, a, 9.0, 1e-6, 1e-12, method="dp5", state=st)
    assert s3["status"] == 0 and s3["t"] == 9.0 and s3["n_accept"] > s1["n_accept"]
    ref, _ = smol.integrate(U, V, lam, n0, 9.0, 1e-6, 1e-12, method="dp5")
    assert np.abs(c.cpu().numpy() - ref.cpu().numpy()).max() < 1e-6 * np.abs(
        ref.cpu().numpy()).max()


def test_state_validation(smol):
    U, V, lam, n0 = _problem(100)
    st = smol.State(100)
    st.c.k1 = None
    with pytest.raises(smol.SmolError):
        smol.integrate(U, V, lam, n0, 1.0, 1e-6, 1e-12, state=st)
    st = smol.State(100)
    st.c.valid, st.c.t, st.c.h = 1, 0.5, 0.0
    with pytest.raises(smol.SmolError):
        smol.integrate(U, V, lam, n0, 1.0, 1e-6, 1e-12, state=st)
    st.c.h = float("nan")
    with pytest.raises(smol.SmolError):
        smol.integrate(U, V, lam, n0, 1.0, 1e-6, 1e-12, state=st)
    with pytest.raises(smol.SmolError):  # batched runs take no checkpoint
        smol.integrate_batch([dict(U=U, V=V, lam=lam, n0=n0, t_end=1.0, rtol=1e-6, atol=1e-12)],
                             state=smol.State(100))
    assert ctypes.sizeof(smol._State) == 8 * 8 + 3 * 8 + 4 * 4 + 8
