"""Learned step proposer: FP32 HIP forward / backward / Adam against the FP64
oracle, dataset rows against oracle features of the actual state, and the
learned controller (PI fallback, accuracy, what it gains)."""
import time

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import normwise, say, t

pytestmark = pytest.mark.gpu
NP = 4865


@pytest.fixture(scope="module")
def smol():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_16559_amd as smol
    return smol


def f32(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def init_params(seed):
    p = W.mlp_init(seed)
    assert p.size == NP
    return p


def rand_rows(n, seed):
    g = W.SplitMix64(seed)
    X = (2 * g.uniforms(n * 9) - 1).reshape(n, 9)
    return X, 0.5 * (2 * g.uniforms(n) - 1)


def test_forward_parity(smol):
    p = init_params(1)
    X, _ = rand_rows(500, 2)
    got = smol.proposer_forward(f32(p), f32(X)).cpu().numpy()
    ref = oracle.mlp_forward(p.astype(np.float32).astype(np.float64),
                             X.astype(np.float32).astype(np.float64))
    assert np.abs(got - ref).max() < 1e-5 * max(1.0, np.abs(ref).max())


def test_loss_gradient_parity(smol):
    p = init_params(3)
    X, tg = rand_rows(2000, 4)
    p32, X32, t32 = (a.astype(np.float32).astype(np.float64) for a in (p, X, tg))
    loss, grad = smol.proposer_loss_grad(f32(p), f32(X), f32(tg), 4.0)
    rl, rg = oracle.mlp_loss_grad(p32, X32, t32, 4.0)
    assert abs(loss.item() - rl) <= 1e-5 * abs(rl)
    err = normwise(grad.cpu().numpy(), rg)
    say(f"proposer gradient: normwise relative error vs FP64 oracle {err:.2e}")
    assert err < 1e-4


def test_one_adam_step(smol):
    """Full-batch training for one step equals one oracle Adam step on the
    oracle gradient (updates of size ~lr, FP32)."""
    p = init_params(5)
    X, tg = rand_rows(256, 6)
    params = f32(p)
    smol.proposer_train(f32(X), f32(tg), params, epochs=1, batch=256, lr=1e-3, over_weight=4.0)
    p32, X32, t32 = (a.astype(np.float32).astype(np.float64) for a in (p, X, tg))
    _, g = oracle.mlp_loss_grad(p32, X32, t32, 4.0)
    q = p32.copy()
    m, v = np.zeros(NP), np.zeros(NP)
    oracle.adam(q, g, m, v, 1)
    big = np.abs(g) > 1e-5  # away from the eps-dominated first step
    np.testing.assert_allclose(params.cpu().numpy()[big], q[big], atol=2e-6)


def test_training_reduces_loss(smol):
    X, _ = rand_rows(4096, 7)
    tg = np.tanh(X[:, 0] - 0.5 * X[:, 4])  # a learnable target
    params = f32(init_params(8))
    loss = smol.proposer_train(f32(X), f32(tg), params, epochs=40, batch=256, lr=3e-3).cpu().numpy()
    say(f"training loss first/last epoch {loss[0]:.4f} / {loss[-1]:.4f}")
    assert loss[-1] < 0.2 * loss[0]


def test_dataset_rows_match_oracle_features(smol):
    """Training rows from a logged GPU run equal the oracle's rows built from
    the same log (features to FP32 rounding, targets to FP32 accuracy), and
    the features of the decision after attempt j equal the oracle's features
    of the state reached after attempt j (run again with max_steps = j+1)."""
    import torch
    M = 800
    U, V = W.brownian_rank3(M, 0.4)
    n0 = W.monodisperse(M)
    log = torch.zeros((2000, 9), dtype=torch.float64, device="cuda:0")
    _, st = smol.integrate(t(U), t(V), 0.02, t(n0), 20.0, 1e-6, 1e-12, method="dp5", log=log,
                           h0=0.5)
    rows = st["n_accept"] + st["n_reject"]
    assert st["n_reject"] > 0
    X, tg = smol.proposer_dataset(log, rows, "dp5")
    L = log.cpu().numpy()[:rows]
    Xo, To = oracle.proposer_dataset(L, 5, err_target=0.8)
    assert X.shape[0] == Xo.shape[0] > 0
    np.testing.assert_allclose(X.cpu().numpy(), Xo, rtol=2e-7, atol=1e-7)
    assert np.abs(tg.cpu().numpy() - To).max() < 2e-6
    # rows: accepted attempts with a successor that did not follow a rejection
    acc = [j for j in range(rows - 1) if L[j, 3] == 1 and (j == 0 or L[j - 1, 3] == 1)]
    assert X.shape[0] == len(acc)
    for r, j in list(enumerate(acc))[5::7][:6]:
        nj, sj = smol.integrate(t(U), t(V), 0.02, t(n0), 20.0, 1e-6, 1e-12, method="dp5",
                                max_steps=j + 1, h0=0.5)
        hist = [L[j - q, 2] for q in range(4) if j - q >= 0]
        ref = oracle.features(nj.cpu().numpy(), L[j, 1], hist)
        np.testing.assert_allclose(X[r].cpu().numpy(), ref, rtol=2e-6, atol=2e-7)


@pytest.mark.parametrize("seed,b3", [(21, 0.0), (22, 0.3)])
def test_learned_decisions_match_oracle(smol, seed, b3):
    """Every step the learned controller takes in a logged GPU run equals the
    oracle's learned factor exp(clamp(log PI + network(features))) at that
    decision (FP32 network on the GPU, FP64 in the oracle); decisions after a
    rejection are PI's."""
    import torch
    p = init_params(seed)
    p[-1] = b3
    smol.proposer_set(f32(p))
    M = 3000
    U, V = W.brownian_rank3(M, 0.35)
    n0 = W.exponential_start(M, 4.0)
    log = torch.zeros((6000, 9), dtype=torch.float64, device="cuda:0")
    _, st = smol.integrate(t(U), t(V), 0.01, t(n0), 40.0, 1e-6, 1e-12, method="dp5",
                           controller="learned", log=log)
    rows = st["n_accept"] + st["n_reject"]
    L = log.cpu().numpy()[:rows]
    say(f"learned run seed {seed} b3 {b3}: {st}")
    assert st["status"] == 0 and rows < 6000
    want = oracle.learned_steps(p.astype(np.float32).astype(np.float64), L, 5)
    js = [j for j in range(rows - 2) if np.isfinite(want[j])]  # last successor clipped to t_end
    assert len(js) >= 10
    got = L[np.array(js) + 1, 1] / L[js, 1]
    rel = np.abs(got / want[js] - 1.0)
    say(f"  {len(js)} learned decisions, max relative difference {rel.max():.2e}")
    assert rel.max() < 2e-5
    assert st["n_fallback"] == sum(1 for j in range(rows)
                                   if L[j, 3] == 1 and j > 0 and L[j - 1, 3] != 1)


def test_bad_proposer_falls_back_to_pi(smol):
    """Weights that always propose 10x larger steps: every overshoot is
    rejected, the next step falls back to PI, and the run still meets the
    trajectory bar against a tight reference."""
    p = np.zeros(NP)
    p[-1] = 10.0  # b3: output clamps to log 10
    smol.proposer_set(f32(p))
    M = 1000
    U, V = W.brownian_rank3(M, 0.4)
    n0 = t(W.monodisperse(M))
    a, sa = smol.integrate(t(U), t(V), 0.01, n0, 50.0, 1e-6, 1e-12, method="dp5",
                           controller="learned")
    ref, _ = smol.integrate(t(U), t(V), 0.01, n0, 50.0, 1e-10, 1e-16, method="dp5")
    say(f"bad proposer: {sa}")
    assert sa["status"] == 0 and sa["n_reject"] > 0 and sa["n_fallback"] > 0
    assert normwise(a.cpu().numpy(), ref.cpu().numpy()) < 1e-5


def _training_runs(smol, specs, t_end, err_target=0.8):
    import torch
    insts, logs = [], []
    for M, a, lam, s0 in specs:
        U, V = W.brownian_rank3(M, a)
        log = torch.zeros((20000, 9), dtype=torch.float64, device="cuda:0")
        insts.append(dict(U=t(U), V=t(V), lam=lam, n0=t(W.exponential_start(M, s0)), t_end=t_end,
                          rtol=1e-6, atol=1e-12, log=log))
        logs.append(log)
    _, stats = smol.integrate_batch(insts, method="dp5")
    Xs, Ts = [], []
    for log, st in zip(logs, stats):
        X, tg = smol.proposer_dataset(log, st["n_accept"] + st["n_reject"], "dp5", err_target)
        Xs.append(X)
        Ts.append(tg)
    return torch.cat(Xs).contiguous(), torch.cat(Ts).contiguous()


@pytest.mark.parametrize("err_target", [0.8, 0.5])
def test_trained_proposer_ab(smol, err_target):
    """Train on PI logs of 24 seeded instances, then run a held-out instance
    with the learned controller and with PI: both meet the accuracy bar and
    the learned controller needs fewer right-hand sides (steps, rejections
    and time are reported)."""
    import torch
    draws = W.batch_draws(24, seed=11, m_lo_log2=10, m_hi_log2=13)
    X, tg = _training_runs(smol, [(d["M"], d["a"], d["lam"], d["s0"]) for d in draws], 200.0,
                           err_target)
    say(f"proposer training rows: {X.shape[0]}")
    params = f32(init_params(12345))
    loss = smol.proposer_train(X, tg, params, epochs=100, batch=512, lr=1e-3)
    smol.proposer_set(params)
    M = 16384
    U, V = W.brownian_rank3(M, 0.4)
    n0 = t(W.monodisperse(M))
    ref, _ = smol.integrate(t(U), t(V), 0.01, n0, 500.0, 1e-10, 1e-16, method="dp5")
    res = {}
    for ctrl in ("pi", "learned"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, st = smol.integrate(t(U), t(V), 0.01, n0, 500.0, 1e-6, 1e-12, method="dp5",
                                 controller=ctrl)
        dt = time.perf_counter() - t0
        res[ctrl] = (st, dt, normwise(out.cpu().numpy(), ref.cpu().numpy()))
        assert st["status"] == 0
    say(f"proposer loss {loss[0].item():.4f} -> {loss[-1].item():.4f}")
    for k, (st, dt, e) in res.items():
        say(f"{k} (target {err_target}): accepted {st['n_accept']} rejected {st['n_reject']} rhs {st['n_rhs']} "
            f"fallback {st['n_fallback']} time {dt:.3f}s err vs tight {e:.2e}")
    assert res["learned"][2] < 1e-5
    assert res["learned"][0]["n_rhs"] < res["pi"][0]["n_rhs"]
