"""smol_integrate_batch: many uneven instances advanced together, each with
its own step size, accept/reject and status.  Every instance runs the same
kernels as a single-instance run, so its result and statistics must equal
smol_integrate's exactly."""
import time

import numpy as np
import pytest

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


def _instances(specs):
    out = []
    for M, a, lam, s0, t_end in specs:
        U, V = W.brownian_rank3(M, a)
        out.append(dict(U=t(U), V=t(V), lam=lam, n0=t(W.exponential_start(M, s0)), t_end=t_end,
                        rtol=1e-6, atol=1e-12))
    return out


SPECS = [(3, 0.2, 0.01, 1.0, 2.0), (50, 0.3, 0.05, 3.0, 10.0), (600, 0.45, 0.002, 8.0, 20.0),
         (4096, 0.1, 0.03, 15.0, 30.0), (4097, 0.33, 0.001, 2.0, 5.0), (10000, 0.5, 0.1, 20.0, 8.0),
         (70000, 0.25, 0.01, 5.0, 3.0), (1, 0.3, 0.0, 1.0, 1.0), (2000, 0.4, 0.01, 4.0, 0.0)]


@pytest.mark.parametrize("method,precision", [("bs3", "fp64"), ("dp5", "fp64"), ("bs3", "fp32x2")])
def test_batch_equals_single_runs(smol, method, precision):
    insts = _instances(SPECS)
    say(f"batch {method} {precision}: {len(insts)} instances")
    outs, stats = smol.integrate_batch(insts, method=method, precision=precision)
    for d, o, st in zip(insts, outs, stats):
        ref, rst = smol.integrate(d["U"], d["V"], d["lam"], d["n0"], d["t_end"], d["rtol"],
                                  d["atol"], method=method, precision=precision)
        assert st == rst, (st, rst)
        assert np.array_equal(o.cpu().numpy(), ref.cpu().numpy())
        assert st["status"] == 0 and st["t"] == d["t_end"]


def test_poisoned_instance_fails_alone(smol):
    insts = _instances(SPECS[:5])
    bad = insts[2]["n0"].clone()
    bad[7] = float("nan")
    insts[2]["n0"] = bad
    outs, stats = smol.integrate_batch(insts, method="bs3")
    assert stats[2]["status"] == smol.ENONFINITE
    for i in (0, 1, 3, 4):
        assert stats[i]["status"] == 0 and stats[i]["t"] == insts[i]["t_end"]


def test_batch_limits_per_instance(smol):
    """Options apply to every instance; each stops on its own limit."""
    insts = _instances(SPECS[:4])
    outs, stats = smol.integrate_batch(insts, method="bs3", max_steps=5)
    for st in stats:
        assert st["status"] in (0, smol.EMAXSTEPS)
        assert st["n_accept"] + st["n_reject"] <= 5
    assert any(st["status"] == smol.EMAXSTEPS for st in stats)


def test_batch_small_instances_match_oracle(smol):
    """The batch's small instances (M = 1, 3, 50, 600, 4096) against the
    oracle's integrator run by run: identical accept / reject decisions, t
    and h to 1e-5, end states to 1e-7 (max-norm relative).  The weighted norm
    divides entries far below the largest by about atol, and there the
    transform's round-off (small only relative to the largest entries) is
    not small relative to the entry: err moves by up to ~1e-5 relative when
    it is small, and the PI controller passes that on to h and t."""
    import oracle
    import torch
    for method, name in (("bs3", oracle.BS32), ("dp5", oracle.DP54)):
        specs = [sp for sp in SPECS if sp[0] in (1, 3, 50, 600, 4096)]
        insts = _instances(specs)
        logs = [torch.zeros((20000, 9), dtype=torch.float64, device="cuda:0") for _ in insts]
        for d, lg in zip(insts, logs):
            d["log"] = lg
        outs, stats = smol.integrate_batch(insts, method=method)
        for (M, a, lam, s0, t_end), o, st, lg in zip(specs, outs, stats, logs):
            U, V = W.brownian_rank3(M, a)
            ref, rst, rlog = oracle.integrate(U, V, lam, W.exponential_start(M, s0), t_end,
                                              1e-6, 1e-12, method=name, log_cap=20000)
            say(f"batch {method} M={M}: gpu {st} oracle {rst}")
            assert st["status"] == 0 and rst["status"] == 0
            assert (st["n_accept"], st["n_reject"], st["n_rhs"]) == \
                (rst["n_accept"], rst["n_reject"], rst["n_rhs"])
            g = lg.cpu().numpy()[: st["n_accept"] + st["n_reject"]]
            np.testing.assert_array_equal(g[:, 3], rlog[:, 3])
            np.testing.assert_allclose(g[:, 0], rlog[:, 0], rtol=1e-5)
            np.testing.assert_allclose(g[:, 1], rlog[:, 1], rtol=1e-5)
            assert normwise(o.cpu().numpy(), ref) < 1e-7


def test_config3_draws_short_window(smol):
    """The batched sweep's 256 seeded instances (M in [2^12, 2^17]) over a
    short window: every instance finishes and a sample equals its single run
    (the two forms' times are reported, not compared)."""
    import torch
    draws = W.batch_draws(256, seed=0)
    insts = []
    for d in draws:
        U, V, lam, n0 = W.batch_instance(d)
        insts.append(dict(U=t(U), V=t(V), lam=lam, n0=t(n0), t_end=5.0, rtol=1e-6, atol=1e-12))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs, stats = smol.integrate_batch(insts, method="bs3")
    tb = time.perf_counter() - t0
    assert all(st["status"] == 0 and st["t"] == 5.0 for st in stats)
    t0 = time.perf_counter()
    for i in range(0, 256, 32):
        d = insts[i]
        ref, rst = smol.integrate(d["U"], d["V"], d["lam"], d["n0"], 5.0, 1e-6, 1e-12, method="bs3")
        assert rst == stats[i] and np.array_equal(ref.cpu().numpy(), outs[i].cpu().numpy())
    ts = (time.perf_counter() - t0) * 256 / 8
    say(f"batched-sweep draws to t=5: batch {tb:.3f} s, single runs (extrapolated from 8) "
        f"{ts:.3f} s, accepted steps {sum(s['n_accept'] for s in stats)}")


def test_config3_full_length(smol):
    """The batched sweep as specified (256 seeded instances, BS3, rtol 1e-6,
    atol 1e-12, t_end = 1e3): every instance reaches t_end; mass is conserved
    to 1e-6 where the tail above M/2 carries (almost) no mass; the instance
    with the smallest M equals the oracle's trajectory to 1e-6."""
    import oracle
    c = W.WORKLOADS["batched-sweep"]
    draws = W.batch_draws(c["n_inst"], seed=c["seed"])
    insts, host = [], []
    for d in draws:
        U, V, lam, n0 = W.batch_instance(d)
        host.append((U, V, lam, n0))
        insts.append(dict(U=t(U), V=t(V), lam=lam, n0=t(n0), t_end=c["t_end"], rtol=c["rtol"],
                          atol=c["atol"]))
    say("batched sweep to t_end = 1e3")
    t0 = time.perf_counter()
    outs, stats = smol.integrate_batch(insts, method=c["method"])
    say(f"  {time.perf_counter() - t0:.2f} s, accepted {sum(s['n_accept'] for s in stats)}, "
        f"rejected {sum(s['n_reject'] for s in stats)}")
    assert all(st["status"] == 0 and st["t"] == c["t_end"] for st in stats)
    checked = 0
    for (U, V, lam, n0), o in zip(host, outs):
        n = o.cpu().numpy()
        s = np.arange(1, n.size + 1)
        tail = np.sum((s * np.abs(n))[n.size // 2:])
        if tail < 1e-9:
            # the mass leaves only through the truncation flux; round-off in
            # the tail entries, weighted by s, sets the 1e-6 scale
            assert abs(np.sum(s * n) - np.sum(s * n0)) < 1e-6
            checked += 1
    say(f"  mass conserved on {checked} of {len(outs)} instances with a massless tail")
    assert checked > 0
    i = int(np.argmin([d["M"] for d in draws]))
    U, V, lam, n0 = host[i]
    say(f"  oracle trajectory of instance {i} (M = {draws[i]['M']})")
    ref, rst, _ = oracle.integrate(U, V, lam, n0, c["t_end"], c["rtol"], c["atol"],
                                   method=oracle.BS32)
    say(f"  gpu {stats[i]} oracle {rst}")
    assert normwise(outs[i].cpu().numpy(), ref) < 1e-6
