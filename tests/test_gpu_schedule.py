"""Launch schedules (radix and tile variants of the three right-hand-side
kernels): every variant computes the right-hand side to the same tolerance
against the FP64 oracle and drives the integrator to the same trajectory as
the default schedule; the autotuner installs a schedule that exists."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import normwise, say, t

pytestmark = pytest.mark.gpu
TOL_RHS = 1e-10


@pytest.fixture(scope="module")
def smol():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_16559_amd as smol
    return smol


def _variants(logL):
    """(phase, variant) pairs that exist at this length, besides variant 0."""
    N1, N2 = 2 ** ((logL + 1) // 2), 2 ** (logL // 2)
    out = []
    for ph, N in ((0, N1), (1, N2), (2, N1)):
        for v in (1, 2, 3):
            if (v < 2 or N <= 256) and not (logL == 20 and ph == 1 and v == 1):
                out.append((ph, v))
    return out


def _m_for(logL):
    """A ragged size whose transform length is 2^logL."""
    return 2 ** (logL - 2) + 3


@pytest.fixture
def restore(smol):
    saved = {L: smol.get_schedule(L) for L in range(12, 21)}
    yield
    for L, v in saved.items():
        smol.set_schedule(L, v)


@pytest.mark.parametrize("logL", [12, 13, 14])
def test_variant_rhs_vs_oracle(smol, restore, logL):
    M = _m_for(logL)
    U, V = W.random_factors(M, 3, seed=logL)
    n = W.random_state(M, seed=logL + 1)
    ref = oracle.rhs(U, V, 0.03, n)
    for ph, v in [(0, 0)] + _variants(logL):
        sched = [0, 0, 0]
        sched[ph] = v
        smol.set_schedule(logL, sched)
        got = smol.rhs(t(U), t(V), 0.03, t(n)).cpu().numpy()
        err = normwise(got, ref)
        say(f"logL={logL} M={M} schedule {sched}: normwise error {err:.2e}")
        assert err < TOL_RHS, (sched, err)


@pytest.mark.parametrize("logL", [15, 16, 17, 18, 19, 20])
def test_variant_rhs_large(smol, restore, logL):
    """Large lengths: each variant against the default schedule (normwise)
    and sampled entries against the oracle."""
    M = _m_for(logL) if logL < 20 else 2 ** 19
    U, V = W.brownian_rank3(M, 0.4)
    n = W.exponential_start(M, 50.0)
    smol.set_schedule(logL, [0, 0, 0])
    base = smol.rhs(t(U), t(V), 0.01, t(n)).cpu().numpy()
    idx = np.array([0, 1, 2, 77, M // 3, M - 2, M - 1])
    ref = oracle.rhs_entries(U, V, 0.01, n, idx)
    scale = np.abs(base).max()
    for ph, v in _variants(logL):
        sched = [0, 0, 0]
        sched[ph] = v
        smol.set_schedule(logL, sched)
        got = smol.rhs(t(U), t(V), 0.01, t(n)).cpu().numpy()
        e_base, e_or = normwise(got, base), np.abs(got[idx] - ref).max() / scale
        say(f"logL={logL} schedule {sched}: vs default {e_base:.2e}, sampled vs oracle {e_or:.2e}")
        assert e_base < 1e-12 and e_or < TOL_RHS, (sched, e_base, e_or)


@pytest.mark.parametrize("logL,split,whole", [(15, 2, 3), (16, 2, 3), (17, 0, 1)])
def test_split_finish_bitwise(smol, restore, logL, split, whole):
    """Phase C with two workgroups per packed column (four waves, one packed
    column per unit) computes exactly what one eight-wave workgroup per
    packed column does: the same inverse transform and finish per output,
    only spread over twice the workgroups."""
    import torch
    L = 2 ** logL
    for M in (L // 2 - 1234, L // 2 + 1):
        for R in (3, 5):
            U, V = W.random_factors(M, R, seed=logL + R)
            n = W.random_state(M, seed=M)
            out = []
            for v in (whole, split):
                smol.set_schedule(logL, [0, 0, v])
                out.append(smol.rhs(t(U), t(V), 0.01, t(n)))
            same = bool(torch.equal(out[0], out[1]))
            say(f"logL={logL} M={M} R={R}: C variant {split} bitwise equal to {whole}: {same}")
            assert same


@pytest.mark.parametrize("logL", [13, 17])
def test_variant_integration(smol, restore, logL):
    """DP5 runs under every variant (fused finish + column pass included)
    land on the default schedule's end state."""
    M = _m_for(logL)
    U, V = W.brownian_rank3(M, 0.45)
    n0 = t(W.monodisperse(M))
    smol.set_schedule(logL, [0, 0, 0])
    base, sb = smol.integrate(t(U), t(V), 0.005, n0, 20.0, 1e-6, 1e-12, method="dp5")
    base = base.cpu().numpy()
    for ph, v in _variants(logL):
        sched = [0, 0, 0]
        sched[ph] = v
        smol.set_schedule(logL, sched)
        out, st = smol.integrate(t(U), t(V), 0.005, n0, 20.0, 1e-6, 1e-12, method="dp5")
        err = normwise(out.cpu().numpy(), base)
        say(f"logL={logL} schedule {sched}: accepted {st['n_accept']} vs {sb['n_accept']}, "
            f"end-state difference {err:.2e}")
        assert st["status"] == 0 and err < 1e-8, (sched, err)


def test_autotune(smol, restore):
    M = _m_for(16)
    U, V = W.brownian_rank3(M, 0.45)
    n0 = t(W.monodisperse(M))
    smol.set_schedule(16, (0, 0, 0))
    sched, ms0, ms = smol.autotune(t(U), t(V), 0.005, n0, method="dp5", attempts=100, reps=2)
    say(f"autotune logL=16: schedule {sched}, {ms0:.4f} -> {ms:.4f} ms per attempt")
    assert smol.get_schedule(16) == sched and 0 < ms <= ms0
    n = W.random_state(M, seed=5)
    got = smol.rhs(t(U), t(V), 0.005, t(n)).cpu().numpy()
    idx = np.array([0, 1, 500, M - 1])
    ref = oracle.rhs_entries(U, V, 0.005, n, idx)
    assert np.abs(got[idx] - ref).max() / np.abs(got).max() < TOL_RHS


@pytest.mark.parametrize("method", ["bs3", "dp5"])
def test_profile_step_times_and_leaves_inputs(smol, method):
    """The stage-kernel timing hook returns positive times, does not touch
    the caller's arrays, and a later integration is unaffected."""
    import torch
    M = 5000
    U, V = W.brownian_rank3(M, 0.4)
    n0 = W.exponential_start(M, 10.0)
    Ud, Vd, nd = t(U), t(V), t(n0)
    before = nd.clone()
    ref, st_ref = smol.integrate(Ud, Vd, 0.01, nd, 2.0, 1e-6, 1e-12, method="dp5")
    ref = ref.cpu().numpy()
    ms = smol.profile_step(Ud, Vd, 0.01, nd, method=method, iters=5)
    torch.cuda.synchronize()
    say(f"profile_step {method} M={M}: {ms}")
    assert set(ms) == {"int_a", "int_b", "int_c_fused", "int_c_last"}
    assert all(np.isfinite(v) and v > 0 for v in ms.values())
    assert torch.equal(nd, before)
    out, st = smol.integrate(Ud, Vd, 0.01, nd, 2.0, 1e-6, 1e-12, method="dp5")
    assert st["n_accept"] == st_ref["n_accept"] and st["n_reject"] == st_ref["n_reject"]
    assert np.array_equal(out.cpu().numpy(), ref)
