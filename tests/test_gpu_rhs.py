"""smol_rhs (HIP) against the FP64 oracle's direct double sums.

Bar: max-norm relative error <= 1e-10 in FP64 (normwise, since FFT round-off
is relative to the largest entries, not to each tail entry)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import normwise, say, t

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module")
def smol():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_16559_amd as smol
    return smol


@pytest.mark.parametrize("M", [1, 2, 3, 7, 31, 33, 64, 100, 257, 512, 1000, 2049, 4096, 5000])
@pytest.mark.parametrize("R", [1, 3, 4])
def test_rhs_full_parity(smol, M, R):
    say(f"rhs parity M={M} R={R}")
    U, V = W.random_factors(M, R, seed=M * 31 + R)
    n = W.random_state(M, seed=M + 7)
    got = smol.rhs(t(U), t(V), 0.013, t(n)).cpu().numpy()
    ref = oracle.rhs(U, V, 0.013, n)
    assert normwise(got, ref) < TOL


@pytest.mark.parametrize("M", [512, 8192])
def test_rhs_config_kernel_monodisperse_and_spread(smol, M):
    U, V = W.brownian_rank3(M, 0.45)
    for n in (W.monodisperse(M), W.exponential_start(M, 50.0), W.random_state(M, 3, decay=False)):
        got = smol.rhs(t(U), t(V), 0.005, t(n)).cpu().numpy()
        assert normwise(got, oracle.rhs(U, V, 0.005, n)) < TOL


def _spread_state(M):
    return W.exponential_start(M, 200.0) + 1e-3 * W.random_state(M, seed=5, decay=False) / M


@pytest.mark.parametrize("M,R,a", [(65536, 3, 0.45), (65536, 4, 0.3), (262144, 3, 0.4)])
def test_rhs_full_size_every_entry(smol, M, R, a):
    """The full-size kernels (the single-large and learned-proposer
    instances' rank-3 kernel, the precision workload's rank-4 product):
    every entry against the oracle's direct sums, normalised by the oracle."""
    say(f"rhs full size M={M} R={R}")
    U, V = W.brownian_rank3(M, a) if R == 3 else W.product_rank4(M, a)
    n = _spread_state(M)
    got = smol.rhs(t(U), t(V), 0.01, t(n)).cpu().numpy()
    ref = oracle.rhs(U, V, 0.01, n)
    err = normwise(got, ref)
    say(f"  normwise error {err:.2e}")
    assert err < TOL


@pytest.mark.parametrize("M", [5000, 65536])
@pytest.mark.parametrize("R", [2, 5, 8, 16, 32])
def test_rhs_ranks_beyond_prefetch(smol, M, R):
    """Ranks 2 (the paper's Brownian kernel without constant term) and 5..32
    (32 is the largest the library takes): the row-pair pass takes several
    rounds of ranks and the finish reads the ranks beyond its prefetched
    four, under the installed schedule."""
    say(f"rhs rank M={M} R={R}")
    U, V = W.random_factors(M, R, seed=1000 * R + M % 997)
    n = _spread_state(M)
    got = smol.rhs(t(U), t(V), 0.017, t(n)).cpu().numpy()
    ref = oracle.rhs(U, V, 0.017, n)
    err = normwise(got, ref)
    say(f"  normwise error {err:.2e}")
    assert err < TOL


def test_rhs_largest_size(smol):
    """M = 2^19 + 1, the largest size (transform length 2^20): sampled
    entries against the oracle, ragged tail included; one size more is
    refused (SMOL_EUNSUPPORTED) by smol_rhs and smol_integrate."""
    M = 2 ** 19 + 1
    U, V = W.random_factors(M, 3, seed=19)
    n = _spread_state(M)
    got = smol.rhs(t(U), t(V), 0.01, t(n)).cpu().numpy()
    idx = np.array([0, 1, 2, 1000, M // 2, M - 3, M - 2, M - 1])
    ref = oracle.rhs_entries(U, V, 0.01, n, idx)
    err = np.abs(got[idx] - ref).max() / np.abs(got).max()
    say(f"rhs M={M}: sampled error vs oracle {err:.2e}")
    assert err < TOL
    M += 1
    U, V = W.random_factors(M, 1, seed=20)
    n = t(W.random_state(M, seed=21))
    with pytest.raises(smol.SmolError) as e:
        smol.rhs(t(U), t(V), 0.01, n)
    assert e.value.code == smol.EUNSUPPORTED
    with pytest.raises(smol.SmolError) as e:
        smol.integrate(t(U), t(V), 0.01, n, 1.0, 1e-6, 1e-12, raise_on_error=True)
    assert e.value.code == smol.EUNSUPPORTED


def test_rhs_rank4_equals_rank3(smol):
    M = 65536
    n = W.exponential_start(M, 300.0)
    a = smol.rhs(*map(t, W.product_rank4(M, 0.3)), 0.02, t(n)).cpu().numpy()
    b = smol.rhs(*map(t, W.brownian_rank3(M, 0.3)), 0.02, t(n)).cpu().numpy()
    assert normwise(a, b) < TOL


def test_rhs_mass_balance_large(smol):
    """sum_s s S_s = -F_trunc; with a state that vanishes above M/2 the
    truncation flux is zero, so the GPU RHS must conserve mass to round-off."""
    M = 65536
    U, V = W.brownian_rank3(M, 0.45)
    n = W.exponential_start(M, 500.0)
    n[M // 2:] = 0.0
    S = smol.rhs(t(U), t(V), 0.005, t(n)).cpu().numpy()
    s = np.arange(1, M + 1)
    assert abs(np.sum(s * S)) < 1e-11 * np.sum(s * np.abs(S))


def test_rhs_deterministic(smol):
    M = 65536
    U, V = W.brownian_rank3(M, 0.45)
    n = t(W.exponential_start(M, 100.0))
    a = smol.rhs(t(U), t(V), 0.005, n).cpu().numpy()
    b = smol.rhs(t(U), t(V), 0.005, n).cpu().numpy()
    assert np.array_equal(a, b)


def test_rhs_two_streams_share_plan(smol):
    """Calls with the same plan on two streams, issued back to back without
    host synchronisation: the library orders the shared workspaces, so every
    result equals the one computed alone."""
    import torch
    M = 65536
    U, V = W.brownian_rank3(M, 0.45)
    Ut, Vt = t(U), t(V)
    n1, n2 = t(W.exponential_start(M, 100.0)), t(W.exponential_start(M, 20.0))
    r1 = smol.rhs(Ut, Vt, 0.005, n1).cpu().numpy()
    r2 = smol.rhs(Ut, Vt, 0.005, n2).cpu().numpy()
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for _ in range(6):
        with torch.cuda.stream(sa):
            a = smol.rhs(Ut, Vt, 0.005, n1)
        with torch.cuda.stream(sb):
            b = smol.rhs(Ut, Vt, 0.005, n2)
        outs.append((a, b))
    torch.cuda.synchronize()
    for a, b in outs:
        assert np.array_equal(a.cpu().numpy(), r1)
        assert np.array_equal(b.cpu().numpy(), r2)

