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


@pytest.mark.parametrize("M,R,a", [(65536, 3, 0.45), (65536, 4, 0.3), (262144, 3, 0.4)])
def test_rhs_full_size_sampled(smol, M, R, a):
    """Full-size configurations: sampled entries against the oracle, which
    evaluates each sampled S_s by its direct sums."""
    say(f"rhs sampled M={M} R={R}")
    U, V = W.brownian_rank3(M, a) if R == 3 else W.product_rank4(M, a)
    n = W.exponential_start(M, 200.0) + 1e-3 * W.random_state(M, seed=5, decay=False) / M
    got = smol.rhs(t(U), t(V), 0.01, t(n)).cpu().numpy()
    first = [0] if M <= 65536 else []  # S_1's double sum is O(M^2 R) in the oracle
    idx = np.unique(np.concatenate([np.array(first + [1, 2, 3, M // 2, M - 2, M - 1]),
                                    np.random.default_rng(M).integers(1, M, 24)])).astype(np.int64)
    ref = oracle.rhs_entries(U, V, 0.01, n, idx)
    scale = np.abs(got).max()
    assert np.abs(got[idx] - ref).max() / scale < TOL


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
