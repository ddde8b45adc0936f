"""Float-float (SMOL_FP32X2) variant: the convolution transforms in hi/lo FP32
pairs, everything else FP64.  Checked against the FP64 oracle (RHS) and the
FP64 GPU path (whole vectors at every transform length up to 2^20;
trajectories of the precision workload to t = 1e3)."""
import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import normwise, say, t

pytestmark = pytest.mark.gpu
# float-float carries ~48 significand bits (u^2 = 2^-48 ~ 3.6e-15 per
# operation); with log2(L) <= 20 butterfly levels the normwise error of the
# transforms stays near 1e-13.  The bar leaves a factor of ~100.
TOL_RHS = 1e-11


@pytest.fixture(scope="module")
def smol():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2407_16559_amd as smol
    return smol


@pytest.mark.parametrize("M", [2, 7, 33, 100, 1000, 5000])
def test_rhs_fp32x2_parity(smol, M):
    U, V = W.random_factors(M, 3, seed=M + 11)
    n = W.random_state(M, seed=M + 3)
    got = smol.rhs(t(U), t(V), 0.02, t(n), precision="fp32x2").cpu().numpy()
    err = normwise(got, oracle.rhs(U, V, 0.02, n))
    say(f"fp32x2 rhs M={M}: normwise error {err:.2e}")
    assert err < TOL_RHS


@pytest.mark.parametrize("kernel", ["rank3", "rank4"])
def test_rhs_fp32x2_full_size(smol, kernel):
    M = 65536
    U, V = W.brownian_rank3(M, 0.45) if kernel == "rank3" else W.product_rank4(M, 0.3)
    n = W.exponential_start(M, 300.0)
    a = smol.rhs(t(U), t(V), 0.01, t(n), precision="fp32x2").cpu().numpy()
    b = smol.rhs(t(U), t(V), 0.01, t(n)).cpu().numpy()
    idx = np.array([0, 1, 2, 500, 30000, M - 1])
    ref = oracle.rhs_entries(U, V, 0.01, n, idx)
    err = np.abs(a[idx] - ref).max() / np.abs(a).max()
    say(f"fp32x2 rhs M=65536 {kernel}: sampled error vs oracle {err:.2e}, "
        f"normwise vs FP64 GPU {normwise(a, b):.2e}")
    assert err < TOL_RHS and normwise(a, b) < TOL_RHS


@pytest.mark.parametrize("M,R", [(131072, 3), (262144, 3), (524288, 3), (65536, 5), (5000, 8)])
def test_rhs_fp32x2_long_transforms_and_ranks(smol, M, R):
    """Float-float at transform lengths 2^18 .. 2^20 and at ranks that take
    several rounds of the row-pair pass: sampled entries against the oracle's
    direct sums and the whole vector against the FP64 path (which the RHS
    tests check against the oracle on every entry at M = 5000, 65536 and
    262144, and on sampled entries at the other lengths)."""
    U, V = W.random_factors(M, R, seed=M + R)
    n = W.exponential_start(M, M / 200.0) + 1e-3 * W.random_state(M, seed=R, decay=False) / M
    a = smol.rhs(t(U), t(V), 0.01, t(n), precision="fp32x2").cpu().numpy()
    b = smol.rhs(t(U), t(V), 0.01, t(n)).cpu().numpy()
    idx = np.unique(np.array([0, 1, 2, 3, 77, M // 7, M // 2, M - 2, M - 1]))
    ref = oracle.rhs_entries(U, V, 0.01, n, idx)
    err = np.abs(a[idx] - ref).max() / np.abs(a).max()
    # sizes s >= 2 on their own scale: S_1 (mostly the FP64 reductions) is
    # the largest entry here and would hide the convolution's error
    e2 = np.abs(a[idx[idx > 0]] - ref[idx > 0]).max() / np.abs(b[1:]).max()
    n2 = normwise(a[1:], b[1:])
    say(f"fp32x2 rhs M={M} R={R}: sampled error vs oracle {err:.2e} (sizes >= 2: {e2:.2e}), "
        f"normwise vs FP64 GPU {normwise(a, b):.2e} (sizes >= 2: {n2:.2e})")
    assert err < TOL_RHS and e2 < TOL_RHS and n2 < TOL_RHS


@pytest.mark.parametrize("name,kernel,a,lam", [("rank3", "rank3", 0.45, 0.005),
                                               ("rank4", "rank4", 0.3, 0.02)])
def test_precision_workload_trajectory(smol, name, kernel, a, lam):
    """Precision workload: M = 65536 monodisperse, DP5, rtol 1e-6, to t = 1e3,
    float-float against FP64.  The difference is reported (and must stay
    within the trajectory bar)."""
    M = 65536
    U, V = W.brownian_rank3(M, a) if kernel == "rank3" else W.product_rank4(M, a)
    n0 = W.monodisperse(M)
    x, sx = smol.integrate(t(U), t(V), lam, t(n0), 1e3, 1e-6, 1e-12, method="dp5",
                           precision="fp32x2")
    y, sy = smol.integrate(t(U), t(V), lam, t(n0), 1e3, 1e-6, 1e-12, method="dp5")
    err = normwise(x.cpu().numpy(), y.cpu().numpy())
    say(f"precision workload {name}: max rel err fp32x2 vs fp64 at t=1e3 = {err:.3e}; "
        f"steps {sx['n_accept']} vs {sy['n_accept']}")
    assert sx["status"] == 0 and sy["status"] == 0
    assert err < 1e-6


@pytest.mark.parametrize("M", [131072, 262144, 524288])
def test_fp32x2_integration_long_transform(smol, M):
    """DP5 with float-float convolutions at L = 2^18, 2^19 and 2^20 (monodisperse
    start, rank-3 kernel a = 0.45, lam = 0.005, t = 20): within the
    trajectory bar of the FP64 run, with the same step counts to within
    two."""
    U, V = W.brownian_rank3(M, 0.45)
    n0 = t(W.monodisperse(M))
    a, sa = smol.integrate(t(U), t(V), 0.005, n0, 20.0, 1e-6, 1e-12, method="dp5",
                           precision="fp32x2")
    b, sb = smol.integrate(t(U), t(V), 0.005, n0, 20.0, 1e-6, 1e-12, method="dp5")
    err = normwise(a.cpu().numpy(), b.cpu().numpy())
    say(f"fp32x2 DP5 M={M} t=20: accepted {sa['n_accept']} vs {sb['n_accept']}, "
        f"difference {err:.2e}")
    assert sa["status"] == 0 and sb["status"] == 0
    assert abs(sa["n_accept"] - sb["n_accept"]) <= 2 and err < 1e-6
