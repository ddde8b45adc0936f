"""smol_rhs_noalloc (fixed device workspaces, no allocation in the call)
against smol_rhs on the same inputs: two calls in a row, the second smaller,
at the FP64 right-hand-side bar (max-norm relative error <= 1e-10), plus the
size limits it rejects."""
import ctypes

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


def _case(M, R, seed):
    U, V = W.random_factors(M, R, seed=seed)
    n = W.random_state(M, seed=seed + 1)
    return U, V, n


@pytest.mark.parametrize("sizes", [((65537, 4), (5000, 3)), ((4096, 3), (1, 1)),
                                   ((65536, 3), (65536, 3))])
def test_noalloc_matches_rhs_two_calls(smol, sizes):
    import torch
    for k, (M, R) in enumerate(sizes):
        say(f"noalloc call {k}: M={M} R={R}")
        U, V, n = _case(M, R, seed=17 * M + R + k)
        Ut, Vt, nt = t(U), t(V), t(n)
        out = torch.full_like(nt, float("nan"))
        before = torch.cuda.memory_allocated()
        smol.rhs_noalloc(Ut, Vt, 0.011, nt, out)
        assert torch.cuda.memory_allocated() == before
        got = out.cpu().numpy()
        ref = smol.rhs(Ut, Vt, 0.011, nt).cpu().numpy()
        assert np.isfinite(got).all()
        err = normwise(got, ref)
        say(f"  vs smol_rhs: {err:.2e}")
        assert err < TOL
        if M <= 5000:
            assert normwise(got, oracle.rhs(U, V, 0.011, n)) < TOL


def test_noalloc_config_state_against_oracle_samples(smol):
    """The single-large instance's kernel at M = 65536 (R = 3) on a spread
    state, sampled entries against the oracle's direct sums."""
    import torch
    M = 65536
    U, V = W.brownian_rank3(M, 0.45)
    n = W.exponential_start(M, 200.0)
    out = torch.empty(M, dtype=torch.float64, device="cuda:0")
    got = smol.rhs_noalloc(t(U), t(V), 0.005, t(n), out).cpu().numpy()
    idx = np.array([0, 1, 2, 100, 5000, M // 2, M - 1], dtype=np.int64)
    ref = oracle.rhs_entries(U, V, 0.005, n, idx)
    full = smol.rhs(t(U), t(V), 0.005, t(n)).cpu().numpy()
    assert np.abs(got[idx] - ref).max() / np.abs(full).max() < TOL


def test_noalloc_rejects_beyond_limits(smol):
    import torch
    lib = smol.lib()
    for M, R in ((65538, 3), (4096, 5)):
        U, V, n = (torch.ones((R, M), dtype=torch.float64, device="cuda:0"),
                   torch.ones((R, M), dtype=torch.float64, device="cuda:0"),
                   torch.ones(M, dtype=torch.float64, device="cuda:0"))
        out = torch.empty_like(n)
        rc = lib.smol_rhs_noalloc(M, R, U.data_ptr(), V.data_ptr(), 0.01, n.data_ptr(),
                                  out.data_ptr(), ctypes.c_void_p(0))
        assert rc == smol.EUNSUPPORTED
        with pytest.raises(ValueError):
            smol.rhs_noalloc(U, V, 0.01, n, out)
    n = torch.ones(8, dtype=torch.float64, device="cuda:0")
    rc = lib.smol_rhs_noalloc(8, 1, n.data_ptr(), n.data_ptr(), 0.01, n.data_ptr(), n.data_ptr(),
                              ctypes.c_void_p(0))
    assert rc == smol.EINVAL  # dndt aliases n
