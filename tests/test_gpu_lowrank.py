"""smol_lowrank: low-rank factors of kernels given by a formula (adaptive cross
approximation on the GPU), measured against the oracle's kernel entries, and
the right-hand side with those factors against the oracle's direct sums
with the exact kernel (Sec. 3.1's free-molecular kernel has no exact
low-rank form)."""
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


def _errors(U, V, formula, M, p0=0.0, p1=0.0):
    """max entrywise relative and max-norm relative error of U^T V against
    the oracle's kernel matrix."""
    K = oracle.kernel_matrix(formula, M, p0, p1)
    A = U.cpu().numpy().T @ V.cpu().numpy()
    return float(np.max(np.abs(K - A) / np.abs(K))), float(np.abs(K - A).max() / np.abs(K).max())


@pytest.mark.parametrize("M", [1, 2, 7, 512, 4096])
def test_free_molecular_error_against_rank(smol, M):
    """Tightening tol raises the rank and lowers the error; the max-norm
    error stays within a small multiple of tol."""
    prev = None
    for tol in (1e-4, 1e-7, 1e-10, 1e-13):
        U, V, est = smol.lowrank(M, "free_molecular", tol=tol)
        rel, nw = _errors(U, V, oracle.K_FREE_MOLECULAR, M)
        say(f"free-molecular M={M} tol={tol:.0e}: rank {U.shape[0]}, estimate {est:.1e}, "
            f"max entrywise {rel:.2e}, max-norm {nw:.2e}")
        assert nw <= 100 * tol + 1e-14
        if prev is not None:
            assert U.shape[0] >= prev[0] and nw <= prev[1] * 1.01 + 1e-15
        prev = (U.shape[0], nw)
    assert prev[0] <= 32 and prev[1] < 1e-11


@pytest.mark.parametrize("a,c", [(1.0 / 3.0, 2.0), (0.45, 0.0)])
def test_exactly_low_rank_kernels(smol, a, c):
    """The Brownian kernel has rank 3 (2 without its constant term) and the
    constant kernel rank 1: the approximation stops there, exact to
    round-off."""
    M = 2000
    U, V, _ = smol.lowrank(M, "brownian", p0=a, p1=c, tol=1e-12)
    assert U.shape[0] == (3 if c else 2)
    rel, _ = _errors(U, V, oracle.K_BROWNIAN, M, a, c)
    assert rel < 1e-12
    U, V, _ = smol.lowrank(M, "constant", p0=2.5, tol=1e-12)
    assert U.shape[0] == 1
    assert _errors(U, V, oracle.K_CONSTANT, M, 2.5)[0] < 1e-15


@pytest.mark.parametrize("M", [4096, 32768])
def test_rhs_with_free_molecular_factors(smol, M):
    """S(n) with the factors: against the oracle's direct sums with the same
    factors (the right-hand side's own bar, 1e-10), and against the oracle's
    direct sums with the exact kernel, within the approximation error
    measured on sampled pairs."""
    U, V, est = smol.lowrank(M, "free_molecular", tol=1e-13)
    R = U.shape[0]
    g = W.SplitMix64(M)
    i = 1 + (g.uniforms(4000) * M).astype(np.int64)
    j = 1 + (g.uniforms(4000) * M).astype(np.int64)
    Uh, Vh = U.cpu().numpy(), V.cpu().numpy()
    approx = np.einsum("ak,ak->k", Uh[:, i - 1], Vh[:, j - 1])
    exact = oracle.kernel_entries(oracle.K_FREE_MOLECULAR, i, j)
    eps = float(np.max(np.abs(approx - exact) / exact))
    n = W.exponential_start(M, M / 20.0) + 1e-4 * W.random_state(M, seed=3, decay=False) / M
    got = smol.rhs(U, V, 0.01, t(n)).cpu().numpy()
    e_fac = normwise(got, oracle.rhs(Uh, Vh, 0.01, n))
    e_ker = normwise(got, oracle.rhs_kernel(oracle.K_FREE_MOLECULAR, 0.01, n))
    say(f"free-molecular M={M}: rank {R}, sampled entrywise error {eps:.2e}, RHS vs factors "
        f"{e_fac:.2e}, RHS vs exact kernel {e_ker:.2e}")
    assert e_fac < 1e-10
    assert e_ker < 10 * eps + 1e-10


def test_lowrank_arguments(smol):
    import ctypes
    lib = smol.lib()
    p = ctypes.c_void_p(16)
    r = ctypes.c_int32()
    assert lib.smol_lowrank(0, 3, 0.0, 0.0, 1e-8, 8, p, ctypes.c_void_p(32), ctypes.byref(r),
                            None, None) == smol.EINVAL
    assert lib.smol_lowrank(10, 9, 0.0, 0.0, 1e-8, 8, p, ctypes.c_void_p(32), ctypes.byref(r),
                            None, None) == smol.EINVAL
    assert lib.smol_lowrank(10, 3, 0.0, 0.0, 1e-8, 33, p, ctypes.c_void_p(32), ctypes.byref(r),
                            None, None) == smol.EINVAL
    assert lib.smol_lowrank(10, 3, 0.0, 0.0, -1.0, 8, p, ctypes.c_void_p(32), ctypes.byref(r),
                            None, None) == smol.EINVAL
    assert lib.smol_lowrank(10, 3, 0.0, 0.0, 1e-8, 8, p, p, ctypes.byref(r), None,
                            None) == smol.EINVAL
