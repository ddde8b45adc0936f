"""Pins of the oracle's formula kernels (Sec. 3.1) and of its right-hand side
with K_ij evaluated from a formula for every pair (CPU only): the Brownian
formula against its exact rank-3 factors, the constant kernel against rank 1,
hand values and the degree-1/6 homogeneity of the free-molecular kernel, the
M = 2 hand-expanded right-hand side, and the mass balance."""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def test_brownian_formula_equals_rank3_factors():
    M = 300
    n = W.random_state(M, seed=4)
    for a, c in ((1.0 / 3.0, 2.0), (0.45, 0.0), (0.1, 1.5)):
        U, V = W.brownian_rank3(M, a, c)
        ref = oracle.rhs(U, V, 0.02, n)
        got = oracle.rhs_kernel(oracle.K_BROWNIAN, 0.02, n, p0=a, p1=c)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_constant_formula_equals_rank1():
    M = 200
    n = W.random_state(M, seed=5)
    U, V = W.constant_kernel(M, 1.7)
    ref = oracle.rhs(U, V, 0.05, n)
    got = oracle.rhs_kernel(oracle.K_CONSTANT, 0.05, n, p0=1.7)
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-15 * np.abs(ref).max())


def test_free_molecular_hand_values():
    """K_ij = (i^(1/3) + j^(1/3))^2 sqrt(1/i + 1/j) at pairs worked out by hand."""
    i = np.array([1, 1, 8, 1, 27, 8])
    j = np.array([1, 8, 8, 27, 27, 64])
    want = np.array([4.0 * math.sqrt(2.0),            # (1+1)^2 sqrt(2)
                     9.0 * math.sqrt(9.0 / 8.0),       # (1+2)^2 sqrt(1 + 1/8)
                     8.0,                              # (2+2)^2 sqrt(1/4)
                     16.0 * math.sqrt(28.0 / 27.0),    # (1+3)^2 sqrt(1 + 1/27)
                     36.0 * math.sqrt(2.0 / 27.0),     # (3+3)^2 sqrt(2/27)
                     36.0 * math.sqrt(9.0 / 64.0)])    # (2+4)^2 sqrt(1/8 + 1/64)
    got = oracle.kernel_entries(oracle.K_FREE_MOLECULAR, i, j)
    np.testing.assert_allclose(got, want, rtol=1e-15)


def test_free_molecular_homogeneity_and_symmetry():
    """Scaling both sizes by 8 multiplies K by 8^(2/3 - 1/2) = sqrt(2)."""
    g = W.SplitMix64(8)
    i = 1 + (g.uniforms(500) * 5000).astype(np.int64)
    j = 1 + (g.uniforms(500) * 5000).astype(np.int64)
    k = oracle.kernel_entries(oracle.K_FREE_MOLECULAR, i, j)
    np.testing.assert_allclose(oracle.kernel_entries(oracle.K_FREE_MOLECULAR, 8 * i, 8 * j),
                               math.sqrt(2.0) * k, rtol=1e-14)
    np.testing.assert_array_equal(oracle.kernel_entries(oracle.K_FREE_MOLECULAR, j, i), k)


@pytest.mark.parametrize("formula", [oracle.K_FREE_MOLECULAR, oracle.K_BROWNIAN])
def test_formula_rhs_m2_hand_expanded(formula):
    """M = 2 from Eq. (4): S1 = -n1 (K11 n1 + K12 n2) + 2 lam K22 n2^2
    + 2 lam K12 n1 n2, S2 = K11 n1^2 / 2 - (1 + lam) n2 (K21 n1 + K22 n2)."""
    K = oracle.kernel_matrix(formula, 2, p0=0.3, p1=1.0)
    n1, n2, lam = 0.6, 0.45, 0.2
    S = oracle.rhs_kernel(formula, lam, np.array([n1, n2]), p0=0.3, p1=1.0)
    S1 = -n1 * (K[0, 0] * n1 + K[0, 1] * n2) + 2 * lam * K[1, 1] * n2 ** 2 \
        + 2 * lam * K[0, 1] * n1 * n2
    S2 = 0.5 * K[0, 0] * n1 ** 2 - (1 + lam) * n2 * (K[1, 0] * n1 + K[1, 1] * n2)
    np.testing.assert_allclose(S, [S1, S2], rtol=1e-14)


@pytest.mark.parametrize("lam", [0.0, 0.05])
def test_free_molecular_mass_balance(lam):
    """sum_s s S_s = -(1/2) sum_{i,j<=M, i+j>M} (i+j) K_ij n_i n_j."""
    M = 120
    n = W.random_state(M, seed=12, s0=40.0)
    S = oracle.rhs_kernel(oracle.K_FREE_MOLECULAR, lam, n)
    K = oracle.kernel_matrix(oracle.K_FREE_MOLECULAR, M)
    s = np.arange(1, M + 1)
    I, J = np.meshgrid(s, s, indexing="ij")
    F = 0.5 * np.sum(((I + J) * K * np.outer(n, n))[(I + J) > M])
    assert abs(np.sum(s * S) + F) <= 1e-13 * (np.sum(s * np.abs(S)) + F)
