"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method itself: it only builds kernel
factors U, V (alpha-major, shape (R, M), size s at column s-1), initial states
and the batch draws, from a SplitMix64 stream.  The workloads follow the
kernels the paper uses: the generalized Brownian kernel
(i/j)^a + (j/i)^a + c (Sec. 1 introductory example, Sec. 3.1 and 3.2) and the
constant kernel (Sec. 3.1), with the monodisperse start n_s(0) = delta_{s,1}
(Sec. 3.1, 3.2).
"""
import math

import numpy as np

MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea, Flood 2014) with 53-bit uniforms in [0, 1)."""

    def __init__(self, seed):
        self.state = seed & MASK64

    def next_u64(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self):
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniforms(self, n):
        """The next n uniforms (the same numbers as n calls of uniform()):
        the k-th state is seed + k * 0x9E3779B97F4A7C15 mod 2^64, so the
        whole run is mixed at once in wrapping uint64 arithmetic."""
        if n <= 0:
            return np.zeros(0)
        k = np.arange(1, n + 1, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = np.uint64(self.state) + k * np.uint64(0x9E3779B97F4A7C15)
            z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
            z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
            z = z ^ (z >> np.uint64(31))
        self.state = (self.state + n * 0x9E3779B97F4A7C15) & MASK64
        return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def sizes(M):
    return np.arange(1, M + 1, dtype=np.float64)


def brownian_rank3(M, a, c=2.0):
    """K_ij = (i/j)^a + (j/i)^a + c as U = (i^a, i^-a, 1), V = (j^-a, j^a, c)."""
    s = sizes(M)
    U = np.stack([s ** a, s ** -a, np.ones(M)])
    V = np.stack([s ** -a, s ** a, np.full(M, c)])
    return U, V


def brownian_rank2(M, a):
    """K_ij = (i/j)^a + (j/i)^a (no constant term)."""
    s = sizes(M)
    return np.stack([s ** a, s ** -a]), np.stack([s ** -a, s ** a])


def product_rank4(M, a):
    """K_ij = (i^a + j^a)(i^-a + j^-a), written out term by term as a rank-4
    product: U = (1, i^a, i^-a, 1), V = (1, j^-a, j^a, 1)."""
    s = sizes(M)
    one = np.ones(M)
    return np.stack([one, s ** a, s ** -a, one]), np.stack([one, s ** -a, s ** a, one])


def constant_kernel(M, value=1.0):
    return np.ones((1, M)), np.full((1, M), value)


def monodisperse(M):
    n = np.zeros(M)
    n[0] = 1.0
    return n


def exponential_start(M, s0):
    """n_s proportional to exp(-s/s0), scaled to unit mass sum_s s n_s = 1."""
    s = sizes(M)
    n = np.exp(-s / s0)
    return n / float(np.sum(s * n))


def random_state(M, seed, s0=None, decay=True):
    """Nonnegative test state: uniform(0.5, 1.5) times an exponential decay."""
    g = SplitMix64(seed)
    u = 0.5 + g.uniforms(M)
    if not decay:
        return u
    if s0 is None:
        s0 = max(2.0, M / 8.0)
    return u * np.exp(-sizes(M) / s0)


def random_factors(M, R, seed, lo=0.1, hi=2.0):
    """Random nonnegative (generally non-symmetric) factors."""
    g = SplitMix64(seed)
    U = lo + (hi - lo) * g.uniforms(R * M).reshape(R, M)
    V = lo + (hi - lo) * g.uniforms(R * M).reshape(R, M)
    return U, V


# ---------------------------------------------------------------------------
# The five benchmark workloads.
# ---------------------------------------------------------------------------

WORKLOADS = {
    "plain-small": dict(M=512, a=1.0 / 3.0, lam=0.01, method="bs3", rtol=1e-6, atol=1e-12,
                        t_end=50.0),
    "single-large": dict(M=65536, a=0.45, lam=0.005, method="dp5", rtol=1e-6, atol=1e-12,
                         t_end=1e4),
    "batched-sweep": dict(n_inst=256, method="bs3", rtol=1e-6, atol=1e-12, t_end=1e3, seed=0),
    "precision": dict(M=65536, a=0.3, lam=0.02, t_eval=1e3),
    "learned-proposer": dict(M=262144, a=0.4, lam=0.01, method="dp5", rtol=1e-6, atol=1e-12,
                             t_end=1e4),
}


def workload_instance(name):
    """(U, V, lam, n0) of a single-instance workload: rank-3 kernel
    (i/j)^a + (j/i)^a + 2, monodisperse start."""
    c = WORKLOADS[name]
    U, V = brownian_rank3(c["M"], c["a"])
    return U, V, c["lam"], monodisperse(c["M"])


def batch_draws(n_inst=256, seed=0, m_lo_log2=12, m_hi_log2=17):
    """Per-instance (M, a, lam, s0) of the batched sweep: M log-uniform in
    [2^12, 2^17], a uniform in [0.05, 0.5], lam log-uniform in [1e-3, 1e-1],
    s0 uniform in [1, 20]."""
    g = SplitMix64(seed)
    out = []
    span = m_hi_log2 - m_lo_log2
    for _ in range(n_inst):
        M = int(math.floor(2.0 ** (m_lo_log2 + span * g.uniform())))
        a = 0.05 + 0.45 * g.uniform()
        lam = 10.0 ** (-3.0 + 2.0 * g.uniform())
        s0 = 1.0 + 19.0 * g.uniform()
        out.append(dict(M=M, a=a, lam=lam, s0=s0))
    return out


def batch_instance(d):
    U, V = brownian_rank3(d["M"], d["a"])
    return U, V, d["lam"], exponential_start(d["M"], d["s0"])


# Layer shapes (fan_in, fan_out) of the step proposer network; the flat
# parameter vector holds each layer's weights (fan_out x fan_in, row-major)
# followed by its biases.
MLP_LAYERS = ((9, 64), (64, 64), (64, 1))


def mlp_init(seed):
    """Initial proposer parameters: weights uniform in +-sqrt(6/(fan_in+fan_out))
    (Glorot and Bengio 2010) from SplitMix64 draws, biases zero."""
    g = SplitMix64(seed)
    n = sum(i * o + o for i, o in MLP_LAYERS)
    p = np.zeros(n)
    off = 0
    for fan_in, fan_out in MLP_LAYERS:
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        p[off:off + fan_in * fan_out] = lim * (2.0 * g.uniforms(fan_in * fan_out) - 1.0)
        off += fan_in * fan_out + fan_out
    return p
