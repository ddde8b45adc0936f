"""The seeded input generator: SplitMix64's published reference outputs, and
the vectorised uniforms equal to one-at-a-time draws (CPU only)."""
import numpy as np

import workloads as W


def test_splitmix64_reference_outputs():
    # first outputs of SplitMix64 from state 0 (Steele, Lea and Flood's
    # generator as published in Vigna's reference implementation)
    g = W.SplitMix64(0)
    assert [g.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                0x06C45D188009454F]


def test_vectorised_uniforms_equal_scalar_draws():
    for seed in (0, 1, 12345, 2 ** 64 - 1):
        a, b = W.SplitMix64(seed), W.SplitMix64(seed)
        x = np.array([a.uniform() for _ in range(700)])
        y = np.concatenate([b.uniforms(1), b.uniforms(400), b.uniforms(299)])
        assert np.array_equal(x, y)
        assert a.state == b.state
        assert ((0.0 <= y) & (y < 1.0)).all()
