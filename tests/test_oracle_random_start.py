"""The oracle's counter-based start block: Philox4x32-10 against the
published known-answer vectors of the generator (Salmon et al., SC 2011, and
the Random123 distribution that accompanies it), the 53-bit uniforms against
their definition at the ends of the range, and the Box-Muller deviates
against the standard normal law (moments, and a Kolmogorov-Smirnov test
against scipy's normal CDF)."""
import numpy as np
import scipy.stats as ss

from oracle import random_start as rs


def test_philox_known_answer_vectors():
    M = 0xFFFFFFFF
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
        ((M, M, M, M), (M, M), (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
        ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
         (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
    ]
    for ctr, key, out in cases:
        got = rs.philox4x32_10(np.array(ctr, dtype=np.uint64), np.array(key, dtype=np.uint64))
        assert [int(v) for v in got] == list(out)


def test_uniforms_cover_the_53_bit_range():
    assert rs.uniforms53(0, 0) == 0.0
    assert rs.uniforms53(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert rs.uniforms53(0, 1 << 11) == 2.0 ** -53
    assert rs.uniforms53(1, 0) == 2.0 ** -32


def test_start_block_is_standard_normal_and_reproducible():
    X = rs.start_block(20001, 7, 3, 12345)
    assert X.shape == (20001, 7) and np.isfinite(X).all()
    v = X.ravel()
    assert abs(v.mean()) < 0.02 and abs(v.var() - 1.0) < 0.02
    assert ss.kstest(v, "norm").pvalue > 1e-3
    # any column (element, seed) is its own stream
    assert np.array_equal(X, rs.start_block(20001, 7, 3, 12345))
    assert not np.allclose(X[:, 0], rs.start_block(20001, 7, 4, 12345)[:, 0])
    assert not np.allclose(X[:, 0], rs.start_block(20001, 7, 3, 12346)[:, 0])
    # an odd N_g's last row is the cosine deviate of its pair
    Y = rs.start_block(20002, 7, 3, 12345)
    assert np.array_equal(Y[:20001], X)
