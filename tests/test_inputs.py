"""Input generators shared by both sides: the counter-based seeded normal
stream (the twin of the library's seed path of fctn_plan) against its
published definition and distribution, and its independence of the factor
split."""

import numpy as np

from workloads import seeded_normal_factors, factor_shapes_of


def test_seeded_stream_first_words_match_splitmix64_reference_values():
    # SplitMix64 with state 0: the first outputs are the published reference
    # values of the generator (state advanced by the golden-ratio increment
    # before mixing)
    M = (1 << 64) - 1

    def splitmix(state):
        state = (state + 0x9E3779B97F4A7C15) & M
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return state, z ^ (z >> 31)

    st, w0 = splitmix(0)
    st, w1 = splitmix(st)
    assert w0 == 0xE220A8397B1DCDAF
    assert w1 == 0x6E789E6AA1B965F4
    # the same two words drive the first Box-Muller pair of the stream
    u1 = ((w0 >> 11) + 1.0) * 2.0 ** -53
    u2 = (w1 >> 11) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    f = seeded_normal_factors(0, (2, 2, 2), (1, 1, 1))
    assert f[0].ravel()[0] == r * np.cos(2 * np.pi * u2)
    assert f[0].ravel()[1] == r * np.sin(2 * np.pi * u2)


def test_seeded_stream_is_standard_normal_and_deterministic():
    dims, ranks = (40, 30, 20), (6, 5, 4)
    a = seeded_normal_factors(123, dims, ranks)
    b = seeded_normal_factors(123, dims, ranks)
    c = seeded_normal_factors(124, dims, ranks)
    for x, y, sh in zip(a, b, factor_shapes_of(dims, ranks)):
        assert x.shape == sh
        np.testing.assert_array_equal(x, y)
    z = np.concatenate([x.ravel() for x in a])
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 0.2
    assert not np.array_equal(a[0], c[0])


def test_seeded_stream_is_one_stream_over_the_factors():
    # factor 2 continues where factor 1 stops: the draws depend on the
    # position in the concatenated factors only
    a = seeded_normal_factors(7, (5, 4, 3), (2, 2, 2))
    b = seeded_normal_factors(7, (5, 4, 3, 2), (2, 2, 2, 1, 1, 1))
    za = np.concatenate([x.ravel() for x in a])
    zb = np.concatenate([x.ravel() for x in b])
    np.testing.assert_array_equal(za, zb[:za.size])
