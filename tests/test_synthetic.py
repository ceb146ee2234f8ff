"""The shared input generator follows the published SplitMix64 definition."""
import numpy as np

import synthetic as syn


def test_splitmix64_reference_outputs():
    # First outputs of the SplitMix64 reference generator seeded with 1234567
    # (Steele, Lea & Flood 2014; the widely used reference implementation).
    out = syn.splitmix64(1234567, np.arange(5))
    assert [int(v) for v in out] == [6457827717110365317, 3203168211198807973,
                                     9817491932198370423, 4593380528125082431,
                                     16408922859458223821]


def test_counter_based_and_layout_free():
    a = syn.uniform(7, 3, 1000)
    b = syn.uniform(7, 3, 400, offset=600)
    assert np.array_equal(a[600:], b)
    assert a.min() >= 0.0 and a.max() < 1.0
    assert not np.array_equal(syn.uniform(7, 4, 10), a[:10])


def test_chunked_generation_matches_direct():
    n = (1 << 22) + 12345
    big = syn.uniform(9, 1, n)
    idx = np.array([0, 1, (1 << 22) - 1, 1 << 22, n - 1], dtype=np.uint64)
    direct = (syn.splitmix64(syn._key(9, 1), idx) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    assert np.array_equal(big[idx.astype(np.int64)], direct)
