"""Pins of the oracle's counter-based generator (Philox4x64-10, Salmon et al.
SC'11) against numpy's independent implementation of the same generator,
and of the multiply-high index map it feeds."""
import numpy as np
import pytest

MASK = (1 << 64) - 1


def _numpy_block(ctr, key):
    """numpy's Philox advances its 256-bit counter before each block, so the
    block for counter c is the first output of a generator started at c - 1."""
    c = sum(int(w) << (64 * i) for i, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = [(c >> (64 * i)) & MASK for i in range(4)]
    g = np.random.Philox(counter=np.array(words, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return g.random_raw(4)


def test_philox_matches_numpy_on_random_counters_and_keys(orc):
    rng = np.random.default_rng(7)
    for _ in range(400):
        ctr = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=4, dtype=np.uint64)
        key = rng.integers(0, 2 ** 63, size=2, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=2, dtype=np.uint64)
        assert np.array_equal(orc.philox4x64_10(ctr, key), _numpy_block(ctr, key))


def test_philox_matches_numpy_on_the_hypothesis_counters(orc):
    key = [0x5EED0002, 17]
    for j in (0, 1, 255, 1023, 4095):
        for r in (0, 5, 11):
            for b in (0, 1, 15):
                ctr = [j, r, b, 0]
                assert np.array_equal(orc.philox4x64_10(ctr, key), _numpy_block(ctr, key))


def test_philox_zero_counter_zero_key_differs_from_input(orc):
    out = orc.philox4x64_10([0, 0, 0, 0], [0, 0])
    assert np.any(out != 0)
    # counter increments give unrelated blocks
    out2 = orc.philox4x64_10([1, 0, 0, 0], [0, 0])
    assert np.count_nonzero(out ^ out2) == 4


@pytest.mark.parametrize("M", [3, 1000, 307200])
def test_multiply_high_index_map_is_in_range_and_uniform(M):
    g = np.random.Philox(key=np.array([1, 2], dtype=np.uint64))
    w = g.random_raw(200000)
    k = np.array([(int(x) * M) >> 64 for x in w[:20000]])
    assert k.min() >= 0 and k.max() < M
    nb = min(M, 10)
    bins = np.bincount((k * nb) // M, minlength=nb)
    expected = len(k) / nb
    chi2 = ((bins - expected) ** 2 / expected).sum()
    assert chi2 < 40  # 9 dof: p ~ 5e-6
