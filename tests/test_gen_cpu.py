"""CPU checks of the seeded input generators (tqgen)."""
import numpy as np

import tqgen


def bits_of(words):
    return np.unpackbits(np.ascontiguousarray(words).view(np.uint8), bitorder="little")


def test_splitmix_reference_value():
    # SplitMix64 with state 0: the first output is the published 0xE220A8397B1DCDAF
    assert tqgen.rand64_scalar(0, 0) == 0xE220A8397B1DCDAF
    assert int(tqgen.rand64(0, np.array([0], dtype=np.uint64))[0]) == 0xE220A8397B1DCDAF


def test_determinism_and_random_access():
    bs = tqgen.large_set(2, n=3, r_bits=64 * 300 + 5)
    a = bs.words(1)
    assert np.array_equal(a, tqgen.large_set(2, n=3, r_bits=64 * 300 + 5).words(1))
    assert np.array_equal(bs.words(1, 17, 123), a[17:123])
    ms = tqgen.rle_set(3, n=2, r_bits=1 << 18)
    m = ms.words(1)
    for lo, hi in ((0, 1), (5, 77), (4000, 4096)):
        assert np.array_equal(ms.words(1, lo, hi), m[lo:hi])


def test_bernoulli_density():
    bs = tqgen.bernoulli_fixed(9, 2, 1 << 20, 0.05)
    d = bits_of(bs.words(0)).mean()
    assert abs(d - 0.05) < 5 * np.sqrt(0.05 * 0.95 / (1 << 20))


def test_markov_run_lengths():
    ms = tqgen.markov_fixed(11, 1, 1 << 24, mean_ones=64.0, mean_zeros=4096.0)
    b = bits_of(ms.words(0)).astype(np.int8)
    edges = np.flatnonzero(np.diff(b)) + 1
    runs = np.diff(np.concatenate([[0], edges, [b.size]]))
    vals = b[np.concatenate([[0], edges])]
    ones, zeros = runs[vals == 1][1:-1], runs[vals == 0][1:-1]
    assert abs(ones.mean() / 64.0 - 1) < 0.05
    assert abs(zeros.mean() / 4096.0 - 1) < 0.1
    assert abs(b.mean() / (64 / 4160) - 1) < 0.15


def test_markov_general_flip_regime():
    # mean ones-run 1 and density near 1/2: the coupling has "flip" positions
    ms = tqgen.markov_density_runlength(5, 1, 64 * 2000, density=0.45, mean_ones=1.0)
    w = ms.words(0)
    assert np.array_equal(ms.words(0, 999, 1500), w[999:1500])
    b = bits_of(w)
    assert not (b[1:] & b[:-1]).any()          # ones-runs of length exactly 1
    assert abs(b.mean() - 0.45) < 0.02


def test_exhaustive_fixture():
    n = 6
    for j in range(n):
        b = bits_of(tqgen.exhaustive_words(j, n))
        assert np.array_equal(b, (np.arange(64) >> j) & 1)


def test_workload_shapes():
    qs = tqgen.selector_queries(4, count=200)
    assert all(2 <= q.n <= 4096 and 1 <= q.theta <= q.n for q in qs)
    sq = tqgen.serving_queries(5, count=100)
    for q in sq:
        assert len(set(q.members)) == len(q.members)
        assert 1 <= q.theta <= len(q.members)
        assert all(0 <= m < 8192 for m in q.members)
    assert all(a.arrival_s < b.arrival_s for a, b in zip(sq, sq[1:]))
