"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against something fixed by the paper or by
mathematics: the exhaustive-combination fixture (every input combination
appears at a known position, so the count is popcount of the position), the
Looped recurrence of section 4.5 evaluated with whole-bitmap AND/OR, the
sorting view of section 4.4.1 (the T-th largest input bit is the threshold),
library reductions (OR, AND, XOR), and identities of section 2.3.
"""
import os

import numpy as np
import pytest

import tqgen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.txt")


def popcount_int(p: int) -> int:
    return bin(p).count("1")


def unpack(words: np.ndarray, r_bits: int) -> np.ndarray:
    return np.unpackbits(np.ascontiguousarray(words).view(np.uint8), bitorder="little")[:r_bits]


def pack(bits: np.ndarray) -> np.ndarray:
    bits = np.asarray(bits, dtype=np.uint8)
    pad = (-bits.size) % 64
    if pad:
        bits = np.concatenate([bits, np.zeros(pad, dtype=np.uint8)])
    return np.packbits(bits, bitorder="little").view("<u8").astype(np.uint64)


def tail_mask_words(r_bits: int) -> np.ndarray:
    return pack(np.ones(r_bits, dtype=np.uint8))


def rand_bitmaps(rng, n, r_bits, p=0.3):
    nw = (r_bits + 63) // 64
    out = []
    for _ in range(n):
        bits = (rng.random(nw * 64) < p).astype(np.uint8)
        out.append(pack(bits))           # garbage past r on purpose
    return out


# ------------------------------------------------------- exhaustive fixture
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10])
def test_exhaustive_threshold(orc, n):
    r = 1 << n
    bm = [tqgen.exhaustive_words(j, n) for j in range(n)]
    pc = np.array([popcount_int(p) for p in range(r)])
    for theta in range(0, n + 2):
        got = unpack(orc.threshold(bm, r, theta), r)
        assert np.array_equal(got, (pc >= theta).astype(np.uint8)), theta


@pytest.mark.parametrize("n", [4, 7, 9])
def test_exhaustive_symmetric(orc, n):
    r = 1 << n
    rng = np.random.default_rng(n)
    bm = [tqgen.exhaustive_words(j, n) for j in range(n)]
    pc = np.array([popcount_int(p) for p in range(r)])
    for _ in range(5):
        f = rng.integers(0, 2, n + 1).astype(np.uint8)
        got = unpack(orc.symmetric(bm, r, f), r)
        assert np.array_equal(got, f[pc])


def test_exhaustive_ragged_tail(orc):
    # r not a multiple of 64: positions >= r must come out zero
    n = 7
    r = (1 << n) - 37
    bm = [tqgen.exhaustive_words(j, n) for j in range(n)]
    pc = np.array([popcount_int(p) for p in range(1 << n)])
    for theta in (0, 1, 3, 7):
        out = orc.threshold(bm, r, theta)
        allbits = np.unpackbits(out.view(np.uint8), bitorder="little")
        assert np.array_equal(allbits[:r], (pc[:r] >= theta).astype(np.uint8))
        assert not allbits[r:].any()


# ------------------------------------------------ independent algorithms
def looped(bitmaps, theta):
    """Looped recurrence (section 4.5): C_j holds the j-threshold of the
    inputs seen so far; adding input b turns C_j into C_j OR (C_{j-1} AND b)."""
    n = len(bitmaps)
    if theta == 0:
        return np.full_like(bitmaps[0], np.uint64(0xFFFFFFFFFFFFFFFF))
    if theta > n:
        return np.zeros_like(bitmaps[0])
    C = [np.zeros_like(bitmaps[0]) for _ in range(theta + 1)]
    C[0] = np.full_like(bitmaps[0], np.uint64(0xFFFFFFFFFFFFFFFF))
    for b in bitmaps:
        for j in range(theta, 0, -1):
            C[j] = C[j] | (C[j - 1] & b)
    return C[theta]


def test_looped_recurrence_all_thetas(orc):
    rng = np.random.default_rng(7)
    r = 64 * 40 + 11
    for n in (1, 2, 3, 6, 13, 31):
        bm = rand_bitmaps(rng, n, r, p=rng.uniform(0.05, 0.9))
        mask = tail_mask_words(r)
        for theta in range(0, n + 2):
            assert np.array_equal(orc.threshold(bm, r, theta), looped(bm, theta) & mask), (n, theta)


def test_sorting_view(orc):
    # T-th largest of the N input bits at each position is the T-threshold
    rng = np.random.default_rng(11)
    r = 3000
    n = 23
    bm = rand_bitmaps(rng, n, r, p=0.4)
    bits = np.stack([unpack(b, r) for b in bm])          # (n, r)
    srt = -np.sort(-bits.astype(np.int8), axis=0)        # descending per position
    for theta in range(1, n + 1):
        want = pack(srt[theta - 1].astype(np.uint8))
        assert np.array_equal(orc.threshold(bm, r, theta), want), theta


def test_library_reductions(orc):
    rng = np.random.default_rng(3)
    r = 64 * 100 + 5
    mask = tail_mask_words(r)
    for n in (1, 2, 9, 40):
        bm = rand_bitmaps(rng, n, r, p=0.5)
        st = np.stack(bm)
        assert np.array_equal(orc.threshold(bm, r, 1), np.bitwise_or.reduce(st, axis=0) & mask)
        assert np.array_equal(orc.threshold(bm, r, n), np.bitwise_and.reduce(st, axis=0) & mask)
        assert np.array_equal(orc.symmetric(bm, r, orc.truth_parity(n)),
                              np.bitwise_xor.reduce(st, axis=0) & mask)


# ---------------------------------------------------------------- identities
def test_monotone_and_sum_identity(orc):
    rng = np.random.default_rng(5)
    r = 64 * 64 + 17
    n = 19
    bm = rand_bitmaps(rng, n, r, p=0.35)
    mask = tail_mask_words(r)
    outs = [orc.threshold(bm, r, t) for t in range(1, n + 1)]
    for a, b in zip(outs, outs[1:]):
        assert not (b & ~a).any()                      # T_{t+1} subset of T_t
    total = sum(int(np.unpackbits((x & mask).view(np.uint8)).sum()) for x in bm)
    assert sum(int(np.unpackbits(o.view(np.uint8)).sum()) for o in outs) == total


def test_permutation_and_complement(orc):
    rng = np.random.default_rng(9)
    r = 64 * 30 + 3
    n = 12
    bm = rand_bitmaps(rng, n, r, p=0.2)
    mask = tail_mask_words(r)
    perm = [bm[i] for i in rng.permutation(n)]
    neg = [~b for b in bm]
    for t in range(0, n + 2):
        a = orc.threshold(bm, r, t)
        assert np.array_equal(a, orc.threshold(perm, r, t))
        # complement identity of section 2.3; the printed N-T is off by one,
        # the identity that holds is  not T_t(B) = T_{N-t+1}(not B)
        if 1 <= t <= n:
            assert np.array_equal(~a & mask, orc.threshold(neg, r, n - t + 1))


def test_padding_rule(orc):
    # section 4.4.5: an (N, T) circuit answers (N', T') with N' <= N and
    # T' in [T-(N-N'), T] by adding T-T' all-ones and the rest all-zeros inputs
    rng = np.random.default_rng(13)
    r = 64 * 12 + 9
    nprime = 6
    bm = rand_bitmaps(rng, nprime, r, p=0.45)
    ones = np.full_like(bm[0], np.uint64(0xFFFFFFFFFFFFFFFF))
    zeros = np.zeros_like(bm[0])
    for N, T in ((8, 4), (10, 7), (16, 8)):
        for tp in range(max(1, T - (N - nprime)), T + 1):
            pad = [ones] * (T - tp) + [zeros] * (N - nprime - (T - tp))
            assert np.array_equal(orc.threshold(bm + pad, r, T), orc.threshold(bm, r, tp))


def test_weights_by_replication(orc):
    # section 2.3: integer weight w_i == w_i copies of input i
    rng = np.random.default_rng(17)
    r = 1000
    bm = rand_bitmaps(rng, 4, r, p=0.5)
    w = [3, 1, 2, 1]
    rep = [b for b, k in zip(bm, w) for _ in range(k)]
    bits = np.stack([unpack(b, r) for b in bm]).astype(np.int64)
    wsum = (bits * np.array(w)[:, None]).sum(axis=0)
    for t in range(1, 8):
        assert np.array_equal(unpack(orc.threshold(rep, r, t), r), (wsum >= t).astype(np.uint8))


# --------------------------------------------------------- sampled columns
def test_cols_match_full(orc):
    rng = np.random.default_rng(21)
    r = 64 * 50 + 1
    n = 11
    bm = rand_bitmaps(rng, n, r)
    cols = np.array([0, 3, 17, 49, 50])
    words = np.stack([b[cols] for b in bm])
    for t in (1, 4, 11):
        assert np.array_equal(orc.threshold_cols(words, cols, r, t), orc.threshold(bm, r, t)[cols])
    f = rng.integers(0, 2, n + 1)
    assert np.array_equal(orc.symmetric_cols(words, cols, r, f), orc.symmetric(bm, r, f)[cols])


# ---------------------------------------------------------- paper examples
def _golden(kind):
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith(kind + " "):
                yield [x.strip() for x in line[len(kind) + 1:].split(";")]


def test_golden_layout():
    for pos, hexbytes in _golden("layout"):
        positions = [int(x) for x in pos.split(",")]
        bits = np.zeros(64, dtype=np.uint8)
        bits[positions] = 1
        w = pack(bits)
        want = bytes(int(h, 16) for h in hexbytes.split())
        assert w.view(np.uint8)[:len(want)].tobytes() == want
        # the fixture generator packs bits the same way
        e = tqgen.exhaustive_words(0, 6)          # bit p = p & 1
        assert int(e[0]) == 0xAAAAAAAAAAAAAAAA


def test_golden_rle(orc):
    for r, zeros, runs, stream in _golden("rle"):
        r, zeros, runs = int(r), int(zeros), int(runs)
        bits = np.zeros(r, dtype=np.uint8)
        bits[zeros:] = 1
        dense = pack(bits)
        s = orc.rle_encode(dense, r)
        assert [int(x) for x in s] == [int(x, 16) for x in stream.split()]
        assert orc.run_count(dense, r) == runs
        assert np.array_equal(orc.rle_decode(s, r), dense)


def test_golden_allfill(orc):
    for n, r, pattern, theta, want in _golden("allfill"):
        n, r, theta = int(n), int(r), int(theta)
        pat = [int(x) for x in pattern.split(",")]
        bm = [pack(np.full(r, v, dtype=np.uint8)) for v in pat]
        assert sum(orc.run_count(b, r) for b in bm) == n
        out = orc.threshold(bm, r, theta)
        expect = pack(np.full(r, 1 if want == "ones" else 0, dtype=np.uint8))
        assert np.array_equal(out, expect)
        # one marker, plus the ragged tail word as a literal when it holds ones
        assert len(orc.rle_encode(out, r)) == (2 if want == "ones" and r % 64 else 1)


# ----------------------------------------------------------------- RLE codec
def test_rle_roundtrip_and_canonical(orc):
    rng = np.random.default_rng(23)
    for trial in range(20):
        r = int(rng.integers(1, 64 * 200))
        ms = tqgen.markov_fixed(trial, 1, r, mean_ones=float(rng.integers(1, 300)),
                                mean_zeros=float(rng.integers(1, 3000)))
        dense = ms.words(0)
        s = orc.rle_encode(dense, r)
        dec = orc.rle_decode(s, r)
        assert np.array_equal(dec, dense & tail_mask_words(r)[:dense.size])
        assert np.array_equal(orc.rle_encode(dec, r), s)             # canonical is a fixed point
        # canonical structure: no clean literal; markers split only where required
        pos, w = 0, 0
        prev_kind = None
        while pos < len(s):
            m = int(s[pos]); pos += 1
            fill, run, lits = m & 1, (m >> 1) & 0xFFFFFFFF, m >> 33
            if pos > 1:
                assert run > 0                       # only the first marker may have an empty fill
                assert prev_kind == "dirty" or prev_kind != fill
            for k in range(lits):
                x = int(s[pos + k])
                assert x != 0 and x != 0xFFFFFFFFFFFFFFFF
            prev_kind = "dirty" if lits else fill
            pos += lits
            w += run + lits
        assert w == (r + 63) // 64


def test_rle_noncanonical_accepted(orc):
    r = 64 * 10
    dense = np.zeros(10, dtype=np.uint64)
    dense[3] = 5
    dense[4:7] = np.uint64(0xFFFFFFFFFFFFFFFF)
    mk = lambda f, run, lits: (f & 1) | (run << 1) | (lits << 33)
    # a split zero run, a clean word stored as a literal, an empty marker
    s = np.array([mk(0, 2, 0), mk(0, 1, 2), 5, 0xFFFFFFFFFFFFFFFF, mk(0, 0, 0), mk(1, 2, 0),
                  mk(0, 3, 0)], dtype=np.uint64)
    assert np.array_equal(orc.rle_decode(s, r), dense)
    assert np.array_equal(orc.rle_decode(orc.rle_encode(dense, r), r), dense)
    assert len(orc.rle_encode(dense, r)) < len(s)


def test_rle_malformed_rejected(orc):
    r = 64 * 10
    mk = lambda f, run, lits: (f & 1) | (run << 1) | (lits << 33)
    bad = [
        [mk(0, 9, 0)],                      # covers too few words
        [mk(0, 11, 0)],                     # covers too many
        [mk(0, 8, 3), 1, 2, 3],             # literals past the universe
        [mk(0, 8, 2), 1],                   # literals past the stream
        [],                                 # empty stream for a non-empty bitmap
    ]
    for s in bad:
        with pytest.raises(ValueError):
            orc.rle_decode(np.array(s, dtype=np.uint64), r)


def test_rle_encode_ignores_tail(orc):
    """Bits at positions >= r are not part of the bitmap: a dense input with
    garbage past r encodes to the stream of its masked words, and the tail
    word is classified (zero fill, ones fill, literal) after masking."""
    rng = np.random.default_rng(29)
    for r in (1, 37, 64 * 3 + 1, 64 * 9 + 63):
        nw = (r + 63) // 64
        mask = tail_mask_words(r)
        for tail in ("zeros", "ones", "mixed"):
            bits = np.zeros(nw * 64, dtype=np.uint8)
            bits[:r] = {"zeros": 0, "ones": 1}.get(tail, 0)
            if tail == "mixed":
                bits[:r] = rng.random(r) < 0.5
            clean = pack(bits)
            dirty = clean | (~mask & np.uint64(0xA5A5A5A5A5A5A5A5))
            s = orc.rle_encode(dirty, r)
            assert np.array_equal(s, orc.rle_encode(clean, r)), (r, tail)
            assert np.array_equal(orc.rle_decode(s, r), clean), (r, tail)
            if tail == "zeros":
                assert len(s) == 1 and int(s[0]) == (nw << 1)
            if tail == "ones":
                # full words are a ones fill; a ragged last word holds ones
                # below r only, so it is a literal (an empty fill has fill bit 0)
                full = r // 64
                assert int(s[0]) == ((1 if full else 0) | (full << 1) | ((nw - full) << 33))


def test_run_count(orc):
    assert orc.run_count(np.zeros(2, dtype=np.uint64), 100) == 1
    alt = np.full(2, np.uint64(0xAAAAAAAAAAAAAAAA))
    assert orc.run_count(alt, 128) == 128


# -------------------------------------------- consumers of a result bitmap
@pytest.mark.parametrize("n", [1, 3, 6, 10])
def test_count_closed_form(orc, n):
    """On the exhaustive fixture every combination of the N inputs appears
    once, so |T_theta| = sum_{c >= theta} C(N, c), and ANDed with input 0 (a
    filter) sum_{c >= theta} C(N-1, c-1); a symmetric f counts
    sum_c f(c) C(N, c)."""
    from math import comb
    r = 1 << n
    bm = [tqgen.exhaustive_words(j, n) for j in range(n)]
    for theta in range(0, n + 2):
        res = orc.threshold(bm, r, theta)
        _, cnt = orc.consume(res, r)
        assert cnt == sum(comb(n, c) for c in range(theta, n + 1)), theta
        _, cnt_f = orc.consume(res, r, bm[0])
        assert cnt_f == sum(comb(n - 1, c - 1) for c in range(max(theta, 1), n + 1)), theta
    rng = np.random.default_rng(n)
    f = rng.integers(0, 2, n + 1).astype(np.uint8)
    _, cnt = orc.consume(orc.symmetric(bm, r, f), r)
    assert cnt == sum(int(f[c]) * comb(n, c) for c in range(n + 1))


def test_count_against_numpy(orc):
    """Positions below r only, against numpy's bit unpacking; the filter
    against numpy's AND."""
    rng = np.random.default_rng(33)
    for r in (1, 63, 64, 65, 1000, 64 * 77 + 5):
        a, f = rand_bitmaps(rng, 2, r, p=0.4)
        got, cnt = orc.consume(a, r, f)
        assert np.array_equal(got, a & f)
        assert cnt == int(unpack(a & f, r).sum()), r
        assert orc.count(a, r) == int(unpack(a, r).sum())
    assert orc.count(np.zeros(1, dtype=np.uint64), 0) == 0


# -------------------------------------------------------- weighted inputs
def subset_weight_counts(weights):
    """Number of subsets of the inputs with each total weight (a DP over the
    weights, independent of any bitmap)."""
    tot = sum(weights)
    ways = [0] * (tot + 1)
    ways[0] = 1
    for w in weights:
        for s in range(tot, w - 1, -1):
            ways[s] += ways[s - w]
    return ways


@pytest.mark.parametrize("weights", [[1], [3, 1, 2], [5, 5, 1, 7, 2, 2], [1, 2, 4, 8, 16, 32, 64, 100]])
def test_weighted_exhaustive(orc, weights):
    """Weighted threshold on the exhaustive fixture: the number of positions
    with weight sum >= theta equals the number of input subsets of weight >=
    theta; each position's bit equals the weight sum of its bits."""
    n = len(weights)
    r = 1 << n
    bm = [tqgen.exhaustive_words(j, n) for j in range(n)]
    ways = subset_weight_counts(weights)
    wsum_at = np.array([sum(w for j, w in enumerate(weights) if (p >> j) & 1) for p in range(r)])
    for theta in sorted({0, 1, 2, max(weights), sum(weights) // 2, sum(weights), sum(weights) + 1}):
        res = orc.weighted_threshold(bm, weights, r, theta)
        assert orc.count(res, r) == sum(ways[theta:]), theta
        assert np.array_equal(unpack(res, r), (wsum_at >= theta).astype(np.uint8)), theta


def test_weighted_equals_replication(orc):
    """Section 2.3: a positive integer weight w is the same as w copies of
    the input (the unweighted oracle on replicated inputs); weight 0 drops
    the input."""
    rng = np.random.default_rng(18)
    r = 64 * 40 + 9
    bm = rand_bitmaps(rng, 6, r, p=0.35)
    w = [4, 0, 1, 3, 2, 1]
    rep = [b for b, k in zip(bm, w) for _ in range(k)]
    for t in range(0, sum(w) + 2):
        assert np.array_equal(orc.weighted_threshold(bm, w, r, t), orc.threshold(rep, r, t)), t
