"""Dense threshold / symmetric queries on the GPU against the CPU oracle.

Element-by-element comparison of whole outputs at sizes the oracle finishes
in seconds (several tiles, ragged tails) and at the full large
configuration, and the error paths of the ABI.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import tqgen
from gpuhelp import dev_pool, empty_words, tail_mask, to_dev, to_host
from paper_1402_4073_amd import binding as tq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tq.tq_create(0)
    yield c
    tq.tq_destroy(c)


def run_threshold(ctx, rows, r_bits, theta):
    nw = (r_bits + 63) // 64
    out = empty_words(nw)
    tq.tq_threshold(ctx, rows, r_bits, theta, out)
    assert tq.tq_ctx_check(ctx) == 0
    return to_host(out)[:nw]


def run_symmetric(ctx, rows, r_bits, truth):
    nw = (r_bits + 63) // 64
    out = empty_words(nw)
    tq.tq_symmetric(ctx, rows, r_bits, truth, out)
    assert tq.tq_ctx_check(ctx) == 0
    return to_host(out)[:nw]


def rand_words(rng, n, nw, p):
    bits = rng.random((n, nw * 64)) < p
    return np.packbits(bits.astype(np.uint8), axis=1, bitorder="little").view("<u8").astype(np.uint64)


# ------------------------------------------------------------ small config
@pytest.mark.parametrize("p", [0.05, 0.5])
def test_small_config_all_thetas(ctx, p):
    """N=16, r=2^20, Bernoulli(p) (p=0.5 stresses the high thresholds)."""
    bs = tqgen.bernoulli_fixed(1, 16, 1 << 20, p)
    host = [bs.words(j) for j in range(bs.n)]
    pool = torch.zeros((bs.n, bs.nwords), dtype=torch.int64, device="cuda")
    tqgen.fill_gpu(bs, pool.view(-1))
    rows = [pool[j] for j in range(bs.n)]
    for theta in (0, 1, 2, 8, 15, 16, 17):
        got = run_threshold(ctx, rows, bs.r_bits, theta)
        assert np.array_equal(got, oracle.threshold(host, bs.r_bits, theta)), theta


# ------------------------------------------------------ exhaustive fixture
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 11, 13, 15, 16])
def test_exhaustive_combinations(ctx, n):
    r = 1 << n
    host = [tqgen.exhaustive_words(j, n) for j in range(n)]
    pool = dev_pool(host)
    rows = [pool[j] for j in range(n)]
    pc = np.array([bin(p).count("1") for p in range(r)])
    for theta in range(0, n + 2):
        got = run_threshold(ctx, rows, r, theta)
        bits = np.unpackbits(got.view(np.uint8), bitorder="little")[:r]
        assert np.array_equal(bits, (pc >= theta).astype(np.uint8)), theta


# ------------------------------------------------- every counter width
NS = [1, 2, 3, 7, 15, 16, 17, 31, 33, 64, 100, 255, 256, 257, 511, 1000, 1024, 2047, 4095, 4096,
      4097, 8191, 8192, 9000, 40000, 65535]


@pytest.mark.parametrize("n", NS)
def test_many_n(ctx, n):
    rng = np.random.default_rng(n)
    r = 64 * 700 + 13            # several column groups and a ragged tail
    nw = (r + 63) // 64
    distinct = min(n, 300)       # larger N repeats inputs (aliasing)
    dens = rng.uniform(0.02, 0.98, distinct)
    base = np.concatenate([rand_words(rng, 1, nw, d) for d in dens])
    pool = dev_pool(list(base))
    pick = rng.integers(0, distinct, n) if n > distinct else np.arange(n)
    rows = [pool[int(i)] for i in pick]
    host = [base[int(i)] for i in pick]
    counts_mean = float(np.mean(dens)) * n
    thetas = {0, 1, n, n + 1, (n + 1) // 2, max(1, int(counts_mean)), max(1, int(counts_mean) + 3)}
    for theta in sorted(thetas):
        got = run_threshold(ctx, rows, r, theta)
        assert np.array_equal(got, oracle.threshold(host, r, theta)), theta


# ------------------------------------------------------------ split paths
@pytest.mark.parametrize("nw,n", [(1024, 300), (64 * 600, 128), (96000, 80), (200, 5000), (3, 64)])
def test_small_r_large_n(ctx, nw, n):
    rng = np.random.default_rng(nw + n)
    r = nw * 64 - 5
    distinct = min(n, 256)
    base = rand_words(rng, distinct, nw, 0.3)
    pool = dev_pool(list(base))
    pick = rng.integers(0, distinct, n)
    rows = [pool[int(i)] for i in pick]
    host = [base[int(i)] for i in pick]
    for theta in (1, int(0.3 * n), int(0.3 * n) + 1, n):
        got = run_threshold(ctx, rows, r, theta)
        assert np.array_equal(got, oracle.threshold(host, r, theta)), theta


# ------------------------------------------------------------ symmetric
def symmetric_cases(n, rng):
    yield "parity", oracle.truth_parity(n)
    yield "not parity", 1 - oracle.truth_parity(n)
    yield "interval 2..10", oracle.truth_interval(n, 2, 10)
    yield "delta 3", oracle.truth_interval(n, 3, 3)
    yield "below 4", oracle.truth_interval(n, 0, 3)
    yield "majority", oracle.truth_threshold(n, (n + 1) // 2)
    yield "zero", np.zeros(n + 1, dtype=np.uint8)
    yield "one", np.ones(n + 1, dtype=np.uint8)
    f = np.zeros(n + 1, dtype=np.uint8)
    f[::3] = 1
    yield "every third", f
    for k in range(3):
        yield "random %d" % k, rng.integers(0, 2, n + 1).astype(np.uint8)
    g = np.zeros(n + 1, dtype=np.uint8)
    for a in range(1, n, 7):
        g[a:a + 2] = 1
    yield "intervals", g


@pytest.mark.parametrize("n", [5, 16, 37, 256, 300])
def test_symmetric_functions(ctx, n):
    rng = np.random.default_rng(100 + n)
    r = 64 * 300 + 29
    nw = (r + 63) // 64
    base = rand_words(rng, n, nw, 0.05 if n > 100 else 0.4)
    pool = dev_pool(list(base))
    rows = [pool[j] for j in range(n)]
    host = list(base)
    for name, f in symmetric_cases(n, rng):
        got = run_symmetric(ctx, rows, r, f)
        assert np.array_equal(got, oracle.symmetric(host, r, f)), name


# ------------------------------------------------------------- alignment
def test_eight_byte_aligned_inputs(ctx):
    rng = np.random.default_rng(5)
    n, nw = 40, 5001
    r = nw * 64
    base = rand_words(rng, n, nw + 1, 0.35)
    flat = to_dev(base.reshape(-1))
    # views starting one word in: 8-byte but not 16-byte aligned
    rows = [flat[j * (nw + 1) + 1: j * (nw + 1) + 1 + nw] for j in range(n)]
    host = [base[j][1:] for j in range(n)]
    for theta in (2, 13, 40):
        got = run_threshold(ctx, rows, r, theta)
        assert np.array_equal(got, oracle.threshold(host, r, theta))


def test_empty_universe(ctx):
    pool = dev_pool([np.zeros(1, dtype=np.uint64)] * 3)
    out = empty_words(1)
    tq.tq_threshold(ctx, [pool[0], pool[1], pool[2]], 0, 1, out)
    assert tq.tq_ctx_check(ctx) == 0
    assert int(to_host(out)[0]) == 0x5A5A5A5A5A5A5A5A       # nothing written


# ---------------------------------------------------------------- errors
def test_argument_errors(ctx):
    pool = dev_pool([np.zeros(4, dtype=np.uint64)] * 3)
    out = empty_words(4)
    P = tq.ptr_array([pool[0], pool[1], pool[2]])
    assert tq.raw_threshold(ctx, P, 0, 256, 1, out.data_ptr()) == tq.TQ_EINVAL          # N = 0
    assert tq.raw_threshold(ctx, P, 3, 256, 1, 0) == tq.TQ_EINVAL                       # no output
    assert tq.raw_threshold(ctx, P, 3, 256, 1, pool[1].data_ptr()) == tq.TQ_EINVAL      # output aliases input
    bad = tq.ptr_array([pool[0].data_ptr() + 4])
    assert tq.raw_threshold(ctx, bad, 1, 256, 1, out.data_ptr()) == tq.TQ_EINVAL        # misaligned
    nul = tq.ptr_array([0])
    assert tq.raw_threshold(ctx, nul, 1, 256, 1, out.data_ptr()) == tq.TQ_EINVAL        # null input
    big = (ctypes.c_uint64 * (tq.TQ_MAX_INPUTS + 1))(*([pool[0].data_ptr()] * (tq.TQ_MAX_INPUTS + 1)))
    assert tq.raw_threshold(ctx, big, tq.TQ_MAX_INPUTS + 1, 256, 1, out.data_ptr()) == tq.TQ_EINVAL
    assert int(to_host(out)[0]) == 0x5A5A5A5A5A5A5A5A       # nothing was queued


# -------------------------------------------- full large configuration
@pytest.fixture(scope="module")
def large(ctx):
    bs = tqgen.large_set(2)
    pool = torch.empty((bs.n, bs.nwords), dtype=torch.int64, device="cuda")
    tqgen.fill_gpu(bs, pool.view(-1))
    yield bs, pool
    del pool
    torch.cuda.empty_cache()


def test_large_config_full(ctx, large):
    """N=256, r=2^26 (2 GiB): the benchmark's step exactly as timed (inputs
    registered with their cardinality and run count, thresholds 2, 16, 128,
    255 through the carry-save variant with registered input order, pruning
    and the saturating counters on; the interval 2 <= count <= 10 and parity
    through tq_symmetric), then the roofline pass (pruning and saturating
    counters off); every output word of every query equals the oracle's.
    theta = 1 is also checked against torch's OR of all inputs and parity
    against torch's XOR."""
    bs, pool = large
    n, nw, r = bs.n, bs.nwords, bs.r_bits
    rows = [pool[j] for j in range(n)]
    host_all = pool.cpu().numpy().view(np.uint64)
    host = [host_all[j] for j in range(n)]
    stats = torch.zeros((n, 2), dtype=torch.int64, device="cuda")
    for j in range(n):
        tq.tq_bitmap_stats(ctx, rows[j], r, stats[j, 0:1], stats[j, 1:2])
    st = stats.cpu().numpy()
    registered = (tq.bitmap_array([dict(dense=rows[j], rle=None, ones=int(st[j, 0]), runs=int(st[j, 1]))
                                   for j in range(n)]), n)
    queries = [("threshold", t) for t in tqgen.LARGE["thetas"]]
    lo, hi = tqgen.LARGE["interval"]
    queries += [("symmetric", oracle.truth_interval(n, lo, hi)), ("symmetric", oracle.truth_parity(n))]
    wants = [oracle.threshold(host, r, a) if k == "threshold" else oracle.symmetric(host, r, a)
             for k, a in queries]
    out = torch.empty(nw, dtype=torch.int64, device="cuda")
    for prune in (1, 0):
        tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, prune)
        tq.tq_set_option(ctx, tq.TQ_OPTION_LOOPED, prune)
        for (kind, arg), want in zip(queries, wants):
            out.fill_(0x5A5A5A5A)
            if kind == "threshold":
                tq.tq_threshold_variant(ctx, registered, r, arg, tq.TQ_VARIANT_CSA, out)
            else:
                tq.tq_symmetric(ctx, rows, r, arg, out)
            assert tq.tq_ctx_check(ctx) == 0
            assert np.array_equal(to_host(out), want), (kind, prune)
    tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, 1)
    tq.tq_set_option(ctx, tq.TQ_OPTION_LOOPED, 1)
    # theta = 1 is the OR of all inputs, parity their XOR (torch's own ops)
    acc = torch.zeros(nw, dtype=torch.int64, device="cuda")
    x = torch.zeros(nw, dtype=torch.int64, device="cuda")
    for j in range(n):
        acc |= pool[j]
        x ^= pool[j]
    tq.tq_threshold(ctx, rows, r, 1, out)
    assert tq.tq_ctx_check(ctx) == 0
    assert torch.equal(acc, out)
    tq.tq_symmetric(ctx, rows, r, oracle.truth_parity(n), out)
    assert tq.tq_ctx_check(ctx) == 0
    assert torch.equal(x, out)


# ----------------------------------------------------------------- pruning
@pytest.mark.parametrize("n", [40, 200, 1000])
def test_pruning_equivalence(ctx, n):
    """Threshold queries stop reading inputs once every position of a column
    group is decided; the result must not change (against the unpruned run
    and the oracle).  Densities vary per column group so waves stop at
    different inputs."""
    rng = np.random.default_rng(300 + n)
    r = 64 * 64 * 9 + 31
    nw = (r + 63) // 64
    base = []
    for j in range(min(n, 250)):
        col_dens = np.repeat(rng.uniform(0.0, 1.0, (nw + 63) // 64), 64)[:nw]
        bits = rng.random((nw, 64)) < col_dens[:, None] * rng.uniform(0.2, 1.0)
        base.append(np.packbits(bits.astype(np.uint8), axis=1, bitorder="little").view("<u8").reshape(-1).astype(np.uint64))
    pool = dev_pool(base)
    pick = rng.integers(0, len(base), n)
    rows = [pool[int(i)] for i in pick]
    host = [base[int(i)] for i in pick]
    for theta in sorted({1, 3, n // 3, n // 2, (3 * n) // 4, n - 1, n}):
        want = oracle.threshold(host, r, theta)
        outs = []
        for prune in (1, 0):
            tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, prune)
            outs.append(run_threshold(ctx, rows, r, theta))
        tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, 1)
        assert np.array_equal(outs[0], want), theta
        assert np.array_equal(outs[1], want), theta


def test_complement_identity_gpu(ctx):
    """Section 2.3, corrected: NOT T_theta(B) = T_{N-theta+1}(NOT B) on [0, r),
    for the dense kernel and for compressed inputs (the complemented bitmaps
    encoded by the library)."""
    rng = np.random.default_rng(77)
    n, r = 23, 64 * 1500 + 29
    nw = (r + 63) // 64
    host = rand_words(rng, n, nw, 0.2)
    pool = dev_pool(host)
    comp = torch.bitwise_not(pool)
    rows = [pool[j] for j in range(n)]
    crows = [comp[j] for j in range(n)]
    mask = np.full(nw, np.uint64(0xFFFFFFFFFFFFFFFF))
    mask[-1] = np.uint64(tail_mask(r))
    cap = tq.tq_rle_max_words(r)
    enc = []
    for j in range(n):
        s = torch.empty(cap, dtype=torch.int64, device="cuda")
        ln = torch.zeros(1, dtype=torch.int64, device="cuda")
        tq.tq_rle_encode(ctx, crows[j], r, s, cap, ln, None)
        assert tq.tq_ctx_check(ctx) == 0
        enc.append((s, int(ln.item()), None))
    for theta in (1, 2, 7, n // 2, n - 1, n):
        a = run_threshold(ctx, rows, r, theta)
        b = run_threshold(ctx, crows, r, n - theta + 1)
        assert np.array_equal(a, ~b & mask), theta
        c = empty_words(nw)
        tq.tq_threshold_rle_dense(ctx, enc, r, n - theta + 1, c)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(a, ~to_host(c)[:nw] & mask), theta


@pytest.mark.parametrize("p", [0.02, 0.5, 0.97])
def test_looped_extreme_thresholds(ctx, p):
    """Thresholds within 3 of either end run on saturating counters (directly,
    or on the complemented inputs); they must equal the oracle and the
    carry-save kernel, with and without early exit, over ragged tails."""
    rng = np.random.default_rng(int(p * 100))
    for n, r in ((1, 64 * 70 + 3), (2, 640), (3, 64 * 129), (4, 64 * 200 + 1), (5, 64 * 65),
                 (16, 64 * 300 + 17), (40, 64 * 128), (300, 64 * 70 + 63)):
        nw = (r + 63) // 64
        host = rand_words(rng, n, nw, p)
        pool = dev_pool(host)
        rows = [pool[j] for j in range(n)]
        for theta in sorted({t for t in (1, 2, 3, n - 2, n - 1, n) if 1 <= t <= n}):
            want = oracle.threshold(list(host), r, theta)
            for looped, prune in ((1, 1), (1, 0), (0, 1)):
                tq.tq_set_option(ctx, tq.TQ_OPTION_LOOPED, looped)
                tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, prune)
                got = run_threshold(ctx, rows, r, theta)
                assert np.array_equal(got, want), (n, theta, looped, prune)
    tq.tq_set_option(ctx, tq.TQ_OPTION_LOOPED, 1)
    tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, 1)


def test_looped_exhaustive():
    """On the exhaustive fixture (every input combination once) each extreme
    threshold selects exactly the positions with popcount >= theta."""
    c = tq.tq_create(0)
    try:
        for n in (3, 6, 9):
            r = 1 << n
            host = [tqgen.exhaustive_words(j, n) for j in range(n)]
            pool = dev_pool(host)
            rows = [pool[j] for j in range(n)]
            pc = np.array([bin(q).count("1") for q in range(r)])
            for theta in sorted({t for t in (1, 2, 3, n - 2, n - 1, n) if t >= 1}):
                got = run_threshold(c, rows, r, theta)
                bits = np.unpackbits(got.view(np.uint8), bitorder="little")[:r]
                assert np.array_equal(bits, (pc >= theta).astype(np.uint8)), (n, theta)
    finally:
        tq.tq_destroy(c)


def test_max_size_beyond_32bit_word_index(ctx):
    """Bitmaps of 2^32 + 101 words (32 GiB each, r = 64 (2^32 + 100) + 7 bits):
    word indices past 32 bits and a ragged last word.  Sampled columns against
    the oracle, and the whole output against torch's OR / AND of the two
    inputs (theta = 1 / 2), chunk by chunk."""
    nw = (1 << 32) + 101
    r = 64 * ((1 << 32) + 100) + 7
    free, _ = torch.cuda.mem_get_info()
    need = 3 * nw * 8 + (4 << 30)
    if free < need:
        pytest.skip("needs %d GiB of free device memory" % (need >> 30))
    bs = tqgen.bernoulli_fixed(9, 2, r, 0.5)
    assert bs.nwords == nw
    pool = torch.empty((2, nw), dtype=torch.int64, device="cuda")
    tqgen.fill_gpu(bs, pool.view(-1))
    rows = [pool[0], pool[1]]
    out = torch.empty(nw, dtype=torch.int64, device="cuda")
    rng = np.random.default_rng(3)
    cols = np.unique(np.concatenate([[0, 1, (1 << 32) - 1, 1 << 32, (1 << 32) + 1, nw - 2, nw - 1],
                                     rng.integers(0, nw, 24)])).astype(np.int64)
    words = np.stack([np.concatenate([bs.words(j, int(c), int(c) + 1) for c in cols]) for j in range(2)])
    tail = np.uint64(tail_mask(r))
    chunk = 1 << 28
    for theta in (1, 2):
        tq.tq_threshold(ctx, rows, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        got = out[torch.from_numpy(cols).cuda()].cpu().numpy().view(np.uint64)
        assert np.array_equal(got, oracle.threshold_cols(words, cols, r, theta)), theta
        for c0 in range(0, nw, chunk):
            c1 = min(nw, c0 + chunk)
            a, b = pool[0, c0:c1], pool[1, c0:c1]
            ref = (a | b) if theta == 1 else (a & b)
            if c1 == nw:
                ref = ref.clone()
                ref[-1] = ref[-1] & torch.tensor(np.array([tail]).view(np.int64)[0], device="cuda")
            assert torch.equal(out[c0:c1], ref), (theta, c0)
