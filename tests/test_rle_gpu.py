"""Run-length-encoded path on the GPU against the CPU oracle.

The GPU encoder must produce the oracle's canonical stream byte for byte;
threshold queries over compressed inputs must produce the oracle's canonical
encoding of the oracle's threshold; dense-output and hybrid queries must
equal the oracle's dense threshold.  At the full RLE configuration (N=512,
r=2^28) outputs are checked on sampled columns and against the uncompressed
path on the same inputs.
"""
import numpy as np
import pytest
import torch

import oracle
import tqgen
from gpuhelp import dev_pool, empty_words, to_dev, to_host
from paper_1402_4073_amd import binding as tq

pytestmark = pytest.mark.gpu

STRIDE = tq.TQ_RLE_INDEX_STRIDE


@pytest.fixture(scope="module", params=[1, 2], ids=["bitplanes", "swar"])
def ctx(request):
    """Every test runs with each kind of column counters of the tile kernel."""
    c = tq.tq_create(0)
    tq.tq_set_option(c, tq.TQ_OPTION_RLE_COUNTERS, request.param)
    yield c
    tq.tq_destroy(c)


def mk(fill, run, lits):
    return (fill & 1) | (run << 1) | (lits << 33)


def expected_index(stream, r_bits):
    """Checkpoint index by its definition: for checkpoint c, the marker whose
    run covers word c*STRIDE (stream offset, start word)."""
    nw = (r_bits + 63) // 64
    nchk = (nw + STRIDE - 1) // STRIDE
    idx = np.zeros(2 * nchk, dtype=np.uint64)
    pos, w, c = 0, 0, 0
    s = [int(x) for x in stream]
    while pos < len(s):
        m = s[pos]
        run, lits = (m >> 1) & 0xFFFFFFFF, m >> 33
        end = w + run + lits
        while c < nchk and c * STRIDE < end:
            idx[2 * c], idx[2 * c + 1] = pos, w
            c += 1
        pos += 1 + lits
        w = end
    return idx


def markov_bitmaps(seed, n, r, ones, zeros):
    ms = tqgen.markov_fixed(seed, n, r, ones, zeros)
    return [ms.words(j) for j in range(n)]


def special_bitmaps(r):
    nw = (r + 63) // 64
    out = []
    out.append(np.zeros(nw, dtype=np.uint64))
    out.append(np.full(nw, np.uint64(0xFFFFFFFFFFFFFFFF)))
    alt = np.zeros(nw, dtype=np.uint64)
    alt[1::2] = np.uint64(0xFFFFFFFFFFFFFFFF)
    out.append(alt)                                  # alternating fills
    d0 = np.full(nw, np.uint64(0xFFFFFFFFFFFFFFFF))
    d0[0] = 12345                                    # dirty first word
    out.append(d0)
    dc = np.zeros(nw, dtype=np.uint64)
    dc[::2] = np.uint64(0x00FF00FF00FF00FF)          # dirty / clean alternating
    out.append(dc)
    return out


def gpu_encode(ctx, dense_np, r):
    d = to_dev(dense_np)
    cap = tq.tq_rle_max_words(r)
    out = empty_words(cap)
    ln = torch.zeros(1, dtype=torch.int64, device="cuda")
    idx = torch.zeros(max(1, tq.tq_rle_index_words(r)), dtype=torch.int64, device="cuda")
    tq.tq_rle_encode(ctx, d, r, out, cap, ln, idx)
    assert tq.tq_ctx_check(ctx) == 0
    L = int(ln.item())
    return to_host(out)[:L], to_host(idx)


# ------------------------------------------------------------------ encoder
@pytest.mark.parametrize("r", [64, 65, 1000, 64 * 512, 64 * 512 + 1, 64 * 3000 + 17, 1 << 20])
def test_encoder_matches_oracle(ctx, r):
    cases = special_bitmaps(r) + markov_bitmaps(r, 4, r, 50.0, 900.0) + markov_bitmaps(r + 1, 2, r, 2.0, 3.0)
    for k, dense in enumerate(cases):
        got, idx = gpu_encode(ctx, dense, r)
        want = oracle.rle_encode(dense, r)
        assert np.array_equal(got, want), k
        assert np.array_equal(idx, expected_index(want, r)), k


@pytest.mark.parametrize("nw", [7, 8, 9, 2047, 2048, 2049, 4097])
def test_encoder_run_boundaries(ctx, nw):
    """Runs that change exactly where the encoder's per-thread (8-word) and
    per-block (2048-word) spans change, and one word to either side: whether
    a word starts a marker depends on the word before it, which then lies in
    another thread or block.  Bitmaps of nw words and of nw words less five
    bits (a masked tail word)."""
    ones = np.uint64(0xFFFFFFFFFFFFFFFF)
    for r in (nw * 64, nw * 64 - 5):
        cases = []
        for period in (8, 2048, 7, 9, 2047):
            for kinds in ((0, 1), (1, 2), (2, 0), (0, 2, 1)):
                w = np.arange(nw)
                k = np.array(kinds)[(w // period) % len(kinds)]
                x = np.where(k == 0, np.uint64(0), np.where(k == 1, ones, np.uint64(0x0123456789ABCDEF)))
                cases.append(x.astype(np.uint64))
        for k, dense in enumerate(cases):
            got, idx = gpu_encode(ctx, dense, r)
            want = oracle.rle_encode(dense, r)
            assert np.array_equal(got, want), (r, k)
            assert np.array_equal(idx, expected_index(want, r)), (r, k)


def test_encoder_capacity(ctx):
    r = 64 * 100
    dense = markov_bitmaps(7, 1, r, 3.0, 5.0)[0]
    want = oracle.rle_encode(dense, r)
    d = to_dev(dense)
    out = empty_words(len(want))
    ln = torch.zeros(1, dtype=torch.int64, device="cuda")
    cap = len(want) - 3
    tq.tq_rle_encode(ctx, d, r, out, cap, ln)
    assert tq.tq_ctx_check(ctx) == tq.TQ_ECAPACITY
    assert int(ln.item()) == len(want)                # required length reported
    got = to_host(out)
    assert np.all(got[cap:] == np.uint64(0x5A5A5A5A5A5A5A5A))   # nothing past the capacity
    assert tq.tq_ctx_check(ctx) == 0                  # status cleared


# -------------------------------------------------------------- index build
def test_build_index_canonical_and_not(ctx):
    r = 64 * 2000 + 9
    for dense in markov_bitmaps(11, 3, r, 40.0, 700.0):
        s = oracle.rle_encode(dense, r)
        d = to_dev(s)
        idx = torch.zeros(tq.tq_rle_index_words(r), dtype=torch.int64, device="cuda")
        tq.tq_rle_build_index(ctx, d, len(s), r, idx)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(idx), expected_index(s, r))
    # non-canonical: split runs, clean literals, empty markers
    r = 64 * 1300
    parts = [mk(0, 300, 0), mk(0, 300, 2), 5, 0, mk(0, 0, 0), mk(1, 100, 0), mk(1, 0, 1), 7,
             mk(0, 597, 0)]
    s = np.array(parts, dtype=np.uint64)
    idx = torch.zeros(tq.tq_rle_index_words(r), dtype=torch.int64, device="cuda")
    tq.tq_rle_build_index(ctx, to_dev(s), len(s), r, idx)
    assert tq.tq_ctx_check(ctx) == 0
    assert np.array_equal(to_host(idx), expected_index(s, r))


def random_stream(rng, nw, max_run, max_lits, p_empty=0.05):
    """A valid, generally non-canonical stream over nw words: markers with
    random fills, runs and literal counts (empty markers among them), the
    last one cut so that the runs end exactly at nw."""
    parts, w = [], 0
    while w < nw:
        if rng.random() < p_empty:
            parts.append(mk(int(rng.integers(0, 2)), 0, 0))
            continue
        run = int(rng.integers(0, max_run + 1))
        lits = int(rng.integers(0, max_lits + 1))
        if w + run + lits > nw:
            run = min(run, nw - w)
            lits = nw - w - run
        parts.append(mk(int(rng.integers(0, 2)), run, lits))
        parts += [int(x) for x in rng.integers(1, 1 << 62, lits, dtype=np.int64)]
        w += run + lits
    return np.array(parts, dtype=np.uint64)


@pytest.mark.parametrize("case", range(10))
def test_build_index_structures(ctx, case):
    """Index building decodes each stream 64 words at a time: streams whose
    markers sit at chunk boundaries, literal runs spanning several chunks
    (chunks of literal words only are skipped), fills covering hundreds of
    checkpoints (index entries written in several rounds), dense runs of
    empty markers, and streams whose length is a multiple of 64, all against
    the index by its definition."""
    rng = np.random.default_rng(900 + case)
    nw = [64 * STRIDE + 1, 300 * STRIDE, 5000, 64, 2 * STRIDE + 63, 4 * STRIDE, 77 * STRIDE + 5, 7000,
          3 * STRIDE, 20 * STRIDE][case]
    r = nw * 64 - (case % 3)
    streams = {
        0: random_stream(rng, nw, 600, 3),
        1: np.array([mk(1, nw, 0)], dtype=np.uint64),                     # one fill, 300 entries
        2: random_stream(rng, nw, 40, 200),                                # long literal runs
        3: np.array([mk(0, 0, 0)] * 63 + [mk(1, 64, 0)], dtype=np.uint64),  # 64 markers in one chunk
        4: random_stream(rng, nw, 3, 1, p_empty=0.3),                      # a marker every word or two
        5: random_stream(rng, nw, 2 * STRIDE, 62),
        6: random_stream(rng, nw, 5 * STRIDE, 70),
        7: random_stream(rng, nw, 64, 64),
        8: None,
        9: random_stream(rng, nw, STRIDE, 0),
    }
    st = streams[case]
    if st is None:
        # the last literal word of each marker ends a 64-word chunk
        parts, w = [], 0
        while w < nw:
            lits = min(63 - (len(parts) % 64), nw - w)
            parts.append(mk(0, 0, lits))
            parts += [5] * lits
            w += lits
            if w < nw:
                run = min(int(rng.integers(1, 900)), nw - w)
                parts.append(mk(1, run, 0))
                w += run
        st = np.array(parts, dtype=np.uint64)
    assert np.array_equal(oracle.rle_decode(st, r).size, (r + 63) // 64)   # a valid stream
    idx = torch.full((tq.tq_rle_index_words(r),), -1, dtype=torch.int64, device="cuda")
    tq.tq_rle_build_index(ctx, to_dev(st), len(st), r, idx)
    assert tq.tq_ctx_check(ctx) == 0
    assert np.array_equal(to_host(idx), expected_index(st, r))


def test_indexes_built_by_a_query(ctx):
    """A query whose inputs bring no index builds all of them in one launch
    (one wave per stream): varied streams, including non-canonical ones,
    against the oracle's threshold of the decoded inputs."""
    rng = np.random.default_rng(77)
    nw = 40 * STRIDE + 17
    r = nw * 64
    streams = [random_stream(rng, nw, int(m), int(l)) for m, l in
               zip(rng.integers(1, 3000, 24), rng.integers(0, 90, 24))]
    streams += [oracle.rle_encode(d, r) for d in markov_bitmaps(17, 8, r, 60.0, 900.0)]
    dense = [oracle.rle_decode(x, r) for x in streams]
    inputs = [(to_dev(x), len(x), None) for x in streams]
    for theta in (1, 2, 9, len(streams)):
        out = empty_words(nw)
        tq.tq_threshold_rle_dense(ctx, inputs, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.threshold(dense, r, theta)), theta


def test_build_index_rejects_malformed(ctx):
    r = 64 * 1000
    for parts in ([mk(0, 999, 0)], [mk(0, 1001, 0)], [mk(0, 998, 3), 1, 2, 3], [mk(0, 990, 5), 1, 2],
                  [mk(0, 1000, 0), mk(0, 5, 0)], [mk(0, 10, 0)] * 99 + [mk(0, 9, 70)] + [3] * 60,
                  [mk(0, 0, 0)] * 130 + [mk(1, 999, 0)]):
        s = np.array(parts, dtype=np.uint64)
        idx = torch.zeros(tq.tq_rle_index_words(r), dtype=torch.int64, device="cuda")
        tq.tq_rle_build_index(ctx, to_dev(s), len(s), r, idx)
        assert tq.tq_ctx_check(ctx) == tq.TQ_EFORMAT, parts


# ------------------------------------------------------------------- decode
def test_decode(ctx):
    r = 64 * 1500 + 33
    for dense in special_bitmaps(r) + markov_bitmaps(13, 3, r, 30.0, 400.0):
        s = oracle.rle_encode(dense, r)
        d = to_dev(s)
        out = empty_words((r + 63) // 64)
        tq.tq_rle_decode(ctx, (d, len(s), None), r, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.rle_decode(s, r))


def test_decode_rejects_malformed(ctx):
    r = 64 * 1000
    s = np.array([mk(0, 998, 3), 1, 2, 3], dtype=np.uint64)
    idx = np.zeros(tq.tq_rle_index_words(r), dtype=np.uint64)   # claims every tile starts at marker 0
    out = empty_words(1000)
    tq.tq_rle_decode(ctx, (to_dev(s), len(s), to_dev(idx)), r, out)
    assert tq.tq_ctx_check(ctx) == tq.TQ_EFORMAT


# ---------------------------------------------------------------- threshold
@pytest.fixture
def tiles_option(ctx):
    yield lambda v: tq.raw_set_option(ctx, tq.TQ_OPTION_RLE_TILES, v)
    tq.tq_set_option(ctx, tq.TQ_OPTION_RLE_TILES, 0)


def rle_inputs(ctx, dense_list, r, with_index=True, use_oracle_encoding=False):
    keep, inputs = [], []
    for dense in dense_list:
        if use_oracle_encoding:
            s = oracle.rle_encode(dense, r)
            idx = expected_index(s, r) if with_index else None
        else:
            s, idx = gpu_encode(ctx, dense, r)
            idx = idx if with_index else None
        ds = to_dev(s)
        di = to_dev(idx) if idx is not None else None
        keep += [ds, di]
        inputs.append((ds, len(s), di))
    return inputs, keep


@pytest.mark.parametrize("n,r", [(1, 64 * 600), (5, 64 * 1100 + 3), (37, 64 * 2050), (200, 64 * 1025 + 63)])
def test_threshold_rle_matches_oracle(ctx, n, r):
    rng = np.random.default_rng(n)
    dense = markov_bitmaps(100 + n, n, r, float(rng.integers(20, 200)), float(rng.integers(100, 3000)))
    dense[0] = special_bitmaps(r)[int(rng.integers(0, 5))]
    for variant in ("gpu-encoded", "oracle-encoded", "no-index"):
        inputs, keep = rle_inputs(ctx, dense, r, with_index=(variant != "no-index"),
                                  use_oracle_encoding=(variant == "oracle-encoded"))
        for theta in sorted({0, 1, 2, max(1, n // 3), n, n + 1}):
            want_dense = oracle.threshold(dense, r, theta)
            want = oracle.rle_encode(want_dense, r)
            cap = tq.tq_rle_max_words(r)
            out = empty_words(cap)
            ln = torch.zeros(1, dtype=torch.int64, device="cuda")
            tq.tq_threshold_rle(ctx, inputs, r, theta, out, cap, ln)
            assert tq.tq_ctx_check(ctx) == 0
            L = int(ln.item())
            assert L == len(want), (variant, theta)
            assert np.array_equal(to_host(out)[:L], want), (variant, theta)
            dout = empty_words((r + 63) // 64)
            tq.tq_threshold_rle_dense(ctx, inputs, r, theta, dout)
            assert tq.tq_ctx_check(ctx) == 0
            assert np.array_equal(to_host(dout), want_dense), (variant, theta)


def test_threshold_rle_noncanonical_inputs(ctx):
    r = 64 * 1300
    a = np.array([mk(0, 300, 0), mk(0, 300, 2), 5, 0, mk(0, 0, 0), mk(1, 100, 0), mk(1, 0, 1), 7,
                  mk(0, 597, 0)], dtype=np.uint64)
    b = oracle.rle_encode(markov_bitmaps(3, 1, r, 10.0, 10.0)[0], r)
    c = np.array([mk(1, 1300, 0)], dtype=np.uint64)
    dense = [oracle.rle_decode(x, r) for x in (a, b, c)]
    inputs = [(to_dev(x), len(x), None) for x in (a, b, c)]
    for theta in (1, 2, 3):
        out = empty_words((r + 63) // 64)
        tq.tq_threshold_rle_dense(ctx, inputs, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.threshold(dense, r, theta))


def test_threshold_rle_capacity_and_format(ctx):
    r = 64 * 700
    dense = markov_bitmaps(21, 6, r, 5.0, 9.0)
    inputs, keep = rle_inputs(ctx, dense, r)
    want = oracle.rle_encode(oracle.threshold(dense, r, 3), r)
    out = empty_words(len(want))
    ln = torch.zeros(1, dtype=torch.int64, device="cuda")
    tq.tq_threshold_rle(ctx, inputs, r, 3, out, len(want) - 1, ln)
    assert tq.tq_ctx_check(ctx) == tq.TQ_ECAPACITY
    assert int(ln.item()) == len(want)
    bad = np.array([mk(0, 600, 0)], dtype=np.uint64)            # covers too few words
    inputs2 = inputs[:2] + [(to_dev(bad), 1, None)]
    tq.tq_threshold_rle(ctx, inputs2, r, 2, out, len(want), ln)
    assert tq.tq_ctx_check(ctx) == tq.TQ_EFORMAT
    # host-side argument errors
    assert tq.raw_threshold_rle(ctx, [], r, 1, out.data_ptr(), 10, ln.data_ptr()) == tq.TQ_EINVAL
    assert tq.raw_threshold_rle(ctx, inputs, r, 1, out.data_ptr(), 10, 0) == tq.TQ_EINVAL
    # size limits: bitmaps of 2^31 words or more, streams longer than 2^32 - 1024 words
    huge = [(inputs[0][0], inputs[0][1], None)]
    assert tq.raw_threshold_rle(ctx, huge, 64 << 31, 1, out.data_ptr(), 10, ln.data_ptr()) == tq.TQ_EINVAL
    long_stream = [(inputs[0][0], (1 << 32) - 1023, None)]
    assert tq.raw_threshold_rle(ctx, long_stream, r, 1, out.data_ptr(), 10, ln.data_ptr()) == tq.TQ_EINVAL


@pytest.mark.parametrize("n_rle,n_dense", [(3, 2), (0, 4), (20, 20), (1, 0)])
def test_hybrid(ctx, n_rle, n_dense):
    r = 64 * 1700 + 5
    dense_all = markov_bitmaps(300 + n_rle, n_rle + n_dense, r, 60.0, 500.0)
    inputs, keep = rle_inputs(ctx, dense_all[:n_rle], r)
    pool = dev_pool(dense_all[n_rle:]) if n_dense else None
    drows = [pool[j] for j in range(n_dense)] if n_dense else []
    n = n_rle + n_dense
    for theta in sorted({1, 2, max(1, n // 2), n}):
        out = empty_words((r + 63) // 64)
        tq.tq_threshold_hybrid(ctx, inputs, drows, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.threshold(dense_all, r, theta)), theta


# ------------------------------------------------------- full configuration
def test_rle_config_full_size(ctx):
    """N=512 Markov bitmaps of r=2^28 bits (ones-runs mean 64, zeros-runs mean
    4096), encoded on the GPU; thresholds 2, 64, 256, parity and
    2 <= count <= 10 with canonical RLE output.  Every output stream decodes
    (oracle decoder) to a bitmap equal, word for word, to the oracle's result
    on the generator's words (compared in word ranges of 2^18 columns), is
    the oracle's canonical encoding of it, and equals the uncompressed
    kernel's output on the same inputs."""
    ms = tqgen.rle_set(3)
    n, nw, r = ms.n, ms.nwords, ms.r_bits
    dense = torch.empty((n, nw), dtype=torch.int64, device="cuda")
    chunk = 64
    for j0 in range(0, n, chunk):
        tqgen.fill_gpu(ms, dense[j0:j0 + chunk].reshape(-1), first=j0, count=min(chunk, n - j0))
    rows = [dense[j] for j in range(n)]
    pool, offs, lens, index_pool = tq.encode_pool(ctx, rows, r)
    inputs = [(pool[offs[j]:], lens[j], index_pool[j]) for j in range(n)]
    # the GPU-encoded inputs decode back to the generator's words
    for j in (0, 1, n - 1):
        dec = torch.empty(nw, dtype=torch.int64, device="cuda")
        tq.tq_rle_decode(ctx, inputs[j], r, dec)
        assert tq.tq_ctx_check(ctx) == 0
        assert torch.equal(dec, dense[j])
        s_host = to_host(pool[offs[j]:offs[j] + lens[j]])
        assert np.array_equal(oracle.rle_decode(s_host, r), to_host(dense[j]))
    cap = tq.tq_rle_max_words(r)
    out = torch.empty(cap, dtype=torch.int64, device="cuda")
    ln = torch.zeros(1, dtype=torch.int64, device="cuda")
    ref = torch.empty(nw, dtype=torch.int64, device="cuda")
    queries = [("threshold", t) for t in (2, 64, 256)]
    queries += [("symmetric", oracle.truth_parity(n)), ("symmetric", oracle.truth_interval(n, 2, 10))]
    results = []
    for kind, arg in queries:
        if kind == "threshold":
            tq.tq_threshold_rle(ctx, inputs, r, arg, out, cap, ln)
        else:
            tq.tq_symmetric_rle(ctx, inputs, r, arg, out, cap, ln)
        assert tq.tq_ctx_check(ctx) == 0
        stream = to_host(out)[:int(ln.item())]
        got = oracle.rle_decode(stream, r)                       # valid, exact coverage
        assert np.array_equal(oracle.rle_encode(got, r), stream), kind  # canonical
        if kind == "threshold":
            tq.tq_threshold(ctx, rows, r, arg, ref)              # uncompressed path, same inputs
        else:
            tq.tq_symmetric(ctx, rows, r, arg, ref)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(got, to_host(ref)), kind
        results.append(got)
    span = 1 << 18
    for c0 in range(0, nw, span):
        c1 = min(nw, c0 + span)
        words = dense[:, c0:c1].contiguous().cpu().numpy().view(np.uint64)
        cols = np.arange(c0, c1, dtype=np.uint64)
        for (kind, arg), got in zip(queries, results):
            if kind == "threshold":
                want = oracle.threshold_cols(words, cols, r, arg)
            else:
                want = oracle.symmetric_cols(words, cols, r, arg)
            assert np.array_equal(got[c0:c1], want), (kind, c0)


@pytest.mark.parametrize("n,tiles", [(70, 0), (150, 0), (70, 3), (150, 2)])
def test_threshold_rle_many_dirty_words(ctx, tiles_option, n, tiles):
    """Inputs dirty almost everywhere: nearly every column is undecided after
    the fills and its counter receives a literal word from most inputs.  With
    several tiles per workgroup the tiles after the first are done in one
    pass."""
    r = 64 * 1100 + 5
    assert tiles_option(tiles) == tq.TQ_OK
    dense = markov_bitmaps(500 + n, n, r, 2.0, 2.0)
    inputs, keep = rle_inputs(ctx, dense, r)
    for theta in (1, n // 3, n // 2, n - 1, n):
        out = empty_words((r + 63) // 64)
        tq.tq_threshold_rle_dense(ctx, inputs, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.threshold(dense, r, theta)), theta
    # hybrid with the same inputs split between the two forms
    half = n // 2
    pool = dev_pool(dense[half:])
    out = empty_words((r + 63) // 64)
    tq.tq_threshold_hybrid(ctx, inputs[:half], [pool[j] for j in range(n - half)], r, n // 2, out)
    assert tq.tq_ctx_check(ctx) == 0
    assert np.array_equal(to_host(out), oracle.threshold(dense, r, n // 2))


# ------------------------------------------------ tile ranges per workgroup
def test_tiles_option_range(ctx, tiles_option):
    assert tiles_option(-1) == tq.TQ_EINVAL
    assert tiles_option((1 << 20) + 1) == tq.TQ_EINVAL
    assert tiles_option(1 << 20) == tq.TQ_OK
    assert tiles_option(0) == tq.TQ_OK


def undecided_per_tile(dense, r, theta):
    """Columns of each tile where the fills do not decide theta (RBMrg's
    middle case) and some input is dirty, counted from the words."""
    words = np.stack(dense)
    ones = (words == np.uint64(0xFFFFFFFFFFFFFFFF)).sum(axis=0)
    dirty = ((words != 0) & (words != np.uint64(0xFFFFFFFFFFFFFFFF))).sum(axis=0)
    tp = theta - ones.astype(np.int64)
    und = (tp >= 1) & (tp <= dirty) & (dirty > 0)
    nt = (words.shape[1] + STRIDE - 1) // STRIDE
    return np.array([int(und[t * STRIDE:(t + 1) * STRIDE].sum()) for t in range(nt)])


@pytest.mark.parametrize("tiles", [0, 11, 3, 1 << 20])
def test_spans_with_few_undecided_columns(ctx, tiles_option, tiles):
    """Tiles the fills nearly decide are taken several at a time: one marker
    walk over the span, then a literal walk only for the tiles of the span
    that have undecided columns, each stream entered through the index at
    that tile.  Thresholds are picked so that some tiles have a few
    undecided columns and others none (the mixed spans), with ranges that
    end in a partial span, with and without indexes, and hybrid inputs."""
    r = 64 * STRIDE * 26 + 41                      # 27 tiles, the last one short
    n = 160
    dense = markov_bitmaps(710, n, r, 64.0, 1500.0)
    counts = {t: undecided_per_tile(dense, r, t) for t in range(2, n)}
    # thresholds with undecided columns in some tiles, fewer than 32 in every
    # tile, and none in others
    mixed = [t for t, u in counts.items() if u.max() < 32 and (u > 0).sum() >= 3 and (u == 0).sum() >= 3]
    assert mixed, "no threshold leaves a few undecided columns in some tiles"
    picks = sorted({mixed[0], mixed[len(mixed) // 2], mixed[-1]})
    assert tiles_option(tiles) == tq.TQ_OK
    for with_index in (True, False):
        inputs, keep = rle_inputs(ctx, dense, r, with_index=with_index)
        for theta in picks + [n // 2, n]:
            out = empty_words((r + 63) // 64)
            tq.tq_threshold_rle_dense(ctx, inputs, r, theta, out)
            assert tq.tq_ctx_check(ctx) == 0
            assert np.array_equal(to_host(out), oracle.threshold(dense, r, theta)), (with_index, theta)
    inputs, keep = rle_inputs(ctx, dense[:100], r)
    pool = dev_pool(dense[100:])
    for theta in picks:
        out = empty_words((r + 63) // 64)
        tq.tq_threshold_hybrid(ctx, inputs, [pool[j] for j in range(n - 100)], r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.threshold(dense, r, theta)), ("hybrid", theta)
    # symmetric functions whose run table leaves as few columns undecided
    inputs, keep = rle_inputs(ctx, dense, r)
    for t in picks:
        for f in (oracle.truth_interval(n, t, n), oracle.truth_interval(n, t - 1, n - 1)):
            out = empty_words((r + 63) // 64)
            tq.tq_symmetric_rle_dense(ctx, inputs, r, f, out)
            assert tq.tq_ctx_check(ctx) == 0
            assert np.array_equal(to_host(out), oracle.symmetric(dense, r, f)), ("symmetric", t)


@pytest.mark.parametrize("tiles", [1, 2, 3, 7, 1 << 20, 0])
def test_tile_ranges(ctx, tiles_option, tiles):
    """A workgroup that walks several tiles in a row carries every stream's
    position from one tile to the next; any range length, a ragged last
    range and a ragged last tile give the oracle's result, with and without
    checkpoint indexes, and for hybrid queries."""
    r = 64 * STRIDE * 9 + 37                      # 10 tiles, the last one short
    n = 24
    dense = markov_bitmaps(700, n, r, 40.0, 900.0)
    sp = special_bitmaps(r)
    dense[0], dense[1], dense[2] = sp[2], sp[4], sp[3]
    assert tiles_option(tiles) == tq.TQ_OK
    for with_index in (True, False):
        inputs, keep = rle_inputs(ctx, dense, r, with_index=with_index)
        for theta in (1, 2, 8, n - 1, n):
            want_dense = oracle.threshold(dense, r, theta)
            dout = empty_words((r + 63) // 64)
            tq.tq_threshold_rle_dense(ctx, inputs, r, theta, dout)
            assert tq.tq_ctx_check(ctx) == 0
            assert np.array_equal(to_host(dout), want_dense), (with_index, theta)
            want = oracle.rle_encode(want_dense, r)
            cap = tq.tq_rle_max_words(r)
            out = empty_words(cap)
            ln = torch.zeros(1, dtype=torch.int64, device="cuda")
            tq.tq_threshold_rle(ctx, inputs, r, theta, out, cap, ln)
            assert tq.tq_ctx_check(ctx) == 0
            assert np.array_equal(to_host(out)[:int(ln.item())], want), (with_index, theta)
    inputs, keep = rle_inputs(ctx, dense[:10], r)
    pool = dev_pool(dense[10:])
    out = empty_words((r + 63) // 64)
    tq.tq_threshold_hybrid(ctx, inputs, [pool[j] for j in range(n - 10)], r, 9, out)
    assert tq.tq_ctx_check(ctx) == 0
    assert np.array_equal(to_host(out), oracle.threshold(dense, r, 9))


@pytest.mark.parametrize("tiles", [3, 0])
def test_more_inputs_than_lanes(ctx, tiles_option, tiles):
    """600 RLE inputs: a workgroup has 512 lanes, so the inputs past the first
    512 enter each tile through their checkpoint index."""
    r = 64 * STRIDE * 5 + 3
    n = 600
    dense = markov_bitmaps(800, n, r, 50.0, 2000.0)
    assert tiles_option(tiles) == tq.TQ_OK
    inputs, keep = rle_inputs(ctx, dense, r)
    for theta in (1, 2, 30, 300, n):
        out = empty_words((r + 63) // 64)
        tq.tq_threshold_rle_dense(ctx, inputs, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.threshold(dense, r, theta)), theta


@pytest.mark.parametrize("n_rle,n_dense,tiles", [(300, 0, 0), (300, 0, 2), (40, 30, 0), (600, 0, 0)])
def test_threshold_counts_beyond_narrow_counters(ctx, tiles_option, n_rle, n_dense, tiles):
    """Small thresholds keep bit_length(theta - 1) exact counter planes and a
    sticky one, so columns where hundreds of inputs are dirty overflow the
    exact planes many times over: every theta around the powers of two (and
    its complement-side neighbours) must still equal the oracle, with dense
    inputs added in the same column (hybrid) and with one-pass tiles."""
    rng = np.random.default_rng(300 + n_rle + n_dense)
    r = 64 * STRIDE * 3 + 29
    nw = (r + 63) // 64
    dense = []
    for j in range(n_rle + n_dense):
        # almost every word dirty, density varying by input so counts spread
        p = 0.02 + 0.9 * (j % 17) / 17.0
        bits = rng.random(nw * 64) < p
        w = np.packbits(bits.astype(np.uint8), bitorder="little").view("<u8").astype(np.uint64)
        if j % 5 == 0:
            w[100:300] = 0                        # fills among the dirty words
        if j % 7 == 0:
            w[400:700] = np.uint64(0xFFFFFFFFFFFFFFFF)
        dense.append(w)
    assert tiles_option(tiles) == tq.TQ_OK
    inputs, keep = rle_inputs(ctx, dense[:n_rle], r)
    drows = [to_dev(d) for d in dense[n_rle:]]
    n = n_rle + n_dense
    for theta in (1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 32, 63, 64, 65, 127, 128, 129, 255, 256, 257,
                  n // 2, n - 1, n):
        out = empty_words(nw)
        if n_dense:
            tq.tq_threshold_hybrid(ctx, inputs, drows, r, theta, out)
        else:
            tq.tq_threshold_rle_dense(ctx, inputs, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.threshold(dense, r, theta)), theta
    # symmetric functions constant from a small count on (narrow counters with
    # a sticky plane), and their complements
    tables = [oracle.truth_interval(n, 2, 10), oracle.truth_interval(n, 3, 3), 1 - oracle.truth_threshold(n, 5),
              1 - oracle.truth_interval(n, 5, 9), oracle.truth_interval(n, 1, 1) | oracle.truth_interval(n, 6, 14)]
    for t in tables:
        t = np.asarray(t, dtype=np.uint8)
        out = empty_words(nw)
        if n_dense:
            tq.tq_symmetric_hybrid(ctx, inputs, drows, r, t, out)
        else:
            tq.tq_symmetric_rle_dense(ctx, inputs, r, t, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.symmetric(dense, r, t)), list(np.nonzero(t)[0][:12])


# ------------------------------------------- fused consumers over RLE
def count_dev():
    return torch.full((1,), -1, dtype=torch.int64, device="cuda")


@pytest.mark.parametrize("n,r,tiles", [(1, 64 * 700 + 9, 0), (37, 64 * STRIDE * 3 + 17, 2), (300, 64 * 2100 + 1, 0)])
def test_rle_fused_consumers(ctx, tiles_option, n, r, tiles):
    """tq_threshold_rle_fused / tq_symmetric_rle_fused: the result AND a
    filter, and its count, equal the oracle's result, AND and position count,
    for thresholds (constant ones included), symmetric functions (parity,
    interval, random and constant tables), with and without filter, stored
    and count-only, filtered in place, with and without indexes."""
    rng = np.random.default_rng(70 + n)
    nw = (r + 63) // 64
    dense = markov_bitmaps(1700 + n, n, r, float(rng.integers(20, 300)), float(rng.integers(100, 3000)))
    fhost = np.packbits((rng.random(nw * 64) < 0.7).astype(np.uint8), bitorder="little").view("<u8").astype(np.uint64)
    assert tiles_option(tiles) == tq.TQ_OK
    for with_index in (True, False):
        inputs, keep = rle_inputs(ctx, dense, r, with_index=with_index)
        cases = [("t", t) for t in (0, 1, 2, max(1, n // 3), n, n + 1)]
        cases += [("s", t) for t in sym_tables(n, rng)]
        for kind, arg in cases:
            want = oracle.threshold(dense, r, arg) if kind == "t" else oracle.symmetric(dense, r, arg)
            for use_filter in (False, True):
                w_out, w_cnt = oracle.consume(want, r, fhost if use_filter else None)
                filt = to_dev(fhost) if use_filter else None
                out, cnt = empty_words(nw), count_dev()
                if kind == "t":
                    tq.tq_threshold_rle_fused(ctx, inputs, r, arg, filt, out, cnt)
                else:
                    tq.tq_symmetric_rle_fused(ctx, inputs, r, arg, filt, out, cnt)
                assert tq.tq_ctx_check(ctx) == 0
                assert np.array_equal(to_host(out), w_out), (kind, use_filter)
                assert int(cnt.item()) == w_cnt, (kind, use_filter)
                cnt2 = count_dev()                       # count only
                if kind == "t":
                    tq.tq_threshold_rle_fused(ctx, inputs, r, arg, filt, None, cnt2)
                else:
                    tq.tq_symmetric_rle_fused(ctx, inputs, r, arg, filt, None, cnt2)
                assert int(cnt2.item()) == w_cnt
            # in place: the filter is the output buffer
            buf = to_dev(fhost)
            if kind == "t":
                tq.tq_threshold_rle_fused(ctx, inputs, r, arg, buf, buf, None)
            else:
                tq.tq_symmetric_rle_fused(ctx, inputs, r, arg, buf, buf, None)
            assert np.array_equal(to_host(buf), oracle.consume(want, r, fhost)[0])


def test_rle_fused_errors_and_empty(ctx):
    r = 64 * 40
    dense = markov_bitmaps(1800, 3, r, 30.0, 300.0)
    inputs, keep = rle_inputs(ctx, dense, r)
    out = empty_words(40)
    cnt = count_dev()
    assert tq.raw_threshold_rle_fused(ctx, inputs, r, 2, 0, 0, 0) == tq.TQ_EINVAL          # nothing to produce
    assert tq.raw_threshold_rle_fused(ctx, inputs, r, 2, 0, out.data_ptr() + 4, 0) == tq.TQ_EINVAL
    assert tq.raw_threshold_rle_fused(ctx, inputs, r, 2, 0, out.data_ptr(), out.data_ptr() + 16) == tq.TQ_EINVAL
    assert tq.raw_threshold_rle_fused(ctx, inputs, r, 2, out.data_ptr() + 8, out.data_ptr(), 0) == tq.TQ_EINVAL
    assert tq.raw_threshold_rle_fused(ctx, inputs, 0, 2, 0, 0, cnt.data_ptr()) == tq.TQ_OK  # r = 0 counts zero
    assert tq.tq_ctx_check(ctx) == 0
    assert int(cnt.item()) == 0


# ------------------------------------------- symmetric functions over RLE
def sym_tables(n, rng):
    t = [oracle.truth_parity(n), 1 - oracle.truth_parity(n), oracle.truth_interval(n, 2, min(n, 10)),
         oracle.truth_interval(n, min(n, 3), min(n, 3)),                     # delta: count == 3
         1 - oracle.truth_threshold(n, max(1, n // 2)),                       # count < n/2
         rng.integers(0, 2, n + 1).astype(np.uint8),
         np.ones(n + 1, dtype=np.uint8), np.zeros(n + 1, dtype=np.uint8)]
    return [np.asarray(x, dtype=np.uint8) for x in t]


@pytest.mark.parametrize("n,r,tiles", [(1, 64 * 700, 0), (6, 64 * STRIDE * 3 + 17, 2), (33, 64 * 2100 + 5, 0),
                                       (90, 64 * STRIDE * 4 + 64, 1)])
def test_symmetric_rle_matches_oracle(ctx, tiles_option, n, r, tiles):
    """Symmetric functions over compressed inputs: dense and canonical RLE
    outputs equal the oracle's, with and without checkpoint indexes, over
    several tile-range lengths; a threshold written as a truth table equals
    the threshold call."""
    rng = np.random.default_rng(40 + n)
    dense = markov_bitmaps(900 + n, n, r, float(rng.integers(20, 300)), float(rng.integers(100, 3000)))
    sp = special_bitmaps(r)
    for j in range(min(n, 3)):
        dense[j] = sp[(j + n) % 5]
    assert tiles_option(tiles) == tq.TQ_OK
    for with_index in (True, False):
        inputs, keep = rle_inputs(ctx, dense, r, with_index=with_index)
        for t in sym_tables(n, rng):
            want_dense = oracle.symmetric(dense, r, t)
            dout = empty_words((r + 63) // 64)
            tq.tq_symmetric_rle_dense(ctx, inputs, r, t, dout)
            assert tq.tq_ctx_check(ctx) == 0
            assert np.array_equal(to_host(dout), want_dense), (with_index, list(t))
            want = oracle.rle_encode(want_dense, r)
            cap = tq.tq_rle_max_words(r)
            out = empty_words(cap)
            ln = torch.zeros(1, dtype=torch.int64, device="cuda")
            tq.tq_symmetric_rle(ctx, inputs, r, t, out, cap, ln)
            assert tq.tq_ctx_check(ctx) == 0
            assert np.array_equal(to_host(out)[:int(ln.item())], want), (with_index, list(t))
    theta = max(1, n // 3)
    d1 = empty_words((r + 63) // 64)
    d2 = empty_words((r + 63) // 64)
    tq.tq_symmetric_rle_dense(ctx, inputs, r, oracle.truth_threshold(n, theta), d1)
    tq.tq_threshold_rle_dense(ctx, inputs, r, theta, d2)
    assert tq.tq_ctx_check(ctx) == 0
    assert np.array_equal(to_host(d1), to_host(d2))


@pytest.mark.parametrize("n_rle,n_dense", [(4, 3), (0, 5), (25, 25)])
def test_symmetric_hybrid(ctx, n_rle, n_dense):
    r = 64 * 1300 + 9
    n = n_rle + n_dense
    dense_all = markov_bitmaps(950 + n, n, r, 40.0, 300.0)
    inputs, keep = rle_inputs(ctx, dense_all[:n_rle], r)
    pool = dev_pool(dense_all[n_rle:])
    drows = [pool[j] for j in range(n_dense)]
    rng = np.random.default_rng(n)
    for t in sym_tables(n, rng):
        out = empty_words((r + 63) // 64)
        tq.tq_symmetric_hybrid(ctx, inputs, drows, r, t, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.symmetric(dense_all, r, t)), list(t)


@pytest.mark.parametrize("tiles", [0, 3])
def test_symmetric_rle_many_inputs(ctx, tiles_option, tiles):
    """600 inputs (more than one per lane) and inputs dirty almost everywhere,
    one tile per workgroup and three (one-pass tiles)."""
    assert tiles_option(tiles) == tq.TQ_OK
    r = 64 * STRIDE * 2 + 3
    dense = markov_bitmaps(990, 600, r, 3.0, 40.0)
    inputs, keep = rle_inputs(ctx, dense, r)
    for t in (oracle.truth_parity(600), oracle.truth_interval(600, 20, 45), oracle.truth_interval(600, 0, 5)):
        out = empty_words((r + 63) // 64)
        tq.tq_symmetric_rle_dense(ctx, inputs, r, t, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.symmetric(dense, r, t))


def test_symmetric_rle_errors(ctx):
    r = 640
    inputs, keep = rle_inputs(ctx, markov_bitmaps(1, 2, r, 5.0, 5.0), r)
    out = empty_words(10)
    arr = tq.rle_array(inputs)
    assert tq._lib.tq_symmetric_rle_dense(ctx, arr, 2, r, None, out.data_ptr(), None) == tq.TQ_EINVAL
    assert tq._lib.tq_symmetric_rle(ctx, arr, 2, r, None, out.data_ptr(), 10, out.data_ptr(), None) == tq.TQ_EINVAL
