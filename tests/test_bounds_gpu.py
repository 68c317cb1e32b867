"""Writes stay inside the outputs they are given.

Every output of every entry point is placed between guard words holding a
canary pattern; after the call the result must equal the oracle's and every
guard word must be unchanged.  Covered: dense thresholds over all launch
shapes (one input, the single-wave and split-input shapes, thousands of
inputs, Looped thresholds at both ends, constant results), symmetric tables,
weighted thresholds, fused outputs and counts, compressed-input queries with
dense and compressed outputs (capacity exactly the length, and too small:
then only the first out_cap words are written and TQ_ECAPACITY is reported),
encoding, decoding, the per-position counter variant and batches.
"""
import numpy as np
import pytest
import torch

import oracle
import tqgen
from gpuhelp import dev_pool, to_dev, to_host
from paper_1402_4073_amd import binding as tq

pytestmark = pytest.mark.gpu

G = 64                                     # guard words on each side
CANARY = np.uint64(0xC3A5C3A5DEADBEEF)


@pytest.fixture(scope="module")
def ctx():
    c = tq.tq_create(0)
    yield c
    tq.tq_destroy(c)


def guarded(nwords):
    """(whole buffer, view of nwords words between the guards)."""
    buf = torch.full((nwords + 2 * G,), int(CANARY.view(np.int64)), dtype=torch.int64, device="cuda")
    return buf, buf[G:G + max(nwords, 0)]


def guards_intact(buf, nwords):
    h = to_host(buf)
    return bool(np.all(h[:G] == CANARY) and np.all(h[G + nwords:] == CANARY))


def rand_words(rng, n, nw, p):
    bits = rng.random((n, nw * 64)) < p
    return np.packbits(bits.astype(np.uint8), axis=1, bitorder="little").view("<u8").astype(np.uint64)


@pytest.fixture(scope="module")
def dense_pool():
    rng = np.random.default_rng(91)
    nw = 64 * 1000 + 1
    host = rand_words(rng, 300, nw, 0.35)
    return host, dev_pool(list(host)), nw


@pytest.mark.parametrize("n,r", [(1, 64 * 3 + 5), (16, 64 * 1000 + 1), (37, 64 * 513), (300, 64 * 257 + 63),
                                 (5000, 64 * 40 + 7)])
def test_dense_outputs_stay_in_bounds(ctx, dense_pool, n, r):
    host, pool, _ = dense_pool
    nw = (r + 63) // 64
    members = [j % 300 for j in range(n)]            # thousands of inputs repeat rows (aliasing)
    rows = [pool[m] for m in members]
    hb = [host[m][:nw] for m in members]
    for theta in sorted({0, 1, 2, 3, max(1, n // 2), max(1, n - 2), n, n + 1}):
        buf, out = guarded(nw)
        tq.tq_threshold(ctx, rows, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert guards_intact(buf, nw), theta
        assert np.array_equal(to_host(out), oracle.threshold(hb, r, theta)), theta
    c = np.arange(n + 1, dtype=np.uint64)
    f = (((c * np.uint64(2654435761)) >> np.uint64(7)) & np.uint64(1)).astype(np.uint8)
    buf, out = guarded(nw)
    tq.tq_symmetric(ctx, rows, r, f, out)
    assert guards_intact(buf, nw)
    assert np.array_equal(to_host(out), oracle.symmetric(hb, r, f))


def test_weighted_and_fused_stay_in_bounds(ctx, dense_pool):
    host, pool, _ = dense_pool
    r = 64 * 700 + 9
    nw = (r + 63) // 64
    rows = [pool[j] for j in range(10)]
    hb = [host[j][:nw] for j in range(10)]
    w = [1, 2, 3, 4, 1, 2, 3, 4, 5, 9]
    buf, out = guarded(nw)
    tq.tq_threshold_weighted(ctx, rows, w, r, 11, out)
    assert guards_intact(buf, nw)
    assert np.array_equal(to_host(out), oracle.weighted_threshold(hb, w, r, 11))
    filt_host = host[50][:nw]
    filt = to_dev(filt_host)
    for theta in (0, 4, 11):                          # a constant result, then computed ones
        buf, out = guarded(nw)
        cbuf, cnt = guarded(1)
        tq.tq_threshold_fused(ctx, rows, r, theta, filt, out, cnt)
        assert guards_intact(buf, nw) and guards_intact(cbuf, 1), theta
        want, want_c = oracle.consume(oracle.threshold(hb, r, theta), r, filt_host)
        assert np.array_equal(to_host(out), want) and int(to_host(cnt)[0]) == want_c, theta


@pytest.fixture(scope="module")
def rle_set(ctx):
    n, r = 20, 64 * tq.TQ_RLE_INDEX_STRIDE * 2 + 33
    ms = tqgen.markov_fixed(93, n, r, 30.0, 700.0)
    dense = [ms.words(j) for j in range(n)]
    d = dev_pool(dense)
    pool, offs, lens, idx = tq.encode_pool(ctx, [d[j] for j in range(n)], r)
    inputs = [(pool[offs[j]:], lens[j], idx[j]) for j in range(n)]
    return dense, inputs, r, (pool, d)


def test_compressed_outputs_stay_in_bounds(ctx, rle_set):
    dense, inputs, r, keep = rle_set
    nw = (r + 63) // 64
    for theta in (2, 7):
        want = oracle.threshold(dense, r, theta)
        buf, out = guarded(nw)
        tq.tq_threshold_rle_dense(ctx, inputs, r, theta, out)
        assert guards_intact(buf, nw) and np.array_equal(to_host(out), want)
        # compressed output: capacity exactly the length, then too small
        stream = oracle.rle_encode(want, r)
        L = len(stream)
        for cap in (L, L // 2):
            buf, out = guarded(cap)
            lbuf, ln = guarded(1)
            tq.raw_threshold_rle(ctx, inputs, r, theta, out.data_ptr(), cap, ln.data_ptr())
            st = tq.tq_ctx_check(ctx)
            assert st == (tq.TQ_OK if cap == L else tq.TQ_ECAPACITY), (theta, cap)
            assert guards_intact(buf, cap) and guards_intact(lbuf, 1), (theta, cap)
            assert int(to_host(ln)[0]) == L
            assert np.array_equal(to_host(out), stream[:cap]), (theta, cap)
        # count only and filtered in place
        cbuf, cnt = guarded(1)
        tq.tq_threshold_rle_fused(ctx, inputs, r, theta, None, None, cnt)
        assert guards_intact(cbuf, 1) and int(to_host(cnt)[0]) == oracle.count(want, r)
    f = oracle.truth_interval(len(dense), 2, 5)
    want = oracle.rle_encode(oracle.symmetric(dense, r, f), r)
    buf, out = guarded(len(want))
    lbuf, ln = guarded(1)
    tq.tq_symmetric_rle(ctx, inputs, r, f, out, len(want), ln)
    assert guards_intact(buf, len(want)) and guards_intact(lbuf, 1)
    assert np.array_equal(to_host(out), want)


def test_codec_outputs_stay_in_bounds(ctx, rle_set):
    dense, inputs, r, keep = rle_set
    nw = (r + 63) // 64
    src = to_dev(dense[3])
    stream = oracle.rle_encode(dense[3], r)
    L = len(stream)
    for cap in (L, L // 2):
        buf, out = guarded(cap)
        lbuf, ln = guarded(1)
        ibuf, idx = guarded(tq.tq_rle_index_words(r))
        tq.tq_rle_encode(ctx, src, r, out, cap, ln, idx)
        st = tq.tq_ctx_check(ctx)
        assert st == (tq.TQ_OK if cap == L else tq.TQ_ECAPACITY)
        assert guards_intact(buf, cap) and guards_intact(lbuf, 1) and guards_intact(ibuf, tq.tq_rle_index_words(r))
        assert np.array_equal(to_host(out), stream[:cap])
    buf, out = guarded(nw)
    tq.tq_rle_decode(ctx, inputs[3], r, out)
    assert guards_intact(buf, nw)
    assert np.array_equal(to_host(out), oracle.rle_decode(stream, r))


def test_variant_and_batch_outputs_stay_in_bounds(ctx, dense_pool):
    host, pool, _ = dense_pool
    r = 64 * 300 + 17
    nw = (r + 63) // 64
    n = 24
    rows = [pool[j] for j in range(n)]
    hb = [host[j][:nw] for j in range(n)]
    bms = [{"dense": rows[j], "rle": None, "ones": 0, "runs": 0} for j in range(n)]
    buf, out = guarded(nw)
    tq.tq_threshold_variant(ctx, bms, r, 5, tq.TQ_VARIANT_COUNTER, out)
    assert guards_intact(buf, nw) and np.array_equal(to_host(out), oracle.threshold(hb, r, 5))
    specs, bufs, wants = [], [], []
    for i, (k, rr) in enumerate([(1, 64), (3, 65), (17, 64 * 70 + 1), (24, r), (9, 64 * 2 + 63)] * 3):
        nwk = (rr + 63) // 64
        b, o = guarded(nwk)
        theta = 1 + i % k
        specs.append({"inputs": rows[:k], "r_bits": rr, "out": o, "theta": theta, "tag": i})
        bufs.append((b, nwk))
        wants.append(oracle.threshold([h[:nwk] for h in hb[:k]], rr, theta))
    bt = tq.tq_batch_submit(ctx, tq.BatchQueries(specs))
    tq.tq_batch_wait(bt)
    tq.tq_batch_release(bt)
    for (b, nwk), sp, w in zip(bufs, specs, wants):
        assert guards_intact(b, nwk), sp["tag"]
        assert np.array_equal(to_host(sp["out"]), w), sp["tag"]
