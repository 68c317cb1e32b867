"""Queries captured into a HIP graph and replayed, against the oracle.

Five kinds of query (a threshold, a symmetric function with a truth table, a
fused count with a filter, a threshold over compressed inputs with dense
output and a symmetric function with canonical compressed output) are
staged once on a stream, captured on it, and the graph is replayed three
times.  Between replays eager calls stage many other pointer arrays (so that
every array not held by the graph is evicted) and grow the workspace; the
outputs are cleared before each replay and every replay must write the
oracle's results again.  A call whose arguments were never staged is
refused during capture without breaking it.
"""
import numpy as np
import pytest
import torch

import oracle
import tqgen
from gpuhelp import dev_pool, empty_words, to_dev, to_host
from paper_1402_4073_amd import binding as tq

pytestmark = pytest.mark.gpu


def rand_words(rng, n, nw, p):
    bits = rng.random((n, nw * 64)) < p
    return np.packbits(bits.astype(np.uint8), axis=1, bitorder="little").view("<u8").astype(np.uint64)


def table_truth(n):
    c = np.arange(n + 1, dtype=np.uint64)
    f = (((c * np.uint64(2654435761)) >> np.uint64(9)) & np.uint64(1)).astype(np.uint8)
    f[:20] = [1, 0, 1, 0, 1, 1, 0, 1, 0, 1, 0, 0, 1, 0, 1, 0, 1, 0, 1, 0]
    return f


def test_captured_queries_replay():
    ctx = tq.tq_create(0)
    try:
        rng = np.random.default_rng(5)
        s = torch.cuda.Stream()
        # uncompressed inputs
        n, r = 40, 64 * 700 + 13
        nw = (r + 63) // 64
        host = rand_words(rng, n, nw, 0.3)
        pool = dev_pool(host)
        rows = [pool[j] for j in range(n)]
        fhost = rand_words(rng, 1, nw, 0.6)[0]
        filt = to_dev(fhost)
        f_tab = table_truth(n)
        # compressed inputs
        n2, r2 = 30, 64 * tq.TQ_RLE_INDEX_STRIDE * 3 + 5
        nw2 = (r2 + 63) // 64
        ms = tqgen.markov_fixed(77, n2, r2, 40.0, 900.0)
        dense2 = [ms.words(j) for j in range(n2)]
        d2 = dev_pool(dense2)
        cpool, offs, lens, idx = tq.encode_pool(ctx, [d2[j] for j in range(n2)], r2)
        rle_in = [(cpool[offs[j]:], lens[j], idx[j]) for j in range(n2)]
        f2 = oracle.truth_interval(n2, 2, 6)
        cap = tq.tq_rle_max_words(r2)
        # outputs
        out_t, out_s, out_rd = empty_words(nw), empty_words(nw), empty_words(nw2)
        cnt_f = torch.zeros(1, dtype=torch.int64, device="cuda")
        rle_out = torch.zeros(cap, dtype=torch.int64, device="cuda")
        rle_len = torch.zeros(1, dtype=torch.int64, device="cuda")

        def queries():
            tq.tq_threshold(ctx, rows, r, 7, out_t, s)
            tq.tq_symmetric(ctx, rows, r, f_tab, out_s, s)
            tq.tq_threshold_fused(ctx, rows, r, 12, filt, None, cnt_f, s)
            tq.tq_threshold_rle_dense(ctx, rle_in, r2, 3, out_rd, s)
            tq.tq_symmetric_rle(ctx, rle_in, r2, f2, rle_out, cap, rle_len, s)

        want_t = oracle.threshold(list(host), r, 7)
        want_s = oracle.symmetric(list(host), r, f_tab)
        want_c = oracle.consume(oracle.threshold(list(host), r, 12), r, fhost)[1]
        want_rd = oracle.threshold(dense2, r2, 3)
        want_rs = oracle.rle_encode(oracle.symmetric(dense2, r2, f2), r2)

        with torch.cuda.stream(s):
            queries()                       # stages every array on the capture stream
        s.synchronize()
        assert tq.tq_ctx_check(ctx, s) == 0

        g = torch.cuda.CUDAGraph()
        other = [pool[(j + 1) % n] for j in range(n)]       # an array never staged
        with torch.cuda.graph(g, stream=s):
            queries()
            st = tq.raw_threshold(ctx, tq.ptr_array(other), n, r, 5, out_t.data_ptr(), s)
        assert st == tq.TQ_EINVAL

        big_r = 64 * tq.TQ_RLE_INDEX_STRIDE * 40 + 3
        big = tqgen.markov_fixed(78, 8, big_r, 30.0, 500.0)
        big_dev = dev_pool([big.words(j) for j in range(8)])
        bpool, boffs, blens, bidx = tq.encode_pool(ctx, [big_dev[j] for j in range(8)], big_r)
        big_in = [(bpool[boffs[j]:], blens[j], bidx[j]) for j in range(8)]
        big_out = torch.zeros(tq.tq_rle_max_words(big_r), dtype=torch.int64, device="cuda")
        big_len = torch.zeros(1, dtype=torch.int64, device="cuda")
        scratch = empty_words(nw)
        for rep in range(3):
            for t in (out_t, out_s, out_rd, rle_out, rle_len, cnt_f):
                t.zero_()
            # eager work between replays: 70 other pointer arrays (every array
            # the graph does not hold is evicted) and a larger workspace
            for k in range(70):
                perm = [pool[(j * 7 + k) % n] for j in range(1 + k % 9)]
                tq.tq_threshold(ctx, perm, r, 1, scratch)
            tq.tq_threshold_rle(ctx, big_in, big_r, 2 + rep, big_out, big_out.numel(), big_len)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert tq.tq_ctx_check(ctx) == 0
            assert np.array_equal(to_host(out_t), want_t), rep
            assert np.array_equal(to_host(out_s), want_s), rep
            assert int(cnt_f.item()) == want_c, rep
            assert np.array_equal(to_host(out_rd), want_rd), rep
            L = int(rle_len.item())
            assert L == len(want_rs) and np.array_equal(to_host(rle_out)[:L], want_rs), rep
    finally:
        torch.cuda.synchronize()
        tq.tq_destroy(ctx)
