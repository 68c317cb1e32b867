"""The allocation-free fused threshold entry point against tq_threshold_fused.

tq_threshold_fused_noalloc keeps its device scratch (the pointer array and the
per-column-group partial counts) in one fixed array per device.  Its output
words and count must equal those of tq_threshold_fused, called through the C
ABI on the same inputs, bit for bit; the oracle checks both.  Two calls in a
row, the second on a smaller input, show that what the first left in the
scratch array does not leak into the second.  Sizes beyond the array are
refused before anything is queued.
"""
import numpy as np
import pytest
import torch

import oracle
from gpuhelp import dev_pool, empty_words, to_dev, to_host
from paper_1402_4073_amd import binding as tq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tq.tq_create(0)
    yield c
    tq.tq_destroy(c)


def rand_words(rng, n, nw, p):
    bits = rng.random((n, nw * 64)) < p
    return np.packbits(bits.astype(np.uint8), axis=1, bitorder="little").view("<u8").astype(np.uint64)


def count_dev():
    return torch.full((1,), -1, dtype=torch.int64, device="cuda")


def both(ctx, rows, r, theta, filt):
    nw = (r + 63) // 64
    out_a, cnt_a = empty_words(nw), count_dev()
    out_b, cnt_b = empty_words(nw), count_dev()
    tq.tq_threshold_fused(ctx, rows, r, theta, filt, out_a, cnt_a)
    tq.tq_threshold_fused_noalloc(ctx, rows, r, theta, filt, out_b, cnt_b)
    assert tq.tq_ctx_check(ctx) == 0
    return (to_host(out_a)[:nw], int(cnt_a.item())), (to_host(out_b)[:nw], int(cnt_b.item()))


# (n, r) pairs: the second of each pair is smaller than the first in inputs
# and words, so a stale pointer or partial count from the first would show
PAIRS = [
    ((300, 64 * 5000 + 17), (7, 64 * 900 + 3)),          # split-input shapes, then the small-N kernel
    ((40, 64 * 140000 + 5), (33, 64 * 131072 + 63)),     # one wave per column group, pruned
    ((1000, 64 * 2100 + 1), (999, 64 * 2099)),
]


@pytest.mark.parametrize("first,second", PAIRS)
def test_noalloc_matches_fused_twice(ctx, first, second):
    rng = np.random.default_rng(first[0] * 7 + second[0])
    for n, r in (first, second):
        print("noalloc case n=%d r=%d" % (n, r), flush=True)
        nw = (r + 63) // 64
        host = rand_words(rng, n, nw, 0.05 + 0.4 * rng.random())
        pool = dev_pool(host)
        rows = [pool[j] for j in range(n)]
        fhost = rand_words(rng, 1, nw, 0.7)[0]
        filt = to_dev(fhost)
        for theta in sorted({0, 1, 2, max(1, n // 4), n - 1, n, n + 1}):
            want = oracle.threshold(list(host), r, theta)
            for f, fh in ((None, None), (filt, fhost)):
                (wa, ca), (wb, cb) = both(ctx, rows, r, theta, f)
                assert np.array_equal(wb, wa), (n, r, theta, f is None)
                assert cb == ca, (n, r, theta, f is None)
                wo, wc = oracle.consume(want, r, fh)
                assert np.array_equal(wb, wo) and cb == wc, (n, r, theta, f is None)


def test_noalloc_count_only_and_output_only(ctx):
    rng = np.random.default_rng(5)
    n, r = 64, 64 * 3000 + 9
    nw = (r + 63) // 64
    host = rand_words(rng, n, nw, 0.2)
    pool = dev_pool(host)
    rows = [pool[j] for j in range(n)]
    want = oracle.threshold(list(host), r, 13)
    cnt = count_dev()
    tq.tq_threshold_fused_noalloc(ctx, rows, r, 13, None, None, cnt)
    out = empty_words(nw)
    tq.tq_threshold_fused_noalloc(ctx, rows, r, 13, None, out, None)
    assert tq.tq_ctx_check(ctx) == 0
    assert int(cnt.item()) == oracle.consume(want, r, None)[1]
    assert np.array_equal(to_host(out)[:nw], want)
    # r_bits == 0: the count is zero
    tq.tq_threshold_fused_noalloc(ctx, rows, 0, 13, None, None, cnt)
    assert tq.tq_ctx_check(ctx) == 0
    assert int(cnt.item()) == 0


def test_noalloc_refuses_sizes_beyond_scratch(ctx):
    # 2^20 + 1 column groups of partial counts do not fit next to the
    # pointer array in 4 MiB; without a count the same query runs
    nw = (1 << 26) + 64
    r = nw * 64
    src = torch.zeros(nw, dtype=torch.int64, device="cuda")
    src[::4097] = -1
    out = empty_words(nw)
    cnt = count_dev()
    st = tq.raw_threshold_fused_noalloc(ctx, [src, src], r, 2, 0, out.data_ptr(), cnt.data_ptr())
    assert st == tq.TQ_EINVAL
    assert tq.tq_ctx_check(ctx) == 0
    assert int(cnt.item()) == -1            # nothing was queued
    tq.tq_threshold_fused_noalloc(ctx, [src, src], r, 2, None, out, None)
    ref = empty_words(nw)
    tq.tq_threshold_fused(ctx, [src, src], r, 2, None, ref, None)
    assert tq.tq_ctx_check(ctx) == 0
    assert torch.equal(out, ref)
    del src, out, ref
    torch.cuda.empty_cache()


def test_noalloc_argument_errors(ctx):
    nw = 100
    a = to_dev(np.arange(nw, dtype=np.uint64))
    out = empty_words(nw)
    assert tq.raw_threshold_fused_noalloc(ctx, [a], nw * 64, 1, 0, 0, 0) == tq.TQ_EINVAL      # no output, no count
    assert tq.raw_threshold_fused_noalloc(ctx, [], nw * 64, 1, 0, out.data_ptr(), 0) == tq.TQ_EINVAL
    assert tq.raw_threshold_fused_noalloc(ctx, [a], nw * 64, 1, 0, a.data_ptr(), 0) == tq.TQ_EINVAL  # overlap
    assert tq.tq_ctx_check(ctx) == 0
