"""Fused consumers of a dense query result on the GPU against the oracle.

tq_threshold_fused / tq_symmetric_fused write T AND filter and count its set
positions in the same pass.  Every output word and the count are compared
with the oracle (threshold or symmetric, then AND, then a position-by-position
count) on the same inputs, over ragged tails, the split-input launch shapes,
the constant special cases, in-place filtering and the argument errors.
"""
import numpy as np
import pytest
import torch

import oracle
import tqgen
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


def run_fused(ctx, rows, r, theta=None, truth=None, filt=None, want_out=True, want_count=True):
    nw = (r + 63) // 64
    out = empty_words(nw) if want_out else None
    cnt = count_dev() if want_count else None
    if truth is None:
        tq.tq_threshold_fused(ctx, rows, r, theta, filt, out, cnt)
    else:
        tq.tq_symmetric_fused(ctx, rows, r, truth, filt, out, cnt)
    assert tq.tq_ctx_check(ctx) == 0
    words = to_host(out)[:nw] if want_out else None
    c = int(cnt.item()) if want_count else None
    return words, c


@pytest.mark.parametrize("n,r", [(1, 64 * 300 + 5), (5, 64 * 1000 + 13), (16, 1 << 16), (37, 64 * 2000 + 63),
                                 (300, 64 * 200 + 1)])
def test_threshold_fused_matches_oracle(ctx, n, r):
    rng = np.random.default_rng(n)
    nw = (r + 63) // 64
    host = rand_words(rng, n, nw, 0.3)
    pool = dev_pool(host)
    rows = [pool[j] for j in range(n)]
    fhost = rand_words(rng, 1, nw, 0.6)[0]
    filt = to_dev(fhost)
    for theta in sorted({0, 1, 2, max(1, n // 3), n, n + 1}):
        want = oracle.threshold(list(host), r, theta)
        for f in (None, filt):
            wo, wc = oracle.consume(want, r, None if f is None else fhost)
            got, c = run_fused(ctx, rows, r, theta=theta, filt=f)
            assert np.array_equal(got, wo), (theta, f is None)
            assert c == wc, (theta, f is None)
            # count only, and output only
            _, c2 = run_fused(ctx, rows, r, theta=theta, filt=f, want_out=False)
            assert c2 == wc
            got3, _ = run_fused(ctx, rows, r, theta=theta, filt=f, want_count=False)
            assert np.array_equal(got3, wo)


@pytest.mark.parametrize("n", [6, 40])
def test_symmetric_fused_matches_oracle(ctx, n):
    rng = np.random.default_rng(100 + n)
    r = 64 * 777 + 31
    nw = (r + 63) // 64
    host = rand_words(rng, n, nw, 0.4)
    pool = dev_pool(host)
    rows = [pool[j] for j in range(n)]
    fhost = rand_words(rng, 1, nw, 0.5)[0]
    filt = to_dev(fhost)
    tables = [oracle.truth_parity(n), oracle.truth_interval(n, 2, min(n, 10)),
              rng.integers(0, 2, n + 1).astype(np.uint8), np.ones(n + 1, dtype=np.uint8),
              np.zeros(n + 1, dtype=np.uint8)]
    for t in tables:
        want = oracle.symmetric(list(host), r, t)
        wo, wc = oracle.consume(want, r, fhost)
        got, c = run_fused(ctx, rows, r, truth=t, filt=filt)
        assert np.array_equal(got, wo)
        assert c == wc


def test_in_place_filter_and_edges(ctx):
    rng = np.random.default_rng(7)
    n, r = 9, 64 * 500 + 3
    nw = (r + 63) // 64
    host = rand_words(rng, n, nw, 0.5)
    pool = dev_pool(host)
    rows = [pool[j] for j in range(n)]
    fhost = rand_words(rng, 1, nw, 0.5)[0]
    buf = to_dev(fhost)                                   # filter and output in one buffer
    cnt = count_dev()
    tq.tq_threshold_fused(ctx, rows, r, 4, buf, buf, cnt)
    assert tq.tq_ctx_check(ctx) == 0
    wo, wc = oracle.consume(oracle.threshold(list(host), r, 4), r, fhost)
    assert np.array_equal(to_host(buf)[:nw], wo)
    assert int(cnt.item()) == wc
    # r = 0: count 0, nothing written
    cnt = count_dev()
    tq.tq_threshold_fused(ctx, rows, 0, 1, None, None, cnt)
    assert tq.tq_ctx_check(ctx) == 0
    assert int(cnt.item()) == 0
    # a single position
    _, c = run_fused(ctx, rows, 1, theta=1)
    assert c == oracle.consume(oracle.threshold(list(host), 1, 1), 1)[1]


def test_fused_argument_errors(ctx):
    n, r = 3, 640
    pool = torch.zeros((n, 10), dtype=torch.int64, device="cuda")
    ptrs = tq.ptr_array([pool[j] for j in range(n)])
    out = torch.zeros(12, dtype=torch.int64, device="cuda")
    cnt = count_dev()
    # neither output nor count
    assert tq.raw_threshold_fused(ctx, ptrs, n, r, 1, None, None, None) == tq.TQ_EINVAL
    # filter overlapping the output without being it
    assert tq.raw_threshold_fused(ctx, ptrs, n, r, 1, out.data_ptr() + 8, out.data_ptr(), None) == tq.TQ_EINVAL
    # misaligned filter / count
    assert tq.raw_threshold_fused(ctx, ptrs, n, r, 1, out.data_ptr() + 4, None, cnt.data_ptr()) == tq.TQ_EINVAL
    assert tq.raw_threshold_fused(ctx, ptrs, n, r, 1, None, out.data_ptr(), cnt.data_ptr() + 4) == tq.TQ_EINVAL
    # count inside the output
    assert tq.raw_threshold_fused(ctx, ptrs, n, r, 1, None, out.data_ptr(), out.data_ptr() + 16) == tq.TQ_EINVAL
    # output overlapping an input
    assert tq.raw_threshold_fused(ctx, ptrs, n, r, 1, None, pool[1].data_ptr(), None) == tq.TQ_EINVAL
    # valid: count only
    assert tq.raw_threshold_fused(ctx, ptrs, n, r, 1, None, None, cnt.data_ptr()) == tq.TQ_OK
    assert tq.tq_ctx_check(ctx) == 0
    assert int(cnt.item()) == 0


def test_fused_large_config(ctx):
    """N=256, r=2^26 (2 GiB), the large configuration: the fused result of
    T_theta AND filter and its count equal the oracle's consume step on the
    oracle's threshold, every word (stored and count-only)."""
    bs = tqgen.large_set()
    pool = torch.empty((bs.n, bs.nwords), dtype=torch.int64, device="cuda")
    tqgen.fill_gpu(bs, pool.view(-1))
    rows = [pool[j] for j in range(bs.n)]
    r, nw = bs.r_bits, bs.nwords
    host_all = pool.cpu().numpy().view(np.uint64)
    host = [host_all[j] for j in range(bs.n)]
    filt = rows[3]                                     # an input as filter (aliasing allowed)
    for theta in (2, 16, 255):
        want_words, want_count = oracle.consume(oracle.threshold(host, r, theta), r, host[3])
        out = torch.empty(nw, dtype=torch.int64, device="cuda")
        cnt = count_dev()
        tq.tq_threshold_fused(ctx, rows, r, theta, filt, out, cnt)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), want_words), theta
        assert int(cnt.item()) == want_count, theta
        cnt2 = count_dev()
        tq.tq_threshold_fused(ctx, rows, r, theta, filt, None, cnt2)
        assert tq.tq_ctx_check(ctx) == 0
        assert int(cnt2.item()) == want_count, theta
