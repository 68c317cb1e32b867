"""Weighted threshold queries on the GPU against the oracle.

Every output word is compared with the oracle's weighted threshold (the
definition: the sum of the weights of the inputs that have the bit), over
weight classes of every counter width, zero and duplicate weights, totals up
to 2^32 - 1, ragged tails and the theta edges, with pruning on (classes of
at most 16 inputs, heaviest first, lanes stopping once decided) and off;
small weights are also checked against the unweighted kernel on replicated
inputs (section 2.3).
"""
import numpy as np
import pytest
import torch

import oracle
from gpuhelp import dev_pool, empty_words, to_host
from paper_1402_4073_amd import binding as tq

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tq.tq_create(0)
    yield c
    tq.tq_destroy(c)


@pytest.fixture(params=[1, 0], ids=["prune", "noprune"])
def prune(ctx, request):
    tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, request.param)
    yield request.param
    tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, 1)


def rand_words(rng, n, nw, p):
    bits = rng.random((n, nw * 64)) < p
    return np.packbits(bits.astype(np.uint8), axis=1, bitorder="little").view("<u8").astype(np.uint64)


CASES = [
    ("unit", lambda rng, n: [1] * n),
    ("small", lambda rng, n: list(rng.integers(0, 5, n))),
    ("wide", lambda rng, n: list(rng.integers(1, 1000, n))),
    ("powers", lambda rng, n: [1 << int(k) for k in rng.integers(0, 12, n)]),
    ("one-heavy", lambda rng, n: [1] * (n - 1) + [n]),
]


@pytest.mark.parametrize("n,r", [(1, 64 * 100 + 1), (7, 64 * 900 + 13), (40, 64 * 1024), (300, 64 * 150 + 63)])
@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_weighted_matches_oracle(ctx, prune, n, r, case):
    rng = np.random.default_rng(n * 7 + len(case))
    weights = [int(x) for x in dict(CASES)[case](rng, n)]
    nw = (r + 63) // 64
    host = rand_words(rng, n, nw, 0.35)
    pool = dev_pool(host)
    rows = [pool[j] for j in range(n)]
    total = sum(weights)
    thetas = {0, 1, total, total + 1, max(1, total // 2), max(1, total // 7), int(rng.integers(0, total + 2))}
    for theta in sorted(thetas):
        out = empty_words(nw)
        tq.tq_threshold_weighted(ctx, rows, weights, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out)[:nw], oracle.weighted_threshold(list(host), weights, r, theta)), \
            (case, theta)


def test_weighted_equals_replication(ctx, prune):
    rng = np.random.default_rng(5)
    n, r = 12, 64 * 2000 + 7
    nw = (r + 63) // 64
    host = rand_words(rng, n, nw, 0.3)
    pool = dev_pool(host)
    rows = [pool[j] for j in range(n)]
    weights = [int(x) for x in rng.integers(0, 4, n)]
    rep = [rows[j] for j in range(n) for _ in range(weights[j])]
    for theta in range(1, sum(weights) + 2, 3):
        a = empty_words(nw)
        b = empty_words(nw)
        tq.tq_threshold_weighted(ctx, rows, weights, r, theta, a)
        tq.tq_threshold(ctx, rep, r, theta, b)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(a), to_host(b)), theta


def test_weighted_extreme_totals(ctx, prune):
    """Totals near 2^32 - 1 (the widest total counter) and classes of more
    than 8191 equal weights (the widest class counter)."""
    rng = np.random.default_rng(9)
    r = 64 * 70 + 5
    nw = (r + 63) // 64
    host = rand_words(rng, 4, nw, 0.5)
    pool = dev_pool(host)
    rows = [pool[j] for j in range(4)]
    weights = [(1 << 31) - 1, (1 << 30), (1 << 29) + 12345, 7]
    total = sum(weights)
    assert total < (1 << 32)
    for theta in (1, 8, (1 << 30), (1 << 31), (1 << 31) + 1, total - 7, total - 6, total, total + 1):
        out = empty_words(nw)
        tq.tq_threshold_weighted(ctx, rows, weights, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.weighted_threshold(list(host), weights, r, theta)), theta
    # 9000 inputs of weight 2 plus one of weight 5 (aliased rows of a small pool)
    small = rand_words(rng, 64, nw, 0.5)
    spool = dev_pool(small)
    idx = [int(x) for x in rng.integers(0, 64, 9001)]
    rows2 = [spool[i] for i in idx]
    w2 = [2] * 9000 + [5]
    hostlist = [small[i] for i in idx]
    for theta in (1, 2, 9000, 9005, 18000, 18005, 18006):
        out = empty_words(nw)
        tq.tq_threshold_weighted(ctx, rows2, w2, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out), oracle.weighted_threshold(hostlist, w2, r, theta)), theta


def test_weighted_errors(ctx):
    pool = torch.zeros((3, 10), dtype=torch.int64, device="cuda")
    rows = [pool[j] for j in range(3)]
    out = torch.zeros(10, dtype=torch.int64, device="cuda")
    assert tq.raw_threshold_weighted(ctx, rows, None, 640, 1, out.data_ptr()) == tq.TQ_EINVAL
    assert tq.raw_threshold_weighted(ctx, rows, [1 << 31, 1 << 31, 1], 640, 1, out.data_ptr()) == tq.TQ_EINVAL
    assert tq.raw_threshold_weighted(ctx, rows, [1, 2, 3], 640, 1, pool[0].data_ptr()) == tq.TQ_EINVAL
    assert tq.raw_threshold_weighted(ctx, [], [], 640, 1, out.data_ptr()) == tq.TQ_EINVAL
    # all weights zero: nothing reaches theta >= 1
    assert tq.raw_threshold_weighted(ctx, rows, [0, 0, 0], 640, 1, out.data_ptr()) == tq.TQ_OK
    assert tq.tq_ctx_check(ctx) == 0
    assert int(out.abs().sum().item()) == 0
