"""Inputs split over workgroups (short bitmaps, many inputs) against the oracle.

Bitmaps too short to fill the device with 64-word column groups (and at
least 4 MiB of input) are counted in parts of at least 32 inputs on separate
workgroups, and a second kernel
adds the parts' binary counts (section 4.4.2) before the epilogue.  Every
shape below is checked to take that path by the rule the library states
(fewer than one column group per compute unit, at least 4 MiB of input,
at least 8 parts of 32 inputs), then every output word is compared with the oracle for thresholds
(the constant ends included), parity, intervals, a complement and a lookup
table, over ragged tails and part sizes that do not divide N.
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


def num_cus():
    return torch.cuda.get_device_properties(0).multi_processor_count


def split_parts(n, nw):
    """The number of parts the library uses (0: no split)."""
    groups = (nw + 63) // 64
    target = num_cus() * 8
    if groups == 0 or groups * 8 >= target or n < 256 or n * nw * 8 < (4 << 20):
        return 0
    parts = min((target + groups - 1) // groups, n // 32, 256)
    return parts if parts >= 8 else 0


def rand_words(rng, n, nw, p):
    bits = rng.random((n, nw * 64)) < p
    return np.packbits(bits.astype(np.uint8), axis=1, bitorder="little").view("<u8").astype(np.uint64)


def table_truth(n, salt):
    c = np.arange(n + 1, dtype=np.uint64)
    f = ((((c + np.uint64(salt)) * np.uint64(2654435761)) >> np.uint64(7)) & np.uint64(1)).astype(np.uint8)
    f[:12] = [1, 0, 1, 1, 0, 1, 0, 0, 1, 0, 1, 0][:min(12, n + 1)]
    return f


# (words, inputs): one column group, a few, parts of 32 and of many inputs,
# part sizes that do not divide N, the largest counter width
SHAPES = [(64, 8192), (200, 5000), (64 * 7 + 5, 1500), (4096, 4096), (64 * 200 + 1, 300), (150, 65535)]


@pytest.mark.parametrize("nw,n", SHAPES)
def test_split_matches_oracle(ctx, nw, n):
    assert split_parts(n, nw) >= 8, "shape must take the split path"
    rng = np.random.default_rng(nw * 7 + n)
    r = nw * 64 - 19
    distinct = min(n, 512)
    dens = rng.uniform(0.02, 0.6, distinct)
    base = np.stack([rand_words(rng, 1, nw, d)[0] for d in dens])
    pool = dev_pool(list(base))
    pick = rng.integers(0, distinct, n) if n > distinct else np.arange(n)
    rows = [pool[int(i)] for i in pick]
    host = [base[int(i)] for i in pick]
    mean = float(np.mean(dens)) * n
    for theta in sorted({0, 1, 2, int(mean), int(mean) + 1, n - 1, n, n + 1}):
        print("split case nw=%d n=%d theta=%d" % (nw, n, theta), flush=True)
        out = empty_words(nw)
        tq.tq_threshold(ctx, rows, r, theta, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out)[:nw], oracle.threshold(host, r, theta)), theta
    cases = [oracle.truth_parity(n), 1 - oracle.truth_parity(n), oracle.truth_interval(n, 2, max(2, int(mean))),
             oracle.truth_interval(n, 0, int(mean)), table_truth(n, nw)]
    for k, f in enumerate(cases):
        out = empty_words(nw)
        tq.tq_symmetric(ctx, rows, r, f, out)
        assert tq.tq_ctx_check(ctx) == 0
        assert np.array_equal(to_host(out)[:nw], oracle.symmetric(host, r, f)), k


@pytest.mark.parametrize("nw,n", [(200, 5000), (4096, 4096)])
def test_split_option_off_gives_same_bits(ctx, nw, n):
    rng = np.random.default_rng(nw + 3 * n)
    base = rand_words(rng, 256, nw, 0.1)
    pool = dev_pool(list(base))
    rows = [pool[int(i)] for i in rng.integers(0, 256, n)]
    r = nw * 64 - 1
    try:
        for theta in (1, n // 10, n // 2):
            a, b = empty_words(nw), empty_words(nw)
            tq.tq_threshold(ctx, rows, r, theta, a)
            tq.tq_set_option(ctx, tq.TQ_OPTION_SPLIT, 0)
            tq.tq_threshold(ctx, rows, r, theta, b)
            tq.tq_set_option(ctx, tq.TQ_OPTION_SPLIT, 1)
            assert tq.tq_ctx_check(ctx) == 0
            assert torch.equal(a, b), theta
    finally:
        tq.tq_set_option(ctx, tq.TQ_OPTION_SPLIT, 1)


def test_split_equals_unsplit_shapes(ctx):
    """The same query with and without the split (a longer bitmap whose
    prefix is the short one keeps the single-kernel path): equal prefixes."""
    rng = np.random.default_rng(4)
    n, nw_short = 1000, 600
    nw_long = 64 * num_cus()               # one column group per compute unit: no split
    assert split_parts(n, nw_short) >= 8 and split_parts(n, nw_long) == 0
    base = rand_words(rng, n, nw_long, 0.2)
    pool = dev_pool(list(base))
    rows_long = [pool[j] for j in range(n)]
    rows_short = [pool[j][:nw_short] for j in range(n)]
    for theta in (3, 200, 201, 999):
        a, b = empty_words(nw_long), empty_words(nw_short)
        tq.tq_threshold(ctx, rows_long, nw_long * 64, theta, a)
        tq.tq_threshold(ctx, rows_short, nw_short * 64, theta, b)
        assert tq.tq_ctx_check(ctx) == 0
        assert torch.equal(a[:nw_short], b[:nw_short]), theta
