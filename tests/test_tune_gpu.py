"""Autotuner: tuned launch shapes give the oracle's results, the cache
exports and imports as text, malformed or impossible entries are refused,
and tuned batch schedules keep batches exact."""
import numpy as np
import pytest
import torch

import oracle
from gpuhelp import dev_pool, empty_words, to_dev, to_host
from paper_1402_4073_amd import binding as tq

pytestmark = pytest.mark.gpu


def rand_words(rng, n, nw, p):
    bits = rng.random((n, nw * 64)) < p
    return np.packbits(bits.astype(np.uint8), axis=1, bitorder="little").view("<u8").astype(np.uint64)


@pytest.fixture
def tctx():
    c = tq.tq_create(0)
    tq.tq_set_option(c, tq.TQ_OPTION_AUTOTUNE, 1)
    yield c
    tq.tq_destroy(c)


def parse(text):
    rows = []
    for line in text.strip().splitlines():
        cls, params, us = line.split(":")
        rows.append(([int(x) for x in cls.split()], [int(x) for x in params.split()], float(us)))
    return rows


SHAPES = [(16, 1 << 20, True), (300, 64 * 200 + 5, True), (1000, 64 * 64, True), (37, 64 * 1000 + 13, False)]


def run_shapes(ctx, rng):
    results = []
    for n, r, aligned in SHAPES:
        nw = (r + 63) // 64
        host = rand_words(rng, n, nw, 0.2)
        if aligned:
            pool = dev_pool(host)
            rows = [pool[j] for j in range(n)]
        else:
            # every row starts 8 bytes past a 16-byte boundary: two-word lanes are not allowed
            pad = np.zeros(1, dtype=np.uint64)
            pool = to_dev(np.concatenate([np.concatenate([pad, h]) for h in host]))
            rows = [pool[j * (nw + 1) + 1:(j + 1) * (nw + 1)] for j in range(n)]
        for theta in sorted({1, 2, max(1, n // 2), n}):
            out = empty_words(nw)
            tq.tq_threshold(ctx, rows, r, theta, out)
            assert tq.tq_ctx_check(ctx) == 0
            got = to_host(out)[:nw]
            assert np.array_equal(got, oracle.threshold(list(host), r, theta)), (n, r, theta)
            results.append(got)
        for f in (oracle.truth_parity(n), rng.integers(0, 2, n + 1).astype(np.uint8)):
            out = empty_words(nw)
            tq.tq_symmetric(ctx, rows, r, f, out)
            assert tq.tq_ctx_check(ctx) == 0
            got = to_host(out)[:nw]
            assert np.array_equal(got, oracle.symmetric(list(host), r, f)), (n, r)
            results.append(got)
    return results


def test_autotune_dense_matches_oracle(tctx):
    run_shapes(tctx, np.random.default_rng(1))
    rows = parse(tq.tq_tune_export(tctx))
    assert len(rows) >= len(SHAPES)
    for cls, params, us in rows:
        family, K, log_n, log_w, kind, pruned, theta8, a16 = cls
        assert family == 1 and us > 0
        wpl, split, groups, zero = params
        assert zero == 0 and wpl in (1, 2) and split in (1, 2, 4, 8) and groups in (1, 4)
        if not a16:
            assert wpl == 1
        if split > 1:
            assert wpl == 1 and groups == 1


def test_tune_export_import_roundtrip():
    rng = np.random.default_rng(2)
    a = tq.tq_create(0)
    b = tq.tq_create(0)
    try:
        tq.tq_set_option(a, tq.TQ_OPTION_AUTOTUNE, 1)
        tq.tq_set_option(b, tq.TQ_OPTION_AUTOTUNE, 1)
        first = run_shapes(a, rng)
        text = tq.tq_tune_export(a)
        tq.tq_tune_import(b, text)
        assert tq.tq_tune_export(b) == text
        second = run_shapes(b, np.random.default_rng(2))
        assert all(np.array_equal(x, y) for x, y in zip(first, second))
        assert tq.tq_tune_export(b) == text          # every class was already tuned
        tq.tq_tune_clear(b)
        assert tq.tq_tune_export(b) == ""
    finally:
        tq.tq_destroy(a)
        tq.tq_destroy(b)


@pytest.mark.parametrize("text", [
    "1 9 8 20 0 1 3 1 : 1 3 1 0 : 5.0\n",            # split 3 does not exist
    "1 9 8 20 0 1 3 0 : 2 1 1 0 : 5.0\n",            # two-word lanes need 16-byte alignment
    "1 9 8 20 0 1 3 1 : 2 2 1 0 : 5.0\n",            # two-word lanes are not split
    "1 7 8 20 0 1 3 1 : 1 1 1 0 : 5.0\n1 9 8 x\n",   # malformed second line
    "1 9 8 20 0 1 3 1 : 1 1 1 0\n",                  # missing time
    "2 9 8 20 0 0 3 0 : -1 1 0 0 : 5.0\n",           # negative tiles per workgroup
    "2 9 8 20 0 0 3 0 : 4 3 0 0 : 5.0\n",            # counters 3 do not exist
    "7 9 8 20 0 0 3 0 : 1 0 0 0 : 5.0\n",            # unknown family
])
def test_tune_import_rejects(tctx, text):
    assert tq.raw_tune_import(tctx, text) == tq.TQ_EINVAL
    assert tq.tq_tune_export(tctx) == ""


def test_tune_import_accepts_and_uses(tctx):
    """An imported shape is used as is (here a split of 8 waves for N = 16)."""
    rng = np.random.default_rng(4)
    n, r = 16, 1 << 18
    nw = r // 64
    host = rand_words(rng, n, nw, 0.3)
    pool = dev_pool(host)
    rows = [pool[j] for j in range(n)]
    K, log_n, log_w = 5, 4, 12
    text = "1 %d %d %d 0 1 4 1 : 1 8 1 0 : 1.0\n" % (K, log_n, log_w)
    tq.tq_tune_import(tctx, text)
    out = empty_words(nw)
    tq.tq_threshold(tctx, rows, r, 9, out)                 # theta 9 of 16: eighth 4
    assert tq.tq_ctx_check(tctx) == 0
    assert np.array_equal(to_host(out), oracle.threshold(list(host), r, 9))
    assert tq.tq_tune_export(tctx) == "1 5 4 12 0 1 4 1 : 1 8 1 0 : 1.000\n"


def test_autotune_rle(tctx):
    from test_rle_gpu import markov_bitmaps, rle_inputs
    r = 64 * 512 * 6 + 17
    for n, ones, zeros in ((40, 30.0, 600.0), (9, 200.0, 200.0)):
        dense = markov_bitmaps(60 + n, n, r, ones, zeros)
        inputs, keep = rle_inputs(tctx, dense, r)
        for theta in (1, 2, n // 2):
            out = empty_words((r + 63) // 64)
            tq.tq_threshold_rle_dense(tctx, inputs, r, theta, out)
            assert tq.tq_ctx_check(tctx) == 0
            assert np.array_equal(to_host(out), oracle.threshold(dense, r, theta))
        f = oracle.truth_parity(n)
        out = empty_words((r + 63) // 64)
        tq.tq_symmetric_rle_dense(tctx, inputs, r, f, out)
        assert tq.tq_ctx_check(tctx) == 0
        assert np.array_equal(to_host(out), oracle.symmetric(dense, r, f))
    rows = parse(tq.tq_tune_export(tctx))
    rle = [x for x in rows if x[0][0] == 2]
    assert len(rle) >= 4
    assert all(p[0] in (0, 1, 2, 4, 16) and p[1] in (1, 2) and p[2:] == [0, 0] for _, p, _ in rle)


def test_batch_tune_keeps_results(tctx):
    from test_batch_gpu import make_specs
    rng = np.random.default_rng(42)
    nw = 64 * 37 + 11
    dens = rng.uniform(0.01, 0.9, 300)
    base = np.concatenate([rand_words(rng, 1, nw, d) for d in dens])
    dpool = dev_pool(list(base))
    specs, want = make_specs(rng, base, dpool, nw, 60)
    q = tq.BatchQueries(specs)
    ipw, miw = tq.tq_batch_tune(tctx, q)
    assert ipw in (1, 2, 4, 8, 16) and miw in (4, 16, 64)
    for sp, w in zip(specs, want):
        sp["out"].fill_(0x5A5A)
    b = tq.tq_batch_submit(tctx, q)
    tq.tq_batch_wait(b)
    tq.tq_batch_release(b)
    assert tq.tq_ctx_check(tctx) == 0
    for sp, w in zip(specs, want):
        assert np.array_equal(to_host(sp["out"])[:len(w)], w)
    assert tq.tq_batch_set_schedule(tctx, 0, 16) == tq.TQ_EINVAL
    assert tq.tq_batch_set_schedule(tctx, 4, 5000) == tq.TQ_EINVAL
    assert tq.tq_batch_set_schedule(tctx, 2, 8) == tq.TQ_OK
    b = tq.tq_batch_submit(tctx, q)
    tq.tq_batch_release(b)
    assert tq.tq_ctx_check(tctx) == 0
    for sp, w in zip(specs, want):
        assert np.array_equal(to_host(sp["out"])[:len(w)], w)
