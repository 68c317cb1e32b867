"""The carry-save kernel's pruned path at one wave per column group, against
the oracle, element by element.

Threshold pruning (skipping once every position of a lane is decided, the
lower-bound argument of section 1) runs only where one wave owns all inputs
of a column group.  The default launch rule splits the inputs of short
bitmaps over several waves, so these tests either import a one-wave shape
through the tuning cache or use bitmaps long enough (2048 column groups or
more) that the default rule keeps one wave.  Inputs are read in the caller's
order and in order of registered cardinality (true, reversed and equal
registered values), with pruning and the saturating-counter (Looped) kernel
on and off.
"""
import numpy as np
import pytest
import torch

import oracle
import tqgen
from gpuhelp import dev_pool, empty_words, force_dense_shape, to_host
from paper_1402_4073_amd import binding as tq

pytestmark = pytest.mark.gpu


def column_varied_words(rng, count, nw):
    """Bitmaps whose density changes from one 64-word column group to the
    next, so that lanes and waves are decided after different inputs."""
    out = []
    for _ in range(count):
        col_dens = np.repeat(rng.uniform(0.0, 1.0, (nw + 63) // 64), 64)[:nw]
        bits = rng.random((nw, 64)) < col_dens[:, None] * rng.uniform(0.2, 1.0)
        out.append(np.packbits(bits.astype(np.uint8), axis=1, bitorder="little").view("<u8")
                   .reshape(-1).astype(np.uint64))
    return out


def popcounts(host, r):
    return [int(np.unpackbits(h.view(np.uint8), bitorder="little")[:r].sum()) for h in host]


def run(ctx, fn, nw):
    out = empty_words(nw)
    fn(out)
    assert tq.tq_ctx_check(ctx) == 0
    return to_host(out)[:nw]


@pytest.mark.parametrize("n", [40, 256, 1000])
def test_pruned_carry_save_one_wave(n):
    """Forced one-wave shape: the pruned loop with its checks every 16
    inputs (2 to 62 checks here), several column groups and a ragged tail."""
    rng = np.random.default_rng(900 + n)
    r = 64 * 64 * 9 + 31
    nw = (r + 63) // 64
    base = column_varied_words(rng, min(n, 120), nw)
    pool = dev_pool(base)
    pick = rng.integers(0, len(base), n)
    rows = [pool[int(i)] for i in pick]
    host = [base[int(i)] for i in pick]
    ones = popcounts(host, r)
    mean = sum(ones) / r
    thetas = sorted({1, 2, 3, 4, max(1, int(mean / 2)), max(1, int(mean)), int(mean) + 5,
                     n // 3, n // 2, (3 * n) // 4, n - 3, n - 2, n - 1, n})
    ctx = tq.tq_create(0)
    try:
        text = force_dense_shape(tq, ctx, n, nw)
        registered = {
            "true": ones,
            "reversed": ones[::-1],
            "equal": [5] * n,
        }
        for theta in thetas:
            want = oracle.threshold(host, r, theta)
            for looped in (0, 1):
                tq.tq_set_option(ctx, tq.TQ_OPTION_LOOPED, looped)
                for prune in (1, 0):
                    tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, prune)
                    got = run(ctx, lambda o: tq.tq_threshold(ctx, rows, r, theta, o), nw)
                    assert np.array_equal(got, want), ("caller order", theta, looped, prune)
                    for label, reg in registered.items():
                        bms = [dict(dense=rows[j], rle=None, ones=int(reg[j]), runs=1) for j in range(n)]
                        arr = (tq.bitmap_array(bms), n)
                        got = run(ctx, lambda o: tq.tq_threshold_variant(ctx, arr, r, theta, tq.TQ_VARIANT_CSA, o),
                                  nw)
                        assert np.array_equal(got, want), (label, theta, looped, prune)
        # the imported one-wave shape is what ran: nothing was timed or replaced
        assert sorted(tq.tq_tune_export(ctx).splitlines()) == sorted(text.splitlines())
    finally:
        tq.tq_destroy(ctx)


def test_pruned_carry_save_default_shape_long_bitmaps():
    """Bitmaps of 2^17 + 37 words (2049 column groups, ragged tail): the
    default launch rule keeps one wave per column group, so pruning runs on
    the shape the library picks by itself.  Inputs from the seeded
    generator (filled on the GPU, copied back for the oracle)."""
    n = 96
    r = 64 * ((1 << 17) + 36) + 5
    bs = tqgen.bernoulli_loguniform(41, n, r, 1e-3, 0.5)
    pool = torch.empty((n, bs.nwords), dtype=torch.int64, device="cuda")
    tqgen.fill_gpu(bs, pool.view(-1))
    rows = [pool[j] for j in range(n)]
    host_all = pool.cpu().numpy().view(np.uint64)
    host = [host_all[j] for j in range(n)]
    ones = popcounts(host, r)
    mean = sum(ones) / r
    nw = bs.nwords
    ctx = tq.tq_create(0)
    try:
        for theta in sorted({2, 3, max(1, int(mean)), int(mean) + 4, n // 2, n - 3, n - 1}):
            want = oracle.threshold(host, r, theta)
            for prune, looped in ((1, 1), (1, 0), (0, 0)):
                tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, prune)
                tq.tq_set_option(ctx, tq.TQ_OPTION_LOOPED, looped)
                for label, reg in (("true", ones), ("reversed", ones[::-1])):
                    bms = [dict(dense=rows[j], rle=None, ones=int(reg[j]), runs=1) for j in range(n)]
                    arr = (tq.bitmap_array(bms), n)
                    got = run(ctx, lambda o: tq.tq_threshold_variant(ctx, arr, r, theta, tq.TQ_VARIANT_CSA, o), nw)
                    assert np.array_equal(got, want), (label, theta, prune, looped)
    finally:
        tq.tq_destroy(ctx)
