"""Batched queries (persistent kernel, graph replay) against the oracle."""
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


def rand_words(rng, n, nw, p):
    bits = rng.random((n, nw * 64)) < p
    return np.packbits(bits.astype(np.uint8), axis=1, bitorder="little").view("<u8").astype(np.uint64)


@pytest.fixture(scope="module")
def pool():
    rng = np.random.default_rng(42)
    nw = 64 * 37 + 11
    dens = rng.uniform(0.01, 0.9, 300)
    base = np.concatenate([rand_words(rng, 1, nw, d) for d in dens])
    return base, dev_pool(list(base)), nw


def make_specs(rng, base, dpool, nw, count, with_symmetric=True):
    specs, want = [], []
    for i in range(count):
        n = int(rng.choice([1, 2, 3, 7, 15, 16, 17, 40, 130, 299]))
        r = int(rng.integers(1, nw * 64 + 1))
        members = rng.choice(base.shape[0], size=n, replace=False)
        out = empty_words((r + 63) // 64)
        host = [base[m] for m in members]
        sp = {"inputs": [dpool[int(m)] for m in members], "r_bits": r, "out": out, "tag": 1000 + i}
        kind = rng.integers(0, 4) if with_symmetric else 0
        if kind == 1:
            f = oracle.truth_parity(n)
            sp["truth"] = f
            want.append(oracle.symmetric(host, r, f))
        elif kind == 2:
            f = oracle.truth_interval(n, 2, max(2, n // 2))
            sp["truth"] = f
            want.append(oracle.symmetric(host, r, f))
        else:
            theta = int(rng.integers(0, n + 2))
            sp["theta"] = theta
            want.append(oracle.threshold(host, r, theta))
        specs.append(sp)
    return specs, want


@pytest.mark.parametrize("count", [60, 130])    # below and above the graph threshold (64 queries)
@pytest.mark.parametrize("flags", [0, tq.TQ_BATCH_NO_GRAPH])
def test_batch_matches_oracle(ctx, pool, flags, count):
    """Every query of random batches equals the oracle, over repeated
    submissions on the same slot (graph replays for the larger batches): the
    completion counters each batch leaves behind must be zero again."""
    base, dpool, nw = pool
    rng = np.random.default_rng(7 + flags + count)
    for rep in range(3):                      # repeated replays of the same slot graph
        specs, want = make_specs(rng, base, dpool, nw, count)
        bq = tq.BatchQueries(specs)
        b = tq.tq_batch_submit(ctx, bq, flags)
        torch.cuda.synchronize()             # eager work between replays
        tq.tq_batch_wait(b)
        assert tq.tq_batch_poll(b) == len(specs)
        recs = tq.tq_batch_records(b, len(specs))
        for i, (sp, w) in enumerate(zip(specs, want)):
            got = to_host(sp["out"])[:(sp["r_bits"] + 63) // 64]
            assert np.array_equal(got, w), (rep, i)
            rec = recs[i]
            assert rec["user_tag"] == 1000 + i and rec["status"] == 0 and rec["done"] == 1
            assert rec["t_end_ns"] >= rec["t_start_ns"]
        tq.tq_batch_release(b)
        assert tq.tq_ctx_check(ctx) == 0


def test_batch_equals_single_queries(ctx, pool):
    base, dpool, nw = pool
    rng = np.random.default_rng(99)
    specs, _ = make_specs(rng, base, dpool, nw, 40, with_symmetric=False)
    b = tq.tq_batch_submit(ctx, tq.BatchQueries(specs))
    tq.tq_batch_release(b)
    for sp in specs:
        single = empty_words((sp["r_bits"] + 63) // 64)
        tq.tq_threshold(ctx, sp["inputs"], sp["r_bits"], sp["theta"], single)
        assert torch.equal(single, sp["out"])


def test_batch_admission_and_errors(ctx, pool):
    base, dpool, nw = pool
    rng = np.random.default_rng(5)
    handles = []
    for _ in range(4):
        specs, _ = make_specs(rng, base, dpool, nw, 5, with_symmetric=False)
        bq = tq.BatchQueries(specs)
        handles.append((tq.tq_batch_submit(ctx, bq), bq))
    specs, want = make_specs(rng, base, dpool, nw, 5, with_symmetric=False)
    bq = tq.BatchQueries(specs)
    st, h = tq.raw_batch_submit(ctx, bq)
    assert st == tq.TQ_EBUSY and not h             # every slot is in flight
    tq.tq_batch_release(handles[0][0])
    b = tq.tq_batch_submit(ctx, bq)                # a slot is free again
    tq.tq_batch_release(b)
    for h, _ in handles[1:]:
        tq.tq_batch_release(h)
    for sp, w in zip(specs, want):
        assert np.array_equal(to_host(sp["out"])[:(sp["r_bits"] + 63) // 64], w)
    # a truth table that needs a lookup table is not served by the batch kernel
    n = 40
    f = np.zeros(n + 1, dtype=np.uint8)
    f[::2] = 1
    f[1] = 1
    sp = {"inputs": [dpool[j] for j in range(n)], "r_bits": 640, "out": empty_words(10), "truth": f}
    st, h = tq.raw_batch_submit(ctx, tq.BatchQueries([sp]))
    assert st == tq.TQ_ENOTSUP
    sp = {"inputs": [], "r_bits": 640, "out": empty_words(10), "theta": 1}
    st, h = tq.raw_batch_submit(ctx, tq.BatchQueries([sp]))
    assert st == tq.TQ_EINVAL
    assert tq.tq_ctx_check(ctx) == 0
