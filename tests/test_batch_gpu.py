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


def table_truth(n, salt=0):
    """A truth table with many runs of ones and of zeros and not a parity
    function, so that only the lookup-table epilogue can evaluate it."""
    c = np.arange(n + 1, dtype=np.uint64)
    f = (((c + np.uint64(salt)) * np.uint64(2654435761)) >> np.uint64(9)) & np.uint64(1)
    f = f.astype(np.uint8)
    f[:20] = [1, 0, 1, 0, 1, 1, 0, 1, 0, 1, 0, 0, 1, 0, 1, 0, 1, 0, 1, 0][:min(20, n + 1)]
    return f


def make_specs(rng, base, dpool, nw, count, with_symmetric=True):
    specs, want = [], []
    for i in range(count):
        n = int(rng.choice([1, 2, 3, 7, 15, 16, 17, 40, 130, 299]))
        r = int(rng.integers(1, nw * 64 + 1))
        members = rng.choice(base.shape[0], size=n, replace=False)
        out = empty_words((r + 63) // 64)
        host = [base[m] for m in members]
        sp = {"inputs": [dpool[int(m)] for m in members], "r_bits": r, "out": out, "tag": 1000 + i}
        kind = rng.integers(0, 5) if with_symmetric else 0
        if kind == 4 and n >= 19:
            f = table_truth(n, salt=i)
            sp["truth"] = f
            want.append(oracle.symmetric(host, r, f))
        elif kind == 1:
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
    for _ in range(tq.TQ_BATCH_MAX_INFLIGHT):
        specs, _ = make_specs(rng, base, dpool, nw, 5, with_symmetric=False)
        bq = tq.BatchQueries(specs)
        handles.append((tq.tq_batch_submit(ctx, bq), bq))
    specs, want = make_specs(rng, base, dpool, nw, 5, with_symmetric=False)
    bq = tq.BatchQueries(specs)
    st, h = tq.raw_batch_submit(ctx, bq)
    assert st == tq.TQ_EBUSY and not h             # the context holds as many batches as it may
    tq.tq_batch_release(handles[0][0])
    b = tq.tq_batch_submit(ctx, bq)                # room again
    tq.tq_batch_release(b)
    for h, _ in handles[1:]:
        tq.tq_batch_release(h)
    for sp, w in zip(specs, want):
        assert np.array_equal(to_host(sp["out"])[:(sp["r_bits"] + 63) // 64], w)
    # the lookup tables of one batch are bounded (nothing is launched here):
    # 129 functions of 8192 inputs need 129 tables of 2^16 bits
    n = 8192
    f = table_truth(n)
    out = empty_words(1)
    specs = [{"inputs": [dpool[j % 300] for j in range(n)], "r_bits": 64, "out": out, "truth": f}
             for _ in range(tq.TQ_BATCH_MAX_TABLE_BYTES // 8192 + 1)]
    st, h = tq.raw_batch_submit(ctx, tq.BatchQueries(specs))
    assert st == tq.TQ_EINVAL and not h
    sp = {"inputs": [], "r_bits": 640, "out": empty_words(10), "theta": 1}
    st, h = tq.raw_batch_submit(ctx, tq.BatchQueries([sp]))
    assert st == tq.TQ_EINVAL
    assert tq.tq_ctx_check(ctx) == 0


@pytest.mark.parametrize("count", [20, 70])     # direct launch and graph replay
def test_batch_truth_tables(ctx, pool, count):
    """Arbitrary symmetric functions in a batch (lookup-table epilogue), with
    tables small enough to be staged per wave (n < 2048) and larger ones read
    from the packed batch (n = 2500 and 9000, inputs repeated), mixed with
    thresholds; every output equals the oracle's, over repeated submissions."""
    base, dpool, nw = pool
    rng = np.random.default_rng(11 + count)
    for rep in range(2):
        specs, want = [], []
        for i in range(count):
            big = i % 9 == 4
            n = int(rng.choice([2500, 9000])) if big else int(rng.choice([19, 40, 130, 299]))
            r = int(rng.integers(1, (nw * 64 if not big else 64 * 300) + 1))
            members = rng.integers(0, base.shape[0], size=n) if big else rng.choice(base.shape[0], n, replace=False)
            host = [base[m] for m in members]
            sp = {"inputs": [dpool[int(m)] for m in members], "r_bits": r, "out": empty_words((r + 63) // 64),
                  "tag": i}
            if i % 3 == 2:
                theta = int(rng.integers(1, n + 1))
                sp["theta"] = theta
                want.append(oracle.threshold(host, r, theta))
            else:
                f = table_truth(n, salt=97 * rep + i)
                sp["truth"] = f
                want.append(oracle.symmetric(host, r, f))
            specs.append(sp)
        b = tq.tq_batch_submit(ctx, tq.BatchQueries(specs))
        tq.tq_batch_wait(b)
        recs = tq.tq_batch_records(b, len(specs))
        for i, (sp, w) in enumerate(zip(specs, want)):
            assert np.array_equal(to_host(sp["out"])[:(sp["r_bits"] + 63) // 64], w), (rep, i, len(sp["inputs"]))
            assert recs[i]["status"] == 0 and recs[i]["done"] == 1
        tq.tq_batch_release(b)
        # the same functions through the single-query call
        for sp in specs[:6]:
            if "truth" in sp:
                single = empty_words((sp["r_bits"] + 63) // 64)
                tq.tq_symmetric(ctx, sp["inputs"], sp["r_bits"], sp["truth"], single)
                assert torch.equal(single, sp["out"])
    assert tq.tq_ctx_check(ctx) == 0
