"""Batched queries over registered inputs: every variant, compressed inputs
and results, admission by bytes, cancellation and deadlines.

Each batch mixes the carry-save counter (with the Looped forms at thresholds
within 3 of either end), the per-position counter, the run-length merge, the
hybrid and the selector's choice, with dense and compressed results; every
output is compared word for word with the oracle (a compressed result with
the oracle's canonical encoding of the oracle's dense result).  The failure
paths are forced from the host: a small admission limit, a cancel flag set
right after submission, a deadline of a microsecond, an output capacity that
is too small and a malformed stream; every query a stopped batch reports
complete is still checked against the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
from gpuhelp import dev_pool, empty_words, to_dev, to_host
from paper_1402_4073_amd import binding as tq
from paper_1402_4073_amd import selector

pytestmark = pytest.mark.gpu

NW = 64 * 37 + 11
R = NW * 64 - 37          # ragged tail
VARIANTS = (tq.TQ_VARIANT_CSA, tq.TQ_VARIANT_COUNTER, tq.TQ_VARIANT_RLE, tq.TQ_VARIANT_HYBRID, tq.TQ_VARIANT_AUTO)


@pytest.fixture(scope="module")
def ctx():
    c = tq.tq_create(0)
    selector.load_default(c)
    yield c
    tq.tq_destroy(c)


def run_bits(rng, nbits, density, mean_ones):
    """Alternating runs: ones of geometric length (mean mean_ones), zeros sized
    for the given density."""
    mean_zeros = max(1.0, mean_ones * (1 - density) / max(density, 1e-9))
    out = np.zeros(nbits, dtype=np.uint8)
    pos, one = 0, rng.random() < density
    while pos < nbits:
        m = mean_ones if one else mean_zeros
        L = int(rng.geometric(1.0 / max(m, 1.0)))
        if one:
            out[pos:pos + L] = 1
        pos += L
        one = not one
    return out


@pytest.fixture(scope="module")
def pool(ctx):
    """120 registered bitmaps of R bits: i.i.d. and run-structured ones, each
    with its dense form and its canonical stream; every other stream without
    a checkpoint index (built by the batch)."""
    rng = np.random.default_rng(2024)
    rows = []
    for j in range(120):
        if j % 3 == 0:
            bits = (rng.random(NW * 64) < 10 ** rng.uniform(-3, np.log10(0.5))).astype(np.uint8)
        else:
            bits = run_bits(rng, NW * 64, 10 ** rng.uniform(-3, np.log10(0.4)), 10 ** rng.uniform(0, 3))
        w = np.packbits(bits, bitorder="little").view("<u8").astype(np.uint64)
        w[-1] &= np.uint64((1 << (R % 64)) - 1)
        rows.append(w)
    host = np.stack(rows)
    dense = dev_pool(list(host))
    drows = [dense[j] for j in range(len(rows))]
    streams, offs, lens, index = tq.encode_pool(ctx, drows, R)
    bitmaps = []
    for j in range(len(rows)):
        ones = int(sum(bin(int(x)).count("1") for x in host[j]))
        bitmaps.append({"dense": drows[j], "rle": (streams[offs[j]:], lens[j], index[j] if j % 2 else None),
                        "ones": ones, "runs": oracle.run_count(host[j], R)})
    return host, dense, drows, bitmaps, (streams, index)


def theta_for(rng, n):
    return int(rng.choice([0, 1, 2, 3, max(1, n - 2), max(1, n - 1), n, n + 1, int(rng.integers(1, n + 1))]))


def build_batch(rng, pool, count, compressed_every=3, symmetric_every=7):
    host, dense, drows, bitmaps, _ = pool
    specs, want = [], []
    for i in range(count):
        n = int(rng.choice([1, 2, 3, 5, 9, 16, 17, 33, 64, 119]))
        members = rng.choice(len(bitmaps), size=n, replace=False)
        bms = [bitmaps[int(m)] for m in members]
        hrows = [host[int(m)] for m in members]
        sp = {"bitmaps": bms, "r_bits": R, "tag": 500 + i}
        if i % symmetric_every == symmetric_every - 1:
            f = oracle.truth_interval(n, 1, max(1, n // 2)) if i % 2 else oracle.truth_parity(n)
            sp["truth"] = f
            sp["variant"] = tq.TQ_VARIANT_AUTO if i % 3 else tq.TQ_VARIANT_CSA
            w = oracle.symmetric(hrows, R, f)
        else:
            theta = theta_for(rng, n)
            sp["theta"] = theta
            sp["variant"] = VARIANTS[i % len(VARIANTS)]
            w = oracle.threshold(hrows, R, theta)
        if i % compressed_every == compressed_every - 1:
            cap = NW + 1
            sp["out"] = empty_words(cap)
            sp["out_cap"] = cap
            sp["out_len"] = torch.full((1,), -1, dtype=torch.int64, device="cuda")
            want.append(("rle", oracle.rle_encode(w, R)))
        else:
            sp["out"] = empty_words(NW)
            want.append(("dense", w))
        specs.append(sp)
    return specs, want


def check_output(sp, w, where):
    kind, ref = w
    if kind == "dense":
        got = to_host(sp["out"])[:NW]
        assert np.array_equal(got, ref), where
    else:
        L = int(sp["out_len"].item())
        assert L == len(ref), where
        assert np.array_equal(to_host(sp["out"])[:L], ref), where


@pytest.mark.parametrize("count", [40, 150])     # direct launch and graph replay of the persistent kernel
def test_batch_variants_match_oracle(ctx, pool, count):
    rng = np.random.default_rng(31 + count)
    for rep in range(2):
        specs, want = build_batch(rng, pool, count)
        b = tq.tq_batch_submit(ctx, tq.BatchQueries(specs))
        tq.tq_batch_wait(b)
        recs = tq.tq_batch_records(b, count)
        for i, (sp, w) in enumerate(zip(specs, want)):
            check_output(sp, w, (rep, i, sp["variant"], len(sp["bitmaps"]), sp.get("theta")))
            r = recs[i]
            assert r["status"] == 0 and r["done"] == 1 and r["user_tag"] == 500 + i
            assert r["t_end_ns"] >= r["t_start_ns"] > 0
            if sp["variant"] != tq.TQ_VARIANT_AUTO:
                assert r["variant"] == sp["variant"]
            else:
                assert r["variant"] < 4
        tq.tq_batch_release(b)
    assert tq.tq_ctx_check(ctx) == 0


def test_batch_variants_equal_single_calls(ctx, pool):
    """Batched results equal tq_threshold_variant's for the same inputs."""
    host, dense, drows, bitmaps, _ = pool
    rng = np.random.default_rng(77)
    specs = []
    for i in range(24):
        n = int(rng.integers(2, 60))
        members = rng.choice(len(bitmaps), size=n, replace=False)
        specs.append({"bitmaps": [bitmaps[int(m)] for m in members], "r_bits": R, "out": empty_words(NW),
                      "theta": int(rng.integers(1, n + 1)), "variant": i % 4})
    b = tq.tq_batch_submit(ctx, tq.BatchQueries(specs))
    tq.tq_batch_release(b)
    for sp in specs:
        single = empty_words(NW)
        tq.tq_threshold_variant(ctx, sp["bitmaps"], R, sp["theta"], sp["variant"], single)
        assert torch.equal(single, sp["out"])
    assert tq.tq_ctx_check(ctx) == 0


def test_batch_dense_pointers_with_counter_variant(ctx, pool):
    """Queries given as plain pointer arrays may pick the per-position counter."""
    host, dense, drows, bitmaps, _ = pool
    rng = np.random.default_rng(5)
    specs, want = [], []
    for i in range(30):
        n = int(rng.choice([2, 7, 40, 119]))
        members = rng.choice(len(drows), size=n, replace=False)
        r = int(rng.integers(1, R + 1))
        theta = theta_for(rng, n)
        specs.append({"inputs": [drows[int(m)] for m in members], "r_bits": r, "out": empty_words((r + 63) // 64),
                      "theta": theta, "variant": tq.TQ_VARIANT_COUNTER if i % 2 else tq.TQ_VARIANT_CSA})
        want.append(oracle.threshold([host[int(m)] for m in members], r, theta))
    b = tq.tq_batch_submit(ctx, tq.BatchQueries(specs))
    tq.tq_batch_wait(b)
    for sp, w in zip(specs, want):
        assert np.array_equal(to_host(sp["out"])[:(sp["r_bits"] + 63) // 64], w)
    tq.tq_batch_release(b)
    # the counter variant needs thresholds and dense inputs; AUTO needs registered inputs
    bad = [{"inputs": [drows[0], drows[1]], "r_bits": R, "out": empty_words(NW), "truth": oracle.truth_parity(2),
            "variant": tq.TQ_VARIANT_COUNTER},
           {"inputs": [drows[0]], "r_bits": R, "out": empty_words(NW), "theta": 1, "variant": tq.TQ_VARIANT_AUTO},
           {"inputs": [drows[0]], "r_bits": R, "out": empty_words(NW), "theta": 1, "variant": tq.TQ_VARIANT_RLE},
           {"bitmaps": [dict(bitmaps[0], dense=None)], "r_bits": R, "out": empty_words(NW), "theta": 1,
            "variant": tq.TQ_VARIANT_CSA}]
    for sp in bad:
        st, h = tq.raw_batch_submit(ctx, tq.BatchQueries([sp]))
        assert st == tq.TQ_EINVAL and not h, sp.get("variant")
    # a symmetric function over compressed-only inputs is not batched
    sp = {"bitmaps": [dict(bitmaps[0], dense=None), dict(bitmaps[1], dense=None)], "r_bits": R,
          "out": empty_words(NW), "truth": oracle.truth_parity(2), "variant": tq.TQ_VARIANT_AUTO}
    st, h = tq.raw_batch_submit(ctx, tq.BatchQueries([sp]))
    assert st == tq.TQ_ENOTSUP and not h
    assert tq.tq_ctx_check(ctx) == 0


def test_batch_capacity_and_format_errors(ctx, pool):
    """A compressed result larger than its capacity and a malformed input
    stream are reported in their own records; the other queries are right."""
    host, dense, drows, bitmaps, (streams, index) = pool
    rng = np.random.default_rng(8)
    n = 20
    members = rng.choice(len(bitmaps), size=n, replace=False)
    bms = [bitmaps[int(m)] for m in members]
    hrows = [host[int(m)] for m in members]
    want = oracle.threshold(hrows, R, 1)
    enc = oracle.rle_encode(want, R)
    assert len(enc) > 4
    small = {"bitmaps": bms, "r_bits": R, "theta": 1, "variant": tq.TQ_VARIANT_CSA, "out": empty_words(4),
             "out_cap": 4, "out_len": torch.full((1,), -1, dtype=torch.int64, device="cuda")}
    # a stream whose first marker claims more words than the bitmap has
    broken = torch.tensor([(np.uint64(NW + 5) << np.uint64(1)).astype(np.int64), 0], dtype=torch.int64,
                          device="cuda")
    bad_bm = {"dense": None, "rle": (broken, 2, None), "ones": 10, "runs": 3}
    malformed = {"bitmaps": [bad_bm, dict(bms[0], dense=None)], "r_bits": R, "theta": 1,
                 "variant": tq.TQ_VARIANT_RLE, "out": empty_words(NW)}
    good = {"bitmaps": bms, "r_bits": R, "theta": 1, "variant": tq.TQ_VARIANT_RLE, "out": empty_words(NW)}
    specs = [small, malformed, good]
    b = tq.tq_batch_submit(ctx, tq.BatchQueries(specs))
    st = tq.raw_batch_wait(b)
    recs = tq.tq_batch_records(b, 3)
    assert st == tq.TQ_ECAPACITY                     # the first query that did not complete with TQ_OK
    assert recs[0]["status"] == tq.TQ_ECAPACITY and recs[0]["done"] == 1
    assert int(small["out_len"].item()) == len(enc)  # the required length is reported
    assert recs[1]["status"] == tq.TQ_EFORMAT and recs[1]["done"] == 1
    assert recs[2]["status"] == 0 and np.array_equal(to_host(good["out"])[:NW], want)
    tq.tq_batch_release(b)
    assert tq.tq_ctx_check(ctx) == 0                 # per-query errors stay in the records


def small_batch(pool, rng, count=5, n=100):
    host, dense, drows, bitmaps, _ = pool
    specs, want = [], []
    for _ in range(count):
        members = rng.choice(len(drows), size=n, replace=False)
        theta = int(rng.integers(4, n - 3))
        specs.append({"inputs": [drows[int(m)] for m in members], "r_bits": R, "out": empty_words(NW),
                      "theta": theta})
        want.append(oracle.threshold([host[int(m)] for m in members], R, theta))
    return specs, want


def test_batch_admission_counts_bytes(ctx, pool):
    rng = np.random.default_rng(9)
    specs, want = small_batch(pool, rng)
    bq = tq.BatchQueries(specs)
    try:
        # the smallest limit that admits this batch, found from the host
        lo, hi = 1, 1 << 20
        tq.tq_set_option(ctx, tq.TQ_OPTION_BATCH_BYTES, hi)
        st, h = tq.raw_batch_submit(ctx, bq)
        assert st == tq.TQ_OK
        tq.tq_batch_release(h)
        while lo < hi:
            mid = (lo + hi) // 2
            tq.tq_set_option(ctx, tq.TQ_OPTION_BATCH_BYTES, mid)
            st, h = tq.raw_batch_submit(ctx, bq)
            if st == tq.TQ_OK:
                tq.tq_batch_release(h)
                hi = mid
            else:
                assert st == tq.TQ_EINVAL and not h      # larger than the limit on its own
                lo = mid + 1
        need = lo
        assert need > 1000
        # room for one batch: a second is refused until the first is released
        tq.tq_set_option(ctx, tq.TQ_OPTION_BATCH_BYTES, 2 * need - 1)
        a = tq.tq_batch_submit(ctx, bq)
        st, h = tq.raw_batch_submit(ctx, bq)
        assert st == tq.TQ_EBUSY and not h
        tq.tq_batch_release(a)
        b = tq.tq_batch_submit(ctx, bq)
        # room for two
        tq.tq_set_option(ctx, tq.TQ_OPTION_BATCH_BYTES, 2 * need)
        c = tq.tq_batch_submit(ctx, bq)
        st, h = tq.raw_batch_submit(ctx, bq)
        assert st == tq.TQ_EBUSY and not h
        tq.tq_batch_release(b)
        tq.tq_batch_release(c)
        for sp, w in zip(specs, want):
            assert np.array_equal(to_host(sp["out"])[:NW], w)
        # the number of batches held at once is bounded too
        tq.tq_set_option(ctx, tq.TQ_OPTION_BATCH_BYTES, 1 << 34)
        held = [tq.tq_batch_submit(ctx, bq) for _ in range(tq.TQ_BATCH_MAX_INFLIGHT)]
        st, h = tq.raw_batch_submit(ctx, bq)
        assert st == tq.TQ_EBUSY and not h
        for x in held:
            tq.tq_batch_release(x)
        # options reject bad values
        assert tq._lib.tq_set_option(ctx, tq.TQ_OPTION_BATCH_BYTES, 0) == tq.TQ_EINVAL
    finally:
        tq.tq_set_option(ctx, tq.TQ_OPTION_BATCH_BYTES, 1 << 30)
    assert tq.tq_ctx_check(ctx) == 0


def big_batch(pool, rng, count):
    """Enough work items that the first round of every workgroup cannot
    finish them all."""
    host, dense, drows, bitmaps, _ = pool
    specs, want = [], []
    for i in range(count):
        n = 119
        members = rng.choice(len(drows), size=n, replace=False)
        theta = int(rng.integers(4, n - 3))
        specs.append({"inputs": [drows[int(m)] for m in members], "r_bits": R, "out": empty_words(NW),
                      "theta": theta, "tag": i})
        want.append((members, theta))
    return specs, want


def check_stopped(ctx, pool, specs, want, b, expect):
    host = pool[0]
    st = tq.raw_batch_wait(b)
    recs = tq.tq_batch_records(b, len(specs))
    stopped = 0
    for i, (sp, (members, theta)) in enumerate(zip(specs, want)):
        r = recs[i]
        if r["done"]:
            assert r["status"] == 0
            ref = oracle.threshold([host[int(m)] for m in members], R, theta)
            assert np.array_equal(to_host(sp["out"])[:NW], ref), i
        else:
            assert r["status"] == expect, (i, r["status"])
            stopped += 1
    assert (st == expect) == (stopped > 0) and (st == tq.TQ_OK) == (stopped == 0)
    tq.tq_batch_release(b)
    return stopped


def test_batch_cancel(ctx, pool):
    rng = np.random.default_rng(12)
    specs, want = big_batch(pool, rng, 2000)
    bq = tq.BatchQueries(specs)
    b = tq.tq_batch_submit(ctx, bq)
    tq.tq_batch_cancel(b)
    stopped = check_stopped(ctx, pool, specs, want, b, tq.TQ_ECANCELED)
    print("cancelled before completion:", stopped, "of", len(specs))
    # the slot serves a full batch correctly afterwards (its counters were reset)
    for _ in range(2):
        b = tq.tq_batch_submit(ctx, bq)
        assert check_stopped(ctx, pool, specs, want, b, tq.TQ_ECANCELED) == 0
    assert tq.tq_ctx_check(ctx) == 0


def test_batch_deadline(ctx, pool):
    rng = np.random.default_rng(13)
    specs, want = big_batch(pool, rng, 2000)
    bq = tq.BatchQueries(specs)
    try:
        tq.tq_set_option(ctx, tq.TQ_OPTION_BATCH_DEADLINE_US, 1)
        b = tq.tq_batch_submit(ctx, bq)
        stopped = check_stopped(ctx, pool, specs, want, b, tq.TQ_ETIMEDOUT)
        assert stopped > 0
        # compressed results of stopped queries are reported stopped too
        sp2, w2 = build_batch(rng, pool, 200, compressed_every=2, symmetric_every=1000)
        for sp in sp2:
            sp["variant"] = tq.TQ_VARIANT_CSA
        b = tq.tq_batch_submit(ctx, tq.BatchQueries(sp2))
        st = tq.raw_batch_wait(b)
        recs = tq.tq_batch_records(b, len(sp2))
        for i, (sp, w) in enumerate(zip(sp2, w2)):
            if recs[i]["done"]:
                assert recs[i]["status"] == 0
                check_output(sp, w, i)
            else:
                assert recs[i]["status"] == tq.TQ_ETIMEDOUT
        assert st in (tq.TQ_OK, tq.TQ_ETIMEDOUT)
        tq.tq_batch_release(b)
    finally:
        tq.tq_set_option(ctx, tq.TQ_OPTION_BATCH_DEADLINE_US, 0)
    b = tq.tq_batch_submit(ctx, bq)
    assert check_stopped(ctx, pool, specs, want, b, tq.TQ_ETIMEDOUT) == 0
    assert tq._lib.tq_set_option(ctx, tq.TQ_OPTION_BATCH_DEADLINE_US, -1) == tq.TQ_EINVAL
    assert tq.tq_ctx_check(ctx) == 0
