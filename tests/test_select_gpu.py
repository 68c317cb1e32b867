"""Variants, metadata kernels and the selector network on the GPU."""
import numpy as np
import pytest
import torch

import oracle
import tqgen
from gpuhelp import dev_pool, empty_words, to_dev, to_host
from oracle import mlp_ref
from paper_1402_4073_amd import binding as tq
from paper_1402_4073_amd import selector

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = tq.tq_create(0)
    yield c
    tq.tq_destroy(c)


def registered(ctx, dense_list, r, with_dense=True, with_rle=True):
    """Register bitmaps: device dense words, GPU-encoded stream + index, stats."""
    pool = dev_pool(dense_list)
    rows = [pool[j] for j in range(len(dense_list))]
    enc, offs, lens, idx = tq.encode_pool(ctx, rows, r)
    stats = torch.zeros((len(rows), 2), dtype=torch.int64, device="cuda")
    for j, row in enumerate(rows):
        tq.tq_bitmap_stats(ctx, row, r, stats[j, 0:1], stats[j, 1:2])
    st = stats.cpu().numpy()
    bms = []
    for j in range(len(rows)):
        bms.append(dict(dense=rows[j] if with_dense else None,
                        rle=(enc[offs[j]:], lens[j], idx[j]) if with_rle else None,
                        ones=int(st[j, 0]), runs=int(st[j, 1])))
    return bms, (pool, enc, idx)


def test_bitmap_stats(ctx):
    """Cardinality and run count equal the oracle's: tiny and ragged bitmaps,
    several 2048-word chunks with a partial last one, and more chunks than
    workgroups (the grid strides)."""
    big = 64 * (2048 * 1024 + 2048 * 2 + 9) + 33
    for r in (big,):
        bs = tqgen.bernoulli_loguniform(r % 1000, 2, r, 1e-3, 0.5)
        dense = [bs.words(j) for j in range(2)]
        bms, keep = registered(ctx, dense, r, with_rle=False)
        for j, b in enumerate(bms):
            bits = np.unpackbits(dense[j].view(np.uint8), bitorder="little")[:r]
            assert b["ones"] == int(bits.sum())
            assert b["runs"] == oracle.run_count(dense[j], r)
    for r in (1, 63, 64 * 100 + 7, 1 << 16, 64 * 2048 * 3 + 64 * 5 + 17):
        ms = tqgen.markov_fixed(r, 3, r, 5.0, 40.0)
        dense = [ms.words(j) for j in range(3)]
        bms, keep = registered(ctx, dense, r)
        for j, b in enumerate(bms):
            bits = np.unpackbits(dense[j].view(np.uint8), bitorder="little")[:r]
            assert b["ones"] == int(bits.sum())
            assert b["runs"] == oracle.run_count(dense[j], r)


@pytest.mark.parametrize("n,ones,zeros", [(3, 20.0, 300.0), (40, 2.0, 3.0), (300, 64.0, 4096.0)])
def test_variants_match_oracle(ctx, n, ones, zeros):
    r = 64 * 1500 + 21
    ms = tqgen.markov_fixed(n, n, r, ones, zeros)
    dense = [ms.words(j) for j in range(n)]
    bms, keep = registered(ctx, dense, r)
    arr = (tq.bitmap_array(bms), n)
    for theta in sorted({0, 1, 2, max(1, n // 4), n, n + 1}):
        want = oracle.threshold(dense, r, theta)
        for v in range(4):
            out = empty_words((r + 63) // 64)
            tq.tq_threshold_variant(ctx, arr, r, theta, v, out)
            assert tq.tq_ctx_check(ctx) == 0
            assert np.array_equal(to_host(out), want), (theta, tq.VARIANT_NAMES[v])


def test_csa_reads_inputs_by_cardinality(ctx):
    """The CSA variant reads its inputs in order of registered cardinality
    (densest first below half the expected count, sparsest first above),
    with pruning on and off; the result is the oracle's whether the
    registered cardinalities are true, reversed or all equal."""
    n, r = 48, 64 * 2000 + 5
    bs = tqgen.bernoulli_loguniform(31, n, r, 1e-3, 0.5)
    dense = [bs.words(j) for j in range(n)]
    bms, keep = registered(ctx, dense, r, with_rle=False)
    true_ones = [b["ones"] for b in bms]
    mean = sum(true_ones) / r
    thetas = sorted({1, 2, 3, max(1, int(mean / 4)), int(mean), 2 * int(mean) + 1, n - 2, n - 1, n})
    for label, ones in (("true", true_ones), ("reversed", true_ones[::-1]), ("equal", [7] * n)):
        arr = (tq.bitmap_array([dict(b, ones=o) for b, o in zip(bms, ones)]), n)
        for prune in (1, 0):
            tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, prune)
            for theta in thetas:
                out = empty_words((r + 63) // 64)
                tq.tq_threshold_variant(ctx, arr, r, theta, tq.TQ_VARIANT_CSA, out)
                assert tq.tq_ctx_check(ctx) == 0
                assert np.array_equal(to_host(out), oracle.threshold(dense, r, theta)), (label, prune, theta)
    tq.tq_set_option(ctx, tq.TQ_OPTION_PRUNE, 1)


def test_variant_needs_its_form(ctx):
    r = 64 * 100
    dense = [tqgen.markov_fixed(1, 1, r, 5.0, 50.0).words(0)]
    bms, keep = registered(ctx, dense, r, with_rle=False)
    out = empty_words(100)
    with pytest.raises(tq.TQError):
        tq.tq_threshold_variant(ctx, bms, r, 1, tq.TQ_VARIANT_RLE, out)
    tq.tq_threshold_variant(ctx, bms, r, 1, tq.TQ_VARIANT_HYBRID, out)   # dense form suffices
    assert np.array_equal(to_host(out), oracle.threshold(dense, r, 1))


def test_auto_refuses_input_without_a_form(ctx):
    """An input with neither a dense nor a compressed form leaves no variant
    to run: TQ_EINVAL with and without the timing fallback, and nothing is
    written."""
    r = 64 * 100
    dense = [tqgen.markov_fixed(2, 1, r, 5.0, 50.0).words(0)] * 2
    bms, keep = registered(ctx, dense, r)
    bms[1] = dict(dense=None, rle=None, ones=bms[1]["ones"], runs=bms[1]["runs"])
    p = mlp_ref.init_params(3).astype(np.float32)
    tq.tq_selector_set(ctx, p, np.zeros(8), np.ones(8), np.full(8, -1e9), np.full(8, 1e9), 1e9)
    out = empty_words(100)
    for flags in (0, tq.TQ_AUTO_FALLBACK, tq.TQ_AUTO_FALLBACK | tq.TQ_AUTO_RETIME):
        with pytest.raises(tq.TQError) as ei:
            tq.tq_threshold_auto(ctx, bms, r, 1, out, flags)
        assert ei.value.status == tq.TQ_EINVAL, flags
    assert tq.tq_ctx_check(ctx) == 0
    assert np.all(to_host(out) == np.uint64(0x5A5A5A5A5A5A5A5A))


def test_mlp_gradient_matches_fp64_reference(ctx):
    rng = np.random.default_rng(4)
    B = 77
    p = (mlp_ref.init_params(5) + rng.standard_normal(mlp_ref.N_PARAMS) * 0.05).astype(np.float32)
    x = rng.standard_normal((B, 8)).astype(np.float32)
    t = rng.standard_normal((B, 4)).astype(np.float32)
    m = (rng.random((B, 4)) < 0.7).astype(np.float32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = torch.zeros(mlp_ref.N_PARAMS, dtype=torch.float32, device="cuda")
    y = torch.zeros((B, 4), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    tq.tq_mlp_grad(ctx, d(p), d(x), d(t), d(m), B, float(m.sum()), y, g, loss)
    gref = mlp_ref.grad(p.astype(np.float64), x, t, m)
    yref, _ = mlp_ref.forward(p.astype(np.float64), x)
    lref = mlp_ref.loss(p.astype(np.float64), x, t, m)
    gg = g.cpu().numpy()
    assert np.allclose(y.cpu().numpy(), yref, rtol=1e-4, atol=1e-4)
    assert abs(float(loss.item()) - lref) <= 1e-4 * abs(lref) + 1e-6
    scale = np.abs(gref).max()
    assert np.max(np.abs(gg - gref)) <= 2e-4 * scale, np.max(np.abs(gg - gref)) / scale
    # deterministic: a second evaluation gives the same bits
    g2 = torch.zeros_like(g)
    tq.tq_mlp_grad(ctx, d(p), d(x), d(t), d(m), B, float(m.sum()), None, g2, None)
    assert torch.equal(g, g2)


def test_mlp_forward_and_host_inference(ctx):
    rng = np.random.default_rng(6)
    p = mlp_ref.init_params(7).astype(np.float32)
    feats = rng.standard_normal((50, 8)).astype(np.float32)
    mean = rng.standard_normal(8).astype(np.float32)
    std = (rng.random(8) + 0.5).astype(np.float32)
    gpu = selector.predict(ctx, p, (feats - mean) / std)
    ref, _ = mlp_ref.forward(p.astype(np.float64), (feats.astype(np.float64) - mean) / std)
    assert np.allclose(gpu, ref, rtol=1e-4, atol=1e-4)
    tq.tq_selector_set(ctx, p, mean, std, np.full(8, -1e9), np.full(8, 1e9), 0.0)
    for i in range(10):
        host = tq.tq_selector_predict(ctx, feats[i])
        assert np.allclose(host, ref[i], rtol=1e-4, atol=1e-4)


def test_training_reduces_loss(ctx):
    rng = np.random.default_rng(8)
    X = rng.standard_normal((600, 8)).astype(np.float32)
    W = rng.standard_normal((8, 4))
    T = (np.tanh(X @ W) + 0.1 * X[:, :4] ** 2).astype(np.float32)
    params, hist = selector.train(ctx, X, T, epochs=800, lr=3e-3)
    assert hist[-1][1] < 0.1 * hist[0][1], hist
    pred = selector.predict(ctx, params, X)
    ref, _ = mlp_ref.forward(params.astype(np.float64), X)
    assert np.allclose(pred, ref, rtol=1e-4, atol=1e-4)


def test_auto_dispatch(ctx):
    r = 64 * 900 + 3
    n = 24
    ms = tqgen.markov_fixed(9, n, r, 30.0, 600.0)
    dense = [ms.words(j) for j in range(n)]
    bms, keep = registered(ctx, dense, r)
    arr = (tq.bitmap_array(bms), n)
    p = mlp_ref.init_params(9).astype(np.float32)
    f = tq.tq_query_features(arr, r, 3)
    tq.tq_selector_set(ctx, p, np.zeros(8), np.ones(8), f - 100, f + 100, 0.0)
    pred = tq.tq_selector_predict(ctx, f)
    out = empty_words((r + 63) // 64)
    chosen = tq.tq_threshold_auto(ctx, arr, r, 3, out)
    assert chosen == int(np.argmin(pred))
    assert np.array_equal(to_host(out), oracle.threshold(dense, r, 3))
    # a huge margin makes every prediction uncertain: the fallback times all variants
    tq.tq_selector_set(ctx, p, np.zeros(8), np.ones(8), f - 100, f + 100, 1e9)
    out2 = empty_words((r + 63) // 64)
    chosen = tq.tq_threshold_auto(ctx, arr, r, 3, out2, tq.TQ_AUTO_FALLBACK)
    assert chosen & tq.TQ_AUTO_CHOSE_BY_TIMING and (chosen & 0xFF) < 4
    assert np.array_equal(to_host(out2), oracle.threshold(dense, r, 3))
    # the decision is remembered for the query's cell: no timing the second time
    timed = chosen & 0xFF
    for flags, bit in ((tq.TQ_AUTO_FALLBACK, tq.TQ_AUTO_CHOSE_BY_CACHE),
                       (tq.TQ_AUTO_FALLBACK | tq.TQ_AUTO_RETIME, tq.TQ_AUTO_CHOSE_BY_TIMING)):
        out3 = empty_words((r + 63) // 64)
        chosen = tq.tq_threshold_auto(ctx, arr, r, 3, out3, flags)
        assert chosen & bit and (chosen & 0xFF) < 4, (flags, chosen)
        if bit == tq.TQ_AUTO_CHOSE_BY_CACHE:
            assert chosen & 0xFF == timed
        assert np.array_equal(to_host(out3), oracle.threshold(dense, r, 3))
    # a neighbouring query (another threshold) falls in another cell
    chosen = tq.tq_threshold_auto(ctx, arr, r, 12, out3, tq.TQ_AUTO_FALLBACK)
    assert chosen & tq.TQ_AUTO_CHOSE_BY_TIMING
    assert np.array_equal(to_host(out3), oracle.threshold(dense, r, 12))
    # new weights forget the remembered decisions
    tq.tq_selector_set(ctx, p, np.zeros(8), np.ones(8), f - 100, f + 100, 1e9)
    chosen = tq.tq_threshold_auto(ctx, arr, r, 3, out3, tq.TQ_AUTO_FALLBACK)
    assert chosen & tq.TQ_AUTO_CHOSE_BY_TIMING


def test_default_weights_dispatch(ctx):
    """The shipped weights load and drive tq_threshold_auto to a correct result."""
    w = selector.load_default(ctx)
    assert len(w["params"]) == tq.TQ_SEL_PARAMS
    r = 1 << 20
    for n, d, m, theta in ((8, 0.2, 2.0, 3), (100, 1e-3, 500.0, 2)):
        ms = tqgen.markov_density_runlength(n, n, r, d, m)
        dense = [ms.words(j) for j in range(n)]
        bms, keep = registered(ctx, dense, r)
        out = empty_words(r // 64)
        chosen = tq.tq_threshold_auto(ctx, bms, r, theta, out)
        assert chosen < 4
        assert np.array_equal(to_host(out), oracle.threshold(dense, r, theta))
