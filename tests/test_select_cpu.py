"""Host logic of the selector (no GPU): query features from metadata."""
import math

import numpy as np
import pytest

from paper_1402_4073_amd import binding as tq


def test_features_definition():
    r = 1 << 20
    nw = r // 64
    meta = [dict(dense=0x1000, rle=(0x2000, 300, None), ones=500, runs=41),
            dict(dense=0x3000, rle=None, ones=20000, runs=9001),
            dict(dense=0x4000, rle=(0x5000, 9000, None), ones=0, runs=1)]
    f = tq.tq_query_features(meta, r, 2)
    d = np.array([m["ones"] / r for m in meta])
    runlen = [max(1.0, m["ones"] / max(1.0, m["runs"] / 2)) if m["ones"] else 1.0 for m in meta]
    ld = np.log10(d + 1e-9)
    comp = 300 + nw + 9000
    want = [math.log2(3), 2 / 3, math.log10(d.mean() + 1e-9), math.log10(max(1.0, np.mean(runlen))),
            ld.std(), 20.0, math.log2(nw * 3 / comp), math.log2(2 / (1 + d.sum()))]
    assert np.allclose(f, want, rtol=1e-5, atol=1e-6)


def test_features_reject_bad_args():
    with pytest.raises(tq.TQError):
        tq.tq_query_features([], 1024, 1)
