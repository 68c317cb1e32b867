"""The GPU input generator reproduces the numpy definition bit for bit."""
import numpy as np
import pytest
import torch

import tqgen
from gpuhelp import to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("r_bits", [64 * 33 + 7, 1 << 16])
def test_bernoulli_gpu_equals_cpu(r_bits):
    bs = tqgen.large_set(12, n=5, r_bits=r_bits)
    pool = torch.zeros(bs.n * bs.nwords, dtype=torch.int64, device="cuda")
    tqgen.fill_gpu(bs, pool)
    got = to_host(pool).reshape(bs.n, bs.nwords)
    for j in range(bs.n):
        assert np.array_equal(got[j], bs.words(j)), j


@pytest.mark.parametrize("r_bits", [64 * 70 + 3, 1 << 18])
def test_markov_gpu_equals_cpu(r_bits):
    for ms in (tqgen.rle_set(13, n=4, r_bits=r_bits),
               tqgen.markov_density_runlength(14, 3, r_bits, density=0.3, mean_ones=1.0),
               tqgen.markov_density_runlength(15, 3, r_bits, density=1e-4, mean_ones=500.0)):
        stride = ms.nwords + 3
        pool = torch.zeros(ms.n * stride, dtype=torch.int64, device="cuda")
        tqgen.fill_gpu(ms, pool, stride_words=stride)
        got = to_host(pool).reshape(ms.n, stride)[:, :ms.nwords]
        for j in range(ms.n):
            assert np.array_equal(got[j], ms.words(j)), j
