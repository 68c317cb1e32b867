"""Seeded synthetic bitmaps for threshold queries.

This module produces inputs only.  It holds none of the query arithmetic
(no counting, no comparison against a threshold, no run-length coding), so
both the CPU oracle and the GPU library can be fed from it without sharing
any of the method.

Every bit is a pure function of (seed, bitmap id, bit position), drawn from a
counter-based generator: the SplitMix64 output function of Steele, Lea and
Flood ("Fast splittable pseudorandom number generators", OOPSLA 2014) applied
to ``key + (ctr + 1) * GAMMA`` where ``key`` is a per-bitmap stream key.  The
same definition is implemented in ``tqgen/gen.hip`` for filling device
memory; tests check the two bit for bit.

Bit layout (the paper's uncompressed bitmap, section 2.1): position p lives
in bit (p mod 64) of 64-bit word p div 64, little-endian.  Bits of the last
word at positions >= r are left as generated (not zeroed) so that consumers
are exercised on garbage tails.

Two bit processes are provided:

* Bernoulli: bit q is 1 iff u32(q) < thr, thr = round(p * 2**32).
* Two-state Markov chain with P(0->1) = p01, P(1->0) = p10.  Each position q
  draws one u32 u; with A = round(p01 * 2**32) and S = round((1-p10) * 2**32)
  the next state is (u < S) from state 1 and (u < A) from state 0.  Drawing
  one uniform per position for both possible predecessor states is a
  coupling, so the marginal chain is exactly the Markov chain, and it makes
  every position classifiable on its own as "reset to 1", "reset to 0",
  "keep" or "flip".  A bit is then the value of the last reset at or before
  it, flipped once per flip since, which lets any word range be generated
  without running the chain from position 0.  The state before position 0 is
  drawn from the stationary law P(1) = p01 / (p01 + p10).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1
# counter reserved for per-bitmap scalar draws (initial Markov state, densities)
CTR_INIT = 1 << 62
CTR_PARAM = (1 << 62) + 1
CTR_PARAM2 = (1 << 62) + 2

_U64 = np.uint64
# smallest per-position reset probability accepted for Markov bitmaps
MIN_RESET = 2.0 ** -13


def _mix64_int(z: int) -> int:
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=_U64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> _U64(30))) * _U64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> _U64(27))) * _U64(0x94D049BB133111EB)
        return z ^ (z >> _U64(31))


def stream_key(seed: int, stream: int) -> int:
    """Per-bitmap key: mix64(seed * GAMMA + stream)."""
    return _mix64_int((seed * GAMMA + stream) & M64)


def rand64(key: int, ctr: np.ndarray) -> np.ndarray:
    """ctr-th output of the SplitMix64 sequence whose state starts at key."""
    ctr = np.asarray(ctr, dtype=_U64)
    with np.errstate(over="ignore"):
        return mix64(_U64(key) + (ctr + _U64(1)) * _U64(GAMMA))


def rand64_scalar(key: int, ctr: int) -> int:
    return _mix64_int((key + (ctr + 1) * GAMMA) & M64)


def unit_double(key: int, ctr: int) -> float:
    """Uniform in [0, 1) with 53 bits from one draw."""
    return (rand64_scalar(key, ctr) >> 11) * (1.0 / (1 << 53))


def u32_at(key: int, q: np.ndarray) -> np.ndarray:
    """The u32 uniform of bit position q: half (q & 1) of draw q >> 1."""
    q = np.asarray(q, dtype=_U64)
    r = rand64(key, q >> _U64(1))
    return (r >> ((q & _U64(1)) * _U64(32))) & _U64(0xFFFFFFFF)


def prob_to_thr(p: float) -> int:
    """Integer threshold on a u32 uniform; the effective probability is thr / 2**32."""
    if not (0.0 <= p <= 1.0):
        raise ValueError("probability out of range")
    return int(round(p * 4294967296.0))


def _pack_bits(bits: np.ndarray) -> np.ndarray:
    """bits: (m, 64) array of 0/1, bit b of word i -> uint64 words (little-endian)."""
    b = np.packbits(bits.astype(np.uint8), axis=1, bitorder="little")
    return np.ascontiguousarray(b).view("<u8").reshape(-1).astype(_U64)


def words_for_bits(r_bits: int) -> int:
    return (r_bits + 63) // 64


# ----------------------------------------------------------------- Bernoulli
def bernoulli_words(key: int, thr: int, w0: int, w1: int) -> np.ndarray:
    """Words [w0, w1) of a Bernoulli bitmap with stream key `key`."""
    if w1 <= w0:
        return np.zeros(0, dtype=_U64)
    q = np.arange(64 * w0, 64 * w1, dtype=_U64)
    u = u32_at(key, q)
    bits = (u < _U64(thr)).reshape(-1, 64)
    return _pack_bits(bits)


# -------------------------------------------------------------------- Markov
@dataclass(frozen=True)
class MarkovParams:
    A: int        # u < A  => next is 1 from state 0
    S: int        # u < S  => next is 1 from state 1
    init1: int    # 1 if the state before position 0 is 1

    @staticmethod
    def from_probs(key: int, p01: float, p10: float) -> "MarkovParams":
        # A position resets the chain with probability 1 - |1 - (p01 + p10)|;
        # random access scans back to the last reset, so keep that away from 0.
        if not (MIN_RESET <= p01 + p10 <= 2.0 - MIN_RESET):
            raise ValueError("Markov chain too close to constant or periodic for random access")
        A = prob_to_thr(p01)
        S = prob_to_thr(1.0 - p10)
        pi1 = 0.0 if p01 + p10 == 0 else p01 / (p01 + p10)
        u = rand64_scalar(key, CTR_INIT) & 0xFFFFFFFF
        return MarkovParams(A, S, 1 if u < prob_to_thr(pi1) else 0)

    @staticmethod
    def from_density_runlength(key: int, density: float, mean_ones_run: float) -> "MarkovParams":
        """Ones-runs geometric with mean m; zeros-runs mean m(1-d)/d, so the
        stationary density is d."""
        p10 = 1.0 / mean_ones_run
        if density <= 0.0:
            p01 = 0.0
        else:
            p01 = density / (mean_ones_run * (1.0 - density))
        p01 = min(p01, 2.0 - MIN_RESET - p10)
        if p01 + p10 < MIN_RESET:
            p01 = MIN_RESET - p10
        return MarkovParams.from_probs(key, p01, p10)


def _classify(u: np.ndarray, A: int, S: int):
    t1 = u < _U64(A)   # next state from 0
    t2 = u < _U64(S)   # next state from 1
    reset1 = t1 & t2
    reset0 = ~t1 & ~t2
    flip = t1 & ~t2
    return reset1, reset0, flip


def _entry_state(key: int, mp: MarkovParams, q0: int, chunk: int = 1 << 14) -> int:
    """State before bit position q0 (scanning back to the last reset)."""
    parity = 0
    hi = q0
    while hi > 0:
        lo = max(0, hi - chunk)
        u = u32_at(key, np.arange(lo, hi, dtype=_U64))
        r1, r0, fl = _classify(u, mp.A, mp.S)
        rs = np.flatnonzero(r1 | r0)
        if rs.size:
            last = int(rs[-1])
            parity ^= int(np.count_nonzero(fl[last + 1:])) & 1
            return (1 if r1[last] else 0) ^ parity
        parity ^= int(np.count_nonzero(fl)) & 1
        hi = lo
        chunk = min(chunk * 2, 1 << 22)
    return mp.init1 ^ parity


def markov_words(key: int, mp: MarkovParams, w0: int, w1: int) -> np.ndarray:
    """Words [w0, w1) of a Markov bitmap with stream key `key`."""
    if w1 <= w0:
        return np.zeros(0, dtype=_U64)
    q0 = 64 * w0
    s = _entry_state(key, mp, q0)
    u = u32_at(key, np.arange(q0, 64 * w1, dtype=_U64))
    r1, r0, fl = _classify(u, mp.A, mp.S)
    isr = r1 | r0
    idx = np.arange(u.size, dtype=np.int64)
    last = np.maximum.accumulate(np.where(isr, idx, -1))
    cf = np.cumsum(fl.astype(np.int64))
    has = last >= 0
    lastc = np.where(has, last, 0)
    val_reset = r1[lastc].astype(np.int64)
    par_since = (cf - cf[lastc]) & 1
    bits = np.where(has, val_reset ^ par_since, (s + cf) & 1)
    return _pack_bits(bits.reshape(-1, 64))


# ------------------------------------------------------------ fixed patterns
def exhaustive_words(j: int, n: int) -> np.ndarray:
    """Bitmap j of the exhaustive-combination fixture: r = 2**n positions and
    bit p of bitmap j is (p >> j) & 1, so position p sees every input
    combination once and its count is popcount(p)."""
    r = 1 << n
    p = np.arange(r, dtype=np.int64)
    bits = ((p >> j) & 1).astype(np.uint8)
    if r % 64:
        bits = np.concatenate([bits, np.zeros(64 - r % 64, dtype=np.uint8)])
    return _pack_bits(bits.reshape(-1, 64))


# ----------------------------------------------------- workload descriptions
def log_uniform(key: int, ctr: int, lo: float, hi: float) -> float:
    u = unit_double(key, ctr)
    return math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))


@dataclass(frozen=True)
class BernoulliSet:
    """N Bernoulli bitmaps of r bits; bitmap j has density dens[j]."""
    seed: int
    n: int
    r_bits: int
    dens: tuple

    def key(self, j: int) -> int:
        return stream_key(self.seed, j)

    def thr(self, j: int) -> int:
        return prob_to_thr(self.dens[j])

    @property
    def nwords(self) -> int:
        return words_for_bits(self.r_bits)

    def words(self, j: int, w0: int = 0, w1: int | None = None) -> np.ndarray:
        w1 = self.nwords if w1 is None else w1
        return bernoulli_words(self.key(j), self.thr(j), w0, w1)

    def keys_array(self) -> np.ndarray:
        return np.array([self.key(j) for j in range(self.n)], dtype=_U64)

    def thr_array(self) -> np.ndarray:
        return np.array([self.thr(j) for j in range(self.n)], dtype=_U64)


@dataclass(frozen=True)
class MarkovSet:
    """N Markov bitmaps of r bits with per-bitmap parameters."""
    seed: int
    n: int
    r_bits: int
    params: tuple  # MarkovParams per bitmap

    def key(self, j: int) -> int:
        return stream_key(self.seed, j)

    @property
    def nwords(self) -> int:
        return words_for_bits(self.r_bits)

    def words(self, j: int, w0: int = 0, w1: int | None = None) -> np.ndarray:
        w1 = self.nwords if w1 is None else w1
        return markov_words(self.key(j), self.params[j], w0, w1)

    def keys_array(self) -> np.ndarray:
        return np.array([self.key(j) for j in range(self.n)], dtype=_U64)

    def a_array(self) -> np.ndarray:
        return np.array([p.A for p in self.params], dtype=_U64)

    def s_array(self) -> np.ndarray:
        return np.array([p.S for p in self.params], dtype=_U64)

    def init_array(self) -> np.ndarray:
        return np.array([p.init1 for p in self.params], dtype=np.uint32)


def bernoulli_fixed(seed: int, n: int, r_bits: int, p: float) -> BernoulliSet:
    return BernoulliSet(seed, n, r_bits, tuple([p] * n))


def bernoulli_loguniform(seed: int, n: int, r_bits: int, lo: float, hi: float) -> BernoulliSet:
    """Per-bitmap density drawn log-uniform in [lo, hi]."""
    dens = tuple(log_uniform(stream_key(seed, j), CTR_PARAM, lo, hi) for j in range(n))
    return BernoulliSet(seed, n, r_bits, dens)


def markov_fixed(seed: int, n: int, r_bits: int, mean_ones: float, mean_zeros: float) -> MarkovSet:
    params = tuple(MarkovParams.from_probs(stream_key(seed, j), 1.0 / mean_zeros, 1.0 / mean_ones)
                   for j in range(n))
    return MarkovSet(seed, n, r_bits, params)


def markov_density_runlength(seed: int, n: int, r_bits: int, density: float, mean_ones: float) -> MarkovSet:
    params = tuple(MarkovParams.from_density_runlength(stream_key(seed, j), density, mean_ones)
                   for j in range(n))
    return MarkovSet(seed, n, r_bits, params)


# ------------------------------------------------------- the five workloads
# Sizes of the paper-shaped synthetic workloads.
SMALL = dict(n=16, r_bits=1 << 20, p=0.05, thetas=(1, 2, 8, 16))
LARGE = dict(n=256, r_bits=1 << 26, dens=(1e-4, 0.5), thetas=(2, 16, 128, 255), interval=(2, 10))
RLE = dict(n=512, r_bits=1 << 28, mean_ones=64.0, mean_zeros=4096.0, thetas=(2, 64, 256))
SELECTOR = dict(queries=2500, train=2000, r_bits=1 << 22, n=(2, 4096), dens=(1e-5, 0.5), runlen=(1.0, 4096.0))
SERVING = dict(pool=8192, r_bits=1 << 23, dens=(1e-4, 0.3), queries=20000, n=(2, 1024))


def small_set(seed: int = 1) -> BernoulliSet:
    return bernoulli_fixed(seed, SMALL["n"], SMALL["r_bits"], SMALL["p"])


def large_set(seed: int = 2, n: int | None = None, r_bits: int | None = None) -> BernoulliSet:
    return bernoulli_loguniform(seed, n or LARGE["n"], r_bits or LARGE["r_bits"], *LARGE["dens"])


def rle_set(seed: int = 3, n: int | None = None, r_bits: int | None = None) -> MarkovSet:
    return markov_fixed(seed, n or RLE["n"], r_bits or RLE["r_bits"], RLE["mean_ones"], RLE["mean_zeros"])


@dataclass(frozen=True)
class SelectorQuery:
    n: int
    theta: int
    density: float
    mean_run: float
    seed: int


def selector_queries(seed: int = 4, count: int | None = None) -> list:
    """Queries with N log-uniform in [2, 4096], density log-uniform in
    [1e-5, 0.5], mean ones-run log-uniform in [1, 4096], theta = max(1, ceil(u N))
    with u uniform in (0, 1]."""
    count = SELECTOR["queries"] if count is None else count
    out = []
    for qi in range(count):
        k = stream_key(seed, 1_000_000 + qi)
        n = int(min(SELECTOR["n"][1], max(SELECTOR["n"][0], round(log_uniform(k, 1, *SELECTOR["n"])))))
        d = log_uniform(k, 2, *SELECTOR["dens"])
        m = log_uniform(k, 3, *SELECTOR["runlen"])
        u = 1.0 - unit_double(k, 4)            # (0, 1]
        theta = max(1, math.ceil(u * n))
        out.append(SelectorQuery(n, theta, d, m, (seed * 7919 + qi) & M64))
    return out


@dataclass(frozen=True)
class ServingQuery:
    members: tuple   # distinct pool indices
    theta: int
    arrival_s: float


def serving_queries(seed: int = 5, count: int | None = None, pool: int | None = None,
                    rate_qps: float = 1000.0, n_range: tuple | None = None) -> list:
    """Queries choosing N log-uniform in [2, 1024] distinct pool members
    uniformly without replacement, theta uniform in [1, N], Poisson arrivals
    at rate_qps."""
    count = SERVING["queries"] if count is None else count
    pool = SERVING["pool"] if pool is None else pool
    lo, hi = n_range or SERVING["n"]
    t = 0.0
    out = []
    for qi in range(count):
        k = stream_key(seed, 2_000_000 + qi)
        n = int(min(hi, max(lo, round(log_uniform(k, 1, lo, hi)))))
        n = min(n, pool)
        # partial Fisher-Yates over the pool driven by the counter stream
        chosen = {}
        members = []
        for i in range(n):
            j = i + int(unit_double(k, 10 + i) * (pool - i))
            a = chosen.get(j, j)
            chosen[j] = chosen.get(i, i)
            members.append(a)
        theta = 1 + int(unit_double(k, 2) * n)
        theta = min(theta, n)
        t += -math.log(1.0 - unit_double(k, 3)) / rate_qps
        out.append(ServingQuery(tuple(members), theta, t))
    return out


# --------------------------------------------------------- device filling
# The same bit processes as above, generated on the GPU by tqgen/gen.hip.
_gen_lib = None


def _gpu_lib():
    global _gen_lib
    if _gen_lib is None:
        import ctypes
        import os
        import torch  # noqa: F401  (binds the library to torch's HIP runtime)
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtqgen.so")
        if not os.path.exists(path):
            raise RuntimeError("libtqgen.so is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(path)
        P, U32, U64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        L.tqgen_bernoulli_pool.argtypes = [P, U64, U64, U32, P, P, P]
        L.tqgen_markov_pool.argtypes = [P, U64, U64, U32, P, P, P, P, P]
        L.tqgen_bernoulli_pool.restype = ctypes.c_int
        L.tqgen_markov_pool.restype = ctypes.c_int
        _gen_lib = L
    return _gen_lib


def fill_gpu(bset, pool, stride_words: int | None = None, first: int = 0, count: int | None = None):
    """Generate bitmaps [first, first+count) of a BernoulliSet or MarkovSet
    into the int64 CUDA tensor `pool` (bitmap first+i at word i*stride)."""
    import torch
    count = bset.n - first if count is None else count
    stride = bset.nwords if stride_words is None else stride_words
    assert pool.dtype == torch.int64 and pool.is_cuda and pool.is_contiguous()
    assert pool.numel() >= (count - 1) * stride + bset.nwords if count else True
    dev = pool.device
    keys = torch.from_numpy(bset.keys_array()[first:first + count].view(np.int64)).to(dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    L = _gpu_lib()
    if isinstance(bset, BernoulliSet):
        thr = torch.from_numpy(bset.thr_array()[first:first + count].view(np.int64)).to(dev)
        rc = L.tqgen_bernoulli_pool(pool.data_ptr(), stride, bset.nwords, count, keys.data_ptr(),
                                    thr.data_ptr(), stream)
        keep = (keys, thr)
    else:
        A = torch.from_numpy(bset.a_array()[first:first + count].view(np.int64)).to(dev)
        S = torch.from_numpy(bset.s_array()[first:first + count].view(np.int64)).to(dev)
        I = torch.from_numpy(bset.init_array()[first:first + count].view(np.int32)).to(dev)
        rc = L.tqgen_markov_pool(pool.data_ptr(), stride, bset.nwords, count, keys.data_ptr(),
                                 A.data_ptr(), S.data_ptr(), I.data_ptr(), stream)
        keep = (keys, A, S, I)
    if rc != 0:
        raise RuntimeError("tqgen kernel launch failed: %d" % rc)
    torch.cuda.current_stream(dev).synchronize()
    del keep
    return pool
