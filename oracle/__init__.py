"""Oracle for threshold and symmetric queries over bitmaps.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline of bench.py, never by the library.  It shares no code with the GPU
path.  The arithmetic lives in ``tq_oracle.c`` (plain C, per-position
counters, see the comments there for the passages it follows); this module
only marshals numpy arrays and builds the C file with gcc.

``mlp_ref`` holds the fp64 reference of the kernel-selector network.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EFORMAT = -3
EINVAL = -1


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP over word columns)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = _load(_LIB)
    return _lib


def use_library(path: str) -> None:
    """Point this module at another build of the C oracle (the planted-mistake
    tests load deliberately broken copies through this)."""
    global _lib
    _lib = _load(path)


def _load(path: str):
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    U32, U64 = ctypes.c_uint32, ctypes.c_uint64
    L.oracle_threshold_cols.argtypes = [P, U32, U64, P, U64, U32, P]
    L.oracle_symmetric_cols.argtypes = [P, U32, U64, P, U64, P, P]
    L.oracle_threshold.argtypes = [P, U32, U64, U32, P]
    L.oracle_symmetric.argtypes = [P, U32, U64, P, P]
    L.oracle_rle_decode.argtypes = [P, U64, U64, P]
    L.oracle_rle_encode.argtypes = [P, U64, P, U64]
    L.oracle_rle_encode.restype = U64
    L.oracle_run_count.argtypes = [P, U64]
    L.oracle_run_count.restype = U64
    L.oracle_set_threads.argtypes = [ctypes.c_int]
    L.oracle_set_threads.restype = None
    L.oracle_max_threads.argtypes = []
    L.oracle_max_threads.restype = ctypes.c_int
    L.oracle_count.argtypes = [P, U64]
    L.oracle_count.restype = U64
    L.oracle_weighted_threshold.argtypes = [P, U32, P, U64, U64, P]
    L.oracle_weighted_threshold.restype = ctypes.c_int
    for f in ("oracle_threshold_cols", "oracle_symmetric_cols", "oracle_threshold",
              "oracle_symmetric", "oracle_rle_decode"):
        getattr(L, f).restype = ctypes.c_int
    return L


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def nwords(r_bits: int) -> int:
    return (r_bits + 63) // 64


def _ptr_array(bitmaps):
    arrs = [_u64(b) for b in bitmaps]
    ptrs = (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    return arrs, ptrs


def threshold(bitmaps, r_bits: int, theta: int) -> np.ndarray:
    """Output bitmap of the theta-threshold over full bitmaps."""
    n = len(bitmaps)
    arrs, ptrs = _ptr_array(bitmaps)
    for a in arrs:
        assert a.size >= nwords(r_bits)
    out = np.zeros(nwords(r_bits), dtype=np.uint64)
    rc = lib().oracle_threshold(ptrs, n, r_bits, theta, out.ctypes.data)
    if rc:
        raise ValueError("oracle_threshold: %d" % rc)
    return out


def symmetric(bitmaps, r_bits: int, truth) -> np.ndarray:
    """Output bitmap of the symmetric function with truth table truth[0..N]."""
    n = len(bitmaps)
    f = np.ascontiguousarray(np.asarray(truth, dtype=np.uint8))
    assert f.size == n + 1
    arrs, ptrs = _ptr_array(bitmaps)
    out = np.zeros(nwords(r_bits), dtype=np.uint64)
    rc = lib().oracle_symmetric(ptrs, n, r_bits, f.ctypes.data, out.ctypes.data)
    if rc:
        raise ValueError("oracle_symmetric: %d" % rc)
    return out


def weighted_threshold(bitmaps, weights, r_bits: int, theta: int) -> np.ndarray:
    """Output bitmap of sum of weights[j] * bit_j(p) >= theta."""
    n = len(bitmaps)
    wt = np.ascontiguousarray(np.asarray(weights, dtype=np.uint32))
    assert wt.size == n
    arrs, ptrs = _ptr_array(bitmaps)
    out = np.zeros(nwords(r_bits), dtype=np.uint64)
    rc = lib().oracle_weighted_threshold(ptrs, n, wt.ctypes.data, r_bits, theta, out.ctypes.data)
    if rc:
        raise ValueError("oracle_weighted_threshold: %d" % rc)
    return out


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (timing only)."""
    lib().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def count(words, r_bits: int) -> int:
    """Number of set positions p < r_bits of a bitmap."""
    w = _u64(words)
    assert w.size >= nwords(r_bits)
    return int(lib().oracle_count(w.ctypes.data, r_bits))


def consume(result, r_bits: int, filt=None):
    """Consumers of a result bitmap (abstract and introduction: the result
    is again a bitmap, combined with other criteria by AND, or counted):
    returns (result AND filt, number of set positions below r_bits)."""
    out = _u64(result).copy()
    if filt is not None:
        out &= _u64(filt)[:out.size]
    return out, count(out, r_bits)


def threshold_cols(words: np.ndarray, col_index, r_bits: int, theta: int) -> np.ndarray:
    """words: (N, m) matrix of sampled word columns; col_index: word index of each column."""
    w = _u64(words)
    n, m = w.shape
    ci = _u64(col_index)
    out = np.zeros(m, dtype=np.uint64)
    rc = lib().oracle_threshold_cols(w.ctypes.data, n, m, ci.ctypes.data, r_bits, theta, out.ctypes.data)
    if rc:
        raise ValueError("oracle_threshold_cols: %d" % rc)
    return out


def symmetric_cols(words: np.ndarray, col_index, r_bits: int, truth) -> np.ndarray:
    w = _u64(words)
    n, m = w.shape
    f = np.ascontiguousarray(np.asarray(truth, dtype=np.uint8))
    assert f.size == n + 1
    ci = _u64(col_index)
    out = np.zeros(m, dtype=np.uint64)
    rc = lib().oracle_symmetric_cols(w.ctypes.data, n, m, ci.ctypes.data, r_bits, f.ctypes.data,
                                     out.ctypes.data)
    if rc:
        raise ValueError("oracle_symmetric_cols: %d" % rc)
    return out


def rle_encode(dense, r_bits: int) -> np.ndarray:
    """Canonical RLE stream of a dense bitmap (bits >= r cleared)."""
    d = _u64(dense)
    assert d.size >= nwords(r_bits)
    L = lib()
    need = L.oracle_rle_encode(d.ctypes.data, r_bits, None, 0)
    out = np.zeros(max(int(need), 1), dtype=np.uint64)
    got = L.oracle_rle_encode(d.ctypes.data, r_bits, out.ctypes.data, need)
    assert got == need
    return out[:need]


def rle_decode(stream, r_bits: int) -> np.ndarray:
    """Dense words of a stream; raises ValueError on a malformed stream."""
    s = _u64(stream)
    nw = nwords(r_bits)
    out = np.zeros(max(nw, 1), dtype=np.uint64)
    rc = lib().oracle_rle_decode(s.ctypes.data if s.size else None, s.size, nw, out.ctypes.data)
    if rc:
        raise ValueError("malformed RLE stream (%d)" % rc)
    return out[:nw]


def run_count(dense, r_bits: int) -> int:
    d = _u64(dense)
    return int(lib().oracle_run_count(d.ctypes.data, r_bits))


# convenience truth tables (the functions named in section 2.2)
def truth_threshold(n: int, theta: int) -> np.ndarray:
    return np.array([1 if c >= theta else 0 for c in range(n + 1)], dtype=np.uint8)


def truth_interval(n: int, lo: int, hi: int) -> np.ndarray:
    return np.array([1 if lo <= c <= hi else 0 for c in range(n + 1)], dtype=np.uint8)


def truth_parity(n: int) -> np.ndarray:
    return np.array([c & 1 for c in range(n + 1)], dtype=np.uint8)


if __name__ == "__main__":
    build(force=True)
    print(_LIB)
    sys.exit(0)
