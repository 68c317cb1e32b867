"""ctypes binding of libtq.so: argument marshalling only.

Every function here has the name of the C entry point it forwards to and
does nothing but convert Python/torch arguments into plain pointers and
sizes.  All computation runs in the HIP kernels of libtq.so; if the library
is not built this module raises on import instead of falling back to
anything else.

torch is imported first on purpose: PyTorch ships its own copy of the HIP
runtime (same soname as /opt/rocm's), and libtq.so must bind to that copy so
that torch-allocated device memory and torch streams are the library's too.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede loading libtq.so)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtq.so")

TQ_OK = 0
TQ_EINVAL = -1
TQ_ENOMEM = -2
TQ_EFORMAT = -3
TQ_ECAPACITY = -4
TQ_EDEVICE = -5
TQ_EBUSY = -6
TQ_ENOTSUP = -7
TQ_ECANCELED = -8
TQ_ETIMEDOUT = -9
TQ_MAX_INPUTS = 65535

_P = ctypes.c_void_p
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64
_INT = ctypes.c_int


class TQError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s" % (where, status_string(status)))


def _load():
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libtq.so is not built (%s); run __graft_entry__.build() or "
            "python paper_1402_4073_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "tq_create": (_INT, [ctypes.POINTER(_P), _INT]),
        "tq_destroy": (_INT, [_P]),
        "tq_status_string": (ctypes.c_char_p, [_INT]),
        "tq_ctx_check": (_INT, [_P, _P]),
        "tq_set_option": (_INT, [_P, _INT, ctypes.c_int64]),
        "tq_threshold": (_INT, [_P, _P, _U32, _U64, _U32, _P, _P]),
        "tq_symmetric": (_INT, [_P, _P, _U32, _U64, _P, _P, _P]),
        "tq_threshold_fused": (_INT, [_P, _P, _U32, _U64, _U32, _P, _P, _P, _P]),
        "tq_threshold_fused_noalloc": (_INT, [_P, _P, _U32, _U64, _U32, _P, _P, _P, _P]),
        "tq_threshold_weighted": (_INT, [_P, _P, _U32, _P, _U64, _U64, _P, _P]),
        "tq_symmetric_fused": (_INT, [_P, _P, _U32, _U64, _P, _P, _P, _P, _P]),
        "tq_rle_max_words": (_U64, [_U64]),
        "tq_rle_index_words": (_U64, [_U64]),
        "tq_rle_encode": (_INT, [_P, _P, _U64, _P, _U64, _P, _P, _P]),
        "tq_rle_build_index": (_INT, [_P, _P, _U64, _U64, _P, _P]),
        "tq_rle_decode": (_INT, [_P, _P, _U64, _P, _P]),
        "tq_threshold_rle": (_INT, [_P, _P, _U32, _U64, _U32, _P, _U64, _P, _P]),
        "tq_threshold_rle_dense": (_INT, [_P, _P, _U32, _U64, _U32, _P, _P]),
        "tq_threshold_rle_fused": (_INT, [_P, _P, _U32, _U64, _U32, _P, _P, _P, _P]),
        "tq_symmetric_rle_fused": (_INT, [_P, _P, _U32, _U64, _P, _P, _P, _P, _P]),
        "tq_threshold_hybrid": (_INT, [_P, _P, _U32, _P, _U32, _U64, _U32, _P, _P]),
        "tq_symmetric_rle": (_INT, [_P, _P, _U32, _U64, _P, _P, _U64, _P, _P]),
        "tq_symmetric_rle_dense": (_INT, [_P, _P, _U32, _U64, _P, _P, _P]),
        "tq_symmetric_hybrid": (_INT, [_P, _P, _U32, _P, _U32, _U64, _P, _P, _P]),
        "tq_batch_submit": (_INT, [_P, _P, _U32, _U32, _P, ctypes.POINTER(_P)]),
        "tq_batch_poll": (_INT, [_P, ctypes.POINTER(_U32)]),
        "tq_batch_wait": (_INT, [_P]),
        "tq_batch_records": (_INT, [_P, _P]),
        "tq_batch_release": (_INT, [_P]),
        "tq_batch_cancel": (_INT, [_P]),
        "tq_batch_tune": (_INT, [_P, _P, _U32, _P, ctypes.POINTER(_U32), ctypes.POINTER(_U32)]),
        "tq_batch_set_schedule": (_INT, [_P, _U32, _U32]),
        "tq_tune_export": (_INT, [_P, ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
        "tq_tune_import": (_INT, [_P, ctypes.c_char_p]),
        "tq_tune_clear": (_INT, [_P]),
        "tq_bitmap_stats": (_INT, [_P, _P, _U64, _P, _P, _P]),
        "tq_query_features": (_INT, [_P, _U32, _U64, _U32, _P]),
        "tq_threshold_variant": (_INT, [_P, _P, _U32, _U64, _U32, _U32, _P, _P]),
        "tq_selector_param_count": (_U64, []),
        "tq_selector_set": (_INT, [_P, _P, _P, _P, _P, _P, ctypes.c_float]),
        "tq_selector_predict": (_INT, [_P, _P, _P]),
        "tq_threshold_auto": (_INT, [_P, _P, _U32, _U64, _U32, _P, _U32, ctypes.POINTER(_U32), _P]),
        "tq_mlp_forward": (_INT, [_P, _P, _P, _U32, _P, _P]),
        "tq_mlp_grad": (_INT, [_P, _P, _P, _P, _P, _U32, ctypes.c_float, _P, _P, _P, _P]),
        "tq_mlp_adam": (_INT, [_P, _P, _P, _P, _P, _U32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_float, _U32, _P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def lib() -> ctypes.CDLL:
    return _lib


def hip_runtimes_loaded() -> list:
    """Distinct libamdhip64 files mapped into this process (must be one)."""
    paths = set()
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return sorted(paths)


def status_string(status: int) -> str:
    return _lib.tq_status_string(status).decode()


def _check(status: int, where: str) -> None:
    if status != TQ_OK:
        raise TQError(status, where)


def _ptr(x) -> int:
    """Device address of a tensor, or an int taken as an address."""
    if isinstance(x, torch.Tensor):
        return x.data_ptr()
    return int(x)


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def ptr_array(inputs):
    """Host array of device pointers (ctypes), from tensors or addresses."""
    arr = (_U64 * max(1, len(inputs)))(*[_ptr(t) for t in inputs])
    return arr


def _u64_host(words):
    arr = (_U64 * max(1, len(words)))(*[int(w) for w in words])
    return arr


def truth_words(truth) -> list:
    """Pack a 0/1 truth table f[0..n] into 64-bit words (bit c = f(c))."""
    vals = [int(v) & 1 for v in truth]
    words = [0] * ((len(vals) + 63) // 64)
    for c, v in enumerate(vals):
        if v:
            words[c // 64] |= 1 << (c % 64)
    return words


def truth_interval(n: int, lo: int, hi: int) -> list:
    """Truth table f[0..n] of the interval query lo <= count <= hi (section 2.2)."""
    return [1 if lo <= c <= hi else 0 for c in range(n + 1)]


def truth_parity(n: int) -> list:
    """Truth table f[0..n] of parity, 1 iff the count is odd (section 2.2)."""
    return [c & 1 for c in range(n + 1)]


# ------------------------------------------------------------------ context
def tq_create(device: int = 0) -> int:
    h = _P()
    _check(_lib.tq_create(ctypes.byref(h), device), "tq_create")
    return h.value


def tq_destroy(ctx: int) -> None:
    _check(_lib.tq_destroy(ctx), "tq_destroy")


TQ_OPTION_PRUNE = 1
TQ_OPTION_RLE_TILES = 2
TQ_OPTION_AUTOTUNE = 3
TQ_OPTION_RLE_COUNTERS = 4
TQ_OPTION_LOOPED = 5
TQ_OPTION_BATCH_BYTES = 6
TQ_OPTION_SPLIT = 8
TQ_OPTION_BATCH_DEADLINE_US = 7


def tq_set_option(ctx: int, option: int, value: int) -> None:
    _check(_lib.tq_set_option(ctx, option, value), "tq_set_option")


def raw_set_option(ctx: int, option: int, value: int) -> int:
    """tq_set_option returning the status instead of raising."""
    return _lib.tq_set_option(ctx, option, value)


def tq_ctx_check(ctx: int, stream=None) -> int:
    """Return the status (0 or a negative tq_status) without raising."""
    return _lib.tq_ctx_check(ctx, _stream(stream))


# ------------------------------------------------------------------ queries
def tq_threshold(ctx: int, inputs, r_bits: int, theta: int, out, stream=None) -> None:
    ptrs = ptr_array(inputs)
    _check(_lib.tq_threshold(ctx, ptrs, len(inputs), r_bits, theta, _ptr(out), _stream(stream)),
           "tq_threshold")


def tq_symmetric(ctx: int, inputs, r_bits: int, truth, out, stream=None) -> None:
    """truth: sequence of 0/1 values f(0..n) (packed here into words)."""
    ptrs = ptr_array(inputs)
    tw = _u64_host(truth_words(truth))
    _check(_lib.tq_symmetric(ctx, ptrs, len(inputs), r_bits, tw, _ptr(out), _stream(stream)),
           "tq_symmetric")


def _u32_host(values):
    arr = (ctypes.c_uint32 * max(1, len(values)))()
    for i, v in enumerate(values):
        arr[i] = int(v)
    return arr


def tq_threshold_weighted(ctx: int, inputs, weights, r_bits: int, theta: int, out, stream=None) -> None:
    """out bit p = [sum_j weights[j] * bit_j(p) >= theta] (non-negative integer weights)."""
    ptrs = ptr_array(inputs)
    _check(_lib.tq_threshold_weighted(ctx, ptrs, len(inputs), _u32_host(weights), r_bits, theta, _ptr(out),
                                      _stream(stream)), "tq_threshold_weighted")


def raw_threshold_weighted(ctx: int, inputs, weights, r_bits: int, theta: int, out_ptr, stream=None) -> int:
    ptrs = ptr_array(inputs)
    w = _u32_host(weights) if weights is not None else None
    return _lib.tq_threshold_weighted(ctx, ptrs, len(inputs), w, r_bits, theta, out_ptr, _stream(stream))


def _optr(t):
    """Device pointer of an optional tensor (None -> NULL)."""
    return None if t is None else _ptr(t)


def tq_threshold_fused(ctx: int, inputs, r_bits: int, theta: int, filt=None, out=None, count=None,
                       stream=None) -> None:
    """out = T_theta(inputs) AND filt; count[0] = popcount(out) (each optional)."""
    ptrs = ptr_array(inputs)
    _check(_lib.tq_threshold_fused(ctx, ptrs, len(inputs), r_bits, theta, _optr(filt), _optr(out), _optr(count),
                                   _stream(stream)), "tq_threshold_fused")


def tq_threshold_fused_noalloc(ctx: int, inputs, r_bits: int, theta: int, filt=None, out=None, count=None,
                               stream=None) -> None:
    """tq_threshold_fused through the entry point that allocates nothing."""
    ptrs = ptr_array(inputs)
    _check(_lib.tq_threshold_fused_noalloc(ctx, ptrs, len(inputs), r_bits, theta, _optr(filt), _optr(out),
                                           _optr(count), _stream(stream)), "tq_threshold_fused_noalloc")


def raw_threshold_fused_noalloc(ctx: int, inputs, r_bits: int, theta: int, filt_ptr, out_ptr, count_ptr,
                                stream=None) -> int:
    """Status code of tq_threshold_fused_noalloc with raw device addresses (0 = NULL)."""
    ptrs = ptr_array(inputs)
    return _lib.tq_threshold_fused_noalloc(ctx, ptrs, len(inputs), r_bits, theta, filt_ptr, out_ptr, count_ptr,
                                           _stream(stream))


def tq_symmetric_fused(ctx: int, inputs, r_bits: int, truth, filt=None, out=None, count=None,
                       stream=None) -> None:
    ptrs = ptr_array(inputs)
    tw = _u64_host(truth_words(truth))
    _check(_lib.tq_symmetric_fused(ctx, ptrs, len(inputs), r_bits, tw, _optr(filt), _optr(out), _optr(count),
                                   _stream(stream)), "tq_symmetric_fused")


def raw_threshold_fused(ctx: int, ptrs, n: int, r_bits: int, theta: int, filt_ptr, out_ptr, count_ptr,
                        stream=None) -> int:
    return _lib.tq_threshold_fused(ctx, ptrs, n, r_bits, theta, filt_ptr, out_ptr, count_ptr, _stream(stream))


def raw_threshold(ctx: int, ptrs, n: int, r_bits: int, theta: int, out_ptr: int, stream=None) -> int:
    """Unchecked call returning the status (for error-path tests)."""
    return _lib.tq_threshold(ctx, ptrs, n, r_bits, theta, out_ptr, _stream(stream))


# ------------------------------------------------------------------- RLE
TQ_RLE_INDEX_STRIDE = 512
TQ_RLE_MAX_INPUTS = 8192


class TqRle(ctypes.Structure):
    _fields_ = [("words", _U64), ("n_words", _U64), ("index", _U64)]


def rle_array(inputs):
    """Host array of tq_rle from (words, n_words, index) triples; index may be None."""
    arr = (TqRle * max(1, len(inputs)))()
    for i, (w, nw, idx) in enumerate(inputs):
        arr[i].words = _ptr(w)
        arr[i].n_words = int(nw)
        arr[i].index = 0 if idx is None else _ptr(idx)
    return arr


def tq_rle_max_words(r_bits: int) -> int:
    return int(_lib.tq_rle_max_words(r_bits))


def tq_rle_index_words(r_bits: int) -> int:
    return int(_lib.tq_rle_index_words(r_bits))


def tq_rle_encode(ctx: int, dense, r_bits: int, out, out_cap: int, out_len, index=None, stream=None) -> None:
    _check(_lib.tq_rle_encode(ctx, _ptr(dense), r_bits, _ptr(out) if out is not None else 0, out_cap,
                              _ptr(out_len), 0 if index is None else _ptr(index), _stream(stream)),
           "tq_rle_encode")


def tq_rle_build_index(ctx: int, words, n_words: int, r_bits: int, index, stream=None) -> None:
    _check(_lib.tq_rle_build_index(ctx, _ptr(words), n_words, r_bits, _ptr(index), _stream(stream)),
           "tq_rle_build_index")


def tq_rle_decode(ctx: int, rle, r_bits: int, dense, stream=None) -> None:
    """rle: (words, n_words, index-or-None)."""
    arr = rle_array([rle])
    _check(_lib.tq_rle_decode(ctx, arr, r_bits, _ptr(dense), _stream(stream)), "tq_rle_decode")


def tq_threshold_rle(ctx: int, inputs, r_bits: int, theta: int, out, out_cap: int, out_len, stream=None) -> None:
    arr = rle_array(inputs)
    _check(_lib.tq_threshold_rle(ctx, arr, len(inputs), r_bits, theta, _ptr(out) if out is not None else 0,
                                 out_cap, _ptr(out_len), _stream(stream)), "tq_threshold_rle")


def tq_threshold_rle_dense(ctx: int, inputs, r_bits: int, theta: int, out, stream=None) -> None:
    arr = rle_array(inputs)
    _check(_lib.tq_threshold_rle_dense(ctx, arr, len(inputs), r_bits, theta, _ptr(out), _stream(stream)),
           "tq_threshold_rle_dense")


def tq_threshold_rle_fused(ctx: int, inputs, r_bits: int, theta: int, filt=None, out=None, count=None,
                           stream=None) -> None:
    """out = T_theta(compressed inputs) AND filt; count[0] = popcount(out) (each optional)."""
    arr = rle_array(inputs)
    _check(_lib.tq_threshold_rle_fused(ctx, arr, len(inputs), r_bits, theta, _optr(filt), _optr(out), _optr(count),
                                       _stream(stream)), "tq_threshold_rle_fused")


def tq_symmetric_rle_fused(ctx: int, inputs, r_bits: int, truth, filt=None, out=None, count=None,
                           stream=None) -> None:
    arr = rle_array(inputs)
    tw = _u64_host(truth_words(truth))
    _check(_lib.tq_symmetric_rle_fused(ctx, arr, len(inputs), r_bits, tw, _optr(filt), _optr(out), _optr(count),
                                       _stream(stream)), "tq_symmetric_rle_fused")


def tq_threshold_hybrid(ctx: int, rle_inputs, dense_inputs, r_bits: int, theta: int, out, stream=None) -> None:
    arr = rle_array(rle_inputs)
    ptrs = ptr_array(dense_inputs)
    _check(_lib.tq_threshold_hybrid(ctx, arr, len(rle_inputs), ptrs, len(dense_inputs), r_bits, theta, _ptr(out),
                                    _stream(stream)), "tq_threshold_hybrid")


def tq_symmetric_rle(ctx: int, inputs, r_bits: int, truth, out, out_cap: int, out_len, stream=None) -> None:
    """truth: f(0..n) as 0/1 values."""
    arr = rle_array(inputs)
    tw = _u64_host(truth_words(truth))
    _check(_lib.tq_symmetric_rle(ctx, arr, len(inputs), r_bits, tw, _ptr(out) if out is not None else 0,
                                 out_cap, _ptr(out_len), _stream(stream)), "tq_symmetric_rle")


def tq_symmetric_rle_dense(ctx: int, inputs, r_bits: int, truth, out, stream=None) -> None:
    arr = rle_array(inputs)
    tw = _u64_host(truth_words(truth))
    _check(_lib.tq_symmetric_rle_dense(ctx, arr, len(inputs), r_bits, tw, _ptr(out), _stream(stream)),
           "tq_symmetric_rle_dense")


def tq_symmetric_hybrid(ctx: int, rle_inputs, dense_inputs, r_bits: int, truth, out, stream=None) -> None:
    arr = rle_array(rle_inputs)
    ptrs = ptr_array(dense_inputs)
    tw = _u64_host(truth_words(truth))
    _check(_lib.tq_symmetric_hybrid(ctx, arr, len(rle_inputs), ptrs, len(dense_inputs), r_bits, tw, _ptr(out),
                                    _stream(stream)), "tq_symmetric_hybrid")


def raw_threshold_rle_fused(ctx: int, inputs, r_bits: int, theta: int, filt_ptr, out_ptr, count_ptr,
                            stream=None) -> int:
    """Status code of tq_threshold_rle_fused with raw device addresses (0 = NULL)."""
    arr = rle_array(inputs)
    return _lib.tq_threshold_rle_fused(ctx, arr, len(inputs), r_bits, theta, filt_ptr or None, out_ptr or None,
                                       count_ptr or None, _stream(stream))


def raw_threshold_rle(ctx: int, inputs, r_bits: int, theta: int, out_ptr: int, out_cap: int, out_len_ptr: int,
                      stream=None) -> int:
    arr = rle_array(inputs)
    return _lib.tq_threshold_rle(ctx, arr, len(inputs), r_bits, theta, out_ptr, out_cap, out_len_ptr,
                                 _stream(stream))


def encode_pool(ctx: int, dense_rows, r_bits: int, stream=None):
    """Encode dense device bitmaps into one compact device pool of canonical
    streams with their checkpoint indexes (two passes: lengths, then data).
    Returns (pool, offsets, lengths, index_pool)."""
    n = len(dense_rows)
    dev = dense_rows[0].device
    lens = torch.zeros(n, dtype=torch.int64, device=dev)
    for j, row in enumerate(dense_rows):
        tq_rle_encode(ctx, row, r_bits, None, 0, lens[j:j + 1], None, stream)
    # the first pass records "capacity too small" on purpose: clear it
    tq_ctx_check(ctx, stream)
    hl = lens.cpu().tolist()
    offs = [0]
    for L in hl:
        offs.append(offs[-1] + ((L + 1) & ~1))   # keep every stream 16-byte aligned
    pool = torch.zeros(max(offs[-1], 1), dtype=torch.int64, device=dev)
    iw = tq_rle_index_words(r_bits)
    index_pool = torch.zeros((n, max(iw, 1)), dtype=torch.int64, device=dev)
    lens2 = torch.zeros(n, dtype=torch.int64, device=dev)
    for j, row in enumerate(dense_rows):
        tq_rle_encode(ctx, row, r_bits, pool[offs[j]:], hl[j], lens2[j:j + 1], index_pool[j], stream)
    st = tq_ctx_check(ctx, stream)
    if st != TQ_OK:
        raise TQError(st, "encode_pool")
    return pool, offs[:-1], hl, index_pool


# ------------------------------------------------------------------ batch
TQ_QUERY_THRESHOLD = 0
TQ_QUERY_SYMMETRIC = 1
TQ_BATCH_NO_GRAPH = 1
TQ_BATCH_MAX_QUERIES = 8192
TQ_BATCH_MAX_POINTERS = 2097152
TQ_BATCH_MAX_TABLE_BYTES = 1048576
TQ_BATCH_MAX_INFLIGHT = 16
TQ_VARIANT_AUTO = 0xFFFFFFFF


class TqQuery(ctypes.Structure):
    _fields_ = [("kind", _U32), ("n", _U32), ("ptrs", _U64), ("r_bits", _U64), ("theta", _U32),
                ("variant", _U32), ("h_truth", _U64), ("d_out", _U64), ("user_tag", _U64), ("inputs", _U64),
                ("out_cap", _U64), ("d_out_len", _U64)]


class TqQueryRecord(ctypes.Structure):
    _fields_ = [("user_tag", _U64), ("status", ctypes.c_int32), ("done", _U32),
                ("t_start_ns", _U64), ("t_end_ns", _U64), ("variant", _U32), ("pad", _U32)]


def _fill_query(q, keep, r_bits, out, theta=None, truth=None, tag=0, inputs=None, bitmaps=None,
                variant=0, out_cap=0, out_len=None):
    """Fill a TqQuery; host arrays it points to are appended to keep.
    inputs: dense device inputs (tensors/addresses); bitmaps: registered
    inputs (dicts as for bitmap_array, or a prebuilt TqBitmap array)."""
    if (inputs is None) == (bitmaps is None):
        raise ValueError("give exactly one of inputs and bitmaps")
    if inputs is not None:
        ptrs = ptr_array(inputs)
        keep.append(ptrs)
        q.n = len(inputs)
        q.ptrs = ctypes.addressof(ptrs)
    else:
        arr = bitmaps if isinstance(bitmaps, ctypes.Array) else bitmap_array(bitmaps)
        keep.append(arr)
        q.n = len(bitmaps)
        q.inputs = ctypes.addressof(arr)
    q.r_bits = int(r_bits)
    q.d_out = _ptr(out)
    q.user_tag = int(tag)
    q.variant = int(variant)
    q.out_cap = int(out_cap)
    q.d_out_len = 0 if out_len is None else _ptr(out_len)
    if truth is not None:
        tw = _u64_host(truth_words(truth))
        keep.append(tw)
        q.kind = TQ_QUERY_SYMMETRIC
        q.h_truth = ctypes.addressof(tw)
    else:
        q.kind = TQ_QUERY_THRESHOLD
        q.theta = int(theta)


class PreparedQuery:
    """A query with its host arrays and tq_query record already built
    (marshalled once, reusable across submissions)."""
    __slots__ = ("ptrs", "n", "r_bits", "theta", "out", "tag", "keep", "rec")

    def __init__(self, inputs, r_bits, out, theta=None, truth=None, tag=0, bitmaps=None, variant=0, out_cap=0,
                 out_len=None):
        self.keep = []
        q = TqQuery()
        _fill_query(q, self.keep, r_bits, out, theta, truth, tag, inputs=inputs, bitmaps=bitmaps, variant=variant,
                    out_cap=out_cap, out_len=out_len)
        self.ptrs = self.keep[0] if inputs is not None else None
        self.n = q.n
        self.r_bits = int(r_bits)
        self.out = _ptr(out)
        self.theta = theta
        self.tag = int(tag)
        self.rec = q


def tq_threshold_prepared(ctx: int, pq: "PreparedQuery", stream=None) -> None:
    _check(_lib.tq_threshold(ctx, pq.ptrs, pq.n, pq.r_bits, pq.theta, pq.out, _stream(stream)), "tq_threshold")


class BatchQueries:
    """Host-side tq_query array plus the pointer arrays and truth tables it
    points to (kept alive until submission has copied them)."""

    @classmethod
    def from_prepared(cls, prepared):
        self = cls.__new__(cls)
        self.keep = list(prepared)
        self.arr = (TqQuery * max(1, len(prepared)))()
        size = ctypes.sizeof(TqQuery)
        base = ctypes.addressof(self.arr)
        for i, pq in enumerate(prepared):
            ctypes.memmove(base + i * size, ctypes.addressof(pq.rec), size)
        self.count = len(prepared)
        return self

    def __init__(self, specs):
        """specs: list of dicts with keys r_bits, out, theta or truth, and
        either inputs (dense device inputs) or bitmaps (registered inputs);
        optional tag, variant (default TQ_VARIANT_CSA), out_cap and out_len
        (compressed result)."""
        self.keep = []
        self.arr = (TqQuery * max(1, len(specs)))()
        for i, sp in enumerate(specs):
            _fill_query(self.arr[i], self.keep, sp["r_bits"], sp["out"], sp.get("theta"), sp.get("truth"),
                        sp.get("tag", i), inputs=sp.get("inputs"), bitmaps=sp.get("bitmaps"),
                        variant=sp.get("variant", 0), out_cap=sp.get("out_cap", 0), out_len=sp.get("out_len"))
        self.count = len(specs)


def tq_batch_submit(ctx: int, queries: "BatchQueries", flags: int = 0, stream=None) -> int:
    """Returns the batch handle; raises TQError (status TQ_EBUSY when no slot is free)."""
    h = _P()
    _check(_lib.tq_batch_submit(ctx, queries.arr, queries.count, flags, _stream(stream), ctypes.byref(h)),
           "tq_batch_submit")
    return h.value


def raw_batch_submit(ctx: int, queries: "BatchQueries", flags: int = 0, stream=None):
    """Unchecked submission: (status, handle)."""
    h = _P()
    st = _lib.tq_batch_submit(ctx, queries.arr, queries.count, flags, _stream(stream), ctypes.byref(h))
    return st, h.value


def tq_batch_tune(ctx: int, queries: "BatchQueries", stream=None):
    """Time the batch under each candidate schedule; returns (items_per_wave, min_item_work) kept."""
    a, m = _U32(), _U32()
    _check(_lib.tq_batch_tune(ctx, queries.arr, queries.count, _stream(stream), ctypes.byref(a), ctypes.byref(m)),
           "tq_batch_tune")
    return a.value, m.value


def tq_batch_set_schedule(ctx: int, items_per_wave: int, min_item_work: int) -> int:
    return _lib.tq_batch_set_schedule(ctx, items_per_wave, min_item_work)


def tq_tune_export(ctx: int) -> str:
    n = ctypes.c_size_t()
    _check(_lib.tq_tune_export(ctx, None, 0, ctypes.byref(n)), "tq_tune_export")
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(_lib.tq_tune_export(ctx, buf, n.value + 1, ctypes.byref(n)), "tq_tune_export")
    return buf.value.decode()


def tq_tune_import(ctx: int, text: str) -> None:
    _check(_lib.tq_tune_import(ctx, text.encode()), "tq_tune_import")


def raw_tune_import(ctx: int, text: str) -> int:
    return _lib.tq_tune_import(ctx, text.encode())


def tq_tune_clear(ctx: int) -> None:
    _check(_lib.tq_tune_clear(ctx), "tq_tune_clear")


def tq_batch_poll(batch: int) -> int:
    d = _U32()
    _check(_lib.tq_batch_poll(batch, ctypes.byref(d)), "tq_batch_poll")
    return d.value


def tq_batch_wait(batch: int) -> None:
    _check(_lib.tq_batch_wait(batch), "tq_batch_wait")


def raw_batch_wait(batch: int) -> int:
    """Status of tq_batch_wait (the first query that did not complete with TQ_OK)."""
    return _lib.tq_batch_wait(batch)


def tq_batch_cancel(batch: int) -> None:
    _check(_lib.tq_batch_cancel(batch), "tq_batch_cancel")


RECORD_DTYPE = [("user_tag", "<u8"), ("status", "<i4"), ("done", "<u4"), ("t_start_ns", "<u8"),
                ("t_end_ns", "<u8"), ("variant", "<u4"), ("pad", "<u4")]


def tq_batch_records(batch: int, count: int):
    """Per-query records as a numpy structured array (fields of tq_query_record)."""
    import numpy as np
    arr = (TqQueryRecord * max(1, count))()
    _check(_lib.tq_batch_records(batch, arr), "tq_batch_records")
    return np.frombuffer(arr, dtype=np.dtype(RECORD_DTYPE), count=count).copy()


def tq_batch_release(batch: int) -> None:
    _check(_lib.tq_batch_release(batch), "tq_batch_release")


# --------------------------------------------------------- variants, selector
TQ_SEL_FEATURES = 8
TQ_SEL_VARIANTS = 4
TQ_SEL_PARAMS = 4996
TQ_VARIANT_CSA, TQ_VARIANT_COUNTER, TQ_VARIANT_RLE, TQ_VARIANT_HYBRID = 0, 1, 2, 3
VARIANT_NAMES = ("csa", "counter", "rle", "hybrid")
TQ_AUTO_FALLBACK = 1
TQ_AUTO_RETIME = 2
TQ_AUTO_CHOSE_BY_TIMING = 0x100
TQ_AUTO_CHOSE_BY_CACHE = 0x200


class TqBitmap(ctypes.Structure):
    _fields_ = [("dense", _U64), ("rle", TqRle), ("ones", _U64), ("runs", _U64)]


def bitmap_array(bitmaps):
    """bitmaps: sequence of dicts with keys dense (tensor/addr or None),
    rle ((words, n_words, index) or None), ones, runs."""
    arr = (TqBitmap * max(1, len(bitmaps)))()
    for i, b in enumerate(bitmaps):
        arr[i].dense = 0 if b.get("dense") is None else _ptr(b["dense"])
        if b.get("rle") is not None:
            w, nw, idx = b["rle"]
            arr[i].rle.words = _ptr(w)
            arr[i].rle.n_words = int(nw)
            arr[i].rle.index = 0 if idx is None else _ptr(idx)
        arr[i].ones = int(b["ones"])
        arr[i].runs = int(b["runs"])
    return arr


BITMAP_DTYPE = [("dense", "<u8"), ("rle_words", "<u8"), ("rle_n_words", "<u8"), ("rle_index", "<u8"),
                ("ones", "<u8"), ("runs", "<u8")]


def bitmap_table(dense_addrs, rle_addrs, rle_lens, index_addrs, ones, runs):
    """numpy table of registered bitmaps laid out as tq_bitmap (address 0 =
    absent form); rows are picked for a query with bitmap_rows."""
    import numpy as np
    t = np.zeros(len(ones), dtype=np.dtype(BITMAP_DTYPE))
    t["dense"], t["rle_words"], t["rle_n_words"] = dense_addrs, rle_addrs, rle_lens
    t["rle_index"], t["ones"], t["runs"] = index_addrs, ones, runs
    return t


def bitmap_rows(table, members):
    """ctypes tq_bitmap array of the given rows of a bitmap_table."""
    import numpy as np
    sub = np.ascontiguousarray(table[np.asarray(members)])
    arr = (TqBitmap * max(1, len(sub)))()
    ctypes.memmove(ctypes.addressof(arr), sub.ctypes.data, sub.nbytes)
    return arr


def tq_bitmap_stats(ctx: int, dense, r_bits: int, ones_out, runs_out, stream=None) -> None:
    _check(_lib.tq_bitmap_stats(ctx, _ptr(dense), r_bits, _ptr(ones_out), _ptr(runs_out), _stream(stream)),
           "tq_bitmap_stats")


def tq_query_features(bitmaps, r_bits: int, theta: int):
    """Host computation; bitmaps as for bitmap_array (or a prebuilt array with n)."""
    import numpy as np
    arr, n = (bitmaps if isinstance(bitmaps, tuple) else (bitmap_array(bitmaps), len(bitmaps)))
    out = (ctypes.c_float * TQ_SEL_FEATURES)()
    _check(_lib.tq_query_features(arr, n, r_bits, theta, out), "tq_query_features")
    return np.array(out[:], dtype=np.float32)


def tq_threshold_variant(ctx: int, bitmaps, r_bits: int, theta: int, variant: int, out, stream=None) -> None:
    arr, n = (bitmaps if isinstance(bitmaps, tuple) else (bitmap_array(bitmaps), len(bitmaps)))
    _check(_lib.tq_threshold_variant(ctx, arr, n, r_bits, theta, variant, _ptr(out), _stream(stream)),
           "tq_threshold_variant")


def _f32(a):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return a, a.ctypes.data


def tq_selector_param_count() -> int:
    return int(_lib.tq_selector_param_count())


def tq_selector_set(ctx: int, params, mean, std, lo, hi, margin: float) -> None:
    keep = [_f32(a) for a in (params, mean, std, lo, hi)]
    _check(_lib.tq_selector_set(ctx, *[k[1] for k in keep], float(margin)), "tq_selector_set")


def tq_selector_predict(ctx: int, features):
    import numpy as np
    f, fp = _f32(features)
    out = np.zeros(TQ_SEL_VARIANTS, dtype=np.float32)
    _check(_lib.tq_selector_predict(ctx, fp, out.ctypes.data), "tq_selector_predict")
    return out


def tq_threshold_auto(ctx: int, bitmaps, r_bits: int, theta: int, out, flags: int = 0, stream=None) -> int:
    """Returns the chosen variant (with TQ_AUTO_CHOSE_BY_TIMING set if timed)."""
    arr, n = (bitmaps if isinstance(bitmaps, tuple) else (bitmap_array(bitmaps), len(bitmaps)))
    chosen = _U32()
    _check(_lib.tq_threshold_auto(ctx, arr, n, r_bits, theta, _ptr(out), flags, ctypes.byref(chosen),
                                  _stream(stream)), "tq_threshold_auto")
    return chosen.value


def tq_mlp_forward(ctx: int, params, x, batch: int, y, stream=None) -> None:
    _check(_lib.tq_mlp_forward(ctx, _ptr(params), _ptr(x), batch, _ptr(y), _stream(stream)), "tq_mlp_forward")


def tq_mlp_grad(ctx: int, params, x, t, mask, batch: int, mask_count: float, y, grad, loss, stream=None) -> None:
    _check(_lib.tq_mlp_grad(ctx, _ptr(params), _ptr(x), _ptr(t), 0 if mask is None else _ptr(mask), batch,
                            float(mask_count), 0 if y is None else _ptr(y), _ptr(grad),
                            0 if loss is None else _ptr(loss), _stream(stream)), "tq_mlp_grad")


def tq_mlp_adam(ctx: int, params, grad, m, v, count: int, lr: float, beta1: float, beta2: float, eps: float,
                step: int, stream=None) -> None:
    _check(_lib.tq_mlp_adam(ctx, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), count, lr, beta1, beta2, eps, step,
                            _stream(stream)), "tq_mlp_adam")


class Context:
    """Owns a tq context; thin convenience wrapper over the functions above."""

    def __init__(self, device: int = 0):
        self.handle = tq_create(device)

    def close(self):
        if self.handle:
            tq_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def threshold(self, inputs, r_bits, theta, out, stream=None):
        tq_threshold(self.handle, inputs, r_bits, theta, out, stream)

    def symmetric(self, inputs, r_bits, truth, out, stream=None):
        tq_symmetric(self.handle, inputs, r_bits, truth, out, stream)

    def check(self, stream=None) -> int:
        return tq_ctx_check(self.handle, stream)
