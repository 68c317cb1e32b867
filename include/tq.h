/*
 * tq — threshold and symmetric queries over bitmaps on AMD Instinct MI355X.
 *
 * C ABI of libtq.so.  The operations follow the problem statement of Kaser &
 * Lemire, "Threshold and Symmetric Functions over Bitmaps" (TR-14-001):
 *
 *   Given N bitmaps B_1..B_N over positions 0..r-1 and a threshold T, the
 *   T-threshold bitmap has bit p set iff at least T of the inputs have bit p
 *   set (Introduction, "Formulation"; section 2.3).  A symmetric function is
 *   any map f from the per-position count c in [0, N] to {0, 1} (sections 2.2
 *   and 4.2); bit p of its result is f(c(p)).
 *
 * Conventions shared by every call below.
 *
 *   Bitmap layout (section 2.1, uncompressed bitmaps): a bitmap of r bits is
 *   ceil(r/64) little-endian uint64 words in device memory; position p is bit
 *   (p mod 64) of word p div 64.  Input bits at positions >= r are ignored;
 *   output bits at positions >= r are written as zero.  Input words must be
 *   8-byte aligned; 16-byte alignment of every input and of the output lets
 *   the library use 16-byte loads.
 *
 *   Inputs may repeat (the same pointer several times counts several times:
 *   integer weights by replication, section 2.3).  The output must not
 *   overlap any input.
 *
 *   Pointer arrays (`ptrs`) are HOST arrays of N DEVICE pointers.  The
 *   library copies them (and truth tables) at call time; the caller may reuse
 *   or free its host arrays as soon as the call returns.  Device buffers are
 *   owned by the caller and must stay valid until the work queued on
 *   `stream` has completed.  The library never frees or retains caller
 *   memory.
 *
 *   Every call is asynchronous on `stream` (a hipStream_t; NULL is the
 *   default stream).  Argument errors are detected on the host and returned
 *   immediately, with nothing queued.  Errors that only the device can see
 *   (a malformed compressed stream, an output capacity that is too small) are
 *   recorded in the context's status word and returned by tq_ctx_check.
 *
 *   A context is not thread-safe: use one per host thread, or lock around it.
 *
 *   Status codes are the negative values of tq_status; no call throws.
 */
#ifndef TQ_H
#define TQ_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TQ_API_VERSION 2

/* Largest N accepted by the dense calls (the in-register counter has at most
 * 16 bit planes). */
#define TQ_MAX_INPUTS 65535u

typedef enum tq_status {
  TQ_OK = 0,
  TQ_EINVAL = -1,     /* bad argument: NULL pointer, N == 0, N too large, misaligned or overlapping buffers */
  TQ_ENOMEM = -2,     /* device or pinned host allocation failed */
  TQ_EFORMAT = -3,    /* malformed run-length stream (device-detected) */
  TQ_ECAPACITY = -4,  /* output capacity too small; the required length is reported */
  TQ_EDEVICE = -5,    /* a HIP runtime call failed */
  TQ_EBUSY = -6,      /* admission refused: the batch ring or workspace is full, retry later */
  TQ_ENOTSUP = -7,    /* the request is valid but not supported by this library */
  TQ_ECANCELED = -8,  /* batched query not completed: its batch was cancelled (tq_batch_cancel) */
  TQ_ETIMEDOUT = -9   /* batched query not completed: its batch passed its deadline */
} tq_status;

typedef struct tq_ctx tq_ctx;

/* Create a context on HIP device `device` (the device is made current for
 * the call).  *out receives the context, or NULL on failure. */
tq_status tq_create(tq_ctx** out, int device);

/* Destroy a context: waits for the work the context still tracks, then frees
 * its device workspace and pinned staging memory.  NULL is accepted. */
tq_status tq_destroy(tq_ctx* ctx);

/* Static, human-readable name of a status code. */
const char* tq_status_string(int status);

/* Context options. */
#define TQ_OPTION_PRUNE 1  /* value 1 (default): threshold queries, plain and weighted, stop reading
                              inputs for a word once each of its positions is decided, i.e. its
                              (weighted) count already reaches theta or cannot reach it with the
                              remaining inputs (the skipping argument of section 1, "Lower Bound").
                              Results are identical either way; 0 reads every input word. */
#define TQ_OPTION_RLE_TILES 2  /* tiles of TQ_RLE_INDEX_STRIDE words that one workgroup of a query over
                                  RLE inputs walks in a row, each input read front to back across
                                  them; 0 (default) picks one range per resident workgroup.  Any value
                                  gives the same results; values outside [0, 2^20] are TQ_EINVAL. */

#define TQ_OPTION_LOOPED 5  /* value 1 (default): dense thresholds with theta <= 3 use saturating
                              counters (Looped, section 4.5), and theta >= N - 2 the same on the
                              complemented inputs (complement identity, section 2.3, corrected
                              form), testing every 8 inputs whether all positions are decided;
                              0: always the carry-save counter.  Results are identical. */
#define TQ_OPTION_RLE_COUNTERS 4  /* column counters of queries over RLE inputs: 1 = bit planes (a
                                     tile whose columns the fills decide reads no literal word), 2 =
                                     SWAR 16-bit counts (every literal word added once, in the first
                                     pass, without waiting on LDS), 0 (default) = bit planes, or
                                     the tuned choice.  Any value gives the same results. */
#define TQ_OPTION_AUTOTUNE 3  /* value 1: the first dense or compressed-input query of each shape
                                 class (counter width, log2 N, log2 words, epilogue, pruned theta's
                                 eighth, alignment) times every launch shape of its kernel on the
                                 caller's stream, synchronising it once, and caches the fastest in
                                 the context for later queries of the class (skipped while the
                                 stream is being captured into a graph).  0 (default): fixed
                                 shape rules.  Results are identical either way. */

#define TQ_OPTION_BATCH_BYTES 6  /* admission limit of batches (default 2^30): the device bytes that the
                                    batches of the context not yet released may hold together (packed
                                    descriptors, pointer arrays and tables, per-query records and
                                    counters, and the workspace of compressed inputs and compressed
                                    outputs); value >= 1 */
#define TQ_OPTION_BATCH_DEADLINE_US 7  /* deadline of later batches in microseconds after the batch
                                         starts on the device (0, the default: none); see
                                         tq_batch_submit.  Value in [0, 2^40] */

#define TQ_OPTION_SPLIT 8  /* value 1 (default): dense queries over bitmaps too short to fill the device
                              split their inputs over workgroups (see tq_threshold); 0: never.
                              Results are identical either way. */

/* Set a context option; TQ_EINVAL for an unknown option. */
tq_status tq_set_option(tq_ctx* ctx, int option, int64_t value);

/* The tuned launch shapes of a context as text, one shape class per line:
 * "family K log2N log2words epilogue pruned theta8 aligned16 : p0 p1 p2 p3 : us".
 * tq_tune_export writes the text and its terminating NUL into buf (cap
 * bytes; cap == 0 only reports the length in *len, without the NUL;
 * TQ_ECAPACITY if cap is too small).  tq_tune_import adds the lines of a
 * NUL-terminated text to the context (TQ_EINVAL, and nothing added, if any
 * line is malformed or names a shape that does not exist).  tq_tune_clear
 * empties the cache. */
tq_status tq_tune_export(tq_ctx* ctx, char* buf, size_t cap, size_t* len);
tq_status tq_tune_import(tq_ctx* ctx, const char* text);
tq_status tq_tune_clear(tq_ctx* ctx);

/* Wait for `stream`, then return (and clear) the first device-detected error
 * recorded by calls on this context, or TQ_EDEVICE if a HIP call failed. */
tq_status tq_ctx_check(tq_ctx* ctx, hipStream_t stream);

/*
 * Stream capture.  The query calls may be made on a stream that is being
 * captured into a HIP graph; the graph then replays them with the arguments
 * of the capture.  During capture the library copies and allocates nothing:
 * the host arrays a call stages (pointer arrays, truth tables, compressed-
 * input descriptors) must have been staged by an earlier call with the same
 * contents on the same stream, and the context's workspace must already be
 * large enough; otherwise the call returns TQ_EINVAL and records nothing.
 * What a captured call uses is kept for the context's lifetime (staged arrays
 * are never evicted, a workspace a graph refers to is never freed while the
 * context lives), so replays stay valid whatever eager calls run between
 * them.  Replays and other calls that use the workspace must be ordered, as
 * for eager calls.  The autotuner does not time under capture, the
 * selector's timing fallback is skipped, and tq_batch_submit returns
 * TQ_EINVAL (a batch replays its own graph).
 */

/*
 * Threshold query (section 2.3, the function written there as
 * theta(T, {B_1..B_N})):
 *   d_out bit p = [ #{ j : bit p of ptrs[j] is set } >= theta ]   for p < r_bits,
 *   d_out bit p = 0                                                for p >= r_bits.
 * ptrs: host array of n device pointers, each to ceil(r_bits/64) words.
 * n in [1, TQ_MAX_INPUTS].  theta may be any value: theta == 0 gives all ones
 * on [0, r_bits) and theta > n gives all zeros.  r_bits == 0 writes nothing.
 * d_out: ceil(r_bits/64) device words, overwritten.
 * Bitmaps too short to fill the device with 64-word column groups (fewer
 * groups, ceil(r_bits/4096), than compute units) with at least 256 inputs
 * and 4 MiB of input words are counted in parts of at least 32 inputs on
 * separate workgroups (TQ_OPTION_SPLIT), whose partial counts (adding binary
 * counts, section 4.4.2) go through the context's workspace: such calls on
 * one context must be ordered (one stream, or synchronised by the caller), as
 * the compressed-input calls.  The same holds for tq_symmetric.
 */
tq_status tq_threshold(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits,
                       uint32_t theta, uint64_t* d_out, hipStream_t stream);

/*
 * Symmetric query (section 2.2; counter methods take any map [0, N] -> {0,1},
 * section 4.2):
 *   d_out bit p = f(count(p)) for p < r_bits, 0 beyond.
 * h_truth: HOST array of ceil((n+1)/64) words; bit c (bit c mod 64 of word
 * c div 64) is f(c) for c in [0, n].  Bits above n are ignored.  Examples:
 * parity (f(c) = c mod 2), the interval query 2 <= c <= 10, the delta
 * function c == k, majority (c >= ceil(n/2)).
 * Other arguments as for tq_threshold.
 */
tq_status tq_symmetric(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits,
                       const uint64_t* h_truth, uint64_t* d_out, hipStream_t stream);

/*
 * Weighted threshold query (section 2.3: inputs may carry positive integer
 * weights, there realised by replicating input j weights[j] times):
 *   d_out bit p = [ sum_j weights[j] * bit p of ptrs[j] >= theta ]  for p < r_bits.
 * Each input is read at most once whatever its weight (heaviest first; with
 * TQ_OPTION_PRUNE a word stops being read once each of its positions is
 * decided).  h_weights: HOST array of n
 * uint32 weights (0 allowed: the input is ignored); their sum must not exceed
 * 2^32 - 1 (else TQ_EINVAL).  theta == 0 gives all ones on [0, r_bits), theta
 * above the sum gives zeros.  Other arguments and errors as for tq_threshold.
 */
tq_status tq_threshold_weighted(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, const uint32_t* h_weights,
                                uint64_t r_bits, uint64_t theta, uint64_t* d_out, hipStream_t stream);

/*
 * Fused consumers of the result (the result of a threshold or symmetric
 * query is again a bitmap, to be combined with other criteria by AND and
 * friends or counted: abstract and introduction).  In the same pass:
 *   R = T_theta(inputs)  (or f(count) for the symmetric form)  AND  filter,
 *   d_out    = R                               (nullable: R is not stored),
 *   *d_count = number of positions p < r_bits with bit p of R set
 *                                              (nullable; one device uint64).
 * d_filter: ceil(r_bits/64) device words, or NULL for no filter; it may be
 * d_out itself (in place) but must not overlap it otherwise; it may alias
 * the inputs.  At least one of d_out and d_count is given; d_count must not
 * lie inside d_out.  The count uses the context's workspace (one uint32 per
 * 64 output words): calls on one context that use workspace must be ordered.
 * Other arguments, special cases and errors as for tq_threshold / tq_symmetric;
 * r_bits == 0 sets *d_count = 0.
 */
tq_status tq_threshold_fused(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits,
                             uint32_t theta, const uint64_t* d_filter, uint64_t* d_out, uint64_t* d_count,
                             hipStream_t stream);
tq_status tq_symmetric_fused(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits,
                             const uint64_t* h_truth, const uint64_t* d_filter, uint64_t* d_out,
                             uint64_t* d_count, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc, code that must not allocate while a graph
 * is being captured): the query
 * of tq_threshold_fused, with the same arguments, results and errors, that
 * makes no device or pinned allocation.  Its device scratch (the copy of the
 * pointer array, then one uint32 partial count per 64 output words when
 * d_count is given) is a fixed array of TQ_NOALLOC_SCRATCH_BYTES per device,
 * held until the process ends:
 *   roundup(8 n, 256) + 4 ceil(ceil(r_bits/64) / 64)  <=  TQ_NOALLOC_SCRATCH_BYTES
 * when d_count is given (theta in [1, n]); 4 ceil(ceil(r_bits/64) / 256)
 * bytes when theta is 0 or above n; else TQ_EINVAL and nothing is queued.
 * Without d_count only the pointer array is held, which always fits.  The
 * host pointer array is copied with hipMemcpyAsync on `stream`, which stages
 * pageable memory before it returns (under stream capture the copy becomes a
 * graph node that reads the host array at every replay).  The
 * launch shape is the default one (no autotuning).  Every call on a device
 * shares that device's array: calls that overlap in time on one device (two
 * streams, two contexts, two threads) race; calls on one stream are ordered.
 */
#define TQ_NOALLOC_SCRATCH_BYTES (4u << 20)
tq_status tq_threshold_fused_noalloc(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits,
                                     uint32_t theta, const uint64_t* d_filter, uint64_t* d_out,
                                     uint64_t* d_count, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Run-length-encoded bitmaps (section 2.1, word-aligned RLE with markers that
 * carry both a fill-run length and a dirty-word count, as in EWAH).
 *
 * Stream layout: a sequence of 64-bit marker words, each followed by its
 * literal words.  Marker bit 0 = fill value, bits 1..32 = number of fill
 * words, bits 33..63 = number of literal words that follow.  The fill and
 * literal counts of all markers add up to exactly ceil(r/64) words.  Any
 * such stream is accepted as input; outputs are canonical: a marker starts at
 * word 0 and at every clean word (all zeros or all ones) whose predecessor is
 * dirty or the other fill, covers the maximal run of equal clean words there
 * and then the maximal run of dirty words; clean words are never literals.
 * The tail word is encoded with its bits >= r cleared.
 *
 * Checkpoint index: for every TQ_RLE_INDEX_STRIDE uncompressed words, two
 * uint64: the stream offset of the marker whose run covers word
 * c * TQ_RLE_INDEX_STRIDE, and the uncompressed word at which that marker's
 * run starts.  tq_rle_index_words(r) words in device memory.  It makes tiles
 * of the bitmap directly addressable (the paper notes RLE offers no random
 * access, section 1 "Lower Bound"; auxiliary skip structures, section 4.3).
 * ---------------------------------------------------------------------- */
#define TQ_RLE_INDEX_STRIDE 512
/* Largest N accepted by the compressed-input calls. */
#define TQ_RLE_MAX_INPUTS 8192u
/* The threshold calls over compressed inputs (tq_threshold_rle,
 * tq_threshold_rle_dense, tq_threshold_hybrid) accept bitmaps of fewer than
 * 2^31 words (r_bits < 2^37) and streams of at most 2^32 - 1024 words;
 * larger ones are TQ_EINVAL. */

typedef struct tq_rle {
  const uint64_t* words; /* device stream */
  uint64_t n_words;      /* stream length in words */
  const uint64_t* index; /* device checkpoint index, or NULL (then built into the context's workspace) */
} tq_rle;

/* Largest canonical encoding of an r-bit bitmap: ceil(r/64) + 1 words. */
uint64_t tq_rle_max_words(uint64_t r_bits);

/* Words of a checkpoint index: 2 * ceil(ceil(r/64) / TQ_RLE_INDEX_STRIDE). */
uint64_t tq_rle_index_words(uint64_t r_bits);

/*
 * Canonical encoding of the dense bitmap d_dense (ceil(r/64) words; bits
 * >= r ignored) into d_out (capacity out_cap words).  The encoded length is
 * written to *d_out_len (a device uint64).  If it exceeds out_cap, nothing
 * beyond out_cap is written and TQ_ECAPACITY is recorded for tq_ctx_check
 * (the required length is still in *d_out_len).  d_index (nullable) receives
 * the checkpoint index of the encoded stream.  Uses the context's workspace:
 * calls on one context that use workspace must be ordered (one stream, or
 * synchronised by the caller).
 */
tq_status tq_rle_encode(tq_ctx* ctx, const uint64_t* d_dense, uint64_t r_bits, uint64_t* d_out,
                        uint64_t out_cap, uint64_t* d_out_len, uint64_t* d_index, hipStream_t stream);

/* Build the checkpoint index of a stream (validating it: TQ_EFORMAT is
 * recorded if the stream does not cover exactly ceil(r/64) words). */
tq_status tq_rle_build_index(tq_ctx* ctx, const uint64_t* d_words, uint64_t n_words, uint64_t r_bits,
                             uint64_t* d_index, hipStream_t stream);

/* Decode one stream into ceil(r/64) dense words (bits >= r zero). */
tq_status tq_rle_decode(tq_ctx* ctx, const tq_rle* input, uint64_t r_bits, uint64_t* d_dense,
                        hipStream_t stream);

/*
 * Threshold over compressed inputs (section 2.3 for the function; section
 * 4.1, RBMrg, for the run cases: where k inputs are 1-fills, theta - k <= 0
 * gives ones, theta - k greater than the number of dirty inputs gives zeros,
 * and otherwise a (theta - k)-threshold over the dirty words decides).
 * inputs: HOST array of n tq_rle descriptors (device streams).  The result is
 * written as a canonical stream into d_out (capacity out_cap_words), its
 * length into *d_out_len (device).  TQ_ECAPACITY as for tq_rle_encode;
 * TQ_EFORMAT is recorded if an input is malformed.  n in [1,
 * TQ_RLE_MAX_INPUTS].  Uses the context's workspace (see tq_rle_encode).
 */
tq_status tq_threshold_rle(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits, uint32_t theta,
                           uint64_t* d_out, uint64_t out_cap_words, uint64_t* d_out_len, hipStream_t stream);

/* Same query with the result written as a dense bitmap (ceil(r/64) words). */
tq_status tq_threshold_rle_dense(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits,
                                 uint32_t theta, uint64_t* d_out, hipStream_t stream);

/*
 * Hybrid query: n_rle compressed inputs plus n_dense uncompressed inputs
 * (host array of device pointers), each input stored in whichever form is
 * smaller; the threshold counts all n_rle + n_dense of them.  Dense output.
 * n_rle + n_dense in [1, TQ_RLE_MAX_INPUTS].
 */
tq_status tq_threshold_hybrid(tq_ctx* ctx, const tq_rle* rle_inputs, uint32_t n_rle,
                              const uint64_t* const* dense_ptrs, uint32_t n_dense, uint64_t r_bits,
                              uint32_t theta, uint64_t* d_out, hipStream_t stream);

/*
 * Symmetric functions over compressed inputs (section 2.2 for the functions;
 * the run cases of section 4.1 generalised: where k inputs are 1-fills and d
 * are dirty, the count lies in [k, k+d], so f constant on that range decides
 * the word from the markers alone, and otherwise f is evaluated on k plus the
 * counted dirty bits).  h_truth as for tq_symmetric (n + 1 entries); other
 * arguments, outputs and errors as for the threshold forms above.
 */
tq_status tq_symmetric_rle(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits, const uint64_t* h_truth,
                           uint64_t* d_out, uint64_t out_cap_words, uint64_t* d_out_len, hipStream_t stream);
tq_status tq_symmetric_rle_dense(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits,
                                 const uint64_t* h_truth, uint64_t* d_out, hipStream_t stream);
tq_status tq_symmetric_hybrid(tq_ctx* ctx, const tq_rle* rle_inputs, uint32_t n_rle,
                              const uint64_t* const* dense_ptrs, uint32_t n_dense, uint64_t r_bits,
                              const uint64_t* h_truth, uint64_t* d_out, hipStream_t stream);

/*
 * Fused consumers over compressed inputs (the result is again a bitmap to be
 * combined or counted: abstract and introduction), as tq_threshold_fused /
 * tq_symmetric_fused: R = f(inputs) AND filter; d_out = R (dense, nullable),
 * *d_count = |R| below r_bits (nullable).  The filter is dense, ceil(r/64)
 * words (NULL: none), and may be d_out itself.  The count uses the context's
 * workspace (one uint32 per wave of each TQ_RLE_INDEX_STRIDE-word tile, and
 * the indexes the inputs lack).  Inputs and errors as tq_threshold_rle_dense.
 */
tq_status tq_threshold_rle_fused(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits, uint32_t theta,
                                 const uint64_t* d_filter, uint64_t* d_out, uint64_t* d_count, hipStream_t stream);
tq_status tq_symmetric_rle_fused(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits,
                                 const uint64_t* h_truth, const uint64_t* d_filter, uint64_t* d_out,
                                 uint64_t* d_count, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched queries: many threshold / symmetric queries of uneven N, r and
 * theta served by one persistent kernel launch, replayed from a graph.
 * ---------------------------------------------------------------------- */
typedef enum tq_query_kind { TQ_QUERY_THRESHOLD = 0, TQ_QUERY_SYMMETRIC = 1 } tq_query_kind;

/* tq_query.variant: let the installed selector choose (see tq_threshold_auto). */
#define TQ_VARIANT_AUTO 0xFFFFFFFFu

struct tq_bitmap;

typedef struct tq_query {
  uint32_t kind;                /* tq_query_kind */
  uint32_t n;                   /* number of inputs, [1, TQ_MAX_INPUTS]; [1, TQ_RLE_MAX_INPUTS] when
                                   any input is read in compressed form */
  const uint64_t* const* ptrs;  /* HOST array of n dense device inputs, or NULL when `inputs` is given */
  uint64_t r_bits;
  uint32_t theta;               /* TQ_QUERY_THRESHOLD */
  uint32_t variant;             /* tq_variant, or TQ_VARIANT_AUTO (only with `inputs`); with `ptrs`
                                   TQ_VARIANT_CSA (0) or TQ_VARIANT_COUNTER */
  const uint64_t* h_truth;      /* TQ_QUERY_SYMMETRIC: host truth table as for tq_symmetric (copied) */
  uint64_t* d_out;              /* dense result (ceil(r_bits/64) words) when out_cap == 0, else the
                                   canonical compressed result (at most out_cap words) */
  uint64_t user_tag;            /* returned in the query's record */
  const struct tq_bitmap* inputs;  /* HOST array of n registered inputs (either or both forms, with
                                      metadata), or NULL when `ptrs` is given (copied) */
  uint64_t out_cap;             /* 0: dense result; > 0: compressed result of capacity out_cap words */
  uint64_t* d_out_len;          /* out_cap > 0: device uint64 receiving the compressed length */
} tq_query;

typedef struct tq_query_record {
  uint64_t user_tag;
  int32_t status;               /* TQ_OK once done; see tq_batch_records */
  uint32_t done;                /* 1 once the query's output is complete and visible */
  uint64_t t_start_ns;          /* device clock when the first work of the query started */
  uint64_t t_end_ns;            /* device clock when its last work finished */
  uint32_t variant;             /* tq_variant that ran (the selector's choice for TQ_VARIANT_AUTO) */
  uint32_t pad;
} tq_query_record;

typedef struct tq_batch tq_batch;

/* Flags of tq_batch_submit. */
#define TQ_BATCH_NO_GRAPH 1u    /* launch directly instead of replaying the slot's graph (batches of
                                   fewer than 64 queries are always launched directly).  A graph
                                   replay and a direct launch cost the host different times, which
                                   shows in the latency of small batches: the caller picks. */

/* Largest batch: queries and total pointer entries (sum of n). */
#define TQ_BATCH_MAX_QUERIES 8192u
#define TQ_BATCH_MAX_POINTERS 2097152u
#define TQ_BATCH_MAX_TABLE_BYTES 1048576u
/* Batches not yet released that a context holds at once. */
#define TQ_BATCH_MAX_INFLIGHT 16u

/*
 * Submit `count` queries as one batch on `stream`.  Each query has the
 * semantics of tq_threshold or tq_symmetric (the threshold and symmetric
 * functions of sections 2.2-2.3); results are bit-identical to those calls.
 *
 * Inputs: either `ptrs` (dense inputs) or `inputs` (registered bitmaps as
 * for tq_threshold_variant, each with its dense and/or compressed form and
 * its cardinality and run count).  The variant reads them as in
 * tq_threshold_variant: TQ_VARIANT_CSA (with TQ_OPTION_LOOPED, thresholds
 * within 3 of either end by saturating counters; with `inputs` and pruning,
 * inputs read by registered cardinality), TQ_VARIANT_COUNTER (thresholds
 * only), TQ_VARIANT_RLE, TQ_VARIANT_HYBRID (compressed and hybrid reads:
 * thresholds only), or TQ_VARIANT_AUTO: the installed selector's prediction
 * among the variants the inputs allow (features outside its training range
 * are clamped into it; nothing is timed), the carry-save counter without a
 * selector.  A symmetric query with TQ_VARIANT_AUTO runs the carry-save
 * counter (TQ_ENOTSUP if an input has no dense form).  An input lacking the
 * form its variant reads is TQ_EINVAL.
 *
 * Execution: dense-input queries (carry-save, Looped and counter variants)
 * are split into work items of similar byte counts that one persistent
 * kernel serves from one queue; queries over compressed inputs, and the
 * encoding of compressed results, run after it on the stream as their own
 * launches (tile kernel, encoder), with indexes the inputs lack built by one
 * launch per query.  A compressed result (out_cap > 0) behaves as in
 * tq_threshold_rle: its length goes to *d_out_len, and a capacity below it is
 * the query's TQ_ECAPACITY (in its record) with the required length still
 * written.
 *
 * Admission: the device bytes the batch holds (packed descriptors and copies
 * of the pointer arrays and truth tables, per-query records and counters,
 * and the workspace of compressed inputs and results) are counted against
 * TQ_OPTION_BATCH_BYTES together with the batches of the context not yet
 * released; when they do not fit, or TQ_BATCH_MAX_INFLIGHT batches are held,
 * the call returns TQ_EBUSY and queues nothing (retry after releasing a
 * batch).  A batch that alone exceeds the limit is TQ_EINVAL.
 *
 * Deadline and cancellation: the persistent kernel takes no new work item
 * once the batch is cancelled (tq_batch_cancel) or, with
 * TQ_OPTION_BATCH_DEADLINE_US set, once that many microseconds have passed
 * since the batch's kernel started; work items already taken finish.
 * Queries left incomplete are reported TQ_ECANCELED / TQ_ETIMEDOUT and
 * their outputs are undefined.  Queries over compressed inputs, which run
 * after the persistent kernel, are not stopped.
 *
 * count in [1, TQ_BATCH_MAX_QUERIES]; sum of n at most TQ_BATCH_MAX_POINTERS.
 * A symmetric function with more than 8 runs of ones and of zeros in f is
 * evaluated through a lookup table of 2^K bits (K the counter width,
 * bit_length(n)); the tables of one batch may take at most
 * TQ_BATCH_MAX_TABLE_BYTES (each rounded up to 8 bytes), else TQ_EINVAL.
 * All host arrays are copied; *out receives the batch.
 */
tq_status tq_batch_submit(tq_ctx* ctx, const tq_query* queries, uint32_t count, uint32_t flags,
                          hipStream_t stream, tq_batch** out);

/* Number of queries of the batch whose output is complete (non-blocking;
 * completion flags are written by the device into pinned host memory). */
tq_status tq_batch_poll(tq_batch* batch, uint32_t* ndone);

/* Block until the batch's work has finished.  Returns TQ_OK if every query
 * completed with TQ_OK, else the status of the first query (in submission
 * order) that did not. */
tq_status tq_batch_wait(tq_batch* batch);

/* Stop the batch from taking new work items (see tq_batch_submit); does not
 * wait.  Queries already complete keep their results. */
tq_status tq_batch_cancel(tq_batch* batch);

/* Copy the batch's per-query records (count entries, submission order).
 * status: TQ_OK (done = 1 once complete); TQ_ECAPACITY or TQ_EFORMAT for a
 * compressed result too large or a malformed compressed input (done = 1,
 * the record is final); TQ_ECANCELED / TQ_ETIMEDOUT once the batch has
 * finished without completing the query (done = 0). */
tq_status tq_batch_records(tq_batch* batch, tq_query_record* out);

/* Wait for the batch, free its slot and the handle. */
tq_status tq_batch_release(tq_batch* batch);

/*
 * Word-column schedule of batches: the work of a batch (64-word column groups
 * times inputs) is cut into items so that every wave of the persistent grid
 * gets about `items_per_wave` of them, and no item is smaller than
 * `min_item_work` group-inputs.  tq_batch_tune submits the given batch under
 * each candidate schedule (items per wave 1, 2, 4, 8, 16 x smallest item 4,
 * 16, 64; best of three submissions each, timed with HIP events on `stream`,
 * which it synchronises), keeps the fastest for later submissions on this
 * context and returns it (either out pointer may be NULL).  The queries'
 * outputs are written as by tq_batch_submit.  It needs a free batch slot
 * (TQ_EBUSY otherwise) and a stream that is not being captured (TQ_EINVAL).
 * tq_batch_set_schedule sets a schedule directly (items_per_wave in [1, 64],
 * min_item_work in [1, 4096]); the default is 4 and 16.  Results never
 * depend on the schedule.
 */
tq_status tq_batch_tune(tq_ctx* ctx, const tq_query* queries, uint32_t count, hipStream_t stream,
                        uint32_t* items_per_wave, uint32_t* min_item_work);
tq_status tq_batch_set_schedule(tq_ctx* ctx, uint32_t items_per_wave, uint32_t min_item_work);

/* ------------------------------------------------------------------------
 * Kernel variants and the learned selector.
 *
 * Which threshold algorithm is fastest depends on N, T, the density and the
 * run structure of the inputs (sections 5.7-5.10 and 6).  Four GPU variants
 * compute the same bits (sections 2.3, 4.1, 4.2, 4.4):
 *   TQ_VARIANT_CSA      carry-save vertical counter over dense words
 *   TQ_VARIANT_COUNTER  per-position counters over dense words (ScanCount)
 *   TQ_VARIANT_RLE      run-length tile merge over compressed inputs (RBMrg cases)
 *   TQ_VARIANT_HYBRID   each input read in its smaller form
 * A registered bitmap carries either or both forms plus its cardinality and
 * run count; a small network (8 -> 64 -> 64 -> 4, ReLU, fp32) maps eight
 * features of that metadata to predicted log run times of the variants.
 * ---------------------------------------------------------------------- */
#define TQ_SEL_FEATURES 8
#define TQ_SEL_HIDDEN 64
#define TQ_SEL_VARIANTS 4
/* W1[64][8] b1[64] W2[64][64] b2[64] W3[4][64] b3[4], row-major (out x in) */
#define TQ_SEL_PARAMS 4996

typedef enum tq_variant {
  TQ_VARIANT_CSA = 0,
  TQ_VARIANT_COUNTER = 1,
  TQ_VARIANT_RLE = 2,
  TQ_VARIANT_HYBRID = 3
} tq_variant;

typedef struct tq_bitmap {
  const uint64_t* dense;  /* device words, or NULL when only the compressed form exists */
  tq_rle rle;             /* compressed form; rle.words NULL when absent */
  uint64_t ones;          /* registered cardinality (positions < r that are set) */
  uint64_t runs;          /* registered number of runs of equal bits in [0, r) */
} tq_bitmap;

/* Flags of tq_threshold_auto and bits of its *chosen report. */
#define TQ_AUTO_FALLBACK 1u            /* time every variant when the prediction is uncertain */
#define TQ_AUTO_RETIME 2u              /* with TQ_AUTO_FALLBACK: time again even if a decision is remembered */
#define TQ_AUTO_CHOSE_BY_TIMING 0x100u /* set in *chosen when the fallback timed the variants */
#define TQ_AUTO_CHOSE_BY_CACHE 0x200u  /* set in *chosen when a remembered decision was used */

/* Cardinality and run count of a dense bitmap (metadata registered with it,
 * section 2.1: RunCount).  Both results are device uint64. */
tq_status tq_bitmap_stats(tq_ctx* ctx, const uint64_t* d_dense, uint64_t r_bits, uint64_t* d_ones,
                          uint64_t* d_runs, hipStream_t stream);

/* The eight selector features of a query, from metadata only (host):
 * log2 N, theta/N, log10 mean density, log10 mean ones-run length, standard
 * deviation of log10 density, log2 r, log2 compression ratio, and
 * log2(theta / (1 + expected count)). */
tq_status tq_query_features(const tq_bitmap* inputs, uint32_t n, uint64_t r_bits, uint32_t theta, float* out);

/* Threshold query run by the given variant (dense output, semantics of
 * tq_threshold).  TQ_EINVAL if an input lacks the form the variant reads.
 * With pruning on (TQ_OPTION_PRUNE), TQ_VARIANT_CSA reads the inputs in order
 * of their registered cardinality: densest first when theta is below half
 * the expected count (sum of ones / r_bits), so that positions reach theta
 * sooner, else sparsest first, so that they are written off sooner (section
 * 1, lower bound and skipping).  The result does not depend on the order or
 * on the registered values. */
tq_status tq_threshold_variant(tq_ctx* ctx, const tq_bitmap* inputs, uint32_t n, uint64_t r_bits,
                               uint32_t theta, uint32_t variant, uint64_t* d_out, hipStream_t stream);

uint64_t tq_selector_param_count(void);

/* Install trained weights (TQ_SEL_PARAMS floats, host), the feature
 * normalisation (mean, std) and the feature range seen in training (lo, hi),
 * and the decision margin in predicted log time below which a prediction
 * counts as uncertain. */
tq_status tq_selector_set(tq_ctx* ctx, const float* params, const float* feat_mean, const float* feat_std,
                          const float* feat_lo, const float* feat_hi, float margin);

/* Host inference: predicted log run times of the four variants. */
tq_status tq_selector_predict(tq_ctx* ctx, const float* features, float* predicted);

/* Threshold query with the variant the selector predicts fastest among those
 * the inputs allow.  With TQ_AUTO_FALLBACK, an uncertain prediction (top two
 * within the margin, or features outside the training range) makes the call
 * time every available variant once and keep the fastest; that path
 * synchronises the stream.  The decision is remembered for the query's cell
 * (each feature in quarters of its training standard deviation, and the set
 * of variants the inputs allow; up to 65536 cells, forgotten by
 * tq_selector_set): a later uncertain query of the same cell runs that
 * variant without timing (TQ_AUTO_CHOSE_BY_CACHE) unless TQ_AUTO_RETIME is
 * given.  All variants give the same bits, so a remembered decision changes
 * only the time.  *chosen (nullable) receives the variant. */
tq_status tq_threshold_auto(tq_ctx* ctx, const tq_bitmap* inputs, uint32_t n, uint64_t r_bits, uint32_t theta,
                            uint64_t* d_out, uint32_t flags, uint32_t* chosen, hipStream_t stream);

/* Selector network kernels (device arrays, fp32).  x: batch x 8 features,
 * y: batch x 4 outputs, t: targets, mask (nullable): 0/1 per target; the
 * loss is sum(mask * (y - t)^2) / mask_count.  tq_mlp_grad writes the
 * gradient of the loss w.r.t. the parameters (and the loss, and y if
 * non-NULL); tq_mlp_adam applies one Adam step (step counts from 1). */
tq_status tq_mlp_forward(tq_ctx* ctx, const float* d_params, const float* d_x, uint32_t batch, float* d_y,
                         hipStream_t stream);
tq_status tq_mlp_grad(tq_ctx* ctx, const float* d_params, const float* d_x, const float* d_t, const float* d_mask,
                      uint32_t batch, float mask_count, float* d_y, float* d_grad, float* d_loss,
                      hipStream_t stream);
tq_status tq_mlp_adam(tq_ctx* ctx, float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t count,
                      float lr, float beta1, float beta2, float eps, uint32_t step, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* TQ_H */
