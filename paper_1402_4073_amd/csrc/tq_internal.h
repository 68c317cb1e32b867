// Internal declarations of libtq (host side).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <unordered_map>
#include <functional>
#include <vector>

#include "../../include/tq.h"

namespace tq {

// ---------------------------------------------------------------- epilogue
// How the per-position count c is turned into the output bit.  Compiled on
// the host from the threshold or the truth table, evaluated on the bit
// planes of the count in the kernel.
enum EpiKind : int32_t {
  EPI_THRESH = 0,     // c >= theta (compare against theta - 1)
  EPI_INTERVALS = 1,  // OR of lo_i <= c <= hi_i
  EPI_PARITY = 2,     // c odd
  EPI_TABLE = 3,      // generic: f looked up per bit position from a table
};

constexpr int kMaxIntervals = 8;

struct EpiParams {
  int32_t kind;
  int32_t invert;       // complement the result
  uint32_t theta;       // EPI_THRESH: theta in [1, n]
  int32_t nint;         // EPI_INTERVALS
  uint32_t lo[kMaxIntervals];   // c >= lo   (0 means no lower bound)
  uint32_t hi1[kMaxIntervals];  // c <  hi1  (> n means no upper bound)
  const uint32_t* table;        // EPI_TABLE: bit c of the table is f(c)
  uint32_t table_words;
  uint32_t prune;               // EPI_THRESH: stop loading once every position is decided
};

// Plan of a symmetric function: a constant, or an epilogue.
struct SymPlan {
  bool constant;
  uint64_t const_word;  // all ones or zero when constant
  EpiParams epi;
  std::vector<uint32_t> table;  // EPI_TABLE contents
};

SymPlan plan_threshold(uint32_t n, uint32_t theta);
SymPlan plan_symmetric(uint32_t n, const uint64_t* truth);

// --------------------------------------------------------- dense launches
struct DenseConfig {
  int K;     // bit planes of the counter: the count must fit, count <= n < 2^K
  int wpl;   // 64-bit words per lane (1 or 2)
  int split; // waves per workgroup sharing the same columns (inputs split among them)
  int groups; // column groups per workgroup
};

bool dense_config_valid(const DenseConfig& c);

int dense_planes_for(uint32_t n);

// can_prune: the query is a threshold the kernel may stop reading early for
// (which needs one wave per column group)
DenseConfig choose_dense_config(uint32_t n, uint64_t nwords, bool aligned16, int num_cus, bool can_prune = true);

// Work-items of one launch stay below this: the dispatch packet holds the
// grid size in 32 bits, and a larger launch is silently cut short.  Longer
// bitmaps are processed by several launches over consecutive word ranges.
constexpr uint64_t kMaxLaunchItems = 1ull << 31;

// Consumers fused into the store of a result word: AND with a filter bitmap
// (nullable) and per-column-group popcounts of the stored word (nullable;
// one uint32 per column group, summed afterwards by launch_count_reduce).
struct Sink {
  const uint64_t* filter = nullptr;
  uint32_t* partial = nullptr;     // dense kernels: one count per column group
  uint64_t* partial64 = nullptr;   // tile kernel over compressed inputs: one per wave of each workgroup
};

// Column groups (= partial slots) of a dense launch over nwords words.
uint64_t dense_groups(const DenseConfig& cfg, uint64_t nwords);

hipError_t launch_dense(const DenseConfig& cfg, const uint64_t* const* d_ptrs, uint32_t n,
                        uint64_t nwords, uint64_t tail_mask, uint64_t* d_out,
                        const EpiParams& epi, hipStream_t stream, const Sink& sink = Sink());

hipError_t launch_fill(uint64_t* d_out, uint64_t nwords, uint64_t value, uint64_t tail_mask,
                       hipStream_t stream);

// Inputs split over workgroups (adding binary counts, section 4.4.2): for
// bitmaps too short to fill the device with column groups, `parts` parts of
// `per` inputs each are counted by their own waves into kp-plane partial
// counters in workspace (split_workspace_bytes), which a second kernel adds
// before the epilogue.  parts == 0: not worth it for this shape.
struct SplitPlan {
  uint32_t parts = 0, per = 0;
  int kp = 0;
  uint64_t stride = 0;   // words per partial plane (column groups * 64)
};
SplitPlan plan_split(uint32_t n, uint64_t nwords, int num_cus);
size_t split_workspace_bytes(const SplitPlan& sp);
hipError_t launch_dense_split(const SplitPlan& sp, const uint64_t* const* d_ptrs, uint32_t n, uint64_t nwords,
                              uint64_t tail_mask, uint64_t* d_out, const EpiParams& epi, uint64_t* d_part,
                              hipStream_t stream);

// Saturating counters for theta <= 3, or theta >= n - 2 on the complemented
// inputs (Looped, section 4.5; complement identity, section 2.3).
bool looped_applies(uint32_t n, uint32_t theta, uint32_t* t, bool* comp);
hipError_t launch_looped(const uint64_t* const* d_ptrs, uint32_t n, uint64_t nwords, uint64_t tail_mask,
                         uint32_t theta, bool prune, uint64_t* d_out, hipStream_t stream);

// Weighted threshold: inputs [begin, end) of the (reordered) pointer array
// all carry `weight`.
struct WeightClass {
  uint32_t weight, begin, end, pad;
};
// prune: after each class a lane whose positions are all decided (weighted
// sum already >= theta, or below theta even with every class left) stops.
hipError_t launch_weighted(const uint64_t* const* d_ptrs, const WeightClass* d_classes, uint32_t nclasses,
                           uint32_t max_class, uint64_t nwords, uint64_t tail_mask, uint32_t theta,
                           uint32_t total_weight, bool prune, uint64_t* d_out, hipStream_t stream);

// Constant result with consumers: out = value AND filter (tail cleared),
// partial popcounts per 256-word block (fill_groups(nwords) slots).
uint64_t fill_groups(uint64_t nwords);
hipError_t launch_fill_sink(uint64_t* d_out, uint64_t nwords, uint64_t value, uint64_t tail_mask,
                            const Sink& sink, hipStream_t stream);

// *d_count = sum of partial[0..m)
hipError_t launch_count_reduce(const uint32_t* d_partial, uint64_t m, uint64_t* d_count, hipStream_t stream);
hipError_t launch_count_reduce(const uint64_t* d_partial, uint64_t m, uint64_t* d_count, hipStream_t stream);

// Arguments of the dense calls: n in [1, TQ_MAX_INPUTS], non-null 8-byte
// aligned inputs, an 8-byte aligned output (nullable if out_optional) that
// overlaps no input.  *aligned16: every buffer is 16-byte aligned.
tq_status check_dense_args(const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits, const uint64_t* d_out,
                           bool* aligned16, bool out_optional = false);

// Device address of the fixed scratch array of the allocation-free entry
// point on `device` (set by noalloc_init, which tq_create calls with the
// device current); nullptr before.
tq_status noalloc_init(int device);
void* noalloc_scratch(int device);

// Arguments of the fused-consumer calls: at least one of d_out / d_count,
// 8-byte alignment, a filter equal to d_out or disjoint from it, d_count
// outside d_out.
tq_status check_sink_args(uint64_t r_bits, const uint64_t* d_filter, const uint64_t* d_out,
                          const uint64_t* d_count);

// -------------------------------------------------------------------- RLE
// Device-side description of one compressed input (3 words, staged as a blob).
struct RleDesc {
  const uint64_t* words;
  uint64_t len;
  const uint64_t* index;
};

// Largest stream length accepted by the queries over RLE inputs (bitmaps
// are limited to fewer than 2^31 words): the tile kernel keeps positions in
// 32 bits.
constexpr uint64_t kRleMaxWords = (1ull << 32) - 1024;
// A symmetric function over compressed inputs.  A column with k ones fills
// and d dirty inputs has a count in [k, k + d]; it is decided when f is
// constant there, i.e. when k + d <= run_end[k].
struct RleSym {
  const uint32_t* run_end;  // per count c in [0, n]: last count of the run of equal f values from c
  const uint64_t* f;        // f(c) is bit c of this array, c in [0, n]
  EpiParams epi;            // f(count) on the planes of the full count
  uint32_t tail_from;       // f is constant (tail_value) on [tail_from, n]
  uint32_t tail_value;
};

size_t rle_tile_lds_bytes(int K, bool swar);
// sym == nullptr: threshold theta; otherwise the symmetric function *sym
// (host copy, which picks the kernel), d_sym its copy in device memory (which
// the kernel reads).
// swar: SWAR column counters (every tile in one pass) instead of bit planes.
// sink (filter and/or partial64 set): consumers of each result word (AND
// filter; popcounts into sink.partial64, one slot per wave of each
// workgroup: *slots_used slots, at most rle_tile_partials(nwords)); d_out may
// then be null.
hipError_t launch_rle_tile(const RleDesc* d_descs, uint32_t n_rle, const uint64_t* const* d_dense,
                           uint32_t n_dense, uint64_t nwords, uint64_t tail_mask, uint32_t theta,
                           const RleSym* sym, const RleSym* d_sym, bool swar, int num_cus,
                           uint32_t tiles_per_group, uint64_t* d_out, int* d_status, hipStream_t stream,
                           const Sink& sink = Sink(), uint64_t* slots_used = nullptr);
uint64_t rle_tile_partials(uint64_t nwords);
size_t rle_encode_workspace_bytes(uint64_t nwords);
hipError_t launch_rle_encode(const uint64_t* d_dense, uint64_t nwords, uint64_t tail_mask, uint64_t* d_out,
                             uint64_t cap, uint64_t* d_out_len, uint64_t* d_index, void* workspace,
                             int* d_status, hipStream_t stream);
hipError_t launch_build_index(const uint64_t* d_words, uint64_t len, uint64_t nwords, uint64_t* d_index,
                              int* d_status, hipStream_t stream);
// Validate n compressed inputs over bitmaps of nwords words (nwords below
// 2^31, streams non-empty, aligned and not longer than kRleMaxWords); counts
// those without an index.
tq_status check_rle_inputs(const tq_rle* inputs, uint32_t n, uint64_t nwords, uint32_t* missing_index);
// Device descriptors (3 words each: stream, length, index) of n_rle
// compressed inputs into desc; an input without an index is given the next
// slot of idx_area (rle_index_bytes each) and its position in *missing.
// TQ_EINVAL if an index is missing and idx_area is null.
tq_status rle_describe(const tq_rle* inputs, uint32_t n_rle, uint64_t nwords, uint64_t* idx_area, uint64_t* desc,
                       std::vector<uint32_t>* missing);
size_t rle_index_bytes(uint64_t nwords);
// Indexes of the streams d_descs[d_list[0..count)], one wave per stream in
// one launch; each is written where its descriptor's index points.
hipError_t launch_build_indexes(const RleDesc* d_descs, const uint32_t* d_list, uint32_t count, uint64_t nwords,
                                int* d_status, hipStream_t stream);
hipError_t launch_set_u64(uint64_t* d_dst, uint64_t value, hipStream_t stream);

// --------------------------------------------------------------- autotuner
constexpr int kTuneDense = 1;   // dense_kernel: p = {wpl, split, groups}
constexpr int kTuneRle = 2;     // rle_tile_kernel: p = {tiles per workgroup (0: one range per slot),
                                //                    counters (1: bit planes, 2: SWAR)}

struct TuneClass {
  int family = 0, K = 0, log_n = 0, log_words = 0, kind = 0, pruned = 0, theta_class = 0, aligned16 = 0;
};
struct TuneEntry {
  int32_t p[4] = {0, 0, 0, 0};
  float us = 0.f;   // measured time of the chosen shape
};

uint64_t tune_key(const TuneClass& c);
bool tune_lookup(tq_ctx* ctx, const TuneClass& c, TuneEntry* e);
void tune_store(tq_ctx* ctx, const TuneClass& c, const TuneEntry& e);
bool tune_entry_valid(const TuneClass& c, const TuneEntry& e);
void tuner_destroy(tq_ctx* ctx);
// true while the stream records a graph (tuning is skipped then)
bool stream_capturing(hipStream_t stream);
// mean microseconds of `reps` launches after one warm-up, or < 0 on error
float time_launches(hipStream_t stream, const std::function<hipError_t()>& launch, int reps);

// -------------------------------------------------------------- blob cache
// Small host arrays that kernels read (pointer arrays, truth tables) are
// staged through pinned memory into device memory and cached by content, so
// a repeated query does not copy them again.
struct Blob {
  std::vector<uint64_t> content;
  uint64_t hash = 0;
  void* d = nullptr;
  uint64_t* h_pinned = nullptr;
  size_t cap_words = 0;
  hipEvent_t copied = nullptr;
  hipStream_t copy_stream = nullptr;
  std::vector<std::pair<hipStream_t, hipEvent_t>> uses;
  uint64_t lru = 0;
  bool valid = false;
  bool frozen = false;   // staged for a captured graph: never evicted or rewritten
};

}  // namespace tq

struct tq_ctx {
  int device = 0;
  int num_cus = 256;
  int* d_status = nullptr;     // first device-detected error (0 = none)
  int sticky_host_error = 0;   // HIP failures seen by the host
  std::vector<tq::Blob> blobs;
  uint64_t lru_clock = 0;
  void* ws = nullptr;          // grow-only device workspace (RLE paths)
  size_t ws_bytes = 0;
  bool ws_frozen = false;      // ws is referenced by a captured graph: retire it instead of freeing
  std::vector<void*> ws_retired;   // workspaces of captured graphs, freed with the context
  tq_status staging_status = TQ_OK;   // why the last blob_get / workspace call failed
  void* batch = nullptr;       // batch slots (created on first submission)
  void* selector = nullptr;    // selector network and feature ranges
  int prune = 1;               // TQ_OPTION_PRUNE
  uint32_t rle_tiles = 0;      // TQ_OPTION_RLE_TILES (0: automatic)
  int rle_counters = 0;        // TQ_OPTION_RLE_COUNTERS (0: automatic, 1: bit planes, 2: SWAR)
  int autotune = 0;            // TQ_OPTION_AUTOTUNE
  int looped = 1;              // TQ_OPTION_LOOPED
  int split = 1;               // TQ_OPTION_SPLIT
  uint64_t batch_bytes = 1ull << 30;   // TQ_OPTION_BATCH_BYTES: device bytes of batches in flight
  uint64_t batch_deadline_us = 0;      // TQ_OPTION_BATCH_DEADLINE_US (0: none)
  void* tuner = nullptr;       // tuned launch shapes by shape class
};

namespace tq {

// Returns a device copy of `words` (count words), staged on `stream`.
// Returns nullptr on failure (ctx->sticky_host_error is set).
const void* blob_get(tq_ctx* ctx, const uint64_t* words, size_t count, hipStream_t stream,
                     Blob** which);
// Records that work using the blob was queued on `stream`.
void blob_used(tq_ctx* ctx, Blob* b, hipStream_t stream);

inline uint64_t words_for_bits(uint64_t r) { return (r + 63) / 64; }
inline uint64_t tail_mask_for(uint64_t r) {
  uint64_t rem = r % 64;
  return rem ? ((uint64_t)1 << rem) - 1 : ~(uint64_t)0;
}
inline int bit_length(uint64_t x) {
  int k = 0;
  while (x) { ++k; x >>= 1; }
  return k;
}

tq_status record_hip(tq_ctx* ctx, hipError_t e);

void batch_destroy(tq_ctx* ctx);

// Variants (bit v for tq_variant v) that can read every input of a query.
uint32_t variants_available(const tq_bitmap* in, uint32_t n);
// The variant the installed selector predicts fastest among `avail`
// (features outside the training range clamped into it); without a selector
// the carry-save counter if available, else the hybrid, else the first.
int select_variant(tq_ctx* ctx, const tq_bitmap* in, uint32_t n, uint64_t r_bits, uint32_t theta, uint32_t avail);
// Dense input pointers of a carry-save threshold in the order it reads them
// (by registered cardinality when pruning).
void csa_input_order(const tq_bitmap* in, uint32_t n, uint64_t r_bits, uint32_t theta, bool prune,
                     std::vector<const uint64_t*>* dense);
void selector_destroy(tq_ctx* ctx);

// Device workspace of at least `bytes` (grown with a device synchronisation).
// Grow-only device workspace.  Under stream capture it cannot grow (nullptr,
// staging_status = TQ_EINVAL) and is kept alive for the captured graph.
void* workspace(tq_ctx* ctx, size_t bytes, hipStream_t stream);
// Status to return after blob_get or workspace failed: TQ_EINVAL when stream
// capture refused the staging, else dflt.
tq_status staging_error(tq_ctx* ctx, tq_status dflt);

}  // namespace tq
