// Fused threshold query that allocates nothing.
//
// The query is tq_threshold_fused's (threshold of section 2.3, result ANDed
// with a filter and counted).  Its two pieces of device scratch -- the device
// copy of the input pointer array and the per-column-group popcounts that the
// count sums -- live in one fixed file-scope array instead of the context's
// grow-only workspace and staging cache, so a call makes no hipMalloc,
// hipHostMalloc, hipFree or event creation.  Every call on one device shares
// that device's array: calls that overlap in time on one device race, and
// calls on one stream are ordered by the stream.
#include <mutex>

#include "tq_internal.h"

namespace tq {
namespace {

constexpr size_t kScratchBytes = TQ_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

// The pointer array (at most TQ_MAX_INPUTS entries) and the partial counts.
// In host code this name stands for the symbol, not for device memory: the
// device address is taken once per device with hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices];   // device address of `scratch` on each device

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

tq_status noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return TQ_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return TQ_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return TQ_EDEVICE;
  g_scratch[device] = p;
  return TQ_OK;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_scratch[device];
}

}  // namespace tq

using namespace tq;

extern "C" {

tq_status tq_threshold_fused_noalloc(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits,
                                     uint32_t theta, const uint64_t* d_filter, uint64_t* d_out,
                                     uint64_t* d_count, hipStream_t stream) {
  if (!ctx) return TQ_EINVAL;
  tq_status st = check_sink_args(r_bits, d_filter, d_out, d_count);
  if (st != TQ_OK) return st;
  bool a16 = false;
  st = check_dense_args(ptrs, n, r_bits, d_out, &a16, true);
  if (st != TQ_OK) return st;
  char* base = static_cast<char*>(noalloc_scratch(ctx->device));
  if (!base) return TQ_EDEVICE;
  const uint64_t nw = words_for_bits(r_bits);
  const uint64_t tmask = tail_mask_for(r_bits);
  if (nw == 0) return d_count ? record_hip(ctx, launch_set_u64(d_count, 0, stream)) : TQ_OK;
  const SymPlan plan = plan_threshold(n, theta);
  Sink sink;
  sink.filter = d_filter;
  if (plan.constant) {
    // every partial slot is written by the fill kernel before it is summed
    const uint64_t slots = fill_groups(nw);
    if (d_count && slots > kScratchBytes / sizeof(uint32_t)) return TQ_EINVAL;
    if (d_count) sink.partial = reinterpret_cast<uint32_t*>(base);
    st = record_hip(ctx, launch_fill_sink(d_out, nw, plan.const_word, tmask, sink, stream));
    if (st == TQ_OK && d_count) st = record_hip(ctx, launch_count_reduce(sink.partial, slots, d_count, stream));
    return st;
  }
  // the default launch shape: the autotuner times candidates with events,
  // which this entry point does not create
  const DenseConfig cfg = choose_dense_config(n, nw, a16, ctx->num_cus);
  const size_t ptr_bytes = align256((size_t)n * sizeof(uint64_t));
  const uint64_t groups = dense_groups(cfg, nw);
  if (d_count && groups > (kScratchBytes - ptr_bytes) / sizeof(uint32_t)) return TQ_EINVAL;
  // the pointer array goes into the scratch array on the stream; the caller's
  // host array is staged by the runtime before the copy call returns
  hipError_t e = hipMemcpyAsync(base, ptrs, (size_t)n * sizeof(uint64_t), hipMemcpyHostToDevice, stream);
  if (e != hipSuccess) return record_hip(ctx, e);
  EpiParams epi = plan.epi;
  epi.prune = ctx->prune ? 1u : 0u;
  // one partial count per column group, each written by the group's wave
  if (d_count) sink.partial = reinterpret_cast<uint32_t*>(base + ptr_bytes);
  st = record_hip(ctx, launch_dense(cfg, reinterpret_cast<const uint64_t* const*>(base), n, nw, tmask, d_out, epi,
                                    stream, sink));
  if (st == TQ_OK && d_count) st = record_hip(ctx, launch_count_reduce(sink.partial, groups, d_count, stream));
  return st;
}

}  // extern "C"
