// Host side of libtq: context, staging cache, query planning, ABI entry points.
#include <string.h>

#include <algorithm>
#include <functional>
#include <new>

#include "tq_internal.h"

namespace tq {

tq_status record_hip(tq_ctx* ctx, hipError_t e) {
  if (e == hipSuccess) return TQ_OK;
  if (ctx && !ctx->sticky_host_error) ctx->sticky_host_error = (int)e;
  return e == hipErrorOutOfMemory ? TQ_ENOMEM : TQ_EDEVICE;
}

// ------------------------------------------------------------ blob cache
namespace {

constexpr size_t kMaxBlobs = 64;

uint64_t hash_words(const uint64_t* w, size_t n) {
  uint64_t h = 0x84222325CBF29CE4ull ^ n;
  for (size_t i = 0; i < n; ++i) {
    h ^= w[i];
    h *= 0x100000001B3ull;
    h ^= h >> 29;
  }
  return h;
}

hipError_t blob_wait_idle(Blob& b) {
  for (auto& u : b.uses) {
    hipError_t e = hipEventSynchronize(u.second);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void blob_release(Blob& b) {
  (void)blob_wait_idle(b);
  for (auto& u : b.uses) (void)hipEventDestroy(u.second);
  b.uses.clear();
  if (b.copied) (void)hipEventDestroy(b.copied);
  b.copied = nullptr;
  if (b.d) (void)hipFree(b.d);
  if (b.h_pinned) (void)hipHostFree(b.h_pinned);
  b.d = nullptr;
  b.h_pinned = nullptr;
  b.cap_words = 0;
  b.valid = false;
}

}  // namespace

const void* blob_get(tq_ctx* ctx, const uint64_t* words, size_t count, hipStream_t stream,
                     Blob** which) {
  // Under stream capture nothing is copied: the array must have been staged
  // by an earlier call on the same stream, and it is then frozen (kept as it
  // is for the captured graph, which reads it at every replay).
  const bool capturing = stream_capturing(stream);
  const uint64_t h = hash_words(words, count);
  for (auto& b : ctx->blobs) {
    if (b.valid && b.hash == h && b.content.size() == count &&
        memcmp(b.content.data(), words, count * 8) == 0) {
      if (b.copy_stream != stream) {
        if (capturing) {
          ctx->staging_status = TQ_EINVAL;
          return nullptr;
        }
        hipError_t e = hipStreamWaitEvent(stream, b.copied, 0);
        if (e != hipSuccess) { record_hip(ctx, e); return nullptr; }
      }
      if (capturing) b.frozen = true;
      b.lru = ++ctx->lru_clock;
      *which = &b;
      return b.d;
    }
  }
  if (capturing) {
    ctx->staging_status = TQ_EINVAL;
    return nullptr;
  }
  Blob* victim = nullptr;
  if (ctx->blobs.size() < kMaxBlobs) {
    ctx->blobs.emplace_back();
    victim = &ctx->blobs.back();
  } else {
    for (auto& b : ctx->blobs)
      if (!b.frozen && (!victim || b.lru < victim->lru)) victim = &b;
    if (!victim) {   // every slot holds an array of a captured graph
      ctx->staging_status = TQ_ENOMEM;
      return nullptr;
    }
  }
  hipError_t e = blob_wait_idle(*victim);
  if (e != hipSuccess) { record_hip(ctx, e); return nullptr; }
  victim->valid = false;
  if (victim->cap_words < count) {
    if (victim->d) (void)hipFree(victim->d);
    if (victim->h_pinned) (void)hipHostFree(victim->h_pinned);
    victim->d = nullptr;
    victim->h_pinned = nullptr;
    size_t cap = std::max<size_t>(count, 512);
    if ((e = hipMalloc(&victim->d, cap * 8)) != hipSuccess) { record_hip(ctx, e); victim->d = nullptr; return nullptr; }
    if ((e = hipHostMalloc((void**)&victim->h_pinned, cap * 8, hipHostMallocDefault)) != hipSuccess) {
      record_hip(ctx, e);
      victim->h_pinned = nullptr;
      return nullptr;
    }
    victim->cap_words = cap;
  }
  if (!victim->copied) {
    if ((e = hipEventCreateWithFlags(&victim->copied, hipEventDisableTiming)) != hipSuccess) {
      record_hip(ctx, e);
      return nullptr;
    }
  }
  memcpy(victim->h_pinned, words, count * 8);
  if ((e = hipMemcpyAsync(victim->d, victim->h_pinned, count * 8, hipMemcpyHostToDevice, stream)) !=
      hipSuccess) {
    record_hip(ctx, e);
    return nullptr;
  }
  if ((e = hipEventRecord(victim->copied, stream)) != hipSuccess) { record_hip(ctx, e); return nullptr; }
  victim->copy_stream = stream;
  victim->content.assign(words, words + count);
  victim->hash = h;
  victim->lru = ++ctx->lru_clock;
  victim->valid = true;
  *which = victim;
  return victim->d;
}

void blob_used(tq_ctx* ctx, Blob* b, hipStream_t stream) {
  // a frozen array is never rewritten, so its readers need no tracking (and
  // an event recorded under capture is not one the host could wait for)
  if (b->frozen) return;
  for (auto& u : b->uses) {
    if (u.first == stream) {
      record_hip(ctx, hipEventRecord(u.second, stream));
      return;
    }
  }
  hipEvent_t ev = nullptr;
  if (record_hip(ctx, hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != TQ_OK) return;
  record_hip(ctx, hipEventRecord(ev, stream));
  b->uses.emplace_back(stream, ev);
}

// --------------------------------------------------------------- planning
static SymPlan constant_plan(bool one) {
  SymPlan p{};
  p.constant = true;
  p.const_word = one ? ~(uint64_t)0 : 0;
  return p;
}

SymPlan plan_threshold(uint32_t n, uint32_t theta) {
  if (theta == 0) return constant_plan(true);
  if (theta > n) return constant_plan(false);
  SymPlan p{};
  p.constant = false;
  p.epi.kind = EPI_THRESH;
  p.epi.theta = theta;
  return p;
}

// Runs of ones of f over [0, n] as half-open [lo, hi1).
static std::vector<std::pair<uint32_t, uint32_t>> runs_of(const std::vector<uint8_t>& f, uint8_t v) {
  std::vector<std::pair<uint32_t, uint32_t>> r;
  const uint32_t m = (uint32_t)f.size();
  for (uint32_t c = 0; c < m;) {
    if (f[c] != v) { ++c; continue; }
    uint32_t d = c;
    while (d < m && f[d] == v) ++d;
    r.emplace_back(c, d);
    c = d;
  }
  return r;
}

SymPlan plan_symmetric(uint32_t n, const uint64_t* truth) {
  std::vector<uint8_t> f(n + 1);
  for (uint32_t c = 0; c <= n; ++c) f[c] = (truth[c / 64] >> (c % 64)) & 1;
  auto ones = runs_of(f, 1);
  if (ones.empty()) return constant_plan(false);
  if (ones.size() == 1 && ones[0].first == 0 && ones[0].second == n + 1) return constant_plan(true);
  SymPlan p{};
  p.constant = false;
  // a single run reaching n is a threshold; a single run starting at 0 is its complement
  if (ones.size() == 1 && ones[0].second == n + 1) {
    p.epi.kind = EPI_THRESH;
    p.epi.theta = ones[0].first;
    return p;
  }
  if (ones.size() == 1 && ones[0].first == 0) {
    p.epi.kind = EPI_THRESH;
    p.epi.theta = ones[0].second;
    p.epi.invert = 1;
    return p;
  }
  bool parity = true, nparity = true;
  for (uint32_t c = 0; c <= n; ++c) {
    parity &= f[c] == (c & 1);
    nparity &= f[c] != (c & 1);
  }
  if (parity || nparity) {
    p.epi.kind = EPI_PARITY;
    p.epi.invert = nparity ? 1 : 0;
    return p;
  }
  auto zeros = runs_of(f, 0);
  const bool use_zeros = zeros.size() < ones.size();
  const auto& iv = use_zeros ? zeros : ones;
  if ((int)iv.size() <= kMaxIntervals) {
    p.epi.kind = EPI_INTERVALS;
    p.epi.invert = use_zeros ? 1 : 0;
    p.epi.nint = (int32_t)iv.size();
    for (size_t t = 0; t < iv.size(); ++t) {
      p.epi.lo[t] = iv[t].first;
      p.epi.hi1[t] = iv[t].second;  // == n + 1 means no upper bound
    }
    return p;
  }
  p.epi.kind = EPI_TABLE;
  // table sized for the counter's full range so any count indexes it
  const uint32_t entries = 1u << dense_planes_for(n);
  p.table.assign((entries + 31) / 32, 0);
  for (uint32_t c = 0; c <= n; ++c)
    if (f[c]) p.table[c / 32] |= 1u << (c % 32);
  p.epi.table_words = (uint32_t)p.table.size();
  return p;
}

// Arguments of the fused-consumer calls (filter, output, count).
tq_status check_sink_args(uint64_t r_bits, const uint64_t* d_filter, const uint64_t* d_out,
                          const uint64_t* d_count) {
  if (!d_out && !d_count) return TQ_EINVAL;
  if (((uintptr_t)d_filter & 7) || ((uintptr_t)d_count & 7)) return TQ_EINVAL;
  const uint64_t nw = words_for_bits(r_bits);
  if (d_filter && d_out && d_filter != d_out) {
    const uintptr_t f0 = (uintptr_t)d_filter, o0 = (uintptr_t)d_out;
    if (f0 < o0 + nw * 8 && o0 < f0 + nw * 8) return TQ_EINVAL;
  }
  if (d_count && d_out) {
    const uintptr_t c0 = (uintptr_t)d_count, o0 = (uintptr_t)d_out;
    if (c0 < o0 + nw * 8 && o0 < c0 + 8) return TQ_EINVAL;
  }
  return TQ_OK;
}

}  // namespace tq

using namespace tq;

// ----------------------------------------------------------------- ABI
extern "C" {

const char* tq_status_string(int s) {
  switch (s) {
    case TQ_OK: return "TQ_OK";
    case TQ_EINVAL: return "TQ_EINVAL: invalid argument";
    case TQ_ENOMEM: return "TQ_ENOMEM: out of memory";
    case TQ_EFORMAT: return "TQ_EFORMAT: malformed run-length stream";
    case TQ_ECAPACITY: return "TQ_ECAPACITY: output capacity too small";
    case TQ_EDEVICE: return "TQ_EDEVICE: HIP runtime error";
    case TQ_EBUSY: return "TQ_EBUSY: admission refused, retry";
    case TQ_ECANCELED: return "TQ_ECANCELED: batch cancelled before the query completed";
    case TQ_ETIMEDOUT: return "TQ_ETIMEDOUT: batch deadline passed before the query completed";
    case TQ_ENOTSUP: return "TQ_ENOTSUP: not supported";
  }
  return "unknown tq status";
}

tq_status tq_create(tq_ctx** out, int device) {
  if (!out) return TQ_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return TQ_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return TQ_EDEVICE;
  tq_ctx* c = new (std::nothrow) tq_ctx();
  if (!c) return TQ_ENOMEM;
  c->device = device;
  // scratch array of the allocation-free entry point, located once per device
  const tq_status ns = noalloc_init(device);
  if (ns != TQ_OK) {
    delete c;
    return ns;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cus = prop.multiProcessorCount;
  if (hipMalloc((void**)&c->d_status, 256) != hipSuccess) {
    delete c;
    return TQ_ENOMEM;
  }
  if (hipMemset(c->d_status, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(c->d_status);
    delete c;
    return TQ_EDEVICE;
  }
  c->blobs.reserve(64);
  *out = c;
  return TQ_OK;
}

// Teardown is best effort: every resource is released whatever the device
// reports on the way.
tq_status tq_destroy(tq_ctx* ctx) {
  if (!ctx) return TQ_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  batch_destroy(ctx);
  selector_destroy(ctx);
  tuner_destroy(ctx);
  for (auto& b : ctx->blobs) blob_release(b);
  if (ctx->ws) (void)hipFree(ctx->ws);
  for (void* p : ctx->ws_retired) (void)hipFree(p);
  if (ctx->d_status) (void)hipFree(ctx->d_status);
  delete ctx;
  return TQ_OK;
}

tq_status tq_set_option(tq_ctx* ctx, int option, int64_t value) {
  if (!ctx) return TQ_EINVAL;
  switch (option) {
    case TQ_OPTION_PRUNE:
      ctx->prune = value ? 1 : 0;
      return TQ_OK;
    case TQ_OPTION_RLE_TILES:
      if (value < 0 || value > (1 << 20)) return TQ_EINVAL;
      ctx->rle_tiles = (uint32_t)value;
      return TQ_OK;
    case TQ_OPTION_AUTOTUNE:
      ctx->autotune = value ? 1 : 0;
      return TQ_OK;
    case TQ_OPTION_LOOPED:
      ctx->looped = value ? 1 : 0;
      return TQ_OK;
    case TQ_OPTION_SPLIT:
      ctx->split = value ? 1 : 0;
      return TQ_OK;
    case TQ_OPTION_BATCH_BYTES:
      if (value < 1) return TQ_EINVAL;
      ctx->batch_bytes = (uint64_t)value;
      return TQ_OK;
    case TQ_OPTION_BATCH_DEADLINE_US:
      if (value < 0 || value > (1ll << 40)) return TQ_EINVAL;
      ctx->batch_deadline_us = (uint64_t)value;
      return TQ_OK;
    case TQ_OPTION_RLE_COUNTERS:
      if (value < 0 || value > 2) return TQ_EINVAL;
      ctx->rle_counters = (int)value;
      return TQ_OK;
  }
  return TQ_EINVAL;
}

tq_status tq_ctx_check(tq_ctx* ctx, hipStream_t stream) {
  if (!ctx) return TQ_EINVAL;
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return record_hip(ctx, e);
  if (ctx->sticky_host_error) {
    ctx->sticky_host_error = 0;
    return TQ_EDEVICE;
  }
  int st = 0;
  if ((e = hipMemcpy(&st, ctx->d_status, sizeof(int), hipMemcpyDeviceToHost)) != hipSuccess)
    return record_hip(ctx, e);
  if (st != 0) {
    int zero = 0;
    if ((e = hipMemcpy(ctx->d_status, &zero, sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
      return record_hip(ctx, e);
    return (tq_status)st;
  }
  return TQ_OK;
}

}  // extern "C"

// Validate the pointer array and the output; returns whether every buffer is 16-byte aligned.
tq_status tq::check_dense_args(const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits, const uint64_t* d_out,
                               bool* aligned16, bool out_optional) {
  if (!ptrs || n == 0 || n > TQ_MAX_INPUTS) return TQ_EINVAL;
  const uint64_t nw = words_for_bits(r_bits);
  if (r_bits > 0 && !d_out && !out_optional) return TQ_EINVAL;
  uintptr_t any = (uintptr_t)d_out;
  const uintptr_t o0 = (uintptr_t)d_out, o1 = o0 + nw * 8;
  for (uint32_t j = 0; j < n; ++j) {
    const uintptr_t p = (uintptr_t)ptrs[j];
    if (!p || (p & 7)) return TQ_EINVAL;
    any |= p;
    if (d_out && r_bits > 0 && p < o1 && o0 < p + nw * 8) return TQ_EINVAL;  // output overlaps an input
  }
  if ((uintptr_t)d_out & 7) return TQ_EINVAL;
  *aligned16 = (any & 15) == 0;
  return TQ_OK;
}

namespace {

// Arguments of the fused consumers: the filter is nullable and may be the
// output itself but must not overlap it otherwise; the count is nullable;
// at least one of output and count is given.

// The launch shape of a dense query: the tuned shape of its class if the
// autotuner is on (timing every candidate on the first query of the class),
// else the default rule.
DenseConfig dense_shape(tq_ctx* ctx, uint32_t n, uint64_t nw, const EpiParams& epi, bool aligned16,
                        const std::function<hipError_t(const DenseConfig&)>& launch, hipStream_t stream) {
  const bool can_prune = epi.kind == EPI_THRESH && epi.prune && epi.theta >= 1 && epi.theta <= n;
  const DenseConfig dflt = choose_dense_config(n, nw, aligned16, ctx->num_cus, can_prune);
  if (!ctx->autotune) return dflt;
  TuneClass c;
  c.family = kTuneDense;
  c.K = dflt.K;
  c.log_n = bit_length(n) - 1;
  c.log_words = bit_length(nw) - 1;
  c.kind = epi.kind;
  c.pruned = (epi.kind == EPI_THRESH && epi.prune) ? 1 : 0;
  c.theta_class = c.pruned ? (int)((8ull * epi.theta) / ((uint64_t)n + 1)) : 0;
  c.aligned16 = aligned16 ? 1 : 0;
  TuneEntry e;
  if (tune_lookup(ctx, c, &e)) return DenseConfig{dflt.K, e.p[0], e.p[1], e.p[2]};
  if (stream_capturing(stream)) return dflt;
  static const int cand[][3] = {{1, 1, 1}, {1, 2, 1}, {1, 4, 1}, {1, 8, 1}, {1, 1, 4}, {2, 1, 1}, {2, 1, 4}};
  DenseConfig best = dflt;
  float best_us = -1.f;
  for (const auto& q : cand) {
    const DenseConfig cfg{dflt.K, q[0], q[1], q[2]};
    if (cfg.wpl == 2 && !aligned16) continue;
    if (!dense_config_valid(cfg)) continue;
    const float us = time_launches(stream, [&]() { return launch(cfg); }, 5);
    if (us > 0.f && (best_us < 0.f || us < best_us)) {
      best = cfg;
      best_us = us;
    }
  }
  if (best_us > 0.f) {
    e.p[0] = best.wpl;
    e.p[1] = best.split;
    e.p[2] = best.groups;
    e.p[3] = 0;
    e.us = best_us;
    tune_store(ctx, c, e);
  }
  return best;
}

tq_status run_dense(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits,
                    const SymPlan& plan, uint64_t* d_out, hipStream_t stream, bool aligned16,
                    const uint64_t* d_filter = nullptr, uint64_t* d_count = nullptr) {
  const uint64_t nw = words_for_bits(r_bits);
  const uint64_t tmask = tail_mask_for(r_bits);
  if (nw == 0) return d_count ? record_hip(ctx, launch_set_u64(d_count, 0, stream)) : TQ_OK;
  const bool fused = d_filter || d_count;
  Sink sink;
  sink.filter = d_filter;
  if (plan.constant) {
    if (!fused) return record_hip(ctx, launch_fill(d_out, nw, plan.const_word, tmask, stream));
    const uint64_t slots = fill_groups(nw);
    if (d_count) {
      sink.partial = static_cast<uint32_t*>(workspace(ctx, slots * sizeof(uint32_t), stream));
      if (!sink.partial) return staging_error(ctx, TQ_ENOMEM);
    }
    tq_status st = record_hip(ctx, launch_fill_sink(d_out, nw, plan.const_word, tmask, sink, stream));
    if (st == TQ_OK && d_count) st = record_hip(ctx, launch_count_reduce(sink.partial, slots, d_count, stream));
    return st;
  }
  Blob* pb = nullptr;
  const void* d_ptrs = blob_get(ctx, reinterpret_cast<const uint64_t*>(ptrs), n, stream, &pb);
  if (!d_ptrs) return staging_error(ctx, TQ_EDEVICE);
  EpiParams epi = plan.epi;
  epi.prune = ctx->prune ? 1u : 0u;
  Blob* tb = nullptr;
  if (epi.kind == EPI_TABLE) {
    std::vector<uint64_t> t64((plan.table.size() + 1) / 2, 0);
    memcpy(t64.data(), plan.table.data(), plan.table.size() * 4);
    const void* d_t = blob_get(ctx, t64.data(), t64.size(), stream, &tb);
    if (!d_t) return staging_error(ctx, TQ_EDEVICE);
    epi.table = reinterpret_cast<const uint32_t*>(d_t);
  }
  const uint64_t* const* dp = reinterpret_cast<const uint64_t* const*>(d_ptrs);
  // thresholds within 3 of either end: saturating counters (no consumers)
  uint32_t lt = 0;
  bool lcomp = false;
  if (ctx->looped && !fused && epi.kind == EPI_THRESH && !epi.invert && looped_applies(n, epi.theta, &lt, &lcomp)) {
    tq_status st = record_hip(ctx, launch_looped(dp, n, nw, tmask, epi.theta, epi.prune != 0, d_out, stream));
    blob_used(ctx, pb, stream);
    if (tb) blob_used(ctx, tb, stream);
    return st;
  }
  // short bitmaps with many inputs: the inputs are split over workgroups
  // and their partial counts added by a second kernel (no consumers)
  if (!fused && ctx->split) {
    const SplitPlan sp = plan_split(n, nw, ctx->num_cus);
    if (sp.parts) {
      uint64_t* part = static_cast<uint64_t*>(workspace(ctx, split_workspace_bytes(sp), stream));
      if (!part) return staging_error(ctx, TQ_ENOMEM);
      tq_status st = record_hip(ctx, launch_dense_split(sp, dp, n, nw, tmask, d_out, epi, part, stream));
      blob_used(ctx, pb, stream);
      if (tb) blob_used(ctx, tb, stream);
      return st;
    }
  }
  const DenseConfig cfg = dense_shape(
      ctx, n, nw, epi, aligned16,
      [&](const DenseConfig& c) { return launch_dense(c, dp, n, nw, tmask, d_out, epi, stream); }, stream);
  if (d_count) {
    sink.partial = static_cast<uint32_t*>(workspace(ctx, dense_groups(cfg, nw) * sizeof(uint32_t), stream));
    if (!sink.partial) return staging_error(ctx, TQ_ENOMEM);
  }
  tq_status st = record_hip(ctx, launch_dense(cfg, dp, n, nw, tmask, d_out, epi, stream, sink));
  if (st == TQ_OK && d_count)
    st = record_hip(ctx, launch_count_reduce(sink.partial, dense_groups(cfg, nw), d_count, stream));
  blob_used(ctx, pb, stream);
  if (tb) blob_used(ctx, tb, stream);
  return st;
}

}  // namespace

// An imported tuning entry must name a shape that exists.
bool tq::tune_entry_valid(const TuneClass& c, const TuneEntry& e) {
  if (!(e.us >= 0.f)) return false;
  if (c.family == kTuneDense) {
    const DenseConfig cfg{c.K, e.p[0], e.p[1], e.p[2]};
    if (e.p[0] == 2 && !c.aligned16) return false;
    return dense_config_valid(cfg) && e.p[3] == 0;
  }
  if (c.family == kTuneRle)
    return e.p[0] >= 0 && e.p[0] <= (1 << 20) && (e.p[1] == 1 || e.p[1] == 2) && e.p[2] == 0 && e.p[3] == 0;
  return false;
}

extern "C" {

tq_status tq_threshold(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits,
                       uint32_t theta, uint64_t* d_out, hipStream_t stream) {
  if (!ctx) return TQ_EINVAL;
  bool a16 = false;
  tq_status st = check_dense_args(ptrs, n, r_bits, d_out, &a16);
  if (st != TQ_OK) return st;
  return run_dense(ctx, ptrs, n, r_bits, plan_threshold(n, theta), d_out, stream, a16);
}

tq_status tq_symmetric(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits,
                       const uint64_t* h_truth, uint64_t* d_out, hipStream_t stream) {
  if (!ctx || !h_truth) return TQ_EINVAL;
  bool a16 = false;
  tq_status st = check_dense_args(ptrs, n, r_bits, d_out, &a16);
  if (st != TQ_OK) return st;
  return run_dense(ctx, ptrs, n, r_bits, plan_symmetric(n, h_truth), d_out, stream, a16);
}

tq_status tq_threshold_weighted(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, const uint32_t* h_weights,
                                uint64_t r_bits, uint64_t theta, uint64_t* d_out, hipStream_t stream) {
  if (!ctx || !h_weights) return TQ_EINVAL;
  bool a16 = false;
  tq_status st = check_dense_args(ptrs, n, r_bits, d_out, &a16);
  if (st != TQ_OK) return st;
  uint64_t total = 0;
  for (uint32_t j = 0; j < n; ++j) total += h_weights[j];
  if (total > 0xFFFFFFFFull) return TQ_EINVAL;
  const uint64_t nw = words_for_bits(r_bits);
  const uint64_t tmask = tail_mask_for(r_bits);
  if (nw == 0) return TQ_OK;
  if (theta == 0 || theta > total)
    return record_hip(ctx, launch_fill(d_out, nw, theta == 0 ? ~(uint64_t)0 : 0, tmask, stream));
  // group the inputs of equal weight (weight 0 contributes nothing), heaviest
  // first; with pruning, classes of at most kPruneClass inputs, after each of
  // which the kernel checks whether a lane's positions are all decided
  // (measured on 256 inputs of weights 1..4: 16 against 64 is 10-40 % faster
  // where theta lets it prune, 1 % slower where it cannot)
  constexpr uint32_t kPruneClass = 16;
  std::vector<uint32_t> order;
  order.reserve(n);
  for (uint32_t j = 0; j < n; ++j)
    if (h_weights[j]) order.push_back(j);
  std::stable_sort(order.begin(), order.end(),
                   [&](uint32_t a, uint32_t b) { return h_weights[a] > h_weights[b]; });
  std::vector<uint64_t> sorted(order.size());
  std::vector<WeightClass> classes;
  uint32_t max_class = 0;
  for (size_t i = 0; i < order.size(); ++i) {
    sorted[i] = (uint64_t)(uintptr_t)ptrs[order[i]];
    const uint32_t wt = h_weights[order[i]];
    if (classes.empty() || classes.back().weight != wt ||
        (ctx->prune && classes.back().end - classes.back().begin >= kPruneClass))
      classes.push_back(WeightClass{wt, (uint32_t)i, (uint32_t)i, 0});
    classes.back().end = (uint32_t)i + 1;
    const uint32_t size = classes.back().end - classes.back().begin;
    if (size > max_class) max_class = size;
  }
  Blob* pb = nullptr;
  Blob* cb = nullptr;
  const void* d_ptrs = blob_get(ctx, sorted.data(), sorted.size(), stream, &pb);
  if (!d_ptrs) return staging_error(ctx, TQ_EDEVICE);
  const void* d_cls = blob_get(ctx, reinterpret_cast<const uint64_t*>(classes.data()), classes.size() * 2, stream,
                               &cb);
  if (!d_cls) return staging_error(ctx, TQ_EDEVICE);
  st = record_hip(ctx, launch_weighted(reinterpret_cast<const uint64_t* const*>(d_ptrs),
                                       reinterpret_cast<const WeightClass*>(d_cls), (uint32_t)classes.size(),
                                       max_class, nw, tmask, (uint32_t)theta, (uint32_t)total, ctx->prune != 0,
                                       d_out, stream));
  blob_used(ctx, pb, stream);
  blob_used(ctx, cb, stream);
  return st;
}

tq_status tq_threshold_fused(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits,
                             uint32_t theta, const uint64_t* d_filter, uint64_t* d_out, uint64_t* d_count,
                             hipStream_t stream) {
  if (!ctx) return TQ_EINVAL;
  tq_status st = check_sink_args(r_bits, d_filter, d_out, d_count);
  if (st != TQ_OK) return st;
  bool a16 = false;
  st = check_dense_args(ptrs, n, r_bits, d_out, &a16, true);
  if (st != TQ_OK) return st;
  return run_dense(ctx, ptrs, n, r_bits, plan_threshold(n, theta), d_out, stream, a16, d_filter, d_count);
}

tq_status tq_symmetric_fused(tq_ctx* ctx, const uint64_t* const* ptrs, uint32_t n, uint64_t r_bits,
                             const uint64_t* h_truth, const uint64_t* d_filter, uint64_t* d_out,
                             uint64_t* d_count, hipStream_t stream) {
  if (!ctx || !h_truth) return TQ_EINVAL;
  tq_status st = check_sink_args(r_bits, d_filter, d_out, d_count);
  if (st != TQ_OK) return st;
  bool a16 = false;
  st = check_dense_args(ptrs, n, r_bits, d_out, &a16, true);
  if (st != TQ_OK) return st;
  return run_dense(ctx, ptrs, n, r_bits, plan_symmetric(n, h_truth), d_out, stream, a16, d_filter, d_count);
}

}  // extern "C"
