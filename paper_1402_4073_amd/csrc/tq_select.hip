// Kernel-variant selection: per-bitmap metadata, query features, the four
// bit-exact variants behind one call, host-side inference of the selector
// network, and the MLP training entry points.
//
// The paper observes that which threshold algorithm is fastest depends on N,
// T, the density and the run structure of the inputs (sections 5.7-5.10 and
// 6).  Here that choice is made per query among four GPU
// variants that all produce the same bits: the carry-save counter over dense
// words, per-position counters over dense words, the run-length tile merge over
// compressed inputs, and the hybrid that reads each input in its smaller form.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <unordered_map>
#include <vector>

#include "tq_internal.h"

namespace tq {

hipError_t launch_counter(const uint64_t* const* d_ptrs, uint32_t n, uint64_t nwords, uint64_t tail_mask,
                          uint32_t theta, const uint32_t* d_table, uint64_t* d_out, hipStream_t stream);
hipError_t launch_stats(const uint64_t* d_dense, uint64_t r_bits, uint64_t* d_ones, uint64_t* d_runs,
                        hipStream_t stream);
uint32_t mlp_chunks(uint32_t batch);
hipError_t launch_mlp_forward(const float* d_params, const float* d_x, uint32_t batch, float* d_y,
                              hipStream_t stream);
hipError_t launch_mlp_grad(const float* d_params, const float* d_x, const float* d_t, const float* d_mask,
                           uint32_t batch, float inv_count, float* d_y, float* d_grad, float* d_loss, void* ws,
                           hipStream_t stream);
size_t mlp_grad_workspace_bytes(uint32_t batch);
hipError_t launch_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t n, float lr,
                       float beta1, float beta2, float eps, uint32_t step, hipStream_t stream);

struct Selector {
  bool ready = false;
  std::vector<float> params;   // TQ_SEL_PARAMS
  float mean[TQ_SEL_FEATURES], stdev[TQ_SEL_FEATURES], lo[TQ_SEL_FEATURES], hi[TQ_SEL_FEATURES];
  float margin = 0.f;
  // decisions of the timing fallback by feature cell (see decision_key)
  std::unordered_map<uint64_t, uint8_t> decided;
};

namespace {

constexpr int kIn = TQ_SEL_FEATURES, kHid = TQ_SEL_HIDDEN, kOut = TQ_SEL_VARIANTS;

bool has_dense(const tq_bitmap& b) { return b.dense != nullptr; }
bool has_rle(const tq_bitmap& b) { return b.rle.words != nullptr && b.rle.n_words > 0; }

// variant availability for a query
bool variant_available(const tq_bitmap* in, uint32_t n, int v) {
  for (uint32_t j = 0; j < n; ++j) {
    if ((v == TQ_VARIANT_CSA || v == TQ_VARIANT_COUNTER) && !has_dense(in[j])) return false;
    if (v == TQ_VARIANT_RLE && !has_rle(in[j])) return false;
    if (v == TQ_VARIANT_HYBRID && !has_dense(in[j]) && !has_rle(in[j])) return false;
  }
  return true;
}

void host_forward(const Selector& s, const float* f, float* y) {
  const float* P = s.params.data();
  const float* W1 = P;
  const float* B1 = W1 + kHid * kIn;
  const float* W2 = B1 + kHid;
  const float* B2 = W2 + kHid * kHid;
  const float* W3 = B2 + kHid;
  const float* B3 = W3 + kOut * kHid;
  float x[kIn], h1[kHid], h2[kHid];
  for (int i = 0; i < kIn; ++i) x[i] = (f[i] - s.mean[i]) / s.stdev[i];
  for (int j = 0; j < kHid; ++j) {
    float z = B1[j];
    for (int i = 0; i < kIn; ++i) z += W1[j * kIn + i] * x[i];
    h1[j] = z > 0.f ? z : 0.f;
  }
  for (int j = 0; j < kHid; ++j) {
    float z = B2[j];
    for (int i = 0; i < kHid; ++i) z += W2[j * kHid + i] * h1[i];
    h2[j] = z > 0.f ? z : 0.f;
  }
  for (int k = 0; k < kOut; ++k) {
    float z = B3[k];
    for (int i = 0; i < kHid; ++i) z += W3[k * kHid + i] * h2[i];
    y[k] = z;
  }
}

// Cell of a query for the fallback's remembered decisions: each feature in
// quarters of its training standard deviation (raw quarters without weights),
// and which variants the inputs allow.  Keys are FNV-1a hashes; two cells
// sharing a key only share a choice of variant, and every variant gives the
// same bits.
constexpr size_t kMaxDecisions = 1u << 16;

uint64_t decision_key(const Selector& s, const float* f, uint32_t avail) {
  uint64_t h = 1469598103934665603ull ^ avail;
  for (int i = 0; i < kIn; ++i) {
    float z = s.ready ? (f[i] - s.mean[i]) / s.stdev[i] : f[i];
    z = std::min(std::max(z * 4.f, -1e6f), 1e6f);
    const uint32_t q = (uint32_t)(int32_t)lrintf(z);
    for (int b = 0; b < 4; ++b) h = (h ^ ((q >> (8 * b)) & 0xFFu)) * 1099511628211ull;
  }
  return h;
}

}  // namespace

uint32_t variants_available(const tq_bitmap* in, uint32_t n) {
  uint32_t avail = 0;
  for (int v = 0; v < kOut; ++v)
    if (variant_available(in, n, v)) avail |= 1u << v;
  return avail;
}

int select_variant(tq_ctx* ctx, const tq_bitmap* in, uint32_t n, uint64_t r_bits, uint32_t theta, uint32_t avail) {
  const Selector* s = static_cast<const Selector*>(ctx->selector);
  float f[kIn], y[kOut];
  if (s && s->ready && r_bits > 0 && tq_query_features(in, n, r_bits, theta, f) == TQ_OK) {
    // no variant can be timed here: features outside the training range are
    // taken at the nearest edge of it
    for (int i = 0; i < kIn; ++i) f[i] = std::min(std::max(f[i], s->lo[i]), s->hi[i]);
    host_forward(*s, f, y);
    int best = -1;
    for (int v = 0; v < kOut; ++v)
      if (((avail >> v) & 1u) && (best < 0 || y[v] < y[best])) best = v;
    if (best >= 0) return best;
  }
  if (avail & (1u << TQ_VARIANT_CSA)) return TQ_VARIANT_CSA;
  if (avail & (1u << TQ_VARIANT_HYBRID)) return TQ_VARIANT_HYBRID;
  return avail ? __builtin_ctz(avail) : -1;
}

void csa_input_order(const tq_bitmap* in, uint32_t n, uint64_t r_bits, uint32_t theta, bool prune,
                     std::vector<const uint64_t*>* dense) {
  // Inputs in order of registered cardinality (the lower-bound skipping of
  // section 1, with pruning on): a lane stops reading once each of its
  // positions has reached theta, which dense inputs read first bring about
  // sooner, or can no longer reach it with the inputs left, which sparse
  // inputs read first bring about sooner (the count stays low while the
  // inputs left run out).  Dense first when theta is below half the expected
  // count, else sparse first; equal cardinalities keep the caller's order.
  // The result does not depend on the order.
  dense->resize(n);
  if (!(prune && r_bits > 0) || n > TQ_MAX_INPUTS) {   // (more inputs are rejected by the query)
    for (uint32_t j = 0; j < n; ++j) (*dense)[j] = in[j].dense;
    return;
  }
  double total = 0;
  for (uint32_t j = 0; j < n; ++j) total += (double)in[j].ones;
  const bool dense_first = 2.0 * (double)theta < total / (double)r_bits;
  // one 64-bit key per input: its cardinality (complemented for dense first;
  // at most 2^47, above any bitmap the library admits) above its position
  // (n <= 65535), so a plain sort of the keys gives the stable order
  constexpr uint64_t kMaxOnes = (1ull << 48) - 1;
  std::vector<uint64_t> key(n);
  for (uint32_t j = 0; j < n; ++j) {
    const uint64_t c = in[j].ones < kMaxOnes ? in[j].ones : kMaxOnes;
    key[j] = ((dense_first ? kMaxOnes - c : c) << 16) | j;
  }
  std::sort(key.begin(), key.end());
  for (uint32_t j = 0; j < n; ++j) (*dense)[j] = in[(uint32_t)(key[j] & 0xFFFF)].dense;
}

void selector_destroy(tq_ctx* ctx) {
  delete static_cast<Selector*>(ctx->selector);
  ctx->selector = nullptr;
}

}  // namespace tq

using namespace tq;

extern "C" {

tq_status tq_bitmap_stats(tq_ctx* ctx, const uint64_t* d_dense, uint64_t r_bits, uint64_t* d_ones,
                          uint64_t* d_runs, hipStream_t stream) {
  if (!ctx || !d_ones || !d_runs || (r_bits && !d_dense)) return TQ_EINVAL;
  if (((uintptr_t)d_dense & 7) || ((uintptr_t)d_ones & 7) || ((uintptr_t)d_runs & 7)) return TQ_EINVAL;
  return record_hip(ctx, launch_stats(d_dense, r_bits, d_ones, d_runs, stream));
}

tq_status tq_query_features(const tq_bitmap* inputs, uint32_t n, uint64_t r_bits, uint32_t theta, float* out) {
  if (!inputs || n == 0 || !out || r_bits == 0) return TQ_EINVAL;
  const double r = (double)r_bits;
  const double nw = (double)words_for_bits(r_bits);
  double dsum = 0.0, runlen = 0.0, ld_sum = 0.0, ld_sq = 0.0, comp = 0.0;
  for (uint32_t j = 0; j < n; ++j) {
    const double d = (double)inputs[j].ones / r;
    dsum += d;
    // runs alternate between zeros and ones: about half of them are runs of ones
    const double one_runs = std::max(1.0, (double)inputs[j].runs / 2.0);
    runlen += inputs[j].ones ? (double)inputs[j].ones / one_runs : 1.0;
    const double ld = log10(d + 1e-9);
    ld_sum += ld;
    ld_sq += ld * ld;
    comp += has_rle(inputs[j]) ? (double)inputs[j].rle.n_words : nw;
  }
  const double mean_ld = ld_sum / n;
  out[0] = (float)log2((double)n);
  out[1] = (float)((double)theta / n);
  out[2] = (float)log10(dsum / n + 1e-9);
  out[3] = (float)log10(std::max(1.0, runlen / n));
  out[4] = (float)sqrt(std::max(0.0, ld_sq / n - mean_ld * mean_ld));
  out[5] = (float)log2(r);
  out[6] = (float)log2(nw * n / std::max(1.0, comp));
  out[7] = (float)log2(std::max(1.0, (double)theta) / (1.0 + dsum));
  return TQ_OK;
}

tq_status tq_threshold_variant(tq_ctx* ctx, const tq_bitmap* inputs, uint32_t n, uint64_t r_bits,
                               uint32_t theta, uint32_t variant, uint64_t* d_out, hipStream_t stream) {
  if (!ctx || !inputs || n == 0) return TQ_EINVAL;
  if (variant >= TQ_SEL_VARIANTS) return TQ_EINVAL;
  if (!variant_available(inputs, n, (int)variant)) return TQ_EINVAL;
  std::vector<const uint64_t*> dense;
  std::vector<tq_rle> rle;
  switch (variant) {
    case TQ_VARIANT_CSA:
      csa_input_order(inputs, n, r_bits, theta, ctx->prune != 0, &dense);
      return tq_threshold(ctx, dense.data(), n, r_bits, theta, d_out, stream);
    case TQ_VARIANT_COUNTER: {
      for (uint32_t j = 0; j < n; ++j) dense.push_back(inputs[j].dense);
      if (n > TQ_MAX_INPUTS || !d_out || ((uintptr_t)d_out & 7)) return TQ_EINVAL;
      const uint64_t nw = words_for_bits(r_bits);
      for (uint32_t j = 0; j < n; ++j) {
        const uintptr_t p = (uintptr_t)dense[j];
        if (p & 7) return TQ_EINVAL;
        if (p < (uintptr_t)(d_out + nw) && (uintptr_t)d_out < p + nw * 8) return TQ_EINVAL;
      }
      if (nw == 0) return TQ_OK;
      if (theta == 0 || theta > n)
        return record_hip(ctx, launch_fill(d_out, nw, theta == 0 ? ~(uint64_t)0 : 0, tail_mask_for(r_bits), stream));
      Blob* pb = nullptr;
      const void* d_ptrs = blob_get(ctx, reinterpret_cast<const uint64_t*>(dense.data()), n, stream, &pb);
      if (!d_ptrs) return staging_error(ctx, TQ_EDEVICE);
      tq_status st = record_hip(ctx, launch_counter(reinterpret_cast<const uint64_t* const*>(d_ptrs), n, nw,
                                                    tail_mask_for(r_bits), theta, nullptr, d_out, stream));
      blob_used(ctx, pb, stream);
      return st;
    }
    case TQ_VARIANT_RLE:
      for (uint32_t j = 0; j < n; ++j) rle.push_back(inputs[j].rle);
      return tq_threshold_rle_dense(ctx, rle.data(), n, r_bits, theta, d_out, stream);
    default: {  // hybrid: each input in its smaller form
      const uint64_t nw = words_for_bits(r_bits);
      for (uint32_t j = 0; j < n; ++j) {
        const bool use_rle = has_rle(inputs[j]) && (!has_dense(inputs[j]) || inputs[j].rle.n_words < nw);
        if (use_rle) rle.push_back(inputs[j].rle);
        else dense.push_back(inputs[j].dense);
      }
      return tq_threshold_hybrid(ctx, rle.data(), (uint32_t)rle.size(), dense.data(), (uint32_t)dense.size(),
                                 r_bits, theta, d_out, stream);
    }
  }
}

uint64_t tq_selector_param_count(void) { return TQ_SEL_PARAMS; }

tq_status tq_selector_set(tq_ctx* ctx, const float* params, const float* feat_mean, const float* feat_std,
                          const float* feat_lo, const float* feat_hi, float margin) {
  if (!ctx || !params || !feat_mean || !feat_std || !feat_lo || !feat_hi) return TQ_EINVAL;
  Selector* s = static_cast<Selector*>(ctx->selector);
  if (!s) {
    s = new (std::nothrow) Selector();
    if (!s) return TQ_ENOMEM;
    ctx->selector = s;
  }
  s->params.assign(params, params + TQ_SEL_PARAMS);
  for (int i = 0; i < kIn; ++i) {
    if (!(feat_std[i] > 0.f)) return TQ_EINVAL;
    s->mean[i] = feat_mean[i];
    s->stdev[i] = feat_std[i];
    s->lo[i] = feat_lo[i];
    s->hi[i] = feat_hi[i];
  }
  s->margin = margin;
  s->ready = true;
  s->decided.clear();   // cells are defined by the normalisation just set
  return TQ_OK;
}

tq_status tq_selector_predict(tq_ctx* ctx, const float* features, float* predicted) {
  if (!ctx || !features || !predicted) return TQ_EINVAL;
  Selector* s = static_cast<Selector*>(ctx->selector);
  if (!s || !s->ready) return TQ_EINVAL;
  host_forward(*s, features, predicted);
  return TQ_OK;
}

tq_status tq_threshold_auto(tq_ctx* ctx, const tq_bitmap* inputs, uint32_t n, uint64_t r_bits, uint32_t theta,
                            uint64_t* d_out, uint32_t flags, uint32_t* chosen, hipStream_t stream) {
  if (!ctx || !inputs || n == 0) return TQ_EINVAL;
  // a query no variant can read (an input with neither form) is refused
  // whatever the flags, before any prediction or timing
  const uint32_t avail = variants_available(inputs, n);
  if (avail == 0) return TQ_EINVAL;
  Selector* s = static_cast<Selector*>(ctx->selector);
  float f[kIn], y[kOut];
  int best = -1, second = -1;
  bool uncertain = true;
  const bool have_f = r_bits > 0 && tq_query_features(inputs, n, r_bits, theta, f) == TQ_OK;
  if (s && s->ready && have_f) {
    host_forward(*s, f, y);
    for (int v = 0; v < kOut; ++v) {
      if (!variant_available(inputs, n, v)) continue;
      if (best < 0 || y[v] < y[best]) { second = best; best = v; }
      else if (second < 0 || y[v] < y[second]) second = v;
    }
    bool in_range = true;
    for (int i = 0; i < kIn; ++i) in_range &= (f[i] >= s->lo[i] && f[i] <= s->hi[i]);
    uncertain = !in_range || (second >= 0 && y[second] - y[best] < s->margin);
  }
  if (best < 0) {
    // no selector: the carry-save counter when dense words exist, else the hybrid
    best = variant_available(inputs, n, TQ_VARIANT_CSA) ? TQ_VARIANT_CSA : TQ_VARIANT_HYBRID;
    uncertain = true;
  }
  // the fallback times the variants and synchronises: not under stream capture
  if ((flags & TQ_AUTO_FALLBACK) && uncertain && !stream_capturing(stream)) {
    if (!s && have_f) {
      s = new (std::nothrow) Selector();   // holds the remembered decisions only
      ctx->selector = s;
    }
    const bool cache = s && have_f;
    const uint64_t key = cache ? decision_key(*s, f, avail) : 0;
    if (cache && !(flags & TQ_AUTO_RETIME)) {
      auto it = s->decided.find(key);
      if (it != s->decided.end() && ((avail >> it->second) & 1u)) {
        if (chosen) *chosen = (uint32_t)it->second | TQ_AUTO_CHOSE_BY_CACHE;
        return tq_threshold_variant(ctx, inputs, n, r_bits, theta, it->second, d_out, stream);
      }
    }
    // exhaustive fallback: time every available variant once on this query
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    };
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      release();
      return TQ_EDEVICE;
    }
    float best_ms = 0.f;
    int fastest = -1;
    for (int v = 0; v < kOut; ++v) {
      if (!variant_available(inputs, n, v)) continue;
      hipError_t e = hipEventRecord(e0, stream);
      tq_status st = e == hipSuccess ? tq_threshold_variant(ctx, inputs, n, r_bits, theta, (uint32_t)v, d_out, stream)
                                     : record_hip(ctx, e);
      if (st == TQ_OK) st = record_hip(ctx, hipEventRecord(e1, stream));
      if (st == TQ_OK) st = record_hip(ctx, hipEventSynchronize(e1));
      float ms = 0.f;
      if (st == TQ_OK) st = record_hip(ctx, hipEventElapsedTime(&ms, e0, e1));
      if (st != TQ_OK) {
        release();
        return st;
      }
      if (fastest < 0 || ms < best_ms) { best_ms = ms; fastest = v; }
    }
    release();
    if (cache && fastest >= 0) {
      if (s->decided.size() >= kMaxDecisions) s->decided.clear();
      s->decided[key] = (uint8_t)fastest;
    }
    if (chosen) *chosen = (uint32_t)fastest | TQ_AUTO_CHOSE_BY_TIMING;
    // every variant wrote the same bits into d_out; nothing more to run
    return TQ_OK;
  }
  if (chosen) *chosen = (uint32_t)best;
  return tq_threshold_variant(ctx, inputs, n, r_bits, theta, (uint32_t)best, d_out, stream);
}

tq_status tq_mlp_forward(tq_ctx* ctx, const float* d_params, const float* d_x, uint32_t batch, float* d_y,
                         hipStream_t stream) {
  if (!ctx || !d_params || (batch && (!d_x || !d_y))) return TQ_EINVAL;
  return record_hip(ctx, launch_mlp_forward(d_params, d_x, batch, d_y, stream));
}

tq_status tq_mlp_grad(tq_ctx* ctx, const float* d_params, const float* d_x, const float* d_t, const float* d_mask,
                      uint32_t batch, float mask_count, float* d_y, float* d_grad, float* d_loss,
                      hipStream_t stream) {
  if (!ctx || !d_params || !d_grad || batch == 0 || !d_x || !d_t || !(mask_count > 0.f)) return TQ_EINVAL;
  void* ws = workspace(ctx, mlp_grad_workspace_bytes(batch), stream);
  if (!ws) return staging_error(ctx, TQ_ENOMEM);
  return record_hip(ctx, launch_mlp_grad(d_params, d_x, d_t, d_mask, batch, 1.f / mask_count, d_y, d_grad, d_loss,
                                         ws, stream));
}

tq_status tq_mlp_adam(tq_ctx* ctx, float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t count,
                      float lr, float beta1, float beta2, float eps, uint32_t step, hipStream_t stream) {
  if (!ctx || !d_params || !d_grad || !d_m || !d_v || step == 0) return TQ_EINVAL;
  return record_hip(ctx, launch_adam(d_params, d_grad, d_m, d_v, count, lr, beta1, beta2, eps, step, stream));
}

}  // extern "C"
