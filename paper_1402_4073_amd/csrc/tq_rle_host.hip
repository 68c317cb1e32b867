// Host side of the run-length-encoded calls: validation, index provisioning,
// workspace, and the kernel sequence of each call.
#include <string.h>

#include <vector>

#include "tq_internal.h"

namespace tq {

namespace {

__global__ void set_u64_kernel(uint64_t* dst, uint64_t v) { *dst = v; }

uint64_t index_entries(uint64_t nwords) { return (nwords + TQ_RLE_INDEX_STRIDE - 1) / TQ_RLE_INDEX_STRIDE; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

hipError_t launch_set_u64(uint64_t* d_dst, uint64_t value, hipStream_t stream) {
  hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(1), 0, stream, d_dst, value);
  return hipGetLastError();
}

void* workspace(tq_ctx* ctx, size_t bytes, hipStream_t stream) {
  const bool capturing = stream_capturing(stream);
  if (bytes <= ctx->ws_bytes && ctx->ws) {
    if (capturing) ctx->ws_frozen = true;   // a captured graph now refers to it
    return ctx->ws;
  }
  if (capturing) {   // no allocation under capture
    ctx->staging_status = TQ_EINVAL;
    return nullptr;
  }
  // the old buffer may still be read by queued work
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) { record_hip(ctx, e); return nullptr; }
  if (ctx->ws) {
    if (ctx->ws_frozen)
      ctx->ws_retired.push_back(ctx->ws);   // captured graphs still read it
    else
      (void)hipFree(ctx->ws);
  }
  ctx->ws = nullptr;
  ctx->ws_bytes = 0;
  ctx->ws_frozen = false;
  size_t want = align256(bytes + bytes / 4);
  if ((e = hipMalloc(&ctx->ws, want)) != hipSuccess) {
    record_hip(ctx, e);
    ctx->ws = nullptr;
    return nullptr;
  }
  ctx->ws_bytes = want;
  return ctx->ws;
}

tq_status staging_error(tq_ctx* ctx, tq_status dflt) {
  const tq_status st = ctx->staging_status;
  ctx->staging_status = TQ_OK;
  return st != TQ_OK ? st : dflt;
}

// Validate compressed inputs; counts those without an index.
tq_status check_rle_inputs(const tq_rle* inputs, uint32_t n, uint64_t nwords, uint32_t* missing_index) {
  *missing_index = 0;
  // the tile kernel keeps word positions in 32 bits
  if (nwords >= (1ull << 31)) return TQ_EINVAL;
  for (uint32_t j = 0; j < n; ++j) {
    const tq_rle& x = inputs[j];
    if (nwords > 0 && (!x.words || x.n_words == 0)) return TQ_EINVAL;
    if (x.n_words > kRleMaxWords) return TQ_EINVAL;
    if (((uintptr_t)x.words & 7) || ((uintptr_t)x.index & 7)) return TQ_EINVAL;
    if (!x.index) ++*missing_index;
  }
  return TQ_OK;
}

tq_status rle_describe(const tq_rle* inputs, uint32_t n_rle, uint64_t nwords, uint64_t* idx_area, uint64_t* desc,
                       std::vector<uint32_t>* missing) {
  const uint64_t nchk = index_entries(nwords);
  missing->clear();
  for (uint32_t j = 0; j < n_rle; ++j) {
    const uint64_t* index = inputs[j].index;
    if (!index) {
      if (!idx_area) return TQ_EINVAL;
      index = idx_area + (size_t)missing->size() * nchk * 2;
      missing->push_back(j);
    }
    desc[3 * j] = (uint64_t)(uintptr_t)inputs[j].words;
    desc[3 * j + 1] = inputs[j].n_words;
    desc[3 * j + 2] = (uint64_t)(uintptr_t)index;
  }
  return TQ_OK;
}

size_t rle_index_bytes(uint64_t nwords) { return (size_t)index_entries(nwords) * 16; }

namespace {

// Bytes of workspace needed for the indexes the caller did not supply.
tq_status missing_index_bytes(const tq_rle* inputs, uint32_t n_rle, uint64_t nw, size_t* bytes) {
  uint32_t missing = 0;
  tq_status st = check_rle_inputs(inputs, n_rle, nw, &missing);
  *bytes = align256((size_t)missing * index_entries(nw) * 16);
  return st;
}

// The function of a query over compressed inputs: a threshold, or (truth
// non-null) the symmetric function whose truth table is truth[0..n].
struct RleFn {
  uint32_t theta;
  const uint64_t* truth;
};

// Device tables of a symmetric function for the tile kernel (cached blobs).
struct SymTables {
  RleSym sym{};
  const RleSym* d_sym = nullptr;   // sym itself in device memory, for the kernel
  Blob* blobs[4] = {nullptr, nullptr, nullptr, nullptr};
};

tq_status sym_tables(tq_ctx* ctx, uint32_t n, const uint64_t* truth, const SymPlan& plan, hipStream_t stream,
                     SymTables* t) {
  const uint32_t fw = n / 64 + 1;
  std::vector<uint64_t> f(truth, truth + fw);
  if ((n + 1) % 64) f[fw - 1] &= ((uint64_t)1 << ((n + 1) % 64)) - 1;
  // run_end[c]: last count of the run of equal f values that starts at c
  std::vector<uint32_t> run_end(n + 2, 0);
  run_end[n] = n;
  for (uint32_t c = n; c-- > 0;) {
    const bool fc = (f[c / 64] >> (c % 64)) & 1, fn = (f[(c + 1) / 64] >> ((c + 1) % 64)) & 1;
    run_end[c] = fc == fn ? run_end[c + 1] : c;
  }
  std::vector<uint64_t> re64((n + 2) / 2, 0);
  memcpy(re64.data(), run_end.data(), (size_t)(n + 1) * 4);
  const void* d_f = blob_get(ctx, f.data(), f.size(), stream, &t->blobs[0]);
  const void* d_re = blob_get(ctx, re64.data(), re64.size(), stream, &t->blobs[1]);
  if (!d_f || !d_re) return staging_error(ctx, TQ_EDEVICE);
  t->sym.f = static_cast<const uint64_t*>(d_f);
  t->sym.run_end = static_cast<const uint32_t*>(d_re);
  t->sym.epi = plan.epi;
  uint32_t tail = n;
  while (tail > 0 && run_end[tail - 1] == n) --tail;
  t->sym.tail_from = tail;
  t->sym.tail_value = (uint32_t)((f[n / 64] >> (n % 64)) & 1);
  if (plan.epi.kind == EPI_TABLE) {
    std::vector<uint64_t> t64((plan.table.size() + 1) / 2, 0);
    memcpy(t64.data(), plan.table.data(), plan.table.size() * 4);
    const void* d_t = blob_get(ctx, t64.data(), t64.size(), stream, &t->blobs[2]);
    if (!d_t) return staging_error(ctx, TQ_EDEVICE);
    t->sym.epi.table = static_cast<const uint32_t*>(d_t);
  }
  // The kernel reads the plan from memory: passed by value it would take
  // some 30 scalar registers for the whole launch.  Every field is set and
  // the struct has no padding, so equal plans stage equal bytes.
  static_assert(sizeof(RleSym) % 8 == 0, "staged as whole words");
  uint64_t words[sizeof(RleSym) / 8];
  memcpy(words, &t->sym, sizeof(RleSym));
  const void* d_s = blob_get(ctx, words, sizeof(RleSym) / 8, stream, &t->blobs[3]);
  if (!d_s) return staging_error(ctx, TQ_EDEVICE);
  t->d_sym = static_cast<const RleSym*>(d_s);
  return TQ_OK;
}

// Tiles per workgroup of a query over compressed inputs: the tuned value of
// its shape class if the autotuner is on, else 0 (one range per resident
// workgroup).
struct RleShape {
  uint32_t tiles = 0;   // tiles per workgroup (0: one range per resident workgroup)
  bool swar = false;    // SWAR column counters instead of bit planes
};

// Default counters when nothing is tuned or forced: bit planes.  Measured on
// MI355X, SWAR counters cost 16 LDS atomics per literal word where bit planes
// take about two, which outweighs the round trips they save unless literal
// words hold few ones (isolated bits: about 5 % faster); the tuner weighs
// both per shape class.
bool default_swar(const RleFn&) { return false; }

RleShape rle_shape(tq_ctx* ctx, uint32_t n, uint64_t nw, const RleFn& qf, const SymPlan& plan,
                   const std::function<hipError_t(const RleShape&)>& launch, hipStream_t stream) {
  RleShape dflt;
  dflt.tiles = ctx->rle_tiles;
  dflt.swar = ctx->rle_counters ? ctx->rle_counters == 2 : default_swar(qf);
  if (!ctx->autotune || (ctx->rle_tiles && ctx->rle_counters)) return dflt;
  TuneClass c;
  c.family = kTuneRle;
  c.K = dense_planes_for(n);
  c.log_n = bit_length(n) - 1;
  c.log_words = bit_length(nw) - 1;
  c.kind = qf.truth ? 1 + plan.epi.kind : 0;
  c.theta_class = qf.truth ? 0 : (int)((8ull * qf.theta) / ((uint64_t)n + 1));
  TuneEntry e;
  if (tune_lookup(ctx, c, &e)) {
    RleShape t;
    t.tiles = ctx->rle_tiles ? ctx->rle_tiles : (uint32_t)e.p[0];
    t.swar = ctx->rle_counters ? ctx->rle_counters == 2 : e.p[1] == 2;
    return t;
  }
  if (stream_capturing(stream)) return dflt;
  static const uint32_t tiles[] = {0, 1, 2, 4, 16};
  RleShape best = dflt;
  float best_us = -1.f;
  for (int sw = 0; sw < 2; ++sw) {
    if (ctx->rle_counters && (ctx->rle_counters == 2) != (sw == 1)) continue;
    for (uint32_t t : tiles) {
      if (ctx->rle_tiles && t != ctx->rle_tiles) continue;
      RleShape cand;
      cand.tiles = t;
      cand.swar = sw == 1;
      const float us = time_launches(stream, [&]() { return launch(cand); }, 3);
      if (us > 0.f && (best_us < 0.f || us < best_us)) {
        best = cand;
        best_us = us;
      }
    }
  }
  if (best_us > 0.f) {
    e.p[0] = (int32_t)best.tiles;
    e.p[1] = best.swar ? 2 : 1;
    e.us = best_us;
    tune_store(ctx, c, e);
  }
  return best;
}

// Common part of the compressed-input queries: tile kernel into d_dense_out.
// idx_area: workspace for the indexes the caller did not supply (sized with
// missing_index_bytes), allocated by the caller before any pointer into the
// workspace is taken.
tq_status run_rle_tiles(tq_ctx* ctx, const tq_rle* inputs, uint32_t n_rle, const uint64_t* const* dense_ptrs,
                        uint32_t n_dense, uint64_t r_bits, const RleFn& qf, uint64_t* d_dense_out,
                        uint64_t* idx_area, hipStream_t stream, const Sink& sink = Sink(),
                        uint64_t* slots_used = nullptr) {
  const uint64_t nw = words_for_bits(r_bits);
  const uint64_t tmask = tail_mask_for(r_bits);
  const uint32_t n = n_rle + n_dense;
  SymPlan plan = qf.truth ? plan_symmetric(n, qf.truth) : plan_threshold(n, qf.theta);
  if (plan.constant) return record_hip(ctx, launch_fill(d_dense_out, nw, plan.const_word, tmask, stream));
  SymTables tabs;
  if (qf.truth) {
    tq_status st = sym_tables(ctx, n, qf.truth, plan, stream, &tabs);
    if (st != TQ_OK) return st;
  }
  std::vector<uint64_t> desc(3 * (size_t)(n_rle ? n_rle : 1), 0);
  // inputs without an index get one in idx_area, all built by one launch
  std::vector<uint32_t> missing;
  if (rle_describe(inputs, n_rle, nw, idx_area, desc.data(), &missing) != TQ_OK) return TQ_EINVAL;
  Blob* bd = nullptr;
  const void* d_desc = blob_get(ctx, desc.data(), desc.size(), stream, &bd);
  if (!d_desc) return staging_error(ctx, TQ_EDEVICE);
  tq_status st = TQ_OK;
  if (!missing.empty()) {
    std::vector<uint64_t> list64((missing.size() + 1) / 2, 0);
    memcpy(list64.data(), missing.data(), missing.size() * 4);
    Blob* bl = nullptr;
    const void* d_list = blob_get(ctx, list64.data(), list64.size(), stream, &bl);
    if (!d_list) return staging_error(ctx, TQ_EDEVICE);
    st = record_hip(ctx, launch_build_indexes(static_cast<const RleDesc*>(d_desc),
                                              static_cast<const uint32_t*>(d_list), (uint32_t)missing.size(), nw,
                                              ctx->d_status, stream));
    blob_used(ctx, bl, stream);
    if (st != TQ_OK) {
      blob_used(ctx, bd, stream);
      return st;
    }
  }
  Blob* bp = nullptr;
  const void* d_dense = nullptr;
  if (n_dense) {
    d_dense = blob_get(ctx, reinterpret_cast<const uint64_t*>(dense_ptrs), n_dense, stream, &bp);
    if (!d_dense) return staging_error(ctx, TQ_EDEVICE);
  }
  auto launch = [&](const RleShape& sh) {
    return launch_rle_tile(reinterpret_cast<const RleDesc*>(d_desc), n_rle,
                           reinterpret_cast<const uint64_t* const*>(d_dense), n_dense, nw, tmask, qf.theta,
                           qf.truth ? &tabs.sym : nullptr, qf.truth ? tabs.d_sym : nullptr, sh.swar,
                           ctx->num_cus, sh.tiles, d_dense_out,
                           ctx->d_status, stream, sink, slots_used);
  };
  st = record_hip(ctx, launch(rle_shape(ctx, n, nw, qf, plan, launch, stream)));
  blob_used(ctx, bd, stream);
  if (bp) blob_used(ctx, bp, stream);
  for (Blob* b : tabs.blobs)
    if (b) blob_used(ctx, b, stream);
  return st;
}

// Query with a dense result written to d_out; workspace holds only built indexes.
tq_status rle_query_dense(tq_ctx* ctx, const tq_rle* inputs, uint32_t n_rle, const uint64_t* const* dense_ptrs,
                          uint32_t n_dense, uint64_t r_bits, const RleFn& qf, uint64_t* d_out, hipStream_t stream) {
  const uint64_t nw = words_for_bits(r_bits);
  size_t idx_bytes = 0;
  tq_status st = missing_index_bytes(inputs, n_rle, nw, &idx_bytes);
  if (st != TQ_OK) return st;
  uint64_t* idx_area = nullptr;
  if (idx_bytes) {
    idx_area = static_cast<uint64_t*>(workspace(ctx, idx_bytes, stream));
    if (!idx_area) return staging_error(ctx, TQ_ENOMEM);
  }
  return run_rle_tiles(ctx, inputs, n_rle, dense_ptrs, n_dense, r_bits, qf, d_out, idx_area, stream);
}

// Dense-output query over compressed inputs (argument checks included).
tq_status rle_dense_entry(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits, const RleFn& qf,
                          uint64_t* d_out, hipStream_t stream) {
  if (!ctx || !inputs || n == 0 || n > TQ_RLE_MAX_INPUTS) return TQ_EINVAL;
  const uint64_t nw = words_for_bits(r_bits);
  if (nw >= (1ull << 31)) return TQ_EINVAL;
  if (nw == 0) return TQ_OK;
  if (!d_out || ((uintptr_t)d_out & 7)) return TQ_EINVAL;
  return rle_query_dense(ctx, inputs, n, nullptr, 0, r_bits, qf, d_out, stream);
}

tq_status hybrid_entry(tq_ctx* ctx, const tq_rle* rle_inputs, uint32_t n_rle, const uint64_t* const* dense_ptrs,
                       uint32_t n_dense, uint64_t r_bits, const RleFn& qf, uint64_t* d_out, hipStream_t stream) {
  if (!ctx || (n_rle && !rle_inputs) || (n_dense && !dense_ptrs)) return TQ_EINVAL;
  const uint64_t n = (uint64_t)n_rle + n_dense;
  if (n == 0 || n > TQ_RLE_MAX_INPUTS) return TQ_EINVAL;
  const uint64_t nw = words_for_bits(r_bits);
  if (nw >= (1ull << 31)) return TQ_EINVAL;
  if (nw == 0) return TQ_OK;
  if (!d_out || ((uintptr_t)d_out & 7)) return TQ_EINVAL;
  for (uint32_t j = 0; j < n_dense; ++j) {
    const uintptr_t p = (uintptr_t)dense_ptrs[j];
    if (!p || (p & 7)) return TQ_EINVAL;
    if (p < (uintptr_t)(d_out + nw) && (uintptr_t)d_out < p + nw * 8) return TQ_EINVAL;
  }
  return rle_query_dense(ctx, rle_inputs, n_rle, dense_ptrs, n_dense, r_bits, qf, d_out, stream);
}

// Dense query with fused consumers (filter AND, count) over compressed or
// hybrid inputs.
tq_status rle_fused_entry(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits, const RleFn& qf,
                          const uint64_t* d_filter, uint64_t* d_out, uint64_t* d_count, hipStream_t stream) {
  if (!ctx || !inputs || n == 0 || n > TQ_RLE_MAX_INPUTS) return TQ_EINVAL;
  const uint64_t nw = words_for_bits(r_bits);
  if (nw >= (1ull << 31)) return TQ_EINVAL;
  tq_status st = check_sink_args(r_bits, d_filter, d_out, d_count);
  if (st != TQ_OK) return st;
  if ((uintptr_t)d_out & 7) return TQ_EINVAL;
  if (nw == 0) return d_count ? record_hip(ctx, launch_set_u64(d_count, 0, stream)) : TQ_OK;
  size_t idx_bytes = 0;
  st = missing_index_bytes(inputs, n, nw, &idx_bytes);
  if (st != TQ_OK) return st;
  const SymPlan plan = qf.truth ? plan_symmetric(n, qf.truth) : plan_threshold(n, qf.theta);
  const uint64_t tmask = tail_mask_for(r_bits);
  Sink sink;
  sink.filter = d_filter;
  // partial counts: uint32 per 256-word block for a constant result, uint64
  // per wave of each tile-kernel workgroup otherwise
  const size_t part_bytes =
      !d_count ? 0 : align256(plan.constant ? fill_groups(nw) * sizeof(uint32_t) : rle_tile_partials(nw) * 8);
  // workspace: [partial counts | built indexes], sized before any pointer into it is taken
  char* ws = nullptr;
  if (part_bytes + idx_bytes) {
    ws = static_cast<char*>(workspace(ctx, part_bytes + idx_bytes, stream));
    if (!ws) return staging_error(ctx, TQ_ENOMEM);
  }
  if (plan.constant) {
    if (d_count) sink.partial = reinterpret_cast<uint32_t*>(ws);
    st = record_hip(ctx, launch_fill_sink(d_out, nw, plan.const_word, tmask, sink, stream));
    if (st == TQ_OK && d_count)
      st = record_hip(ctx, launch_count_reduce(sink.partial, fill_groups(nw), d_count, stream));
    return st;
  }
  if (d_count) sink.partial64 = reinterpret_cast<uint64_t*>(ws);
  uint64_t* idx_area = idx_bytes ? reinterpret_cast<uint64_t*>(ws + part_bytes) : nullptr;
  uint64_t slots = 0;
  st = run_rle_tiles(ctx, inputs, n, nullptr, 0, r_bits, qf, d_out, idx_area, stream, sink, &slots);
  if (st == TQ_OK && d_count) {
    const uint64_t* partial = sink.partial64;
    st = record_hip(ctx, launch_count_reduce(partial, slots, d_count, stream));
  }
  return st;
}

// Query with a canonical RLE result.
tq_status rle_rle_entry(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits, const RleFn& qf,
                        uint64_t* d_out, uint64_t out_cap_words, uint64_t* d_out_len, hipStream_t stream) {
  if (!ctx || !inputs || n == 0 || n > TQ_RLE_MAX_INPUTS || !d_out_len) return TQ_EINVAL;
  const uint64_t nw = words_for_bits(r_bits);
  if (nw >= (1ull << 31)) return TQ_EINVAL;
  if (nw == 0) return record_hip(ctx, launch_set_u64(d_out_len, 0, stream));
  if ((!d_out && out_cap_words) || ((uintptr_t)d_out & 7)) return TQ_EINVAL;
  // workspace: [dense result | encoder scratch | built indexes], sized once
  // before any pointer into it is taken
  const size_t dense_bytes = align256(nw * 8);
  const size_t enc_bytes = align256(rle_encode_workspace_bytes(nw));
  size_t idx_bytes = 0;
  tq_status st = missing_index_bytes(inputs, n, nw, &idx_bytes);
  if (st != TQ_OK) return st;
  char* ws = static_cast<char*>(workspace(ctx, dense_bytes + enc_bytes + idx_bytes, stream));
  if (!ws) return staging_error(ctx, TQ_ENOMEM);
  uint64_t* dense = reinterpret_cast<uint64_t*>(ws);
  uint64_t* idx_area = idx_bytes ? reinterpret_cast<uint64_t*>(ws + dense_bytes + enc_bytes) : nullptr;
  st = run_rle_tiles(ctx, inputs, n, nullptr, 0, r_bits, qf, dense, idx_area, stream);
  if (st != TQ_OK) return st;
  return record_hip(ctx, launch_rle_encode(dense, nw, tail_mask_for(r_bits), d_out, out_cap_words, d_out_len,
                                           nullptr, ws + dense_bytes, ctx->d_status, stream));
}

}  // namespace

}  // namespace tq

using namespace tq;

extern "C" {

uint64_t tq_rle_max_words(uint64_t r_bits) { return words_for_bits(r_bits) + 1; }

uint64_t tq_rle_index_words(uint64_t r_bits) { return 2 * index_entries(words_for_bits(r_bits)); }

tq_status tq_rle_encode(tq_ctx* ctx, const uint64_t* d_dense, uint64_t r_bits, uint64_t* d_out, uint64_t out_cap,
                        uint64_t* d_out_len, uint64_t* d_index, hipStream_t stream) {
  if (!ctx || !d_out_len) return TQ_EINVAL;
  const uint64_t nw = words_for_bits(r_bits);
  if (nw >= (1ull << 31)) return TQ_EINVAL;
  if (nw == 0) return record_hip(ctx, launch_set_u64(d_out_len, 0, stream));
  if (!d_dense || (!d_out && out_cap > 0)) return TQ_EINVAL;
  if (((uintptr_t)d_dense & 7) || ((uintptr_t)d_out & 7) || ((uintptr_t)d_index & 7)) return TQ_EINVAL;
  void* ws = workspace(ctx, rle_encode_workspace_bytes(nw), stream);
  if (!ws) return staging_error(ctx, TQ_ENOMEM);
  return record_hip(ctx, launch_rle_encode(d_dense, nw, tail_mask_for(r_bits), d_out, out_cap, d_out_len, d_index,
                                           ws, ctx->d_status, stream));
}

tq_status tq_rle_build_index(tq_ctx* ctx, const uint64_t* d_words, uint64_t n_words, uint64_t r_bits,
                             uint64_t* d_index, hipStream_t stream) {
  if (!ctx || !d_index || !d_words || n_words == 0) return TQ_EINVAL;
  const uint64_t nw = words_for_bits(r_bits);
  if (nw == 0 || nw >= (1ull << 31)) return TQ_EINVAL;
  if (((uintptr_t)d_words & 7) || ((uintptr_t)d_index & 7)) return TQ_EINVAL;
  return record_hip(ctx, launch_build_index(d_words, n_words, nw, d_index, ctx->d_status, stream));
}

tq_status tq_rle_decode(tq_ctx* ctx, const tq_rle* input, uint64_t r_bits, uint64_t* d_dense, hipStream_t stream) {
  if (!ctx || !input || !d_dense) return TQ_EINVAL;
  const uint64_t nw = words_for_bits(r_bits);
  if (nw >= (1ull << 31)) return TQ_EINVAL;
  if (nw == 0) return TQ_OK;
  if ((uintptr_t)d_dense & 7) return TQ_EINVAL;
  // the 1-threshold of a single input is the input itself
  return rle_query_dense(ctx, input, 1, nullptr, 0, r_bits, RleFn{1, nullptr}, d_dense, stream);
}

tq_status tq_threshold_rle_dense(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits, uint32_t theta,
                                 uint64_t* d_out, hipStream_t stream) {
  return rle_dense_entry(ctx, inputs, n, r_bits, RleFn{theta, nullptr}, d_out, stream);
}

tq_status tq_threshold_hybrid(tq_ctx* ctx, const tq_rle* rle_inputs, uint32_t n_rle, const uint64_t* const* dense_ptrs,
                              uint32_t n_dense, uint64_t r_bits, uint32_t theta, uint64_t* d_out, hipStream_t stream) {
  return hybrid_entry(ctx, rle_inputs, n_rle, dense_ptrs, n_dense, r_bits, RleFn{theta, nullptr}, d_out, stream);
}

tq_status tq_threshold_rle(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits, uint32_t theta,
                           uint64_t* d_out, uint64_t out_cap_words, uint64_t* d_out_len, hipStream_t stream) {
  return rle_rle_entry(ctx, inputs, n, r_bits, RleFn{theta, nullptr}, d_out, out_cap_words, d_out_len, stream);
}

tq_status tq_symmetric_rle_dense(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits,
                                 const uint64_t* h_truth, uint64_t* d_out, hipStream_t stream) {
  if (!h_truth) return TQ_EINVAL;
  return rle_dense_entry(ctx, inputs, n, r_bits, RleFn{0, h_truth}, d_out, stream);
}

tq_status tq_symmetric_hybrid(tq_ctx* ctx, const tq_rle* rle_inputs, uint32_t n_rle, const uint64_t* const* dense_ptrs,
                              uint32_t n_dense, uint64_t r_bits, const uint64_t* h_truth, uint64_t* d_out,
                              hipStream_t stream) {
  if (!h_truth) return TQ_EINVAL;
  return hybrid_entry(ctx, rle_inputs, n_rle, dense_ptrs, n_dense, r_bits, RleFn{0, h_truth}, d_out, stream);
}

tq_status tq_symmetric_rle(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits, const uint64_t* h_truth,
                           uint64_t* d_out, uint64_t out_cap_words, uint64_t* d_out_len, hipStream_t stream) {
  if (!h_truth) return TQ_EINVAL;
  return rle_rle_entry(ctx, inputs, n, r_bits, RleFn{0, h_truth}, d_out, out_cap_words, d_out_len, stream);
}

tq_status tq_threshold_rle_fused(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits, uint32_t theta,
                                 const uint64_t* d_filter, uint64_t* d_out, uint64_t* d_count, hipStream_t stream) {
  return rle_fused_entry(ctx, inputs, n, r_bits, RleFn{theta, nullptr}, d_filter, d_out, d_count, stream);
}

tq_status tq_symmetric_rle_fused(tq_ctx* ctx, const tq_rle* inputs, uint32_t n, uint64_t r_bits,
                                 const uint64_t* h_truth, const uint64_t* d_filter, uint64_t* d_out,
                                 uint64_t* d_count, hipStream_t stream) {
  if (!h_truth) return TQ_EINVAL;
  return rle_fused_entry(ctx, inputs, n, r_bits, RleFn{0, h_truth}, d_filter, d_out, d_count, stream);
}

}  // extern "C"
