// Autotuner for launch shapes.
//
// Every launch shape of a kernel family computes the same bits; only the
// time differs, and the best shape depends on the query's size (N, r), the
// epilogue, the threshold (pruning) and the part.  With TQ_OPTION_AUTOTUNE on,
// the first query of a shape class times every candidate shape on the
// caller's stream (a few launches each, HIP events) and caches the fastest in
// the context; later queries of the class look it up.  The cache can be
// exported as text and imported into another context.
//
// Shape classes: the kernel family, the counter width K, floor(log2 N),
// floor(log2 words), the epilogue kind, whether a pruned threshold runs and
// then theta's eighth of [0, N], and 16-byte alignment of the inputs.
#include <stdio.h>
#include <string.h>

#include <map>
#include <new>
#include <string>

#include "tq_internal.h"

namespace tq {

struct Tuner {
  std::map<uint64_t, TuneEntry> entries;
};

static Tuner* tuner(tq_ctx* ctx) {
  if (!ctx->tuner) ctx->tuner = new (std::nothrow) Tuner();
  return static_cast<Tuner*>(ctx->tuner);
}

void tuner_destroy(tq_ctx* ctx) {
  delete static_cast<Tuner*>(ctx->tuner);
  ctx->tuner = nullptr;
}

uint64_t tune_key(const TuneClass& c) {
  // 4 bits family, 5 bits K, 5 bits log n, 6 bits log words, 3 bits kind,
  // 1 bit pruned, 4 bits theta class, 1 bit alignment
  uint64_t k = (uint64_t)(c.family & 15);
  k = (k << 5) | (uint64_t)(c.K & 31);
  k = (k << 5) | (uint64_t)(c.log_n & 31);
  k = (k << 6) | (uint64_t)(c.log_words & 63);
  k = (k << 3) | (uint64_t)(c.kind & 7);
  k = (k << 1) | (uint64_t)(c.pruned & 1);
  k = (k << 4) | (uint64_t)(c.theta_class & 15);
  k = (k << 1) | (uint64_t)(c.aligned16 & 1);
  return k;
}

static TuneClass class_of(uint64_t k) {
  TuneClass c;
  c.aligned16 = (int)(k & 1); k >>= 1;
  c.theta_class = (int)(k & 15); k >>= 4;
  c.pruned = (int)(k & 1); k >>= 1;
  c.kind = (int)(k & 7); k >>= 3;
  c.log_words = (int)(k & 63); k >>= 6;
  c.log_n = (int)(k & 31); k >>= 5;
  c.K = (int)(k & 31); k >>= 5;
  c.family = (int)(k & 15);
  return c;
}

bool tune_lookup(tq_ctx* ctx, const TuneClass& c, TuneEntry* e) {
  Tuner* t = tuner(ctx);
  if (!t) return false;
  auto it = t->entries.find(tune_key(c));
  if (it == t->entries.end()) return false;
  *e = it->second;
  return true;
}

void tune_store(tq_ctx* ctx, const TuneClass& c, const TuneEntry& e) {
  Tuner* t = tuner(ctx);
  if (t) t->entries[tune_key(c)] = e;
}

bool stream_capturing(hipStream_t stream) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &st) != hipSuccess) return true;
  return st != hipStreamCaptureStatusNone;
}

float time_launches(hipStream_t stream, const std::function<hipError_t()>& launch, int reps) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return -1.f;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.f;
  }
  float ms = -1.f;
  bool ok = launch() == hipSuccess;   // warm-up
  ok = ok && hipEventRecord(e0, stream) == hipSuccess;
  for (int i = 0; ok && i < reps; ++i) ok = launch() == hipSuccess;
  ok = ok && hipEventRecord(e1, stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
  if (ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
    ms = ms * 1000.f / (float)reps;
  else
    ms = -1.f;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

}  // namespace tq

using namespace tq;

extern "C" {

tq_status tq_tune_export(tq_ctx* ctx, char* buf, size_t cap, size_t* len) {
  if (!ctx || !len || (cap && !buf)) return TQ_EINVAL;
  std::string s;
  Tuner* t = tuner(ctx);
  if (t) {
    char line[192];
    for (const auto& kv : t->entries) {
      const TuneClass c = class_of(kv.first);
      const TuneEntry& e = kv.second;
      snprintf(line, sizeof(line), "%d %d %d %d %d %d %d %d : %d %d %d %d : %.3f\n", c.family, c.K, c.log_n,
               c.log_words, c.kind, c.pruned, c.theta_class, c.aligned16, e.p[0], e.p[1], e.p[2], e.p[3], e.us);
      s += line;
    }
  }
  *len = s.size();
  if (cap == 0) return TQ_OK;
  if (cap < s.size() + 1) return TQ_ECAPACITY;
  memcpy(buf, s.c_str(), s.size() + 1);
  return TQ_OK;
}

tq_status tq_tune_import(tq_ctx* ctx, const char* text) {
  if (!ctx || !text) return TQ_EINVAL;
  std::map<uint64_t, TuneEntry> parsed;
  const char* p = text;
  while (*p) {
    const char* eol = strchr(p, '\n');
    const size_t n = eol ? (size_t)(eol - p) : strlen(p);
    std::string line(p, n);
    p += n + (eol ? 1 : 0);
    if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
    TuneClass c;
    TuneEntry e;
    int used = 0;
    if (sscanf(line.c_str(), "%d %d %d %d %d %d %d %d : %d %d %d %d : %f%n", &c.family, &c.K, &c.log_n,
               &c.log_words, &c.kind, &c.pruned, &c.theta_class, &c.aligned16, &e.p[0], &e.p[1], &e.p[2],
               &e.p[3], &e.us, &used) != 13)
      return TQ_EINVAL;
    if (line.find_first_not_of(" \t\r", (size_t)used) != std::string::npos) return TQ_EINVAL;
    if (!tune_entry_valid(c, e)) return TQ_EINVAL;
    parsed[tune_key(c)] = e;
  }
  Tuner* t = tuner(ctx);
  if (!t) return TQ_ENOMEM;
  for (const auto& kv : parsed) t->entries[kv.first] = kv.second;
  return TQ_OK;
}

tq_status tq_tune_clear(tq_ctx* ctx) {
  if (!ctx) return TQ_EINVAL;
  Tuner* t = tuner(ctx);
  if (t) t->entries.clear();
  return TQ_OK;
}

}  // extern "C"
