// Batched queries: one persistent kernel serves many threshold / symmetric
// queries of uneven N, r and theta.
//
// A batch is uploaded as one packed buffer (header, query descriptors, the
// first work item of each query, all pointer arrays, truth tables, and the
// descriptors of compressed inputs).  The work of a dense-input query is cut
// into items of `groups` column groups (64 words each); item sizes grow as N
// shrinks so that every item streams about the same number of bytes.  Waves
// pop items from one atomic counter in increasing order, find the query of an
// item with a cursor that only moves forward, run the query's variant on each
// column group -- the register-resident carry-save counter of the
// single-query kernel, saturating counters for thresholds within 3 of either
// end (Looped), or packed per-position counters -- and write the output
// words.  The wave that finishes a query's last item writes the query's
// device timestamps and a done flag into coherent pinned host memory, so the
// host sees completions without waiting for the whole launch.
//
// Queries over compressed inputs (run-length tile merge, or the hybrid that
// reads each input in its smaller form) and the encoding of compressed
// results run after the persistent kernel on the same stream, each between
// two one-thread kernels that stamp its record.
//
// Admission counts bytes: a batch holds its packed buffer, its per-query
// records and counters, and the workspace of its compressed inputs and
// results until it is released, and the batches a context holds together
// stay within TQ_OPTION_BATCH_BYTES.  Each batch slot keeps its buffers (grown
// to the largest batch it served) and a graph built on them (copy of the
// packed buffer, the persistent kernel); a submission updates the copy size
// and replays it.
//
// A batch stops taking work items once the host cancels it (a flag in pinned
// host memory, read by every workgroup at each round) or once its deadline
// has passed on the device clock.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "tq_csa.hpp"
#include "tq_variants.hpp"

namespace tq {
namespace {

using namespace csa;

struct BatchHeader {
  uint32_t nq;           // queries served by the persistent kernel
  uint32_t total_items;
  uint32_t next;         // work counter
  uint32_t pad0;
  uint64_t off_queries;  // byte offsets inside the packed buffer
  uint64_t off_item_begin;
  uint64_t off_ptrs;
  uint64_t deadline;     // wall-clock ticks after the first workgroup starts (0: none)
  uint64_t t0;           // wall clock when the first workgroup started (0 until then)
  uint64_t pad1;
};

enum BatchPath : uint32_t { BP_CSA = 0, BP_LOOPED = 1, BP_COUNTER = 2 };
constexpr uint32_t QF_COMP = 1;    // Looped on the complemented inputs
constexpr uint32_t QF_DEFER = 2;   // completion is recorded after the query's encoding

struct BatchQuery {
  uint64_t ptrs;        // device address of this query's pointer array
  uint64_t out;
  uint64_t nwords;
  uint64_t tail_mask;
  uint32_t n;
  uint32_t K;           // BP_CSA: counter planes; BP_LOOPED: T; BP_COUNTER: counter width
  uint32_t groups;      // 64-word column groups per item
  uint32_t items;
  uint32_t item_begin;
  uint32_t constant;    // 0: compute, 1: all ones, 2: all zeros
  uint32_t path;        // BatchPath
  uint32_t flags;       // QF_*
  uint32_t rec;         // index of the query's record (submission order)
  uint32_t pad;
  EpiParams epi;
};

struct BatchRecord {    // in pinned host memory, one per query
  uint64_t t_start;
  uint64_t t_end;
  uint32_t done;
  int32_t status;
  uint64_t pad;
};

struct BatchCtl {       // in pinned host memory, one per slot
  uint32_t cancel;      // set by tq_batch_cancel
  uint32_t stopped;     // set by the kernel: 1 cancelled, 2 past the deadline
};

// record status written by the device for a query its batch did not complete
constexpr int32_t kStoppedStatus = -100;

constexpr int kBatchWavesPerCU = 16;
constexpr uint64_t kMinItemWork = 16;

// Completion of a query is counted on kShards sub-counters (item i of the
// query counts on shard i mod kShards) so that the items of one query, which
// tend to finish together, do not all hit one address; the item that fills a
// shard bumps the query's top counter, and the item that fills the last shard
// completes the query.  A counter that has reached its final value is set
// back to zero by the lane that saw it get there (nothing else touches it in
// this batch), so the next batch of the slot finds them all zero without a
// reset launch.  They are zeroed when the slot's arrays are created, and
// again before the next batch when a batch stopped early left some behind.
constexpr uint32_t kShards = 64;
// Batches of fewer queries are launched directly (copy + kernel) rather than
// by replaying the slot's graph: on this runtime a graph launch costs more
// host time than the two direct calls, which shows in the latency of small
// batches.
constexpr uint32_t kGraphMinQueries = 64;

// The packed batch is not written while the kernel runs (only the work
// counter and start time in its header are), so descriptors, item starts and
// pointer arrays are read through the constant address space: uniform reads
// become scalar loads instead of vector loads of one address.
#define TQ_CONST __attribute__((address_space(4)))
typedef const uint64_t* const TQ_CONST* CPtrArr;   // constant array of input pointers

template <typename T>
__device__ __forceinline__ const T TQ_CONST* as_const(const void* p) {
  return (const T TQ_CONST*)(p);
}

typedef const BatchQuery TQ_CONST CBatchQuery;

__device__ __forceinline__ void store_word(CBatchQuery& Q, uint64_t w, uint64_t v) {
  uint64_t* out = reinterpret_cast<uint64_t*>(Q.out);
  if (w < Q.nwords) out[w] = (w == Q.nwords - 1) ? (v & Q.tail_mask) : v;
}

// N >= 16: one column group (64 words) per wave, 16 inputs folded per step
template <int K>
__device__ __forceinline__ void run_group(CBatchQuery& Q, CPtrArr ptrs, uint64_t base, const uint32_t* table) {
  const int lane = threadIdx.x & 63;
  const uint64_t w = base + lane;
  Vec<1> r;
  if (Q.constant) {
    r.w[0] = Q.constant == 1 ? ~(uint64_t)0 : 0;
  } else {
    Vec<1> P[K];
#pragma unroll
    for (int k = 0; k < K; ++k) P[k].w[0] = 0;
    // a threshold item stops reading once its positions are decided, as in
    // the single-query kernel
    const bool prune = Q.epi.kind == EPI_THRESH && Q.epi.prune && Q.epi.theta >= 1 && Q.epi.theta <= Q.n;
    if (base + 64 <= Q.nwords) {
      if (prune)
        accumulate_pruned<K, 1, false>(P, ptrs, Q.n, w, Q.nwords, Q.epi.theta);
      else
        accumulate<K, 1, false>(P, ptrs, 0, Q.n, w, Q.nwords);
    } else {
      if (prune)
        accumulate_pruned<K, 1, true>(P, ptrs, Q.n, w, Q.nwords, Q.epi.theta);
      else
        accumulate<K, 1, true>(P, ptrs, 0, Q.n, w, Q.nwords);
    }
    r = epilogue<K, 1>(P, Q.epi, Q.n, table);
  }
  store_word(Q, w, r.w[0]);
}

// N <= 15: four interleaved column groups per wave (lane l owns words
// base + 64g + l), four inputs folded per step, so that a wave keeps as many
// loads in flight as with larger N
constexpr int kSmallGroups = 4;

__device__ __forceinline__ void run_small(CBatchQuery& Q, CPtrArr ptrs, uint64_t base, const uint32_t* table) {
  const int lane = threadIdx.x & 63;
  Vec<kSmallGroups> r;
  if (Q.constant) {
#pragma unroll
    for (int g = 0; g < kSmallGroups; ++g) r.w[g] = Q.constant == 1 ? ~(uint64_t)0 : 0;
  } else {
    Vec<kSmallGroups> P[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int g = 0; g < kSmallGroups; ++g) P[k].w[g] = 0;
    for (uint32_t i = 0; i < Q.n; i += 4) {
      Vec<kSmallGroups> x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool live = i + u < Q.n;
        const uint64_t* p = live ? ptrs[i + u] : nullptr;
#pragma unroll
        for (int g = 0; g < kSmallGroups; ++g) {
          const uint64_t w = base + (uint64_t)g * 64 + lane;
          x[u].w[g] = (live && w < Q.nwords) ? __builtin_nontemporal_load(p + w) : 0;
        }
      }
      add_block_l<2, 4, kSmallGroups>(P, x);
    }
    r = epilogue<4, kSmallGroups>(P, Q.epi, Q.n, table);
  }
#pragma unroll
  for (int g = 0; g < kSmallGroups; ++g) store_word(Q, base + (uint64_t)g * 64 + lane, r.w[g]);
}

// Thresholds within 3 of either end: saturating counters over the inputs or
// their complements (Looped, section 4.5; complement identity, section 2.3)
template <int T, bool Comp>
__device__ __forceinline__ void run_looped(CBatchQuery& Q, CPtrArr ptrs, uint64_t base) {
  const uint64_t w = base + (threadIdx.x & 63);
  const uint64_t valid = w < Q.nwords ? (w == Q.nwords - 1 ? Q.tail_mask : ~(uint64_t)0) : 0;
  uint64_t B[T];
#pragma unroll
  for (int t = 0; t < T; ++t) B[t] = 0;
  const bool prune = Q.epi.prune != 0;
  if (base + 64 <= Q.nwords)
    var::looped_accumulate<T, Comp, false>(B, ptrs, Q.n, w, Q.nwords, valid, prune);
  else
    var::looped_accumulate<T, Comp, true>(B, ptrs, Q.n, w, Q.nwords, valid, prune);
  store_word(Q, w, (Comp ? ~B[T - 1] : B[T - 1]) & valid);
}

// Per-position packed counters (ScanCount, section 4.2), thresholds
template <int W>
__device__ __forceinline__ void run_counter(CBatchQuery& Q, CPtrArr ptrs, uint64_t base) {
  const uint64_t w = base + (threadIdx.x & 63);
  uint64_t C[W];
#pragma unroll
  for (int k = 0; k < W; ++k) C[k] = 0;
  if (base + 64 <= Q.nwords)
    var::count_inputs<W, false>(C, ptrs, Q.n, w, Q.nwords);
  else
    var::count_inputs<W, true>(C, ptrs, Q.n, w, Q.nwords);
  store_word(Q, w, var::counter_word<W>(C, Q.epi.theta, nullptr));
}

__device__ __forceinline__ void run_item_group(CBatchQuery& Q, CPtrArr ptrs, uint64_t base, const uint32_t* table) {
  if (Q.path == BP_LOOPED && !Q.constant) {
    const bool comp = (Q.flags & QF_COMP) != 0;
    switch (Q.K) {
      case 1: comp ? run_looped<1, true>(Q, ptrs, base) : run_looped<1, false>(Q, ptrs, base); break;
      case 2: comp ? run_looped<2, true>(Q, ptrs, base) : run_looped<2, false>(Q, ptrs, base); break;
      default: comp ? run_looped<3, true>(Q, ptrs, base) : run_looped<3, false>(Q, ptrs, base); break;
    }
    return;
  }
  if (Q.path == BP_COUNTER && !Q.constant) {
    if (Q.K == 8) run_counter<8>(Q, ptrs, base);
    else run_counter<16>(Q, ptrs, base);
    return;
  }
  switch (Q.K) {
    case 4: run_small(Q, ptrs, base, table); break;
    case 5: run_group<5>(Q, ptrs, base, table); break;
    case 6: run_group<6>(Q, ptrs, base, table); break;
    case 7: run_group<7>(Q, ptrs, base, table); break;
    case 8: run_group<8>(Q, ptrs, base, table); break;
    case 9: run_group<9>(Q, ptrs, base, table); break;
    case 10: run_group<10>(Q, ptrs, base, table); break;
    case 11: run_group<11>(Q, ptrs, base, table); break;
    case 12: run_group<12>(Q, ptrs, base, table); break;
    case 13: run_group<13>(Q, ptrs, base, table); break;
    default: run_group<16>(Q, ptrs, base, table); break;
  }
}

// Whether the batch must stop taking work items: cancelled by the host, or
// past its deadline.  Records the reason for the host.
__device__ __forceinline__ bool batch_stop(uint32_t cancel, uint64_t deadline, uint64_t t0, BatchCtl* ctl) {
  uint32_t why = cancel ? 1u : 0u;
  if (!why && deadline && wall_clock64() - t0 > deadline) why = 2u;
  if (why) __hip_atomic_store(&ctl->stopped, why, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  return why != 0;
}

// A workgroup of kItemWaves waves takes kItemWaves consecutive items per
// round (one per wave).  Publishing a finished item needs a device-scope
// release, which on this part writes back the XCD's L2; doing it once per
// round for all the workgroup's items, from one instruction of wave 0, costs
// one write-back instead of one per wave.  The barrier orders every wave's
// output stores before that release.
constexpr int kItemWaves = 8;
// Truth tables (arbitrary symmetric functions) of up to this many 32-bit
// words, i.e. counters of up to 11 bits (n < 2048), are staged in LDS by the
// wave that uses them; larger ones are read from the packed batch.
constexpr uint32_t kWaveTableWords = 64;

__global__ __launch_bounds__(64 * kItemWaves) void batch_kernel(char* buf, uint32_t* qshard, uint32_t* qtop,
                                                               uint32_t* qcomplete, BatchRecord* rec,
                                                               BatchCtl* ctl) {
  __shared__ uint32_t s_q[kItemWaves];
  __shared__ uint32_t s_local[kItemWaves];
  __shared__ uint32_t s_next;
  __shared__ uint64_t s_t0;
  __shared__ uint32_t s_table[kItemWaves][kWaveTableWords];
  BatchHeader* hdr = reinterpret_cast<BatchHeader*>(buf);
  const BatchHeader TQ_CONST* chdr = as_const<BatchHeader>(buf);
  const BatchQuery TQ_CONST* qs = as_const<BatchQuery>(buf + chdr->off_queries);
  const uint32_t TQ_CONST* item_begin = as_const<uint32_t>(buf + chdr->off_item_begin);
  const uint32_t nq = chdr->nq, total = chdr->total_items;
  const uint64_t deadline = chdr->deadline;
  const uint32_t nrounds = (total + kItemWaves - 1) / kItemWaves;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // the batch's start time (the first workgroup to get here sets it) and a
  // first look at the cancel flag
  if (threadIdx.x == 0) {
    const uint64_t now = wall_clock64();
    const uint64_t old = atomicCAS(reinterpret_cast<unsigned long long*>(&hdr->t0), 0ull,
                                   (unsigned long long)now);
    s_t0 = old ? old : now;
    const uint32_t cancel = __hip_atomic_load(&ctl->cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    s_next = batch_stop(cancel, deadline, s_t0, ctl) ? nrounds : blockIdx.x;
  }
  __syncthreads();
  const uint64_t t0 = s_t0;
  uint32_t q = 0;
  uint32_t staged = 0xFFFFFFFFu;   // query whose truth table this wave holds in s_table
  // the first round of every workgroup is its own index; later ones come from the counter
  uint32_t round = s_next;
  while (round < nrounds) {
    // the cancel flag for the end of this round, read now so that the trip
    // to host memory overlaps the round's work
    uint32_t cancel = 0;
    if (threadIdx.x == 0) cancel = __hip_atomic_load(&ctl->cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    const uint32_t item = round * kItemWaves + wave;
    uint32_t my_q = 0xFFFFFFFFu, my_local = 0;
    if (item < total) {
      // items of a wave come in increasing order: move the cursor forward
      if (q + 1 < nq && item_begin[q + 1] <= item) {
        uint32_t lo = q + 1, hi = nq - 1;
        while (lo < hi) {
          const uint32_t mid = (lo + hi + 1) / 2;
          if (item_begin[mid] <= item) lo = mid; else hi = mid - 1;
        }
        q = lo;
      }
      CBatchQuery& Q = qs[q];
      const uint64_t local = item - Q.item_begin;
      if (lane == 0 && local == 0) rec[Q.rec].t_start = wall_clock64();
      CPtrArr ptrs = as_const<const uint64_t*>(reinterpret_cast<const void*>(Q.ptrs));
      const uint32_t* table = nullptr;
      if (!Q.constant && Q.epi.kind == EPI_TABLE) {
        table = Q.epi.table;
        if (Q.epi.table_words <= kWaveTableWords) {
          if (staged != q) {
            for (uint32_t t = lane; t < Q.epi.table_words; t += 64) s_table[wave][t] = table[t];
            // the other lanes of this wave read what this wave wrote
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            staged = q;
          }
          table = s_table[wave];
        }
      }
      const uint32_t step = (Q.path == BP_CSA && Q.K == 4) ? kSmallGroups : 1;
      for (uint32_t g = 0; g < Q.groups; g += step) {
        const uint64_t base = (local * Q.groups + g) * 64;
        if (base >= Q.nwords) break;
        run_item_group(Q, ptrs, base, table);
      }
      my_q = q;
      my_local = (uint32_t)local;
    }
    if (lane == 0) {
      s_q[wave] = my_q;
      s_local[wave] = my_local;
    }
    __syncthreads();
    if (wave == 0) {
      if (lane < kItemWaves && s_q[lane] != 0xFFFFFFFFu) {
        const uint32_t qq = s_q[lane];
        const uint32_t items = qs[qq].items;
        const uint32_t shard = s_local[lane] % kShards;
        const uint32_t nshards = items < kShards ? items : kShards;
        const uint32_t shard_items = (items - shard + kShards - 1) / kShards;
        uint32_t* sc = &qshard[(uint64_t)qq * kShards + shard];
        bool last = __hip_atomic_fetch_add(sc, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1 == shard_items;
        if (last) {
          __hip_atomic_store(sc, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          last = __hip_atomic_fetch_add(&qtop[qq], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1 == nshards;
          if (last) __hip_atomic_store(&qtop[qq], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (last) {
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
          const uint32_t r = qs[qq].rec;
          if (qs[qq].flags & QF_DEFER) {
            // the encoder that follows completes the record
            __hip_atomic_store(&qcomplete[r], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
          } else {
            rec[r].t_end = wall_clock64();
            rec[r].status = 0;
            __hip_atomic_store(&rec[r].done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
          }
        }
      }
      if (lane == 0) {
        if (batch_stop(cancel, deadline, t0, ctl))
          s_next = nrounds;
        else
          s_next = nrounds > gridDim.x ? gridDim.x + atomicAdd(&hdr->next, 1u) : nrounds;
      }
    }
    __syncthreads();
    round = s_next;
  }
}

// Record stamps around the work of a query that runs after the persistent
// kernel.  end: the query's status (a deferred query the kernel did not
// complete is reported stopped), its end time and done flag; the status slot
// and completion flag are cleared for the slot's next batch.
__global__ void batch_mark_kernel(BatchRecord* rec, uint32_t* qcomplete, int32_t* qstatus, uint32_t r,
                                  uint32_t end, uint32_t deferred) {
  if (!end) {
    rec[r].t_start = wall_clock64();
    return;
  }
  int32_t st = qstatus[r];
  if (deferred && !__hip_atomic_load(&qcomplete[r], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) st = kStoppedStatus;
  qstatus[r] = 0;
  qcomplete[r] = 0;
  rec[r].t_end = wall_clock64();
  rec[r].status = st;
  __hip_atomic_store(&rec[r].done, st == kStoppedStatus ? 0u : 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void zero_u32_kernel(uint32_t* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t pow2_at_least(size_t x, size_t lo) {
  size_t c = lo;
  while (c < x) c <<= 1;
  return c;
}

}  // namespace

struct BatchSlot {
  bool in_use = false;
  bool dirty = false;          // completion counters may be non-zero (a batch stopped early)
  char* d_buf = nullptr;       // packed batch (device)
  char* h_buf = nullptr;       // packed batch (pinned staging)
  size_t buf_cap = 0;
  uint32_t q_cap = 0;          // queries the per-query arrays hold
  uint32_t* d_qarr = nullptr;  // q_cap x (kShards shard counters), q_cap top counters, q_cap
                               // completion flags, q_cap int32 statuses
  BatchRecord* h_rec = nullptr;  // pinned, coherent, written by the GPU
  BatchRecord* d_rec = nullptr;  // device view of h_rec
  BatchCtl* h_ctl = nullptr;
  BatchCtl* d_ctl = nullptr;
  char* d_ws = nullptr;        // workspace of compressed inputs and results
  size_t ws_cap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t copy_node = nullptr;
  hipEvent_t done_ev = nullptr;
  size_t held = 0;             // bytes counted against the admission limit while in use

  uint32_t* qshard() const { return d_qarr; }
  uint32_t* qtop() const { return d_qarr + (size_t)q_cap * kShards; }
  uint32_t* qcomplete() const { return qtop() + q_cap; }
  int32_t* qstatus() const { return reinterpret_cast<int32_t*>(qcomplete() + q_cap); }
  size_t qarr_words() const { return (size_t)q_cap * (kShards + 3); }
  size_t allocated() const {
    return buf_cap + qarr_words() * 4 + (size_t)q_cap * sizeof(BatchRecord) + ws_cap;
  }
};

struct BatchState {
  BatchSlot slots[TQ_BATCH_MAX_INFLIGHT];
  int grid = 0;
  double tick_ns = 10.0;
  // word-column schedule: items per wave of the grid the work is cut into,
  // and the smallest item (in 64-word group-inputs); set by tq_batch_tune
  uint32_t items_per_wave = 4;
  uint32_t min_item_work = (uint32_t)kMinItemWork;
};

}  // namespace tq

struct tq_batch {
  tq_ctx* ctx;
  int slot;
  uint32_t nq;
  std::vector<uint64_t> tags;
  std::vector<uint8_t> variants;
};

namespace tq {
namespace {

BatchState* batch_state(tq_ctx* ctx) {
  if (!ctx->batch) {
    BatchState* b = new (std::nothrow) BatchState();
    if (!b) return nullptr;
    b->grid = ctx->num_cus * kBatchWavesPerCU / kItemWaves;   // workgroups of kItemWaves waves
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, ctx->device) == hipSuccess && rate_khz > 0)
      b->tick_ns = 1e6 / (double)rate_khz;
    ctx->batch = b;
  }
  return static_cast<BatchState*>(ctx->batch);
}

void free_graph(BatchSlot& s) {
  if (s.exec) (void)hipGraphExecDestroy(s.exec);
  if (s.graph) (void)hipGraphDestroy(s.graph);
  s.exec = nullptr;
  s.graph = nullptr;
  s.copy_node = nullptr;
}

// Frees the buffers of an idle slot (its last batch has been waited for).
void free_slot_memory(BatchSlot& s) {
  free_graph(s);
  if (s.d_buf) (void)hipFree(s.d_buf);
  if (s.h_buf) (void)hipHostFree(s.h_buf);
  if (s.d_qarr) (void)hipFree(s.d_qarr);
  if (s.h_rec) (void)hipHostFree(s.h_rec);
  if (s.d_ws) (void)hipFree(s.d_ws);
  s.d_buf = nullptr;
  s.h_buf = nullptr;
  s.d_qarr = nullptr;
  s.h_rec = nullptr;
  s.d_rec = nullptr;
  s.d_ws = nullptr;
  s.buf_cap = 0;
  s.q_cap = 0;
  s.ws_cap = 0;
}

// Buffers of a slot of at least the given sizes.  A slot's buffers only
// grow; a grown packed buffer or per-query array needs a new graph, and new
// per-query arrays are zeroed (on the stream) before first use.
tq_status slot_reserve(tq_ctx* ctx, BatchState* bs, BatchSlot& s, size_t buf_bytes, uint32_t queries,
                       size_t ws_bytes, hipStream_t stream) {
  hipError_t e;
  if (!s.done_ev && (e = hipEventCreateWithFlags(&s.done_ev, hipEventDisableTiming)) != hipSuccess)
    return record_hip(ctx, e);
  if (!s.h_ctl) {
    if ((e = hipHostMalloc((void**)&s.h_ctl, sizeof(BatchCtl), hipHostMallocMapped | hipHostMallocCoherent)) !=
        hipSuccess)
      return record_hip(ctx, e);
    if ((e = hipHostGetDevicePointer((void**)&s.d_ctl, s.h_ctl, 0)) != hipSuccess) return record_hip(ctx, e);
    memset(s.h_ctl, 0, sizeof(BatchCtl));
  }
  bool regraph = !s.exec;
  if (buf_bytes > s.buf_cap) {
    free_graph(s);
    if (s.d_buf) (void)hipFree(s.d_buf);
    if (s.h_buf) (void)hipHostFree(s.h_buf);
    s.d_buf = nullptr;
    s.h_buf = nullptr;
    s.buf_cap = 0;
    const size_t cap = pow2_at_least(buf_bytes, 64 << 10);
    if ((e = hipMalloc((void**)&s.d_buf, cap)) != hipSuccess) return record_hip(ctx, e);
    if ((e = hipHostMalloc((void**)&s.h_buf, cap, hipHostMallocDefault)) != hipSuccess) return record_hip(ctx, e);
    s.buf_cap = cap;
    regraph = true;
  }
  if (queries > s.q_cap) {
    free_graph(s);
    if (s.d_qarr) (void)hipFree(s.d_qarr);
    if (s.h_rec) (void)hipHostFree(s.h_rec);
    s.d_qarr = nullptr;
    s.h_rec = nullptr;
    s.d_rec = nullptr;
    s.q_cap = 0;
    const uint32_t cap = (uint32_t)pow2_at_least(queries, 64);
    if ((e = hipMalloc((void**)&s.d_qarr, (size_t)cap * (kShards + 3) * 4)) != hipSuccess) return record_hip(ctx, e);
    if ((e = hipHostMalloc((void**)&s.h_rec, (size_t)cap * sizeof(BatchRecord),
                           hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
      return record_hip(ctx, e);
    if ((e = hipHostGetDevicePointer((void**)&s.d_rec, s.h_rec, 0)) != hipSuccess) return record_hip(ctx, e);
    s.q_cap = cap;
    s.dirty = true;   // fresh counters are zeroed before the batch
    regraph = true;
  }
  if (ws_bytes > s.ws_cap) {
    if (s.d_ws) (void)hipFree(s.d_ws);
    s.d_ws = nullptr;
    s.ws_cap = 0;
    const size_t cap = pow2_at_least(ws_bytes, 1 << 20);
    if ((e = hipMalloc((void**)&s.d_ws, cap)) != hipSuccess) return record_hip(ctx, e);
    s.ws_cap = cap;
  }
  if (regraph) {
    // graph: copy the packed buffer, run the persistent kernel
    free_graph(s);
    if ((e = hipGraphCreate(&s.graph, 0)) != hipSuccess) return record_hip(ctx, e);
    if ((e = hipGraphAddMemcpyNode1D(&s.copy_node, s.graph, nullptr, 0, s.d_buf, s.h_buf, sizeof(BatchHeader),
                                     hipMemcpyHostToDevice)) != hipSuccess)
      return record_hip(ctx, e);
    // kernel parameter values are copied when the node is created
    char* buf = s.d_buf;
    uint32_t* qsh = s.qshard();
    uint32_t* qt = s.qtop();
    uint32_t* qc = s.qcomplete();
    BatchRecord* rec = s.d_rec;
    BatchCtl* ctl = s.d_ctl;
    hipGraphNode_t kernel_node;
    void* kargs[6] = {&buf, &qsh, &qt, &qc, &rec, &ctl};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(batch_kernel);
    kp.gridDim = dim3(bs->grid);
    kp.blockDim = dim3(64 * kItemWaves);
    kp.sharedMemBytes = 0;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    if ((e = hipGraphAddKernelNode(&kernel_node, s.graph, &s.copy_node, 1, &kp)) != hipSuccess)
      return record_hip(ctx, e);
    if ((e = hipGraphInstantiate(&s.exec, s.graph, nullptr, nullptr, 0)) != hipSuccess) return record_hip(ctx, e);
  }
  if (s.dirty) {
    const uint64_t words = s.qarr_words();
    const uint32_t grid = (uint32_t)std::min<uint64_t>(1024, (words + 255) / 256);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(grid), dim3(256), 0, stream, s.d_qarr, words);
    if ((e = hipGetLastError()) != hipSuccess) return record_hip(ctx, e);
    s.dirty = false;
  }
  return TQ_OK;
}

// How one query of a batch runs.
struct QueryPlan {
  bool in_kernel = true;    // served by the persistent kernel
  int variant = TQ_VARIANT_CSA;
  uint32_t path = BP_CSA;
  uint32_t K = 0;
  uint32_t flags = 0;
  SymPlan plan;
  std::vector<const uint64_t*> dense;   // dense inputs in reading order (in-kernel, hybrid)
  std::vector<tq_rle> rle;              // compressed inputs (RLE, hybrid)
  uint32_t missing_index = 0;
  size_t dense_tmp = 0;                 // dense result bytes held in workspace (compressed result)
  size_t tail_ws = 0;                   // workspace of its work after the kernel
};

// Validates one query and decides how it runs.
tq_status plan_query(tq_ctx* ctx, const tq_query& q, QueryPlan* p) {
  if (q.kind != TQ_QUERY_THRESHOLD && q.kind != TQ_QUERY_SYMMETRIC) return TQ_EINVAL;
  if (q.n == 0 || q.n > TQ_MAX_INPUTS) return TQ_EINVAL;
  if ((q.ptrs == nullptr) == (q.inputs == nullptr)) return TQ_EINVAL;
  if (q.kind == TQ_QUERY_SYMMETRIC && !q.h_truth) return TQ_EINVAL;
  const uint64_t nw = words_for_bits(q.r_bits);
  if (nw >= (1ull << 31)) return TQ_EINVAL;
  const bool rle_out = q.out_cap > 0;
  if (rle_out) {
    if (!q.d_out || ((uintptr_t)q.d_out & 7) || !q.d_out_len || ((uintptr_t)q.d_out_len & 7)) return TQ_EINVAL;
  } else {
    if (!q.d_out || ((uintptr_t)q.d_out & 7)) return TQ_EINVAL;
  }
  const bool thresh = q.kind == TQ_QUERY_THRESHOLD;
  if (q.ptrs) {
    if (q.variant != TQ_VARIANT_CSA && q.variant != TQ_VARIANT_COUNTER) return TQ_EINVAL;
    p->variant = (int)q.variant;
    p->dense.assign(q.ptrs, q.ptrs + q.n);
  } else {
    const tq_bitmap* in = q.inputs;
    const uint32_t avail = variants_available(in, q.n);
    if (avail == 0) return TQ_EINVAL;
    if (q.variant == TQ_VARIANT_AUTO) {
      if (thresh) {
        p->variant = select_variant(ctx, in, q.n, q.r_bits, q.theta, avail);
      } else {
        if (!(avail & (1u << TQ_VARIANT_CSA))) return TQ_ENOTSUP;
        p->variant = TQ_VARIANT_CSA;
      }
    } else {
      if (q.variant >= TQ_SEL_VARIANTS) return TQ_EINVAL;
      if (!((avail >> q.variant) & 1u)) return TQ_EINVAL;
      p->variant = (int)q.variant;
    }
    switch (p->variant) {
      case TQ_VARIANT_CSA:
        csa_input_order(in, q.n, q.r_bits, thresh ? q.theta : 0, thresh && ctx->prune != 0, &p->dense);
        break;
      case TQ_VARIANT_COUNTER:
        for (uint32_t j = 0; j < q.n; ++j) p->dense.push_back(in[j].dense);
        break;
      case TQ_VARIANT_RLE:
        for (uint32_t j = 0; j < q.n; ++j) p->rle.push_back(in[j].rle);
        break;
      default:   // hybrid: each input in its smaller form
        for (uint32_t j = 0; j < q.n; ++j) {
          const bool has_r = in[j].rle.words && in[j].rle.n_words > 0;
          if (has_r && (!in[j].dense || in[j].rle.n_words < nw)) p->rle.push_back(in[j].rle);
          else p->dense.push_back(in[j].dense);
        }
        break;
    }
  }
  if (p->variant == TQ_VARIANT_COUNTER && !thresh) return TQ_EINVAL;
  for (const uint64_t* d : p->dense) {
    const uintptr_t a = (uintptr_t)d;
    if (!a || (a & 7)) return TQ_EINVAL;
    if (!rle_out && a < (uintptr_t)(q.d_out + nw) && (uintptr_t)q.d_out < a + nw * 8) return TQ_EINVAL;
  }
  try {
    p->plan = thresh ? plan_threshold(q.n, q.theta) : plan_symmetric(q.n, q.h_truth);
  } catch (const std::bad_alloc&) {
    return TQ_ENOMEM;
  }
  p->in_kernel = p->variant == TQ_VARIANT_CSA || p->variant == TQ_VARIANT_COUNTER;
  if (!p->in_kernel) {
    if (!thresh) return TQ_ENOTSUP;
    if (q.n > TQ_RLE_MAX_INPUTS) return TQ_EINVAL;
    tq_status st = check_rle_inputs(p->rle.data(), (uint32_t)p->rle.size(), nw, &p->missing_index);
    if (st != TQ_OK) return st;
  }
  if (p->in_kernel && !p->plan.constant) {
    uint32_t lt = 0;
    bool lcomp = false;
    if (p->variant == TQ_VARIANT_COUNTER) {
      p->path = BP_COUNTER;
      p->K = q.n <= 255 ? 8 : 16;
    } else if (ctx->looped && p->plan.epi.kind == EPI_THRESH && !p->plan.epi.invert &&
               looped_applies(q.n, p->plan.epi.theta, &lt, &lcomp)) {
      p->path = BP_LOOPED;
      p->K = lt;
      p->flags |= lcomp ? QF_COMP : 0;
    } else {
      p->path = BP_CSA;
      p->K = (uint32_t)dense_planes_for(q.n);
    }
  } else {
    p->path = BP_CSA;
    p->K = (uint32_t)dense_planes_for(q.n);
  }
  // workspace: a compressed result is computed dense into workspace, then
  // encoded; missing indexes of compressed inputs are built into workspace
  if (rle_out && nw > 0) {
    p->dense_tmp = align_up(nw * 8, 256);
    p->tail_ws = align_up(rle_encode_workspace_bytes(nw), 256);
  }
  if (!p->in_kernel) p->tail_ws += align_up((size_t)p->missing_index * rle_index_bytes(nw), 256);
  if (p->in_kernel && rle_out) p->flags |= QF_DEFER;
  return TQ_OK;
}

}  // namespace

void batch_destroy(tq_ctx* ctx) {
  BatchState* bs = static_cast<BatchState*>(ctx->batch);
  if (!bs) return;
  for (auto& s : bs->slots) {
    if (s.done_ev) (void)hipEventSynchronize(s.done_ev);
    free_slot_memory(s);
    if (s.done_ev) (void)hipEventDestroy(s.done_ev);
    if (s.h_ctl) (void)hipHostFree(s.h_ctl);
  }
  delete bs;
  ctx->batch = nullptr;
}

}  // namespace tq

using namespace tq;

namespace {

// Status of a record as the caller sees it.
int32_t public_status(const BatchRecord& r, uint32_t stopped, bool finished) {
  const uint32_t done = __atomic_load_n(&r.done, __ATOMIC_ACQUIRE);
  if (done) return r.status;
  if (r.status == kStoppedStatus || finished) {
    if (stopped == 1) return TQ_ECANCELED;
    if (stopped == 2) return TQ_ETIMEDOUT;
  }
  return 0;
}

}  // namespace

extern "C" {

tq_status tq_batch_submit(tq_ctx* ctx, const tq_query* queries, uint32_t count, uint32_t flags,
                          hipStream_t stream, tq_batch** out) {
  if (!ctx || !out || (count && !queries)) return TQ_EINVAL;
  *out = nullptr;
  // a batch replays its slot's own graph and reports through host memory:
  // it cannot be captured into another graph
  if (stream_capturing(stream)) return TQ_EINVAL;
  if (count == 0 || count > TQ_BATCH_MAX_QUERIES) return TQ_EINVAL;
  BatchState* bs = batch_state(ctx);
  if (!bs) return TQ_ENOMEM;
  // validate and plan every query
  std::vector<QueryPlan> plans;
  try {
    plans.resize(count);
  } catch (const std::bad_alloc&) {
    return TQ_ENOMEM;
  }
  uint64_t nptrs = 0, table_bytes = 0, ndesc = 0, nlist = 0;
  size_t ws_kernel = 0, ws_tail = 0;
  uint32_t nk = 0;
  for (uint32_t i = 0; i < count; ++i) {
    tq_status st = plan_query(ctx, queries[i], &plans[i]);
    if (st != TQ_OK) return st;
    const QueryPlan& p = plans[i];
    nptrs += p.dense.size();
    ndesc += p.rle.size();
    nlist += p.missing_index;
    if (!p.plan.constant && p.plan.epi.kind == EPI_TABLE) table_bytes += align_up(p.plan.table.size() * 4, 8);
    if (p.in_kernel) {
      ++nk;
      ws_kernel += p.dense_tmp;
      ws_tail = std::max(ws_tail, p.tail_ws);
    } else {
      ws_tail = std::max(ws_tail, p.dense_tmp + p.tail_ws);
    }
  }
  if (nptrs > TQ_BATCH_MAX_POINTERS) return TQ_EINVAL;
  if (table_bytes > TQ_BATCH_MAX_TABLE_BYTES) return TQ_EINVAL;

  // pack: header | queries | item_begin | pointer arrays | tables | compressed-input descriptors | index lists
  const size_t off_q = align_up(sizeof(BatchHeader), 256);
  const size_t off_ib = align_up(off_q + (size_t)nk * sizeof(BatchQuery), 256);
  const size_t off_p = align_up(off_ib + (size_t)nk * 4, 256);
  const size_t off_t = align_up(off_p + nptrs * 8, 256);
  const size_t off_d = align_up(off_t + table_bytes, 256);
  const size_t off_l = align_up(off_d + ndesc * sizeof(RleDesc), 256);
  const size_t used = align_up(off_l + nlist * 4, 256);
  const size_t ws_bytes = ws_kernel + ws_tail;

  // admission by bytes
  const size_t need = used + ws_bytes + (size_t)count * (sizeof(BatchRecord) + (kShards + 3) * 4);
  if (need > ctx->batch_bytes) return TQ_EINVAL;
  size_t held = 0;
  int si = -1;
  for (int k = 0; k < (int)TQ_BATCH_MAX_INFLIGHT; ++k) {
    const BatchSlot& c = bs->slots[k];
    if (c.in_use) {
      held += c.held;
    } else if (si < 0 || (c.buf_cap >= used && c.q_cap >= count && bs->slots[si].buf_cap < used)) {
      si = k;
    }
  }
  if (si < 0 || held + need > ctx->batch_bytes) return TQ_EBUSY;
  // idle slots keep their buffers for reuse, but not beyond the limit
  {
    size_t total = 0;
    for (int k = 0; k < (int)TQ_BATCH_MAX_INFLIGHT; ++k) total += bs->slots[k].allocated();
    for (int k = 0; k < (int)TQ_BATCH_MAX_INFLIGHT && total + need > 2 * ctx->batch_bytes; ++k) {
      BatchSlot& c = bs->slots[k];
      if (k == si || c.in_use || !c.allocated()) continue;
      total -= c.allocated();
      free_slot_memory(c);
    }
  }
  BatchSlot& s = bs->slots[si];
  tq_status st = slot_reserve(ctx, bs, s, used, count, ws_bytes, stream);
  if (st != TQ_OK) return st;

  BatchHeader* h = reinterpret_cast<BatchHeader*>(s.h_buf);
  BatchQuery* qd = reinterpret_cast<BatchQuery*>(s.h_buf + off_q);
  uint32_t* ib = reinterpret_cast<uint32_t*>(s.h_buf + off_ib);
  uint64_t* pa = reinterpret_cast<uint64_t*>(s.h_buf + off_p);
  uint64_t* da = reinterpret_cast<uint64_t*>(s.h_buf + off_d);
  uint32_t* la = reinterpret_cast<uint32_t*>(s.h_buf + off_l);
  uint64_t pcur = 0, dcur = 0, lcur = 0;
  size_t tcur = off_t;
  uint64_t items = 0;
  // Item size: enough items to give every wave of the grid several, but no
  // item smaller than kMinItemWork group-inputs (64 words x 1 input each).
  // A lone query is spread over the whole chip; a large batch gets items of
  // up to 64 column groups, which keeps the work counter cold.
  uint64_t work = 0;
  for (uint32_t i = 0; i < count; ++i)
    if (plans[i].in_kernel) work += ((words_for_bits(queries[i].r_bits) + 63) / 64) * (uint64_t)queries[i].n;
  const uint64_t target_items = (uint64_t)bs->grid * kItemWaves * bs->items_per_wave;
  const uint64_t item_work = std::max<uint64_t>(bs->min_item_work, (work + target_items - 1) / target_items);
  tq_batch* b = new (std::nothrow) tq_batch();
  if (!b) return TQ_ENOMEM;
  b->ctx = ctx;
  b->slot = si;
  b->nq = count;
  try {
    b->tags.resize(count);
    b->variants.resize(count);
  } catch (const std::bad_alloc&) {
    delete b;
    return TQ_ENOMEM;
  }
  // where each query's dense result goes: its output, or workspace when it
  // is encoded afterwards
  std::vector<uint64_t*> dense_target(count, nullptr);
  size_t wk = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const tq_query& q = queries[i];
    if (q.out_cap == 0) {
      dense_target[i] = q.d_out;
    } else if (plans[i].in_kernel) {
      dense_target[i] = reinterpret_cast<uint64_t*>(s.d_ws + wk);
      wk += plans[i].dense_tmp;
    } else {
      dense_target[i] = reinterpret_cast<uint64_t*>(s.d_ws + ws_kernel);
    }
  }
  uint32_t kq = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const tq_query& q = queries[i];
    const QueryPlan& p = plans[i];
    b->tags[i] = q.user_tag;
    b->variants[i] = (uint8_t)p.variant;
    s.h_rec[i].t_start = 0;
    s.h_rec[i].t_end = 0;
    s.h_rec[i].status = 0;
    s.h_rec[i].done = 0;
    if (!p.in_kernel) continue;
    const uint64_t nw = words_for_bits(q.r_bits);
    BatchQuery& d = qd[kq];
    memset(&d, 0, sizeof(d));
    d.ptrs = (uint64_t)(uintptr_t)(reinterpret_cast<uint64_t*>(s.d_buf + off_p) + pcur);
    d.out = (uint64_t)(uintptr_t)dense_target[i];
    d.nwords = nw;
    d.tail_mask = tail_mask_for(q.r_bits);
    d.n = q.n;
    d.K = p.K;
    d.path = p.path;
    d.flags = p.flags;
    d.rec = i;
    // every item streams roughly the same number of bytes
    uint64_t g64 = (item_work + q.n - 1) / q.n;
    uint32_t groups = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(64, g64));
    if (p.path == BP_CSA && p.K == 4) groups = (groups + kSmallGroups - 1) / kSmallGroups * kSmallGroups;
    const uint64_t ngroups = (nw + 63) / 64;
    d.groups = groups;
    d.items = (uint32_t)std::max<uint64_t>(1, (ngroups + groups - 1) / groups);
    d.item_begin = (uint32_t)items;
    d.constant = p.plan.constant ? (p.plan.const_word ? 1u : 2u) : 0u;
    d.epi = p.plan.epi;
    d.epi.prune = ctx->prune ? 1u : 0u;
    if (!p.plan.constant && p.plan.epi.kind == EPI_TABLE) {
      memcpy(s.h_buf + tcur, p.plan.table.data(), p.plan.table.size() * 4);
      d.epi.table = reinterpret_cast<const uint32_t*>(s.d_buf + tcur);
      tcur += align_up(p.plan.table.size() * 4, 8);
    }
    ib[kq] = (uint32_t)items;
    items += d.items;
    memcpy(pa + pcur, p.dense.data(), p.dense.size() * 8);
    pcur += p.dense.size();
    ++kq;
  }
  if (items >= 0xFFFFFFFFull) {
    delete b;
    return TQ_EINVAL;
  }
  // descriptors of compressed inputs (indexes the inputs lack go to the
  // tail workspace, after a compressed query's dense result and encoder area)
  struct TailRun {
    uint64_t d_desc, d_dense, d_list;
    uint32_t nlist;
  };
  std::vector<TailRun> tails;
  std::vector<int32_t> tail_of(count, -1);
  for (uint32_t i = 0; i < count; ++i) {
    const QueryPlan& p = plans[i];
    if (p.in_kernel) continue;
    tail_of[i] = (int32_t)tails.size();
    const uint64_t nw = words_for_bits(queries[i].r_bits);
    TailRun t{};
    t.d_desc = (uint64_t)(uintptr_t)(s.d_buf + off_d + dcur * sizeof(RleDesc));
    uint64_t* idx_area = reinterpret_cast<uint64_t*>(s.d_ws + ws_kernel + p.dense_tmp + p.tail_ws -
                                                     align_up((size_t)p.missing_index * rle_index_bytes(nw), 256));
    std::vector<uint32_t> missing;
    if (rle_describe(p.rle.data(), (uint32_t)p.rle.size(), nw, idx_area, da + dcur * 3, &missing) != TQ_OK) {
      delete b;
      return TQ_EINVAL;
    }
    dcur += p.rle.size();
    t.d_list = (uint64_t)(uintptr_t)(s.d_buf + off_l + lcur * 4);
    t.nlist = (uint32_t)missing.size();
    memcpy(la + lcur, missing.data(), missing.size() * 4);
    lcur += missing.size();
    t.d_dense = (uint64_t)(uintptr_t)(reinterpret_cast<uint64_t*>(s.d_buf + off_p) + pcur);
    memcpy(pa + pcur, p.dense.data(), p.dense.size() * 8);
    pcur += p.dense.size();
    tails.push_back(t);
  }
  memset(h, 0, sizeof(*h));
  h->nq = nk;
  h->total_items = (uint32_t)items;
  h->off_queries = off_q;
  h->off_item_begin = off_ib;
  h->off_ptrs = off_p;
  h->deadline = ctx->batch_deadline_us ? (uint64_t)((double)ctx->batch_deadline_us * 1000.0 / bs->tick_ns) : 0;
  if (ctx->batch_deadline_us && h->deadline == 0) h->deadline = 1;
  s.h_ctl->cancel = 0;
  s.h_ctl->stopped = 0;
  hipError_t e = hipSuccess;
  if (items == 0 || (flags & TQ_BATCH_NO_GRAPH) || nk < kGraphMinQueries) {
    // no more workgroups than rounds of items (a small batch starts no idle ones)
    const uint64_t rounds = (items + kItemWaves - 1) / kItemWaves;
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)bs->grid, rounds));
    if ((e = hipMemcpyAsync(s.d_buf, s.h_buf, used, hipMemcpyHostToDevice, stream)) == hipSuccess && items) {
      hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(64 * kItemWaves), 0, stream, s.d_buf, s.qshard(), s.qtop(),
                         s.qcomplete(), s.d_rec, s.d_ctl);
      e = hipGetLastError();
    }
  } else {
    e = hipGraphExecMemcpyNodeSetParams1D(s.exec, s.copy_node, s.d_buf, s.h_buf, used, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipGraphLaunch(s.exec, stream);
  }
  // work after the persistent kernel: compressed-input queries and the
  // encoding of compressed results, each between its record stamps
  char* enc_ws = s.d_ws + ws_kernel;
  for (uint32_t i = 0; i < count && e == hipSuccess; ++i) {
    const tq_query& q = queries[i];
    const QueryPlan& p = plans[i];
    if (p.in_kernel && q.out_cap == 0) continue;
    const uint64_t nw = words_for_bits(q.r_bits);
    const uint64_t tmask = tail_mask_for(q.r_bits);
    int32_t* qst = s.qstatus() + i;
    if (!p.in_kernel) {
      hipLaunchKernelGGL(batch_mark_kernel, dim3(1), dim3(1), 0, stream, s.d_rec, s.qcomplete(), s.qstatus(), i, 0u,
                         0u);
      e = hipGetLastError();
      const TailRun* t = &tails[tail_of[i]];
      if (e == hipSuccess && nw > 0) {
        if (p.plan.constant) {
          e = launch_fill(dense_target[i], nw, p.plan.const_word, tmask, stream);
        } else {
          if (t->nlist)
            e = launch_build_indexes(reinterpret_cast<const RleDesc*>(t->d_desc),
                                     reinterpret_cast<const uint32_t*>(t->d_list), t->nlist, nw, qst, stream);
          if (e == hipSuccess)
            e = launch_rle_tile(reinterpret_cast<const RleDesc*>(t->d_desc), (uint32_t)p.rle.size(),
                                reinterpret_cast<const uint64_t* const*>(t->d_dense), (uint32_t)p.dense.size(), nw,
                                tmask, q.theta, nullptr, nullptr, ctx->rle_counters == 2, ctx->num_cus,
                                ctx->rle_tiles, dense_target[i], qst, stream);
        }
      }
      enc_ws = s.d_ws + ws_kernel + p.dense_tmp;
    } else {
      enc_ws = s.d_ws + ws_kernel;
    }
    if (e == hipSuccess && q.out_cap > 0) {
      if (nw == 0)
        e = launch_set_u64(q.d_out_len, 0, stream);
      else
        e = launch_rle_encode(dense_target[i], nw, tmask, q.d_out, q.out_cap, q.d_out_len, nullptr, enc_ws, qst,
                              stream);
    }
    if (e == hipSuccess) {
      hipLaunchKernelGGL(batch_mark_kernel, dim3(1), dim3(1), 0, stream, s.d_rec, s.qcomplete(), s.qstatus(), i, 1u,
                         (p.flags & QF_DEFER) ? 1u : 0u);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipEventRecord(s.done_ev, stream);
  if (e != hipSuccess) {
    delete b;
    // queued work may have run part way: the slot's counters are reset
    s.dirty = true;
    return record_hip(ctx, e);
  }
  s.in_use = true;
  s.held = need;
  *out = b;
  return TQ_OK;
}

tq_status tq_batch_poll(tq_batch* b, uint32_t* ndone) {
  if (!b || !ndone) return TQ_EINVAL;
  BatchState* bs = static_cast<BatchState*>(b->ctx->batch);
  const BatchRecord* rec = bs->slots[b->slot].h_rec;
  uint32_t d = 0;
  for (uint32_t i = 0; i < b->nq; ++i)
    d += __atomic_load_n(&rec[i].done, __ATOMIC_ACQUIRE) ? 1 : 0;
  *ndone = d;
  return TQ_OK;
}

tq_status tq_batch_wait(tq_batch* b) {
  if (!b) return TQ_EINVAL;
  BatchState* bs = static_cast<BatchState*>(b->ctx->batch);
  BatchSlot& s = bs->slots[b->slot];
  tq_status st = record_hip(b->ctx, hipEventSynchronize(s.done_ev));
  if (st != TQ_OK) return st;
  const uint32_t stopped = __atomic_load_n(&s.h_ctl->stopped, __ATOMIC_ACQUIRE);
  for (uint32_t i = 0; i < b->nq; ++i) {
    const int32_t r = public_status(s.h_rec[i], stopped, true);
    if (r != 0) return (tq_status)r;
  }
  return TQ_OK;
}

tq_status tq_batch_cancel(tq_batch* b) {
  if (!b) return TQ_EINVAL;
  BatchState* bs = static_cast<BatchState*>(b->ctx->batch);
  __atomic_store_n(&bs->slots[b->slot].h_ctl->cancel, 1u, __ATOMIC_RELEASE);
  return TQ_OK;
}

tq_status tq_batch_records(tq_batch* b, tq_query_record* out) {
  if (!b || !out) return TQ_EINVAL;
  BatchState* bs = static_cast<BatchState*>(b->ctx->batch);
  BatchSlot& s = bs->slots[b->slot];
  const bool finished = hipEventQuery(s.done_ev) == hipSuccess;
  const uint32_t stopped = __atomic_load_n(&s.h_ctl->stopped, __ATOMIC_ACQUIRE);
  const BatchRecord* rec = s.h_rec;
  for (uint32_t i = 0; i < b->nq; ++i) {
    const uint32_t done = __atomic_load_n(&rec[i].done, __ATOMIC_ACQUIRE);
    out[i].user_tag = b->tags[i];
    out[i].done = done;
    out[i].status = public_status(rec[i], stopped, finished);
    out[i].t_start_ns = (uint64_t)((double)rec[i].t_start * bs->tick_ns);
    out[i].t_end_ns = done ? (uint64_t)((double)rec[i].t_end * bs->tick_ns) : 0;
    out[i].variant = b->variants[i];
    out[i].pad = 0;
  }
  return TQ_OK;
}

tq_status tq_batch_release(tq_batch* b) {
  if (!b) return TQ_OK;
  BatchState* bs = static_cast<BatchState*>(b->ctx->batch);
  BatchSlot& s = bs->slots[b->slot];
  hipError_t e = hipEventSynchronize(s.done_ev);
  // a batch that stopped early leaves completion counters behind
  if (e != hipSuccess || __atomic_load_n(&s.h_ctl->stopped, __ATOMIC_ACQUIRE)) s.dirty = true;
  s.in_use = false;
  s.held = 0;
  tq_ctx* ctx = b->ctx;
  delete b;
  return record_hip(ctx, e);
}

tq_status tq_batch_tune(tq_ctx* ctx, const tq_query* queries, uint32_t count, hipStream_t stream,
                        uint32_t* items_per_wave, uint32_t* min_item_work) {
  if (!ctx) return TQ_EINVAL;
  BatchState* bs = batch_state(ctx);
  if (!bs) return TQ_ENOMEM;
  if (stream_capturing(stream)) return TQ_EINVAL;
  static const uint32_t ipw[] = {1, 2, 4, 8, 16};
  static const uint32_t miw[] = {4, 16, 64};
  const uint32_t keep_ipw = bs->items_per_wave, keep_miw = bs->min_item_work;
  uint32_t best_ipw = keep_ipw, best_miw = keep_miw;
  float best_us = -1.f;
  tq_status st = TQ_OK;
  for (uint32_t a : ipw) {
    for (uint32_t m : miw) {
      bs->items_per_wave = a;
      bs->min_item_work = m;
      float us = -1.f;
      // best of three submissions (packing, upload and kernels, on the stream)
      for (int rep = 0; rep < 3 && st == TQ_OK; ++rep) {
        tq_batch* b = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
          if (e0) (void)hipEventDestroy(e0);
          st = record_hip(ctx, hipErrorOutOfMemory);
          break;
        }
        (void)hipEventRecord(e0, stream);
        st = tq_batch_submit(ctx, queries, count, 0, stream, &b);
        if (st == TQ_OK) {
          (void)hipEventRecord(e1, stream);
          float ms = 0.f;
          if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            us = us < 0.f ? ms * 1000.f : std::min(us, ms * 1000.f);
          st = tq_batch_release(b);
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
      }
      if (st != TQ_OK) break;
      if (us > 0.f && (best_us < 0.f || us < best_us)) {
        best_us = us;
        best_ipw = a;
        best_miw = m;
      }
    }
    if (st != TQ_OK) break;
  }
  bs->items_per_wave = st == TQ_OK ? best_ipw : keep_ipw;
  bs->min_item_work = st == TQ_OK ? best_miw : keep_miw;
  if (items_per_wave) *items_per_wave = bs->items_per_wave;
  if (min_item_work) *min_item_work = bs->min_item_work;
  return st;
}

tq_status tq_batch_set_schedule(tq_ctx* ctx, uint32_t items_per_wave, uint32_t min_item_work) {
  if (!ctx || items_per_wave == 0 || items_per_wave > 64 || min_item_work == 0 || min_item_work > 4096)
    return TQ_EINVAL;
  BatchState* bs = batch_state(ctx);
  if (!bs) return TQ_ENOMEM;
  bs->items_per_wave = items_per_wave;
  bs->min_item_work = min_item_work;
  return TQ_OK;
}

}  // extern "C"
