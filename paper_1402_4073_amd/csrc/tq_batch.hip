// Batched queries: one persistent kernel serves many threshold / symmetric
// queries of uneven N, r and theta.
//
// A batch is uploaded as one packed buffer (header, query descriptors, the
// first work item of each query, and all pointer arrays).  The work of query
// q is cut into items of `groups` column groups (64 words each); item sizes
// grow as N shrinks so that every item streams about the same number of
// bytes.  Waves pop items from one atomic counter in increasing order, find
// the query of an item with a cursor that only moves forward, run the same
// register-resident carry-save counter as the single-query kernel on each
// column group and write the output words.  The wave that finishes a query's
// last item writes the query's device timestamps and a done flag into
// coherent pinned host memory, so the host sees completions without waiting
// for the whole launch.
//
// Per context there are a few batch slots with fixed capacity (queries and
// pointer entries).  A submission that finds no free slot is refused with
// TQ_EBUSY: the memory a batch can hold in flight is bounded up front.  Each
// slot owns a graph built once (copy of the packed buffer, a reset kernel,
// the persistent kernel); a submission updates the copy size and replays it.
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "tq_csa.hpp"

namespace tq {
namespace {

using namespace csa;

struct BatchHeader {
  uint32_t nq;
  uint32_t total_items;
  uint32_t next;         // work counter
  uint32_t pad0;
  uint64_t off_queries;  // byte offsets inside the packed buffer
  uint64_t off_item_begin;
  uint64_t off_ptrs;
  uint64_t pad1[3];
};

struct BatchQuery {
  uint64_t ptrs;        // device address of this query's pointer array
  uint64_t out;
  uint64_t nwords;
  uint64_t tail_mask;
  uint32_t n;
  uint32_t K;
  uint32_t groups;      // 64-word column groups per item
  uint32_t items;
  uint32_t item_begin;
  uint32_t constant;    // 0: compute, 1: all ones, 2: all zeros
  EpiParams epi;
};

struct BatchRecord {    // in pinned host memory, one per query
  uint64_t t_start;
  uint64_t t_end;
  uint32_t done;
  int32_t status;
  uint64_t pad;
};

constexpr uint32_t kSlotQueries = 8192;
constexpr uint64_t kSlotPtrs = 1u << 21;
// room for the truth tables of a batch's arbitrary symmetric functions
constexpr uint64_t kSlotTableBytes = TQ_BATCH_MAX_TABLE_BYTES;
constexpr int kSlots = 4;
constexpr int kBatchWavesPerCU = 16;
constexpr uint64_t kMinItemWork = 16;

// Completion of a query is counted on kShards sub-counters (item i of the
// query counts on shard i mod kShards) so that the items of one query, which
// tend to finish together, do not all hit one address; the item that fills a
// shard bumps the query's top counter, and the item that fills the last shard
// completes the query.  A counter that has reached its final value is set
// back to zero by the lane that saw it get there (nothing else touches it in
// this batch), so the next batch of the slot finds them all zero without a
// reset launch; they are zeroed once when the slot is created.
constexpr uint32_t kShards = 64;
// Batches of fewer queries are launched directly (copy + kernel) rather than
// by replaying the slot's graph: on this runtime a graph launch costs more
// host time than the two direct calls, which shows in the latency of small
// batches.
constexpr uint32_t kGraphMinQueries = 64;

// The packed batch is not written while the kernel runs (only the work
// counter in its header is), so descriptors, item starts and pointer arrays
// are read through the constant address space: uniform reads become scalar
// loads instead of vector loads of one address.
#define TQ_CONST __attribute__((address_space(4)))
typedef const uint64_t* const TQ_CONST* CPtrArr;   // constant array of input pointers

template <typename T>
__device__ __forceinline__ const T TQ_CONST* as_const(const void* p) {
  return (const T TQ_CONST*)(p);
}

typedef const BatchQuery TQ_CONST CBatchQuery;

template <int K>
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
  store_word<K>(Q, w, r.w[0]);
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
  for (int g = 0; g < kSmallGroups; ++g) store_word<4>(Q, base + (uint64_t)g * 64 + lane, r.w[g]);
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
                                                               BatchRecord* rec) {
  __shared__ uint32_t s_q[kItemWaves];
  __shared__ uint32_t s_local[kItemWaves];
  __shared__ uint32_t s_next;
  __shared__ uint32_t s_table[kItemWaves][kWaveTableWords];
  BatchHeader* hdr = reinterpret_cast<BatchHeader*>(buf);
  const BatchHeader TQ_CONST* chdr = as_const<BatchHeader>(buf);
  const BatchQuery TQ_CONST* qs = as_const<BatchQuery>(buf + chdr->off_queries);
  const uint32_t TQ_CONST* item_begin = as_const<uint32_t>(buf + chdr->off_item_begin);
  const uint32_t nq = chdr->nq, total = chdr->total_items;
  const uint32_t nrounds = (total + kItemWaves - 1) / kItemWaves;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t q = 0;
  uint32_t staged = 0xFFFFFFFFu;   // query whose truth table this wave holds in s_table
  // the first round of every workgroup is its own index; later ones come from the counter
  uint32_t round = blockIdx.x;
  while (round < nrounds) {
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
      if (lane == 0 && local == 0) rec[q].t_start = wall_clock64();
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
      const uint32_t step = Q.K == 4 ? kSmallGroups : 1;
      for (uint32_t g = 0; g < Q.groups; g += step) {
        const uint64_t base = (local * Q.groups + g) * 64;
        if (base >= Q.nwords) break;
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
          rec[qq].t_end = wall_clock64();
          rec[qq].status = 0;
          __hip_atomic_store(&rec[qq].done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
      }
      if (lane == 0) s_next = nrounds > gridDim.x ? gridDim.x + atomicAdd(&hdr->next, 1u) : nrounds;
    }
    __syncthreads();
    round = s_next;
  }
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

struct BatchSlot {
  bool in_use = false;
  char* d_buf = nullptr;       // packed batch (device)
  char* h_buf = nullptr;       // packed batch (pinned staging)
  size_t cap_bytes = 0;
  uint32_t* d_qdone = nullptr;     // per query: kShards completion sub-counters
  uint32_t* d_qstarted = nullptr;  // per query: completed shards
  BatchRecord* h_rec = nullptr;  // pinned, coherent, written by the GPU
  BatchRecord* d_rec = nullptr;  // device view of h_rec
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t copy_node = nullptr;
  hipEvent_t done_ev = nullptr;
};

struct BatchState {
  BatchSlot slots[kSlots];
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

tq_status slot_init(tq_ctx* ctx, BatchState* bs, BatchSlot& s) {
  if (s.d_buf) return TQ_OK;
  const size_t bytes =
      sizeof(BatchHeader) + kSlotQueries * (sizeof(BatchQuery) + 4) + kSlotPtrs * 8 + kSlotTableBytes + 4096;
  hipError_t e;
  if ((e = hipMalloc((void**)&s.d_buf, bytes)) != hipSuccess) return record_hip(ctx, e);
  if ((e = hipHostMalloc((void**)&s.h_buf, bytes, hipHostMallocDefault)) != hipSuccess) return record_hip(ctx, e);
  s.cap_bytes = bytes;
  if ((e = hipMalloc((void**)&s.d_qdone, (size_t)kSlotQueries * (kShards + 1) * 4)) != hipSuccess)
    return record_hip(ctx, e);
  // the completion counters start at zero and every batch leaves them at zero
  if ((e = hipMemset(s.d_qdone, 0, (size_t)kSlotQueries * (kShards + 1) * 4)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess)
    return record_hip(ctx, e);
  s.d_qstarted = s.d_qdone + (size_t)kSlotQueries * kShards;
  if ((e = hipHostMalloc((void**)&s.h_rec, kSlotQueries * sizeof(BatchRecord),
                         hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
    return record_hip(ctx, e);
  if ((e = hipHostGetDevicePointer((void**)&s.d_rec, s.h_rec, 0)) != hipSuccess) return record_hip(ctx, e);
  if ((e = hipEventCreateWithFlags(&s.done_ev, hipEventDisableTiming)) != hipSuccess) return record_hip(ctx, e);
  // graph: copy the packed buffer, run the persistent kernel
  if ((e = hipGraphCreate(&s.graph, 0)) != hipSuccess) return record_hip(ctx, e);
  if ((e = hipGraphAddMemcpyNode1D(&s.copy_node, s.graph, nullptr, 0, s.d_buf, s.h_buf, sizeof(BatchHeader),
                                   hipMemcpyHostToDevice)) != hipSuccess)
    return record_hip(ctx, e);
  // kernel parameter values are copied when the node is created
  uint32_t* qd = s.d_qdone;
  uint32_t* qs = s.d_qstarted;
  char* buf = s.d_buf;
  BatchRecord* rec = s.d_rec;
  hipGraphNode_t kernel_node;
  void* kargs[4] = {&buf, &qd, &qs, &rec};
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
  return TQ_OK;
}

}  // namespace

void batch_destroy(tq_ctx* ctx) {
  BatchState* bs = static_cast<BatchState*>(ctx->batch);
  if (!bs) return;
  for (auto& s : bs->slots) {
    if (s.done_ev) (void)hipEventSynchronize(s.done_ev);
    if (s.exec) (void)hipGraphExecDestroy(s.exec);
    if (s.graph) (void)hipGraphDestroy(s.graph);
    if (s.done_ev) (void)hipEventDestroy(s.done_ev);
    if (s.d_buf) (void)hipFree(s.d_buf);
    if (s.h_buf) (void)hipHostFree(s.h_buf);
    if (s.d_qdone) (void)hipFree(s.d_qdone);
    if (s.h_rec) (void)hipHostFree(s.h_rec);
  }
  delete bs;
  ctx->batch = nullptr;
}

}  // namespace tq

using namespace tq;

extern "C" {

tq_status tq_batch_submit(tq_ctx* ctx, const tq_query* queries, uint32_t count, uint32_t flags,
                          hipStream_t stream, tq_batch** out) {
  if (!ctx || !out || (count && !queries)) return TQ_EINVAL;
  *out = nullptr;
  // a batch replays its slot's own graph and reports through host memory:
  // it cannot be captured into another graph
  if (stream_capturing(stream)) return TQ_EINVAL;
  if (count == 0 || count > kSlotQueries) return TQ_EINVAL;
  BatchState* bs = batch_state(ctx);
  if (!bs) return TQ_ENOMEM;
  // validate and size
  uint64_t nptrs = 0;
  for (uint32_t i = 0; i < count; ++i) {
    const tq_query& q = queries[i];
    if (q.kind != TQ_QUERY_THRESHOLD && q.kind != TQ_QUERY_SYMMETRIC) return TQ_EINVAL;
    if (q.n == 0 || q.n > TQ_MAX_INPUTS || !q.ptrs || !q.d_out || ((uintptr_t)q.d_out & 7)) return TQ_EINVAL;
    if (q.kind == TQ_QUERY_SYMMETRIC && !q.h_truth) return TQ_EINVAL;
    const uint64_t nw = words_for_bits(q.r_bits);
    if (nw >= (1ull << 31)) return TQ_EINVAL;
    for (uint32_t j = 0; j < q.n; ++j) {
      const uintptr_t p = (uintptr_t)q.ptrs[j];
      if (!p || (p & 7)) return TQ_EINVAL;
      if (p < (uintptr_t)(q.d_out + nw) && (uintptr_t)q.d_out < p + nw * 8) return TQ_EINVAL;
    }
    nptrs += q.n;
  }
  if (nptrs > kSlotPtrs) return TQ_EINVAL;
  // plans (arbitrary truth tables are packed with the batch)
  std::vector<SymPlan> plans;
  try {
    plans.reserve(count);
    for (uint32_t i = 0; i < count; ++i) {
      const tq_query& q = queries[i];
      plans.push_back(q.kind == TQ_QUERY_THRESHOLD ? plan_threshold(q.n, q.theta) : plan_symmetric(q.n, q.h_truth));
    }
  } catch (const std::bad_alloc&) {
    return TQ_ENOMEM;
  }
  uint64_t table_bytes = 0;
  for (const SymPlan& p : plans)
    if (!p.constant && p.epi.kind == EPI_TABLE) table_bytes += align_up(p.table.size() * 4, 8);
  if (table_bytes > kSlotTableBytes) return TQ_EINVAL;
  int si = -1;
  for (int k = 0; k < kSlots; ++k)
    if (!bs->slots[k].in_use) { si = k; break; }
  if (si < 0) return TQ_EBUSY;
  BatchSlot& s = bs->slots[si];
  tq_status st = slot_init(ctx, bs, s);
  if (st != TQ_OK) return st;

  // pack: header | queries | item_begin | pointer arrays
  const size_t off_q = align_up(sizeof(BatchHeader), 256);
  const size_t off_ib = align_up(off_q + (size_t)count * sizeof(BatchQuery), 256);
  const size_t off_p = align_up(off_ib + (size_t)count * 4, 256);
  const size_t off_t = align_up(off_p + nptrs * 8, 256);
  const size_t used = off_t + table_bytes;
  if (used > s.cap_bytes) return TQ_EINVAL;
  BatchHeader* h = reinterpret_cast<BatchHeader*>(s.h_buf);
  BatchQuery* qd = reinterpret_cast<BatchQuery*>(s.h_buf + off_q);
  uint32_t* ib = reinterpret_cast<uint32_t*>(s.h_buf + off_ib);
  uint64_t* pa = reinterpret_cast<uint64_t*>(s.h_buf + off_p);
  uint64_t pcur = 0;
  size_t tcur = off_t;
  uint64_t items = 0;
  // Item size: enough items to give every wave of the grid several, but no
  // item smaller than kMinItemWork group-inputs (64 words x 1 input each).
  // A lone query is spread over the whole chip; a large batch gets items of
  // up to 64 column groups, which keeps the work counter cold.
  uint64_t work = 0;
  for (uint32_t i = 0; i < count; ++i)
    work += ((words_for_bits(queries[i].r_bits) + 63) / 64) * (uint64_t)queries[i].n;
  const uint64_t target_items = (uint64_t)bs->grid * kItemWaves * bs->items_per_wave;
  const uint64_t item_work = std::max<uint64_t>(bs->min_item_work, (work + target_items - 1) / target_items);
  tq_batch* b = new (std::nothrow) tq_batch();
  if (!b) return TQ_ENOMEM;
  b->ctx = ctx;
  b->slot = si;
  b->nq = count;
  b->tags.resize(count);
  for (uint32_t i = 0; i < count; ++i) {
    const tq_query& q = queries[i];
    const uint64_t nw = words_for_bits(q.r_bits);
    const SymPlan& plan = plans[i];
    BatchQuery& d = qd[i];
    memset(&d, 0, sizeof(d));
    d.ptrs = (uint64_t)(uintptr_t)(reinterpret_cast<uint64_t*>(s.d_buf + off_p) + pcur);
    d.out = (uint64_t)(uintptr_t)q.d_out;
    d.nwords = nw;
    d.tail_mask = tail_mask_for(q.r_bits);
    d.n = q.n;
    d.K = (uint32_t)dense_planes_for(q.n);
    // every item streams roughly the same number of bytes
    uint64_t g64 = (item_work + q.n - 1) / q.n;
    uint32_t groups = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(64, g64));
    if (dense_planes_for(q.n) == 4) groups = (groups + kSmallGroups - 1) / kSmallGroups * kSmallGroups;
    const uint64_t ngroups = (nw + 63) / 64;
    d.groups = groups;
    d.items = (uint32_t)std::max<uint64_t>(1, (ngroups + groups - 1) / groups);
    d.item_begin = (uint32_t)items;
    d.constant = plan.constant ? (plan.const_word ? 1u : 2u) : 0u;
    d.epi = plan.epi;
    d.epi.prune = ctx->prune ? 1u : 0u;
    if (!plan.constant && plan.epi.kind == EPI_TABLE) {
      memcpy(s.h_buf + tcur, plan.table.data(), plan.table.size() * 4);
      d.epi.table = reinterpret_cast<const uint32_t*>(s.d_buf + tcur);
      tcur += align_up(plan.table.size() * 4, 8);
    }
    ib[i] = (uint32_t)items;
    items += d.items;
    memcpy(pa + pcur, q.ptrs, (size_t)q.n * 8);
    pcur += q.n;
    b->tags[i] = q.user_tag;
    s.h_rec[i].t_start = 0;
    s.h_rec[i].t_end = 0;
    s.h_rec[i].status = 0;
    s.h_rec[i].done = 0;
  }
  if (items >= 0xFFFFFFFFull) {
    delete b;
    return TQ_EINVAL;
  }
  memset(h, 0, sizeof(*h));
  h->nq = count;
  h->total_items = (uint32_t)items;
  h->off_queries = off_q;
  h->off_item_begin = off_ib;
  h->off_ptrs = off_p;
  hipError_t e;
  if ((flags & TQ_BATCH_NO_GRAPH) || count < kGraphMinQueries) {
    // no more workgroups than rounds of items (a small batch starts no idle ones)
    const uint64_t rounds = (items + kItemWaves - 1) / kItemWaves;
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)bs->grid, rounds));
    if ((e = hipMemcpyAsync(s.d_buf, s.h_buf, used, hipMemcpyHostToDevice, stream)) == hipSuccess) {
      hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(64 * kItemWaves), 0, stream, s.d_buf, s.d_qdone,
                         s.d_qstarted, s.d_rec);
      e = hipGetLastError();
    }
  } else {
    e = hipGraphExecMemcpyNodeSetParams1D(s.exec, s.copy_node, s.d_buf, s.h_buf, used, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipGraphLaunch(s.exec, stream);
  }
  if (e == hipSuccess) e = hipEventRecord(s.done_ev, stream);
  if (e != hipSuccess) {
    delete b;
    return record_hip(ctx, e);
  }
  s.in_use = true;
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
  return record_hip(b->ctx, hipEventSynchronize(bs->slots[b->slot].done_ev));
}

tq_status tq_batch_records(tq_batch* b, tq_query_record* out) {
  if (!b || !out) return TQ_EINVAL;
  BatchState* bs = static_cast<BatchState*>(b->ctx->batch);
  const BatchRecord* rec = bs->slots[b->slot].h_rec;
  for (uint32_t i = 0; i < b->nq; ++i) {
    const uint32_t done = __atomic_load_n(&rec[i].done, __ATOMIC_ACQUIRE);
    out[i].user_tag = b->tags[i];
    out[i].done = done;
    out[i].status = done ? rec[i].status : 0;
    out[i].t_start_ns = (uint64_t)((double)rec[i].t_start * bs->tick_ns);
    out[i].t_end_ns = done ? (uint64_t)((double)rec[i].t_end * bs->tick_ns) : 0;
  }
  return TQ_OK;
}

tq_status tq_batch_release(tq_batch* b) {
  if (!b) return TQ_OK;
  BatchState* bs = static_cast<BatchState*>(b->ctx->batch);
  BatchSlot& s = bs->slots[b->slot];
  hipError_t e = hipEventSynchronize(s.done_ev);
  s.in_use = false;
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
