// Dense threshold / symmetric kernels for gfx950.
//
// One lane owns WPL consecutive 64-bit word columns.  For every input bitmap
// it loads its WPL words (a wave reads 64*WPL*8 contiguous bytes per input)
// and adds them into a bit-sliced vertical counter held in registers: plane k
// holds bit k of the per-position count of 64*WPL positions.
//
// The counter is fed by a carry-save adder tree.  Sixteen inputs at a time
// are reduced Harley-Seal style: full adders (sum = a^b^c, carry =
// majority(a,b,c), each one v_bitop3_b32 per 32-bit half) fold pairs of
// equal-weight bit vectors into the accumulator planes 0..3 and pass one
// carry of weight 16 upward, which is rippled into planes 4..K-1 with half
// adders.  This is the sideways-sum arrangement of full adders of section
// 4.4.3 (about one full adder per input) run as a stream over the inputs,
// with the live state being the K = O(log N) planes, as in the carry-save
// vertical counter (CSvCkt) of section 4.5.1.
//
// The count is then compared with the query (section 4.4.2, comparison
// against a constant): count > a is the OR, over the zero bits j of a, of
// plane j ANDed with every plane above j where a has a one.  The bits of a
// are the same for the whole grid, so the walk over them compiles to scalar
// branches.  Symmetric functions use that comparator on interval ends, the
// low plane for parity, or a per-bit table lookup for arbitrary truth tables.
#include "tq_csa.hpp"

namespace tq {
namespace {

using namespace csa;

// K: counter planes, WPL: words per lane, S: waves that split the inputs of
// one column group, G: column groups per workgroup.  Small workgroups (one
// wave) spread best over the CUs of the eight XCDs: the kernel has no data
// reuse between workgroups, so nothing is gained by co-locating them.
template <int K, int WPL, int S, int G>
__global__ __launch_bounds__(64 * S * G) void dense_kernel(
    const uint64_t* const* __restrict__ ptrs, uint32_t n, uint64_t nwords, uint64_t tail_mask,
    uint64_t* __restrict__ out, EpiParams epi, Sink sink, uint64_t block0) {
  extern __shared__ uint64_t lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = wave / S;
  const int s = wave - g * S;
  const uint64_t group = (block0 + blockIdx.x) * G + g;   // column group of this wave
  const uint64_t base = group * (64 * WPL);
  const uint64_t w = base + (uint64_t)lane * WPL;

  // truth table for the generic epilogue, staged once per workgroup
  uint32_t* lds_table = reinterpret_cast<uint32_t*>(lds);
  constexpr int red_slots = S / 2;
  uint64_t* lds_red = lds;
  if (epi.kind == EPI_TABLE) {
    for (uint32_t t = threadIdx.x; t < epi.table_words; t += blockDim.x) lds_table[t] = epi.table[t];
    lds_red = lds + (epi.table_words + 1) / 2;
    __syncthreads();
  }

  const uint32_t per = (n + S - 1) / S;
  const uint32_t i0 = (uint32_t)s * per < n ? (uint32_t)s * per : n;
  const uint32_t i1 = i0 + per < n ? i0 + per : n;

  Vec<WPL> P[K];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int i = 0; i < WPL; ++i) P[k].w[i] = 0;

  if (base < nwords) {
    // a threshold query whose inputs all go through this wave can stop early
    const bool prune = S == 1 && epi.kind == EPI_THRESH && epi.prune && epi.theta >= 1 && epi.theta <= n;
    if (base + 64 * WPL <= nwords) {
      if (prune)
        accumulate_pruned<K, WPL, false>(P, ptrs, n, w, nwords, epi.theta);
      else
        accumulate<K, WPL, false>(P, ptrs, i0, i1, w, nwords);
    } else {
      if (prune)
        accumulate_pruned<K, WPL, true>(P, ptrs, n, w, nwords, epi.theta);
      else
        accumulate<K, WPL, true>(P, ptrs, i0, i1, w, nwords);
    }
  }

  if constexpr (S > 1) {
    // tree-add the partial counts of the S waves of this column group
#pragma unroll
    for (int step = 1; step < S; step <<= 1) {
      const int slot = s / (2 * step);
      uint64_t* red = lds_red + (((size_t)g * red_slots + slot) * K) * WPL * 64;
      if ((s % (2 * step)) == step) {
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
          for (int i = 0; i < WPL; ++i) red[(k * WPL + i) * 64 + lane] = P[k].w[i];
      }
      __syncthreads();
      if ((s % (2 * step)) == 0 && s + step < S) {
        Vec<WPL> c;
#pragma unroll
        for (int i = 0; i < WPL; ++i) c.w[i] = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
#pragma unroll
          for (int i = 0; i < WPL; ++i) {
            const uint64_t q = red[(k * WPL + i) * 64 + lane];
            const uint64_t p = P[k].w[i];
            P[k].w[i] = xor3(p, q, c.w[i]);
            c.w[i] = maj3(p, q, c.w[i]);
          }
        }
      }
      __syncthreads();
    }
    if (s != 0) return;
  }

  if (base >= nwords) return;
  Vec<WPL> v = epilogue<K, WPL>(P, epi, n, lds_table);
  const bool full = base + 64 * WPL <= nwords;
#pragma unroll
  for (int i = 0; i < WPL; ++i) {
    if (w + i == nwords - 1) v.w[i] &= tail_mask;
    if (!full && w + i >= nwords) v.w[i] = 0;
  }
  // fused consumers: AND with a filter bitmap, popcount of the result
  if (sink.filter) {
#pragma unroll
    for (int i = 0; i < WPL; ++i)
      if (full || w + i < nwords) v.w[i] &= __builtin_nontemporal_load(sink.filter + w + i);
  }
  if (out) {
    if (full) {
      if constexpr (WPL == 2) {
        u64x2 t;
        t[0] = v.w[0];
        t[1] = v.w[1];
        __builtin_nontemporal_store(t, reinterpret_cast<u64x2*>(out + w));
      } else {
        __builtin_nontemporal_store(v.w[0], out + w);
      }
    } else {
#pragma unroll
      for (int i = 0; i < WPL; ++i)
        if (w + i < nwords) out[w + i] = v.w[i];
    }
  }
  if (sink.partial) {
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < WPL; ++i) c += (uint32_t)__popcll(v.w[i]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (lane == 0) sink.partial[group] = c;
  }
}

__global__ void fill_kernel(uint64_t* __restrict__ out, uint64_t nwords, uint64_t value,
                            uint64_t tail_mask) {
  for (uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords;
       w += (uint64_t)gridDim.x * blockDim.x)
    out[w] = (w == nwords - 1) ? (value & tail_mask) : value;
}

constexpr int kFillBlock = 256;

// one word per thread: out = value AND filter, popcount per block
__global__ __launch_bounds__(kFillBlock) void fill_sink_kernel(uint64_t* __restrict__ out, uint64_t nwords,
                                                               uint64_t value, uint64_t tail_mask, Sink sink,
                                                               uint64_t block0) {
  __shared__ uint32_t wave_sum[kFillBlock / 64];
  const uint64_t block = block0 + blockIdx.x;
  const uint64_t w = block * kFillBlock + threadIdx.x;
  uint64_t v = 0;
  if (w < nwords) {
    v = (w == nwords - 1) ? (value & tail_mask) : value;
    if (sink.filter) v &= sink.filter[w];
    if (out) out[w] = v;
  }
  if (sink.partial) {
    uint32_t c = (uint32_t)__popcll(v);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) wave_sum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
#pragma unroll
      for (int i = 0; i < kFillBlock / 64; ++i) t += wave_sum[i];
      sink.partial[block] = t;
    }
  }
}

constexpr int kReduceBlock = 1024;

template <typename T>
__global__ __launch_bounds__(kReduceBlock) void count_reduce_kernel(const T* __restrict__ partial,
                                                                    uint64_t m, uint64_t* __restrict__ count) {
  __shared__ uint64_t wave_sum[kReduceBlock / 64];
  uint64_t c = 0;
  for (uint64_t i = threadIdx.x; i < m; i += kReduceBlock) c += partial[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) wave_sum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
#pragma unroll
    for (int i = 0; i < kReduceBlock / 64; ++i) t += wave_sum[i];
    *count = t;
  }
}

// Inputs split over workgroups (bitmaps too short to fill the device with
// column groups, many inputs): adding binary counts, section 4.4.2.
//
// Pass 1: one wave per (column group, part of the inputs) counts its part
// into KP planes and stores them, plane by plane, into the partial area:
// part[(p * KP + k) * stride + w] for part p, plane k and word w (stride =
// column groups * 64, so every wave writes whole 512-byte rows).
template <int KP>
__global__ __launch_bounds__(64) void dense_part_kernel(const uint64_t* const* __restrict__ ptrs, uint32_t n,
                                                       uint32_t per, uint64_t nwords, uint64_t* __restrict__ part,
                                                       uint64_t stride, uint64_t group0) {
  const int lane = threadIdx.x;
  const uint32_t p = blockIdx.y;
  const uint64_t base = (group0 + blockIdx.x) * 64;
  const uint64_t w = base + lane;
  const uint32_t i0 = p * per;
  const uint32_t i1 = i0 + per < n ? i0 + per : n;
  Vec<1> P[KP];
#pragma unroll
  for (int k = 0; k < KP; ++k) P[k].w[0] = 0;
  if (base + 64 <= nwords)
    accumulate<KP, 1, false>(P, ptrs, i0, i1, w, nwords);
  else
    accumulate<KP, 1, true>(P, ptrs, i0, i1, w, nwords);
#pragma unroll
  for (int k = 0; k < KP; ++k)
    __builtin_nontemporal_store(P[k].w[0], part + ((uint64_t)p * KP + k) * stride + w);
}

// Pass 2: one workgroup of kCombineWaves waves per column group.  Wave v
// adds parts v, v + kCombineWaves, ... to its K-plane counter (each part a
// kp-bit number: a ripple of full adders from plane 0), the waves' counters
// are added in LDS, and wave 0 applies the epilogue and stores the word.
constexpr int kCombineWaves = 8;

template <int K>
__global__ __launch_bounds__(64 * kCombineWaves) void dense_combine_kernel(
    const uint64_t* __restrict__ part, uint32_t parts, uint32_t kp, uint64_t stride, uint32_t n, uint64_t nwords,
    uint64_t tail_mask, uint64_t* __restrict__ out, EpiParams epi, uint64_t group0) {
  extern __shared__ uint64_t lds[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t w = (group0 + blockIdx.x) * 64 + lane;
  uint32_t* lds_table = reinterpret_cast<uint32_t*>(lds);
  uint64_t* red = lds;
  if (epi.kind == EPI_TABLE) {
    for (uint32_t t = threadIdx.x; t < epi.table_words; t += blockDim.x) lds_table[t] = epi.table[t];
    red = lds + (epi.table_words + 1) / 2;
  }
  Vec<1> P[K];
#pragma unroll
  for (int k = 0; k < K; ++k) P[k].w[0] = 0;
  // two parts per step, their loads issued together
  for (uint32_t p = wave; p < parts; p += 2 * kCombineWaves) {
    const uint32_t q = p + kCombineWaves;
    uint64_t x[K], y[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      x[k] = (uint32_t)k < kp ? part[((uint64_t)p * kp + k) * stride + w] : 0;
      y[k] = ((uint32_t)k < kp && q < parts) ? part[((uint64_t)q * kp + k) * stride + w] : 0;
    }
    uint64_t c = 0, d = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint64_t a = P[k].w[0];
      const uint64_t s1 = xor3(a, x[k], c);
      c = maj3(a, x[k], c);
      P[k].w[0] = xor3(s1, y[k], d);
      d = maj3(s1, y[k], d);
    }
  }
  if (wave != 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[((wave - 1) * K + k) * 64 + lane] = P[k].w[0];
  }
  __syncthreads();
  if (wave != 0) return;
#pragma unroll
  for (int v = 0; v < kCombineWaves - 1; ++v) {
    uint64_t c = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const uint64_t a = P[k].w[0], b = red[(v * K + k) * 64 + lane];
      P[k].w[0] = xor3(a, b, c);
      c = maj3(a, b, c);
    }
  }
  if (w >= nwords) return;
  uint64_t v = epilogue<K, 1>(P, epi, n, lds_table).w[0];
  if (w == nwords - 1) v &= tail_mask;
  out[w] = v;
}

typedef void (*PartFn)(const uint64_t* const*, uint32_t, uint32_t, uint64_t, uint64_t*, uint64_t, uint64_t);
typedef void (*CombineFn)(const uint64_t*, uint32_t, uint32_t, uint64_t, uint32_t, uint64_t, uint64_t, uint64_t*,
                          EpiParams, uint64_t);

PartFn pick_part(int K) {
  switch (K) {
    case 4: return dense_part_kernel<4>;
    case 5: return dense_part_kernel<5>;
    case 6: return dense_part_kernel<6>;
    case 7: return dense_part_kernel<7>;
    case 8: return dense_part_kernel<8>;
    case 9: return dense_part_kernel<9>;
    case 10: return dense_part_kernel<10>;
    case 11: return dense_part_kernel<11>;
    case 12: return dense_part_kernel<12>;
    case 13: return dense_part_kernel<13>;
    case 16: return dense_part_kernel<16>;
  }
  return nullptr;
}

CombineFn pick_combine(int K) {
  switch (K) {
    case 4: return dense_combine_kernel<4>;
    case 5: return dense_combine_kernel<5>;
    case 6: return dense_combine_kernel<6>;
    case 7: return dense_combine_kernel<7>;
    case 8: return dense_combine_kernel<8>;
    case 9: return dense_combine_kernel<9>;
    case 10: return dense_combine_kernel<10>;
    case 11: return dense_combine_kernel<11>;
    case 12: return dense_combine_kernel<12>;
    case 13: return dense_combine_kernel<13>;
    case 16: return dense_combine_kernel<16>;
  }
  return nullptr;
}

typedef void (*DenseFn)(const uint64_t* const*, uint32_t, uint64_t, uint64_t, uint64_t*, EpiParams, Sink,
                        uint64_t);

// Instantiated shapes: one word per lane with S in {1,2,4,8} and G = 1 (the
// default family), plus two-word lanes and four-wave workgroups for the tuner.
template <int K>
DenseFn pick_ws(int wpl, int split, int groups) {
  if (wpl == 1 && groups == 1) {
    switch (split) {
      case 1: return dense_kernel<K, 1, 1, 1>;
      case 2: return dense_kernel<K, 1, 2, 1>;
      case 4: return dense_kernel<K, 1, 4, 1>;
      case 8: return dense_kernel<K, 1, 8, 1>;
    }
  }
  if (split == 1) {
    if (wpl == 1 && groups == 4) return dense_kernel<K, 1, 1, 4>;
    if (wpl == 2 && groups == 1) return dense_kernel<K, 2, 1, 1>;
    if (wpl == 2 && groups == 4) return dense_kernel<K, 2, 1, 4>;
  }
  return nullptr;
}

DenseFn pick(int K, int wpl, int split, int groups) {
  switch (K) {
    case 4: return pick_ws<4>(wpl, split, groups);
    case 5: return pick_ws<5>(wpl, split, groups);
    case 6: return pick_ws<6>(wpl, split, groups);
    case 7: return pick_ws<7>(wpl, split, groups);
    case 8: return pick_ws<8>(wpl, split, groups);
    case 9: return pick_ws<9>(wpl, split, groups);
    case 10: return pick_ws<10>(wpl, split, groups);
    case 11: return pick_ws<11>(wpl, split, groups);
    case 12: return pick_ws<12>(wpl, split, groups);
    case 13: return pick_ws<13>(wpl, split, groups);
    case 16: return pick_ws<16>(wpl, split, groups);
  }
  return nullptr;
}

}  // namespace

int dense_planes_for(uint32_t n) {
  int k = bit_length(n);
  if (k < 4) k = 4;
  if (k > 13) k = 16;
  return k;
}

bool dense_config_valid(const DenseConfig& c) {
  return pick(c.K, c.wpl, c.split, c.groups) != nullptr;
}

DenseConfig choose_dense_config(uint32_t n, uint64_t nwords, bool aligned16, int num_cus, bool can_prune) {
  (void)aligned16;
  DenseConfig c;
  c.K = dense_planes_for(n);
  // one 8-byte word per lane and one wave per workgroup measured fastest
  // (8-byte coalesced loads, the most waves in flight)
  c.wpl = 1;
  c.groups = 1;
  // enough waves to keep every SIMD streaming: aim for >= 8 waves per CU,
  // splitting the inputs of a column group over up to 8 waves when the
  // bitmaps are short
  const uint64_t target_waves = (uint64_t)num_cus * 8;
  const uint64_t colgroups = (nwords + 63) / 64;
  c.split = 1;
  while (c.split < 8 && colgroups * c.split < target_waves && n / (2 * c.split) >= (uint32_t)kBlock)
    c.split *= 2;
  // a query that reads every word anyway (no pruning) with 256 inputs or
  // more: 8 waves share each column group's inputs, more independent input
  // streams in flight per CU (N = 256, r = 2^26: 1.8 % shorter launches)
  if (!can_prune && n >= 256) c.split = 8;
  return c;
}

uint64_t dense_groups(const DenseConfig& cfg, uint64_t nwords) {
  const uint64_t cols = (uint64_t)64 * cfg.wpl;
  return (nwords + cols - 1) / cols;
}

hipError_t launch_dense(const DenseConfig& cfg, const uint64_t* const* d_ptrs, uint32_t n,
                        uint64_t nwords, uint64_t tail_mask, uint64_t* d_out, const EpiParams& epi,
                        hipStream_t stream, const Sink& sink) {
  DenseFn fn = pick(cfg.K, cfg.wpl, cfg.split, cfg.groups);
  if (!fn) return hipErrorInvalidValue;
  const int G = cfg.groups;
  const uint64_t cols_per_block = (uint64_t)64 * cfg.wpl * G;
  const uint64_t blocks = (nwords + cols_per_block - 1) / cols_per_block;
  if (blocks == 0) return hipSuccess;
  size_t lds = 0;
  if (epi.kind == EPI_TABLE) lds += ((size_t)epi.table_words + 1) / 2 * 8;
  if (cfg.split > 1) lds += (size_t)G * (cfg.split / 2) * cfg.K * cfg.wpl * 64 * 8;
  const uint64_t per_launch = kMaxLaunchItems / (64ull * cfg.split * G);
  for (uint64_t b0 = 0; b0 < blocks; b0 += per_launch) {
    const uint64_t nb = blocks - b0 < per_launch ? blocks - b0 : per_launch;
    hipLaunchKernelGGL(fn, dim3((uint32_t)nb), dim3(64 * cfg.split * G), lds, stream, d_ptrs, n, nwords,
                       tail_mask, d_out, epi, sink, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fill(uint64_t* d_out, uint64_t nwords, uint64_t value, uint64_t tail_mask,
                       hipStream_t stream) {
  if (nwords == 0) return hipSuccess;
  uint64_t blocks = (nwords + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(fill_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, d_out, nwords, value,
                     tail_mask);
  return hipGetLastError();
}

uint64_t fill_groups(uint64_t nwords) { return (nwords + kFillBlock - 1) / kFillBlock; }

hipError_t launch_fill_sink(uint64_t* d_out, uint64_t nwords, uint64_t value, uint64_t tail_mask,
                            const Sink& sink, hipStream_t stream) {
  const uint64_t blocks = fill_groups(nwords);
  const uint64_t per_launch = kMaxLaunchItems / kFillBlock;
  for (uint64_t b0 = 0; b0 < blocks; b0 += per_launch) {
    const uint64_t nb = blocks - b0 < per_launch ? blocks - b0 : per_launch;
    hipLaunchKernelGGL(fill_sink_kernel, dim3((uint32_t)nb), dim3(kFillBlock), 0, stream, d_out, nwords, value,
                       tail_mask, sink, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

SplitPlan plan_split(uint32_t n, uint64_t nwords, int num_cus) {
  SplitPlan sp;
  const uint64_t groups = (nwords + 63) / 64;
  const uint64_t target = (uint64_t)(num_cus > 0 ? num_cus : 1) * 8;
  // worth it where even eight waves per column group leave most of the
  // device idle, the inputs are large enough for their reading to outweigh
  // a second launch (4 MiB), and every part keeps at least 32 inputs
  if (groups == 0 || groups * 8 >= target || n < 256 || (uint64_t)n * nwords * 8 < (4ull << 20)) return sp;
  uint64_t parts = (target + groups - 1) / groups;
  if (parts > n / 32) parts = n / 32;
  if (parts > 256) parts = 256;
  if (parts < 8) return sp;
  sp.per = (uint32_t)((n + parts - 1) / parts);
  sp.parts = (n + sp.per - 1) / sp.per;
  sp.kp = dense_planes_for(sp.per);
  sp.stride = groups * 64;
  return sp;
}

size_t split_workspace_bytes(const SplitPlan& sp) { return (size_t)sp.parts * sp.kp * sp.stride * 8; }

hipError_t launch_dense_split(const SplitPlan& sp, const uint64_t* const* d_ptrs, uint32_t n, uint64_t nwords,
                              uint64_t tail_mask, uint64_t* d_out, const EpiParams& epi, uint64_t* d_part,
                              hipStream_t stream) {
  const int K = dense_planes_for(n);
  PartFn pf = pick_part(sp.kp);
  CombineFn cf = pick_combine(K);
  if (!pf || !cf || sp.parts == 0 || sp.parts > 65535) return hipErrorInvalidValue;
  const uint64_t groups = sp.stride / 64;
  // grid x below 2^31 work-items per launch for both passes
  const uint64_t per_launch = kMaxLaunchItems / (64ull * kCombineWaves);
  for (uint64_t g0 = 0; g0 < groups; g0 += per_launch) {
    const uint64_t ng = groups - g0 < per_launch ? groups - g0 : per_launch;
    hipLaunchKernelGGL(pf, dim3((uint32_t)ng, sp.parts), dim3(64), 0, stream, d_ptrs, n, sp.per, nwords, d_part,
                       sp.stride, g0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  size_t lds = (size_t)(kCombineWaves - 1) * K * 64 * 8;
  if (epi.kind == EPI_TABLE) lds += ((size_t)epi.table_words + 1) / 2 * 8;
  for (uint64_t g0 = 0; g0 < groups; g0 += per_launch) {
    const uint64_t ng = groups - g0 < per_launch ? groups - g0 : per_launch;
    hipLaunchKernelGGL(cf, dim3((uint32_t)ng), dim3(64 * kCombineWaves), lds, stream, d_part, sp.parts, sp.kp,
                       sp.stride, n, nwords, tail_mask, d_out, epi, g0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_count_reduce(const uint32_t* d_partial, uint64_t m, uint64_t* d_count, hipStream_t stream) {
  hipLaunchKernelGGL(count_reduce_kernel<uint32_t>, dim3(1), dim3(kReduceBlock), 0, stream, d_partial, m, d_count);
  return hipGetLastError();
}

hipError_t launch_count_reduce(const uint64_t* d_partial, uint64_t m, uint64_t* d_count, hipStream_t stream) {
  hipLaunchKernelGGL(count_reduce_kernel<uint64_t>, dim3(1), dim3(kReduceBlock), 0, stream, d_partial, m, d_count);
  return hipGetLastError();
}

}  // namespace tq
