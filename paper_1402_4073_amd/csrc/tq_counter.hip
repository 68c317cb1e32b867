// Per-position counter variant (the GPU form of ScanCount, section 4.2) and
// per-bitmap statistics used as selector metadata.
//
// Counter variant: one lane owns one 64-bit word column and keeps a counter
// for each of its 64 positions, packed SIMD-within-a-register: with W-bit
// counters, register k holds the counters of positions k, k + W, k + 2W, ...
// (64/W of them), and adding an input word x is C[k] += (x >> k) & E for the
// W registers, E having a 1 at the bottom of every W-bit field.  W = 8 serves
// N <= 255 and W = 16 any N <= 65535, so a counter never overflows.  The
// threshold (or any truth table) is then applied per position.  Compared with
// the carry-save counter this spends W times more ALU work per input word,
// which is the trade the selector weighs.
#include "tq_variants.hpp"

namespace tq {
namespace {

using var::count_inputs;
using var::counter_word;

// W-bit counters per lane; the epilogue compares each counter with theta or
// looks f up in a table of n + 1 bits (one of the two is used).
template <int W>
__global__ __launch_bounds__(256) void counter_kernel(const uint64_t* const* __restrict__ ptrs, uint32_t n,
                                                     uint64_t nwords, uint64_t tail_mask, uint32_t theta,
                                                     const uint32_t* __restrict__ table, uint64_t* __restrict__ out,
                                                     uint64_t block0) {
  const uint64_t w = (block0 + blockIdx.x) * blockDim.x + threadIdx.x;
  const uint64_t wave_base = w & ~(uint64_t)63;
  uint64_t C[W];
#pragma unroll
  for (int k = 0; k < W; ++k) C[k] = 0;
  if (wave_base + 64 <= nwords)
    count_inputs<W, false>(C, ptrs, n, w, nwords);
  else
    count_inputs<W, true>(C, ptrs, n, w, nwords);
  if (w >= nwords) return;
  const uint64_t o = counter_word<W>(C, theta, table);
  out[w] = (w == nwords - 1) ? (o & tail_mask) : o;
}

// ones and runs of one bitmap: runs = 1 + number of positions p in [1, r)
// where bit p differs from bit p-1.  Each workgroup adds its two sums with
// one atomic each: atomics on one address are served one at a time, so the
// grid is kept to at most kStatsMaxBlocks workgroups, and a thread loads its
// kStatsWordsPerThread words of a chunk (and the word before each) before
// using any.
constexpr int kStatsBlock = 256;
constexpr uint64_t kStatsWordsPerThread = 8;
constexpr uint64_t kStatsMaxBlocks = 1024;
__global__ __launch_bounds__(kStatsBlock) void stats_kernel(const uint64_t* __restrict__ d, uint64_t nwords,
                                                            uint64_t tail_mask, uint64_t r_bits,
                                                            unsigned long long* __restrict__ ones,
                                                            unsigned long long* __restrict__ changes) {
  __shared__ unsigned long long s_sum[2][kStatsBlock / 64];
  unsigned long long so = 0, sc = 0;
  const uint64_t chunk = (uint64_t)kStatsBlock * kStatsWordsPerThread;
  for (uint64_t base = (uint64_t)blockIdx.x * chunk; base < nwords; base += (uint64_t)gridDim.x * chunk) {
    uint64_t x[kStatsWordsPerThread], before[kStatsWordsPerThread];
#pragma unroll
    for (uint64_t k = 0; k < kStatsWordsPerThread; ++k) {
      const uint64_t w = base + threadIdx.x + k * kStatsBlock;
      x[k] = w < nwords ? d[w] : 0;
      before[k] = (w < nwords && w > 0) ? d[w - 1] : 0;   // never the tail word
    }
#pragma unroll
    for (uint64_t k = 0; k < kStatsWordsPerThread; ++k) {
      const uint64_t w = base + threadIdx.x + k * kStatsBlock;
      if (w >= nwords) continue;
      const uint64_t m = (w == nwords - 1) ? tail_mask : ~(uint64_t)0;
      const uint64_t xv = x[k] & m;
      so += __popcll(xv);
      // bit p vs bit p-1 inside the word, and the first bit vs the previous word's last
      const uint64_t prev_last = w ? (before[k] >> 63) : (xv & 1);
      const uint64_t shifted = (xv << 1) | prev_last;
      sc += __popcll((xv ^ shifted) & m);
    }
  }
  // wave reduction, then the workgroup's sums, then one atomic per sum
  for (int off = 32; off > 0; off >>= 1) {
    so += __shfl_down(so, off, 64);
    sc += __shfl_down(sc, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_sum[0][threadIdx.x >> 6] = so;
    s_sum[1][threadIdx.x >> 6] = sc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long to = 0, tc = 0;
#pragma unroll
    for (int w = 0; w < kStatsBlock / 64; ++w) {
      to += s_sum[0][w];
      tc += s_sum[1][w];
    }
    atomicAdd(ones, to);
    atomicAdd(changes, tc);
  }
}

__global__ void stats_finish_kernel(unsigned long long* changes, uint64_t r_bits) {
  *changes = r_bits ? *changes + 1 : 0;   // runs = changes + 1
}

__global__ void zero2_kernel(unsigned long long* a, unsigned long long* b) {
  *a = 0;
  *b = 0;
}

}  // namespace

hipError_t launch_counter(const uint64_t* const* d_ptrs, uint32_t n, uint64_t nwords, uint64_t tail_mask,
                          uint32_t theta, const uint32_t* d_table, uint64_t* d_out, hipStream_t stream) {
  const uint64_t blocks = (nwords + 255) / 256;
  const uint64_t per_launch = kMaxLaunchItems / 256;
  for (uint64_t b0 = 0; b0 < blocks; b0 += per_launch) {
    const uint64_t nb = blocks - b0 < per_launch ? blocks - b0 : per_launch;
    if (n <= 255)
      hipLaunchKernelGGL(counter_kernel<8>, dim3((uint32_t)nb), dim3(256), 0, stream, d_ptrs, n, nwords,
                         tail_mask, theta, d_table, d_out, b0);
    else
      hipLaunchKernelGGL(counter_kernel<16>, dim3((uint32_t)nb), dim3(256), 0, stream, d_ptrs, n, nwords,
                         tail_mask, theta, d_table, d_out, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_stats(const uint64_t* d_dense, uint64_t r_bits, uint64_t* d_ones, uint64_t* d_runs,
                        hipStream_t stream) {
  const uint64_t nw = words_for_bits(r_bits);
  unsigned long long* o = reinterpret_cast<unsigned long long*>(d_ones);
  unsigned long long* c = reinterpret_cast<unsigned long long*>(d_runs);
  hipLaunchKernelGGL(zero2_kernel, dim3(1), dim3(1), 0, stream, o, c);
  if (nw) {
    const uint64_t per_block = kStatsBlock * kStatsWordsPerThread;
    uint64_t blocks = (nw + per_block - 1) / per_block;
    if (blocks > kStatsMaxBlocks) blocks = kStatsMaxBlocks;
    hipLaunchKernelGGL(stats_kernel, dim3((uint32_t)blocks), dim3(kStatsBlock), 0, stream, d_dense, nw,
                       tail_mask_for(r_bits), r_bits, o, c);
  }
  hipLaunchKernelGGL(stats_finish_kernel, dim3(1), dim3(1), 0, stream, c, r_bits);
  return hipGetLastError();
}

}  // namespace tq
