// Seeded synthetic bitmaps on the GPU: the same counter-based definitions as
// tqgen/__init__.py (SplitMix64 output function over per-bitmap stream keys),
// used only to fill device memory with test and benchmark inputs quickly.
// Nothing here counts, compares or encodes: it is input generation only.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t rand64(uint64_t key, uint64_t ctr) {
  return mix64(key + (ctr + 1) * kGamma);
}

// u32 uniform of bit position q
__device__ __forceinline__ uint64_t u32_at(uint64_t key, uint64_t q) {
  uint64_t r = rand64(key, q >> 1);
  return (q & 1) ? (r >> 32) : (r & 0xFFFFFFFFull);
}

__global__ void bernoulli_kernel(uint64_t* __restrict__ pool, uint64_t stride, uint64_t nwords,
                                 uint32_t nmaps, const uint64_t* __restrict__ keys,
                                 const uint64_t* __restrict__ thr) {
  const uint64_t total = nwords * (uint64_t)nmaps;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t j = t / nwords;
    const uint64_t w = t - j * nwords;
    const uint64_t key = keys[j];
    const uint64_t th = thr[j];
    uint64_t word = 0;
    const uint64_t c0 = w * 32;  // two bits per draw
#pragma unroll 8
    for (int k = 0; k < 32; ++k) {
      uint64_t r = rand64(key, c0 + k);
      uint64_t lo = r & 0xFFFFFFFFull, hi = r >> 32;
      word |= (uint64_t)(lo < th) << (2 * k);
      word |= (uint64_t)(hi < th) << (2 * k + 1);
    }
    pool[j * stride + w] = word;
  }
}

// next state from state s given the u32 uniform u
__device__ __forceinline__ uint32_t step(uint32_t s, uint64_t u, uint64_t A, uint64_t S) {
  return s ? (u < S) : (u < A);
}

constexpr uint64_t kChunkWords = 64;

__global__ void markov_kernel(uint64_t* __restrict__ pool, uint64_t stride, uint64_t nwords,
                              uint32_t nmaps, const uint64_t* __restrict__ keys,
                              const uint64_t* __restrict__ Aarr, const uint64_t* __restrict__ Sarr,
                              const uint32_t* __restrict__ init) {
  const uint64_t nchunks = (nwords + kChunkWords - 1) / kChunkWords;
  const uint64_t total = nchunks * (uint64_t)nmaps;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t j = t / nchunks;
    const uint64_t c = t - j * nchunks;
    const uint64_t key = keys[j], A = Aarr[j], S = Sarr[j];
    const uint64_t w0 = c * kChunkWords;
    const uint64_t w1 = (w0 + kChunkWords < nwords) ? w0 + kChunkWords : nwords;
    // state before position 64*w0: value of the last reset, flipped once per flip since
    uint32_t parity = 0, s = 0;
    bool found = false;
    for (uint64_t q = 64 * w0; q > 0;) {
      --q;
      const uint64_t u = u32_at(key, q);
      const bool t1 = u < A, t2 = u < S;
      if (t1 == t2) { s = (t1 ? 1u : 0u) ^ parity; found = true; break; }
      if (t1 && !t2) parity ^= 1u;
    }
    if (!found) s = init[j] ^ parity;
    for (uint64_t w = w0; w < w1; ++w) {
      uint64_t word = 0;
      for (int k = 0; k < 32; ++k) {
        uint64_t r = rand64(key, w * 32 + k);
        s = step(s, r & 0xFFFFFFFFull, A, S);
        word |= (uint64_t)s << (2 * k);
        s = step(s, r >> 32, A, S);
        word |= (uint64_t)s << (2 * k + 1);
      }
      pool[j * stride + w] = word;
    }
  }
}

int grid_for(uint64_t total, int block) {
  uint64_t g = (total + block - 1) / block;
  if (g > 65536) g = 65536;
  if (g == 0) g = 1;
  return (int)g;
}

}  // namespace

extern "C" {

// Fill nmaps Bernoulli bitmaps of nwords words each; bitmap j starts at
// d_pool + j*stride_words.  d_keys/d_thr are device arrays of nmaps entries.
// Returns 0 or a hipError_t value.
int tqgen_bernoulli_pool(uint64_t* d_pool, uint64_t stride_words, uint64_t nwords, uint32_t nmaps,
                         const uint64_t* d_keys, const uint64_t* d_thr, hipStream_t stream) {
  if (nwords == 0 || nmaps == 0) return 0;
  const uint64_t total = nwords * (uint64_t)nmaps;
  hipLaunchKernelGGL(bernoulli_kernel, dim3(grid_for(total, 256)), dim3(256), 0, stream, d_pool,
                     stride_words, nwords, nmaps, d_keys, d_thr);
  return (int)hipGetLastError();
}

// Fill nmaps Markov bitmaps (parameters per bitmap as in tqgen.MarkovParams).
int tqgen_markov_pool(uint64_t* d_pool, uint64_t stride_words, uint64_t nwords, uint32_t nmaps,
                      const uint64_t* d_keys, const uint64_t* d_A, const uint64_t* d_S,
                      const uint32_t* d_init, hipStream_t stream) {
  if (nwords == 0 || nmaps == 0) return 0;
  const uint64_t nchunks = (nwords + kChunkWords - 1) / kChunkWords;
  const uint64_t total = nchunks * (uint64_t)nmaps;
  hipLaunchKernelGGL(markov_kernel, dim3(grid_for(total, 128)), dim3(128), 0, stream, d_pool,
                     stride_words, nwords, nmaps, d_keys, d_A, d_S, d_init);
  return (int)hipGetLastError();
}

}  // extern "C"
