// Device building blocks of the two dense variants besides the carry-save
// counter, shared by their single-query kernels and the batch kernel:
// saturating counters for small thresholds (Looped, section 4.5) and packed
// per-position counters (ScanCount, section 4.2).  PtrArr is any indexable
// array of input pointers (a generic pointer, or one in the constant address
// space).
#pragma once

#include "tq_internal.h"

namespace tq {
namespace var {

// ---------------------------------------------------------------- Looped
// For T <= 3, plane B[t] holds "at least t + 1 of the inputs so far have
// this bit": adding an input word x is B[t] |= B[t-1] & x from the top plane
// down, then B[0] |= x (no carries).  A position is decided once B[T-1] is
// set; the planes only grow, so a lane whose positions are all decided stops
// reading and the wave ends once no lane reads (tested every
// looped_block<Comp>() inputs).  Comp reads the complemented inputs.
// Inputs per test: 8, and 4 on the complemented inputs, where a lane is
// typically decided within the first few (theta >= N - 2 needs only T zeros).
template <bool Comp>
constexpr int looped_block() { return Comp ? 4 : 8; }

typedef const __attribute__((address_space(1))) uint64_t GlobalInputWord;

// Words w of inputs i .. i + KB - 1 (zero past the last input, and
// past the bitmap when Guard).  A full block takes its pointers in one go
// and issues all its loads before any is used.
template <int KB, bool Comp, bool Guard, typename PtrArr>
__device__ __forceinline__ void looped_load(uint64_t (&x)[KB], PtrArr ptrs, uint32_t i, uint32_t n, uint64_t w,
                                            uint64_t nwords) {
  if (i + KB <= n) {
    const uint64_t* p[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) p[u] = ptrs[i + u];
#pragma unroll
    for (int u = 0; u < KB; ++u) {
      uint64_t v = 0;
      if (!Guard || w < nwords) v = __builtin_nontemporal_load((GlobalInputWord*)p[u] + w);
      x[u] = Comp ? ~v : v;
    }
    if (Guard && w >= nwords)
#pragma unroll
      for (int u = 0; u < KB; ++u) x[u] = 0;
    return;
  }
#pragma unroll
  for (int u = 0; u < KB; ++u) {
    uint64_t v = 0;
    if (i + u < n && (!Guard || w < nwords)) {
      v = __builtin_nontemporal_load((GlobalInputWord*)ptrs[i + u] + w);
      if (Comp) v = ~v;
    }
    x[u] = v;
  }
}

template <int T, bool Comp, bool Guard, typename PtrArr>
__device__ __forceinline__ void looped_accumulate(uint64_t (&B)[T], PtrArr ptrs, uint32_t n, uint64_t w,
                                                  uint64_t nwords, uint64_t valid, bool prune) {
  constexpr int KB = looped_block<Comp>();
  bool alive = true;   // this lane has positions that have not reached T
  for (uint32_t i = 0; i < n; i += KB) {
    if (alive) {
      uint64_t x[KB];
      looped_load<KB, Comp, Guard>(x, ptrs, i, n, w, nwords);
#pragma unroll
      for (int u = 0; u < KB; ++u) {
#pragma unroll
        for (int t = T - 1; t >= 1; --t) B[t] |= B[t - 1] & x[u];
        B[0] |= x[u];
      }
    }
    if (prune) {
      // positions outside the bitmap count as decided
      alive = (B[T - 1] | ~valid) != ~(uint64_t)0;
      if (!__any(alive)) return;
    }
  }
}

// ------------------------------------------------------- packed counters
// With W-bit counters, register k holds the counters of positions k, k + W,
// k + 2W, ... (64/W of them); adding an input word x is C[k] += (x >> k) & E
// for the W registers, E having a 1 at the bottom of every W-bit field.
// W = 8 serves N <= 255 and W = 16 any N <= 65535: a counter never overflows.
template <int W>
struct Packed {
  static constexpr uint64_t E = W == 8 ? 0x0101010101010101ull : 0x0001000100010001ull;
  static constexpr int F = 64 / W;                          // counters per register
  static constexpr uint64_t M = W == 8 ? 0xFFull : 0xFFFFull;
};

template <int W, bool Guard, typename PtrArr>
__device__ __forceinline__ void count_inputs(uint64_t (&C)[W], PtrArr ptrs, uint32_t n, uint64_t w,
                                             uint64_t nwords) {
  constexpr uint64_t E = Packed<W>::E;
  uint32_t i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = (!Guard || w < nwords) ? __builtin_nontemporal_load(ptrs[i + u] + w) : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int k = 0; k < W; ++k) C[k] += (x[u] >> k) & E;
  }
  for (; i < n; ++i) {
    const uint64_t x = (!Guard || w < nwords) ? ptrs[i][w] : 0;
#pragma unroll
    for (int k = 0; k < W; ++k) C[k] += (x >> k) & E;
  }
}

// Output word of packed counters: bit p is [count(p) >= theta], or f(count(p))
// from a table of n + 1 bits when `table` is not null.
template <int W>
__device__ __forceinline__ uint64_t counter_word(const uint64_t (&C)[W], uint32_t theta, const uint32_t* table) {
  constexpr int F = Packed<W>::F;
  constexpr uint64_t M = Packed<W>::M;
  uint64_t o = 0;
#pragma unroll
  for (int k = 0; k < W; ++k) {
#pragma unroll
    for (int f = 0; f < F; ++f) {
      const uint32_t c = (uint32_t)((C[k] >> (W * f)) & M);
      const uint32_t bit = table ? ((table[c >> 5] >> (c & 31)) & 1u) : (c >= theta ? 1u : 0u);
      o |= (uint64_t)bit << (k + W * f);
    }
  }
  return o;
}

}  // namespace var
}  // namespace tq
