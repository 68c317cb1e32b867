// Device building blocks of the bit-sliced vertical counter, shared by the
// single-query kernels and the batch kernel.  See tq_dense.hip for the
// description of the method.
#pragma once

#include "tq_internal.h"

namespace tq {
namespace csa {

template <int WPL>
struct Vec {
  uint64_t w[WPL];
};

typedef uint64_t u64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t lo32(uint64_t x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }
__device__ __forceinline__ uint64_t join(uint32_t lo, uint32_t hi) {
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

// three-input XOR and majority, one v_bitop3_b32 per 32-bit half
__device__ __forceinline__ uint64_t xor3(uint64_t a, uint64_t b, uint64_t c) {
  return join(__builtin_amdgcn_bitop3_b32(lo32(a), lo32(b), lo32(c), 0x96),
              __builtin_amdgcn_bitop3_b32(hi32(a), hi32(b), hi32(c), 0x96));
}
__device__ __forceinline__ uint64_t maj3(uint64_t a, uint64_t b, uint64_t c) {
  return join(__builtin_amdgcn_bitop3_b32(lo32(a), lo32(b), lo32(c), 0xE8),
              __builtin_amdgcn_bitop3_b32(hi32(a), hi32(b), hi32(c), 0xE8));
}

// full adder: h <- h ^ a ^ b, c <- majority(h, a, b)
template <int WPL>
__device__ __forceinline__ void csa(Vec<WPL>& h, const Vec<WPL>& a, const Vec<WPL>& b, Vec<WPL>& c) {
#pragma unroll
  for (int i = 0; i < WPL; ++i) {
    const uint64_t hh = h.w[i];
    c.w[i] = maj3(hh, a.w[i], b.w[i]);
    h.w[i] = xor3(hh, a.w[i], b.w[i]);
  }
}

// Fold 2^L inputs of weight 1 into planes 0..L-1; return the carry of weight 2^L.
template <int L, int K, int WPL>
__device__ __forceinline__ Vec<WPL> fold(Vec<WPL> (&P)[K], const Vec<WPL>* x) {
  Vec<WPL> c;
  if constexpr (L == 1) {
    csa<WPL>(P[0], x[0], x[1], c);
  } else {
    const Vec<WPL> a = fold<L - 1, K, WPL>(P, x);
    const Vec<WPL> b = fold<L - 1, K, WPL>(P, x + (1 << (L - 1)));
    csa<WPL>(P[L - 1], a, b, c);
  }
  return c;
}

constexpr int kBlockLog = 4;
constexpr int kBlock = 1 << kBlockLog;  // inputs folded per step

// add 2^L input vectors to the counter
template <int L, int K, int WPL>
__device__ __forceinline__ void add_block_l(Vec<WPL> (&P)[K], const Vec<WPL>* x) {
  Vec<WPL> c = fold<L, K, WPL>(P, x);
#pragma unroll
  for (int k = L; k < K; ++k) {
#pragma unroll
    for (int i = 0; i < WPL; ++i) {
      const uint64_t t = P[k].w[i] & c.w[i];
      P[k].w[i] ^= c.w[i];
      c.w[i] = t;
    }
  }
}

// add 16 input vectors to the counter
template <int K, int WPL>
__device__ __forceinline__ void add_block(Vec<WPL> (&P)[K], const Vec<WPL>* x) {
  add_block_l<kBlockLog, K, WPL>(P, x);
}

template <int WPL, bool Guard>
__device__ __forceinline__ Vec<WPL> load_cols(const uint64_t* __restrict__ p, uint64_t w,
                                             uint64_t nwords) {
  Vec<WPL> v;
  if constexpr (!Guard) {
    if constexpr (WPL == 2) {
      const u64x2 t = __builtin_nontemporal_load(reinterpret_cast<const u64x2*>(p + w));
      v.w[0] = t[0];
      v.w[1] = t[1];
    } else {
      v.w[0] = __builtin_nontemporal_load(p + w);
    }
  } else {
#pragma unroll
    for (int i = 0; i < WPL; ++i) v.w[i] = (w + i < nwords) ? p[w + i] : 0;
  }
  return v;
}

// stream inputs [i0, i1) into the counter; PtrArr is any indexable array of
// input pointers (a generic pointer, or one in the constant address space)
template <int K, int WPL, bool Guard, typename PtrArr>
__device__ __forceinline__ void accumulate(Vec<WPL> (&P)[K], PtrArr ptrs,
                                           uint32_t i0, uint32_t i1, uint64_t w, uint64_t nwords) {
  uint32_t i = i0;
  for (; i + kBlock <= i1; i += kBlock) {
    Vec<WPL> x[kBlock];
#pragma unroll
    for (int u = 0; u < kBlock; ++u) x[u] = load_cols<WPL, Guard>(ptrs[i + u], w, nwords);
    add_block<K, WPL>(P, x);
  }
  if (i < i1) {
    Vec<WPL> x[kBlock];
#pragma unroll
    for (int u = 0; u < kBlock; ++u) {
      if (i + u < i1) {
        x[u] = load_cols<WPL, Guard>(ptrs[i + u], w, nwords);
      } else {
#pragma unroll
        for (int q = 0; q < WPL; ++q) x[u].w[q] = 0;
      }
    }
    add_block<K, WPL>(P, x);
  }
}

// Threshold pruning (the skipping argument of section 1, "Lower Bound"):
// after i of the inputs, a position whose count already reaches theta, or
// could not reach it with all remaining inputs, is decided.  Every kPruneEvery
// inputs each lane checks whether its positions are all decided and stops
// loading if so (the wave stops once no lane loads); the counter then still
// gives the right answer, because count >= theta holds exactly at the
// positions that were going to pass.  Measured: every 16 inputs is 10 %
// faster than every 32 at theta = 128 of 256, and costs under 1 % elsewhere.
constexpr int kPruneEvery = 16;

template <int K, int WPL>
__device__ __forceinline__ Vec<WPL> greater_than(const Vec<WPL> (&P)[K], uint32_t a);

template <int K, int WPL, bool Guard, typename PtrArr>
__device__ __forceinline__ void accumulate_pruned(Vec<WPL> (&P)[K], PtrArr ptrs, uint32_t n, uint64_t w,
                                                  uint64_t nwords, uint32_t theta) {
  uint32_t i = 0;
  // A lane whose positions are all decided (count >= theta, or too low to
  // reach theta with the inputs left) loads nothing more: adding nothing
  // keeps every decided position's result, and its memory requests stop.
  bool alive = true;
  while (i + kBlock <= n) {
    if (alive) {
      Vec<WPL> x[kBlock];
#pragma unroll
      for (int u = 0; u < kBlock; ++u) x[u] = load_cols<WPL, Guard>(ptrs[i + u], w, nwords);
      add_block<K, WPL>(P, x);
    }
    i += kBlock;
    if ((i % kPruneEvery) == 0 && i < n) {
      const uint32_t rem = n - i;
      // undecided: count >= theta - rem (could still pass) and count < theta (has not passed)
      uint64_t und = 0;
      if (theta > rem) {
        const Vec<WPL> lo = greater_than<K, WPL>(P, theta - rem - 1);
        const Vec<WPL> hi = greater_than<K, WPL>(P, theta - 1);
#pragma unroll
        for (int q = 0; q < WPL; ++q) und |= lo.w[q] & ~hi.w[q];
      } else {
        const Vec<WPL> hi = greater_than<K, WPL>(P, theta - 1);
#pragma unroll
        for (int q = 0; q < WPL; ++q) und |= ~hi.w[q];
      }
      if (Guard && w >= nwords) und = 0;
      alive = und != 0;
      if (!__any(alive)) return;
    }
  }
  if (i < n && alive) {
    Vec<WPL> x[kBlock];
#pragma unroll
    for (int u = 0; u < kBlock; ++u) {
      if (i + u < n) {
        x[u] = load_cols<WPL, Guard>(ptrs[i + u], w, nwords);
      } else {
#pragma unroll
        for (int q = 0; q < WPL; ++q) x[u].w[q] = 0;
      }
    }
    add_block<K, WPL>(P, x);
  }
}

// count > a, for a < 2^K (a is grid-uniform)
template <int K, int WPL>
__device__ __forceinline__ Vec<WPL> greater_than(const Vec<WPL> (&P)[K], uint32_t a) {
  Vec<WPL> pm, r;
#pragma unroll
  for (int i = 0; i < WPL; ++i) { pm.w[i] = ~(uint64_t)0; r.w[i] = 0; }
#pragma unroll
  for (int j = K - 1; j >= 0; --j) {
    if ((a >> j) & 1u) {
#pragma unroll
      for (int i = 0; i < WPL; ++i) pm.w[i] &= P[j].w[i];
    } else {
#pragma unroll
      for (int i = 0; i < WPL; ++i) r.w[i] |= pm.w[i] & P[j].w[i];
    }
  }
  return r;
}

// count >= x for any x (x == 0: everything; x > n: nothing)
template <int K, int WPL>
__device__ __forceinline__ Vec<WPL> at_least(const Vec<WPL> (&P)[K], uint32_t x, uint32_t n) {
  Vec<WPL> r;
  if (x == 0) {
#pragma unroll
    for (int i = 0; i < WPL; ++i) r.w[i] = ~(uint64_t)0;
  } else if (x > n) {
#pragma unroll
    for (int i = 0; i < WPL; ++i) r.w[i] = 0;
  } else {
    r = greater_than<K, WPL>(P, x - 1);
  }
  return r;
}

// EPT: EpiParams, possibly qualified with an address space (kernel argument
// or constant memory)
template <int K, int WPL, typename EPT>
__device__ __forceinline__ Vec<WPL> epilogue(const Vec<WPL> (&P)[K], EPT& e, uint32_t n,
                                            const uint32_t* lds_table) {
  Vec<WPL> r;
  if (e.kind == EPI_THRESH) {
    r = at_least<K, WPL>(P, e.theta, n);
  } else if (e.kind == EPI_PARITY) {
    r = P[0];
  } else if (e.kind == EPI_INTERVALS) {
#pragma unroll
    for (int i = 0; i < WPL; ++i) r.w[i] = 0;
    for (int t = 0; t < e.nint; ++t) {
      const Vec<WPL> a = at_least<K, WPL>(P, e.lo[t], n);
      const Vec<WPL> b = at_least<K, WPL>(P, e.hi1[t], n);
#pragma unroll
      for (int i = 0; i < WPL; ++i) r.w[i] |= a.w[i] & ~b.w[i];
    }
  } else {
    // generic truth table: rebuild each position's count from the planes
#pragma unroll
    for (int i = 0; i < WPL; ++i) {
      uint64_t o = 0;
      for (int b = 0; b < 64; ++b) {
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) c |= (uint32_t)((P[k].w[i] >> b) & 1) << k;
        o |= (uint64_t)((lds_table[c >> 5] >> (c & 31)) & 1u) << b;
      }
      r.w[i] = o;
    }
  }
  if (e.invert) {
#pragma unroll
    for (int i = 0; i < WPL; ++i) r.w[i] = ~r.w[i];
  }
  return r;
}

}  // namespace csa
}  // namespace tq
