// Weighted threshold queries: output bit p = [ sum_j w_j * bit_j(p) >= theta ]
// for non-negative integer weights (section 2.3 allows positive integer
// weights and realises them by replicating input j w_j times, which reads it
// w_j times).  Here each input is read once.
//
// The host groups the inputs by weight.  For every weight class the kernel
// counts the class's inputs with the carry-save vertical counter of the
// unweighted kernels (planes C), then adds weight * C into a wider bit-sliced
// total T: for every set bit b of the weight, C shifted up by b planes is
// added with a ripple of full adders.  The shift is a choice of planes, so it
// costs nothing; the additions run once per class and column, against one
// full adder per input for the counting.  The comparison with theta is the
// same scalar walk over the bits of theta - 1 as in the unweighted kernels.
//
// Pruning (the skipping argument of section 1 with weights): the classes come
// heaviest first, and after each class a lane whose positions all have a
// total of at least theta, or a total below theta even with the weight of
// every class left, stops loading; the wave stops once no lane loads.  The
// total then still gives the right answer at every position.
#include "tq_csa.hpp"

namespace tq {
namespace {

using namespace csa;

// KC: planes of a class count, KT: planes of the weighted total
template <int KC, int KT>
__global__ __launch_bounds__(64) void weighted_kernel(const uint64_t* const* __restrict__ ptrs,
                                                      const WeightClass* __restrict__ classes, uint32_t nclasses,
                                                      uint64_t nwords, uint64_t tail_mask, uint32_t theta,
                                                      uint32_t total_weight, bool prune,
                                                      uint64_t* __restrict__ out, uint64_t block0) {
  const int lane = threadIdx.x;
  const uint64_t base = (block0 + blockIdx.x) * 64;
  const uint64_t w = base + lane;
  const bool full = base + 64 <= nwords;
  Vec<1> T[KT];
#pragma unroll
  for (int t = 0; t < KT; ++t) T[t].w[0] = 0;

  const uint64_t valid = w < nwords ? (w == nwords - 1 ? tail_mask : ~(uint64_t)0) : 0;
  uint32_t left = total_weight;   // weight of the classes not read yet
  bool alive = true;
  for (uint32_t c = 0; c < nclasses; ++c) {
    const WeightClass cl = classes[c];
    Vec<1> C[KC];
#pragma unroll
    for (int q = 0; q < KC; ++q) C[q].w[0] = 0;
    if (alive) {
      if (full)
        accumulate<KC, 1, false>(C, ptrs, cl.begin, cl.end, w, nwords);
      else
        accumulate<KC, 1, true>(C, ptrs, cl.begin, cl.end, w, nwords);
    }
    // T += weight * C, one shifted addition per set bit of the weight
#pragma unroll
    for (int b = 0; b < KT; ++b) {
      if ((cl.weight >> b) & 1u) {
        uint64_t carry = 0;
#pragma unroll
        for (int t = b; t < KT; ++t) {
          const uint64_t a = (t - b < KC) ? C[t - b].w[0] : 0;
          const uint64_t s = xor3(T[t].w[0], a, carry);
          carry = maj3(T[t].w[0], a, carry);
          T[t].w[0] = s;
        }
      }
    }
    if (prune) {
      left -= cl.weight * (cl.end - cl.begin);
      const uint64_t yes = at_least<KT, 1>(T, theta, total_weight).w[0];
      const uint64_t no = left < theta ? ~at_least<KT, 1>(T, theta - left, total_weight).w[0] : 0;
      alive = ((yes | no) & valid) != valid;
      if (!__any(alive)) break;
    }
  }
  if (w >= nwords) return;
  uint64_t r = at_least<KT, 1>(T, theta, total_weight).w[0];
  if (w == nwords - 1) r &= tail_mask;
  out[w] = r;
}

typedef void (*WeightedFn)(const uint64_t* const*, const WeightClass*, uint32_t, uint64_t, uint64_t, uint32_t,
                           uint32_t, bool, uint64_t*, uint64_t);

template <int KC>
WeightedFn pick_kt(int kt) {
  switch (kt) {
    case 8: if constexpr (KC <= 8) return weighted_kernel<KC, 8>; break;
    case 12: if constexpr (KC <= 12) return weighted_kernel<KC, 12>; break;
    case 16: return weighted_kernel<KC, 16>;
    case 24: return weighted_kernel<KC, 24>;
    case 32: return weighted_kernel<KC, 32>;
  }
  return nullptr;
}

WeightedFn pick_weighted(int kc, int kt) {
  switch (kc) {
    case 5: return pick_kt<5>(kt);
    case 9: return pick_kt<9>(kt);
    case 13: return pick_kt<13>(kt);
    case 16: return pick_kt<16>(kt);
  }
  return nullptr;
}

}  // namespace

void weighted_planes(uint32_t max_class, uint64_t total_weight, int* kc, int* kt) {
  const int bc = bit_length(max_class);
  *kc = bc <= 5 ? 5 : bc <= 9 ? 9 : bc <= 13 ? 13 : 16;
  const int bt = bit_length((uint32_t)total_weight);
  int t = bt <= 8 ? 8 : bt <= 12 ? 12 : bt <= 16 ? 16 : bt <= 24 ? 24 : 32;
  if (t < *kc) t = *kc <= 8 ? 8 : *kc <= 12 ? 12 : 16;
  *kt = t;
}

hipError_t launch_weighted(const uint64_t* const* d_ptrs, const WeightClass* d_classes, uint32_t nclasses,
                           uint32_t max_class, uint64_t nwords, uint64_t tail_mask, uint32_t theta,
                           uint32_t total_weight, bool prune, uint64_t* d_out, hipStream_t stream) {
  int kc, kt;
  weighted_planes(max_class, total_weight, &kc, &kt);
  WeightedFn fn = pick_weighted(kc, kt);
  if (!fn) return hipErrorInvalidValue;
  const uint64_t blocks = (nwords + 63) / 64;
  const uint64_t per_launch = kMaxLaunchItems / 64;
  for (uint64_t b0 = 0; b0 < blocks; b0 += per_launch) {
    const uint64_t nb = blocks - b0 < per_launch ? blocks - b0 : per_launch;
    hipLaunchKernelGGL(fn, dim3((uint32_t)nb), dim3(64), 0, stream, d_ptrs, d_classes, nclasses, nwords,
                       tail_mask, theta, total_weight, prune, d_out, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tq
