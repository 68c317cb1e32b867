// Small thresholds by saturating counters (the Looped algorithm of section
// 4.5), and large ones through the complement identity of section 2.3.
//
// For T <= 3, bit plane B[t] of a lane holds "at least t + 1 of the inputs so
// far have this bit": adding an input word x is B[t] |= B[t-1] & x from the
// top plane down, then B[0] |= x (2T - 1 operations, no carries).  A position
// is decided once B[T-1] is set, and because the planes only grow, a lane
// whose positions are all decided stops reading and the wave ends once no
// lane reads; the test runs every 8 inputs (every 16 in the carry-save
// kernel).
//
// A threshold theta close to N is the complement of a small one over the
// complemented inputs: NOT T_theta(B) = T_{N - theta + 1}(NOT B) (the
// corrected form of the identity), so theta >= N - 2 runs with T = N - theta
// + 1 <= 3 on the zeros of the inputs and inverts the result.  There a lane
// stops once every position has seen T zeros, typically after a few inputs.
#include "tq_variants.hpp"

namespace tq {
namespace {

using var::looped_accumulate;

template <int T, bool Comp>
__global__ __launch_bounds__(64) void looped_kernel(const uint64_t* const* __restrict__ ptrs, uint32_t n,
                                                    uint64_t nwords, uint64_t tail_mask, uint32_t prune,
                                                    uint64_t* __restrict__ out, uint64_t block0) {
  const uint64_t base = (block0 + blockIdx.x) * 64;
  const uint64_t w = base + threadIdx.x;
  const uint64_t valid = w < nwords ? (w == nwords - 1 ? tail_mask : ~(uint64_t)0) : 0;
  uint64_t B[T];
#pragma unroll
  for (int t = 0; t < T; ++t) B[t] = 0;
  if (base + 64 <= nwords)
    looped_accumulate<T, Comp, false>(B, ptrs, n, w, nwords, valid, prune != 0);
  else
    looped_accumulate<T, Comp, true>(B, ptrs, n, w, nwords, valid, prune != 0);
  if (w >= nwords) return;
  const uint64_t r = Comp ? ~B[T - 1] : B[T - 1];
  out[w] = r & valid;
}

typedef void (*LoopedFn)(const uint64_t* const*, uint32_t, uint64_t, uint64_t, uint32_t, uint64_t*, uint64_t);

LoopedFn pick_looped(int t, bool comp) {
  switch (t) {
    case 1: return comp ? looped_kernel<1, true> : looped_kernel<1, false>;
    case 2: return comp ? looped_kernel<2, true> : looped_kernel<2, false>;
    case 3: return comp ? looped_kernel<3, true> : looped_kernel<3, false>;
  }
  return nullptr;
}

}  // namespace

bool looped_applies(uint32_t n, uint32_t theta, uint32_t* t, bool* comp) {
  if (theta == 0 || theta > n) return false;
  if (theta <= 3) {
    *t = theta;
    *comp = false;
    return true;
  }
  if (n - theta + 1 <= 3) {
    *t = n - theta + 1;
    *comp = true;
    return true;
  }
  return false;
}

hipError_t launch_looped(const uint64_t* const* d_ptrs, uint32_t n, uint64_t nwords, uint64_t tail_mask,
                         uint32_t theta, bool prune, uint64_t* d_out, hipStream_t stream) {
  uint32_t t = 0;
  bool comp = false;
  if (!looped_applies(n, theta, &t, &comp)) return hipErrorInvalidValue;
  LoopedFn fn = pick_looped((int)t, comp);
  const uint64_t blocks = (nwords + 63) / 64;
  const uint64_t per_launch = kMaxLaunchItems / 64;
  for (uint64_t b0 = 0; b0 < blocks; b0 += per_launch) {
    const uint64_t nb = blocks - b0 < per_launch ? blocks - b0 : per_launch;
    hipLaunchKernelGGL(fn, dim3((uint32_t)nb), dim3(64), 0, stream, d_ptrs, n, nwords, tail_mask,
                       prune ? 1u : 0u, d_out, b0);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tq
