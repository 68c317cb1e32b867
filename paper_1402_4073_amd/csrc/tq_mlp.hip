// Kernel-selector network: a multilayer perceptron 8 -> 64 -> 64 -> 4 with
// ReLU hidden layers, fp32, trained with mean squared error on the log of
// measured run times and Adam.  Forward, backward and the optimiser are
// hand-written kernels; nothing here touches the query results (the selector
// only picks which bit-exact variant runs).
//
// Parameter layout (row-major, out x in):
//   W1[64][8]  b1[64]  W2[64][64]  b2[64]  W3[4][64]  b3[4]   (4996 floats)
//
// One wave handles a chunk of samples.  Lane j owns hidden unit j of both
// layers (its rows of W1 and W2) and, for j < 4, output j.  The gradient of
// each chunk is accumulated in registers and written to its own slot; a
// second kernel sums the slots in a fixed order, so results do not depend on
// scheduling.
#include "tq_internal.h"

namespace tq {
namespace {

constexpr int kIn = TQ_SEL_FEATURES;
constexpr int kHid = TQ_SEL_HIDDEN;
constexpr int kOut = TQ_SEL_VARIANTS;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kOut * kHid, kParams = oB3 + kOut;
constexpr int kChunk = 32;  // samples per wave

template <bool Backward>
__global__ __launch_bounds__(64) void mlp_kernel(const float* __restrict__ P, const float* __restrict__ X,
                                                 const float* __restrict__ T, const float* __restrict__ Mask,
                                                 uint32_t B, float inv_count, float* __restrict__ Y,
                                                 float* __restrict__ partial_grad, float* __restrict__ partial_loss) {
  __shared__ float sW2[kHid * (kHid + 1)];  // padded rows: column reads stay conflict-free
  __shared__ float sW3[kOut * kHid];
  __shared__ float sx[kIn], sh1[kHid], sh2[kHid], sy[kOut], sdy[kOut], sdz2[kHid];
  const int j = threadIdx.x;
  for (int t = j; t < kHid * kHid; t += 64) sW2[(t / kHid) * (kHid + 1) + t % kHid] = P[oW2 + t];
  for (int t = j; t < kOut * kHid; t += 64) sW3[t] = P[oW3 + t];
  float w1[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i) w1[i] = P[oW1 + j * kIn + i];
  const float b1 = P[oB1 + j], b2 = P[oB2 + j];
  const float b3 = j < kOut ? P[oB3 + j] : 0.f;
  // gradient accumulators of the parameters this lane owns
  float gW1[kIn], gW2[kHid], gW3[kOut];
  float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, loss = 0.f;
#pragma unroll
  for (int i = 0; i < kIn; ++i) gW1[i] = 0.f;
#pragma unroll
  for (int i = 0; i < kHid; ++i) gW2[i] = 0.f;
#pragma unroll
  for (int k = 0; k < kOut; ++k) gW3[k] = 0.f;
  __syncthreads();

  const uint32_t s0 = blockIdx.x * kChunk;
  const uint32_t s1 = s0 + kChunk < B ? s0 + kChunk : B;
  for (uint32_t s = s0; s < s1; ++s) {
    if (j < kIn) sx[j] = X[(uint64_t)s * kIn + j];
    __syncthreads();
    float z1 = b1;
#pragma unroll
    for (int i = 0; i < kIn; ++i) z1 += w1[i] * sx[i];
    const float h1 = z1 > 0.f ? z1 : 0.f;
    sh1[j] = h1;
    __syncthreads();
    float z2 = b2;
#pragma unroll 8
    for (int i = 0; i < kHid; ++i) z2 += sW2[j * (kHid + 1) + i] * sh1[i];
    const float h2 = z2 > 0.f ? z2 : 0.f;
    sh2[j] = h2;
    __syncthreads();
    if (j < kOut) {
      float y = b3;
#pragma unroll 8
      for (int i = 0; i < kHid; ++i) y += sW3[j * kHid + i] * sh2[i];
      sy[j] = y;
      if (!Backward) Y[(uint64_t)s * kOut + j] = y;
      if (Backward) {
        const float m = Mask ? Mask[(uint64_t)s * kOut + j] : 1.f;
        const float d = y - T[(uint64_t)s * kOut + j];
        loss += m * d * d * inv_count;
        sdy[j] = 2.f * m * d * inv_count;
        if (Y) Y[(uint64_t)s * kOut + j] = y;
      }
    }
    __syncthreads();
    if (Backward) {
      // output layer: lane j owns column j of W3 (one weight per output) and b3[j] for j < 4
#pragma unroll
      for (int k = 0; k < kOut; ++k) gW3[k] += sdy[k] * h2;
      if (j < kOut) gb3 += sdy[j];
      float dh2 = 0.f;
#pragma unroll
      for (int k = 0; k < kOut; ++k) dh2 += sW3[k * kHid + j] * sdy[k];
      const float dz2 = z2 > 0.f ? dh2 : 0.f;
      sdz2[j] = dz2;
      gb2 += dz2;
#pragma unroll 8
      for (int i = 0; i < kHid; ++i) gW2[i] += dz2 * sh1[i];
      __syncthreads();
      float dh1 = 0.f;
#pragma unroll 8
      for (int i = 0; i < kHid; ++i) dh1 += sW2[i * (kHid + 1) + j] * sdz2[i];
      const float dz1 = z1 > 0.f ? dh1 : 0.f;
      gb1 += dz1;
#pragma unroll
      for (int i = 0; i < kIn; ++i) gW1[i] += dz1 * sx[i];
    }
    __syncthreads();
  }
  if (Backward) {
    float* g = partial_grad + (uint64_t)blockIdx.x * kParams;
#pragma unroll
    for (int i = 0; i < kIn; ++i) g[oW1 + j * kIn + i] = gW1[i];
    g[oB1 + j] = gb1;
#pragma unroll 8
    for (int i = 0; i < kHid; ++i) g[oW2 + j * kHid + i] = gW2[i];
    g[oB2 + j] = gb2;
#pragma unroll
    for (int k = 0; k < kOut; ++k) g[oW3 + k * kHid + j] = gW3[k];
    if (j < kOut) g[oB3 + j] = gb3;
    // loss of this chunk: lanes 0..3 hold parts
    float l = loss;
    for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off, 64);
    if (j == 0) partial_loss[blockIdx.x] = l;
  }
}

// fixed-order sum of the per-chunk gradients and losses
__global__ void mlp_reduce_kernel(const float* __restrict__ partial_grad, const float* __restrict__ partial_loss,
                                  uint32_t chunks, float* __restrict__ grad, float* __restrict__ loss) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < (uint32_t)kParams) {
    float acc = 0.f;
    for (uint32_t c = 0; c < chunks; ++c) acc += partial_grad[(uint64_t)c * kParams + p];
    grad[p] = acc;
  }
  if (p == 0 && loss) {
    float acc = 0.f;
    for (uint32_t c = 0; c < chunks; ++c) acc += partial_loss[c];
    *loss = acc;
  }
}

__global__ void adam_kernel(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ Mo,
                            float* __restrict__ V, uint32_t n, float lr, float beta1, float beta2, float eps,
                            float bc1, float bc2) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float m = beta1 * Mo[i] + (1.f - beta1) * g;
  const float v = beta2 * V[i] + (1.f - beta2) * g * g;
  Mo[i] = m;
  V[i] = v;
  P[i] -= lr * (m / bc1) / (sqrtf(v / bc2) + eps);
}

}  // namespace

uint32_t mlp_chunks(uint32_t batch) { return (batch + kChunk - 1) / kChunk; }

hipError_t launch_mlp_forward(const float* d_params, const float* d_x, uint32_t batch, float* d_y,
                              hipStream_t stream) {
  if (batch == 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_kernel<false>, dim3(mlp_chunks(batch)), dim3(64), 0, stream, d_params, d_x, nullptr,
                     nullptr, batch, 0.f, d_y, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* d_params, const float* d_x, const float* d_t, const float* d_mask,
                           uint32_t batch, float inv_count, float* d_y, float* d_grad, float* d_loss, void* ws,
                           hipStream_t stream) {
  if (batch == 0) return hipSuccess;
  const uint32_t chunks = mlp_chunks(batch);
  float* pg = static_cast<float*>(ws);
  float* pl = pg + (size_t)chunks * kParams;
  hipLaunchKernelGGL(mlp_kernel<true>, dim3(chunks), dim3(64), 0, stream, d_params, d_x, d_t, d_mask, batch,
                     inv_count, d_y, pg, pl);
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + 255) / 256), dim3(256), 0, stream, pg, pl, chunks,
                     d_grad, d_loss);
  return hipGetLastError();
}

size_t mlp_grad_workspace_bytes(uint32_t batch) {
  return ((size_t)mlp_chunks(batch) * (kParams + 1) + 64) * sizeof(float);
}

hipError_t launch_adam(float* d_params, const float* d_grad, float* d_m, float* d_v, uint32_t n, float lr,
                       float beta1, float beta2, float eps, uint32_t step, hipStream_t stream) {
  const float bc1 = 1.f - powf(beta1, (float)step);
  const float bc2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, d_params, d_grad, d_m, d_v, n, lr,
                     beta1, beta2, eps, bc1, bc2);
  return hipGetLastError();
}

}  // namespace tq
