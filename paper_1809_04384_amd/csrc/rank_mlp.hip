// Inference of the learned rank predictor: 12 -> 128 -> 128 -> 128 -> 1 with
// ReLU, BF16 weights, FP32 accumulation, inputs standardised by the training
// mean and deviation; one workgroup of 128 threads per feature row, thread j
// computes hidden unit j of each layer.  Output: round(2^y - 1) clamped at 0,
// y the predicted log2(1 + rank).
#include "rank_model.hpp"

namespace dh2 {

#include "rank_mlp_weights.inc"   // kMlpMean, kMlpStd, kMlpW1..W4 (bf16 bits), kMlpB1..B4

__device__ __forceinline__ float bf16f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__global__ void __launch_bounds__(kRankHidden) k_rank_mlp(const float* __restrict__ x, int32_t* __restrict__ rank) {
  __shared__ float xin[kRankFeatures];
  __shared__ float h[2][kRankHidden];
  const int j = threadIdx.x;
  const int64_t row = blockIdx.x;
  if (j < kRankFeatures) xin[j] = (x[row * kRankFeatures + j] - kMlpMean[j]) / kMlpStd[j];
  __syncthreads();
  float a = kMlpB1[j];
  for (int i = 0; i < kRankFeatures; ++i) a += bf16f(kMlpW1[j * kRankFeatures + i]) * xin[i];
  h[0][j] = fmaxf(a, 0.0f);
  __syncthreads();
  a = kMlpB2[j];
  for (int i = 0; i < kRankHidden; ++i) a += bf16f(kMlpW2[j * kRankHidden + i]) * h[0][i];
  h[1][j] = fmaxf(a, 0.0f);
  __syncthreads();
  a = kMlpB3[j];
  for (int i = 0; i < kRankHidden; ++i) a += bf16f(kMlpW3[j * kRankHidden + i]) * h[1][i];
  __syncthreads();
  h[0][j] = fmaxf(a, 0.0f) * bf16f(kMlpW4[j]);
  __syncthreads();
  for (int s = kRankHidden / 2; s > 0; s >>= 1) {
    if (j < s) h[0][j] += h[0][j + s];
    __syncthreads();
  }
  if (j == 0) rank[row] = max(0, (int)lrintf(exp2f(h[0][0] + kMlpB4) - 1.0f));
}

void launch_rank_mlp(const float* x, int64_t n, int32_t* rank, hipStream_t st) {
  for (int64_t r0 = 0; r0 < n; r0 += (1 << 30)) {
    const int64_t cnt = n - r0 < (1 << 30) ? n - r0 : (1 << 30);
    hipLaunchKernelGGL(k_rank_mlp, dim3((unsigned)cnt), dim3(kRankHidden), 0, st, x + r0 * kRankFeatures, rank + r0);
  }
}

}  // namespace dh2
