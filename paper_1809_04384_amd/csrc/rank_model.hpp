// Learned rank predictor of the truncation (the learned-rank form): per
// (cluster, direction) slot, 12 features of geometry, direction, wave number
// and tolerance, and a multilayer perceptron (12 -> 128 -> 128 -> 128 -> 1,
// BF16 weights, FP32 accumulation) that predicts log2(1 + rank) of the
// recompressed basis.  The prediction only sizes a randomized sketch; the
// exact FP64 truncation is the fallback whenever the sketch misses the
// tolerance.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "plan.hpp"

namespace dh2 {

constexpr int kRankFeatures = 12;
constexpr int kRankHidden = 128;

// Features of every slot (ns x kRankFeatures, row-major) for the row basis
// (row = true: blocks in which the cluster is the row cluster) or the column
// basis:
//   0 log2 #t                      6 log2(1 + blocks of the slot's list)
//   1 level / depth                7 log2(1 + blocks of the lists of all ancestors)
//   2 kappa diam(B_t)              8 leaf (0 / 1)
//   3 log10 tol (clamped to -16)   9 shortest / longest side of B_t
//   4 order m                     10 log2(1 + triangles of the other clusters of the list)
//   5 directional (|c| > 0)       11 eta (admissibility)
void rank_features(const Plan& p, double tol, bool row, std::vector<float>& out);

// Predicted ranks rank[i] = round(2^y - 1) >= 0 of the feature rows x (n x
// kRankFeatures, device) with the compiled-in weights.
void launch_rank_mlp(const float* x, int64_t n, int32_t* rank, hipStream_t st);

}  // namespace dh2
