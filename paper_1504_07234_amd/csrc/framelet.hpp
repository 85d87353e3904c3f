// Constants of the undecimated linear B-spline framelet shared by the
// explicit-state kernels (framelet.hip) and the implicit-state ones
// (shrink.hip).
#pragma once

namespace mlba {

constexpr int FR_TY = 8;  // rows per strip of the thresholded synthesis
constexpr int AN_TY = 8;  // rows per strip of the analysis and the low-pass levels
constexpr float kB1 = 0.35355339059327376f;  // sqrt(2) / 4

// pair (i, j) != (0, 0) -> position in the level's band block
__host__ __device__ constexpr int pair_slot(int i, int j) { return i * 3 + j - 1; }

}  // namespace mlba
