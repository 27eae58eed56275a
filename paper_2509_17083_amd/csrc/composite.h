#pragma once
#include "internal.h"

namespace hyrf {

struct CompArgs {
  int W, H, tiles_x, tiles_y;
  const float* rec;          // [V][n_max][12]
  uint32_t n_rec;            // V * n_max
  const uint32_t* vals;      // sorted splat ids
  const uint32_t* ranges;    // [V*tiles][2]
  float tau_T;
  float* out_rgb;            // [V][3][H][W]  (foreground colour)
  float* out_T;              // [V][H][W]
  int32_t* out_last;         // [V][H][W] or NULL
  uint32_t* list;            // render mode: pixels needing the background, or NULL
  uint32_t* list_count;
};

// Gaussian exponent of a splat with conic (a, b, c) at offset (dx, dy):
// -(a dx^2 + c dy^2)/2 - b dx dy.
__device__ __forceinline__ float splat_power(float ca, float cb, float cc, float dx, float dy) {
  return -0.5f * fmaf(ca * dx, dx, cc * dy * dy) - cb * dx * dy;
}

void launch_composite(const CompArgs& a, int V, hipStream_t st);

}  // namespace hyrf
