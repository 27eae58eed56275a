#pragma once
#include "internal.h"

namespace hyrf {

struct ProjArgs {
  Cams cams;
  int n;            // Gaussian count (stride of planar per-Gaussian arrays)
  int n_max;        // splat slots per view
  int tiles_x, tiles_y;
  const int32_t* count;
  const int32_t* vis_idx;
  const void* pos;
  bool pos_f16;
  const float* opacity;
  const float* scale;
  const float* quat;
  const float* rgb;
  float* rec;
  int32_t* rect;
  float* depth;
  int64_t* total;
};

void launch_project(const ProjArgs& a, int n_cap, int V, hipStream_t st);

}  // namespace hyrf
