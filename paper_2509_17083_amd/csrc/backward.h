#pragma once
#include "internal.h"

namespace hyrf {

// ---- loss.hip
size_t l1_ws_elems(int64_t n);
void launch_l1(const float* img, const float* target, int64_t n, float* loss, float* grad, float* ws,
               hipStream_t st);

}  // namespace hyrf
