#pragma once
#include "internal.h"

namespace hyrf {

struct BinArgs {
  int V, n_max, tiles_x, tiles_y;
  const int32_t* count;
  const float* depth;
  const int32_t* rect;
  int64_t n_entries;
  uint32_t* keys;     // may be NULL
  uint32_t* vals;
  uint32_t* ranges;
};

struct BinWs {
  uint32_t* dk[2];
  uint32_t* dv[2];
  uint32_t* cnt;
  int4* srect;          // tile rectangles in depth order
  uint32_t* ek[2];
  uint32_t* ev;
  uint32_t* temp;
  size_t bytes;
};

BinWs carve_bin_ws(void* ws, int V, int n_max, int64_t capacity, int tiles_total);
void launch_bin_sort(const BinArgs& a, const BinWs& w, hipStream_t st);

}  // namespace hyrf
