// Device-wide exclusive prefix sum (reduce, scan of partials, down-sweep).
// Every workgroup owns SCAN_ITEMS consecutive values, 16 per thread.
#include "block.h"
#include "kernels.h"

namespace hyrf {

namespace {
constexpr int NT = 256;
constexpr int PER = SCAN_ITEMS / NT;   // 16

__device__ __forceinline__ void load16(const uint32_t* in, int64_t n, int64_t base, uint32_t v[PER]) {
  const int64_t i0 = base + (int64_t)threadIdx.x * PER;
  if (i0 + PER <= n && ((reinterpret_cast<uintptr_t>(in + i0) & 15) == 0)) {
    const uint4* p = reinterpret_cast<const uint4*>(in + i0);
#pragma unroll
    for (int q = 0; q < PER / 4; ++q) {
      uint4 x = p[q];
      v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < PER; ++k) v[k] = (i0 + k < n) ? in[i0 + k] : 0u;
  }
}

__global__ __launch_bounds__(NT) void k_scan_reduce(const uint32_t* __restrict__ in, int64_t n,
                                                    uint32_t* __restrict__ partial) {
  __shared__ uint32_t sh[NT / WAVE + 1];
  uint32_t v[PER];
  load16(in, n, (int64_t)blockIdx.x * SCAN_ITEMS, v);
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) s += v[k];
  uint32_t tot;
  block_excl_scan<NT>(s, sh, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Scans SCAN_ITEMS-sized chunks; `offs` (may be NULL) adds a per-chunk base.
__global__ __launch_bounds__(NT) void k_scan_down(const uint32_t* in, uint32_t* out, int64_t n,
                                                  const uint32_t* __restrict__ offs,
                                                  uint32_t* total) {
  __shared__ uint32_t sh[NT / WAVE + 1];
  const int64_t base = (int64_t)blockIdx.x * SCAN_ITEMS;
  uint32_t v[PER];
  load16(in, n, base, v);
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) s += v[k];
  uint32_t tot;
  uint32_t ex = block_excl_scan<NT>(s, sh, &tot);
  uint32_t b = offs ? offs[blockIdx.x] : 0u;
  uint32_t run = b + ex;
  const int64_t i0 = base + (int64_t)threadIdx.x * PER;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    uint32_t x = v[k];
    if (i0 + k < n) out[i0 + k] = run;
    run += x;
  }
  if (total && threadIdx.x == 0 && blockIdx.x == gridDim.x - 1) *total = b + tot;
}
__global__ void k_store_zero(uint32_t* p) {
  if (threadIdx.x == 0) *p = 0u;
}
}  // namespace

size_t scan_temp_elems(int64_t n) {
  size_t s = 0;
  while (n > SCAN_ITEMS) {
    int64_t nb = (n + SCAN_ITEMS - 1) / SCAN_ITEMS;
    s += (size_t)nb;
    n = nb;
  }
  return s + 1;
}

void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* temp,
                        uint32_t* total, hipStream_t st) {
  if (n <= 0) {
    // a kernel, not a memset node, so that the call can sit in a captured graph
    if (total) k_store_zero<<<1, 64, 0, st>>>(total);
    return;
  }
  if (n <= SCAN_ITEMS) {
    k_scan_down<<<1, NT, 0, st>>>(in, out, n, nullptr, total);
    return;
  }
  int64_t nb = (n + SCAN_ITEMS - 1) / SCAN_ITEMS;
  uint32_t* partial = temp;
  k_scan_reduce<<<(unsigned)nb, NT, 0, st>>>(in, n, partial);
  scan_exclusive_u32(partial, partial, nb, temp + nb, nullptr, st);
  k_scan_down<<<(unsigned)nb, NT, 0, st>>>(in, out, n, partial, total);
}

}  // namespace hyrf
