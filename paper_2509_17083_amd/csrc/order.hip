// Spatial (Morton / Z-order) permutation of the Gaussians.  A data-layout
// utility, run once outside the render step: Gaussians that are close in
// space then sit in the same wavefront, so the coarse hash-grid levels they
// read and the table rows they update coincide (cache reuse in the gather,
// register pre-reduction of the gradient atomics).
#include "kernels.h"

namespace hyrf {

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__global__ __launch_bounds__(256) void k_morton(const float* __restrict__ pos, int n, GridP g,
                                                uint32_t* __restrict__ key, uint32_t* __restrict__ val) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double x[3];
  contract_f64(g, (double)pos[i], (double)pos[n + i], (double)pos[2 * n + i], x);
  uint32_t q[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) q[d] = (uint32_t)fmin(fmax(x[d] * 1024.0, 0.0), 1023.0);
  key[i] = spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2);
  val[i] = (uint32_t)i;
}

size_t order_ws_bytes(int n) {
  Carve c(nullptr);
  for (int k = 0; k < 3; ++k) c.take<uint32_t>(n > 0 ? n : 1);
  c.take<uint32_t>(radix_temp_elems(n));
  return c.off;
}

hipError_t launch_order(const float* pos, int n, const GridP& g, uint32_t* perm, void* ws, hipStream_t st) {
  Carve c(ws);
  uint32_t* k0 = c.take<uint32_t>(n > 0 ? n : 1);
  uint32_t* k1 = c.take<uint32_t>(n > 0 ? n : 1);
  uint32_t* v0 = c.take<uint32_t>(n > 0 ? n : 1);
  uint32_t* temp = c.take<uint32_t>(radix_temp_elems(n));
  if (n <= 0) return hipSuccess;
  k_morton<<<(n + 255) / 256, 256, 0, st>>>(pos, n, g, k0, v0);
  uint32_t* K[2] = {k0, k1};
  uint32_t* V[2] = {v0, perm};
  // 30 key bits: 4 passes of 8 bits; an even pass count leaves the result in
  // slot 0, so start from slot 1 when needed to land in `perm`
  const int passes = 4;
  if ((passes & 1) == 0) {
    // sort (k0, v0) -> ... -> (k0, v0), then copy v0 -> perm
    const int cur = radix_sort_pairs(K, V, 0, n, 30, temp, st);
    if (V[cur] != perm) return hipMemcpyAsync(perm, V[cur], (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st);
  }
  return hipSuccess;
}

}  // namespace hyrf
