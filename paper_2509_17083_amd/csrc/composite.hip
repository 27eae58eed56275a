// Front-to-back alpha blending per 16x16 tile (Sec. 3.1 Eq. 1, 3DGS rules),
// then the background blend (Sec. 3.3 Eqs. 10-11).
//
// One workgroup of 256 threads per (tile, view), one thread per pixel.  The
// tile's depth-ordered splats are staged through LDS in batches of 256
// (one 48-byte record per thread); every pixel walks the batch from LDS
// (broadcast reads).  A batch is skipped as soon as every pixel of the tile
// has terminated.
#include "block.h"
#include "composite.h"
#include "kernels.h"

namespace hyrf {

__global__ __launch_bounds__(256) void k_composite(CompArgs a) {
  __shared__ float4 s0[256], s1[256], s2[256];
  const int tx = blockIdx.x, ty = blockIdx.y, v = blockIdx.z;
  const int x = tx * TILE + (threadIdx.x & 15);
  const int y = ty * TILE + (threadIdx.x >> 4);
  const bool inside = x < a.W && y < a.H;
  const int tile = (v * a.tiles_y + ty) * a.tiles_x + tx;
  const uint32_t start = a.ranges[2 * tile], end = a.ranges[2 * tile + 1];
  const float pxc = (float)x + 0.5f, pyc = (float)y + 0.5f;
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  uint32_t last = 0;
  bool done = !inside;
  const float4* rec = reinterpret_cast<const float4*>(a.rec);
  for (uint32_t b = start; b < end; b += 256) {
    if (__syncthreads_count(done) == 256) break;
    const uint32_t e = b + threadIdx.x;
    if (e < end) {
      const uint32_t id = a.vals[e];
      if (id < a.n_rec) {
        s0[threadIdx.x] = rec[(size_t)id * 3];
        s1[threadIdx.x] = rec[(size_t)id * 3 + 1];
        s2[threadIdx.x] = rec[(size_t)id * 3 + 2];
      } else {   // inconsistent entry list: an invisible splat
        s0[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
        s1[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
        s2[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
    __syncthreads();
    const int nb = (int)min(256u, end - b);
    if (!done) {
      // branch-free body (this loop is bound by VALU and SALU issue; the
      // skips as branches cost more in execution-mask bookkeeping than the
      // arithmetic they save): a splat that does not blend adds w = 0
      for (int k = 0; k < nb; ++k) {
        const float4 q0 = s0[k], q1 = s1[k];
        const float dx = q0.x - pxc, dy = q0.y - pyc;
        const float power = splat_power(q0.z, q0.w, q1.x, dx, dy);
        const float alpha = fminf(ALPHA_MAX, q1.y * __expf(power));
        const bool take = power <= 0.f && alpha >= ALPHA_MIN;
        const float tT = T * (1.f - alpha);
        if (take && tT < T_EPS) {
          done = true;
          break;
        }
        const float w = take ? alpha * T : 0.f;
        const float bb = s2[k].x;
        C0 = fmaf(q1.z, w, C0);
        C1 = fmaf(q1.w, w, C1);
        C2 = fmaf(bb, w, C2);
        T = take ? tT : T;
        last = take ? (uint32_t)(b - start + k + 1) : last;
      }
    }
  }
  if (inside) {
    const size_t HW = (size_t)a.W * a.H;
    const size_t p = (size_t)y * a.W + x;
    a.out_rgb[((size_t)v * 3 + 0) * HW + p] = C0;
    a.out_rgb[((size_t)v * 3 + 1) * HW + p] = C1;
    a.out_rgb[((size_t)v * 3 + 2) * HW + p] = C2;
    a.out_T[(size_t)v * HW + p] = T;
    if (a.out_last) a.out_last[(size_t)v * HW + p] = (int32_t)last;
  }
  if (a.list) {
    // pixels that receive the background in render mode (T > tau_T)
    const bool need = inside && T > a.tau_T;
    const uint64_t m = __ballot(need);
    if (m) {
      const int lane = lane_id();
      const int leader = __ffsll((long long)m) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(a.list_count, (uint32_t)__popcll(m));
      base = __shfl(base, leader, 64);
      if (need) {
        const uint32_t off = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        a.list[base + off] = (uint32_t)((size_t)v * a.W * a.H + (size_t)y * a.W + x);
      }
    }
  }
}

__global__ void k_zero_u32(uint32_t* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

void launch_composite(const CompArgs& a, int V, hipStream_t st) {
  if (a.list_count) k_zero_u32<<<1, 64, 0, st>>>(a.list_count, 1);
  dim3 grid(a.tiles_x, a.tiles_y, V);
  k_composite<<<grid, 256, 0, st>>>(a);
}

}  // namespace hyrf
