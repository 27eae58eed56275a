// 8-bit min-max quantisation of a hash table (Sec. 4.3, compressed model):
// per level, min and max over its T x 2 values, step = (max - min) / 255 and
// code = rint((x - min) / step) clamped to [0, 255].  The field gather
// decodes min + step * code (field.h).  Three launches: per-block partial
// min/max, per-level parameters, encode.  Min and max are exact, so the
// result does not depend on the reduction order.
#include "block.h"
#include "kernels.h"

namespace hyrf {

namespace {
constexpr int NT = 256;
constexpr int VALS_PER_BLOCK = 4096;   // minimum values per partial
constexpr int MAX_BPL = 256;           // partial blocks per level

int blocks_per_level(int log2_T) {
  const int64_t vals = (int64_t)2 << log2_T;
  int64_t b = (vals + VALS_PER_BLOCK - 1) / VALS_PER_BLOCK;
  return (int)(b < 1 ? 1 : (b > MAX_BPL ? MAX_BPL : b));
}

__device__ __forceinline__ void block_minmax(float& mn, float& mx, float* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, off, WAVE));
    mx = fmaxf(mx, __shfl_xor(mx, off, WAVE));
  }
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) {
    sh[2 * w] = mn;
    sh[2 * w + 1] = mx;
  }
  __syncthreads();
  mn = sh[0];
  mx = sh[1];
  for (int k = 1; k < NT / WAVE; ++k) {
    mn = fminf(mn, sh[2 * k]);
    mx = fmaxf(mx, sh[2 * k + 1]);
  }
}

__global__ __launch_bounds__(NT) void k_quant_minmax(const float* __restrict__ table, int64_t per_level,
                                                     float* __restrict__ part) {
  __shared__ float sh[2 * NT / WAVE];
  const int lev = blockIdx.y, bpl = gridDim.x;
  const float* t = table + (size_t)lev * per_level;
  const int64_t chunk = (per_level + bpl - 1) / bpl;
  const int64_t b0 = (int64_t)blockIdx.x * chunk;
  const int64_t b1 = b0 + chunk < per_level ? b0 + chunk : per_level;
  float mn = INFINITY, mx = -INFINITY;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += NT) {
    const float v = t[i];
    mn = fminf(mn, v);
    mx = fmaxf(mx, v);
  }
  block_minmax(mn, mx, sh);
  if (threadIdx.x == 0) {
    part[2 * ((size_t)lev * bpl + blockIdx.x)] = mn;
    part[2 * ((size_t)lev * bpl + blockIdx.x) + 1] = mx;
  }
}

__global__ __launch_bounds__(NT) void k_quant_params(const float* __restrict__ part, int bpl,
                                                     float* __restrict__ qparams) {
  __shared__ float sh[2 * NT / WAVE];
  const int lev = blockIdx.x;
  float mn = INFINITY, mx = -INFINITY;
  for (int i = threadIdx.x; i < bpl; i += NT) {
    mn = fminf(mn, part[2 * ((size_t)lev * bpl + i)]);
    mx = fmaxf(mx, part[2 * ((size_t)lev * bpl + i) + 1]);
  }
  block_minmax(mn, mx, sh);
  if (threadIdx.x == 0) {
    qparams[2 * lev] = mn;
    qparams[2 * lev + 1] = (mx - mn) / 255.f;
  }
}

__device__ __forceinline__ uint32_t encode(float x, float mn, float step) {
  if (step == 0.f) return 0u;
  const float q = rintf((x - mn) / step);
  return (uint32_t)fminf(fmaxf(q, 0.f), 255.f);
}

// four values (two table entries) per thread and step
__global__ __launch_bounds__(NT) void k_quant_encode(const float4* __restrict__ table, int64_t n4,
                                                     int64_t per_level4, const float* __restrict__ qparams,
                                                     uchar4* __restrict__ codes) {
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n4; i += (int64_t)gridDim.x * NT) {
    const int lev = (int)(i / per_level4);
    const float mn = qparams[2 * lev], step = qparams[2 * lev + 1];
    const float4 v = table[i];
    codes[i] = make_uchar4((unsigned char)encode(v.x, mn, step), (unsigned char)encode(v.y, mn, step),
                           (unsigned char)encode(v.z, mn, step), (unsigned char)encode(v.w, mn, step));
  }
}
}  // namespace

size_t quant_ws_elems(int levels, int log2_T) { return (size_t)levels * blocks_per_level(log2_T) * 2; }

void launch_quantize(const float* table, int levels, int log2_T, uint8_t* codes, float* qparams, float* ws,
                     hipStream_t st) {
  const int64_t per_level = (int64_t)2 << log2_T;
  const int bpl = blocks_per_level(log2_T);
  k_quant_minmax<<<dim3(bpl, levels), NT, 0, st>>>(table, per_level, ws);
  k_quant_params<<<levels, NT, 0, st>>>(ws, bpl, qparams);
  const int64_t n4 = per_level / 4 * levels;
  int64_t blocks = (n4 + NT - 1) / NT;
  if (blocks > 8192) blocks = 8192;
  k_quant_encode<<<(int)blocks, NT, 0, st>>>(reinterpret_cast<const float4*>(table), n4, per_level / 4, qparams,
                                             reinterpret_cast<uchar4*>(codes));
}

}  // namespace hyrf
