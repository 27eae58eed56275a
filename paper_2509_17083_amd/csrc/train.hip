// Training-loop steps after the backward (Sec. 3.4): Adam over every
// parameter tensor in one launch, the densify / prune decisions and the
// explicit-opacity reset.  All three are HBM-bound streams.
#include <math.h>

#include "block.h"
#include "kernels.h"

namespace hyrf {

namespace {
constexpr int NT = 256;
constexpr int ADAM_VEC_PER_BLOCK = 1024;   // float4 per workgroup (4096 values)

struct AdamGroupP {
  float* param;
  float* grad;
  float* m;
  float* v;
  _Float16* half;
  int64_t n;
  float lr;
};

struct AdamArgs {
  AdamGroupP g[HYRF_ADAM_MAX_GROUPS];
  int block_start[HYRF_ADAM_MAX_GROUPS + 1];   // first workgroup of each group
  int n_groups;
  float b1, b2, c1, c2;   // c1 = 1 - b1, c2 = 1 - b2
  float inv_bc1, inv_sqrt_bc2, eps;
  int zero_grad;
};

__device__ __forceinline__ void adam_one(float& p, float& g, float& m, float& v, const AdamArgs& a, float lr) {
  m = a.b1 * m + a.c1 * g;
  v = a.b2 * v + a.c2 * (g * g);
  const float mh = m * a.inv_bc1;
  const float vh = sqrtf(v) * a.inv_sqrt_bc2;   // sqrt(v / (1 - b2^t))
  p = p - lr * (mh / (vh + a.eps));
}

__global__ __launch_bounds__(NT) void k_adam(AdamArgs a) {
  const int b = blockIdx.x;
  int gi = 0;
  while (gi + 1 < a.n_groups && b >= a.block_start[gi + 1]) ++gi;
  const AdamGroupP& G = a.g[gi];
  const int64_t base = (int64_t)(b - a.block_start[gi]) * ADAM_VEC_PER_BLOCK * 4;
  const int64_t n4 = G.n >> 2;
#pragma unroll 1
  for (int k = 0; k < ADAM_VEC_PER_BLOCK / NT; ++k) {
    const int64_t e = base + 4 * ((int64_t)k * NT + threadIdx.x);
    if ((e >> 2) < n4) {
      float4 p = *reinterpret_cast<const float4*>(G.param + e);
      float4 g = *reinterpret_cast<const float4*>(G.grad + e);
      float4 m = *reinterpret_cast<const float4*>(G.m + e);
      float4 v = *reinterpret_cast<const float4*>(G.v + e);
      adam_one(p.x, g.x, m.x, v.x, a, G.lr);
      adam_one(p.y, g.y, m.y, v.y, a, G.lr);
      adam_one(p.z, g.z, m.z, v.z, a, G.lr);
      adam_one(p.w, g.w, m.w, v.w, a, G.lr);
      *reinterpret_cast<float4*>(G.param + e) = p;
      *reinterpret_cast<float4*>(G.m + e) = m;
      *reinterpret_cast<float4*>(G.v + e) = v;
      if (a.zero_grad) *reinterpret_cast<float4*>(G.grad + e) = make_float4(0.f, 0.f, 0.f, 0.f);
      if (G.half) {
        _Float16* h = G.half + e;
        h[0] = (_Float16)p.x; h[1] = (_Float16)p.y; h[2] = (_Float16)p.z; h[3] = (_Float16)p.w;
      }
    } else if (e < G.n) {   // ragged tail of the group (< 4 values)
      for (int64_t i = e; i < G.n; ++i) {
        float p = G.param[i], g = G.grad[i], m = G.m[i], v = G.v[i];
        adam_one(p, g, m, v, a, G.lr);
        G.param[i] = p;
        G.m[i] = m;
        G.v[i] = v;
        if (a.zero_grad) G.grad[i] = 0.f;
        if (G.half) G.half[i] = (_Float16)p;
      }
    }
  }
}

__global__ __launch_bounds__(NT) void k_densify_masks(int n, int n_max, const int32_t* __restrict__ vis_count,
                                                      const int32_t* __restrict__ vis_idx,
                                                      const float* __restrict__ opacity,
                                                      const float* __restrict__ scale,
                                                      const float* __restrict__ accum,
                                                      const float* __restrict__ count, float thr, float extent,
                                                      float min_op, uint8_t* __restrict__ flags) {
  const int s = blockIdx.x * NT + threadIdx.x;
  if (s >= *vis_count) return;
  const int gi = vis_idx[s];
  const float c = count[gi];
  const float mean = c > 0.f ? accum[gi] / c : 0.f;
  const float smax = fmaxf(fmaxf(scale[s], scale[(size_t)n_max + s]), scale[2 * (size_t)n_max + s]);
  uint32_t f = HYRF_JUDGED;
  if (mean >= thr) f |= smax <= extent ? HYRF_CLONE : HYRF_SPLIT;
  if (opacity[s] < min_op) f |= HYRF_PRUNE;
  flags[gi] = (uint8_t)f;
}

__global__ __launch_bounds__(NT) void k_zero_u8(uint8_t* p, int n) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(NT) void k_reset_opacity(float* __restrict__ opac_e, int n, float cap) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < n) opac_e[i] = fminf(opac_e[i], cap);
}
}  // namespace

int adam_launch(const hyrf_adam_group* groups, int n_groups, int step, float b1, float b2, float eps,
                int zero_grad, hipStream_t st) {
  AdamArgs a{};
  a.n_groups = n_groups;
  int blocks = 0;
  for (int k = 0; k < n_groups; ++k) {
    const hyrf_adam_group& g = groups[k];
    a.g[k] = AdamGroupP{g.param, g.grad, g.m, g.v, (_Float16*)g.param_half, g.n, g.lr};
    a.block_start[k] = blocks;
    const int64_t per = (int64_t)ADAM_VEC_PER_BLOCK * 4;
    const int64_t nb = (g.n + per - 1) / per;
    if (blocks + nb > INT32_MAX / 2) return -1;
    blocks += (int)nb;
  }
  a.block_start[n_groups] = blocks;
  a.b1 = b1;
  a.b2 = b2;
  a.c1 = (float)(1.0 - (double)b1);
  a.c2 = (float)(1.0 - (double)b2);
  a.inv_bc1 = (float)(1.0 / (1.0 - pow((double)b1, step)));
  a.inv_sqrt_bc2 = (float)(1.0 / sqrt(1.0 - pow((double)b2, step)));
  a.eps = eps;
  a.zero_grad = zero_grad;
  if (blocks > 0) k_adam<<<blocks, NT, 0, st>>>(a);
  return 0;
}

void launch_densify_masks(int n, int n_max, const int32_t* vis_count, const int32_t* vis_idx,
                          const float* opacity, const float* scale, const float* accum, const float* count,
                          float thr, float extent, float min_op, uint8_t* flags, hipStream_t st) {
  k_zero_u8<<<(n + NT - 1) / NT, NT, 0, st>>>(flags, n);
  k_densify_masks<<<(n + NT - 1) / NT, NT, 0, st>>>(n, n_max, vis_count, vis_idx, opacity, scale, accum, count,
                                                    thr, extent, min_op, flags);
}

void launch_reset_opacity(float* opac_e, int n, float value, hipStream_t st) {
  const float cap = (float)log((double)value / (1.0 - (double)value));
  k_reset_opacity<<<(n + NT - 1) / NT, NT, 0, st>>>(opac_e, n, cap);
}

}  // namespace hyrf
