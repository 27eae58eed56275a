// EWA projection of the surviving Gaussians into every view (the 3DGS
// rasterizer's preprocessing, Sec. 3.1) and the conservative tile rectangle
// of each splat.
#include "block.h"
#include "kernels.h"
#include "project.h"

namespace hyrf {

__global__ __launch_bounds__(256) void k_project(ProjArgs a) {
  __shared__ uint32_t sh_sum[256 / WAVE];
  const int v = blockIdx.y;
  const int s = blockIdx.x * 256 + threadIdx.x;
  const int count = *a.count;
  const CamP& c = a.cams.c[v];
  uint32_t tiles = 0;
  if (s < count) {
    const int n = a.n;
    const int gi = a.vis_idx[s];
    const float pxf = load_pos(a.pos, a.pos_f16, gi), pyf = load_pos(a.pos, a.pos_f16, (size_t)n + gi),
                pzf = load_pos(a.pos, a.pos_f16, 2 * (size_t)n + gi);
    double t[3];
    cam_space_f64(c, (double)pxf, (double)pyf, (double)pzf, t);
    const bool vis = precull_f64(c, t);
    const float depth = (float)t[2];
    const size_t slot = (size_t)v * a.n_max + s;
    int4 rect = make_int4(0, 0, 0, 0);
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0, r2 = r0;
    if (vis) {
      const float tx = (float)t[0], ty = (float)t[1], tz = (float)t[2];
      // rotation of the Gaussian (w, x, y, z)
      const float qw = a.quat[s], qx = a.quat[(size_t)n + s], qy = a.quat[2 * (size_t)n + s],
                  qz = a.quat[3 * (size_t)n + s];
      float Rq[3][3] = {{1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy)},
                        {2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx)},
                        {2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)}};
      float s2[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float sc = a.scale[(size_t)d * n + s];
        s2[d] = sc * sc;
      }
      // M = J W (2x3): J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]]
      const float iz = 1.0f / tz;
      const float j00 = c.fx * iz, j02 = -c.fx * tx * iz * iz;
      const float j11 = c.fy * iz, j12 = -c.fy * ty * iz * iz;
      float m0[3], m1[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        m0[k] = j00 * c.R[k] + j02 * c.R[6 + k];
        m1[k] = j11 * c.R[3 + k] + j12 * c.R[6 + k];
      }
      // A = M Rq (2x3); cov = A diag(s^2) A^T
      float A0[3], A1[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        A0[k] = m0[0] * Rq[0][k] + m0[1] * Rq[1][k] + m0[2] * Rq[2][k];
        A1[k] = m1[0] * Rq[0][k] + m1[1] * Rq[1][k] + m1[2] * Rq[2][k];
      }
      float ca = DILATION, cb = 0.f, cc = DILATION;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        ca += A0[k] * A0[k] * s2[k];
        cb += A0[k] * A1[k] * s2[k];
        cc += A1[k] * A1[k] * s2[k];
      }
      const float det = ca * cc - cb * cb;
      const float u = c.fx * tx * iz + c.cx;
      const float vv = c.fy * ty * iz + c.cy;
      const float op = a.opacity[s];
      const float lo = 255.f * op;
      if (det > 0.f && lo > 1.f && isfinite(u) && isfinite(vv)) {
        const float idet = 1.0f / det;
        const float k = sqrtf(2.f * logf(lo));
        const float rx = k * sqrtf(ca) + 1.f, ry = k * sqrtf(cc) + 1.f;
        const float tw = (float)a.tiles_x, th = (float)a.tiles_y;
        const float fx0 = fminf(fmaxf(floorf((u - rx) * (1.f / TILE)), 0.f), tw);
        const float fx1 = fminf(fmaxf(floorf((u + rx) * (1.f / TILE)) + 1.f, 0.f), tw);
        const float fy0 = fminf(fmaxf(floorf((vv - ry) * (1.f / TILE)), 0.f), th);
        const float fy1 = fminf(fmaxf(floorf((vv + ry) * (1.f / TILE)) + 1.f, 0.f), th);
        if (fx1 > fx0 && fy1 > fy0) {
          rect = make_int4((int)fx0, (int)fy0, (int)fx1, (int)fy1);
          tiles = (uint32_t)((rect.z - rect.x) * (rect.w - rect.y));
        }
        const size_t cs = (size_t)a.n;
        r0 = make_float4(u, vv, cc * idet, -cb * idet);
        r1 = make_float4(ca * idet, op, a.rgb[((size_t)v * 3 + 0) * cs + s], a.rgb[((size_t)v * 3 + 1) * cs + s]);
        r2 = make_float4(a.rgb[((size_t)v * 3 + 2) * cs + s], depth, 0.f, 0.f);
      }
    }
    float4* rec = reinterpret_cast<float4*>(a.rec) + slot * 3;
    rec[0] = r0;
    rec[1] = r1;
    rec[2] = r2;
    reinterpret_cast<int4*>(a.rect)[slot] = rect;
    a.depth[slot] = depth;
  }
  // workgroup sum of tile entries -> one 64-bit atomic
  uint32_t tot;
  block_excl_scan<256>(tiles, sh_sum, &tot);
  if (threadIdx.x == 0 && tot) atomicAdd(reinterpret_cast<unsigned long long*>(a.total), (unsigned long long)tot);
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

void launch_project(const ProjArgs& a, int n_cap, int V, hipStream_t st) {
  k_zero_i64<<<1, 1, 0, st>>>(a.total);
  dim3 grid((n_cap + 255) / 256, V);
  if (grid.x == 0) grid.x = 1;
  k_project<<<grid, 256, 0, st>>>(a);
}

}  // namespace hyrf
