// Internal declarations shared by the HyRF gfx950 kernels and the C ABI.
//
// Build note: the library is compiled with -ffp-contract=off so that every
// float64 "decision" expression below rounds once per operation, exactly as
// written; hot float32 loops use explicit fmaf where a fused multiply-add is
// wanted.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hyrf.h"

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

namespace hyrf {

// Coordinate i of a planar position array stored as float32 or, for the
// compressed model, float16 (widened exactly).
__device__ __forceinline__ float load_pos(const void* pos, bool f16, size_t i) {
  return f16 ? (float)reinterpret_cast<const _Float16*>(pos)[i] : reinterpret_cast<const float*>(pos)[i];
}

constexpr int TILE = HYRF_TILE;
constexpr int MAXV = HYRF_MAX_VIEWS;
constexpr float ALPHA_MIN = 1.0f / 255.0f;   // 3DGS: skip splats below this alpha
constexpr float ALPHA_MAX = 0.99f;           // 3DGS: alpha clamp
constexpr float T_EPS = 1e-4f;               // 3DGS: stop before T falls below this
constexpr float DILATION = 0.3f;             // 3DGS: 2D covariance low-pass (px^2)
constexpr uint32_t PRIME_Y = 2654435761u;    // Instant-NGP spatial-hash primes
constexpr uint32_t PRIME_Z = 805459861u;     //   (the x prime is 1)

struct CamP {
  float R[9], t[3];
  float fx, fy, cx, cy;
  int W, H;
  float z_near, cull_tol;
};

struct Cams {
  CamP c[MAXV];
  int V;
};

constexpr int GRID_MAX_LEVELS = 16;

struct GridP {
  int L;                 // levels
  int res[GRID_MAX_LEVELS];   // N_l
  uint32_t dense_geo;    // bit l set: level l of the geometry table is dense
  uint32_t dense_rad;
  uint32_t mask_geo;     // T_geo - 1
  uint32_t mask_rad;
  int log2_T_geo, log2_T_rad;
  float center[3], inv_half[3];
  float bg_radius, tau_T;
  const float* qp_geo;   // 8-bit tables: [L][2] (min, step) per level, else NULL
  const float* qp_rad;
  int single;            // one field (the radiance table) feeds both decoders
};

inline CamP to_camp(const hyrf_camera& c) {
  CamP p;
  for (int i = 0; i < 9; ++i) p.R[i] = c.R[i];
  for (int i = 0; i < 3; ++i) p.t[i] = c.t[i];
  p.fx = c.fx; p.fy = c.fy; p.cx = c.cx; p.cy = c.cy;
  p.W = c.width; p.H = c.height;
  p.z_near = c.z_near; p.cull_tol = c.cull_tol;
  return p;
}

// ---------------------------------------------------------------------------
// Float64 decisions.  Every integer or branch decision of the step (pre-cull,
// depth key, contraction branch, grid cell) is taken here, with the order of
// operations fixed and each operation rounded once.

// Camera space t = R p + t (Sec. 3.3 Eq. 8), sums left to right.
__device__ __forceinline__ void cam_space_f64(const CamP& c, double px, double py, double pz,
                                              double t[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
    t[r] = (((double)c.R[3 * r] * px + (double)c.R[3 * r + 1] * py) + (double)c.R[3 * r + 2] * pz) +
           (double)c.t[r];
}

// Pre-cull predicate (Sec. 3.3 Eq. 9): depth beyond z_near and projected
// centre inside the frame widened by tol, in normalised frame coordinates.
__device__ __forceinline__ bool precull_f64(const CamP& c, const double t[3]) {
  if (!(t[2] > (double)c.z_near)) return false;
  double u = ((double)c.fx * t[0]) / t[2] + (double)c.cx;
  double v = ((double)c.fy * t[1]) / t[2] + (double)c.cy;
  double nx = (2.0 * u) / (double)c.W - 1.0;
  double ny = (2.0 * v) / (double)c.H - 1.0;
  double lim = 1.0 + (double)c.cull_tol;
  return fabs(nx) <= lim && fabs(ny) <= lim;
}

// Scene-box normalisation and contraction into (0,1)^3 (Sec. 3.2 Eq. 2,
// App. A.1 Eqs. 13-14; affine map 0.25 m + 0.5).
__device__ __forceinline__ void contract_f64(const GridP& g, double px, double py, double pz,
                                             double x[3]) {
  double q0 = (px - (double)g.center[0]) * (double)g.inv_half[0];
  double q1 = (py - (double)g.center[1]) * (double)g.inv_half[1];
  double q2 = (pz - (double)g.center[2]) * (double)g.inv_half[2];
  double n2 = (q0 * q0 + q1 * q1) + q2 * q2;
  if (n2 > 1.0) {
    double n = sqrt(n2);
    double s = (2.0 - 1.0 / n) / n;
    q0 = q0 * s; q1 = q1 * s; q2 = q2 * s;
  }
  x[0] = q0 * 0.25 + 0.5;
  x[1] = q1 * 0.25 + 0.5;
  x[2] = q2 * 0.25 + 0.5;
}

// Grid cell of x at resolution res: i = clamp(floor(x res), 0, res-1),
// local coordinate w = x res - i (returned in float32).
__device__ __forceinline__ void grid_cell(const double x[3], int res, int ci[3], float w[3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double gg = x[d] * (double)res;
    // fmax/fmin return the non-NaN operand, so a NaN position lands in cell 0
    double fl = fmin(fmax(floor(gg), 0.0), (double)(res - 1));
    ci[d] = (int)fl;
    w[d] = (float)(gg - fl);
  }
}

// Table row of vertex (cx, cy, cz): dense x-fastest when the level fits,
// else the XOR-prime hash masked to the power-of-two table size.
__device__ __forceinline__ uint32_t corner_row(uint32_t cx, uint32_t cy, uint32_t cz, bool dense,
                                               uint32_t side, uint32_t mask) {
  if (dense) return cx + cy * side + cz * side * side;
  return (cx ^ (cy * PRIME_Y) ^ (cz * PRIME_Z)) & mask;
}

// World ray of pixel (x, y) sampled at its centre: origin o = -R^T t,
// direction d = R^T ((x+.5-cx)/fx, (y+.5-cy)/fy, 1); then the positive root
// of |o + s d| = r (App. A.2) and the hit point.
__device__ __forceinline__ void sphere_point_f64(const CamP& c, int x, int y, double radius,
                                                 double ps[3], double d[3]) {
  double dc0 = (((double)x + 0.5) - (double)c.cx) / (double)c.fx;
  double dc1 = (((double)y + 0.5) - (double)c.cy) / (double)c.fy;
  double dc2 = 1.0;
  double o[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    d[j] = ((double)c.R[j] * dc0 + (double)c.R[3 + j] * dc1) + (double)c.R[6 + j] * dc2;
    o[j] = -(((double)c.R[j] * (double)c.t[0] + (double)c.R[3 + j] * (double)c.t[1]) +
             (double)c.R[6 + j] * (double)c.t[2]);
  }
  double A = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
  double od = (o[0] * d[0] + o[1] * d[1]) + o[2] * d[2];
  double B = 2.0 * od;
  double oo = (o[0] * o[0] + o[1] * o[1]) + o[2] * o[2];
  double C = oo - radius * radius;
  double disc = B * B - (4.0 * A) * C;
  double s = (sqrt(disc) - B) / (2.0 * A);
#pragma unroll
  for (int j = 0; j < 3; ++j) ps[j] = o[j] + s * d[j];
}

// ---------------------------------------------------------------------------
// Float32 helpers.
__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + __expf(-z)); }

__device__ __forceinline__ void cam_center_f32(const CamP& c, float o[3]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) o[j] = -((c.R[j] * c.t[0] + c.R[3 + j] * c.t[1]) + c.R[6 + j] * c.t[2]);
}

// Launch helpers
#define HYRF_LAUNCH_CHECK()                              \
  do {                                                   \
    hipError_t e_ = hipGetLastError();                   \
    if (e_ != hipSuccess) return launch_error(e_);       \
  } while (0)

}  // namespace hyrf
