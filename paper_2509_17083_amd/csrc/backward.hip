// Adjoint of the render step (train mode).
//
//  k_composite_bwd  per 16x16 tile, back to front: the 3DGS blending adjoint
//                   with the background term, transmittance recovered by
//                   division from the final value; per-splat gradients of
//                   (u, v, conic, opacity, rgb) summed over each wave's 64
//                   pixels, then added by 9 lanes of one atomic instruction.
//  k_project_bwd    per surviving Gaussian, looping over views: EWA
//                   projection adjoint (no atomics: one lane per Gaussian).
//  k_field_bwd      per 16 Gaussians per wave (or 16 background pixels):
//                   decoder adjoints on MFMA with dW accumulated through LDS
//                   staging; feature gradients out, plus the view-direction
//                   part of the position gradient.  For background pixels
//                   the radiance-table scatter-add follows in the same
//                   kernel, round by round.
//  k_grid_scatter   per Gaussian, when the forward saved the feature
//                   derivatives: hash-table scatter-add (cell runs summed,
//                   lane-combined atomics).
//  k_grid_bwd       the same when no derivatives were saved, plus the
//                   position gradient through the interpolation weights and
//                   the contraction.
//  k_dw_reduce      sums the per-workgroup dW partials in a fixed order.
#include "backward.h"
#include "block.h"
#include "composite.h"
#include "field_bwd.h"
#include "kernels.h"
#include "query.h"

#include <type_traits>

namespace hyrf {

constexpr int GS = 9;   // per-splat gradient record: u, v, conic a, b, c, opacity, r, g, b

__global__ void k_zero_f32(float* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// ---------------------------------------------------------------- compositing
__global__ __launch_bounds__(256) void k_composite_bwd(CompBwdArgs a) {
  __shared__ float4 s0[256], s1[256], s2[256];
  __shared__ uint32_t sid[256];
  __shared__ int smax[4];
  const int tx = blockIdx.x, ty = blockIdx.y, v = blockIdx.z;
  const int x = tx * TILE + (threadIdx.x & 15);
  const int y = ty * TILE + (threadIdx.x >> 4);
  const bool inside = x < a.W && y < a.H;
  const int tile = (v * a.tiles_y + ty) * a.tiles_x + tx;
  const uint32_t start = a.ranges[2 * tile];
  const size_t HW = (size_t)a.W * a.H;
  const size_t p = (size_t)y * a.W + x;
  const float pxc = (float)x + 0.5f, pyc = (float)y + 0.5f;
  float Tfin = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f, bgd = 0.f;
  int last = 0;
  if (inside) {
    Tfin = a.T_final[(size_t)v * HW + p];
    last = a.last[(size_t)v * HW + p];
    g0 = a.dL[((size_t)v * 3 + 0) * HW + p];
    g1 = a.dL[((size_t)v * 3 + 1) * HW + p];
    g2 = a.dL[((size_t)v * 3 + 2) * HW + p];
    if (a.bg)
      bgd = a.bg[((size_t)v * 3 + 0) * HW + p] * g0 + a.bg[((size_t)v * 3 + 1) * HW + p] * g1 +
            a.bg[((size_t)v * 3 + 2) * HW + p] * g2;
  }
  // entries to walk: up to the furthest last contributor of the tile
  int m = last;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
  if (lane_id() == 0) smax[threadIdx.x >> 6] = m;
  __syncthreads();
  const int maxlast = max(max(smax[0], smax[1]), max(smax[2], smax[3]));
  float T = Tfin;
  float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f, la = 0.f, lc0 = 0.f, lc1 = 0.f, lc2 = 0.f;
  const float4* rec = reinterpret_cast<const float4*>(a.rec);
  for (int b = ((maxlast - 1) / 256) * 256; maxlast > 0 && b >= 0; b -= 256) {
    __syncthreads();
    const int idx = b + (int)threadIdx.x;
    if (idx < maxlast) {
      const uint32_t id = a.vals[start + idx];
      if (id < a.n_rec) {
        s0[threadIdx.x] = rec[(size_t)id * 3];
        s1[threadIdx.x] = rec[(size_t)id * 3 + 1];
        s2[threadIdx.x] = rec[(size_t)id * 3 + 2];
      } else {
        s1[threadIdx.x] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
      sid[threadIdx.x] = id;
    }
    __syncthreads();
    const int nb = min(256, maxlast - b);
    for (int k = nb - 1; k >= 0; --k) {
      const float4 q0 = s0[k], q1 = s1[k];
      const float dx = q0.x - pxc, dy = q0.y - pyc;
      const float power = splat_power(q0.z, q0.w, q1.x, dx, dy);
      const float G = __expf(power);
      const float og = q1.y * G;
      const float alpha = fminf(ALPHA_MAX, og);
      const bool contrib = (b + k) < last && power <= 0.f && alpha >= ALPHA_MIN;
      // most splats of a batch blend into no pixel of the wave: skip them
      // before anything else (this loop is bound by VALU issue, and the
      // gradient registers' zeroing alone was a third of its instructions)
      if (!__ballot(contrib)) continue;
      float gu = 0.f, gv = 0.f, ga = 0.f, gb = 0.f, gc = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gbb = 0.f;
      if (contrib) {
        const float cb = s2[k].x;
        // 1 - alpha >= 0.01: the hardware reciprocal (1 ulp) replaces two
        // full divisions
        const float inv1ma = __builtin_amdgcn_rcpf(1.f - alpha);
        T = T * inv1ma;
        const float wgt = alpha * T;
        gr = wgt * g0;
        gg = wgt * g1;
        gbb = wgt * g2;
        // colour blended behind this splat: la lc + (1 - la) acc
        acc0 = fmaf(la, lc0 - acc0, acc0);
        acc1 = fmaf(la, lc1 - acc1, acc1);
        acc2 = fmaf(la, lc2 - acc2, acc2);
        lc0 = q1.z; lc1 = q1.w; lc2 = cb;
        float dLda = ((q1.z - acc0) * g0 + (q1.w - acc1) * g1 + (cb - acc2) * g2) * T;
        la = alpha;
        dLda += (-Tfin * inv1ma) * bgd;
        // a clamped alpha passes no gradient on (a select, not a branch:
        // this loop is bound by VALU issue)
        const float dLdo = og <= ALPHA_MAX ? dLda : 0.f;
        go = G * dLdo;
        const float dp = alpha * dLdo;
        gu = -dp * (q0.z * dx + q0.w * dy);
        gv = -dp * (q1.x * dy + q0.w * dx);
        ga = -0.5f * dp * dx * dx;
        gb = -dp * dx * dy;
        gc = -0.5f * dp * dy * dy;
      }
      {
        // record fields 0..7 summed transposed (lane 2f holds field f),
        // field 8 by a plain reduction
        const float v8[8] = {gu, gv, ga, gb, gc, go, gr, gg};
        const float t8 = wave_sum8_transposed(v8);
        const float t9 = wave_sum_dpp(gbb);
        // the record's 9 floats from 9 lanes of one instruction: one or two
        // 64-byte lines, so the atomics combine into one or two requests
        const int ln = lane_id();
        const uint32_t id = sid[k];
        if (ln < 16 && ((ln & 1) == 0 || ln == 1) && id < a.n_rec) {
          const int field = ln == 1 ? 8 : ln >> 1;
          atomicAdd(a.gs + (size_t)id * GS + field, ln == 1 ? t9 : t8);
        }
      }
    }
  }
}

// ---------------------------------------------------------------- projection
__global__ __launch_bounds__(256) void k_project_bwd(ProjBwdArgs a) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= *a.count) return;
  const int n = a.n;
  const int gi = a.vis_idx[s];
  const float pxf = a.pos[gi], pyf = a.pos[n + gi], pzf = a.pos[2 * n + gi];
  const float qw = a.quat[s], qx = a.quat[(size_t)n + s], qy = a.quat[2 * (size_t)n + s],
              qz = a.quat[3 * (size_t)n + s];
  const float Rq[3][3] = {{1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy)},
                          {2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx)},
                          {2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)}};
  float sc[3], s2[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    sc[d] = a.scale[(size_t)d * n + s];
    s2[d] = sc[d] * sc[d];
  }
  float Sig[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) Sig[k][l] = Rq[k][0] * s2[0] * Rq[l][0] + Rq[k][1] * s2[1] * Rq[l][1] + Rq[k][2] * s2[2] * Rq[l][2];
  float Gs[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  float dpos[3] = {0.f, 0.f, 0.f};
  float do_sum = 0.f;
  float dce[3] = {0.f, 0.f, 0.f};
  const float op = a.opacity[s];
  float dens_g = 0.f, dens_n = 0.f;
  for (int v = 0; v < a.cams.V; ++v) {
    const int4 rc = reinterpret_cast<const int4*>(a.rect)[(size_t)v * a.n_max + s];
    if (!(rc.z > rc.x && rc.w > rc.y)) {   // no tile entries in this view: no gradient
#pragma unroll
      for (int c = 0; c < 3; ++c) a.dcol[((size_t)v * 3 + c) * a.n_max + s] = 0.f;
      continue;
    }
    const float* gq = a.gs + ((size_t)v * a.n_max + s) * GS;
    const float du = gq[0], dv = gq[1], dca = gq[2], dcb = gq[3], dcc = gq[4];
    do_sum += gq[5];
    if (a.dens_accum) {
      // gradient with respect to the projected centre in NDC: d ndc_x = du * W/2
      const float nx = du * (0.5f * (float)a.cams.c[v].W), ny = dv * (0.5f * (float)a.cams.c[v].H);
      dens_g += sqrtf(nx * nx + ny * ny);
      dens_n += 1.f;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float col = a.rgb[((size_t)v * 3 + c) * n + s];
      const float dpre = gq[6 + c] * col * (1.f - col);
      dce[c] += dpre;
      a.dcol[((size_t)v * 3 + c) * a.n_max + s] = dpre;
    }
    const CamP& c = a.cams.c[v];
    double t[3];
    cam_space_f64(c, (double)pxf, (double)pyf, (double)pzf, t);
    const float tx = (float)t[0], ty = (float)t[1], tz = (float)t[2];
    const float iz = 1.0f / tz;
    const float j00 = c.fx * iz, j02 = -c.fx * tx * iz * iz;
    const float j11 = c.fy * iz, j12 = -c.fy * ty * iz * iz;
    float m0[3], m1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      m0[k] = j00 * c.R[k] + j02 * c.R[6 + k];
      m1[k] = j11 * c.R[3 + k] + j12 * c.R[6 + k];
    }
    float Sm0[3], Sm1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Sm0[k] = Sig[k][0] * m0[0] + Sig[k][1] * m0[1] + Sig[k][2] * m0[2];
      Sm1[k] = Sig[k][0] * m1[0] + Sig[k][1] * m1[1] + Sig[k][2] * m1[2];
    }
    const float A = DILATION + (m0[0] * Sm0[0] + m0[1] * Sm0[1] + m0[2] * Sm0[2]);
    const float B = m0[0] * Sm1[0] + m0[1] * Sm1[1] + m0[2] * Sm1[2];
    const float C = DILATION + (m1[0] * Sm1[0] + m1[1] * Sm1[1] + m1[2] * Sm1[2]);
    const float D = A * C - B * B;
    const float iD = 1.f / D, iD2 = iD * iD;
    // conic (C/D, -B/D, A/D) -> 2D covariance entries
    const float dA = dca * (-C * C * iD2) + dcb * (B * C * iD2) + dcc * (iD - A * C * iD2);
    const float dB = dca * (2.f * B * C * iD2) + dcb * (-iD - 2.f * B * B * iD2) + dcc * (2.f * A * B * iD2);
    const float dC = dca * (iD - A * C * iD2) + dcb * (A * B * iD2) + dcc * (-A * A * iD2);
    float dm0[3], dm1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      dm0[k] = 2.f * dA * Sm0[k] + dB * Sm1[k];
      dm1[k] = 2.f * dC * Sm1[k] + dB * Sm0[k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int l = 0; l < 3; ++l)
        Gs[k][l] += dA * m0[k] * m0[l] + 0.5f * dB * (m0[k] * m1[l] + m1[k] * m0[l]) + dC * m1[k] * m1[l];
    const float dJ00 = dm0[0] * c.R[0] + dm0[1] * c.R[1] + dm0[2] * c.R[2];
    const float dJ02 = dm0[0] * c.R[6] + dm0[1] * c.R[7] + dm0[2] * c.R[8];
    const float dJ11 = dm1[0] * c.R[3] + dm1[1] * c.R[4] + dm1[2] * c.R[5];
    const float dJ12 = dm1[0] * c.R[6] + dm1[1] * c.R[7] + dm1[2] * c.R[8];
    const float iz2 = iz * iz, iz3 = iz2 * iz;
    const float dtx = du * c.fx * iz - dJ02 * c.fx * iz2;
    const float dty = dv * c.fy * iz - dJ12 * c.fy * iz2;
    const float dtz = -du * c.fx * tx * iz2 - dv * c.fy * ty * iz2 - dJ00 * c.fx * iz2 +
                      dJ02 * 2.f * c.fx * tx * iz3 - dJ11 * c.fy * iz2 + dJ12 * 2.f * c.fy * ty * iz3;
#pragma unroll
    for (int k = 0; k < 3; ++k) dpos[k] += c.R[k] * dtx + c.R[3 + k] * dty + c.R[6 + k] * dtz;
  }
  // Sigma = Rq diag(s^2) Rq^T
  float dRq[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int m = 0; m < 3; ++m)
      dRq[k][m] = 2.f * (Gs[k][0] * Rq[0][m] + Gs[k][1] * Rq[1][m] + Gs[k][2] * Rq[2][m]) * s2[m];
  float ds_pre[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    float dd = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      dd += Rq[k][m] * (Gs[k][0] * Rq[0][m] + Gs[k][1] * Rq[1][m] + Gs[k][2] * Rq[2][m]);
    const float dsc = 2.f * sc[m] * dd;
    ds_pre[m] = dsc * sc[m] * (1.f - sc[m]);
  }
  const float dqw = 2.f * (-qz * dRq[0][1] + qy * dRq[0][2] + qz * dRq[1][0] - qx * dRq[1][2] - qy * dRq[2][0] + qx * dRq[2][1]);
  const float dqx = 2.f * (qy * dRq[0][1] + qz * dRq[0][2] + qy * dRq[1][0] - 2.f * qx * dRq[1][1] - qw * dRq[1][2] +
                           qz * dRq[2][0] + qw * dRq[2][1] - 2.f * qx * dRq[2][2]);
  const float dqy = 2.f * (-2.f * qy * dRq[0][0] + qx * dRq[0][1] + qw * dRq[0][2] + qx * dRq[1][0] + qz * dRq[1][2] -
                           qw * dRq[2][0] + qz * dRq[2][1] - 2.f * qy * dRq[2][2]);
  const float dqz = 2.f * (-2.f * qz * dRq[0][0] - qw * dRq[0][1] + qx * dRq[0][2] + qw * dRq[1][0] - 2.f * qz * dRq[1][1] +
                           qy * dRq[1][2] + qx * dRq[2][0] + qy * dRq[2][1]);
  const float do_pre = do_sum * op * (1.f - op);
  float* dg = a.dgeo + (size_t)s * 8;
  dg[0] = do_pre;
  dg[1] = ds_pre[0]; dg[2] = ds_pre[1]; dg[3] = ds_pre[2];
  dg[4] = dqw; dg[5] = dqx; dg[6] = dqy; dg[7] = dqz;
  // the gradient accumulators: every read first, then every write (the
  // compiler cannot tell the arrays apart, so interleaved read-add-writes
  // would each wait for the previous one)
  float cur[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) cur[k] = 0.f;
  if (a.dens_accum) { cur[0] = a.dens_accum[gi]; cur[1] = a.dens_count[gi]; }
  if (a.g_pos)
#pragma unroll
    for (int k = 0; k < 3; ++k) cur[2 + k] = a.g_pos[(size_t)k * n + gi];
  if (a.g_opac_e) cur[5] = a.g_opac_e[gi];
  if (a.g_scale_e)
#pragma unroll
    for (int k = 0; k < 3; ++k) cur[6 + k] = a.g_scale_e[(size_t)k * n + gi];
  if (a.g_col_e)
#pragma unroll
    for (int k = 0; k < 3; ++k) cur[9 + k] = a.g_col_e[(size_t)k * n + gi];
  if (a.dens_accum) {
    a.dens_accum[gi] = cur[0] + dens_g;
    a.dens_count[gi] = cur[1] + dens_n;
  }
  if (a.g_pos)
#pragma unroll
    for (int k = 0; k < 3; ++k) a.g_pos[(size_t)k * n + gi] = cur[2 + k] + dpos[k];
  if (a.g_opac_e) a.g_opac_e[gi] = cur[5] + do_pre;
  if (a.g_scale_e)
#pragma unroll
    for (int k = 0; k < 3; ++k) a.g_scale_e[(size_t)k * n + gi] = cur[6 + k] + ds_pre[k];
  if (a.g_col_e)
#pragma unroll
    for (int k = 0; k < 3; ++k) a.g_col_e[(size_t)k * n + gi] = cur[9 + k] + dce[k];
}

// ---------------------------------------------------------------- fields
template <class Sh, bool BF>
__global__ void k_prep_weights(const float* wg, const float* wc, void* fg, void* fc, void* bg, void* bc) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  if constexpr (BF) {
    permute_mlp_fwd_bf16<Sh>((__bf16*)fg, wg, false, tid, stride);
    permute_mlp_fwd_bf16<Sh>((__bf16*)fc, wc, true, tid, stride);
    permute_mlp_bwd_bf16<Sh>((__bf16*)bg, wg, false, tid, stride);
    permute_mlp_bwd_bf16<Sh>((__bf16*)bc, wc, true, tid, stride);
  } else {
    permute_mlp_fwd<Sh>((float*)fg, wg, false, tid, stride);
    permute_mlp_fwd<Sh>((float*)fc, wc, true, tid, stride);
    permute_mlp_bwd<Sh>((float*)bg, wg, false, tid, stride);
    permute_mlp_bwd<Sh>((float*)bc, wc, true, tid, stride);
  }
}

// Decoder recompute / adjoint in the chosen operand precision.
template <class Sh, bool BF>
struct Dec {
  using T = typename std::conditional<BF, __bf16, float>::type;
  static constexpr int SG = BF ? Sh::S_GEO1_8 : Sh::S_GEO1;
  static constexpr int SC = BF ? Sh::S_COL1_8 : Sh::S_COL1;
  template <int S1>
  static __device__ void fwd(const void* W, const float (&x)[S1], float (&h)[Sh::NH][Sh::S_HID], v4f& o, int lane) {
    if constexpr (BF) mlp_forward_keep_bf16<Sh, S1>((const __bf16*)W, x, h, o, lane);
    else mlp_forward_keep<Sh, S1>((const float*)W, x, h, o, lane);
  }
  template <bool COL, int S1, int ACC, int NWV, int CB = -1>
  static __device__ void bwd(const void* W, const float (&x)[S1], const float (&h)[Sh::NH][Sh::S_HID], v4f dout,
                             float (&dx)[S1], float* Xs, float* Ys, v4f (&acc)[ACC], int w, int lane) {
    if constexpr (BF) mlp_backward_bf16<Sh, COL, S1, ACC, NWV, CB>((const __bf16*)W, x, h, dout, dx, Xs, Ys, acc, w, lane);
    else mlp_backward<Sh, COL, S1, ACC, NWV, CB>((const float*)W, x, h, dout, dx, Xs, Ys, acc, w, lane);
  }
  // Colour decoder over several views with its input [f_rad ; PE(d_v)]
  // (Eq. 6): the first layer's product with the radiance features (lane
  // k-steps [0, FPL)) is formed once per point (col_first), each view adds
  // its direction part (col_fwd_rest); in the adjoint each view handles the
  // direction columns of the first layer (col_bwd_view) and sums its
  // first-layer output gradient, whose product with the features
  // (col_bwd_features: their dW tiles and dL/df_rad) is formed once.
  static constexpr int SPLIT = Sh::FPL;
  static constexpr int TIF = 2 * Sh::L / 16;   // first-layer input tiles of the features
  static_assert((2 * Sh::L) % 16 == 0 && SPLIT % (BF ? 8 : 4) == 0, "feature columns must fill whole tiles");
  static __device__ void col_first(const void* W, const float (&x)[SC], v4f (&acc)[Sh::NT], int lane) {
    if constexpr (BF) mlp_first_part_bf16<Sh, SC, SPLIT>((const __bf16*)W, x, acc, lane);
    else mlp_first_part<Sh, SC, SPLIT>((const float*)W, x, acc, lane);
  }
  static __device__ void col_fwd_rest(const void* W, const float (&x)[SC], v4f (&acc)[Sh::NT],
                                      float (&h)[Sh::NH][Sh::S_HID], v4f& o, int lane) {
    if constexpr (BF) mlp_forward_keep_rest_bf16<Sh, SC, SPLIT>((const __bf16*)W, x, acc, h, o, lane);
    else mlp_forward_keep_rest<Sh, SC, SPLIT>((const float*)W, x, acc, h, o, lane);
  }
  template <int ACC, int NWV>
  static __device__ void col_bwd_view(const void* W, const float (&x)[SC], const float (&h)[Sh::NH][Sh::S_HID],
                                      v4f dout, float (&dx)[SC], float (&dh_sum)[Sh::S_HID], float* Xs, float* Ys,
                                      v4f (&acc)[ACC], int w, int lane) {
    using B = BwdShape<Sh>;
    float dh[Sh::S_HID];
    if constexpr (BF) {
      const __bf16* W1 = mlp_backward_upper_bf16<Sh, true, ACC, NWV>((const __bf16*)W, h, dout, dh, Xs, Ys, acc, w, lane);
      mlp_backward_first_bf16<Sh, true, SC, SPLIT, SC, TIF, B::TI_COL1, ACC, NWV>(W1, x, dh, dx, Xs, Ys, acc, w, lane);
    } else {
      const float* W1 = mlp_backward_upper<Sh, true, ACC, NWV>((const float*)W, h, dout, dh, Xs, Ys, acc, w, lane);
      mlp_backward_first<Sh, true, SC, SPLIT, SC, TIF, B::TI_COL1, ACC, NWV>(W1, x, dh, dx, Xs, Ys, acc, w, lane);
    }
#pragma unroll
    for (int k = 0; k < Sh::S_HID; ++k) dh_sum[k] += dh[k];
  }
  template <int ACC, int NWV>
  static __device__ void col_bwd_features(const void* W, const float (&x)[SC], const float (&dh_sum)[Sh::S_HID],
                                          float (&dx)[SC], float* Xs, float* Ys, v4f (&acc)[ACC], int w, int lane) {
    // the first layer's adjoint operands follow the output and hidden layers'
    if constexpr (BF) {
      const __bf16* W1 = (const __bf16*)W + Sh::NT * 8 * 64 + (Sh::NH - 1) * Sh::NT * Sh::S_HID * 64;
      mlp_backward_first_bf16<Sh, true, SC, 0, SPLIT, 0, TIF, ACC, NWV>(W1, x, dh_sum, dx, Xs, Ys, acc, w, lane);
    } else {
      const float* W1 = (const float*)W + Sh::NT * 4 * 64 + (Sh::NH - 1) * Sh::NT * Sh::S_HID * 64;
      mlp_backward_first<Sh, true, SC, 0, SPLIT, 0, TIF, ACC, NWV>(W1, x, dh_sum, dx, Xs, Ys, acc, w, lane);
    }
  }
};

// Write the dW tiles of one layer (tile ids ID0 ..) owned by this wave.
template <int ID0, int TO, int TI, int ACC, int NWV, bool ITMAJ = false>
__device__ __forceinline__ void write_dw_layer(float* dst, int rows, int in, const v4f (&acc)[ACC], int w, int lane) {
  const int j = lane & 15, g = lane >> 4;
  static_for<0, TO * TI>([&](auto tc) {
    constexpr int t = decltype(tc)::value;
    constexpr int id = ID0 + t;
    constexpr int ot = tile_ot<TO, TI, ITMAJ>(t), it = tile_it<TO, TI, ITMAJ>(t);
    if (id % NWV == w) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * ot + 4 * g + r, col = 16 * it + j;
        if (row < rows && col < in) dst[row * in + col] = acc[id / NWV][r];
      }
    }
  });
}

// WITH_GEO false: the kernel ran no geometry decoder and numbers the colour
// decoder's tiles from 0; its geometry partials are written as zeros.
template <class Sh, int ACC, int NWV, bool WITH_GEO = true>
__device__ void write_dw(float* part, const v4f (&acc)[ACC], int w, int lane) {
  using B = BwdShape<Sh>;
  constexpr int TH = Sh::HID / 16;
  float* dst = part;
  constexpr int N_GEO = Sh::N_GEO;
  if constexpr (WITH_GEO) {
    write_dw_layer<0, Sh::NT, B::TI_GEO1, ACC, NWV>(dst, Sh::HID, Sh::IN_GEO, acc, w, lane);
    dst += Sh::HID * Sh::IN_GEO;
    constexpr int G1 = Sh::NT * B::TI_GEO1;
    if constexpr (Sh::NH == 2) {
      write_dw_layer<G1, Sh::NT, TH, ACC, NWV>(dst, Sh::HID, Sh::HID, acc, w, lane);
      dst += Sh::HID * Sh::HID;
    }
    constexpr int G2 = G1 + (Sh::NH - 1) * Sh::NT * TH;
    write_dw_layer<G2, 1, TH, ACC, NWV>(dst, HYRF_GEO_OUT, Sh::HID, acc, w, lane);
    dst += HYRF_GEO_OUT * Sh::HID;
  } else {
    for (int e = w * 64 + lane; e < N_GEO; e += NWV * 64) dst[e] = 0.f;
    dst += N_GEO;
  }
  // colour MLP
  constexpr int C0 = WITH_GEO ? B::TILES_GEO : 0;
  write_dw_layer<C0, Sh::NT, B::TI_COL1, ACC, NWV, true>(dst, Sh::HID, Sh::IN_COL, acc, w, lane);
  dst += Sh::HID * Sh::IN_COL;
  constexpr int C1 = C0 + Sh::NT * B::TI_COL1;
  if constexpr (Sh::NH == 2) {
    write_dw_layer<C1, Sh::NT, TH, ACC, NWV>(dst, Sh::HID, Sh::HID, acc, w, lane);
    dst += Sh::HID * Sh::HID;
  }
  constexpr int C2 = C1 + (Sh::NH - 1) * Sh::NT * TH;
  write_dw_layer<C2, 1, TH, ACC, NWV>(dst, HYRF_COL_OUT, Sh::HID, acc, w, lane);
}

// Contraction Jacobian transpose: dL/dp from dL/dx (App. A.1 map).
__device__ __forceinline__ void contract_vjp(const GridP& gp, float px, float py, float pz, const float dx[3],
                                             float dp[3]) {
  const float q[3] = {(px - gp.center[0]) * gp.inv_half[0], (py - gp.center[1]) * gp.inv_half[1],
                      (pz - gp.center[2]) * gp.inv_half[2]};
  const float dm[3] = {0.25f * dx[0], 0.25f * dx[1], 0.25f * dx[2]};
  const float n2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
  float dq[3];
  if (n2 > 1.f) {
    const float nn = sqrtf(n2);
    const float s = (2.f - 1.f / nn) / nn;
    const float k = 2.f * (1.f - nn) / (n2 * n2);
    const float qd = q[0] * dm[0] + q[1] * dm[1] + q[2] * dm[2];
#pragma unroll
    for (int d = 0; d < 3; ++d) dq[d] = s * dm[d] + k * q[d] * qd;
  } else {
#pragma unroll
    for (int d = 0; d < 3; ++d) dq[d] = dm[d];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) dp[d] = dq[d] * gp.inv_half[d];
}

// ---- cell-run scatter of a level's 8 corners x 2 features
//
// A float atomic costs one memory request per 64-byte line touched by a wave
// instruction: lanes of one instruction that hit the same line combine, lanes
// that hit the same ADDRESS do not, and requests to distinct lines issue at
// one per clock of the memory-side atomic units.  So the table adjoints (1)
// sum, in registers, the contributions of consecutive lanes whose points lie
// in the same grid cell (runs: spatially ordered Gaussians, adjacent pixels),
// then (2) stage each run total's 16 floats in LDS and issue them 16 lanes
// per cell, corner-major: corners c and c^1 differ in x only and are adjacent
// rows whenever the cell's x index is even, so one instruction touches a few
// lines per cell instead of one line per float.
// Run totals staged per wave and pass: NC cells of 16 words (144 B each).
template <int NC>
struct CellStageN {
  uint32_t idx[NC * 16];
  float val[NC * 16];
  int4 cell[NC];                    // grid coordinates of each staged cell
};
// Gaussian scatters: a wave has at most 64 cells, so every level takes one
// pass (9 KB per wave; the kernels' registers, not LDS, bound occupancy)
constexpr int STAGE_CELLS = 64;
using CellStage = CellStageN<STAGE_CELLS>;
static_assert(sizeof(CellStage) <= 9216, "cell stage size");

// Word of corner c (feature 0; feature 1 follows) of staged cell `slot`.
__device__ __forceinline__ int stage_at(int slot, int c) { return slot * 16 + 4 * ((c >> 1) ^ (slot & 3)) + 2 * (c & 1); }

// Order of LDS accesses between the lanes of one wave (staging writes, then
// other lanes' reads, then rewrites).  The LDS performs one wave's
// operations in issue order, so a compiler fence that keeps the program
// order suffices; no wait for the counter is needed (a loaded value is
// still waited for where it is used).
__device__ __forceinline__ void wave_lds_sync() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

// Lanes whose cell differs from the previous lane's (lane 0 always).
__device__ __forceinline__ uint64_t cell_heads(const int (&ci)[3]) {
  const int lane = lane_id();
  const int p0 = wave_shr1(ci[0]), p1 = wave_shr1(ci[1]), p2 = wave_shr1(ci[2]);
  return __ballot(lane == 0 || p0 != ci[0] || p1 != ci[1] || p2 != ci[2]);
}

// Segmented inclusive sums of v over the runs that start at the set bits of
// `heads`: every lane ends with the sum of its run up to itself (so the last
// lane of a run holds the run's totals).  All lane moves are DPP, none goes
// through LDS: doubling steps inside each 16-lane row (row_shr 1, 2, 4, 8),
// then the rows' last lanes carried across (row_bcast 15, row_bcast 31) to
// the lanes whose run began in an earlier row.  Only as many in-row steps
// as the longest run needs are taken (every run is at most 2^k lanes long
// exactly when each lane has a head among itself and its 2^k - 1
// predecessors), and a carry only where a row's first lane is no head.
template <int N>
__device__ __forceinline__ void run_sums(uint64_t heads, float (&v)[N]) {
  int steps = 0;
  for (uint64_t cover = heads; cover != ~0ull && steps < 6; ++steps) cover |= cover << (1 << steps);
  if (steps == 0) return;   // every lane its own run
  const int lane = lane_id();
  const uint64_t upto = lane == 63 ? heads : heads & ((2ull << lane) - 1ull);
  const int head = 63 - __clzll((long long)upto);
  const int col = lane & 15, row0 = lane & ~15;
  static_for<0, 4>([&](auto sc) {
    constexpr int off = 1 << decltype(sc)::value;
    if (decltype(sc)::value < steps) {
      const bool take = col >= off && lane - off >= head;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const float t = row_shr<off>(v[k]);
        if (take) v[k] += t;
      }
    }
  });
  // rows 1 and 3: lanes 15 and 47 hold their run's sum over rows 0 and 2
  if (!((heads >> 16) & 1ull) || !((heads >> 48) & 1ull)) {
    const bool take = ((lane >> 4) & 1) && head < row0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const float t = row_bcast15(v[k]);
      if (take) v[k] += t;
    }
  }
  // rows 2 and 3: lane 31 holds its run's sum over rows 0 and 1
  if (!((heads >> 32) & 1ull)) {
    const bool take = lane >= 32 && head < 32;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const float t = row_bcast31(v[k]);
      if (take) v[k] += t;
    }
  }
}

// Add the run totals of one level to a table-gradient level g ([T][2]):
// the last lane of each run holds 16 floats, row[c] * 2 + f <- v[2c + f],
// for the cell ci.  Every lane of the wave must call it.  A staged cell
// occupies 16 consecutive words; its four 16-byte quarters are XOR-swizzled
// by the cell's slot so that tail lanes of consecutive slots write
// different banks.  The issue loop reads the slots linearly: every
// instruction covers whole cells.
//
// MERGE: consecutive cells are usually grid neighbours (along a pixel row,
// or in spatial order) and then share corners: the same addresses in one
// instruction, which cost one request each.  So before issue, a corner that
// a cell shares with the next staged cell moves there (the next cell adds
// the original value, this cell drops it); the totals are unchanged.  Along
// pixel rows this removes 39% of the background scatter's requests; it pays
// where the scatter is bound by them (see the callers).
template <bool MERGE, int NC>
__device__ __forceinline__ void scatter_tails(float* __restrict__ g, uint64_t heads, const int (&ci)[3],
                                              const uint32_t (&row)[8], const float* v, CellStageN<NC>& st) {
  const int lane = lane_id();
  const uint64_t tails = (heads >> 1) | (1ull << 63);
  const bool tail = (tails >> lane) & 1ull;
  const int rank = __popcll(tails & ((1ull << lane) - 1ull));
  const int K = __popcll(tails);
  for (int b = 0; b < K; b += NC) {
    const bool mine = tail && rank >= b && rank < b + NC;
    const int cell = rank - b;
    const int nc = min(K - b, NC);
    if (mine) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int at = stage_at(cell, c);
        st.idx[at] = row[c] * 2u;
        st.idx[at + 1] = row[c] * 2u + 1u;
        st.val[at] = v[2 * c];
        st.val[at + 1] = v[2 * c + 1];
      }
      st.cell[cell] = make_int4(ci[0], ci[1], ci[2], 0);
    }
    wave_lds_sync();
    if constexpr (MERGE) {
    // corners shared with the neighbouring slots, from the original values
    float nv[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) nv[k] = v[k];
    if (mine && cell + 1 < nc) {
      const int4 s = st.cell[cell + 1];
      const int dx = s.x - ci[0], dy = s.y - ci[1], dz = s.z - ci[2];
      if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          // the next cell holds this corner if its offset there lies in {0,1}^3
          const int ox = (c & 1) - dx, oy = ((c >> 1) & 1) - dy, oz = ((c >> 2) & 1) - dz;
          if ((unsigned)ox <= 1u && (unsigned)oy <= 1u && (unsigned)oz <= 1u) {
            nv[2 * c] = 0.f;
            nv[2 * c + 1] = 0.f;
          }
        }
      }
    }
    if (mine && cell > 0) {
      const int4 p = st.cell[cell - 1];
      const int dx = ci[0] - p.x, dy = ci[1] - p.y, dz = ci[2] - p.z;
      if (abs(dx) <= 1 && abs(dy) <= 1 && abs(dz) <= 1) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int ox = (c & 1) + dx, oy = ((c >> 1) & 1) + dy, oz = ((c >> 2) & 1) + dz;
          if ((unsigned)ox <= 1u && (unsigned)oy <= 1u && (unsigned)oz <= 1u) {
            const int at = stage_at(cell - 1, ox | (oy << 1) | (oz << 2));
            nv[2 * c] += st.val[at];
            nv[2 * c + 1] += st.val[at + 1];
          }
        }
      }
    }
    wave_lds_sync();   // every original read before any slot is rewritten
    if (mine) {
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int at = stage_at(cell, c);
        st.val[at] = nv[2 * c];
        st.val[at + 1] = nv[2 * c + 1];
      }
    }
    wave_lds_sync();
    }
    const int n = nc * 16;
    for (int s2 = lane; s2 < n; s2 += 64) {
      const float x = st.val[s2];
      if (x != 0.f) atomicAdd(g + st.idx[s2], x);
    }
    wave_lds_sync();
  }
}



// One level of one table for the whole wave: the 8 corner rows and trilinear
// weights of each lane's cell, w_c * dL/df summed over cell runs, then the
// staged scatter.  Every lane of the wave must call it.
template <bool MERGE, int NC>
__device__ __forceinline__ void scatter_level(float* __restrict__ g, uint64_t heads, const int (&ci)[3],
                                              const float (&wv)[3], float2 df, bool dense, uint32_t side,
                                              uint32_t mask, CellStageN<NC>& st) {
  uint32_t row[8];
  float sv[16];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
    const float wc = ((bx ? wv[0] : 1.f - wv[0]) * (by ? wv[1] : 1.f - wv[1])) * (bz ? wv[2] : 1.f - wv[2]);
    row[c] = corner_row((uint32_t)ci[0] + bx, (uint32_t)ci[1] + by, (uint32_t)ci[2] + bz, dense, side, mask);
    sv[2 * c] = wc * df.x;
    sv[2 * c + 1] = wc * df.y;
  }
  run_sums<16>(heads, sv);
  scatter_tails<MERGE, NC>(g, heads, ci, row, sv, st);
}

// Radiance-table scatter of one round of background pixels, inside the
// background decoder adjoint (Sec. 3.3): the round's feature gradients sit
// in LDS ([pixel][BG_DF_STRIDE], pixel-major), and the 8 waves split the
// work as 2 halves of 64 consecutive pixels x 4 level groups (levels
// lg, lg + 4, ...).  The pixels' contracted sphere points (float64, the
// same cells as the forward gather) come from LDS too.  The atomics do not
// return; the wave's next global read waits for them (its memory counter
// completes in issue order).
constexpr int BG_DF_STRIDE = 34;   // 2L + 2 floats: float2 rows spread over the LDS banks
// Cells staged per wave and pass: at the finest levels each of a wave's 64
// pixels has a cell of its own, and every pass repeats the staging and
// merging code for the whole wave.  40 (5.8 KB per wave) fit beside the
// feature gradients in the dW staging space; 64 would push the kernel's LDS
// to 159 KB, leaving no room for the blending adjoint's workgroups that run
// beside it on the CU
constexpr int BG_STAGE_CELLS = 40;
using BgCellStage = CellStageN<BG_STAGE_CELLS>;

template <int L, bool MERGE>
__device__ __forceinline__ void bg_round_scatter(const FieldBwdArgs& a, const float* sdf, const double* sx,
                                                 BgCellStage& st, int w) {
  static_assert(2 * L + 2 <= BG_DF_STRIDE, "LDS row too short");
  const int lane = lane_id();
  const int pl = (w & 1) * 64 + lane;
  const int lg = w >> 1;
  // the pixel's contracted sphere point, computed once by the decoder phase
  const double x[3] = {sx[3 * pl], sx[3 * pl + 1], sx[3 * pl + 2]};
  const uint32_t Tr = a.grid.mask_rad + 1u;
#pragma unroll 1
  for (int k = 0; k < L / 4; ++k) {
    const int lev = lg + 4 * k;
    const int res = a.grid.res[lev];
    int ci[3];
    float wv[3];
    grid_cell(x, res, ci, wv);
    const float2 df = *reinterpret_cast<const float2*>(sdf + pl * BG_DF_STRIDE + 2 * lev);
    scatter_level<MERGE, BG_STAGE_CELLS>(a.g_table_rad + (size_t)lev * Tr * 2, cell_heads(ci), ci, wv, df, (a.grid.dense_rad >> lev) & 1u,
                  (uint32_t)res + 1u, a.grid.mask_rad, st);
  }
}

// Waves per workgroup.  Background pixels run only the colour decoder: its
// weights and the staging of 8 waves fit LDS, and 8 waves hide latency.
// Gaussians run both decoders: with 4 waves the staging shrinks enough that
// both decoders' weights sit in LDS too.
template <bool RAY>
constexpr int bwd_waves() { return RAY ? 8 : 4; }

// SAVED (background points): the forward kept their radiance features
// (a.bg_feat), and the kernel carries no gather (60 fewer registers per
// lane); else the adjoint gathers them again.
template <class Sh, bool RAY, class TT, bool BF, bool SAVED = false>
__global__ __launch_bounds__(bwd_waves<RAY>() * 64) void k_field_bwd(FieldBwdArgs a) {
  using B = BwdShape<Sh>;
  using D = Dec<Sh, BF>;
  constexpr int NWV = bwd_waves<RAY>();
  constexpr int NT = NWV * 64;
  constexpr int PPR = NWV * 16;   // points per round
  // background points run only the colour decoder: its tiles numbered from 0
  constexpr int CB = RAY ? 0 : B::TILES_GEO;
  constexpr int ACC = RAY ? (B::TILES_COL + NWV - 1) / NWV : B::template ACC<NWV>;
  // the dW operand staging X (inputs) and Y (output gradients) of a round
  __shared__ __attribute__((aligned(16))) float XY[2 * PPR * STAGE_W];
  float* const Xs = XY;
  float* const Ys = XY + PPR * STAGE_W;
  // the colour decoder's permuted weights (forward and adjoint operand
  // orders; float32 or bfloat16 bytes) live in LDS for the whole persistent
  // loop: every MFMA A operand is then an LDS read, not an L2 round trip
  __shared__ __attribute__((aligned(16))) float s_wf_col[Sh::W_COL];
  __shared__ __attribute__((aligned(16))) float s_wb_col[B::WB_COL];
  // the geometry decoder's too, for the Gaussians; for background pixels
  // the same space holds the round's contracted sphere points (float64,
  // two buffers by round parity: a wave may still scatter round r while
  // another starts round r + 1)
  __shared__ __attribute__((aligned(16))) float s_wf_geo[RAY ? 2 * PPR * 3 * 2 : Sh::W_GEO];
  __shared__ __attribute__((aligned(16))) float s_wb_geo[RAY ? 4 : B::WB_GEO];
  {
    const float4* src_f = reinterpret_cast<const float4*>(a.wf_col);
    const float4* src_b = reinterpret_cast<const float4*>(a.wb_col);
    for (int i = threadIdx.x; i < Sh::W_COL / 4; i += NT) reinterpret_cast<float4*>(s_wf_col)[i] = src_f[i];
    for (int i = threadIdx.x; i < B::WB_COL / 4; i += NT) reinterpret_cast<float4*>(s_wb_col)[i] = src_b[i];
    if constexpr (!RAY) {
      const float4* gf = reinterpret_cast<const float4*>(a.wf_geo);
      const float4* gb = reinterpret_cast<const float4*>(a.wb_geo);
      for (int i = threadIdx.x; i < Sh::W_GEO / 4; i += NT) reinterpret_cast<float4*>(s_wf_geo)[i] = gf[i];
      for (int i = threadIdx.x; i < B::WB_GEO / 4; i += NT) reinterpret_cast<float4*>(s_wb_geo)[i] = gb[i];
    }
    __syncthreads();
  }
  const int lane = lane_id();
  const int j = lane & 15, g = lane >> 4;
  const int w = threadIdx.x / 64;
  v4f accW[ACC];
#pragma unroll
  for (int k = 0; k < ACC; ++k) accW[k] = v4f{0.f, 0.f, 0.f, 0.f};
  const int HW = a.W * a.H;
  const int count = RAY ? a.cams.V * HW : *a.count;
  const int rounds = (count + PPR - 1) / PPR;
  const uint32_t Tg = a.grid.mask_geo + 1u, Tr = a.grid.mask_rad + 1u;
  const int V = a.cams.V;
  // Gaussians: rounds strided over workgroups; background pixels: each
  // workgroup owns a contiguous band of rounds (image rows), so the coarse
  // cells it touches repeat and stay in its private map
  const int per_blk = (rounds + (int)gridDim.x - 1) / (int)gridDim.x;
  const int r_begin = RAY ? (int)blockIdx.x * per_blk : (int)blockIdx.x;
  const int r_end = RAY ? min(rounds, r_begin + per_blk) : rounds;
  const int r_step = RAY ? 1 : (int)gridDim.x;
  for (int round = r_begin; round < r_end; round += r_step) {
    const int item = round * PPR + w * 16 + j;
    const bool valid = item < count;
    float fg[Sh::FPL], fr[Sh::FPL];
    double x[3];
    float pxf = 0.f, pyf = 0.f, pzf = 0.f;
    int gi = 0, v_r = 0, pix = 0;
    float dfr[Sh::FPL], dxg[D::SG];
    float dgeo_in[4] = {0.f, 0.f, 0.f, 0.f}, rot_in[4] = {0.f, 0.f, 0.f, 0.f}, dcol_in[3] = {0.f, 0.f, 0.f};
    float bg_T = 0.f, bg_dL[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < Sh::FPL; ++s) dfr[s] = 0.f;
#pragma unroll
    for (int s = 0; s < D::SG; ++s) dxg[s] = 0.f;
    float dp_dir[3] = {0.f, 0.f, 0.f};
    if constexpr (!RAY) {
      // the features (indexed by the list position) are read before the
      // Gaussian's index, whose wait then covers them too
#pragma unroll
      for (int k = 0; k < Sh::L / 4; ++k) {
        const int lev = g + 4 * k;
        const int itc = valid ? item : 0;
        const float2 vg = *reinterpret_cast<const float2*>(a.feat_geo + (size_t)itc * 2 * Sh::L + 2 * lev);
        const float2 vr = *reinterpret_cast<const float2*>(a.feat_rad + (size_t)itc * 2 * Sh::L + 2 * lev);
        fg[2 * k] = valid ? vg.x : 0.f; fg[2 * k + 1] = valid ? vg.y : 0.f;
        fr[2 * k] = valid ? vr.x : 0.f; fr[2 * k + 1] = valid ? vr.y : 0.f;
      }
      gi = valid ? a.vis_idx[item] : a.vis_idx[0];
      pxf = a.pos[gi]; pyf = a.pos[a.n + gi]; pzf = a.pos[2 * a.n + gi];
      // the output gradients of both decoders (view 0) and the explicit
      // rotation are read here, so that their latency hides under the
      // forward recomputation (the MFMA layers' scheduling barriers keep
      // later reads from moving up); rows of item 0 for an invalid lane
      {
        const int itc = valid ? item : 0;
        const float4 d4 = *reinterpret_cast<const float4*>(a.dgeo + (size_t)itc * 8 + 4 * (g & 1));
        dgeo_in[0] = d4.x; dgeo_in[1] = d4.y; dgeo_in[2] = d4.z; dgeo_in[3] = d4.w;
#pragma unroll
        for (int k = 0; k < 4; ++k) rot_in[k] = a.rot_e ? a.rot_e[(size_t)k * a.n + gi] : 0.f;
#pragma unroll
        for (int c = 0; c < 3; ++c) dcol_in[c] = a.dcol[(size_t)c * a.n_max + itc];
      }
      // ---- geometry decoder adjoint
      float x1g[D::SG];
#pragma unroll
      for (int s = 0; s < D::SG; ++s) x1g[s] = s < Sh::FPL ? fg[s] : 0.f;
      float hg[Sh::NH][Sh::S_HID];
      v4f og;
      D::template fwd<D::SG>(s_wf_geo, x1g, hg, og, lane);
      v4f dg = v4f{0.f, 0.f, 0.f, 0.f};
      if (valid && g == 0) dg = v4f{dgeo_in[0], dgeo_in[1], dgeo_in[2], dgeo_in[3]};
      if (valid && g == 1) {
        // rotation rows: q = r / |r| with r = r_n (+ r_e)
        const float* d = dgeo_in;
        float r[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) r[k] = og[k] + rot_in[k];
        const float nr = sqrtf((r[0] * r[0] + r[1] * r[1]) + (r[2] * r[2] + r[3] * r[3]));
        const float inr = 1.f / nr;
        float q[4], qd = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          q[k] = r[k] * inr;
          qd += q[k] * d[k];
        }
        float dr[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) dr[k] = (d[k] - q[k] * qd) * inr;
        dg = v4f{dr[0], dr[1], dr[2], dr[3]};
        if (a.g_rot_e && a.rot_e) {
          // the four reads first (the compiler cannot tell the rows apart,
          // so an interleaved read-add-write would serialise them)
          float cur[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) cur[k] = a.g_rot_e[(size_t)k * a.n + gi];
#pragma unroll
          for (int k = 0; k < 4; ++k) a.g_rot_e[(size_t)k * a.n + gi] = cur[k] + dr[k];
        }
      }
      D::template bwd<false, D::SG, ACC, NWV>(s_wb_geo, x1g, hg, dg, dxg, Xs, Ys, accW, w, lane);
    } else {
      pix = valid ? item : 0;
      v_r = pix / HW;
      const int rem = pix - v_r * HW;
      const int yy = rem / a.W, xx = rem - yy * a.W;
      double ps[3], d[3];
      sphere_point_f64(a.cams.c[v_r], xx, yy, (double)a.grid.bg_radius, ps, d);
      contract_f64(a.grid, ps[0], ps[1], ps[2], x);
      if (g == 0 && a.g_table_rad) {
        double* sx = reinterpret_cast<double*>(s_wf_geo) + (round & 1) * PPR * 3;
        const int pl = w * 16 + j;
        sx[3 * pl] = x[0];
        sx[3 * pl + 1] = x[1];
        sx[3 * pl + 2] = x[2];
      }
      if constexpr (SAVED) {
        // features saved by the forward
#pragma unroll
        for (int k = 0; k < Sh::L / 4; ++k) {
          const float2 f2 = *reinterpret_cast<const float2*>(a.bg_feat + (size_t)pix * 2 * Sh::L + 2 * (g + 4 * k));
          fr[2 * k] = f2.x;
          fr[2 * k + 1] = f2.y;
        }
      }
      // the pixel's final transmittance and dL/dC, read here so that their
      // latency hides under the forward recomputation (every lane reads
      // them; the lanes of group 0 use them)
      {
        const int rem = pix - v_r * HW;
        bg_T = a.T_final[pix];
#pragma unroll
        for (int c = 0; c < 3; ++c) bg_dL[c] = a.dL[((size_t)v_r * 3 + c) * HW + rem];
      }
      if constexpr (!SAVED) {
        gather_lane<Sh::L, false, TT>(a.grid, x, g, nullptr, (const TT*)a.table_rad, fg, fr, nullptr, nullptr);
      }
      const double dn = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
      pxf = (float)(d[0] / dn); pyf = (float)(d[1] / dn); pzf = (float)(d[2] / dn);
      if (!valid) {
#pragma unroll
        for (int s = 0; s < Sh::FPL; ++s) fr[s] = 0.f;
      }
    }
    // Gaussians: the saved feature derivatives this lane combines at the
    // end of the round are read before the colour decoder's adjoint, whose
    // work hides their latency
    float jv[RAY ? 1 : Sh::L / 4][12];
    if constexpr (!RAY) {
      if (a.jac) {
        const int itc = valid ? item : 0;
#pragma unroll
        for (int k = 0; k < Sh::L / 4; ++k) {
          const float4* J4 = reinterpret_cast<const float4*>(a.jac + ((size_t)itc * Sh::L + g + 4 * k) * 12);
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            const float4 t = J4[q];
            jv[k][4 * q] = t.x; jv[k][4 * q + 1] = t.y; jv[k][4 * q + 2] = t.z; jv[k][4 * q + 3] = t.w;
          }
        }
      }
    }
    // ---- colour decoder adjoint, once per view (one pass in ray mode).
    // With several views the first layer's radiance-feature part is shared
    // (Eq. 6): formed once forward, its adjoint once after the views.
    const int nviews = RAY ? 1 : V;
    const bool shared = !RAY && V > 1;
    v4f col1[Sh::NT];
    float dh_sum[Sh::S_HID];
    float x1f[D::SC];
#pragma unroll
    for (int s = 0; s < D::SC; ++s) x1f[s] = (valid && s < Sh::FPL) ? fr[s] : 0.f;
    if (shared) {
      D::col_first(s_wf_col, x1f, col1, lane);
#pragma unroll
      for (int k = 0; k < Sh::S_HID; ++k) dh_sum[k] = 0.f;
    }
    for (int v = 0; v < nviews; ++v) {
      // Gaussians: the next view's colour gradient is read ahead (the
      // current view's arrived during the previous view or the round start)
      float dcol_next[3] = {0.f, 0.f, 0.f};
      if constexpr (!RAY) {
        if (v + 1 < nviews) {
          const int itc = valid ? item : 0;
#pragma unroll
          for (int c = 0; c < 3; ++c) dcol_next[c] = a.dcol[((size_t)(v + 1) * 3 + c) * a.n_max + itc];
        }
      }
      float dir[3];
      float inv_len = 0.f;
      if constexpr (!RAY) {
        float oc[3];
        cam_center_f32(a.cams.c[v], oc);
        dir[0] = pxf - oc[0]; dir[1] = pyf - oc[1]; dir[2] = pzf - oc[2];
        inv_len = 1.0f / sqrtf((dir[0] * dir[0] + dir[1] * dir[1]) + dir[2] * dir[2]);
        dir[0] *= inv_len; dir[1] *= inv_len; dir[2] *= inv_len;
      } else {
        dir[0] = pxf; dir[1] = pyf; dir[2] = pzf;
      }
      float pe[6];
      pe_lane(g, dir[0], dir[1], dir[2], pe);
      float x1c[D::SC];
#pragma unroll
      for (int s = 0; s < D::SC; ++s)
        x1c[s] = !valid ? 0.f : (s < Sh::FPL ? fr[s] : (s < Sh::FPL + 6 ? pe[s < Sh::FPL + 6 ? (s - Sh::FPL) : 0] : 0.f));
      float hc[Sh::NH][Sh::S_HID];
      v4f oc4;
      if (shared) {
        v4f acc1[Sh::NT];
#pragma unroll
        for (int t = 0; t < Sh::NT; ++t) acc1[t] = col1[t];
        D::col_fwd_rest(s_wf_col, x1c, acc1, hc, oc4, lane);
      } else {
        D::template fwd<D::SC>(s_wf_col, x1c, hc, oc4, lane);
      }
      v4f dc = v4f{0.f, 0.f, 0.f, 0.f};
      if (valid && g == 0) {
        if constexpr (!RAY) {
          dc = v4f{dcol_in[0], dcol_in[1], dcol_in[2], 0.f};
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float cs = sigmoidf_(oc4[c]);
            dc[c] = bg_T * bg_dL[c] * cs * (1.f - cs);
          }
        }
      }
      float dxc[D::SC];
      // background rounds: the previous round's scatter (LDS staging in Xs,
      // feature gradients in Ys) may still run on other waves up to here;
      // the forward above needs no LDS staging, so the wait sits just
      // before the adjoint's first staging write
      if constexpr (RAY) __syncthreads();
      if (shared) {
        // background points never share (and their dW tiles are numbered
        // without the geometry decoder's): not instantiated for them
        if constexpr (!RAY) D::template col_bwd_view<ACC, NWV>(s_wb_col, x1c, hc, dc, dxc, dh_sum, Xs, Ys, accW, w, lane);
      } else {
        D::template bwd<true, D::SC, ACC, NWV, CB>(s_wb_col, x1c, hc, dc, dxc, Xs, Ys, accW, w, lane);
#pragma unroll
        for (int s = 0; s < Sh::FPL; ++s) dfr[s] += dxc[s];
      }
      if constexpr (!RAY) {
        // PE of octave g: d sin(a d)/dd = a cos(a d), d cos(a d)/dd = -a sin(a d)
        const float af = 3.14159265358979323846f * (float)(1 << g);
        float dd[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) dd[k] = af * (dxc[Sh::FPL + k] * pe[3 + k] - dxc[Sh::FPL + 3 + k] * pe[k]);
        const float dot = dir[0] * dd[0] + dir[1] * dd[1] + dir[2] * dd[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) dp_dir[k] += (dd[k] - dir[k] * dot) * inv_len;
#pragma unroll
        for (int c = 0; c < 3; ++c) dcol_in[c] = dcol_next[c];
      }
    }
    if (shared) {
      float dxf[D::SC];
      D::template col_bwd_features<ACC, NWV>(s_wb_col, x1f, dh_sum, dxf, Xs, Ys, accW, w, lane);
#pragma unroll
      for (int s = 0; s < Sh::FPL; ++s) dfr[s] += dxf[s];
    }
    if constexpr (!RAY) {
      // decoder-side results: feature gradients (canonical order) for the
      // grid adjoint, and the view-direction part of the position gradient
      if (valid) {
#pragma unroll
        for (int k = 0; k < Sh::L / 4; ++k) {
          const int lev = g + 4 * k;
          *reinterpret_cast<float2*>(a.dfeat_geo + (size_t)item * 2 * Sh::L + 2 * lev) = make_float2(dxg[2 * k], dxg[2 * k + 1]);
          *reinterpret_cast<float2*>(a.dfeat_rad + (size_t)item * 2 * Sh::L + 2 * lev) = make_float2(dfr[2 * k], dfr[2 * k + 1]);
        }
      }
      // dL/dx through the interpolation weights from the feature derivatives
      // the forward saved: dL/dx_d = sum_(l,f) dL/df (d f / d x_d)
      float dxv[3] = {0.f, 0.f, 0.f};
      if (a.jac && valid) {
#pragma unroll
        for (int k = 0; k < Sh::L / 4; ++k) {
          const float* Jg = jv[k];       // d(geometry features)/dx, 2 x 3
          const float* Jr = jv[k] + 6;   // d(radiance features)/dx, 2 x 3
#pragma unroll
          for (int d = 0; d < 3; ++d)
            dxv[d] += (dxg[2 * k] * Jg[d] + dxg[2 * k + 1] * Jg[3 + d]) +
                      (dfr[2 * k] * Jr[d] + dfr[2 * k + 1] * Jr[3 + d]);
        }
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        dp_dir[k] += __shfl_xor(dp_dir[k], 16, 64);
        dp_dir[k] += __shfl_xor(dp_dir[k], 32, 64);
        dxv[k] += __shfl_xor(dxv[k], 16, 64);
        dxv[k] += __shfl_xor(dxv[k], 32, 64);
      }
      if (valid && g == 0 && a.g_pos) {
        float dpw[3] = {0.f, 0.f, 0.f};
        if (a.jac) contract_vjp(a.grid, pxf, pyf, pzf, dxv, dpw);
        float cur[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) cur[k] = a.g_pos[(size_t)k * a.n + gi];
#pragma unroll
        for (int k = 0; k < 3; ++k) a.g_pos[(size_t)k * a.n + gi] = cur[k] + (dp_dir[k] + dpw[k]);
      }
    } else if (a.g_table_rad) {
      // background points: the round's feature gradients to LDS (the dW
      // staging is free once every wave has left the decoder adjoint), then
      // the radiance-table scatter of the round
      // layout in the staging space: the 8 waves' cell stages from its
      // start, the feature gradients ([pixel][BG_DF_STRIDE]) at its end
      constexpr int SDF_OFF = 2 * PPR * STAGE_W - PPR * BG_DF_STRIDE;
      static_assert(NWV == 8 && NWV * sizeof(BgCellStage) <= SDF_OFF * sizeof(float) && SDF_OFF % 4 == 0,
                    "background scatter layout");
      float* const sdf = XY + SDF_OFF;
      __syncthreads();
      const int pl = w * 16 + j;
#pragma unroll
      for (int k = 0; k < Sh::L / 4; ++k) {
        const int lev = g + 4 * k;
        *reinterpret_cast<float2*>(sdf + pl * BG_DF_STRIDE + 2 * lev) =
            valid ? make_float2(dfr[2 * k], dfr[2 * k + 1]) : make_float2(0.f, 0.f);
      }
      __syncthreads();
      // shared-corner merging (the default: 39% fewer atomic requests along
      // pixel rows); the choice is uniform over the launch
      const double* sx = reinterpret_cast<const double*>(s_wf_geo) + (round & 1) * PPR * 3;
      BgCellStage& st = reinterpret_cast<BgCellStage*>(XY)[w];
      if (a.merge)
        bg_round_scatter<Sh::L, true>(a, sdf, sx, st, w);
      else
        bg_round_scatter<Sh::L, false>(a, sdf, sx, st, w);
    }
  }
  write_dw<Sh, ACC, NWV, !RAY>(a.dw_part + (size_t)blockIdx.x * a.n_w, accW, w, lane);
}

// Hash-table adjoint of the surviving Gaussians when the decoder adjoint has
// already formed dL/dp from the saved feature derivatives: only the
// scatter-add of w_c * dL/df into both tables remains.  One lane per
// Gaussian, all levels per lane, one table at a time (fewer live registers,
// more waves per SIMD to cover the atomics' issue).
__global__ __launch_bounds__(256) void k_grid_scatter(GridBwdArgs a) {
  __shared__ CellStage stage[4];
  CellStage& st = stage[threadIdx.x / 64];
  const int item = blockIdx.x * 256 + threadIdx.x;
  const int count = *a.count;
  if (blockIdx.x * 256 >= count) return;          // whole workgroup idle (uniform)
  const bool valid = item < count;
  const int gi = valid ? a.vis_idx[item] : 0;
  double x[3];
  contract_f64(a.grid, (double)a.pos[gi], (double)a.pos[a.n + gi], (double)a.pos[2 * a.n + gi], x);
  const uint32_t Tg = a.grid.mask_geo + 1u, Tr = a.grid.mask_rad + 1u;
  const bool single = a.grid.single != 0;
  const bool do_geo = a.g_table_geo && !single;
  // every level's feature gradients are read before the first atomic: a
  // wave's memory counter completes in issue order, so a read issued after
  // a level's atomics would wait for all of them.  Two levels per float4;
  // the pairs shift down one register slot per step of the (rolled) loop
  // over level pairs, so that no register array is indexed at run time.
  float4 fgeo[GRID_MAX_LEVELS / 2], frad[GRID_MAX_LEVELS / 2];
  const int itc = valid ? item : 0;
#pragma unroll
  for (int k = 0; k < GRID_MAX_LEVELS / 2; ++k) {
    fgeo[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    frad[k] = fgeo[k];
    if (valid && 2 * k < a.grid.L) {
      fgeo[k] = *reinterpret_cast<const float4*>(a.dfeat_geo + (size_t)itc * 2 * a.grid.L + 4 * k);
      frad[k] = *reinterpret_cast<const float4*>(a.dfeat_rad + (size_t)itc * 2 * a.grid.L + 4 * k);
    }
  }
  for (int lp = 0; lp < a.grid.L; lp += 2) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int lev = lp + h;
      if (lev < a.grid.L) {
        const int res = a.grid.res[lev];
        int ci[3];
        float wv[3];
        grid_cell(x, res, ci, wv);
        const uint32_t side = (uint32_t)res + 1u;
        float2 dg = h ? make_float2(fgeo[0].z, fgeo[0].w) : make_float2(fgeo[0].x, fgeo[0].y);
        float2 dr = h ? make_float2(frad[0].z, frad[0].w) : make_float2(frad[0].x, frad[0].y);
        if (single) {
          // one field read by both decoders: its feature gradient is the sum
          dr.x += dg.x;
          dr.y += dg.y;
        }
        const uint64_t heads = cell_heads(ci);
        if (do_geo)
          scatter_level<false>(a.g_table_geo + (size_t)lev * Tg * 2, heads, ci, wv, dg, (a.grid.dense_geo >> lev) & 1u,
                               side, a.grid.mask_geo, st);
        if (a.g_table_rad)
          scatter_level<false>(a.g_table_rad + (size_t)lev * Tr * 2, heads, ci, wv, dr, (a.grid.dense_rad >> lev) & 1u,
                               side, a.grid.mask_rad, st);
      }
    }
#pragma unroll
    for (int k = 0; k + 1 < GRID_MAX_LEVELS / 2; ++k) {
      fgeo[k] = fgeo[k + 1];
      frad[k] = frad[k + 1];
    }
  }
}

// Hash-grid adjoint of the surviving Gaussians, one lane per Gaussian and all
// levels per lane: scatter-add of w_c * dL/df into both tables (cell runs of
// consecutive Gaussians summed first; they share cells at the coarse levels
// when the Gaussians are stored in spatial order) and
// dL/dx = sum_c (dL/df . table[c]) dw_c/dx, then the contraction Jacobian ->
// dL/dp.
template <class TT>
__global__ __launch_bounds__(256) void k_grid_bwd(GridBwdArgs a) {
  __shared__ CellStage stage[4];
  CellStage& st = stage[threadIdx.x / 64];
  const TT* table_geo = (const TT*)a.table_geo;
  const TT* table_rad = (const TT*)a.table_rad;
  const int item = blockIdx.x * 256 + threadIdx.x;
  const int count = *a.count;
  if (blockIdx.x * 256 >= count) return;          // whole workgroup idle (uniform)
  const bool valid = item < count;
  const int gi = valid ? a.vis_idx[item] : 0;
  float pxf = 0.f, pyf = 0.f, pzf = 0.f;
  if (valid) {
    pxf = a.pos[gi]; pyf = a.pos[a.n + gi]; pzf = a.pos[2 * a.n + gi];
  }
  const uint32_t Tg = a.grid.mask_geo + 1u, Tr = a.grid.mask_rad + 1u;
  const bool single = a.grid.single != 0;
  const bool do_geo = a.g_table_geo && !single;
  double x[3];
  contract_f64(a.grid, (double)pxf, (double)pyf, (double)pzf, x);
  float dxv[3] = {0.f, 0.f, 0.f};
  for (int lev = 0; lev < a.grid.L; ++lev) {
    const int res = a.grid.res[lev];
    int ci[3];
    float wv[3];
    grid_cell(x, res, ci, wv);
    const uint32_t side = (uint32_t)res + 1u;
    const bool dgn = (a.grid.dense_geo >> lev) & 1u;
    const bool drn = (a.grid.dense_rad >> lev) & 1u;
    float2 dg = make_float2(0.f, 0.f), dr = dg;
    if (valid) {
      dg = *reinterpret_cast<const float2*>(a.dfeat_geo + (size_t)item * 2 * a.grid.L + 2 * lev);
      dr = *reinterpret_cast<const float2*>(a.dfeat_rad + (size_t)item * 2 * a.grid.L + 2 * lev);
    }
    if (single) {
      // one field read by both decoders: its feature gradient is the sum
      dr.x += dg.x;
      dr.y += dg.y;
      dg = make_float2(0.f, 0.f);
    }
    const float fres = (float)res;
    uint32_t rg[8], rr[8];
    float2 vg[8], vr[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const uint32_t cx = (uint32_t)ci[0] + (c & 1), cy = (uint32_t)ci[1] + ((c >> 1) & 1),
                     cz = (uint32_t)ci[2] + ((c >> 2) & 1);
      rg[c] = corner_row(cx, cy, cz, dgn, side, a.grid.mask_geo);
      rr[c] = corner_row(cx, cy, cz, drn, side, a.grid.mask_rad);
      vg[c] = valid && !single ? load_entry(table_geo, (size_t)lev * Tg + rg[c]) : make_float2(0.f, 0.f);
      vr[c] = valid ? load_entry(table_rad, (size_t)lev * Tr + rr[c]) : make_float2(0.f, 0.f);
    }
    float sg[16], sr[16];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
      const float wx = bx ? wv[0] : 1.f - wv[0];
      const float wy = by ? wv[1] : 1.f - wv[1];
      const float wz = bz ? wv[2] : 1.f - wv[2];
      const float wc = (wx * wy) * wz;
      sg[2 * c] = wc * dg.x;
      sg[2 * c + 1] = wc * dg.y;
      sr[2 * c] = wc * dr.x;
      sr[2 * c + 1] = wc * dr.y;
      const float val = (dg.x * vg[c].x + dg.y * vg[c].y) + (dr.x * vr[c].x + dr.y * vr[c].y);
      dxv[0] += val * fres * (bx ? 1.f : -1.f) * (wy * wz);
      dxv[1] += val * fres * (by ? 1.f : -1.f) * (wx * wz);
      dxv[2] += val * fres * (bz ? 1.f : -1.f) * (wx * wy);
    }
    const uint64_t heads = cell_heads(ci);
    if (do_geo) {
      run_sums<16>(heads, sg);
      scatter_tails<false>(a.g_table_geo + (size_t)lev * Tg * 2, heads, ci, rg, sg, st);
    }
    if (a.g_table_rad) {
      run_sums<16>(heads, sr);
      scatter_tails<false>(a.g_table_rad + (size_t)lev * Tr * 2, heads, ci, rr, sr, st);
    }
  }
  if (valid && a.g_pos) {
    float dp[3];
    contract_vjp(a.grid, pxf, pyf, pzf, dxv, dp);
    float cur[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) cur[k] = a.g_pos[(size_t)k * a.n + gi];
#pragma unroll
    for (int k = 0; k < 3; ++k) a.g_pos[(size_t)k * a.n + gi] = cur[k] + dp[k];
  }
}

// dW partials [nparts][nw] -> grads: 64 weights x 4 part-slices per
// workgroup, slices combined in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_dw_reduce(const float* __restrict__ part, int nparts, int nw,
                                                   float* __restrict__ gg, float* __restrict__ gc, int n_geo) {
  __shared__ float sh[4][64];
  const int wi = blockIdx.x * 64 + (threadIdx.x & 63);
  const int sl = threadIdx.x >> 6;
  float s = 0.f;
  if (wi < nw)
    for (int b = sl; b < nparts; b += 4) s += part[(size_t)b * nw + wi];
  sh[sl][threadIdx.x & 63] = s;
  __syncthreads();
  if (sl == 0 && wi < nw) {
    const float t = (sh[0][threadIdx.x] + sh[1][threadIdx.x]) + (sh[2][threadIdx.x] + sh[3][threadIdx.x]);
    if (wi < n_geo) {
      if (gg) gg[wi] += t;
    } else if (gc) {
      gc[wi - n_geo] += t;
    }
  }
}

// ---------------------------------------------------------------- launchers
static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

template <class Sh, class TT, bool BF>
static void launch_bwd_t(const BwdLaunch& L, hipStream_t st) {
  FieldBwdArgs a = L.field;
  a.wf_geo = L.wf_geo; a.wf_col = L.wf_col; a.wb_geo = L.wb_geo; a.wb_col = L.wb_col;
  a.n_w = Sh::N_GEO + Sh::N_COL;
  if (L.stages & BWD_STAGE_WEIGHTS)
    k_prep_weights<Sh, BF><<<64, 256, 0, st>>>(L.w_geo, L.w_col, L.wf_geo, L.wf_col, L.wb_geo, L.wb_col);
  if (L.stages & BWD_STAGE_SPLATS) {
    // per-splat gradient records, then the projection adjoint
    k_zero_f32<<<nblk(L.n_gs), 256, 0, st>>>(L.comp.gs, L.n_gs);
    dim3 grid(L.comp.tiles_x, L.comp.tiles_y, L.V);
    k_composite_bwd<<<grid, 256, 0, st>>>(L.comp);
    k_project_bwd<<<nblk(L.proj.n > 0 ? L.proj.n : 1), 256, 0, st>>>(L.proj);
  }
  if (L.stages & BWD_STAGE_DECODERS)
    k_field_bwd<Sh, false, TT, BF><<<L.blocks_g, bwd_waves<false>() * 64, 0, st>>>(a);
  if ((L.stages & BWD_STAGE_BG_DECODERS) && L.with_bg) {
    FieldBwdArgs b = a;
    b.dw_part = a.dw_part + (size_t)L.blocks_g * a.n_w;
    if (b.bg_feat)
      k_field_bwd<Sh, true, TT, BF, true><<<L.blocks_r, bwd_waves<true>() * 64, 0, st>>>(b);
    else
      k_field_bwd<Sh, true, TT, BF, false><<<L.blocks_r, bwd_waves<true>() * 64, 0, st>>>(b);
  }
  if (L.stages & BWD_STAGE_DW) {
    const int parts = L.blocks_g + (L.with_bg ? L.blocks_r : 0);
    k_dw_reduce<<<(unsigned)((a.n_w + 63) / 64), 256, 0, st>>>(a.dw_part, parts, a.n_w, L.g_mlp_geo, L.g_mlp_col,
                                                               Sh::N_GEO);
  }
  if (L.stages & BWD_STAGE_TABLES) {
    GridBwdArgs gb{};
    gb.grid = a.grid;
    gb.n = a.n;
    gb.count = a.count;
    gb.vis_idx = a.vis_idx;
    gb.pos = a.pos;
    gb.table_geo = a.table_geo;
    gb.table_rad = a.table_rad;
    gb.dfeat_geo = a.dfeat_geo;
    gb.dfeat_rad = a.dfeat_rad;
    gb.g_pos = a.g_pos;
    gb.g_table_geo = a.g_table_geo;
    gb.g_table_rad = a.g_table_rad;
    const unsigned blocks = (unsigned)((a.n + 255) / 256 > 0 ? (a.n + 255) / 256 : 1);
    if (a.jac)
      k_grid_scatter<<<blocks, 256, 0, st>>>(gb);   // dL/dp already formed by the decoder adjoint
    else
      k_grid_bwd<TT><<<blocks, 256, 0, st>>>(gb);
  }
  // BWD_STAGE_BG_TABLES: the background decoder adjoint scatters its table
  // gradients itself; the stage launches nothing.
}

void launch_backward(int Lv, int hid, int nh, const BwdLaunch& L, hipStream_t st) {
  if (Lv == 16 && hid == 64 && nh == 2) {
    using Sh = Shape<16, 64, 2>;
    if (!L.f16 && !L.bf) return launch_bwd_t<Sh, float, false>(L, st);
    if (!L.f16 && L.bf) return launch_bwd_t<Sh, float, true>(L, st);
    if (L.f16 && !L.bf) return launch_bwd_t<Sh, _Float16, false>(L, st);
    return launch_bwd_t<Sh, _Float16, true>(L, st);
  }
  if (L.f16 || L.bf) return;
#define X(l, h, k) if (Lv == l && hid == h && nh == k) return launch_bwd_t<Shape<l, h, k>, float, false>(L, st);
  X(8, 32, 1) X(16, 64, 1) X(8, 64, 2)
#undef X
}

size_t bwd_weight_floats(int Lv, int hid, int nh, size_t* fwd_geo, size_t* fwd_col, size_t* bwd_geo,
                         size_t* bwd_col, size_t* n_w) {
#define X(l, h, k)                                                          \
  if (Lv == l && hid == h && nh == k) {                                     \
    using Sh = Shape<l, h, k>;                                              \
    *fwd_geo = Sh::W_GEO; *fwd_col = Sh::W_COL;                             \
    *bwd_geo = BwdShape<Sh>::WB_GEO; *bwd_col = BwdShape<Sh>::WB_COL;       \
    *n_w = Sh::N_GEO + Sh::N_COL;                                           \
    return *fwd_geo + *fwd_col + *bwd_geo + *bwd_col;                       \
  }
  X(16, 64, 2) X(8, 32, 1) X(16, 64, 1) X(8, 64, 2)
#undef X
  return 0;
}

}  // namespace hyrf
