// Pre-cull + compaction, field query of the survivors, and the background
// query of pixel rays (Sec. 3.2 Eqs. 2-7, Sec. 3.3).
#include "block.h"
#include "field.h"
#include "kernels.h"
#include "query.h"

#include <type_traits>

namespace hyrf {

// ---------------------------------------------------------------- pre-cull
__global__ __launch_bounds__(256) void k_cull_flags(const void* __restrict__ pos, bool pos_f16, int n, Cams cams,
                                                    uint32_t* __restrict__ flag) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double px = load_pos(pos, pos_f16, i), py = load_pos(pos, pos_f16, (size_t)n + i),
               pz = load_pos(pos, pos_f16, 2 * (size_t)n + i);
  bool keep = false;
  for (int v = 0; v < cams.V; ++v) {
    double t[3];
    cam_space_f64(cams.c[v], px, py, pz, t);
    keep |= precull_f64(cams.c[v], t);
  }
  flag[i] = keep ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_cull_write(const uint32_t* __restrict__ flag,
                                                    const uint32_t* __restrict__ pos_, int n,
                                                    int32_t* __restrict__ vis_idx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) vis_idx[pos_[i]] = i;
}

// ---------------------------------------------------------------- field query
// Weight storage of one MLP in LDS: permuted FP32 A operands, or BF16.
template <class Sh, bool BF>
struct MlpLds {
  using T = typename std::conditional<BF, __bf16, float>::type;
  static constexpr int GEO = BF ? Sh::WB16_GEO : Sh::W_GEO;
  static constexpr int COL = BF ? Sh::WB16_COL : Sh::W_COL;
  static constexpr int SG = BF ? Sh::S_GEO1_8 : Sh::S_GEO1;   // first-layer k-steps (lane inputs)
  static constexpr int SC = BF ? Sh::S_COL1_8 : Sh::S_COL1;
  static __device__ void load(T* dst, const float* W, bool colour) {
    if constexpr (BF) permute_mlp_fwd_bf16<Sh>(dst, W, colour, threadIdx.x, blockDim.x);
    else permute_mlp_fwd<Sh>(dst, W, colour, threadIdx.x, blockDim.x);
  }
  template <int S1>
  static __device__ void run(const T* W, const float (&x)[S1], v4f& out, int lane) {
    if constexpr (BF) mlp_forward_bf16<Sh, S1>(W, x, out, lane);
    else mlp_forward<Sh, S1>(W, x, out, lane);
  }
  // colour decoder: the view-independent first-layer part (radiance
  // features, k-steps [0, FPL)) once, then per view the direction part and
  // the remaining layers
  static_assert(Sh::FPL % (BF ? 8 : 4) == 0, "feature k-steps must fill whole MFMA k-groups");
  static __device__ void col_first(const T* W, const float (&x)[SC], v4f (&acc)[Sh::NT], int lane) {
    if constexpr (BF) mlp_first_part_bf16<Sh, SC, Sh::FPL>(W, x, acc, lane);
    else mlp_first_part<Sh, SC, Sh::FPL>(W, x, acc, lane);
  }
  static __device__ void col_rest(const T* W, const float (&x)[SC], v4f (&acc)[Sh::NT], v4f& out, int lane) {
    if constexpr (BF) mlp_forward_rest_bf16<Sh, SC, Sh::FPL>(W, x, acc, out, lane);
    else mlp_forward_rest<Sh, SC, Sh::FPL>(W, x, acc, out, lane);
  }
};

template <class Sh, class TT, bool BF>
__global__ __launch_bounds__(QUERY_NT, 2) void k_field_query(QueryArgs a) {
  using M = MlpLds<Sh, BF>;
  __shared__ __attribute__((aligned(16))) typename M::T w_geo[M::GEO];
  __shared__ __attribute__((aligned(16))) typename M::T w_col[M::COL];
  M::load(w_geo, a.w_geo, false);
  M::load(w_col, a.w_col, true);
  __syncthreads();
  const TT* table_geo = reinterpret_cast<const TT*>(a.table_geo);
  const TT* table_rad = reinterpret_cast<const TT*>(a.table_rad);

  const int lane = lane_id();
  const int j = lane & 15, g = lane >> 4;
  const int count = *a.count;
  const int groups = (count + 15) >> 4;
  const int wave_g = blockIdx.x * (QUERY_NT / 64) + threadIdx.x / 64;
  const int wave_n = gridDim.x * (QUERY_NT / 64);
  const int n = a.n;

  for (int grp = wave_g; grp < groups; grp += wave_n) {
    const int slot = grp * 16 + j;
    const bool valid = slot < count;
    const int gi = valid ? a.vis_idx[slot] : a.vis_idx[0];
    const float pxf = load_pos(a.pos, a.pos_f16, gi), pyf = load_pos(a.pos, a.pos_f16, (size_t)n + gi),
                pzf = load_pos(a.pos, a.pos_f16, 2 * (size_t)n + gi);
    double x[3];
    contract_f64(a.grid, (double)pxf, (double)pyf, (double)pzf, x);
    float fg[Sh::FPL], fr[Sh::FPL];
    uint32_t* dg = nullptr;
    uint32_t* dr = nullptr;
    if (a.dbg && valid) {
      dg = a.dbg + (size_t)slot * 2 * Sh::L * 8;
      dr = dg + Sh::L * 8;
    }
    float* jac = a.jac && valid ? a.jac + (size_t)slot * Sh::L * 12 : nullptr;
    if (a.grid.single) {
      // one field feeds both decoders: gather it once
      gather_lane<Sh::L, false, TT>(a.grid, x, g, nullptr, table_rad, fg, fr, nullptr, dr, jac);
#pragma unroll
      for (int s = 0; s < Sh::FPL; ++s) fg[s] = fr[s];
      if (dg) {
#pragma unroll
        for (int k = 0; k < Sh::L / 4; ++k)
#pragma unroll
          for (int c = 0; c < 8; ++c) dg[(g + 4 * k) * 8 + c] = dr[(g + 4 * k) * 8 + c];
      }
    } else {
      gather_lane<Sh::L, true, TT>(a.grid, x, g, table_geo, table_rad, fg, fr, dg, dr, jac);
    }
    if (a.feat_geo && valid) {
#pragma unroll
      for (int k = 0; k < Sh::L / 4; ++k) {
        const int lev = g + 4 * k;
        *reinterpret_cast<float2*>(a.feat_geo + (size_t)slot * 2 * Sh::L + 2 * lev) = make_float2(fg[2 * k], fg[2 * k + 1]);
        *reinterpret_cast<float2*>(a.feat_rad + (size_t)slot * 2 * Sh::L + 2 * lev) = make_float2(fr[2 * k], fr[2 * k + 1]);
      }
    }
    // geometry decoder
    float xg[M::SG];
#pragma unroll
    for (int s = 0; s < M::SG; ++s) xg[s] = s < Sh::FPL ? fg[s] : 0.f;
    v4f og;
    M::template run<M::SG>(w_geo, xg, og, lane);
    // rows 4..7 (rotation) live in lane group 1: bring them to group 0
    float rn[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) rn[r] = __shfl(og[r], j + 16, 64);
    if (g == 0 && valid) {
      const float op = sigmoidf_(og[0] + a.opac_e[gi]);
      a.opacity[slot] = op;
#pragma unroll
      for (int d = 0; d < 3; ++d) a.scale[(size_t)d * n + slot] = sigmoidf_(og[1 + d] + a.scale_e[(size_t)d * n + gi]);
      float q[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) q[r] = rn[r] + (a.rot_e ? a.rot_e[(size_t)r * n + gi] : 0.f);
      const float inv = 1.0f / sqrtf((q[0] * q[0] + q[1] * q[1]) + (q[2] * q[2] + q[3] * q[3]));
#pragma unroll
      for (int r = 0; r < 4; ++r) a.quat[(size_t)r * n + slot] = q[r] * inv;
    }
    // colour decoder (Eq. 6): the first layer's product with the radiance
    // features once, then per view the direction encoding and the rest
    v4f col1[Sh::NT];
    {
      float xf[M::SC];
#pragma unroll
      for (int s = 0; s < M::SC; ++s) xf[s] = s < Sh::FPL ? fr[s] : 0.f;
      M::col_first(w_col, xf, col1, lane);
    }
    for (int v = 0; v < a.cams.V; ++v) {
      float oc[3];
      cam_center_f32(a.cams.c[v], oc);
      float dx = pxf - oc[0], dy = pyf - oc[1], dz = pzf - oc[2];
      const float inv = 1.0f / sqrtf((dx * dx + dy * dy) + dz * dz);
      dx *= inv; dy *= inv; dz *= inv;
      float pe[6];
      pe_lane(g, dx, dy, dz, pe);
      float xc[M::SC];
#pragma unroll
      for (int s = 0; s < M::SC; ++s)
        xc[s] = s < Sh::FPL ? 0.f : (s < Sh::FPL + 6 ? pe[s < Sh::FPL + 6 ? (s - Sh::FPL) : 0] : 0.f);
      v4f acc[Sh::NT];
#pragma unroll
      for (int t = 0; t < Sh::NT; ++t) acc[t] = col1[t];
      v4f oc4;
      M::col_rest(w_col, xc, acc, oc4, lane);
      if (g == 0 && valid) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
          a.rgb[((size_t)v * 3 + c) * n + slot] = sigmoidf_(oc4[c] + a.col_e[(size_t)c * n + gi]);
      }
    }
  }
}

// ---------------------------------------------------------------- background
// Background query: 4 waves per workgroup, 3 workgroups per CU (at most 168
// registers per lane, 3 waves per SIMD).
constexpr int BG_NT = 256;
constexpr int BG_WAVES_PER_SIMD = 3;
constexpr int BG_MAX_BLOCKS = 768;

template <class Sh, class TT, bool BF>
__global__ __launch_bounds__(BG_NT, BG_WAVES_PER_SIMD) void k_bg_query(BgArgs a) {
  using M = MlpLds<Sh, BF>;
  __shared__ __attribute__((aligned(16))) typename M::T w_col[M::COL];
  M::load(w_col, a.w_col, true);
  __syncthreads();
  const TT* table_rad = reinterpret_cast<const TT*>(a.table_rad);
  const int lane = lane_id();
  const int j = lane & 15, g = lane >> 4;
  const int HW = a.W * a.H;
  const int count = a.list_count ? *a.list_count : a.cams.V * HW;
  const int groups = (count + 15) >> 4;
  const int wave_g = blockIdx.x * (BG_NT / 64) + threadIdx.x / 64;
  const int wave_n = gridDim.x * (BG_NT / 64);
  const double radius = (double)a.grid.bg_radius;
  for (int grp = wave_g; grp < groups; grp += wave_n) {
    const int item = grp * 16 + j;
    const bool valid = item < count;
    const int pix = valid ? (a.list ? (int)a.list[item] : item) : 0;
    const int v = pix / HW;
    const int rem = pix - v * HW;
    const int y = rem / a.W, xq = rem - y * a.W;
    double ps[3], d[3];
    sphere_point_f64(a.cams.c[v], xq, y, radius, ps, d);
    double x[3];
    contract_f64(a.grid, ps[0], ps[1], ps[2], x);
    float fg[Sh::FPL], fr[Sh::FPL];
    gather_lane<Sh::L, false, TT>(a.grid, x, g, nullptr, table_rad, fg, fr, nullptr, nullptr);
    const double dn = sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
    float pe[6];
    pe_lane(g, (float)(d[0] / dn), (float)(d[1] / dn), (float)(d[2] / dn), pe);
    float xc[M::SC];
#pragma unroll
    for (int s = 0; s < M::SC; ++s)
      xc[s] = s < Sh::FPL ? fr[s] : (s < Sh::FPL + 6 ? pe[s < Sh::FPL + 6 ? (s - Sh::FPL) : 0] : 0.f);
    v4f o;
    M::template run<M::SC>(w_col, xc, o, lane);
    if (a.feat_save && valid) {
#pragma unroll
      for (int k = 0; k < Sh::L / 4; ++k)
        *reinterpret_cast<float2*>(a.feat_save + (size_t)pix * 2 * Sh::L + 2 * (g + 4 * k)) =
            make_float2(fr[2 * k], fr[2 * k + 1]);
    }
    if (g == 0 && valid) {
      const float T = a.out_rgb ? a.T[pix] : 0.f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float cs = sigmoidf_(o[c]);
        const size_t at = ((size_t)v * 3 + c) * HW + rem;
        if (a.out_rgb) a.out_rgb[at] = fmaf(T, cs, a.out_rgb[at]);
        if (a.bg_save) a.bg_save[at] = cs;
      }
    }
  }
}

// ---------------------------------------------------------------- launchers
template <class Sh, class TT, bool BF>
static void launch_query_t(const QueryArgs& a, int n_cap, hipStream_t st) {
  int groups = (n_cap + 15) / 16;
  int blocks = (groups + QUERY_NT / 64 - 1) / (QUERY_NT / 64);
  if (blocks > QUERY_MAX_BLOCKS) blocks = QUERY_MAX_BLOCKS;
  if (blocks < 1) blocks = 1;
  k_field_query<Sh, TT, BF><<<blocks, QUERY_NT, 0, st>>>(a);
}

template <class Sh, class TT, bool BF>
static void launch_bg_t(const BgArgs& a, int n_cap, hipStream_t st) {
  int groups = (n_cap + 15) / 16;
  int blocks = (groups + BG_NT / 64 - 1) / (BG_NT / 64);
  if (blocks > BG_MAX_BLOCKS) blocks = BG_MAX_BLOCKS;
  if (blocks < 1) blocks = 1;
  k_bg_query<Sh, TT, BF><<<blocks, BG_NT, 0, st>>>(a);
}

bool shape_supported(int L, int hid, int nh) {
  return (L == 16 && hid == 64 && nh == 2) || (L == 8 && hid == 32 && nh == 1) ||
         (L == 16 && hid == 64 && nh == 1) || (L == 8 && hid == 64 && nh == 2);
}

#define HYRF_SHAPES(X) X(16, 64, 2) X(8, 32, 1) X(16, 64, 1) X(8, 64, 2)

// tdt: table dtype (HYRF_F32, HYRF_F16, HYRF_U8); bf: bfloat16 decoders.
#define HYRF_DISPATCH(FN, ...)                                                                  \
  do {                                                                                          \
    if (L == 16 && hid == 64 && nh == 2) {                                                      \
      using Sh = Shape<16, 64, 2>;                                                              \
      if (tdt == HYRF_F32) return bf ? FN<Sh, float, true>(__VA_ARGS__) : FN<Sh, float, false>(__VA_ARGS__); \
      if (tdt == HYRF_F16)                                                                      \
        return bf ? FN<Sh, _Float16, true>(__VA_ARGS__) : FN<Sh, _Float16, false>(__VA_ARGS__); \
      if (tdt == HYRF_U8) return bf ? FN<Sh, uint8_t, true>(__VA_ARGS__) : FN<Sh, uint8_t, false>(__VA_ARGS__); \
      return;                                                                                   \
    }                                                                                           \
    if (bf || (tdt != HYRF_F32 && tdt != HYRF_U8)) return;                                      \
    if (L == 8 && hid == 32 && nh == 1)                                                         \
      return tdt == HYRF_U8 ? FN<Shape<8, 32, 1>, uint8_t, false>(__VA_ARGS__)                  \
                            : FN<Shape<8, 32, 1>, float, false>(__VA_ARGS__);                   \
    if (L == 16 && hid == 64 && nh == 1)                                                        \
      return tdt == HYRF_U8 ? FN<Shape<16, 64, 1>, uint8_t, false>(__VA_ARGS__)                 \
                            : FN<Shape<16, 64, 1>, float, false>(__VA_ARGS__);                  \
    if (L == 8 && hid == 64 && nh == 2)                                                         \
      return tdt == HYRF_U8 ? FN<Shape<8, 64, 2>, uint8_t, false>(__VA_ARGS__)                  \
                            : FN<Shape<8, 64, 2>, float, false>(__VA_ARGS__);                   \
  } while (0)

void launch_query(int L, int hid, int nh, int tdt, bool bf, const QueryArgs& a, int n_cap, hipStream_t st) {
  HYRF_DISPATCH(launch_query_t, a, n_cap, st);
}

void launch_bg(int L, int hid, int nh, int tdt, bool bf, const BgArgs& a, int n_cap, hipStream_t st) {
  HYRF_DISPATCH(launch_bg_t, a, n_cap, st);
}

bool precision_supported(int L, int hid, int nh, int tdt, bool bf) {
  if ((tdt == HYRF_F32 || tdt == HYRF_U8) && !bf) return shape_supported(L, hid, nh);
  return L == 16 && hid == 64 && nh == 2;
}

__global__ __launch_bounds__(256) void k_blend_bg(const float* __restrict__ bg, const float* __restrict__ T,
                                                  float* __restrict__ rgb, int HW, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;   // over V * 3 * HW
  if (i >= n) return;
  const int64_t v = i / (3 * (int64_t)HW);
  const int64_t p = i - (i / HW) * HW;
  rgb[i] = fmaf(T[v * HW + p], bg[i], rgb[i]);
}

void launch_blend_bg(const float* bg, const float* T, float* rgb, int V, int HW, hipStream_t st) {
  const int64_t n = (int64_t)V * 3 * HW;
  k_blend_bg<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(bg, T, rgb, HW, n);
}

void launch_cull(const void* pos, bool pos_f16, int n, const Cams& cams, uint32_t* flag, uint32_t* pos_,
                 uint32_t* scan_temp, int32_t* vis_idx, int32_t* vis_count, hipStream_t st) {
  if (n <= 0) {
    scan_exclusive_u32(nullptr, nullptr, 0, scan_temp, (uint32_t*)vis_count, st);
    return;
  }
  const int nb = (n + 255) / 256;
  k_cull_flags<<<nb, 256, 0, st>>>(pos, pos_f16, n, cams, flag);
  scan_exclusive_u32(flag, pos_, n, scan_temp, (uint32_t*)vis_count, st);
  k_cull_write<<<nb, 256, 0, st>>>(flag, pos_, n, vis_idx);
}

}  // namespace hyrf
