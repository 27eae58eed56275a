// Kernel argument blocks and launchers of the field query / background query.
#pragma once
#include "internal.h"

namespace hyrf {

constexpr int QUERY_NT = 512;          // 8 waves per workgroup
constexpr int QUERY_MAX_BLOCKS = 512;  // 2 workgroups per CU on 256 CUs (persistent)

struct QueryArgs {
  GridP grid;
  Cams cams;
  const void* table_geo;       // float32 or float16 pairs
  const void* table_rad;
  const float* w_geo;
  const float* w_col;
  int n;                      // Gaussian count (stride of the planar arrays)
  const int32_t* count;       // survivors
  const int32_t* vis_idx;
  const void* pos;
  bool pos_f16;
  const float* scale_e;
  const float* rot_e;
  const float* opac_e;
  const float* col_e;
  float* opacity;
  float* scale;
  float* quat;
  float* rgb;
  float* feat_geo;
  float* feat_rad;
  uint32_t* dbg;
  float* jac;                 // [n][L][12] feature derivatives d f / d x, or NULL
};

struct BgArgs {
  GridP grid;
  Cams cams;
  const void* table_rad;
  const float* w_col;
  int W, H;
  const uint32_t* list;        // pixel ids v*H*W + y*W + x, or NULL = every pixel
  const uint32_t* list_count;  // device count of `list`, or NULL
  const float* T;              // [V][H][W] final transmittance (with out_rgb)
  float* out_rgb;              // [V][3][H][W]: C_fg in, C_fg + T c_s out; or NULL (c_s only)
  float* bg_save;              // [V][3][H][W] c_s, or NULL
  float* feat_save;            // [V*H*W][2L] radiance features of the sphere points, or NULL
};

bool shape_supported(int L, int hid, int nh);
// f16: tables in float16; bf: decoder operands in bfloat16 (FP32 accumulate).
bool precision_supported(int L, int hid, int nh, int tdt, bool bf);
void launch_query(int L, int hid, int nh, int tdt, bool bf, const QueryArgs& a, int n_cap, hipStream_t st);
void launch_bg(int L, int hid, int nh, int tdt, bool bf, const BgArgs& a, int n_cap, hipStream_t st);
// rgb[v][c][p] += T[v][p] * bg[v][c][p]
void launch_blend_bg(const float* bg, const float* T, float* rgb, int V, int HW, hipStream_t st);
void launch_cull(const void* pos, bool pos_f16, int n, const Cams& cams, uint32_t* flag, uint32_t* pos_,
                 uint32_t* scan_temp, int32_t* vis_idx, int32_t* vis_count, hipStream_t st);

}  // namespace hyrf
