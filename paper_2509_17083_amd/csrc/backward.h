#pragma once
#include "internal.h"

namespace hyrf {

// ---- loss.hip
size_t l1_ws_elems(int64_t n);
void launch_l1(const float* img, const float* target, int64_t n, float* loss, float* grad, float* ws,
               hipStream_t st);

// ---- ssim.hip
size_t l1_dssim_ws_elems(int planes, int H, int W);
void launch_l1_dssim(const float* img, const float* target, int planes, int H, int W, float lambda,
                     float* loss, float* grad, float* ws, hipStream_t st);

// ---- backward.hip
struct CompBwdArgs {
  int W, H, tiles_x, tiles_y;
  const float* rec;
  uint32_t n_rec;
  const uint32_t* vals;
  const uint32_t* ranges;
  const float* T_final;
  const int32_t* last;
  const float* bg;       // [V][3][H][W] background colours, or NULL
  const float* dL;       // [V][3][H][W]
  float* gs;             // [V*n_max][9]
};

struct ProjBwdArgs {
  Cams cams;
  int n, n_max;
  const int32_t* count;
  const int32_t* vis_idx;
  const float* pos;
  const float* opacity;
  const float* scale;
  const float* quat;
  const float* rgb;
  const int32_t* rect;
  const float* gs;
  float* g_pos;
  float* g_scale_e;
  float* g_opac_e;
  float* g_col_e;
  float* dgeo;           // [n][8] to the decoder adjoint
  float* dcol;           // [V][3][n_max]: planar, so that the stores coalesce
  float* dens_accum;     // [n] densification statistics, nullable
  float* dens_count;
};

struct FieldBwdArgs {
  GridP grid;
  Cams cams;
  const void* table_geo;       // float32 or float16 pairs
  const void* table_rad;
  const void* wf_geo;          // permuted decoder weights (float32 or bfloat16)
  const void* wf_col;
  const void* wb_geo;
  const void* wb_col;
  int n;
  const int32_t* count;
  const int32_t* vis_idx;
  const float* pos;
  const float* rot_e;
  const float* feat_geo;
  const float* feat_rad;
  const float* dgeo;
  const float* dcol;     // [V][3][n_max]
  int n_max;
  float* dfeat_geo;      // [n][2L] feature gradients handed to the grid adjoint
  float* dfeat_rad;
  float* g_pos;
  float* g_rot_e;
  float* g_table_geo;
  float* g_table_rad;
  float* dw_part;
  int n_w;
  int W, H;
  const float* T_final;
  const float* dL;
  const float* bg_feat;  // [V*H*W][2L] saved background features, or NULL (gather)
  const float* jac;      // [n][L][12] saved feature derivatives, or NULL
  int merge;             // background scatter: merge corners shared by consecutive cells
};

struct GridBwdArgs {
  GridP grid;
  int n;
  const int32_t* count;
  const int32_t* vis_idx;
  const float* pos;
  const void* table_geo;
  const void* table_rad;
  const float* dfeat_geo;
  const float* dfeat_rad;
  float* g_pos;
  float* g_table_geo;
  float* g_table_rad;
};

// Stages of the adjoint.  WEIGHTS first; then two independent branches --
// Gaussians (SPLATS, DECODERS, TABLES) and background points (BG_DECODERS;
// BG_TABLES launches nothing since the background decoder adjoint scatters
// its table gradients itself) -- which may run concurrently on two streams;
// DW after both decoder stages.
enum : int {
  BWD_STAGE_WEIGHTS = 1,       // decoder weights permuted into the MFMA operand order
  BWD_STAGE_SPLATS = 2,        // blending + projection adjoints
  BWD_STAGE_DECODERS = 4,      // decoder adjoints of the Gaussians -> dW partials, feature grads
  BWD_STAGE_TABLES = 8,        // Gaussians' hash-table adjoint -> table grads
  BWD_STAGE_BG_DECODERS = 16,  // colour-decoder + radiance-table adjoint of the background points
  BWD_STAGE_BG_TABLES = 32,    // empty (kept so that stage numbers stay stable)
  BWD_STAGE_DW = 64,           // dW partials -> decoder weight gradients
  BWD_STAGE_ALL = 127
};

struct BwdLaunch {
  int stages;
  int V;
  CompBwdArgs comp;
  int64_t n_gs;
  ProjBwdArgs proj;
  FieldBwdArgs field;
  const float* w_geo;
  const float* w_col;
  float* wf_geo;
  float* wf_col;
  float* wb_geo;
  float* wb_col;
  int blocks_g, blocks_r;
  bool with_bg;
  bool f16, bf;          // float16 tables / bfloat16 decoder operands
  float* g_mlp_geo;
  float* g_mlp_col;
};

void launch_backward(int L, int hid, int nh, const BwdLaunch& a, hipStream_t st);
size_t bwd_weight_floats(int L, int hid, int nh, size_t* fwd_geo, size_t* fwd_col, size_t* bwd_geo,
                         size_t* bwd_col, size_t* n_w);

}  // namespace hyrf
