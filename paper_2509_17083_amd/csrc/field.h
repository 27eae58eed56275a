// Field query building blocks shared by the forward and backward kernels:
// hash-grid gather for a lane's share of the levels and the tiny MLPs on
// MFMA (v_mfma_f32_16x16x4_f32).
//
// Work unit: one wave evaluates 16 points.  Lane l serves point j = l & 15
// and lane group g = l >> 4 (0..3).  Group g gathers the levels g, g+4, g+8,
// g+12, so a point's 2L features are spread over its 4 lanes (L/2 each).
//
// The MLPs run transposed, D[out x points] = W[out x in] * X^T[in x points]:
// the B operand of v_mfma_f32_16x16x4_f32 at lane l is element
// (k = l>>4, column = l&15), so each lane feeds one of ITS OWN inputs per
// k-step, and the accumulator lands as (row = 4(l>>4)+r, column = l&15) --
// again in the lane that owns the point.  A layer's output therefore feeds
// the next layer's B operand straight from registers; the weights (A
// operand) are stored pre-permuted in LDS in the matching k order:
//   input from features:  k-step s of group g = feature 2(g + 4(s>>1)) + (s&1)
//   input from PE:        k-step L/2 + m of group g = PE value 6g + m
//   input from a hidden layer: k-step s = 4b + r of group g = unit 16b + 4g + r.
#pragma once
#include <type_traits>
#include "internal.h"

namespace hyrf {

constexpr int pad4(int x) { return (x + 3) & ~3; }
constexpr int pad8(int x) { return (x + 7) & ~7; }

template <int L_, int HID_, int NH_>
struct Shape {
  static constexpr int L = L_, HID = HID_, NH = NH_;
  static constexpr int NT = HID / 16;          // 16-row output tiles of a hidden layer
  static constexpr int LPG = L / 4;            // levels per lane group
  static constexpr int FPL = L / 2;            // features per lane (per field)
  static constexpr int S_GEO1 = pad4(L / 2);
  static constexpr int S_COL1 = pad4(L / 2 + 6);
  static constexpr int S_HID = HID / 4;
  // bf16 path: 8 lane inputs per k-step
  static constexpr int S_GEO1_8 = pad8(L / 2);
  static constexpr int S_COL1_8 = pad8(L / 2 + 6);
  static constexpr int WB16_GEO = NT * S_GEO1_8 * 64 + (NH - 1) * NT * S_HID * 64 + S_HID * 64;
  static constexpr int WB16_COL = NT * S_COL1_8 * 64 + (NH - 1) * NT * S_HID * 64 + S_HID * 64;
  static constexpr int IN_GEO = 2 * L;
  static constexpr int IN_COL = 2 * L + 6 * HYRF_PE_OCTAVES;
  // LDS floats per MLP
  static constexpr int W_GEO = NT * S_GEO1 * 64 + (NH - 1) * NT * S_HID * 64 + S_HID * 64;
  static constexpr int W_COL = NT * S_COL1 * 64 + (NH - 1) * NT * S_HID * 64 + S_HID * 64;
  // flat float32 weight counts
  static constexpr int N_GEO = HID * IN_GEO + (NH - 1) * HID * HID + HYRF_GEO_OUT * HID;
  static constexpr int N_COL = HID * IN_COL + (NH - 1) * HID * HID + HYRF_COL_OUT * HID;
};

// k index (input column) fed by lane group g at k-step s of a first layer.
template <int L>
__device__ __forceinline__ int first_layer_col(int s, int g, bool colour) {
  if (s < L / 2) return 2 * (g + 4 * (s >> 1)) + (s & 1);
  if (colour && s < L / 2 + 6) return 2 * L + 6 * g + (s - L / 2);
  return -1;
}

// Forward A-operand permutation of one MLP's weights.  Layout per layer:
// [out_tile][s/4][lane][s%4]; element e of the whole MLP is written by the
// caller's thread that owns it (tid, stride), so the same routine fills LDS
// (per workgroup) or a global buffer (whole grid).
template <class Sh>
__device__ void permute_mlp_fwd(float* dst, const float* __restrict__ W, bool colour, int tid, int stride) {
  const int n_out = colour ? HYRF_COL_OUT : HYRF_GEO_OUT;
  const int in1 = colour ? Sh::IN_COL : Sh::IN_GEO;
  const int S1 = colour ? Sh::S_COL1 : Sh::S_GEO1;
  int dst_off = 0, g_off = 0;
  for (int layer = 0; layer <= Sh::NH; ++layer) {
    const bool first = layer == 0;
    const bool last = layer == Sh::NH;
    const int S = first ? S1 : Sh::S_HID;
    const int NTo = last ? 1 : Sh::NT;
    const int rows = last ? n_out : Sh::HID;
    const int in = first ? in1 : Sh::HID;
    const int cnt = NTo * S * 64;
    for (int e = tid; e < cnt; e += stride) {
      const int s4 = e & 3;
      const int lane = (e >> 2) & 63;
      const int rest = e >> 8;                 // ot * (S/4) + sq
      const int sq = rest % (S / 4);
      const int ot = rest / (S / 4);
      const int s = sq * 4 + s4;
      const int g = lane >> 4;
      const int row = ot * 16 + (lane & 15);
      const int col = first ? first_layer_col<Sh::L>(s, g, colour) : (16 * sq + 4 * g + s4);
      float val = 0.f;
      if (row < rows && col >= 0 && col < in) val = W[g_off + row * in + col];
      dst[dst_off + e] = val;
    }
    dst_off += cnt;
    g_off += rows * in;
  }
}

template <class Sh>
__device__ void load_mlp_lds(float* lds, const float* __restrict__ W, bool colour) {
  permute_mlp_fwd<Sh>(lds, W, colour, threadIdx.x, blockDim.x);
}

// Output tiles [OT0, OT1) of one layer of S k-steps, accumulated over its
// k-steps [K0, K1): acc[ot - OT0] += sum_s W(ot, s) * x[s]  (x: this lane's
// B operands).  Per accumulator the MFMA sequence is that of the whole
// layer restricted to the range, so splitting a layer's k-steps into
// consecutive ranges gives the same bits as one pass.
template <int OT0, int OT1, int S, int K0, int K1>
__device__ __forceinline__ void mfma_accum(const float* __restrict__ Wl, const float (&x)[S],
                                           v4f (&acc)[OT1 - OT0], int lane) {
  static_assert(K0 % 4 == 0 && K1 % 4 == 0 && 0 <= K0 && K0 <= K1 && K1 <= S, "k-step range");
  constexpr int NO = OT1 - OT0;
  // the next k-quad's weights are read while the current quad's MFMAs run
  float4 w[2][NO];
  if constexpr (K0 < K1) {
#pragma unroll
    for (int ot = OT0; ot < OT1; ++ot)
      w[0][ot - OT0] = *reinterpret_cast<const float4*>(Wl + ((ot * (S / 4) + K0 / 4) * 64 + lane) * 4);
  }
#pragma unroll
  for (int sq = K0 / 4; sq < K1 / 4; ++sq) {
    const int cur = (sq - K0 / 4) & 1;
    if (sq + 1 < K1 / 4) {
#pragma unroll
      for (int ot = OT0; ot < OT1; ++ot)
        w[cur ^ 1][ot - OT0] = *reinterpret_cast<const float4*>(Wl + ((ot * (S / 4) + sq + 1) * 64 + lane) * 4);
    }
    // the reads above issue before this k-quad's MFMAs (a scheduling
    // barrier: the scheduler would otherwise sink them below), and no later
    // read moves above them, so at most two k-quads of weights are in
    // flight (register budget)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int ot = OT0; ot < OT1; ++ot) {
      const float4 wv = w[cur][ot - OT0];
      v4f& c = acc[ot - OT0];
      c = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.x, x[4 * sq + 0], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.y, x[4 * sq + 1], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.z, x[4 * sq + 2], c, 0, 0, 0);
      c = __builtin_amdgcn_mfma_f32_16x16x4f32(wv.w, x[4 * sq + 3], c, 0, 0, 0);
    }
  }
}

// One layer: acc[ot] = sum_s W(ot, s) * x[s].
template <int NTO, int S>
__device__ __forceinline__ void mfma_layer(const float* __restrict__ Wl, const float (&x)[S],
                                           v4f (&acc)[NTO], int lane) {
#pragma unroll
  for (int ot = 0; ot < NTO; ++ot) acc[ot] = v4f{0.f, 0.f, 0.f, 0.f};
  mfma_accum<0, NTO, S, 0, S>(Wl, x, acc, lane);
}

template <int NTO>
__device__ __forceinline__ void relu_to_inputs(const v4f (&acc)[NTO], float (&x)[NTO * 4]) {
#pragma unroll
  for (int b = 0; b < NTO; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) x[4 * b + r] = fmaxf(acc[b][r], 0.f);
}

// Hidden and output layers from the first layer's pre-activations `acc`;
// W: the weights that follow the first layer's.
template <class Sh>
__device__ __forceinline__ void mlp_tail(const float* __restrict__ W, const v4f (&acc1)[Sh::NT], v4f& out,
                                         int lane) {
  float h[Sh::S_HID];
  relu_to_inputs<Sh::NT>(acc1, h);
  v4f acc[Sh::NT];
#pragma unroll
  for (int k = 1; k < Sh::NH; ++k) {
    mfma_layer<Sh::NT, Sh::S_HID>(W, h, acc, lane);
    W += Sh::NT * Sh::S_HID * 64;
    relu_to_inputs<Sh::NT>(acc, h);
  }
  v4f o[1];
  mfma_layer<1, Sh::S_HID>(W, h, o, lane);
  out = o[0];
}

// Whole MLP from first-layer inputs x1 to the 16-row output tile `out`
// (lane holds rows 4g..4g+3).
template <class Sh, int S1>
__device__ __forceinline__ void mlp_forward(const float* __restrict__ Wlds, const float (&x1)[S1],
                                            v4f& out, int lane) {
  v4f acc[Sh::NT];
  mfma_layer<Sh::NT, S1>(Wlds, x1, acc, lane);
  mlp_tail<Sh>(Wlds + Sh::NT * S1 * 64, acc, out, lane);
}

// The colour decoder over several views of one point (Eq. 6): its input is
// [f_rad ; PE(d_v)], so the first layer's product with the radiance features
// (k-steps [0, SPLIT)) does not depend on the view.  mlp_first_part forms it
// once; mlp_forward_rest adds the view's direction part (k-steps [SPLIT, S1))
// to a copy and runs the remaining layers.  Same bits as mlp_forward.
template <class Sh, int S1, int SPLIT>
__device__ __forceinline__ void mlp_first_part(const float* __restrict__ Wlds, const float (&x1)[S1],
                                               v4f (&acc)[Sh::NT], int lane) {
#pragma unroll
  for (int ot = 0; ot < Sh::NT; ++ot) acc[ot] = v4f{0.f, 0.f, 0.f, 0.f};
  mfma_accum<0, Sh::NT, S1, 0, SPLIT>(Wlds, x1, acc, lane);
}

template <class Sh, int S1, int SPLIT>
__device__ __forceinline__ void mlp_forward_rest(const float* __restrict__ Wlds, const float (&x1)[S1],
                                                 v4f (&acc)[Sh::NT], v4f& out, int lane) {
  mfma_accum<0, Sh::NT, S1, SPLIT, S1>(Wlds, x1, acc, lane);
  mlp_tail<Sh>(Wlds + Sh::NT * S1 * 64, acc, out, lane);
}


// ---------------------------------------------------------------------------
// BF16 operands (v_mfma_f32_16x16x32_bf16, FP32 accumulate).  Same k order
// as the FP32 path, 8 consecutive lane inputs per k-step: per layer
// [out_tile][s/8][lane][8] bf16 (one 16-byte A operand per lane and step).
template <class Sh>
__device__ void permute_mlp_fwd_bf16(__bf16* dst, const float* __restrict__ W, bool colour, int tid, int stride) {
  const int n_out = colour ? HYRF_COL_OUT : HYRF_GEO_OUT;
  const int in1 = colour ? Sh::IN_COL : Sh::IN_GEO;
  const int S1 = colour ? Sh::S_COL1_8 : Sh::S_GEO1_8;
  int dst_off = 0, g_off = 0;
  for (int layer = 0; layer <= Sh::NH; ++layer) {
    const bool first = layer == 0;
    const bool last = layer == Sh::NH;
    const int S = first ? S1 : Sh::S_HID;
    const int NTo = last ? 1 : Sh::NT;
    const int rows = last ? n_out : Sh::HID;
    const int in = first ? in1 : Sh::HID;
    const int cnt = NTo * S * 64;
    for (int e = tid; e < cnt; e += stride) {
      const int s8 = e & 7;
      const int lane = (e >> 3) & 63;
      const int rest = e >> 9;                 // ot * (S/8) + q
      const int q = rest % (S / 8);
      const int ot = rest / (S / 8);
      const int s = q * 8 + s8;
      const int g = lane >> 4;
      const int row = ot * 16 + (lane & 15);
      const int col = first ? first_layer_col<Sh::L>(s, g, colour) : (16 * (s >> 2) + 4 * g + (s & 3));
      float val = 0.f;
      if (row < rows && col >= 0 && col < in) val = W[g_off + row * in + col];
      dst[dst_off + e] = (__bf16)val;
    }
    dst_off += cnt;
    g_off += rows * in;
  }
}

template <int OT0, int OT1, int S, int K0, int K1>
__device__ __forceinline__ void mfma_accum_bf16(const __bf16* __restrict__ Wl, const float (&x)[S],
                                                v4f (&acc)[OT1 - OT0], int lane) {
  static_assert(S % 8 == 0 && K0 % 8 == 0 && K1 % 8 == 0 && 0 <= K0 && K0 <= K1 && K1 <= S, "bf16 k-step range");
  constexpr int NO = OT1 - OT0;
  // the next k-step's weights are read while the current step's MFMAs run
  v8bf w[2][NO];
  if constexpr (K0 < K1) {
#pragma unroll
    for (int ot = OT0; ot < OT1; ++ot)
      w[0][ot - OT0] = *reinterpret_cast<const v8bf*>(Wl + ((ot * (S / 8) + K0 / 8) * 64 + lane) * 8);
  }
#pragma unroll
  for (int q = K0 / 8; q < K1 / 8; ++q) {
    const int cur = (q - K0 / 8) & 1;
    if (q + 1 < K1 / 8) {
#pragma unroll
      for (int ot = OT0; ot < OT1; ++ot)
        w[cur ^ 1][ot - OT0] = *reinterpret_cast<const v8bf*>(Wl + ((ot * (S / 8) + q + 1) * 64 + lane) * 8);
    }
    // the reads above issue before this k-step's MFMAs (scheduling
    // barrier); at most two k-steps of weights in flight (register budget)
    __builtin_amdgcn_sched_barrier(0);
    v8bf b;
#pragma unroll
    for (int e = 0; e < 8; ++e) b[e] = (__bf16)x[8 * q + e];
#pragma unroll
    for (int ot = OT0; ot < OT1; ++ot)
      acc[ot - OT0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w[cur][ot - OT0], b, acc[ot - OT0], 0, 0, 0);
  }
}

template <int NTO, int S>
__device__ __forceinline__ void mfma_layer_bf16(const __bf16* __restrict__ Wl, const float (&x)[S],
                                                v4f (&acc)[NTO], int lane) {
#pragma unroll
  for (int ot = 0; ot < NTO; ++ot) acc[ot] = v4f{0.f, 0.f, 0.f, 0.f};
  mfma_accum_bf16<0, NTO, S, 0, S>(Wl, x, acc, lane);
}

template <class Sh>
__device__ __forceinline__ void mlp_tail_bf16(const __bf16* __restrict__ W, const v4f (&acc1)[Sh::NT], v4f& out,
                                              int lane) {
  float h[Sh::S_HID];
  relu_to_inputs<Sh::NT>(acc1, h);
  v4f acc[Sh::NT];
#pragma unroll
  for (int k = 1; k < Sh::NH; ++k) {
    mfma_layer_bf16<Sh::NT, Sh::S_HID>(W, h, acc, lane);
    W += Sh::NT * Sh::S_HID * 64;
    relu_to_inputs<Sh::NT>(acc, h);
  }
  v4f o[1];
  mfma_layer_bf16<1, Sh::S_HID>(W, h, o, lane);
  out = o[0];
}

template <class Sh, int S1>
__device__ __forceinline__ void mlp_forward_bf16(const __bf16* __restrict__ Wlds, const float (&x1)[S1],
                                                 v4f& out, int lane) {
  v4f acc[Sh::NT];
  mfma_layer_bf16<Sh::NT, S1>(Wlds, x1, acc, lane);
  mlp_tail_bf16<Sh>(Wlds + Sh::NT * S1 * 64, acc, out, lane);
}

template <class Sh, int S1, int SPLIT>
__device__ __forceinline__ void mlp_first_part_bf16(const __bf16* __restrict__ Wlds, const float (&x1)[S1],
                                                    v4f (&acc)[Sh::NT], int lane) {
#pragma unroll
  for (int ot = 0; ot < Sh::NT; ++ot) acc[ot] = v4f{0.f, 0.f, 0.f, 0.f};
  mfma_accum_bf16<0, Sh::NT, S1, 0, SPLIT>(Wlds, x1, acc, lane);
}

template <class Sh, int S1, int SPLIT>
__device__ __forceinline__ void mlp_forward_rest_bf16(const __bf16* __restrict__ Wlds, const float (&x1)[S1],
                                                      v4f (&acc)[Sh::NT], v4f& out, int lane) {
  mfma_accum_bf16<0, Sh::NT, S1, SPLIT, S1>(Wlds, x1, acc, lane);
  mlp_tail_bf16<Sh>(Wlds + Sh::NT * S1 * 64, acc, out, lane);
}

// Table entry loads: FP32 pairs or FP16 pairs widened to FP32.
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 load_entry(const float* t, size_t i) {
  return *reinterpret_cast<const float2*>(t + i * 2);
}
__device__ __forceinline__ float2 load_entry(const _Float16* t, size_t i) {
  const h2_t v = *reinterpret_cast<const h2_t*>(t + i * 2);
  return make_float2((float)v.x, (float)v.y);
}

// 8-bit min-max codes: the two codes of the entry as floats; the level's
// affine decode is applied once to the interpolated code (the trilinear
// weights sum to one).
__device__ __forceinline__ float2 load_entry(const uint8_t* t, size_t i) {
  const uchar2 v = *reinterpret_cast<const uchar2*>(t + i * 2);
  return make_float2((float)v.x, (float)v.y);
}

// Gather this lane's levels from both tables at contracted position x.
// fg / fr: lane features (level g + 4k, feature f) at index 2k + f.
//
// jac (nullable): this point's [L][12] row of spatial feature derivatives,
// written for the lane's levels: d f / d x = sum_c table[c] d w_c / d x with
// d w_c / d x_d = N_l * (+-1) * (product of the other two 1D weights); the
// geometry half repeats the radiance half when GEO is false.
template <int L, bool GEO, class TT>
__device__ __forceinline__ void gather_lane(const GridP& gp, const double x[3], int g,
                                            const TT* __restrict__ tg, const TT* __restrict__ tr,
                                            float (&fg)[L / 2], float (&fr)[L / 2],
                                            uint32_t* dbg_geo, uint32_t* dbg_rad, float* jac = nullptr) {
  const uint32_t Tg = gp.mask_geo + 1u, Tr = gp.mask_rad + 1u;
#pragma unroll
  for (int k = 0; k < L / 4; ++k) {
    const int lev = g + 4 * k;
    const int res = gp.res[lev];
    int ci[3];
    float w[3];
    grid_cell(x, res, ci, w);
    const uint32_t side = (uint32_t)res + 1u;
    const bool dg = (gp.dense_geo >> lev) & 1u;
    const bool dr = (gp.dense_rad >> lev) & 1u;
    float2 vg[8], vr[8];
    float wc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const uint32_t cx = (uint32_t)ci[0] + (c & 1);
      const uint32_t cy = (uint32_t)ci[1] + ((c >> 1) & 1);
      const uint32_t cz = (uint32_t)ci[2] + ((c >> 2) & 1);
      const float wx = (c & 1) ? w[0] : 1.f - w[0];
      const float wy = ((c >> 1) & 1) ? w[1] : 1.f - w[1];
      const float wz = ((c >> 2) & 1) ? w[2] : 1.f - w[2];
      wc[c] = (wx * wy) * wz;
      const uint32_t rr = corner_row(cx, cy, cz, dr, side, gp.mask_rad);
      vr[c] = load_entry(tr, (size_t)lev * Tr + rr);
      if (dbg_rad) dbg_rad[lev * 8 + c] = rr;
      if (GEO) {
        const uint32_t rg = corner_row(cx, cy, cz, dg, side, gp.mask_geo);
        vg[c] = load_entry(tg, (size_t)lev * Tg + rg);
        if (dbg_geo) dbg_geo[lev * 8 + c] = rg;
      }
    }
    float a0 = 0.f, a1 = 0.f, b0 = 0.f, b1 = 0.f;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      a0 = fmaf(wc[c], vr[c].x, a0);
      a1 = fmaf(wc[c], vr[c].y, a1);
      if (GEO) {
        b0 = fmaf(wc[c], vg[c].x, b0);
        b1 = fmaf(wc[c], vg[c].y, b1);
      }
    }
    // (8-bit tables are a render-only format: no derivatives for them)
    if (!std::is_same<TT, uint8_t>::value && jac) {
      float jr[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, jg[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      const float fres = (float)res;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const float wx = (c & 1) ? w[0] : 1.f - w[0];
        const float wy = ((c >> 1) & 1) ? w[1] : 1.f - w[1];
        const float wz = ((c >> 2) & 1) ? w[2] : 1.f - w[2];
        const float dw[3] = {fres * ((c & 1) ? 1.f : -1.f) * (wy * wz),
                             fres * (((c >> 1) & 1) ? 1.f : -1.f) * (wx * wz),
                             fres * (((c >> 2) & 1) ? 1.f : -1.f) * (wx * wy)};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          jr[d] = fmaf(vr[c].x, dw[d], jr[d]);
          jr[3 + d] = fmaf(vr[c].y, dw[d], jr[3 + d]);
          if (GEO) {
            jg[d] = fmaf(vg[c].x, dw[d], jg[d]);
            jg[3 + d] = fmaf(vg[c].y, dw[d], jg[3 + d]);
          }
        }
      }
      float4* o = reinterpret_cast<float4*>(jac + (size_t)lev * 12);
      if (GEO) {
        o[0] = make_float4(jg[0], jg[1], jg[2], jg[3]);
        o[1] = make_float4(jg[4], jg[5], jr[0], jr[1]);
      } else {
        o[0] = make_float4(jr[0], jr[1], jr[2], jr[3]);
        o[1] = make_float4(jr[4], jr[5], jr[0], jr[1]);
      }
      o[2] = make_float4(jr[2], jr[3], jr[4], jr[5]);
    }
    if constexpr (std::is_same<TT, uint8_t>::value) {
      const float2 qr = *reinterpret_cast<const float2*>(gp.qp_rad + 2 * lev);
      a0 = qr.x + qr.y * a0;
      a1 = qr.x + qr.y * a1;
      if (GEO) {
        const float2 qg = *reinterpret_cast<const float2*>(gp.qp_geo + 2 * lev);
        b0 = qg.x + qg.y * b0;
        b1 = qg.x + qg.y * b1;
      }
    }
    fr[2 * k] = a0;
    fr[2 * k + 1] = a1;
    if (GEO) {
      fg[2 * k] = b0;
      fg[2 * k + 1] = b1;
    }
    // one level's 16 loads in flight per lane at a time (register budget)
    asm volatile("" ::: "memory");
  }
}

// PE values of lane group g (octave g): sin(2^g pi d) then cos(2^g pi d).
__device__ __forceinline__ void pe_lane(int g, float dx, float dy, float dz, float pe[6]) {
  const float sc = (float)(1 << g);
  sincospif(sc * dx, &pe[0], &pe[3]);
  sincospif(sc * dy, &pe[1], &pe[4]);
  sincospif(sc * dz, &pe[2], &pe[5]);
}

}  // namespace hyrf
