// Adjoint of the tiny MLPs on MFMA, in the transposed lane layout of
// field.h (a point's activations stay in the lanes that own the point).
//
//  * dX = W^T dY runs as D[in x points] = W^T[in x out] * dY[out x points];
//    its A operand (W^T) is pre-permuted like the forward weights, with the
//    rows of the first layer ordered so that the result lands in each lane's
//    own input order (row 16*ot + 4g + r <-> the lane's input s = 4*ot + r).
//  * dW = sum over points of dY (x) X needs the point index on the MFMA's k
//    axis, i.e. across lane groups: the workgroup stages X and dY of its
//    NWV * 16 points in LDS ([point][feature], column-swizzled) and
//    every wave accumulates a fixed subset of the 16x16 dW tiles over all
//    staged points in registers, across every round of the persistent loop.
#pragma once
#include <type_traits>

#include "field.h"

namespace hyrf {

// Waves per workgroup (NWV) is a template parameter of the adjoint: a
// workgroup stages NWV * 16 points per round.
constexpr int STAGE_W = 64;                    // staged feature columns

template <class Sh>
struct BwdShape {
  // dW tiles per layer: (rows/16 rounded up) x (in/16 rounded up)
  static constexpr int TI_GEO1 = (Sh::IN_GEO + 15) / 16;
  static constexpr int TI_COL1 = (Sh::IN_COL + 15) / 16;
  static constexpr int TI_H = Sh::HID / 16;
  static constexpr int TILES_GEO = Sh::NT * TI_GEO1 + (Sh::NH - 1) * Sh::NT * TI_H + TI_H;
  static constexpr int TILES_COL = Sh::NT * TI_COL1 + (Sh::NH - 1) * Sh::NT * TI_H + TI_H;
  static constexpr int TILES = TILES_GEO + TILES_COL;
  template <int NWV>
  static constexpr int ACC = (TILES + NWV - 1) / NWV;   // dW tiles per wave
  // backward-permuted weight floats per MLP
  static constexpr int WB_GEO = Sh::NT * 4 * 64 + (Sh::NH - 1) * Sh::NT * Sh::S_HID * 64 +
                                (Sh::S_GEO1 / 4) * Sh::S_HID * 64;
  static constexpr int WB_COL = Sh::NT * 4 * 64 + (Sh::NH - 1) * Sh::NT * Sh::S_HID * 64 +
                                (Sh::S_COL1 / 4) * Sh::S_HID * 64;
};

// Backward A-operand permutation (W^T) of one MLP, layers in the order the
// adjoint uses them: output layer, hidden layers from last to first, first
// layer.  Layout per layer [row_tile][s/4][lane][s%4].
template <class Sh>
__device__ void permute_mlp_bwd(float* dst, const float* __restrict__ W, bool colour, int tid, int stride) {
  const int n_out = colour ? HYRF_COL_OUT : HYRF_GEO_OUT;
  const int in1 = colour ? Sh::IN_COL : Sh::IN_GEO;
  const int S1 = colour ? Sh::S_COL1 : Sh::S_GEO1;
  // global offsets of the layers in the flat [out][in] weight list
  int goff[4];
  goff[0] = 0;
  goff[1] = Sh::HID * in1;
  goff[2] = goff[1] + (Sh::NH >= 2 ? Sh::HID * Sh::HID : 0);
  const int g_out = Sh::NH == 2 ? goff[2] : goff[1];
  int dst_off = 0;
  // step = index into the adjoint sequence: 0 = output layer, 1..NH-1 =
  // hidden layer NH-1..1 (weights W_k, k = NH - step), NH = first layer
  for (int step = 0; step <= Sh::NH; ++step) {
    const bool out_l = step == 0;
    const bool first = step == Sh::NH;
    const int S = out_l ? 4 : Sh::S_HID;                 // k steps: over the layer's output rows
    const int RT = first ? S1 / 4 : Sh::NT;              // row tiles: over the layer's inputs
    const int cnt = RT * S * 64;
    for (int e = tid; e < cnt; e += stride) {
      const int s4 = e & 3;
      const int lane = (e >> 2) & 63;
      const int rest = e >> 8;
      const int sq = rest % (S / 4);
      const int rt = rest / (S / 4);
      const int kk = lane >> 4, i = lane & 15;
      // k index = row of W (the layer's output unit)
      const int wrow = out_l ? (4 * kk + s4) : (16 * sq + 4 * kk + s4);
      float val = 0.f;
      if (out_l) {
        const int wcol = 16 * rt + i;                    // hidden unit
        if (wrow < n_out) val = W[g_out + wrow * Sh::HID + wcol];
      } else if (!first) {
        const int wcol = 16 * rt + i;
        val = W[goff[1] + wrow * Sh::HID + wcol];        // only NH == 2 reaches here
      } else {
        const int s_in = 4 * rt + (i & 3), g_in = i >> 2;
        const int wcol = first_layer_col<Sh::L>(s_in, g_in, colour);
        if (wcol >= 0 && wcol < in1) val = W[wrow * in1 + wcol];
      }
      dst[dst_off + e] = val;
    }
    dst_off += cnt;
  }
}

// Forward pass that keeps the post-ReLU hidden activations (lane order).
template <class Sh, int S1>
__device__ __forceinline__ void mlp_forward_keep(const float* __restrict__ Wf, const float (&x1)[S1],
                                                 float (&h)[Sh::NH][Sh::S_HID], v4f& out, int lane) {
  v4f acc[Sh::NT];
  mfma_layer<Sh::NT, S1>(Wf, x1, acc, lane);
  const float* W = Wf + Sh::NT * S1 * 64;
  relu_to_inputs<Sh::NT>(acc, h[0]);
#pragma unroll
  for (int k = 1; k < Sh::NH; ++k) {
    mfma_layer<Sh::NT, Sh::S_HID>(W, h[k - 1], acc, lane);
    W += Sh::NT * Sh::S_HID * 64;
    relu_to_inputs<Sh::NT>(acc, h[k]);
  }
  v4f o[1];
  mfma_layer<1, Sh::S_HID>(W, h[Sh::NH - 1], o, lane);
  out = o[0];
}

// The same from the first layer's pre-activations (the colour decoder with
// its view-independent part formed once: mlp_first_part, field.h).
template <class Sh, int S1, int SPLIT>
__device__ __forceinline__ void mlp_forward_keep_rest(const float* __restrict__ Wf, const float (&x1)[S1],
                                                      v4f (&acc)[Sh::NT], float (&h)[Sh::NH][Sh::S_HID],
                                                      v4f& out, int lane) {
  mfma_accum<0, Sh::NT, S1, SPLIT, S1>(Wf, x1, acc, lane);
  const float* W = Wf + Sh::NT * S1 * 64;
  relu_to_inputs<Sh::NT>(acc, h[0]);
  v4f a2[Sh::NT];
#pragma unroll
  for (int k = 1; k < Sh::NH; ++k) {
    mfma_layer<Sh::NT, Sh::S_HID>(W, h[k - 1], a2, lane);
    W += Sh::NT * Sh::S_HID * 64;
    relu_to_inputs<Sh::NT>(a2, h[k]);
  }
  v4f o[1];
  mfma_layer<1, Sh::S_HID>(W, h[Sh::NH - 1], o, lane);
  out = o[0];
}

__device__ __forceinline__ int swz(int row, int col) { return row * STAGE_W + (col ^ ((row & 1) << 4)); }

__device__ __forceinline__ float bf16r(float x) { return (float)(__bf16)x; }

// Tile t of a layer with TO output and TI input tiles is (ot, it).  The
// colour decoder's first layer numbers its tiles input-major (ITMAJ), so that
// the tiles of its feature columns and those of its direction columns, when
// accumulated apart, each spread evenly over the waves.
template <int TO, int TI, bool ITMAJ>
__host__ __device__ constexpr int tile_ot(int t) { return ITMAJ ? t % TO : t / TI; }
template <int TO, int TI, bool ITMAJ>
__host__ __device__ constexpr int tile_it(int t) { return ITMAJ ? t / TO : t % TI; }

// Compile-time loop: f(std::integral_constant<int, i>) for i in [I0, I1), so
// that register-array indices derived from i stay constants (a runtime index
// would move the array to scratch memory).
template <int I0, int I1, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I0 < I1) {
    f(std::integral_constant<int, I0>{});
    static_for<I0 + 1, I1>(f);
  }
}

// Accumulate the dW tiles of one layer whose input tile lies in [IT0, IT1)
// from the staged [point][feature] arrays: tile (ot, it) += sum_p
// Y[p][16 ot + i] X[p][16 it + j].  Tile ids TB .. TB + TO*TI - 1; wave w
// owns ids with id % NWV == w.
template <int TB, int TO, int TI, bool ITMAJ, int IT0, int IT1, int ACC, int NWV>
__device__ __forceinline__ void dw_tiles_range(const float* Xs, const float* Ys, v4f (&acc)[ACC], int w, int lane) {
  const int kk = lane >> 4, i = lane & 15;
  constexpr int KS = NWV * 16 / 4;   // MFMA k-steps over the staged points
  // the layer's tile numbers [T0, T1) that hold the input tiles [IT0, IT1)
  constexpr bool FULL = IT0 == 0 && IT1 == TI;
  constexpr int T0 = FULL ? 0 : (ITMAJ ? IT0 * TO : -1);
  constexpr int T1 = FULL ? TO * TI : (ITMAJ ? IT1 * TO : -1);
  if constexpr (T0 >= 0 && TB % NWV == 0 && T0 % NWV == 0 && (T1 - T0) % NWV == 0) {
    // every wave owns the same number of the range's tiles, t = w + NWV m,
    // with accumulators acc[TB / NWV + m]: independent MFMA chains stepped
    // together over k, so that they overlap each other and the operand reads
    constexpr int M0 = T0 / NWV, NM = (T1 - T0) / NWV;
    int ya[NM], xa[NM];
    static_for<0, NM>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      const int t = w + NWV * (M0 + m);
      ya[m] = 16 * tile_ot<TO, TI, ITMAJ>(t) + i;
      xa[m] = 16 * tile_it<TO, TI, ITMAJ>(t) + i;
    });
    // operands of k-step s + 1 are read before the MFMAs of step s (a
    // scheduling barrier between them keeps the reads ahead)
    float av[2][NM], bv[2][NM];
    static_for<0, NM>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      av[0][m] = Ys[swz(kk, ya[m])];
      bv[0][m] = Xs[swz(kk, xa[m])];
    });
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int cur = s & 1;
      if (s + 1 < KS) {
        const int p = 4 * (s + 1) + kk;
        static_for<0, NM>([&](auto mc) {
          constexpr int m = decltype(mc)::value;
          av[cur ^ 1][m] = Ys[swz(p, ya[m])];
          bv[cur ^ 1][m] = Xs[swz(p, xa[m])];
        });
      }
      __builtin_amdgcn_sched_barrier(0);
      static_for<0, NM>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        v4f& c = acc[TB / NWV + M0 + m];
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(av[cur][m], bv[cur][m], c, 0, 0, 0);
      });
    }
  } else {
    static_for<0, TO * TI>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      constexpr int ot = tile_ot<TO, TI, ITMAJ>(t), it = tile_it<TO, TI, ITMAJ>(t);
      constexpr int id = TB + t;
      if constexpr (it >= IT0 && it < IT1) {
        if (id % NWV == w) {
          // k runs over the staged points, 4 per MFMA, in four partial sums
          // (independent MFMA chains); the operands of the next four k-steps
          // are read before the MFMAs of the current four
          static_assert(KS % 4 == 0, "staged points per round");
          v4f c[4] = {acc[id / NWV], v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};
          float av[2][4], bv[2][4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            av[0][u] = Ys[swz(4 * u + kk, 16 * ot + i)];
            bv[0][u] = Xs[swz(4 * u + kk, 16 * it + i)];
          }
#pragma unroll
          for (int q = 0; q < KS / 4; ++q) {
            const int cur = q & 1;
            if (q + 1 < KS / 4) {
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int p = 4 * (4 * (q + 1) + u) + kk;
                av[cur ^ 1][u] = Ys[swz(p, 16 * ot + i)];
                bv[cur ^ 1][u] = Xs[swz(p, 16 * it + i)];
              }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < 4; ++u) c[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[cur][u], bv[cur][u], c[u], 0, 0, 0);
          }
          acc[id / NWV] = (c[0] + c[1]) + (c[2] + c[3]);
        }
      }
    });
  }
}

template <int TB, int TO, int TI, int ACC, int NWV>
__device__ __forceinline__ void dw_tiles(const float* Xs, const float* Ys, v4f (&acc)[ACC], int w, int lane) {
  dw_tiles_range<TB, TO, TI, false, 0, TI, ACC, NWV>(Xs, Ys, acc, w, lane);
}

// Write rows (lane order: unit 16b + 4g + r = v[4b + r]) of this lane's point.
template <int N, bool BF = false>
__device__ __forceinline__ void stage_units(float* S, int pt, int g, const float (&v)[N]) {
#pragma unroll
  for (int b = 0; b < N / 4; ++b) {
    float4 q = make_float4(v[4 * b], v[4 * b + 1], v[4 * b + 2], v[4 * b + 3]);
    if (BF) q = make_float4(bf16r(q.x), bf16r(q.y), bf16r(q.z), bf16r(q.w));
    *reinterpret_cast<float4*>(S + swz(pt, 16 * b + 4 * g)) = q;
  }
}

// Write the first-layer inputs of lane k-steps [S0, SE) (lane order) at
// their canonical columns.
template <class Sh, int S1, int S0, int SE, bool BF = false>
__device__ __forceinline__ void stage_inputs(float* S, int pt, int g, const float (&x)[S1], bool colour) {
#pragma unroll
  for (int s = S0; s < SE; ++s) {
    const int col = first_layer_col<Sh::L>(s, g, colour);
    if (col >= 0) S[swz(pt, col)] = BF ? bf16r(x[s]) : x[s];
  }
}

// Output and hidden layers of one MLP's adjoint for the wave's 16 points:
// their dW tiles, and dh = the gradient of the first layer's pre-activation
// output.  dout: 16-row output gradient tile (lane holds rows 4g..4g+3).
// Returns the first layer's adjoint operands.  Contains workgroup barriers:
// every thread of the workgroup must call it with the same template
// arguments.
template <class Sh, bool COL, int ACC, int NWV, int CB = -1>
__device__ __forceinline__ const float* mlp_backward_upper(const float* __restrict__ Wb,
                                                           const float (&h)[Sh::NH][Sh::S_HID], v4f dout,
                                                           float (&dh)[Sh::S_HID], float* Xs, float* Ys,
                                                           v4f (&accW)[ACC], int w, int lane) {
  using B = BwdShape<Sh>;
  constexpr int TI1 = COL ? B::TI_COL1 : B::TI_GEO1;
  constexpr int TB0 = COL ? (CB < 0 ? B::TILES_GEO : CB) : 0;
  const int j = lane & 15, g = lane >> 4;
  const int pt = w * 16 + j;
  // ---- output layer: dW_out += dout (x) h_last
  *reinterpret_cast<float4*>(Ys + swz(pt, 4 * g)) = make_float4(dout[0], dout[1], dout[2], dout[3]);
  stage_units<Sh::S_HID>(Xs, pt, g, h[Sh::NH - 1]);
  __syncthreads();
  constexpr int TB_OUT = TB0 + Sh::NT * TI1 + (Sh::NH - 1) * Sh::NT * (Sh::HID / 16);
  dw_tiles<TB_OUT, 1, Sh::HID / 16, ACC, NWV>(Xs, Ys, accW, w, lane);
  __syncthreads();
  {
    float din[4] = {dout[0], dout[1], dout[2], dout[3]};
    v4f acc[Sh::NT];
    mfma_layer<Sh::NT, 4>(Wb, din, acc, lane);
#pragma unroll
    for (int b = 0; b < Sh::NT; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) dh[4 * b + r] = h[Sh::NH - 1][4 * b + r] > 0.f ? acc[b][r] : 0.f;
  }
  const float* W = Wb + Sh::NT * 4 * 64;
  // ---- hidden layers, last to first (only NH == 2: one W_2); not
  // instantiated for one hidden layer, whose tile numbers end before them
  if constexpr (Sh::NH >= 2) {
#pragma unroll
    for (int k = Sh::NH - 1; k >= 1; --k) {
      stage_units<Sh::S_HID>(Ys, pt, g, dh);
      stage_units<Sh::S_HID>(Xs, pt, g, h[k - 1]);
      __syncthreads();
      constexpr int TB_H = TB0 + Sh::NT * TI1;
      dw_tiles<TB_H, Sh::NT, Sh::HID / 16, ACC, NWV>(Xs, Ys, accW, w, lane);
      __syncthreads();
      v4f acc[Sh::NT];
      mfma_layer<Sh::NT, Sh::S_HID>(W, dh, acc, lane);
      W += Sh::NT * Sh::S_HID * 64;
#pragma unroll
      for (int b = 0; b < Sh::NT; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) dh[4 * b + r] = h[k - 1][4 * b + r] > 0.f ? acc[b][r] : 0.f;
    }
  }
  return W;
}

// First layer of the adjoint restricted to the lane input k-steps [S0, SE):
// dW_1 += dh (x) x over the input tiles [IT0, IT1) (whose columns those
// k-steps hold) and the rows [S0, SE) of dx = W_1^T dh.  Barriers as above.
template <class Sh, bool COL, int S1, int S0, int SE, int IT0, int IT1, int ACC, int NWV, int CB = -1>
__device__ __forceinline__ void mlp_backward_first(const float* __restrict__ W, const float (&x1)[S1],
                                                   const float (&dh)[Sh::S_HID], float (&dx)[S1], float* Xs,
                                                   float* Ys, v4f (&accW)[ACC], int w, int lane) {
  using B = BwdShape<Sh>;
  constexpr int TI1 = COL ? B::TI_COL1 : B::TI_GEO1;
  constexpr int TB0 = COL ? (CB < 0 ? B::TILES_GEO : CB) : 0;
  const int j = lane & 15, g = lane >> 4;
  const int pt = w * 16 + j;
  stage_units<Sh::S_HID>(Ys, pt, g, dh);
  stage_inputs<Sh, S1, S0, SE>(Xs, pt, g, x1, COL);
  __syncthreads();
  dw_tiles_range<TB0, Sh::NT, TI1, COL, IT0, IT1, ACC, NWV>(Xs, Ys, accW, w, lane);
  __syncthreads();
  v4f acc[(SE - S0) / 4];
#pragma unroll
  for (int b = 0; b < (SE - S0) / 4; ++b) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};
  mfma_accum<S0 / 4, SE / 4, Sh::S_HID, 0, Sh::S_HID>(W, dh, acc, lane);
#pragma unroll
  for (int b = 0; b < (SE - S0) / 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) dx[S0 + 4 * b + r] = acc[b][r];
}

// Full adjoint of one MLP for the wave's 16 points.  Returns dx (lane input
// order).  Tile ids as BwdShape, except that CB >= 0 moves the colour
// decoder's tiles to start at CB (0 for a kernel that has no geometry
// decoder, so that it holds no accumulators for geometry tiles).
template <class Sh, bool COL, int S1, int ACC, int NWV, int CB = -1>
__device__ __forceinline__ void mlp_backward(const float* __restrict__ Wb, const float (&x1)[S1],
                                             const float (&h)[Sh::NH][Sh::S_HID], v4f dout,
                                             float (&dx)[S1], float* Xs, float* Ys, v4f (&accW)[ACC],
                                             int w, int lane) {
  using B = BwdShape<Sh>;
  static_assert(S1 == (COL ? Sh::S_COL1 : Sh::S_GEO1), "first-layer width");
  constexpr int TI1 = COL ? B::TI_COL1 : B::TI_GEO1;
  float dh[Sh::S_HID];
  const float* W = mlp_backward_upper<Sh, COL, ACC, NWV, CB>(Wb, h, dout, dh, Xs, Ys, accW, w, lane);
  mlp_backward_first<Sh, COL, S1, 0, S1, 0, TI1, ACC, NWV, CB>(W, x1, dh, dx, Xs, Ys, accW, w, lane);
}

// ---------------------------------------------------------------------------
// Precision variant: bfloat16 operands, float32 accumulation.  The decoder
// recompute and dX run on v_mfma_f32_16x16x32_bf16 with the weights in the
// same lane order packed 8 per k-step; dW runs on the float32 MFMA over
// staged operands already rounded to bfloat16 (their products are exact in
// float32, so this equals a bfloat16 product with float32 accumulation).
template <class Sh>
__device__ void permute_mlp_bwd_bf16(__bf16* dst, const float* __restrict__ W, bool colour, int tid, int stride) {
  const int n_out = colour ? HYRF_COL_OUT : HYRF_GEO_OUT;
  const int in1 = colour ? Sh::IN_COL : Sh::IN_GEO;
  const int S1 = colour ? Sh::S_COL1_8 : Sh::S_GEO1_8;
  const int g1 = Sh::HID * in1;
  const int g_out = Sh::NH == 2 ? g1 + Sh::HID * Sh::HID : g1;
  int dst_off = 0;
  for (int step = 0; step <= Sh::NH; ++step) {
    const bool out_l = step == 0;
    const bool first = step == Sh::NH;
    const int S = out_l ? 8 : Sh::S_HID;
    const int RT = first ? S1 / 4 : Sh::NT;
    const int cnt = RT * S * 64;
    for (int e = tid; e < cnt; e += stride) {
      const int s8 = e & 7;
      const int lane = (e >> 3) & 63;
      const int rest = e >> 9;
      const int q = rest % (S / 8);
      const int rt = rest / (S / 8);
      const int kk = lane >> 4, i = lane & 15;
      const int s = 8 * q + s8;
      float val = 0.f;
      if (out_l) {
        const int wrow = 4 * kk + s;
        if (s < 4 && wrow < n_out) val = W[g_out + wrow * Sh::HID + 16 * rt + i];
      } else {
        const int wrow = 16 * (s >> 2) + 4 * kk + (s & 3);
        if (!first) {
          val = W[g1 + wrow * Sh::HID + 16 * rt + i];
        } else {
          const int wcol = first_layer_col<Sh::L>(4 * rt + (i & 3), i >> 2, colour);
          if (wcol >= 0 && wcol < in1) val = W[wrow * in1 + wcol];
        }
      }
      dst[dst_off + e] = (__bf16)val;
    }
    dst_off += cnt;
  }
}

template <class Sh, int S1>
__device__ __forceinline__ void mlp_forward_keep_bf16(const __bf16* __restrict__ Wf, const float (&x1)[S1],
                                                      float (&h)[Sh::NH][Sh::S_HID], v4f& out, int lane) {
  v4f acc[Sh::NT];
  mfma_layer_bf16<Sh::NT, S1>(Wf, x1, acc, lane);
  const __bf16* W = Wf + Sh::NT * S1 * 64;
  relu_to_inputs<Sh::NT>(acc, h[0]);
#pragma unroll
  for (int k = 1; k < Sh::NH; ++k) {
    mfma_layer_bf16<Sh::NT, Sh::S_HID>(W, h[k - 1], acc, lane);
    W += Sh::NT * Sh::S_HID * 64;
    relu_to_inputs<Sh::NT>(acc, h[k]);
  }
  v4f o[1];
  mfma_layer_bf16<1, Sh::S_HID>(W, h[Sh::NH - 1], o, lane);
  out = o[0];
}

template <class Sh, int S1, int SPLIT>
__device__ __forceinline__ void mlp_forward_keep_rest_bf16(const __bf16* __restrict__ Wf, const float (&x1)[S1],
                                                           v4f (&acc)[Sh::NT], float (&h)[Sh::NH][Sh::S_HID],
                                                           v4f& out, int lane) {
  mfma_accum_bf16<0, Sh::NT, S1, SPLIT, S1>(Wf, x1, acc, lane);
  const __bf16* W = Wf + Sh::NT * S1 * 64;
  relu_to_inputs<Sh::NT>(acc, h[0]);
  v4f a2[Sh::NT];
#pragma unroll
  for (int k = 1; k < Sh::NH; ++k) {
    mfma_layer_bf16<Sh::NT, Sh::S_HID>(W, h[k - 1], a2, lane);
    W += Sh::NT * Sh::S_HID * 64;
    relu_to_inputs<Sh::NT>(a2, h[k]);
  }
  v4f o[1];
  mfma_layer_bf16<1, Sh::S_HID>(W, h[Sh::NH - 1], o, lane);
  out = o[0];
}

template <class Sh, bool COL, int ACC, int NWV, int CB = -1>
__device__ __forceinline__ const __bf16* mlp_backward_upper_bf16(const __bf16* __restrict__ Wb,
                                                                 const float (&h)[Sh::NH][Sh::S_HID], v4f dout,
                                                                 float (&dh)[Sh::S_HID], float* Xs, float* Ys,
                                                                 v4f (&accW)[ACC], int w, int lane) {
  using B = BwdShape<Sh>;
  constexpr int TI1 = COL ? B::TI_COL1 : B::TI_GEO1;
  constexpr int TB0 = COL ? (CB < 0 ? B::TILES_GEO : CB) : 0;
  const int j = lane & 15, g = lane >> 4;
  const int pt = w * 16 + j;
  *reinterpret_cast<float4*>(Ys + swz(pt, 4 * g)) =
      make_float4(bf16r(dout[0]), bf16r(dout[1]), bf16r(dout[2]), bf16r(dout[3]));
  stage_units<Sh::S_HID, true>(Xs, pt, g, h[Sh::NH - 1]);
  __syncthreads();
  constexpr int TB_OUT = TB0 + Sh::NT * TI1 + (Sh::NH - 1) * Sh::NT * (Sh::HID / 16);
  dw_tiles<TB_OUT, 1, Sh::HID / 16, ACC, NWV>(Xs, Ys, accW, w, lane);
  __syncthreads();
  {
    const float din[8] = {dout[0], dout[1], dout[2], dout[3], 0.f, 0.f, 0.f, 0.f};
    v4f acc[Sh::NT];
    mfma_layer_bf16<Sh::NT, 8>(Wb, din, acc, lane);
#pragma unroll
    for (int b = 0; b < Sh::NT; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) dh[4 * b + r] = h[Sh::NH - 1][4 * b + r] > 0.f ? acc[b][r] : 0.f;
  }
  const __bf16* W = Wb + Sh::NT * 8 * 64;
  if constexpr (Sh::NH >= 2) {   // hidden layers, as in the float32 version
#pragma unroll
    for (int k = Sh::NH - 1; k >= 1; --k) {
      stage_units<Sh::S_HID, true>(Ys, pt, g, dh);
      stage_units<Sh::S_HID, true>(Xs, pt, g, h[k - 1]);
      __syncthreads();
      constexpr int TB_H = TB0 + Sh::NT * TI1;
      dw_tiles<TB_H, Sh::NT, Sh::HID / 16, ACC, NWV>(Xs, Ys, accW, w, lane);
      __syncthreads();
      v4f acc[Sh::NT];
      mfma_layer_bf16<Sh::NT, Sh::S_HID>(W, dh, acc, lane);
      W += Sh::NT * Sh::S_HID * 64;
#pragma unroll
      for (int b = 0; b < Sh::NT; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) dh[4 * b + r] = h[k - 1][4 * b + r] > 0.f ? acc[b][r] : 0.f;
    }
  }
  return W;
}

template <class Sh, bool COL, int S1, int S0, int SE, int IT0, int IT1, int ACC, int NWV, int CB = -1>
__device__ __forceinline__ void mlp_backward_first_bf16(const __bf16* __restrict__ W, const float (&x1)[S1],
                                                        const float (&dh)[Sh::S_HID], float (&dx)[S1], float* Xs,
                                                        float* Ys, v4f (&accW)[ACC], int w, int lane) {
  using B = BwdShape<Sh>;
  constexpr int TI1 = COL ? B::TI_COL1 : B::TI_GEO1;
  constexpr int TB0 = COL ? (CB < 0 ? B::TILES_GEO : CB) : 0;
  const int j = lane & 15, g = lane >> 4;
  const int pt = w * 16 + j;
  stage_units<Sh::S_HID, true>(Ys, pt, g, dh);
  stage_inputs<Sh, S1, S0, SE, true>(Xs, pt, g, x1, COL);
  __syncthreads();
  dw_tiles_range<TB0, Sh::NT, TI1, COL, IT0, IT1, ACC, NWV>(Xs, Ys, accW, w, lane);
  __syncthreads();
  v4f acc[(SE - S0) / 4];
#pragma unroll
  for (int b = 0; b < (SE - S0) / 4; ++b) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};
  mfma_accum_bf16<S0 / 4, SE / 4, Sh::S_HID, 0, Sh::S_HID>(W, dh, acc, lane);
#pragma unroll
  for (int b = 0; b < (SE - S0) / 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) dx[S0 + 4 * b + r] = acc[b][r];
}

template <class Sh, bool COL, int S1, int ACC, int NWV, int CB = -1>
__device__ __forceinline__ void mlp_backward_bf16(const __bf16* __restrict__ Wb, const float (&x1)[S1],
                                                  const float (&h)[Sh::NH][Sh::S_HID], v4f dout,
                                                  float (&dx)[S1], float* Xs, float* Ys, v4f (&accW)[ACC],
                                                  int w, int lane) {
  using B = BwdShape<Sh>;
  static_assert(S1 == (COL ? Sh::S_COL1_8 : Sh::S_GEO1_8), "first-layer width");
  constexpr int TI1 = COL ? B::TI_COL1 : B::TI_GEO1;
  float dh[Sh::S_HID];
  const __bf16* W = mlp_backward_upper_bf16<Sh, COL, ACC, NWV, CB>(Wb, h, dout, dh, Xs, Ys, accW, w, lane);
  mlp_backward_first_bf16<Sh, COL, S1, 0, S1, 0, TI1, ACC, NWV, CB>(W, x1, dh, dx, Xs, Ys, accW, w, lane);
}

}  // namespace hyrf
