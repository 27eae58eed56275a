// Wave64 / workgroup prefix-sum primitives for gfx950.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hyrf {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Inclusive prefix sum across the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    uint32_t o = __shfl_up(v, off, WAVE);
    if (lane >= off) v += o;
  }
  return v;
}

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Sum over the 64 lanes with DPP moves (no LDS crossbar): an inclusive scan
// inside each 16-lane row (row_shr 1, 2, 4, 8), then row_bcast:15 and
// row_bcast:31 carry the row totals upward; the total ends in lane 63 and is
// returned to every lane.
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, BOUND));
}
__device__ __forceinline__ float wave_sum_dpp(float v) {
  v += dpp_mov<0x111, 0xf, true>(v);   // row_shr:1
  v += dpp_mov<0x112, 0xf, true>(v);   // row_shr:2
  v += dpp_mov<0x114, 0xf, true>(v);   // row_shr:4
  v += dpp_mov<0x118, 0xf, true>(v);   // row_shr:8
  v += dpp_mov<0x142, 0xa, false>(v);  // row_bcast:15 -> rows 1, 3
  v += dpp_mov<0x143, 0xc, false>(v);  // row_bcast:31 -> rows 2, 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Lane i receives lane i - 1's value, lane 0 receives 0 (DPP wave_shr:1: a
// VALU move, no LDS crossbar).  Every lane of the wave must be active.
__device__ __forceinline__ int wave_shr1(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ float wave_shr1(float x) { return __int_as_float(wave_shr1(__float_as_int(x))); }
// DPP row_shr:N: lane l takes lane l - N of its own 16-lane row (0 where
// that lies before the row's first lane).
template <int N>
__device__ __forceinline__ float row_shr(float x) {
  static_assert(N >= 1 && N <= 15, "row shift");
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x110 + N, 0xf, 0xf, true));
}
// DPP row_bcast:15 and row_bcast:31: rows 1 and 3 take lanes 15 and 47
// (the last lanes of rows 0 and 2); rows 2 and 3 take lane 31.  The other
// rows read 0.
__device__ __forceinline__ float row_bcast15(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x142, 0xa, 0xf, false));
}
__device__ __forceinline__ float row_bcast31(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x143, 0xc, 0xf, false));
}

// Totals of 8 per-lane values over the wave, transposed: lane l ends with
// the total of value (l >> 1) & 7.  A butterfly over the lane bits inside
// each 16-lane row halves the live values per step (partners l ^ 15, l ^ 7,
// l ^ 3 by DPP row_mirror, row_half_mirror, quad_perm [3,2,1,0]; lanes keep
// the upper half of their values when bit 3, 2, 1 is set), quad_perm
// [1,0,3,2] adds the l ^ 1 partner, and two lane permutes add the other
// rows.  26 lane operations for 8 sums instead of 8 full reductions.
__device__ __forceinline__ float wave_sum8_transposed(const float (&v)[8]) {
  const int lane = lane_id();
  const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0, b1 = (lane & 2) != 0;
  float a[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const float lo = v[m] + dpp_mov<0x140, 0xf, true>(v[m]);          // row_mirror
    const float hi = v[m + 4] + dpp_mov<0x140, 0xf, true>(v[m + 4]);
    a[m] = b3 ? hi : lo;
  }
  float b[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const float lo = a[m] + dpp_mov<0x141, 0xf, true>(a[m]);          // row_half_mirror
    const float hi = a[m + 2] + dpp_mov<0x141, 0xf, true>(a[m + 2]);
    b[m] = b2 ? hi : lo;
  }
  const float lo = b[0] + dpp_mov<0x1B, 0xf, true>(b[0]);             // quad_perm [3,2,1,0]
  const float hi = b[1] + dpp_mov<0x1B, 0xf, true>(b[1]);
  float c = b1 ? hi : lo;
  c += dpp_mov<0xB1, 0xf, true>(c);                                   // quad_perm [1,0,3,2]
  c += __shfl_xor(c, 16, WAVE);
  c += __shfl_xor(c, 32, WAVE);
  return c;
}

// Exclusive prefix sum over a workgroup of NT threads (NT a multiple of 64,
// at most 1024).  `sh` must hold NT/64 + 1 uint32.  Returns the exclusive
// prefix of the calling thread; *total receives the workgroup sum.  Contains
// __syncthreads(): every thread of the workgroup must call it.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  constexpr int NW = NT / WAVE;
  const int lane = lane_id();
  const int w = threadIdx.x / WAVE;
  uint32_t inc = wave_incl_scan(v);
  if (lane == WAVE - 1) sh[w] = inc;
  __syncthreads();
  if (w == 0) {
    uint32_t s = lane < NW ? sh[lane] : 0u;
    uint32_t si = wave_incl_scan(s);
    if (lane < NW) sh[lane] = si - s;
    if (lane == NW - 1) sh[NW] = si;
  }
  __syncthreads();
  uint32_t res = sh[w] + inc - v;
  *total = sh[NW];
  __syncthreads();
  return res;
}

}  // namespace hyrf
