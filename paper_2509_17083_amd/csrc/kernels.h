// Host-side launch helpers shared between the kernel translation units and
// the C ABI (internal; not exported).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "internal.h"

namespace hyrf {

// Carves 256-byte aligned chunks out of a caller workspace; with base == NULL
// it only measures.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// ---- scan.hip
constexpr int SCAN_ITEMS = 4096;   // items per workgroup
size_t scan_temp_elems(int64_t n);
// Exclusive prefix sum of n uint32 values (in may equal out); temp holds
// scan_temp_elems(n) uint32; total (device, may be NULL) receives the sum.
void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* temp,
                        uint32_t* total, hipStream_t s);

// ---- sort.hip
constexpr int SORT_ITEMS = 4096;   // items per workgroup and pass
size_t radix_temp_elems(int64_t n);
// Stable LSD radix sort of (key, value) pairs by key bits [0, bits) (the
// other bits must be zero), ceil(bits / 8) passes sharing the bits evenly,
// ping-ponging between (k[0], v[0]) and (k[1], v[1]); the input is in slot
// `start`; returns the slot that holds the result.
int radix_sort_pairs(uint32_t* k[2], uint32_t* v[2], int start, int64_t n, int bits,
                     uint32_t* temp, hipStream_t s);

// ---- order.hip
size_t order_ws_bytes(int n);
hipError_t launch_order(const float* pos, int n, const GridP& g, uint32_t* perm, void* ws, hipStream_t st);

// ---- quant.hip
size_t quant_ws_elems(int levels, int log2_T);
void launch_quantize(const float* table, int levels, int log2_T, uint8_t* codes, float* qparams, float* ws,
                     hipStream_t st);

// ---- train.hip
// returns non-zero when the total work does not fit one launch
int adam_launch(const hyrf_adam_group* groups, int n_groups, int step, float b1, float b2, float eps,
                int zero_grad, hipStream_t st);
void launch_densify_masks(int n, int n_max, const int32_t* vis_count, const int32_t* vis_idx,
                          const float* opacity, const float* scale, const float* accum, const float* count,
                          float thr, float extent, float min_op, uint8_t* flags, hipStream_t st);
void launch_reset_opacity(float* opac_e, int n, float value, hipStream_t st);

}  // namespace hyrf
