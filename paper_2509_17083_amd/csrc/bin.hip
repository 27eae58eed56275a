// Tile binning with depth ordering.
//
// Instead of sorting (tile | depth) keys of every tile entry, the splats are
// sorted once by their float32 depth (stable, so equal depths keep slot
// order), the entries are then written out in that depth order, and a
// stable sort by the small (view, tile) key groups them per tile while
// keeping depth order inside every tile.  The result equals an ordering of
// entries by (view, tile, depth, slot); the wide sort runs over splats (1M)
// and only a 16-bit sort runs over entries.
#include "bin.h"
#include "block.h"
#include "kernels.h"

namespace hyrf {

// depth keys of every (view, slot); slots without tiles sort last
__global__ __launch_bounds__(256) void k_depth_keys(const float* __restrict__ depth,
                                                    const int4* __restrict__ rect,
                                                    const int32_t* __restrict__ count, int n_max,
                                                    int64_t m, uint32_t* __restrict__ key,
                                                    uint32_t* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  const int slot = (int)(i % n_max);
  uint32_t k = 0xFFFFFFFFu;
  if (slot < *count) {
    const int4 r = rect[i];
    if (r.z > r.x && r.w > r.y) k = __float_as_uint(depth[i]);
  }
  key[i] = k;
  val[i] = (uint32_t)i;
}

// number of tile entries of the splat at each depth-sorted position, and its
// rectangle stored in depth order (one random gather here; the entry
// expansion then reads the rectangles in order)
__global__ __launch_bounds__(256) void k_tile_counts(const uint32_t* __restrict__ skey,
                                                     const uint32_t* __restrict__ sval,
                                                     const int4* __restrict__ rect, int64_t m,
                                                     uint32_t* __restrict__ cnt, int4* __restrict__ srect) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= m) return;
  int4 r = make_int4(0, 0, 0, 0);
  if (skey[i] != 0xFFFFFFFFu) r = rect[sval[i]];
  cnt[i] = (uint32_t)((r.z - r.x) * (r.w - r.y));
  srect[i] = r;
}

// write the entries of each splat in depth order: key = view*tiles + tile.
// A wave expands the entries of its 64 consecutive splats together: their
// exclusive offsets are consecutive, so lane e of each step writes entry
// first + e, found by a binary search over the wave's offsets (coalesced
// stores, large splats spread over all lanes).
__global__ __launch_bounds__(256) void k_dup(const uint32_t* __restrict__ skey,
                                             const uint32_t* __restrict__ sval,
                                             const int4* __restrict__ srect,
                                             const uint32_t* __restrict__ off, int64_t m, int n_max,
                                             int tiles_x, int tiles, int64_t capacity,
                                             uint32_t* __restrict__ ekey, uint32_t* __restrict__ eval) {
  __shared__ uint32_t s_off[4][WAVE];
  __shared__ int4 s_rect[4][WAVE];
  __shared__ uint32_t s_id[4][WAVE];
  const int lane = lane_id();
  const int w = threadIdx.x / WAVE;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i0 = i - lane;                    // the wave's first splat
  if (i0 >= m) return;                            // whole wave idle (uniform)
  const bool ok = i < m && skey[i] != 0xFFFFFFFFu;
  const uint32_t id = ok ? sval[i] : 0u;
  const int4 r = ok ? srect[i] : make_int4(0, 0, 0, 0);
  const uint32_t cnt = ok ? (uint32_t)((r.z - r.x) * (r.w - r.y)) : 0u;
  const uint32_t first = off[i0];
  const uint32_t rel = i < m ? off[i] - first : 0u;
  // entries of the wave: the end of its last in-range splat (offsets plus
  // counts do not decrease along the array)
  const int last = (int)min((int64_t)WAVE - 1, m - 1 - i0);
  const uint32_t total = __shfl(rel + cnt, last, WAVE);
  // lanes past the array sit at the end, so the offsets stay sorted
  s_off[w][lane] = i < m ? rel : total;
  s_rect[w][lane] = r;
  s_id[w][lane] = id;
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
  for (uint32_t e = lane; e < total; e += WAVE) {
    // the splat j with s_off[j] <= e < s_off[j + 1] (empty splats skipped)
    int lo = 0, hi = WAVE - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_off[w][mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int4 rr = s_rect[w][lo];
    const uint32_t k = e - s_off[w][lo];
    const int wdt = rr.z - rr.x;
    const int ty = rr.y + (int)(k / (uint32_t)wdt), tx = rr.x + (int)(k % (uint32_t)wdt);
    const uint32_t sid = s_id[w][lo];
    const int64_t o = (int64_t)first + e;
    if (o < capacity) {
      ekey[o] = (sid / (uint32_t)n_max) * (uint32_t)tiles + (uint32_t)(ty * tiles_x + tx);
      eval[o] = sid;
    }
  }
}

// Per-key [first, last) of the sorted keys: entry e opens its key's range
// where key[e - 1] differs and closes it where key[e + 1] differs.  Each
// thread takes RANGE_PER consecutive entries (one 16-byte load when the
// group is whole and the keys are 16-byte aligned) and their two outer
// neighbours.
constexpr int RANGE_PER = 4;
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ key, int64_t ne,
                                                uint32_t nkeys, uint32_t* __restrict__ ranges) {
  const int64_t e0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * RANGE_PER;
  if (e0 >= ne) return;
  uint32_t k[RANGE_PER + 2];   // key[e0 - 1 .. e0 + RANGE_PER]; out-of-range neighbours differ
  if (e0 + RANGE_PER <= ne && ((uintptr_t)key & 15) == 0) {
    const uint4 q = *reinterpret_cast<const uint4*>(key + e0);
    k[1] = q.x; k[2] = q.y; k[3] = q.z; k[4] = q.w;
  } else {
#pragma unroll
    for (int j = 0; j < RANGE_PER; ++j) k[1 + j] = e0 + j < ne ? key[e0 + j] : 0xFFFFFFFFu;
  }
  k[0] = e0 > 0 ? key[e0 - 1] : ~k[1];
  k[RANGE_PER + 1] = e0 + RANGE_PER < ne ? key[e0 + RANGE_PER] : ~k[RANGE_PER];
#pragma unroll
  for (int j = 0; j < RANGE_PER; ++j) {
    const int64_t e = e0 + j;
    const uint32_t kk = k[1 + j];
    if (e >= ne || kk >= nkeys) continue;   // kk >= nkeys: n_entries disagrees with the device total
    if (k[j] != kk) ranges[2 * (size_t)kk] = (uint32_t)e;
    if (e == ne - 1 || k[2 + j] != kk) ranges[2 * (size_t)kk + 1] = (uint32_t)(e + 1);
  }
}

__global__ __launch_bounds__(256) void k_zero_words(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

static unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

BinWs carve_bin_ws(void* ws, int V, int n_max, int64_t capacity, int tiles_total) {
  Carve c(ws);
  BinWs w;
  const int64_t m = (int64_t)V * n_max;
  w.dk[0] = c.take<uint32_t>(m);
  w.dk[1] = c.take<uint32_t>(m);
  w.dv[0] = c.take<uint32_t>(m);
  w.dv[1] = c.take<uint32_t>(m);
  w.cnt = c.take<uint32_t>(m);
  w.srect = c.take<int4>(m);
  w.ek[0] = c.take<uint32_t>(capacity > 0 ? capacity : 1);
  w.ek[1] = c.take<uint32_t>(capacity > 0 ? capacity : 1);
  w.ev = c.take<uint32_t>(capacity > 0 ? capacity : 1);
  int64_t big = m > capacity ? m : capacity;
  w.temp = c.take<uint32_t>(radix_temp_elems(big) + scan_temp_elems(m));
  w.bytes = c.off;
  (void)tiles_total;
  return w;
}

int key_bits_for(int64_t nkeys) {
  int b = 0;
  while (((int64_t)1 << b) < nkeys) ++b;
  return b;
}

void launch_bin_sort(const BinArgs& a, const BinWs& w, hipStream_t st) {
  const int64_t m = (int64_t)a.V * a.n_max;
  const int tiles = a.tiles_x * a.tiles_y;
  const int64_t nranges = 2 * (int64_t)a.V * tiles;
  // 1. depth order of all splats (stable)
  k_depth_keys<<<nblk(m), 256, 0, st>>>(a.depth, reinterpret_cast<const int4*>(a.rect), a.count,
                                        a.n_max, m, w.dk[0], w.dv[0]);
  uint32_t* dk[2] = {w.dk[0], w.dk[1]};
  uint32_t* dv[2] = {w.dv[0], w.dv[1]};
  const int dcur = radix_sort_pairs(dk, dv, 0, m, 32, w.temp, st);
  // 2. entry offsets in depth order
  k_tile_counts<<<nblk(m), 256, 0, st>>>(dk[dcur], dv[dcur], reinterpret_cast<const int4*>(a.rect), m, w.cnt,
                                         w.srect);
  scan_exclusive_u32(w.cnt, w.cnt, m, w.temp, nullptr, st);
  // 3. entries, then a stable sort by (view, tile)
  const int bits = key_bits_for((int64_t)a.V * tiles);
  const int passes = (bits + 7) / 8;
  uint32_t* K[2] = {w.ek[0], a.keys ? a.keys : w.ek[1]};
  uint32_t* Vv[2] = {w.ev, a.vals};
  const int start = (passes & 1) ? 0 : 1;
  k_dup<<<nblk(m), 256, 0, st>>>(dk[dcur], dv[dcur], w.srect, w.cnt, m,
                                 a.n_max, a.tiles_x, tiles, a.n_entries, K[start], Vv[start]);
  const int ecur = radix_sort_pairs(K, Vv, start, a.n_entries, bits, w.temp, st);
  // 4. per-tile ranges
  k_zero_words<<<nblk(nranges), 256, 0, st>>>(a.ranges, nranges);
  if (a.n_entries > 0)
    k_ranges<<<nblk((a.n_entries + RANGE_PER - 1) / RANGE_PER), 256, 0, st>>>(K[ecur], a.n_entries,
                                                                           (uint32_t)(a.V * tiles), a.ranges);
}

}  // namespace hyrf
