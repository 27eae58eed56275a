// Stable LSD radix sort of (uint32 key, uint32 value) pairs, digits of at
// most 8 bits, reduce-then-scan per pass (no inter-workgroup waiting), three
// launches per pass:
//   1. per-workgroup digit histogram -> hist[digit * nblocks + block]
//      (rows of the digits the pass uses: 2^width of them)
//   2. one workgroup per used digit: exclusive scan of the digit's row of hist
//      over the workgroups, in place, and the row's total -> tot[digit]
//   3. per workgroup: global base of (digit, block) = exclusive sum of the
//      totals of the smaller digits + the scanned hist entry; stable
//      ranking, reorder by digit in LDS, then a write in LDS order:
//      consecutive lanes store consecutive addresses of one digit's run
//      (coalesced), instead of 64 scattered 4-byte stores.
// Each workgroup owns ITEMS consecutive pairs; wave w owns the w-th
// quarter and walks it in 64-item rounds, so the rank of an item among equal
// digits follows input order (stability).
#include "block.h"
#include "kernels.h"

namespace hyrf {

namespace {
constexpr int NT = 256;
constexpr int NW = NT / WAVE;                 // 4 waves
constexpr int RADIX = 256;

template <int ITEMS>
__global__ __launch_bounds__(NT) void k_radix_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                   int shift, uint32_t mask, uint32_t* __restrict__ hist,
                                                   int nblocks) {
  constexpr int ROUNDS = ITEMS / NT;
  __shared__ uint32_t h[RADIX];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * ITEMS;
  uint32_t d[ROUNDS];   // all loads in flight before the first LDS update
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const int64_t i = base + (int64_t)r * NT + threadIdx.x;
    d[r] = i < n ? (keys[i] >> shift) & mask : RADIX;
  }
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r)
    if (d[r] < RADIX) atomicAdd(&h[d[r]], 1u);
  __syncthreads();
  if (threadIdx.x <= mask) hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Workgroup d: hist[d * nblocks + b] <- number of keys with digit d in the
// workgroups below b; tot[d] <- number of keys with digit d.
constexpr int OFF_PER = 4;   // consecutive row entries per thread and chunk
__global__ __launch_bounds__(NT) void k_radix_offsets(uint32_t* __restrict__ hist,
                                                      uint32_t* __restrict__ tot, int nblocks) {
  __shared__ uint32_t sh[NW + 1];
  const int d = blockIdx.x;
  uint32_t carry = 0;
  uint32_t* row = hist + (int64_t)d * nblocks;
  for (int c0 = 0; c0 < nblocks; c0 += NT * OFF_PER) {   // uniform trip count: barriers inside
    const int i0 = c0 + (int)threadIdx.x * OFF_PER;
    uint32_t v[OFF_PER], s = 0;
#pragma unroll
    for (int q = 0; q < OFF_PER; ++q) {
      v[q] = i0 + q < nblocks ? row[i0 + q] : 0u;
      s += v[q];
    }
    uint32_t chunk;
    uint32_t run = carry + block_excl_scan<NT>(s, sh, &chunk);
#pragma unroll
    for (int q = 0; q < OFF_PER; ++q) {
      if (i0 + q < nblocks) row[i0 + q] = run;
      run += v[q];
    }
    carry += chunk;
  }
  if (threadIdx.x == 0) tot[d] = carry;
}

template <int ITEMS>
__global__ __launch_bounds__(NT) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                      const uint32_t* __restrict__ vin,
                                                      uint32_t* __restrict__ kout,
                                                      uint32_t* __restrict__ vout, int64_t n,
                                                      int shift, uint32_t mask,
                                                      const uint32_t* __restrict__ hist,
                                                      const uint32_t* __restrict__ dtot, int nblocks) {
  static_assert(NT == RADIX, "one thread per digit");
  static_assert(ITEMS % NT == 0, "whole rounds of 64 per wave");
  constexpr int ROUNDS = ITEMS / NT;
  __shared__ uint32_t cnt[NW][RADIX];
  __shared__ uint32_t sk[ITEMS], sv[ITEMS];   // the workgroup's pairs, ordered by digit
  __shared__ uint32_t lstart[RADIX], gbase[RADIX];
  __shared__ uint32_t scan_sh[NW + 1];
  const int lane = lane_id();
  const int w = threadIdx.x / WAVE;
  for (int k = threadIdx.x; k < NW * RADIX; k += NT) (&cnt[0][0])[k] = 0;
  __syncthreads();

  const int64_t chunk = (int64_t)blockIdx.x * ITEMS + (int64_t)w * (ROUNDS * WAVE);
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t key[ROUNDS], val[ROUNDS], rank[ROUNDS];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const int64_t i = chunk + (int64_t)r * WAVE + lane;
    const bool ok = i < n;
    uint32_t k = ok ? kin[i] : 0u;
    key[r] = k;
    val[r] = ok ? vin[i] : 0u;
    const uint32_t d = (k >> shift) & mask;
    // lanes holding the same digit (out-of-range lanes form their own group)
    uint64_t m = __ballot(ok);
    if (!ok) m = ~m;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t bb = __ballot((d >> b) & 1u);
      m &= ((d >> b) & 1u) ? bb : ~bb;
    }
    uint32_t before = ok ? cnt[w][d] : 0u;
    rank[r] = before + (uint32_t)__popcll(m & lt);
    const bool leader = (m >> lane) == 1ull;     // highest lane of its group
    if (ok && leader) cnt[w][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  // per digit: prefix over waves, the digit's start in the workgroup's
  // digit order, and the global base of (digit, block)
  {
    const int d = threadIdx.x;
    uint32_t tot = 0;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) {
      const uint32_t c = cnt[ww][d];
      cnt[ww][d] = tot;
      tot += c;
    }
    uint32_t all;
    lstart[d] = block_excl_scan<NT>(tot, scan_sh, &all);
    const bool used = (uint32_t)d <= mask;   // rows of digits the pass cannot produce are not written
    gbase[d] = block_excl_scan<NT>(used ? dtot[d] : 0u, scan_sh, &all) +
               (used ? hist[(int64_t)d * nblocks + blockIdx.x] : 0u);
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const int64_t i = chunk + (int64_t)r * WAVE + lane;
    if (i < n) {
      const uint32_t d = (key[r] >> shift) & mask;
      const uint32_t lp = lstart[d] + cnt[w][d] + rank[r];
      sk[lp] = key[r];
      sv[lp] = val[r];
    }
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * ITEMS;
  const int m = (int)min((int64_t)ITEMS, n - base);
  for (int t = threadIdx.x; t < m; t += NT) {
    const uint32_t k = sk[t];
    const uint32_t d = (k >> shift) & mask;
    const uint32_t pos = gbase[d] + ((uint32_t)t - lstart[d]);
    kout[pos] = k;
    vout[pos] = sv[t];
  }
}
}  // namespace

// Sorts of up to SORT_SMALL_N pairs give each workgroup SORT_ITEMS_SMALL of
// them, so that they still spread over every CU; larger ones SORT_ITEMS.
constexpr int SORT_ITEMS_SMALL = 1024;
constexpr int64_t SORT_SMALL_N = (int64_t)1 << 21;

static int64_t sort_blocks(int64_t n, int items) { return (n + items - 1) / items; }

size_t radix_temp_elems(int64_t n) {
  // enough for any sort of at most n pairs, in either workgroup size
  int64_t nb = sort_blocks(n, SORT_ITEMS);
  const int64_t nb_small = sort_blocks(n < SORT_SMALL_N ? n : SORT_SMALL_N, SORT_ITEMS_SMALL);
  if (nb_small > nb) nb = nb_small;
  if (nb < 1) nb = 1;
  return (size_t)nb * RADIX + RADIX;
}

template <int ITEMS>
static int radix_passes(uint32_t* k[2], uint32_t* v[2], int start, int64_t n, int bits, uint32_t* temp,
                        hipStream_t st) {
  const int nb = (int)sort_blocks(n, ITEMS);
  // as few passes as 8-bit digits need, the bits shared out evenly: fewer
  // distinct digits per pass give longer runs per digit in each workgroup's
  // output, so its stores fill whole lines
  const int passes = (bits + 7) / 8;
  uint32_t* hist = temp;
  uint32_t* tot = temp + (size_t)nb * RADIX;   // [RADIX] digit totals of the pass
  int cur = start, shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int w = bits / passes + (p < bits % passes ? 1 : 0);
    const uint32_t mask = (1u << w) - 1u;
    k_radix_hist<ITEMS><<<nb, NT, 0, st>>>(k[cur], n, shift, mask, hist, nb);
    k_radix_offsets<<<mask + 1, NT, 0, st>>>(hist, tot, nb);
    k_radix_scatter<ITEMS><<<nb, NT, 0, st>>>(k[cur], v[cur], k[cur ^ 1], v[cur ^ 1], n, shift, mask, hist,
                                              tot, nb);
    shift += w;
    cur ^= 1;
  }
  return cur;
}

int radix_sort_pairs(uint32_t* k[2], uint32_t* v[2], int start, int64_t n, int bits,
                     uint32_t* temp, hipStream_t st) {
  if (n <= 1 || bits <= 0) return start;
  if (bits > 32) bits = 32;
  if (n <= SORT_SMALL_N) return radix_passes<SORT_ITEMS_SMALL>(k, v, start, n, bits, temp, st);
  return radix_passes<SORT_ITEMS>(k, v, start, n, bits, temp, st);
}

}  // namespace hyrf
