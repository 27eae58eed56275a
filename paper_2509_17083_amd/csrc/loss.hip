// L1 photometric term of the training loss (Sec. 3.4 Eq. 12) and its
// gradient.  Deterministic: per-workgroup partial sums, then one workgroup
// adds them in a fixed order.
#include "backward.h"
#include "block.h"

namespace hyrf {

namespace {
constexpr int NT = 256;
constexpr int PER_BLOCK = NT * 16;

__global__ __launch_bounds__(NT) void k_l1_partial(const float* __restrict__ img,
                                                   const float* __restrict__ tgt, int64_t n,
                                                   float inv_n, float* __restrict__ grad,
                                                   float* __restrict__ part) {
  __shared__ float sh[NT / WAVE];
  const int64_t base = (int64_t)blockIdx.x * PER_BLOCK;
  float s = 0.f;
#pragma unroll 4
  for (int k = 0; k < 16; ++k) {
    const int64_t i = base + (int64_t)k * NT + threadIdx.x;
    if (i < n) {
      const float d = img[i] - tgt[i];
      s += fabsf(d);
      if (grad) grad[i] = d > 0.f ? inv_n : (d < 0.f ? -inv_n : 0.f);
    }
  }
  s = wave_sum_f32(s);
  if (lane_id() == 0) sh[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ __launch_bounds__(NT) void k_l1_final(const float* __restrict__ part, int nb, float inv_n,
                                                 float* __restrict__ loss) {
  __shared__ float sh[NT / WAVE];
  float s = 0.f;
  for (int i = threadIdx.x; i < nb; i += NT) s += part[i];
  s = wave_sum_f32(s);
  if (lane_id() == 0) sh[threadIdx.x / WAVE] = s;
  __syncthreads();
  if (threadIdx.x == 0) *loss = ((sh[0] + sh[1]) + (sh[2] + sh[3])) * inv_n;
}
}  // namespace

size_t l1_ws_elems(int64_t n) { return (size_t)((n + PER_BLOCK - 1) / PER_BLOCK) + 1; }

void launch_l1(const float* img, const float* target, int64_t n, float* loss, float* grad, float* ws,
               hipStream_t st) {
  const int nb = (int)((n + PER_BLOCK - 1) / PER_BLOCK);
  const float inv_n = (float)(1.0 / (double)n);
  k_l1_partial<<<nb, NT, 0, st>>>(img, target, n, inv_n, grad, ws);
  k_l1_final<<<1, NT, 0, st>>>(ws, nb, inv_n, loss);
}

}  // namespace hyrf
