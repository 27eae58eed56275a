// Training loss with its SSIM term (Sec. 3.4 Eq. 12):
//   loss = (1 - lambda) * mean|x - y| + lambda * (1 - mean SSIM(x, y))
// forward and gradient in one pass over the image.  SSIM as Wang et al. 2004
// (Sec. III-B) with the 3DGS settings: 11 x 11 Gaussian window (sigma 1.5),
// C1 = 0.01^2, C2 = 0.03^2, the image extended by zeros outside its frame.
//
// One workgroup per 32 x 32 output tile of one colour plane.  The separable
// window is applied in four register-blocked LDS passes, each thread sliding
// along a run of outputs so that every LDS value it reads serves several
// outputs:
//   B  row sums of (x, y, x^2, y^2, xy) over the tile + 10 px halo rows
//   C  column sums -> local statistics at tile + 5 px; per pixel SSIM S and
//      the three partial derivatives m = (dS/dmu_x, dS/dE[x^2], dS/dE[xy])
//   D  row sums of m over the tile columns
//   E  column sums -> dS_total/dx = (w*m1) + 2x (w*m2) + y (w*m3)
// Loss partial sums go to the workspace per workgroup and are added in a
// fixed order by one workgroup (deterministic).  The image and its target
// are read once from HBM (the halo re-reads of neighbouring tiles hit L2)
// and the gradient is written once: 12 B per pixel.
#include "backward.h"
#include "block.h"

namespace hyrf {

namespace {
constexpr int NT = 256;
constexpr int TS = 32;           // output tile edge
constexpr int RAD = 5;           // window radius
constexpr int RW = TS + 4 * RAD; // 52: input region edge (tile + 10 px halo)
constexpr int SW = TS + 2 * RAD; // 42: statistics region edge (tile + 5 px)
constexpr float C1 = 0.01f * 0.01f;
constexpr float C2 = 0.03f * 0.03f;

// phase work split (256 threads): B 52 rows x 3 runs of 14 columns;
// C 42 columns x 6 runs of 7 rows; D 42 rows x 4 runs of 8 columns;
// E 32 columns x 8 runs of 4 rows.
constexpr int B_RUN = 14, C_RUN = 7, D_RUN = 8, E_RUN = 4;
static_assert(3 * B_RUN == SW && 6 * C_RUN == SW && 4 * D_RUN == TS && 8 * E_RUN == TS, "runs");

struct Win {
  float g[2 * RAD + 1];
};

// 65 KB: two workgroups share a CU.  The inputs are dead once the row sums
// exist, so the derivative maps reuse their space; the row sums of the
// derivative maps reuse the space of the moment row sums.
struct SsimLds {
  union {
    float2 xy[RW][RW];           // A/B: inputs (zero outside the frame)
    float m[3][SW][SW];          // C/D: derivative maps (zero outside the frame)
  };
  union {
    float hs[5][RW][SW];         // B/C: row sums of the five moments
    float hb[3][SW][TS];         // D/E: row sums of the three derivative maps
  };
  float red[2][NT / WAVE];
};

__global__ __launch_bounds__(NT) void k_l1_dssim(const float* __restrict__ img,
                                                 const float* __restrict__ tgt, int W, int H, Win win,
                                                 float coef_l1, float coef_s, float* __restrict__ grad,
                                                 float* __restrict__ part) {
  __shared__ SsimLds sh;
  const int tid = threadIdx.x;
  const int x0 = blockIdx.x * TS, y0 = blockIdx.y * TS;
  const size_t plane = (size_t)blockIdx.z * W * H;
  const float* X = img + plane;
  const float* Y = tgt + plane;

  // A: region rows/cols [-10, 42) around the tile; every load of the thread
  // is issued before the first LDS store
  {
    constexpr int NLOAD = (RW * RW + NT - 1) / NT;
    float2 v[NLOAD];
#pragma unroll
    for (int k = 0; k < NLOAD; ++k) {
      const int i = tid + k * NT;
      const int r = i / RW, c = i - r * RW;
      const int gy = y0 - 2 * RAD + r, gx = x0 - 2 * RAD + c;
      v[k] = make_float2(0.f, 0.f);
      if (i < RW * RW && gy >= 0 && gy < H && gx >= 0 && gx < W) {
        const size_t o = (size_t)gy * W + gx;
        v[k] = make_float2(X[o], Y[o]);
      }
    }
#pragma unroll
    for (int k = 0; k < NLOAD; ++k) {
      const int i = tid + k * NT;
      if (i < RW * RW) sh.xy[i / RW][i % RW] = v[k];
    }
  }
  __syncthreads();

  // B: hs[k][r][h] = sum_t g[t] * moment_k(xy[r][h + t])
  if (tid < RW * 3) {
    const int r = tid / 3, h0 = (tid - r * 3) * B_RUN;
    float acc[5][B_RUN];
#pragma unroll
    for (int j = 0; j < B_RUN; ++j)
#pragma unroll
      for (int k = 0; k < 5; ++k) acc[k][j] = 0.f;
#pragma unroll
    for (int t = 0; t < B_RUN + 2 * RAD; ++t) {
      const float2 v = sh.xy[r][h0 + t];
      const float mo[5] = {v.x, v.y, v.x * v.x, v.y * v.y, v.x * v.y};
#pragma unroll
      for (int j = 0; j < B_RUN; ++j) {
        const int tap = t - j;
        if (tap >= 0 && tap <= 2 * RAD) {
#pragma unroll
          for (int k = 0; k < 5; ++k) acc[k][j] += win.g[tap] * mo[k];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < B_RUN; ++j)
#pragma unroll
      for (int k = 0; k < 5; ++k) sh.hs[k][r][h0 + j] = acc[k][j];
  }
  __syncthreads();

  // C: local statistics at m-row i (image row y0-5+i), m-column h (image
  // column x0-5+h); SSIM and its derivative maps
  float s_sum = 0.f;
  if (tid < SW * 6) {
    const int h = tid % SW, i0 = (tid / SW) * C_RUN;
    float acc[5][C_RUN];
#pragma unroll
    for (int j = 0; j < C_RUN; ++j)
#pragma unroll
      for (int k = 0; k < 5; ++k) acc[k][j] = 0.f;
#pragma unroll
    for (int t = 0; t < C_RUN + 2 * RAD; ++t) {
      float mo[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) mo[k] = sh.hs[k][i0 + t][h];
#pragma unroll
      for (int j = 0; j < C_RUN; ++j) {
        const int tap = t - j;
        if (tap >= 0 && tap <= 2 * RAD) {
#pragma unroll
          for (int k = 0; k < 5; ++k) acc[k][j] += win.g[tap] * mo[k];
        }
      }
    }
    const int gx = x0 - RAD + h;
    const bool col_in = gx >= 0 && gx < W;
    const bool col_inner = h >= RAD && h < RAD + TS;
#pragma unroll
    for (int j = 0; j < C_RUN; ++j) {
      const int i = i0 + j;
      const int gy = y0 - RAD + i;
      float m1 = 0.f, m2 = 0.f, m3 = 0.f;
      if (col_in && gy >= 0 && gy < H) {
        const float mx = acc[0][j], my = acc[1][j];
        const float vx = acc[2][j] - mx * mx, vy = acc[3][j] - my * my, cxy = acc[4][j] - mx * my;
        const float a1 = 2.f * mx * my + C1, a2 = 2.f * cxy + C2;
        const float b1 = mx * mx + my * my + C1, b2 = vx + vy + C2;
        const float ib1 = 1.f / b1, ib2 = 1.f / b2;
        const float S = a1 * a2 * ib1 * ib2;
        if (col_inner && i >= RAD && i < RAD + TS) s_sum += S;
        // partials with (mu_x, var_x, cov) independent, then chained to the
        // raw moments (mu_x, E[x^2], E[xy])
        const float dmu = 2.f * (my * a2 * ib2 - mx * S) * ib1;
        const float dvar = -S * ib2;
        const float dcov = 2.f * a1 * ib1 * ib2;
        m1 = dmu - 2.f * mx * dvar - my * dcov;
        m2 = dvar;
        m3 = dcov;
      }
      sh.m[0][i][h] = m1;
      sh.m[1][i][h] = m2;
      sh.m[2][i][h] = m3;
    }
  }
  __syncthreads();

  // D: hb[k][i][c] = sum_t g[t] * m[k][i][c + t]
  if (tid < SW * 4) {
    const int i = tid >> 2, c0 = (tid & 3) * D_RUN;
    float acc[3][D_RUN];
#pragma unroll
    for (int j = 0; j < D_RUN; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[k][j] = 0.f;
#pragma unroll
    for (int t = 0; t < D_RUN + 2 * RAD; ++t) {
      float mo[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) mo[k] = sh.m[k][i][c0 + t];
#pragma unroll
      for (int j = 0; j < D_RUN; ++j) {
        const int tap = t - j;
        if (tap >= 0 && tap <= 2 * RAD) {
#pragma unroll
          for (int k = 0; k < 3; ++k) acc[k][j] += win.g[tap] * mo[k];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < D_RUN; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) sh.hb[k][i][c0 + j] = acc[k][j];
  }
  __syncthreads();

  // E: gradient at tile pixel (rho, c)
  float l1_sum = 0.f;
  {
    const int c = tid & (TS - 1), r0 = (tid >> 5) * E_RUN;
    float acc[3][E_RUN];
#pragma unroll
    for (int j = 0; j < E_RUN; ++j)
#pragma unroll
      for (int k = 0; k < 3; ++k) acc[k][j] = 0.f;
#pragma unroll
    for (int t = 0; t < E_RUN + 2 * RAD; ++t) {
      float mo[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) mo[k] = sh.hb[k][r0 + t][c];
#pragma unroll
      for (int j = 0; j < E_RUN; ++j) {
        const int tap = t - j;
        if (tap >= 0 && tap <= 2 * RAD) {
#pragma unroll
          for (int k = 0; k < 3; ++k) acc[k][j] += win.g[tap] * mo[k];
        }
      }
    }
    const int gx = x0 + c;
#pragma unroll
    for (int j = 0; j < E_RUN; ++j) {
      const int gy = y0 + r0 + j;
      if (gx < W && gy < H) {
        const size_t o = plane + (size_t)gy * W + gx;
        const float2 v = make_float2(img[o], tgt[o]);
        const float d = v.x - v.y;
        l1_sum += fabsf(d);
        if (grad) {
          const float dS = acc[0][j] + 2.f * v.x * acc[1][j] + v.y * acc[2][j];
          const float sg = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
          grad[o] = coef_l1 * sg - coef_s * dS;
        }
      }
    }
  }

  s_sum = wave_sum_f32(s_sum);
  l1_sum = wave_sum_f32(l1_sum);
  if (lane_id() == 0) {
    sh.red[0][tid / WAVE] = s_sum;
    sh.red[1][tid / WAVE] = l1_sum;
  }
  __syncthreads();
  if (tid == 0) {
    const size_t b = ((size_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[2 * b] = (sh.red[0][0] + sh.red[0][1]) + (sh.red[0][2] + sh.red[0][3]);
    part[2 * b + 1] = (sh.red[1][0] + sh.red[1][1]) + (sh.red[1][2] + sh.red[1][3]);
  }
}

__global__ __launch_bounds__(NT) void k_l1_dssim_final(const float* __restrict__ part, int nb, double inv_n,
                                                       float lambda, float* __restrict__ loss) {
  __shared__ double sh[2][NT];
  double s = 0.0, l = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT) {
    s += (double)part[2 * i];
    l += (double)part[2 * i + 1];
  }
  sh[0][threadIdx.x] = s;
  sh[1][threadIdx.x] = l;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ssim = sh[0][0] * inv_n, l1 = sh[1][0] * inv_n;
    loss[0] = (float)((1.0 - (double)lambda) * l1 + (double)lambda * (1.0 - ssim));
    loss[1] = (float)l1;
    loss[2] = (float)ssim;
  }
}
}  // namespace

size_t l1_dssim_ws_elems(int planes, int H, int W) {
  const size_t nb = (size_t)planes * ((H + TS - 1) / TS) * ((W + TS - 1) / TS);
  return 2 * nb;
}

void launch_l1_dssim(const float* img, const float* target, int planes, int H, int W, float lambda,
                     float* loss, float* grad, float* ws, hipStream_t st) {
  Win win;
  double g[2 * RAD + 1], sum = 0.0;
  for (int t = 0; t <= 2 * RAD; ++t) {
    const double d = t - RAD;
    g[t] = exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += g[t];
  }
  for (int t = 0; t <= 2 * RAD; ++t) win.g[t] = (float)(g[t] / sum);
  const dim3 grid((W + TS - 1) / TS, (H + TS - 1) / TS, planes);
  const double n = (double)planes * H * W;
  const float coef_l1 = (float)((1.0 - lambda) / n), coef_s = (float)(lambda / n);
  k_l1_dssim<<<grid, NT, 0, st>>>(img, target, W, H, win, coef_l1, coef_s, grad, ws);
  const int nb = (int)(grid.x * grid.y * grid.z);
  k_l1_dssim_final<<<1, NT, 0, st>>>(ws, nb, 1.0 / n, lambda, loss);
}

}  // namespace hyrf
