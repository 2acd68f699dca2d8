// Structural similarity between pairs of rendered images, the measure behind
// the data assignment of Eq. 3 (Sec. 3.2.2): SSIM of Wang et al. (2004) with
// an 11 x 11 Gaussian window of standard deviation 1.5 (normalised, zero
// padding outside the image), C1 = 0.01^2, C2 = 0.03^2, averaged over pixels
// and colour channels.
//
// One work-group per (32 x 32 output tile, image pair): both 42 x 42 input
// patches go to LDS, the horizontal pass writes the five windowed moments
// (x, y, x^2, y^2, xy) of 42 rows x 32 columns to LDS, the vertical pass
// finishes them per output pixel.  FP32 filtering; per-tile sums in FP64 are
// reduced per pair in a fixed order, so the result does not depend on
// scheduling.
#include "gs_common.h"

namespace gs {
namespace {

constexpr int kSsimT = 32;               // output tile side
constexpr int kSsimR = 5;                // window radius
constexpr int kSsimP = kSsimT + 2 * kSsimR;  // patch side (42)
constexpr int kSsimThreads = 256;

__global__ void __launch_bounds__(kSsimThreads) ssim_tile_kernel(const float* __restrict__ images, int64_t n_images,
                                                                 int W, int H, const int32_t* __restrict__ pairs,
                                                                 int tiles_x, double* __restrict__ partial) {
  __shared__ float s_x[kSsimP][kSsimP + 1];
  __shared__ float s_y[kSsimP][kSsimP + 1];
  __shared__ float s_h[5][kSsimP][kSsimT + 1];
  __shared__ float s_w[2 * kSsimR + 1];
  __shared__ double s_red[kSsimThreads / 64];
  const int tile = blockIdx.x, pair = blockIdx.y;
  const int ntiles = gridDim.x;
  const int tx0 = (tile % tiles_x) * kSsimT, ty0 = (tile / tiles_x) * kSsimT;
  if (threadIdx.x == 0) {
    double w[2 * kSsimR + 1], sum = 0.0;
    for (int k = -kSsimR; k <= kSsimR; ++k) {
      w[k + kSsimR] = exp(-(double)(k * k) / (2.0 * 1.5 * 1.5));
      sum += w[k + kSsimR];
    }
    for (int k = 0; k < 2 * kSsimR + 1; ++k) s_w[k] = (float)(w[k] / sum);
  }
  const int64_t ia = pairs[2 * pair], ib = pairs[2 * pair + 1];
  const bool valid = ia >= 0 && ia < n_images && ib >= 0 && ib < n_images;
  const int64_t plane = (int64_t)H * W;
  double acc = 0.0;
  for (int c = 0; c < 3 && valid; ++c) {
    const float* A = images + (ia * 3 + c) * plane;
    const float* Bi = images + (ib * 3 + c) * plane;
    __syncthreads();
    for (int k = threadIdx.x; k < kSsimP * kSsimP; k += kSsimThreads) {
      const int r = k / kSsimP, q = k - r * kSsimP;
      const int gy = ty0 - kSsimR + r, gx = tx0 - kSsimR + q;
      const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H;
      s_x[r][q] = in ? A[(int64_t)gy * W + gx] : 0.0f;
      s_y[r][q] = in ? Bi[(int64_t)gy * W + gx] : 0.0f;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kSsimP * kSsimT; k += kSsimThreads) {
      const int r = k / kSsimT, q = k - r * kSsimT;
      float mx = 0.f, my = 0.f, xx = 0.f, yy = 0.f, xy = 0.f;
#pragma unroll
      for (int t = 0; t < 2 * kSsimR + 1; ++t) {
        const float w = s_w[t], x = s_x[r][q + t], y = s_y[r][q + t];
        mx = fmaf(w, x, mx);
        my = fmaf(w, y, my);
        xx = fmaf(w, x * x, xx);
        yy = fmaf(w, y * y, yy);
        xy = fmaf(w, x * y, xy);
      }
      s_h[0][r][q] = mx;
      s_h[1][r][q] = my;
      s_h[2][r][q] = xx;
      s_h[3][r][q] = yy;
      s_h[4][r][q] = xy;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kSsimT * kSsimT; k += kSsimThreads) {
      const int r = k / kSsimT, q = k - r * kSsimT;
      if (tx0 + q >= W || ty0 + r >= H) continue;
      float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < 2 * kSsimR + 1; ++t) {
        const float w = s_w[t];
#pragma unroll
        for (int u = 0; u < 5; ++u) m[u] = fmaf(w, s_h[u][r + t][q], m[u]);
      }
      const float C1 = 0.01f * 0.01f, C2 = 0.03f * 0.03f;
      const float sxx = m[2] - m[0] * m[0], syy = m[3] - m[1] * m[1], sxy = m[4] - m[0] * m[1];
      const float num = (2.0f * m[0] * m[1] + C1) * (2.0f * sxy + C2);
      const float den = (m[0] * m[0] + m[1] * m[1] + C1) * (sxx + syy + C2);
      acc += (double)(num / den);
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kSsimThreads / 64; ++w) t += s_red[w];
    partial[(int64_t)pair * ntiles + tile] = valid ? t : __builtin_nan("");
  }
}

// per pair: tile sums in index order (fixed tree), divided by the sample count
__global__ void __launch_bounds__(256) ssim_reduce_kernel(const double* __restrict__ partial, int ntiles,
                                                          double count, float* __restrict__ out) {
  __shared__ double s[256];
  const int pair = blockIdx.x;
  double acc = 0.0;
  for (int t = threadIdx.x; t < ntiles; t += 256) acc += partial[(int64_t)pair * ntiles + t];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[pair] = (float)(s[0] / count);
}

}  // namespace
}  // namespace gs

extern "C" size_t gs_ssim_workspace_bytes(int32_t n_pairs, int32_t width, int32_t height) {
  using namespace gs;
  if (n_pairs <= 0 || width <= 0 || height <= 0) return 0;
  const int64_t tiles = (int64_t)((width + kSsimT - 1) / kSsimT) * ((height + kSsimT - 1) / kSsimT);
  return (size_t)(8 * tiles * n_pairs);
}

extern "C" gs_status gs_ssim(const float* images, int32_t n_images, int32_t width, int32_t height,
                             const int32_t* pairs, int32_t n_pairs, float* ssim, void* ws, size_t ws_bytes,
                             void* stream) {
  using namespace gs;
  if (!images || !pairs || !ssim || !ws || n_images <= 0 || n_pairs <= 0 || width <= 0 || height <= 0)
    return GS_ERR_INVALID_ARG;
  if (n_pairs > 65535) return GS_ERR_INVALID_ARG;
  if (ws_bytes < gs_ssim_workspace_bytes(n_pairs, width, height)) return GS_ERR_WORKSPACE;
  const int tiles_x = (width + kSsimT - 1) / kSsimT, tiles_y = (height + kSsimT - 1) / kSsimT;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(ssim_tile_kernel, dim3(tiles_x * tiles_y, n_pairs), dim3(kSsimThreads), 0, s, images,
                     (int64_t)n_images, width, height, pairs, tiles_x, (double*)ws);
  GS_LAUNCH_CHECK();
  hipLaunchKernelGGL(ssim_reduce_kernel, dim3(n_pairs), dim3(256), 0, s, (const double*)ws, tiles_x * tiles_y,
                     3.0 * (double)width * (double)height, ssim);
  GS_LAUNCH_CHECK();
  return GS_OK;
}
