// Block-wise level-of-detail selection and aggregation (Sec. 3.3.2 of the paper).
//
// One work-group handles every (view, block) pair: the work is O(V * B) (a few
// thousand pairs at most), so a single launch with an in-LDS scan beats any
// multi-kernel scheme.  All geometry is FP64 in a fixed operation order (this
// file is compiled with -ffp-contract=off) so the chosen levels are
// reproducible bit for bit.
#include "gs_common.h"

namespace gs {
namespace {

constexpr int kLodThreads = 1024;
constexpr int kMaxLevels = 8;

struct LodArgs {
  const double* lo;
  const double* hi;
  const double* cell;
  const double* contraction;  // NULL, or p_min[3], p_max[3] of a contracted partition
  const int64_t* lvl_cnt;
  const int32_t* exclude;  // kExcludeMode: per view, the block left out (-1: none)
  int32_t B, L, V, mode;
  double thr[kMaxLevels - 1];
};

constexpr int32_t kExcludeMode = 100;  // internal mode of gs_lod_select_exclude

// camera centre of a view
__device__ __forceinline__ void cam_centre(const gs_camera& cam, double& C0, double& C1, double& C2) {
  const double* R = cam.R;
  const double* t = cam.t;
  C0 = -((R[0] * t[0] + R[3] * t[1]) + R[6] * t[2]);
  C1 = -((R[1] * t[0] + R[4] * t[1]) + R[7] * t[2]);
  C2 = -((R[2] * t[0] + R[5] * t[1]) + R[8] * t[2]);
}

// The camera centre in the coordinates of the block cells: world x, y, or,
// with a contracted partition, normalised and contracted (Eq. 2) exactly as a
// Gaussian centre is when it is assigned to a block
__device__ __forceinline__ void cell_coords(const double* pc, double C0, double C1, double C2, double& X, double& Y) {
  X = C0;
  Y = C1;
  if (!pc) return;
  const double q0 = (2.0 * (C0 - pc[0])) / (pc[3] - pc[0]) - 1.0;
  const double q1 = (2.0 * (C1 - pc[1])) / (pc[4] - pc[1]) - 1.0;
  const double q2 = (2.0 * (C2 - pc[2])) / (pc[5] - pc[2]) - 1.0;
  const double m0 = fabs(q0), m1 = fabs(q1), m2 = fabs(q2);
  const bool nan = !(m0 == m0) || !(m1 == m1) || !(m2 == m2);
  double nrm = m0 > m1 ? m0 : m1;
  nrm = m2 > nrm ? m2 : nrm;
  X = q0;
  Y = q1;
  if (!nan && nrm > 1.0) {
    const double sc = 2.0 - 1.0 / nrm;
    X = sc * (q0 / nrm);
    Y = sc * (q1 / nrm);
  }
}

__device__ __forceinline__ bool in_cell(const double* cl, double X, double Y) {
  return (cl[0] <= X) && (X < cl[1]) && (cl[2] <= Y) && (Y < cl[3]);
}

__device__ int select_level(const LodArgs& a, const gs_camera& cam, int v, int b) {
  if (a.mode == GS_LOD_ALL_FINEST) return a.L - 1;
  if (a.mode == kExcludeMode) return b == a.exclude[v] ? -1 : a.L - 1;
  const double* lo = a.lo + 3 * b;
  const double* hi = a.hi + 3 * b;
  if (!(lo[0] <= hi[0])) return -1;  // empty block
  const double* R = cam.R;
  const double* t = cam.t;
  // camera centre C = -R^T t
  const double C0 = -((R[0] * t[0] + R[3] * t[1]) + R[6] * t[2]);
  const double C1 = -((R[1] * t[0] + R[4] * t[1]) + R[7] * t[2]);
  const double C2 = -((R[2] * t[0] + R[5] * t[1]) + R[8] * t[2]);
  double dmin2 = __builtin_inf();
  double umin = __builtin_inf(), vmin = __builtin_inf();
  double umax = -__builtin_inf(), vmax = -__builtin_inf();
  int nfront = 0;
  for (int c = 0; c < 8; ++c) {
    const double p0 = (c & 1) ? hi[0] : lo[0];
    const double p1 = (c & 2) ? hi[1] : lo[1];
    const double p2 = (c & 4) ? hi[2] : lo[2];
    const double e0 = p0 - C0, e1 = p1 - C1, e2 = p2 - C2;
    const double d2 = (e0 * e0 + e1 * e1) + e2 * e2;
    dmin2 = d2 < dmin2 ? d2 : dmin2;
    const double zc = ((R[6] * p0 + R[7] * p1) + R[8] * p2) + t[2];
    if (zc > cam.znear) {
      const double xc = ((R[0] * p0 + R[1] * p1) + R[2] * p2) + t[0];
      const double yc = ((R[3] * p0 + R[4] * p1) + R[5] * p2) + t[1];
      const double rz = 1.0 / zc;
      const double u = cam.fx * (xc * rz) + cam.cx;
      const double v = cam.fy * (yc * rz) + cam.cy;
      umin = u < umin ? u : umin;
      umax = u > umax ? u : umax;
      vmin = v < vmin ? v : vmin;
      vmax = v > vmax ? v : vmax;
      ++nfront;
    }
  }
  bool visible = false;
  if (nfront > 0) {
    // IoU with the screen > 0  <=>  the intersection has positive area
    const double W = (double)cam.width, H = (double)cam.height;
    const double ix1 = umax < W ? umax : W, ix0 = umin > 0.0 ? umin : 0.0;
    const double iy1 = vmax < H ? vmax : H, iy0 = vmin > 0.0 ? vmin : 0.0;
    visible = (ix1 > ix0) && (iy1 > iy0);
  }
  // the block whose cell holds the camera centre (Sec. 3.3.2), taken in the
  // contracted space of the partition when there is one
  double X, Y;
  cell_coords(a.contraction, C0, C1, C2, X, Y);
  const bool cam_in_cell = in_cell(a.cell + 4 * b, X, Y);
  if (!(visible || cam_in_cell)) return -1;
  int level = a.L - 1;
  for (int k = 0; k < a.L - 1; ++k)
    if (dmin2 >= a.thr[k] * a.thr[k]) --level;
  return level;
}

__global__ void __launch_bounds__(kLodThreads) lod_select_kernel(LodArgs a, const gs_camera* __restrict__ cams,
                                                                 int8_t* __restrict__ level_out,
                                                                 int64_t* __restrict__ offsets,
                                                                 int64_t* __restrict__ counts) {
  __shared__ int64_t wave_sums[kLodThreads / 64];
  __shared__ int64_t carry;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  if (tid == 0) carry = 0;
  __syncthreads();
  const int64_t total_pairs = (int64_t)a.V * a.B;
  for (int64_t base = 0; base < total_pairs; base += kLodThreads) {
    const int64_t p = base + tid;
    int64_t cnt = 0;
    if (p < total_pairs) {
      const int v = (int)(p / a.B), b = (int)(p % a.B);
      const int lv = select_level(a, cams[v], v, b);
      level_out[p] = (int8_t)lv;
      cnt = lv >= 0 ? a.lvl_cnt[(int64_t)b * a.L + lv] : 0;
    }
    // block-wide exclusive scan of cnt
    int64_t x = cnt;
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wave_sums[wid] = x;
    __syncthreads();
    if (wid == 0) {
      int64_t s = lane < kLodThreads / 64 ? wave_sums[lane] : 0;
      for (int off = 1; off < 64; off <<= 1) {
        const int64_t y = __shfl_up(s, off, 64);
        if (lane >= off) s += y;
      }
      if (lane < kLodThreads / 64) wave_sums[lane] = s;  // inclusive over waves
    }
    __syncthreads();
    const int64_t wave_excl = wid > 0 ? wave_sums[wid - 1] : 0;
    const int64_t incl = carry + wave_excl + x;
    if (p < total_pairs) offsets[p] = incl - cnt;
    __syncthreads();
    if (tid == kLodThreads - 1) carry = incl;
    __syncthreads();
  }
  if (tid == 0) {
    offsets[total_pairs] = carry;
    counts[GS_COUNT_RECORDS] = carry;
    counts[GS_COUNT_VISIBLE] = 0;
    counts[GS_COUNT_PAIRS] = 0;
    counts[GS_COUNT_FLAGS] = 0;
  }
}

// records of each selection segment that survived the cull (tiles_touched > 0)
__global__ void __launch_bounds__(256) segment_visible_kernel(const int32_t* __restrict__ tiles_touched,
                                                             const int64_t* __restrict__ offsets, int32_t n_seg,
                                                             int64_t capacity, int32_t* __restrict__ visible) {
  __shared__ int32_t s_sum[4];
  for (int p = blockIdx.x; p < n_seg; p += gridDim.x) {
    int64_t lo = offsets[p], hi = offsets[p + 1];
    hi = hi < capacity ? hi : capacity;
    int32_t c = 0;
    for (int64_t g = lo + threadIdx.x; g < hi; g += blockDim.x) c += tiles_touched[g] > 0 ? 1 : 0;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) visible[p] = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
    __syncthreads();
  }
}

// Eqs. 3-5: B1 = (1 - SSIM) > eps, B2 = the camera centre lies in the block's cell, B = B1 or B2
__global__ void assign_kernel(const double* __restrict__ cell, const double* __restrict__ contraction, int32_t B,
                              const gs_camera* __restrict__ cams, int32_t P, const float* __restrict__ ssim,
                              double eps, uint8_t* __restrict__ b1, uint8_t* __restrict__ b2,
                              uint8_t* __restrict__ b) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (int64_t)P * B) return;
  const int p = (int)(k / B), j = (int)(k - (int64_t)p * B);
  double C0, C1, C2, X, Y;
  cam_centre(cams[p], C0, C1, C2);
  cell_coords(contraction, C0, C1, C2, X, Y);
  const bool a2 = in_cell(cell + 4 * j, X, Y);
  const bool a1 = (1.0 - (double)ssim[k]) > eps;
  if (b1) b1[k] = a1;
  if (b2) b2[k] = a2;
  b[k] = a1 || a2;
}

}  // namespace
}  // namespace gs

extern "C" gs_status gs_lod_select(const gs_blocks* blocks, const double* thresholds, int32_t mode,
                                   const gs_camera* cams, int32_t n_views, int8_t* level, int64_t* offsets,
                                   int64_t* counts, void* stream) {
  using namespace gs;
  if (!blocks || !cams || !level || !offsets || !counts || n_views <= 0) return GS_ERR_INVALID_ARG;
  if (blocks->n_blocks <= 0 || blocks->n_levels <= 0 || blocks->n_levels > kMaxLevels) return GS_ERR_INVALID_ARG;
  if (mode != GS_LOD_BLOCKWISE && mode != GS_LOD_ALL_FINEST) return GS_ERR_INVALID_ARG;
  if (!blocks->lvl_cnt) return GS_ERR_INVALID_ARG;
  if (mode == GS_LOD_BLOCKWISE && (!blocks->lo || !blocks->hi || !blocks->cell)) return GS_ERR_INVALID_ARG;
  LodArgs a{};
  a.lo = blocks->lo;
  a.hi = blocks->hi;
  a.cell = blocks->cell;
  a.contraction = blocks->contraction;
  a.lvl_cnt = blocks->lvl_cnt;
  a.B = blocks->n_blocks;
  a.L = blocks->n_levels;
  a.V = n_views;
  a.mode = mode;
  for (int k = 0; k < a.L - 1; ++k) {
    if (mode == GS_LOD_BLOCKWISE) {
      if (!thresholds) return GS_ERR_INVALID_ARG;
      if (!(thresholds[k] >= 0.0)) return GS_ERR_INVALID_ARG;
      if (k > 0 && !(thresholds[k] >= thresholds[k - 1])) return GS_ERR_INVALID_ARG;
      a.thr[k] = thresholds[k];
    } else {
      a.thr[k] = 0.0;
    }
  }
  hipLaunchKernelGGL(lod_select_kernel, dim3(1), dim3(kLodThreads), 0, (hipStream_t)stream, a, cams, level,
                     offsets, counts);
  GS_LAUNCH_CHECK();
  return GS_OK;
}

extern "C" gs_status gs_lod_select_exclude(const gs_blocks* blocks, const gs_camera* cams, int32_t n_views,
                                           const int32_t* exclude, int8_t* level, int64_t* offsets, int64_t* counts,
                                           void* stream) {
  using namespace gs;
  if (!blocks || !cams || !exclude || !level || !offsets || !counts || n_views <= 0) return GS_ERR_INVALID_ARG;
  if (blocks->n_blocks <= 0 || blocks->n_levels <= 0 || blocks->n_levels > kMaxLevels || !blocks->lvl_cnt)
    return GS_ERR_INVALID_ARG;
  LodArgs a{};
  a.lvl_cnt = blocks->lvl_cnt;
  a.exclude = exclude;
  a.B = blocks->n_blocks;
  a.L = blocks->n_levels;
  a.V = n_views;
  a.mode = kExcludeMode;
  hipLaunchKernelGGL(lod_select_kernel, dim3(1), dim3(kLodThreads), 0, (hipStream_t)stream, a, cams, level,
                     offsets, counts);
  GS_LAUNCH_CHECK();
  return GS_OK;
}

extern "C" gs_status gs_segment_visible(const int32_t* tiles_touched, const int64_t* offsets, int32_t n_segments,
                                        int64_t record_capacity, int32_t* visible, void* stream) {
  using namespace gs;
  if (!offsets || !visible || n_segments <= 0 || record_capacity < 0 || (record_capacity > 0 && !tiles_touched))
    return GS_ERR_INVALID_ARG;
  const int grid = n_segments < 4096 ? n_segments : 4096;
  hipLaunchKernelGGL(segment_visible_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, tiles_touched, offsets,
                     n_segments, record_capacity, visible);
  GS_LAUNCH_CHECK();
  return GS_OK;
}

extern "C" gs_status gs_assign(const gs_blocks* blocks, const gs_camera* cams, int32_t n_poses, const float* ssim,
                               double eps, uint8_t* b1, uint8_t* b2, uint8_t* b, void* stream) {
  using namespace gs;
  if (!blocks || !blocks->cell || !cams || !ssim || !b || n_poses <= 0 || blocks->n_blocks <= 0)
    return GS_ERR_INVALID_ARG;
  const int64_t n = (int64_t)n_poses * blocks->n_blocks;
  hipLaunchKernelGGL(assign_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     blocks->cell, blocks->contraction, blocks->n_blocks, cams, n_poses, ssim, eps, b1, b2, b);
  GS_LAUNCH_CHECK();
  return GS_OK;
}

// ---------------------------------------------------------------------------
// Block bounds of Eq. 6 (median absolute deviation box), one work-group per
// (block, axis).  Medians are exact order statistics found by radix selection:
// the f32 centres are mapped to order-preserving u32 keys (4 passes of 8 bits),
// the FP64 absolute deviations, all non-negative, to their u64 bit patterns
// (8 passes).  Every pass re-reads the block's centres; this is a one-off setup
// step per scene.
// ---------------------------------------------------------------------------
namespace gs {
namespace {

constexpr int kMadThreads = 1024;

__device__ __forceinline__ uint32_t f32_order_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Histogram of digit `shift` among keys whose bits above `shift + 8` equal
// `prefix`; returns (in s_sel) the digit holding rank k and the rank inside it.
template <class KeyFn>
__device__ void select_digit(KeyFn key_of, int64_t n, uint64_t prefix, int shift, int64_t& k, uint32_t* s_hist,
                             uint64_t* s_out) {
  for (int d = threadIdx.x; d < 256; d += blockDim.x) s_hist[d] = 0u;
  __syncthreads();
  const int hs = shift + 8;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const uint64_t key = key_of(e);
    const bool match = hs >= 64 ? true : ((key >> hs) == (prefix >> hs));
    if (match) atomicAdd(&s_hist[(key >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    int d = 0;
    for (; d < 256; ++d) {
      if (acc + (int64_t)s_hist[d] > k) break;
      acc += s_hist[d];
    }
    s_out[0] = (uint64_t)d;
    s_out[1] = (uint64_t)(k - acc);
  }
  __syncthreads();
  const uint64_t d = s_out[0];
  k = (int64_t)s_out[1];
  __syncthreads();
  (void)d;
}

__global__ void __launch_bounds__(kMadThreads) mad_kernel(const float* __restrict__ means, int64_t n_total,
                                                          const int64_t* __restrict__ lvl_off,
                                                          const int64_t* __restrict__ lvl_cnt, int L, double n_mad,
                                                          double* __restrict__ lo_out, double* __restrict__ hi_out) {
  __shared__ uint32_t s_hist[256];
  __shared__ uint64_t s_out[2];
  __shared__ float s_minmax[2][kMadThreads / 64];
  const int b = blockIdx.x / 3, ax = blockIdx.x % 3;
  const int64_t off = lvl_off[(int64_t)b * L + (L - 1)];
  const int64_t n = lvl_cnt[(int64_t)b * L + (L - 1)];
  if (n <= 0) {
    if (threadIdx.x == 0) {
      lo_out[3 * b + ax] = __builtin_inf();
      hi_out[3 * b + ax] = -__builtin_inf();
    }
    return;
  }
  const float* x = means + (int64_t)ax * n_total + off;
  // min and max
  float mn = __builtin_inff(), mx = -__builtin_inff();
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const float v = x[e];
    mn = v < mn ? v : mn;
    mx = v > mx ? v : mx;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const float a = __shfl_xor(mn, o, 64), c = __shfl_xor(mx, o, 64);
    mn = a < mn ? a : mn;
    mx = c > mx ? c : mx;
  }
  if ((threadIdx.x & 63) == 0) {
    s_minmax[0][threadIdx.x >> 6] = mn;
    s_minmax[1][threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  mn = s_minmax[0][0];
  mx = s_minmax[1][0];
  for (int w = 1; w < kMadThreads / 64; ++w) {
    mn = s_minmax[0][w] < mn ? s_minmax[0][w] : mn;
    mx = s_minmax[1][w] > mx ? s_minmax[1][w] : mx;
  }
  const int64_t rank = (n - 1) / 2;  // lower median
  // median of the f32 centres
  int64_t k = rank;
  uint64_t prefix = 0;
  auto key32 = [&](int64_t e) { return (uint64_t)f32_order_key(x[e]); };
  for (int shift = 24; shift >= 0; shift -= 8) {
    select_digit(key32, n, prefix, shift, k, s_hist, s_out);
    prefix |= s_out[0] << shift;
    __syncthreads();
  }
  const uint32_t mk = (uint32_t)prefix;
  const uint32_t mu = (mk & 0x80000000u) ? (mk & 0x7FFFFFFFu) : ~mk;
  const double med = (double)__uint_as_float(mu);
  // MAD: median of |x - med| in FP64 (exact for f32 inputs of similar magnitude)
  k = rank;
  prefix = 0;
  auto key64 = [&](int64_t e) {
    const double dv = fabs((double)x[e] - med);
    return (uint64_t)__double_as_longlong(dv);
  };
  for (int shift = 56; shift >= 0; shift -= 8) {
    select_digit(key64, n, prefix, shift, k, s_hist, s_out);
    prefix |= s_out[0] << shift;
    __syncthreads();
  }
  const double mad = __longlong_as_double((long long)prefix);
  if (threadIdx.x == 0) {
    const double lo = med - n_mad * mad, hi = med + n_mad * mad;
    const double fmn = (double)mn, fmx = (double)mx;
    lo_out[3 * b + ax] = fmn < lo ? lo : fmn;
    hi_out[3 * b + ax] = fmx > hi ? hi : fmx;
  }
}

}  // namespace
}  // namespace gs

extern "C" size_t gs_mad_workspace_bytes(int64_t max_block_count) {
  (void)max_block_count;
  return 256;
}

extern "C" gs_status gs_mad_bounds(const gs_gaussians* finest, const int64_t* lvl_off, const int64_t* lvl_cnt,
                                   int32_t n_blocks, int32_t n_levels, int64_t max_block_count, double n_mad,
                                   double* lo, double* hi, void* ws, size_t ws_bytes, void* stream) {
  using namespace gs;
  if (!finest || !lvl_off || !lvl_cnt || !lo || !hi || n_blocks <= 0 || n_levels <= 0) return GS_ERR_INVALID_ARG;
  if (finest->n > 0 && !finest->means) return GS_ERR_INVALID_ARG;
  if (!(n_mad >= 0.0) || max_block_count < 0) return GS_ERR_INVALID_ARG;
  if (ws_bytes < gs_mad_workspace_bytes(max_block_count) || !ws) return GS_ERR_WORKSPACE;
  if ((int64_t)n_blocks * 3 >= ((int64_t)1 << 31)) return GS_ERR_INVALID_ARG;
  hipLaunchKernelGGL(mad_kernel, dim3((unsigned)(3 * n_blocks)), dim3(kMadThreads), 0, (hipStream_t)stream,
                     finest->means, finest->n, lvl_off, lvl_cnt, n_levels, n_mad, lo, hi);
  GS_LAUNCH_CHECK();
  return GS_OK;
}
