// Point-wise level-of-detail selection: the baseline that Sec. 3.3.2 weighs
// against the block-wise strategy (ablated in Table 5).  Every Gaussian of
// every level is tested on its own: level l keeps the Gaussians whose centre
// distance to the camera centre falls in level l's distance interval and whose
// centre lies in the view frustum (camera-space z > znear, projection inside
// the screen widened by 15 % of its size on every side, the rasterizer's 1.3x
// guard band for a centred principal point).
//
// Output: view v's selection is L segments (level 0 first), each listing the
// chosen Gaussians' indices within the level in ascending order.  One stable
// single-pass compaction over the virtual array (view, level, index) writes
// them: work-group tiles never straddle a (view, level) segment, so the
// camera and the level are uniform per tile (scalar registers), and the
// per-element work is three coalesced FP32 loads plus the FP64 tests in the
// fixed operation order of the block-wise selection.
#include "scan.h"

namespace gs {
namespace {

constexpr int kPtThreads = 256;
constexpr int kPtItems = 8;
constexpr int kPtTile = kPtThreads * kPtItems;
constexpr int kPtMaxLevels = 8;
constexpr double kPointGuard = 0.15;
constexpr int kPtChunk = 8;  // consecutive tiles claimed per atomic (one shared counter is a serial point)

struct PointArgs {
  const float* means[kPtMaxLevels];  // [3][n_l] per level
  int64_t n[kPtMaxLevels];           // Gaussians per level
  int64_t tiles[kPtMaxLevels];       // ceil(n_l / kPtTile)
  int64_t tiles_per_view;
  int64_t n_tiles;
  const gs_camera* cams;
  int64_t capacity;
  int32_t L, V;
  double thr[kPtMaxLevels - 1];
};

__global__ void point_clear_kernel(uint64_t* __restrict__ status, int64_t n_status, uint32_t* __restrict__ counter,
                                   int64_t* __restrict__ counts) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_status; i += stride) status[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *counter = 0u;
    counts[GS_COUNT_VISIBLE] = 0;
    counts[GS_COUNT_PAIRS] = 0;
    counts[GS_COUNT_FLAGS] = 0;
  }
}

// nothing to select (every level empty): all offsets and the record count are 0
__global__ void point_empty_kernel(int64_t* __restrict__ offsets, int64_t n_off, int64_t* __restrict__ counts) {
  for (int64_t i = threadIdx.x; i < n_off; i += blockDim.x) offsets[i] = 0;
  if (threadIdx.x == 0) {
    counts[GS_COUNT_RECORDS] = 0;
    counts[GS_COUNT_VISIBLE] = 0;
    counts[GS_COUNT_PAIRS] = 0;
    counts[GS_COUNT_FLAGS] = 0;
  }
}

__global__ void __launch_bounds__(kPtThreads) point_select_kernel(PointArgs a, uint32_t* __restrict__ gather,
                                                                  int64_t* __restrict__ offsets,
                                                                  uint64_t* __restrict__ status,
                                                                  uint32_t* __restrict__ tile_counter,
                                                                  int64_t* __restrict__ counts) {
  __shared__ uint32_t s_cnt[kPtItems][kPtThreads / 64];
  __shared__ uint64_t s_excl;
  __shared__ uint32_t s_tile;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // tiles are claimed kPtChunk at a time, in order, and done in order inside a
  // chunk, so every predecessor a look-back waits on is owned by a running
  // work-group that reaches it
  int64_t t = 0, chunk_end = 0;
  for (;;) {
    if (t == chunk_end) {
      if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
      __syncthreads();
      t = (int64_t)__builtin_amdgcn_readfirstlane(s_tile) * kPtChunk;
      chunk_end = t + kPtChunk;
      if (chunk_end > a.n_tiles) chunk_end = a.n_tiles;
    }
    if (t >= a.n_tiles) break;
    // (view, level, tile within the level), uniform over the work-group
    const int v = (int)(t / a.tiles_per_view);
    int64_t tl = t - (int64_t)v * a.tiles_per_view;
    int l = 0;
    while (tl >= a.tiles[l]) {
      tl -= a.tiles[l];
      ++l;
    }
    const int64_t n = a.n[l];
    const float* mean = a.means[l];
    const gs_camera& cam = a.cams[v];
    const double* R = cam.R;
    const double* tc = cam.t;
    const double C0 = -((R[0] * tc[0] + R[3] * tc[1]) + R[6] * tc[2]);
    const double C1 = -((R[1] * tc[0] + R[4] * tc[1]) + R[7] * tc[2]);
    const double C2 = -((R[2] * tc[0] + R[5] * tc[1]) + R[8] * tc[2]);
    const double W = (double)cam.width, H = (double)cam.height;
    const double ulo = -kPointGuard * W, uhi = (1.0 + kPointGuard) * W;
    const double vlo = -kPointGuard * H, vhi = (1.0 + kPointGuard) * H;
    const int64_t i_base = tl * kPtTile;
    float px[kPtItems], py[kPtItems], pz[kPtItems];
#pragma unroll
    for (int k = 0; k < kPtItems; ++k) {
      const int64_t i = i_base + k * kPtThreads + threadIdx.x;
      const bool ok = i < n;
      px[k] = ok ? mean[i] : 0.0f;
      py[k] = ok ? mean[n + i] : 0.0f;
      pz[k] = ok ? mean[2 * n + i] : 0.0f;
    }
    uint64_t mask[kPtItems];
#pragma unroll
    for (int k = 0; k < kPtItems; ++k) {
      const int64_t i = i_base + k * kPtThreads + threadIdx.x;
      bool sel = false;
      if (i < n) {
        const double x = (double)px[k], y = (double)py[k], z = (double)pz[k];
        const double dx = x - C0, dy = y - C1, dz = z - C2;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        int lev = a.L - 1;
        for (int q = 0; q < a.L - 1; ++q)
          if (d2 >= a.thr[q] * a.thr[q]) --lev;
        if (lev == l) {
          const double zc = ((R[6] * x + R[7] * y) + R[8] * z) + tc[2];
          if (zc > cam.znear) {
            const double xc = ((R[0] * x + R[1] * y) + R[2] * z) + tc[0];
            const double yc = ((R[3] * x + R[4] * y) + R[5] * z) + tc[1];
            const double rz = 1.0 / zc;
            const double u = cam.fx * (xc * rz) + cam.cx;
            const double w = cam.fy * (yc * rz) + cam.cy;
            sel = (u > ulo) && (u < uhi) && (w > vlo) && (w < vhi);
          }
        }
      }
      mask[k] = __ballot(sel);
      if (lane == 0) s_cnt[k][wid] = (uint32_t)__popcll(mask[k]);
    }
    __syncthreads();
    // element order inside the tile is (item, wave, lane): the prefix of this
    // lane's item k counts all earlier items and the earlier waves of item k
    uint32_t base[kPtItems];
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < kPtItems; ++k) {
      uint32_t before = total;
#pragma unroll
      for (int w = 0; w < kPtThreads / 64; ++w) {
        const uint32_t c = s_cnt[k][w];
        before += w < wid ? c : 0u;
        total += c;
      }
      base[k] = before;
    }
    if (threadIdx.x < 64) {
      const uint64_t ex = lookback64_wave(status, t, total, counts);
      if (threadIdx.x == 0) {
        s_excl = ex;
        if (tl == 0) {  // first tile of segment (v, l): its start, and that of empty segments before it
          int64_t s = (int64_t)v * a.L + l;
          offsets[s] = (int64_t)ex;
          for (--s; s >= 0 && a.n[s % a.L] == 0; --s) offsets[s] = (int64_t)ex;
        }
        if (t == a.n_tiles - 1) {
          const int64_t all = (int64_t)(ex + total);
          int64_t s = (int64_t)a.V * a.L;
          offsets[s] = all;
          for (--s; s >= 0 && a.n[s % a.L] == 0; --s) offsets[s] = all;
          counts[GS_COUNT_RECORDS] = all;
          if (all > a.capacity) raise_flag(counts, GS_FLAG_RECORDS);
        }
      }
    }
    __syncthreads();
    const uint64_t ex = s_excl;
#pragma unroll
    for (int k = 0; k < kPtItems; ++k) {
      if ((mask[k] >> lane) & 1ull) {
        const int64_t pos = (int64_t)(ex + base[k] + (uint32_t)lanemask_lt_count(mask[k]));
        if (pos < a.capacity) gather[pos] = (uint32_t)(i_base + k * kPtThreads + threadIdx.x);
      }
    }
    __syncthreads();
    ++t;
  }
}

}  // namespace
}  // namespace gs

extern "C" size_t gs_points_workspace_bytes(const int64_t* level_sizes, int32_t n_levels, int32_t n_views) {
  using namespace gs;
  if (!level_sizes || n_levels <= 0 || n_levels > kPtMaxLevels || n_views <= 0) return 0;
  int64_t tpv = 0;
  for (int l = 0; l < n_levels; ++l) tpv += (level_sizes[l] + kPtTile - 1) / kPtTile;
  return 256 + 8 * (size_t)(tpv * n_views);
}

extern "C" gs_status gs_lod_select_points(const gs_gaussians* levels, int32_t n_levels, const double* thresholds,
                                          const gs_camera* cams, int32_t n_views, int64_t record_capacity,
                                          uint32_t* gather, int64_t* offsets, int64_t* counts, void* ws,
                                          size_t ws_bytes, void* stream) {
  using namespace gs;
  if (!levels || !cams || !offsets || !counts || !ws || n_views <= 0) return GS_ERR_INVALID_ARG;
  if (n_levels <= 0 || n_levels > kPtMaxLevels) return GS_ERR_INVALID_ARG;
  if (n_levels > 1 && !thresholds) return GS_ERR_INVALID_ARG;
  if (record_capacity < 0 || (record_capacity > 0 && !gather)) return GS_ERR_INVALID_ARG;
  PointArgs a{};
  int64_t sizes[kPtMaxLevels];
  for (int l = 0; l < n_levels; ++l) {
    const gs_gaussians& g = levels[l];
    if (g.n < 0 || g.n >= ((int64_t)1 << 32) || (g.n > 0 && !g.means)) return GS_ERR_INVALID_ARG;
    a.means[l] = g.means;
    a.n[l] = g.n;
    a.tiles[l] = (g.n + kPtTile - 1) / kPtTile;
    a.tiles_per_view += a.tiles[l];
    sizes[l] = g.n;
  }
  for (int k = 0; k + 1 < n_levels; ++k) {
    a.thr[k] = thresholds[k];
    if (!(thresholds[k] >= 0.0) || (k > 0 && thresholds[k] < thresholds[k - 1])) return GS_ERR_INVALID_ARG;
  }
  a.n_tiles = a.tiles_per_view * n_views;
  if (a.n_tiles >= ((int64_t)1 << 31)) return GS_ERR_INVALID_ARG;
  if (ws_bytes < gs_points_workspace_bytes(sizes, n_levels, n_views)) return GS_ERR_WORKSPACE;
  a.cams = cams;
  a.capacity = record_capacity;
  a.L = n_levels;
  a.V = n_views;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n_off = (int64_t)n_views * n_levels + 1;
  if (a.n_tiles == 0) {
    hipLaunchKernelGGL(point_empty_kernel, dim3(1), dim3(256), 0, s, offsets, n_off, counts);
    GS_LAUNCH_CHECK();
    return GS_OK;
  }
  uint32_t* counter = (uint32_t*)ws;
  uint64_t* status = (uint64_t*)((char*)ws + 256);
  const int64_t cg = (a.n_tiles + 255) / 256;
  hipLaunchKernelGGL(point_clear_kernel, dim3((unsigned)(cg < 1024 ? cg : 1024)), dim3(256), 0, s, status, a.n_tiles,
                     counter, counts);
  GS_LAUNCH_CHECK();
  const int64_t chunks = (a.n_tiles + kPtChunk - 1) / kPtChunk;
  const int64_t grid = chunks < 2048 ? chunks : 2048;
  hipLaunchKernelGGL(point_select_kernel, dim3((unsigned)grid), dim3(kPtThreads), 0, s, a, gather, offsets, status,
                     counter, counts);
  GS_LAUNCH_CHECK();
  return GS_OK;
}
