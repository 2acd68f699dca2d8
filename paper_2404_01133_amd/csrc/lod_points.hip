// Point-wise level-of-detail selection: the baseline that Sec. 3.3.2 weighs
// against the block-wise strategy (ablated in Table 5).  Every Gaussian of
// every level is tested on its own: level l keeps the Gaussians whose centre
// distance to the camera centre falls in level l's distance interval and whose
// centre lies in the view frustum (camera-space z > znear, projection inside
// the screen widened by 15 % of its size on every side, the rasterizer's 1.3x
// guard band for a centred principal point).
//
// Output: view v's selection is L segments (level 0 first), each listing the
// chosen Gaussians' indices within the level in ascending order.  A stable
// compaction over the virtual array (view, level, index) in three launches,
// no inter-work-group waits:
//   1. flags   one work-group per tile: FP64 tests in the fixed operation
//              order of the block-wise selection, the tile's selection bit
//              masks and count (tiles never straddle a (view, level) segment,
//              so camera and level are uniform per tile: scalar registers)
//   2. scan    one work-group: exclusive prefix of the tile counts, segment
//              offsets, record count
//   3. write   one work-group per tile: gather indices from the bit masks
#include "gs_common.h"

namespace gs {
namespace {

constexpr int kPtThreads = 256;
constexpr int kPtItems = 8;                           // elements per thread per round
constexpr int kPtRounds = 2;                          // rounds per tile
constexpr int kPtSlots = kPtRounds * kPtItems;        // (round, item) slots of a tile
constexpr int kPtWaves = kPtThreads / 64;
constexpr int kPtTile = kPtThreads * kPtSlots;        // 4096 elements per tile
constexpr int kPtMaxLevels = 8;
constexpr int kScanThreads = 1024;
constexpr double kPointGuard = 0.15;

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

// (view, level, first element) of tile t, uniform over the work-group
struct TileRef {
  int v, l;
  int64_t i0;
};
__device__ __forceinline__ TileRef tile_ref(const PointArgs& a, int64_t t) {
  TileRef r;
  r.v = (int)(t / a.tiles_per_view);
  int64_t tl = t - (int64_t)r.v * a.tiles_per_view;
  int l = 0;
  while (tl >= a.tiles[l]) {
    tl -= a.tiles[l];
    ++l;
  }
  r.l = l;
  r.i0 = tl * kPtTile;
  return r;
}

// element of (slot, thread) in a tile: element order is (round, item, wave, lane)
__device__ __forceinline__ int64_t slot_element(int64_t i0, int slot) {
  return i0 + (int64_t)(slot / kPtItems) * (kPtThreads * kPtItems) + (slot % kPtItems) * kPtThreads + threadIdx.x;
}

// exclusive prefix of one u32 per thread over the work-group (thread order)
template <int NT>
__device__ __forceinline__ uint64_t block_prefix(uint64_t x, uint64_t* s_wave, uint64_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint64_t inc = x;
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) s_wave[wid] = inc;
  __syncthreads();
  uint64_t base = 0, tot = 0;
  for (int w = 0; w < NT / 64; ++w) {
    const uint64_t c = s_wave[w];
    base += w < wid ? c : 0u;
    tot += c;
  }
  *total = tot;
  __syncthreads();
  return base + inc - x;
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

__global__ void __launch_bounds__(kPtThreads) point_flags_kernel(PointArgs a, uint64_t* __restrict__ masks,
                                                                 uint32_t* __restrict__ tile_count) {
  __shared__ uint32_t s_cnt[kPtSlots * kPtWaves];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t t = blockIdx.x;
  const TileRef tr = tile_ref(a, t);
  const int l = tr.l;
  const int64_t n = a.n[l];
  const float* mean = a.means[l];
  const gs_camera& cam = a.cams[tr.v];
  const double* R = cam.R;
  const double* tc = cam.t;
  const double C0 = -((R[0] * tc[0] + R[3] * tc[1]) + R[6] * tc[2]);
  const double C1 = -((R[1] * tc[0] + R[4] * tc[1]) + R[7] * tc[2]);
  const double C2 = -((R[2] * tc[0] + R[5] * tc[1]) + R[8] * tc[2]);
  const double W = (double)cam.width, H = (double)cam.height;
  const double ulo = -kPointGuard * W, uhi = (1.0 + kPointGuard) * W;
  const double vlo = -kPointGuard * H, vhi = (1.0 + kPointGuard) * H;
  for (int r = 0; r < kPtRounds; ++r) {
    float px[kPtItems], py[kPtItems], pz[kPtItems];
#pragma unroll
    for (int k = 0; k < kPtItems; ++k) {
      const int64_t i = slot_element(tr.i0, r * kPtItems + k);
      const bool ok = i < n;
      px[k] = ok ? mean[i] : 0.0f;
      py[k] = ok ? mean[n + i] : 0.0f;
      pz[k] = ok ? mean[2 * n + i] : 0.0f;
    }
    // level of every item first (independent chains), then the frustum test
    // where the level matches
    bool sel[kPtItems];
#pragma unroll
    for (int k = 0; k < kPtItems; ++k) {
      const double dx = (double)px[k] - C0, dy = (double)py[k] - C1, dz = (double)pz[k] - C2;
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      int lev = a.L - 1;
      for (int q = 0; q < a.L - 1; ++q)
        if (d2 >= a.thr[q] * a.thr[q]) --lev;
      sel[k] = (lev == l) && (slot_element(tr.i0, r * kPtItems + k) < n);
    }
#pragma unroll
    for (int k = 0; k < kPtItems; ++k) {
      if (sel[k]) {
        const double x = (double)px[k], y = (double)py[k], z = (double)pz[k];
        const double zc = ((R[6] * x + R[7] * y) + R[8] * z) + tc[2];
        const double xc = ((R[0] * x + R[1] * y) + R[2] * z) + tc[0];
        const double yc = ((R[3] * x + R[4] * y) + R[5] * z) + tc[1];
        const double rz = 1.0 / zc;
        const double u = cam.fx * (xc * rz) + cam.cx;
        const double w = cam.fy * (yc * rz) + cam.cy;
        sel[k] = (zc > cam.znear) && (u > ulo) && (u < uhi) && (w > vlo) && (w < vhi);
      }
    }
#pragma unroll
    for (int k = 0; k < kPtItems; ++k) {
      const uint64_t m = __ballot(sel[k]);
      const int slot = r * kPtItems + k;
      if (lane == 0) {
        masks[((int64_t)t * kPtSlots + slot) * kPtWaves + wid] = m;
        s_cnt[slot * kPtWaves + wid] = (uint32_t)__popcll(m);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    uint32_t c = 0;
    for (int k = threadIdx.x; k < kPtSlots * kPtWaves; k += 64) c += s_cnt[k];
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
    if (threadIdx.x == 0) tile_count[t] = c;
  }
}

// One work-group: exclusive prefix of the tile counts; segment (v, l) starts at
// its first tile (an empty segment at the next segment's first tile).
__global__ void __launch_bounds__(kScanThreads) point_scan_kernel(PointArgs a, const uint32_t* __restrict__ tile_count,
                                                                  uint64_t* __restrict__ tile_off,
                                                                  int64_t* __restrict__ offsets,
                                                                  int64_t* __restrict__ counts) {
  __shared__ uint64_t s_wave[kScanThreads / 64];
  __shared__ uint64_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < a.n_tiles; base += kScanThreads) {
    const int64_t t = base + threadIdx.x;
    const uint64_t c = t < a.n_tiles ? tile_count[t] : 0u;
    uint64_t tot;
    const uint64_t ex = block_prefix<kScanThreads>(c, s_wave, &tot);
    const uint64_t carry = s_carry;
    if (t < a.n_tiles) tile_off[t] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + tot;
    __syncthreads();
  }
  const uint64_t total = s_carry;
  const int64_t nseg = (int64_t)a.V * a.L;
  for (int64_t sg = threadIdx.x; sg <= nseg; sg += kScanThreads) {
    int64_t first = a.n_tiles;
    if (sg < nseg) {
      const int v = (int)(sg / a.L), l = (int)(sg - (int64_t)v * a.L);
      first = (int64_t)v * a.tiles_per_view;
      for (int q = 0; q < l; ++q) first += a.tiles[q];
    }
    offsets[sg] = first < a.n_tiles ? (int64_t)tile_off[first] : (int64_t)total;
  }
  if (threadIdx.x == 0) {
    counts[GS_COUNT_RECORDS] = (int64_t)total;
    counts[GS_COUNT_VISIBLE] = 0;
    counts[GS_COUNT_PAIRS] = 0;
    counts[GS_COUNT_FLAGS] = (int64_t)total > a.capacity ? GS_FLAG_RECORDS : 0;
  }
}

__global__ void __launch_bounds__(kPtThreads) point_write_kernel(PointArgs a, const uint64_t* __restrict__ masks,
                                                                 const uint64_t* __restrict__ tile_off,
                                                                 uint32_t* __restrict__ gather) {
  __shared__ uint64_t s_wave[kPtWaves];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t t = blockIdx.x;
  const TileRef tr = tile_ref(a, t);
  // thread q owns the (slot, wave) entry q of the tile: counts in element order
  static_assert(kPtSlots * kPtWaves <= kPtThreads, "one (slot, wave) entry per thread");
  const int64_t mbase = (int64_t)t * kPtSlots * kPtWaves;
  const uint64_t mine = threadIdx.x < kPtSlots * kPtWaves ? masks[mbase + threadIdx.x] : 0ull;
  uint64_t tot;
  const uint64_t ex = block_prefix<kPtThreads>((uint64_t)__popcll(mine), s_wave, &tot);
  __shared__ uint64_t s_ex[kPtSlots * kPtWaves];
  if (threadIdx.x < kPtSlots * kPtWaves) s_ex[threadIdx.x] = ex;
  __syncthreads();
  const uint64_t base = tile_off[t];
#pragma unroll 4
  for (int slot = 0; slot < kPtSlots; ++slot) {
    const int e = slot * kPtWaves + wid;
    const uint64_t m = masks[mbase + e];
    if ((m >> lane) & 1ull) {
      const int64_t pos = (int64_t)(base + s_ex[e] + lanemask_lt_count(m));
      if (pos < a.capacity) gather[pos] = (uint32_t)slot_element(tr.i0, slot);
    }
  }
}

}  // namespace
}  // namespace gs

extern "C" size_t gs_points_workspace_bytes(const int64_t* level_sizes, int32_t n_levels, int32_t n_views) {
  using namespace gs;
  if (!level_sizes || n_levels <= 0 || n_levels > kPtMaxLevels || n_views <= 0) return 0;
  int64_t tpv = 0;
  for (int l = 0; l < n_levels; ++l) tpv += (level_sizes[l] + kPtTile - 1) / kPtTile;
  const size_t nt = (size_t)(tpv * n_views);
  return 256 + nt * (4 + 8 + 8 * kPtSlots * kPtWaves);  // counts, offsets, masks
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
  // workspace: tile counts [n_tiles] u32, tile offsets [n_tiles] u64, masks [n_tiles][slots][waves] u64
  char* w = (char*)ws;
  uint64_t* masks = (uint64_t*)w;
  uint64_t* tile_off = (uint64_t*)(w + (size_t)a.n_tiles * 8 * kPtSlots * kPtWaves);
  uint32_t* tile_count = (uint32_t*)((char*)tile_off + (size_t)a.n_tiles * 8);
  hipLaunchKernelGGL(point_flags_kernel, dim3((unsigned)a.n_tiles), dim3(kPtThreads), 0, s, a, masks, tile_count);
  GS_LAUNCH_CHECK();
  hipLaunchKernelGGL(point_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, a, (const uint32_t*)tile_count, tile_off,
                     offsets, counts);
  GS_LAUNCH_CHECK();
  hipLaunchKernelGGL(point_write_kernel, dim3((unsigned)a.n_tiles), dim3(kPtThreads), 0, s, a,
                     (const uint64_t*)masks, (const uint64_t*)tile_off, gather);
  GS_LAUNCH_CHECK();
  return GS_OK;
}
