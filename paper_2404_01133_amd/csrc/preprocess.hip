// Projection of the selected Gaussians to screen-space records (the "proj"
// operator of Eq. 1 in Sec. 3.1, which the paper takes from 3DGS: EWA splatting
// through the local affine approximation of the pinhole map, 0.3 px^2 low-pass
// dilation, 3-sigma footprint, SH colour).
//
// Memory-bound: each record reads the 44 B of geometry (centre, opacity,
// rotation, scale) in one round of loads, and the 192 B of SH only if it
// survives the footprint cull.  Loads are structure-of-arrays, so consecutive
// lanes touch consecutive words; the (view, block) segment of a record is
// found by binary search in an LDS copy of the segment offsets.
//
// The geometry that decides integers (culls, footprint, depth key) is FP64 in
// a fixed operation order; this file is compiled with -ffp-contract=off so the
// compiler cannot fuse or reorder those operations.
#include "project.h"

namespace gs {
namespace {

constexpr int kPreThreads = 256;
constexpr int kLdsOffsets = 1024;  // segment offsets staged in LDS up to this many; global memory beyond

struct PreArgs {
  LevelPtrs lv[kMaxLevels];
  const int64_t* lvl_off;
  const int8_t* level;
  const int64_t* offsets;
  const uint32_t* gather;  // point-wise selection: record -> index within its level
  const gs_camera* cams;
  int64_t capacity;
  int32_t B, L, V, W, H, tw, th, sh_degree;
  int32_t segs;    // segments per view: B (block-wise), L (point-wise) or 1 (packed)
  int32_t packed;  // gather entries are level << GS_PACKED_INDEX_BITS | index (refined selection)
};

// One record: Gaussian gi of level l, seen by view v, stored at record index g.
template <bool HALF>
__device__ __forceinline__ void preprocess_record_t(const PreArgs& a, int64_t g, int v, int l, int64_t gi,
                                                    Record* __restrict__ records, uint32_t* __restrict__ depth_keys,
                                                    int32_t* __restrict__ tiles_touched) {
  const LevelPtrs& L = a.lv[l];
  const gs_camera& cam = a.cams[v];
  Geo o;
  uint32_t key = kCulledKey;
  int32_t tt = 0;
  if (project_geo<HALF>(L, gi, cam, a.W, a.H, o)) {
    tt = (o.i1 / a.tw - o.i0 / a.tw + 1) * (o.j1 / a.th - o.j0 / a.th + 1);
    key = __float_as_uint(o.depth);
    Record rec;
    rec.du = (float)(o.u - (double)o.i0) - 0.5f;  // exact shift (|u - i0| < 2^22)
    rec.dv = (float)(o.v - (double)o.j0) - 0.5f;
    rec.px = (uint32_t)o.i0 | ((uint32_t)(o.i1 - o.i0) << 16);
    rec.py = (uint32_t)o.j0 | ((uint32_t)(o.j1 - o.j0) << 16);
    rec.ca = (float)(kConicScale * sqrt(o.c / o.det));
    rec.cb = (float)(-kConicScale * o.b / sqrt(o.c * o.det));
    rec.cc = (float)(kConicScale / sqrt(o.c));
    rec.opac = (float)o.opac;
    double C[3];
    camera_centre(cam, C);
    const double d0 = o.m[0] - C[0], d1 = o.m[1] - C[1], d2 = o.m[2] - C[2];
    const double dn = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
    const int deg = a.sh_degree < L.sh_deg ? a.sh_degree : L.sh_deg;
    double col[3] = {0.0, 0.0, 0.0};
    sh_colour<HALF>(d0 / dn, d1 / dn, d2 / dn, deg, L.sh, L.n, gi, col);
    rec.r = (float)dmax_(col[0] + 0.5, 0.0);
    rec.g = (float)dmax_(col[1] + 0.5, 0.0);
    rec.b = (float)dmax_(col[2] + 0.5, 0.0);
    rec.view = (uint32_t)v;
    records[g] = rec;
  }
  depth_keys[g] = key;
  tiles_touched[g] = tt;
}

__device__ __forceinline__ void preprocess_record(const PreArgs& a, int64_t g, int v, int l, int64_t gi,
                                                  Record* __restrict__ records, uint32_t* __restrict__ depth_keys,
                                                  int32_t* __restrict__ tiles_touched) {
  if (a.lv[l].half) preprocess_record_t<true>(a, g, v, l, gi, records, depth_keys, tiles_touched);
  else preprocess_record_t<false>(a, g, v, l, gi, records, depth_keys, tiles_touched);
}

__device__ __forceinline__ int64_t clamp_records(const PreArgs& a, int64_t* counts) {
  int64_t n_rec = counts[GS_COUNT_RECORDS];
  if (n_rec > a.capacity) {
    if (blockIdx.x == 0 && threadIdx.x == 0)
      atomicOr((unsigned long long*)&counts[GS_COUNT_FLAGS], (unsigned long long)GS_FLAG_RECORDS);
    n_rec = a.capacity;
  }
  return n_rec;
}

// View-major: records in index order, each mapped to (view, segment) by a
// binary search of the segment offsets (staged in LDS when they fit).  A
// block-wise segment is (view, block) at the block's chosen level; a
// point-wise segment is (view, level) with the Gaussian read from the gather list.
__global__ void __launch_bounds__(kPreThreads) preprocess_kernel(PreArgs a, Record* __restrict__ records,
                                                                 uint32_t* __restrict__ depth_keys,
                                                                 int32_t* __restrict__ tiles_touched,
                                                                 int64_t* __restrict__ counts) {
  const int64_t n_rec = clamp_records(a, counts);
  const int nseg = a.V * a.segs;
  __shared__ int64_t s_off[kLdsOffsets];
  const bool lds_off = nseg < kLdsOffsets;
  if (lds_off)
    for (int k = threadIdx.x; k <= nseg; k += blockDim.x) s_off[k] = a.offsets[k];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_rec; g += stride) {
    const int p = lds_off ? find_segment(s_off, nseg, g) : find_segment(a.offsets, nseg, g);
    const int v = p / a.segs, b = p - v * a.segs;
    int l;
    int64_t gi;
    if (a.packed) {
      const uint32_t e = a.gather[g];
      l = (int)(e >> GS_PACKED_INDEX_BITS);
      gi = (int64_t)(e & ((1u << GS_PACKED_INDEX_BITS) - 1u));
      if (l >= a.L || gi >= a.lv[l].n) {  // not a stored Gaussian: nothing to project
        depth_keys[g] = kCulledKey;
        tiles_touched[g] = 0;
        continue;
      }
    } else if (a.gather) {
      l = b;
      gi = a.gather[g];
    } else {
      l = a.level[p];
      gi = a.lvl_off[(int64_t)b * a.L + l] + (g - (lds_off ? s_off[p] : a.offsets[p]));
    }
    preprocess_record(a, g, v, l, gi, records, depth_keys, tiles_touched);
  }
}

// Shared-selection precondition, checked by one work-group before the
// Gaussian-major kernel: V times view 0's records, and every view's segment
// offsets and levels equal to view 0's (offsets shifted by v times view 0's
// count).  A violation raises GS_FLAG_SELECTION, which the Gaussian-major
// kernels read before doing anything else.
__global__ void __launch_bounds__(kPreThreads) shared_selection_check_kernel(PreArgs a, int64_t* __restrict__ counts) {
  const int64_t n_view = a.offsets[a.segs];
  bool bad = counts[GS_COUNT_RECORDS] != (int64_t)a.V * n_view;
  const int64_t nseg = (int64_t)a.V * a.segs;
  for (int64_t idx = threadIdx.x; idx <= nseg; idx += blockDim.x) {
    const int64_t v = idx / a.segs, k = idx - v * a.segs;
    bad |= a.offsets[idx] != a.offsets[k] + v * n_view;
    if (idx < nseg) bad |= a.level[idx] != a.level[k];
  }
  if (__syncthreads_or(bad) && threadIdx.x == 0)
    atomicOr((unsigned long long*)&counts[GS_COUNT_FLAGS], (unsigned long long)GS_FLAG_SELECTION);
}

// Gaussian-major, for batches in which every view selected the same records
// (view v's records are [v * n_view, (v + 1) * n_view)): one thread projects a
// Gaussian for all views in turn, so its parameters come from HBM once and
// from cache afterwards.  View 0's segments and levels are used for all views.
__global__ void __launch_bounds__(kPreThreads) preprocess_shared_kernel(PreArgs a, Record* __restrict__ records,
                                                                        uint32_t* __restrict__ depth_keys,
                                                                        int32_t* __restrict__ tiles_touched,
                                                                        int64_t* __restrict__ counts) {
  const int64_t n_rec = clamp_records(a, counts);
  if (counts[GS_COUNT_FLAGS] & GS_FLAG_SELECTION) {
    // the views did not select the same records: an empty frame, nothing projected
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_rec; g += stride) {
      depth_keys[g] = kCulledKey;
      tiles_touched[g] = 0;
    }
    return;
  }
  __shared__ int64_t s_off[kLdsOffsets];
  const bool lds_off = a.segs < kLdsOffsets;
  if (lds_off)
    for (int k = threadIdx.x; k <= a.segs; k += blockDim.x) s_off[k] = a.offsets[k];
  __syncthreads();
  const int64_t n_view = a.offsets[a.segs];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_view; i += stride) {
    const int b = lds_off ? find_segment(s_off, a.segs, i) : find_segment(a.offsets, a.segs, i);
    const int l = a.gather ? b : a.level[b];
    const int64_t gi = a.gather ? (int64_t)a.gather[i]
                                : a.lvl_off[(int64_t)b * a.L + l] + (i - (lds_off ? s_off[b] : a.offsets[b]));
    for (int v = 0; v < a.V; ++v) {
      const int64_t g = (int64_t)v * n_view + i;
      if (g >= n_rec) break;
      preprocess_record(a, g, v, l, gi, records, depth_keys, tiles_touched);
    }
  }
}

}  // namespace
}  // namespace gs

extern "C" gs_status gs_preprocess(const gs_gaussians* levels, const gs_blocks* blocks, const int8_t* level,
                                   const int64_t* offsets, const uint32_t* gather, const gs_camera* cams, int32_t n_views, int32_t width,
                                   int32_t height, int32_t sh_degree, const gs_tuning* tuning,
                                   int64_t record_capacity, void* records, uint32_t* depth_keys,
                                   int32_t* tiles_touched, int64_t* counts, void* stream) {
  using namespace gs;
  if (!levels || !blocks || (!level && !gather) || !offsets || !cams || !tuning || !counts) return GS_ERR_INVALID_ARG;
  if (n_views <= 0 || width <= 0 || height <= 0 || width > 65535 || height > 65535) return GS_ERR_INVALID_ARG;
  if (sh_degree < 0 || sh_degree > 3) return GS_ERR_INVALID_ARG;
  if (blocks->n_levels <= 0 || blocks->n_levels > kMaxLevels) return GS_ERR_INVALID_ARG;
  if (!gather && (blocks->n_blocks <= 0 || !blocks->lvl_off)) return GS_ERR_INVALID_ARG;
  if (!tile_shape_supported(tuning->tile_w, tuning->tile_h)) return GS_ERR_UNSUPPORTED;
  if (record_capacity < 0 || (record_capacity > 0 && (!records || !depth_keys || !tiles_touched)))
    return GS_ERR_INVALID_ARG;
  const bool packed = (tuning->flags & GS_TUNE_PACKED_SELECTION) != 0;
  if (packed && !gather) return GS_ERR_INVALID_ARG;
  const int32_t segs = packed ? 1 : gather ? blocks->n_levels : blocks->n_blocks;
  if ((int64_t)n_views * segs > (int64_t)1 << 30) return GS_ERR_INVALID_ARG;
  if (record_capacity >= ((int64_t)1 << 32)) return GS_ERR_INVALID_ARG;  // record ids are u32
  PreArgs a{};
  for (int l = 0; l < blocks->n_levels; ++l) {
    const gs_gaussians& g = levels[l];
    if (g.n < 0 || (g.n > 0 && (!g.means || !g.scales || !g.quats || !g.opac || !g.sh))) return GS_ERR_INVALID_ARG;
    if (g.sh_degree < 0 || g.sh_degree > 3 || (g.attr_half != 0 && g.attr_half != 1)) return GS_ERR_INVALID_ARG;
    a.lv[l] = level_ptrs(g);
  }
  a.lvl_off = blocks->lvl_off;
  a.level = level;
  a.offsets = offsets;
  a.gather = gather;
  a.segs = segs;
  a.packed = packed ? 1 : 0;
  a.cams = cams;
  a.capacity = record_capacity;
  a.B = blocks->n_blocks;
  a.L = blocks->n_levels;
  a.V = n_views;
  a.W = width;
  a.H = height;
  a.tw = tuning->tile_w;
  a.th = tuning->tile_h;
  a.sh_degree = sh_degree;
  int64_t blocks_needed = (record_capacity + kPreThreads - 1) / kPreThreads;
  int grid = (int)(blocks_needed < 8192 ? (blocks_needed > 0 ? blocks_needed : 1) : 8192);
  if ((tuning->flags & GS_TUNE_SHARED_SELECTION) && n_views > 1) {
    if (gather || packed) return GS_ERR_UNSUPPORTED;
    hipLaunchKernelGGL(shared_selection_check_kernel, dim3(1), dim3(kPreThreads), 0, (hipStream_t)stream, a, counts);
    int64_t per_view = (record_capacity / n_views + kPreThreads - 1) / kPreThreads;
    int g2 = (int)(per_view < 8192 ? (per_view > 0 ? per_view : 1) : 8192);
    hipLaunchKernelGGL(preprocess_shared_kernel, dim3(g2), dim3(kPreThreads), 0, (hipStream_t)stream, a,
                       (Record*)records, depth_keys, tiles_touched, counts);
  } else {
    hipLaunchKernelGGL(preprocess_kernel, dim3(grid), dim3(kPreThreads), 0, (hipStream_t)stream, a,
                       (Record*)records, depth_keys, tiles_touched, counts);
  }
  GS_LAUNCH_CHECK();
  return GS_OK;
}
