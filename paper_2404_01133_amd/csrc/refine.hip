// Chunk refinement of a block-wise selection (an implementation step between
// the LoD selection of Sec. 3.3.2 and the projection of Eq. 1; it changes no
// rendered value).
//
// Each (block, level) run of Gaussians is cut into chunks of GS_CHUNK in storage
// order (Morton order inside a block, so a chunk is a compact piece of space);
// gs_chunk_bounds keeps, per chunk, the box of its centres and its largest scale
// component.  Per view, gs_lod_refine drops the chunks of the selected (block,
// level) runs that the projection would cull whole: every corner of the box
// behind the near plane, or the box in front of the camera with its projection
// (inside the hull of the projected corners) farther outside the image than a
// bound on the 3-sigma radius of any of its Gaussians.  The bound is the one the
// projection's own early test uses for one Gaussian: the trace of the projected
// covariance is at most |J|_F^2 s^2, |J|_F^2 is largest at the smallest depth
// over the box, s at most the chunk's largest scale (and one pixel more covers
// the rounding of the corners' projections); so a Gaussian of a dropped chunk is
// one the exact test culls too, and the records left produce the same visible set.  The survivors are listed as records in the block-wise order (per
// view: blocks in order, chunks and Gaussians in storage order), so the depth
// order and its ties among the visible records are unchanged and the images are
// identical bit for bit.
#include "radix.h"
#include "project.h"

namespace gs {
namespace {

constexpr int kChunk = GS_CHUNK;
constexpr int kScanItems = 16;
constexpr int kScanTile = 256 * kScanItems;  // entries per look-back tile of the count scan
constexpr int kExpandBatch = 256;            // entries per work-group round of the expansion

// first chunk of each (block, level) run, chunk_off[b * L + l]; chunk_off[B * L] = all chunks
__global__ void __launch_bounds__(256) chunk_offsets_kernel(const int64_t* __restrict__ lvl_cnt, int BL,
                                                            int64_t* __restrict__ chunk_off) {
  __shared__ int64_t s_part[256];
  const int per = (BL + 255) / 256;
  const int i0 = threadIdx.x * per, i1 = min(BL, i0 + per);
  int64_t sum = 0;
  for (int i = i0; i < i1; ++i) sum += (lvl_cnt[i] + kChunk - 1) / kChunk;
  s_part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int t = 0; t < 256; ++t) {
      const int64_t v = s_part[t];
      s_part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int64_t run = s_part[threadIdx.x];
  for (int i = i0; i < i1; ++i) {
    chunk_off[i] = run;
    run += (lvl_cnt[i] + kChunk - 1) / kChunk;
  }
  if (threadIdx.x == 255) chunk_off[BL] = run;  // the last thread's running sum is the total
}

// (block, level) run holding chunk k: the largest p with chunk_off[p] <= k
__device__ __forceinline__ int run_of_chunk(const int64_t* __restrict__ chunk_off, int BL, int64_t k) {
  int lo = 0, hi = BL;  // chunk_off[lo] <= k < chunk_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= k) lo = mid; else hi = mid;
  }
  return lo;
}

struct ChunkArgs {
  LevelPtrs lv[kMaxLevels];
  const int64_t* lvl_off;
  const int64_t* lvl_cnt;
  const int64_t* chunk_off;
  int32_t B, L;
};

// largest |scale| component of Gaussian gi
template <bool HALF>
__device__ __forceinline__ float chunk_scale(const LevelPtrs& L, int64_t gi) {
  return fmaxf(fabsf(attr<HALF>(L.scales, gi)),
               fmaxf(fabsf(attr<HALF>(L.scales, L.n + gi)), fabsf(attr<HALF>(L.scales, 2 * L.n + gi))));
}

// one work-group per chunk: box of the centres (lo xyz, hi xyz), the largest |scale| and the run
__global__ void __launch_bounds__(256) chunk_bounds_kernel(ChunkArgs a, int64_t max_chunks,
                                                           float* __restrict__ bounds) {
  __shared__ float s_red[7][4];
  const int BL = a.B * a.L;
  const int64_t C = a.chunk_off[BL];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t k = blockIdx.x; k < C && k < max_chunks; k += gridDim.x) {
    const int p = run_of_chunk(a.chunk_off, BL, k);
    const int l = p % a.L;
    const LevelPtrs& L = a.lv[l];
    const int64_t c = k - a.chunk_off[p];
    const int64_t start = a.lvl_off[p] + c * kChunk;
    const int64_t n = min((int64_t)kChunk, a.lvl_cnt[p] - c * kChunk);
    float v[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0f};
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const int64_t gi = start + i;
      const float x = L.means[gi], y = L.means[L.n + gi], z = L.means[2 * L.n + gi];
      v[0] = fminf(v[0], x), v[1] = fminf(v[1], y), v[2] = fminf(v[2], z);
      v[3] = fmaxf(v[3], x), v[4] = fmaxf(v[4], y), v[5] = fmaxf(v[5], z);
      v[6] = fmaxf(v[6], L.half ? chunk_scale<true>(L, gi) : chunk_scale<false>(L, gi));
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) {
      float x = v[q];
      for (int off = 32; off > 0; off >>= 1) {
        const float y = __shfl_xor(x, off, 64);
        x = q < 3 ? fminf(x, y) : fmaxf(x, y);
      }
      if (lane == 0) s_red[q][wid] = x;
    }
    __syncthreads();
    if (threadIdx.x < 7) {
      const int q = threadIdx.x;
      float x = s_red[q][0];
      for (int w = 1; w < 4; ++w) x = q < 3 ? fminf(x, s_red[q][w]) : fmaxf(x, s_red[q][w]);
      bounds[k * 8 + q] = x;
    }
    if (threadIdx.x == 7) bounds[k * 8 + 7] = __int_as_float(p);  // the chunk's run, b * L + l
    __syncthreads();
  }
}

// true if the projection culls every Gaussian whose centre lies in [lo, hi] and
// whose scale components are at most smax (see the file comment)
__device__ __forceinline__ bool chunk_culled(const float* __restrict__ bx, const gs_camera& cam, int W, int H) {
  const double* R = cam.R;
  const double lo[3] = {bx[0], bx[1], bx[2]}, hi[3] = {bx[3], bx[4], bx[5]};
  const double smax = bx[6];
  for (int q = 0; q < 7; ++q)
    if (!isfinite(bx[q])) return false;  // a non-finite centre or scale: the projection decides
  if (!(lo[0] <= hi[0] && lo[1] <= hi[1] && lo[2] <= hi[2] && smax >= 0.0)) return false;
  double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, zmin = INFINITY;
  int behind = 0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double x = (q & 1) ? hi[0] : lo[0], y = (q & 2) ? hi[1] : lo[1], z = (q & 4) ? hi[2] : lo[2];
    const double tx = ((R[0] * x + R[1] * y) + R[2] * z) + cam.t[0];
    const double ty = ((R[3] * x + R[4] * y) + R[5] * z) + cam.t[1];
    const double tz = ((R[6] * x + R[7] * y) + R[8] * z) + cam.t[2];
    if (!(tz > cam.znear - 1e-6)) {  // behind, with a margin over the rounding of the centres' depths
      ++behind;
      continue;
    }
    const double u = cam.fx * (tx / tz) + cam.cx, v = cam.fy * (ty / tz) + cam.cy;
    umin = fmin(umin, u), umax = fmax(umax, u), vmin = fmin(vmin, v), vmax = fmax(vmax, v);
    zmin = fmin(zmin, tz);
  }
  if (behind == 8) return true;  // depth is affine in the centre: every centre is behind the near plane
  if (behind > 0) return false;  // straddles the near plane: the projection decides
  const double limx = 1.3 * ((0.5 * W) / cam.fx), limy = 1.3 * ((0.5 * H) / cam.fy);
  const double jx = cam.fx / zmin, jy = cam.fy / zmin;
  const double jf2 = jx * jx * (1.0 + limx * limx) + jy * jy * (1.0 + limy * limy);
  // the per-Gaussian bound plus one pixel for the corners' own rounding
  const double rb = 3.0 * sqrt((jf2 * (smax * smax) + 0.6) * (1.0 + 1e-6)) + 3.0;
  return (umax + rb) - 0.5 < 0.0 || (umin - rb) - 0.5 > (double)(W - 1) || (vmax + rb) - 0.5 < 0.0 ||
         (vmin - rb) - 0.5 > (double)(H - 1);
}

struct RefineArgs {
  const int64_t* lvl_cnt;
  const int8_t* level;
  const int64_t* chunk_off;
  const float* bounds;
  const gs_camera* cams;
  int64_t max_chunks;
  int32_t B, L, V, W, H;
};

// chunks in the table, at most max_chunks (the entries the workspace holds); a larger table
// raises GS_FLAG_RECORDS when the view offsets are written, and the frame is invalid
__device__ __forceinline__ int64_t table_chunks(const RefineArgs& a) {
  const int64_t c = a.chunk_off[a.B * a.L];
  return c < a.max_chunks ? c : a.max_chunks;
}

// records kept by entry e = v * C + k (view v, chunk k of C): 0 if the view did not select the
// chunk's level or the chunk is culled, else the chunk's size
__device__ __forceinline__ uint32_t entry_keep(const RefineArgs& a, int64_t e, int64_t C) {
  const int v = (int)(e / C);
  const int64_t k = e - (int64_t)v * C;
  const int p = __float_as_int(a.bounds[k * 8 + 7]);
  if ((unsigned)p >= (unsigned)(a.B * a.L)) return 0u;  // not a table written by gs_chunk_bounds
  const int b = p / a.L, l = p - b * a.L;
  if (a.level[(int64_t)v * a.B + b] != l) return 0u;
  const int64_t c = k - a.chunk_off[p];
  const int64_t n = min((int64_t)kChunk, a.lvl_cnt[p] - c * kChunk);
  return chunk_culled(a.bounds + k * 8, a.cams[v], a.W, a.H) ? 0u : (uint32_t)n;
}

__global__ void refine_clear_kernel(uint64_t* __restrict__ status, int64_t words, uint32_t* __restrict__ counter) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
    status[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0u;
}

// per entry the records kept (0 if the view did not select the chunk's level or the chunk is culled)
__global__ void __launch_bounds__(256) refine_test_kernel(RefineArgs a, uint32_t* __restrict__ sizes) {
  const int64_t C = table_chunks(a);
  const int64_t total = (int64_t)a.V * C;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
    sizes[e] = entry_keep(a, e, C);
}

// exclusive prefix of the sizes in (view, chunk) order: one pass, tiles claimed in order (few, large
// tiles: each claim is an atomic on one counter), decoupled look-back over one count per tile
__global__ void __launch_bounds__(256) refine_scan_kernel(RefineArgs a, const uint32_t* __restrict__ sizes,
                                                          uint32_t* __restrict__ offs, uint64_t* __restrict__ status,
                                                          uint32_t* __restrict__ counter, int64_t* counts) {
  __shared__ uint64_t s_wave64[4];
  __shared__ uint32_t s_tile;
  __shared__ uint64_t s_base;
  const int64_t C = table_chunks(a);
  const int64_t total = (int64_t)a.V * C;
  const int64_t ntiles = (total + kScanTile - 1) / kScanTile;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1u);
    __syncthreads();
    const int64_t t = s_tile;
    if (t >= ntiles) break;
    const int64_t e0 = t * kScanTile + (int64_t)threadIdx.x * kScanItems;  // consecutive entries per thread
    uint32_t loc[kScanItems];
    if (e0 + kScanItems <= total) {  // 64 B aligned: the workspace arrays start on 256 B
#pragma unroll
      for (int q = 0; q < kScanItems; q += 4) {
        const uint4 x = *reinterpret_cast<const uint4*>(sizes + e0 + q);
        loc[q] = x.x, loc[q + 1] = x.y, loc[q + 2] = x.z, loc[q + 3] = x.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < kScanItems; ++q) loc[q] = e0 + q < total ? sizes[e0 + q] : 0u;
    }
    uint64_t mine = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) mine += loc[q];
    uint64_t tile_total;
    uint64_t run = block_excl_scan64(mine, s_wave64, &tile_total);
    if (threadIdx.x < 64) {
      const uint64_t ex = lookback64_wave(status, t, tile_total, counts);
      if (threadIdx.x == 0) s_base = ex;
    }
    __syncthreads();
    run += s_base;
    uint32_t out[kScanItems];
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
      out[q] = (uint32_t)min(run, (uint64_t)0xFFFFFFFFu);
      run += loc[q];
    }
    if (e0 + kScanItems <= total) {
#pragma unroll
      for (int q = 0; q < kScanItems; q += 4)
        *reinterpret_cast<uint4*>(offs + e0 + q) = make_uint4(out[q], out[q + 1], out[q + 2], out[q + 3]);
    } else {
#pragma unroll
      for (int q = 0; q < kScanItems; ++q)
        if (e0 + q < total) offs[e0 + q] = out[q];
    }
    __syncthreads();  // s_tile and s_base are rewritten next round
  }
}

// view offsets and the record count (by one work-group); raises GS_FLAG_RECORDS past the capacity
__device__ __forceinline__ void refine_views(const RefineArgs& a, const uint32_t* __restrict__ sizes,
                                             const uint32_t* __restrict__ offs, int64_t capacity,
                                             int64_t* __restrict__ view_off, int64_t* counts) {
  const int64_t C = table_chunks(a);
  const int64_t total_e = (int64_t)a.V * C;
  for (int v = threadIdx.x; v <= a.V; v += blockDim.x) {
    int64_t o;
    if (total_e == 0) o = 0;
    else if (v < a.V) o = offs[(int64_t)v * C];
    else o = (int64_t)offs[total_e - 1] + sizes[total_e - 1];
    view_off[v] = o;
    if (v == a.V) {
      counts[GS_COUNT_RECORDS] = o;
      if (o > capacity || a.chunk_off[a.B * a.L] > a.max_chunks) raise_flag(counts, GS_FLAG_RECORDS);
    }
  }
}

// the kept chunks' records: level << GS_PACKED_INDEX_BITS | index within the level.  A work-group
// takes kExpandBatch entries at a time, one per thread, strided by the grid (kept chunks come in long
// runs of consecutive entries, so this spreads them over the work-groups; most entries are empty:
// chunks at levels the view did not select, or culled), lists the non-empty ones in LDS and writes
// their records together.  Work-group 0 also writes the view offsets and the record count.
__global__ void __launch_bounds__(256) refine_expand_kernel(RefineArgs a, const int64_t* __restrict__ lvl_off,
                                                            const uint32_t* __restrict__ sizes,
                                                            const uint32_t* __restrict__ offs, int64_t capacity,
                                                            uint32_t* __restrict__ gather, int64_t* __restrict__ view_off,
                                                            int64_t* counts) {
  __shared__ uint32_t s_n[kExpandBatch], s_head[kExpandBatch], s_off[kExpandBatch];
  __shared__ int s_cnt;
  if (blockIdx.x == 0) refine_views(a, sizes, offs, capacity, view_off, counts);
  const int64_t C = table_chunks(a);
  const int64_t total = (int64_t)a.V * C;
  const int64_t G = gridDim.x;
  for (int64_t r0 = 0; r0 * G + blockIdx.x < total; r0 += kExpandBatch) {
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    const int64_t e = (r0 + threadIdx.x) * G + blockIdx.x;
    const uint32_t n = e < total ? sizes[e] : 0u;
    if (n) {
      const int64_t k = e - (e / C) * C;
      const int p = __float_as_int(a.bounds[k * 8 + 7]);  // a valid run: the scan kept the entry
      const int l = p % a.L;
      const int64_t start = lvl_off[p] + (k - a.chunk_off[p]) * kChunk;
      const int slot = atomicAdd(&s_cnt, 1);
      s_n[slot] = n;
      s_head[slot] = ((uint32_t)l << GS_PACKED_INDEX_BITS) | (uint32_t)start;
      s_off[slot] = offs[e];
    }
    __syncthreads();
    const int cnt = s_cnt;
    for (int j = 0; j < cnt; ++j) {
      const uint32_t nj = s_n[j], hj = s_head[j];
      const int64_t oj = s_off[j];
      for (uint32_t i = threadIdx.x; i < nj; i += blockDim.x)
        if (oj + i < capacity) gather[oj + i] = hj + i;
    }
    __syncthreads();  // s_cnt and the lists are rewritten next round
  }
}

struct RefineWs {
  uint32_t* sizes;
  uint32_t* offs;
  uint64_t* status;
  uint32_t* counter;
  int64_t status_words;
  size_t bytes;
};

RefineWs refine_ws_layout(char* base, int32_t n_views, int64_t max_chunks) {
  RefineWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  const int64_t entries = (int64_t)n_views * max_chunks;
  w.status_words = (entries + kScanTile - 1) / kScanTile + 1;
  w.sizes = (uint32_t*)take(4 * (size_t)entries);
  w.offs = (uint32_t*)take(4 * (size_t)entries);
  w.status = (uint64_t*)take(8 * (size_t)w.status_words);
  w.counter = (uint32_t*)take(256);
  w.bytes = off;
  return w;
}

}  // namespace
}  // namespace gs

extern "C" int64_t gs_chunk_capacity(const gs_gaussians* levels, const gs_blocks* blocks) {
  using namespace gs;
  if (!levels || !blocks || blocks->n_levels <= 0 || blocks->n_levels > kMaxLevels || blocks->n_blocks <= 0) return -1;
  int64_t c = (int64_t)blocks->n_blocks * blocks->n_levels;
  for (int l = 0; l < blocks->n_levels; ++l) c += (levels[l].n + GS_CHUNK - 1) / GS_CHUNK;
  return c;
}

extern "C" gs_status gs_chunk_bounds(const gs_gaussians* levels, const gs_blocks* blocks, int64_t* chunk_off,
                                     float* bounds, int64_t max_chunks, void* stream) {
  using namespace gs;
  if (!levels || !blocks || !chunk_off || !bounds || max_chunks <= 0) return GS_ERR_INVALID_ARG;
  if (blocks->n_levels <= 0 || blocks->n_levels > kMaxLevels || blocks->n_blocks <= 0 || !blocks->lvl_off ||
      !blocks->lvl_cnt)
    return GS_ERR_INVALID_ARG;
  if (max_chunks < gs_chunk_capacity(levels, blocks)) return GS_ERR_CAPACITY;
  ChunkArgs a{};
  for (int l = 0; l < blocks->n_levels; ++l) {
    const gs_gaussians& g = levels[l];
    if (g.n < 0 || (g.n > 0 && (!g.means || !g.scales))) return GS_ERR_INVALID_ARG;
    if (g.attr_half != 0 && g.attr_half != 1) return GS_ERR_INVALID_ARG;
    if (g.n >= ((int64_t)1 << GS_PACKED_INDEX_BITS)) return GS_ERR_UNSUPPORTED;  // packed gather entries
    a.lv[l] = level_ptrs(g);
  }
  a.lvl_off = blocks->lvl_off;
  a.lvl_cnt = blocks->lvl_cnt;
  a.chunk_off = chunk_off;
  a.B = blocks->n_blocks;
  a.L = blocks->n_levels;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(chunk_offsets_kernel, dim3(1), dim3(256), 0, s, blocks->lvl_cnt, a.B * a.L, chunk_off);
  const int64_t g = max_chunks < 4096 ? max_chunks : 4096;
  hipLaunchKernelGGL(chunk_bounds_kernel, dim3((unsigned)g), dim3(256), 0, s, a, max_chunks, bounds);
  GS_LAUNCH_CHECK();
  return GS_OK;
}

extern "C" size_t gs_refine_workspace_bytes(int32_t n_views, int64_t max_chunks) {
  if (n_views <= 0 || max_chunks <= 0) return 0;
  return gs::refine_ws_layout(nullptr, n_views, max_chunks).bytes;
}

extern "C" gs_status gs_lod_refine(const gs_blocks* blocks, const int8_t* level, const gs_camera* cams,
                                   int32_t n_views, int32_t width, int32_t height, const int64_t* chunk_off,
                                   const float* bounds, int64_t max_chunks, int64_t record_capacity,
                                   uint32_t* gather, int64_t* view_offsets, int64_t* counts, void* ws,
                                   size_t ws_bytes, void* stream) {
  using namespace gs;
  if (!blocks || !level || !cams || !chunk_off || !bounds || !view_offsets || !counts || !ws) return GS_ERR_INVALID_ARG;
  if (n_views <= 0 || width <= 0 || height <= 0 || width > 65535 || height > 65535 || max_chunks <= 0)
    return GS_ERR_INVALID_ARG;
  if (blocks->n_levels <= 0 || blocks->n_levels > kMaxLevels || blocks->n_blocks <= 0 || !blocks->lvl_off ||
      !blocks->lvl_cnt)
    return GS_ERR_INVALID_ARG;
  if (record_capacity < 0 || (record_capacity > 0 && !gather) || record_capacity >= ((int64_t)1 << 32))
    return GS_ERR_INVALID_ARG;
  if ((int64_t)n_views * max_chunks >= ((int64_t)1 << 31)) return GS_ERR_INVALID_ARG;
  const RefineWs w = refine_ws_layout((char*)ws, n_views, max_chunks);
  if (ws_bytes < w.bytes) return GS_ERR_WORKSPACE;
  RefineArgs a{};
  a.lvl_cnt = blocks->lvl_cnt;
  a.level = level;
  a.chunk_off = chunk_off;
  a.bounds = bounds;
  a.cams = cams;
  a.max_chunks = max_chunks;
  a.B = blocks->n_blocks;
  a.L = blocks->n_levels;
  a.V = n_views;
  a.W = width;
  a.H = height;
  hipStream_t s = (hipStream_t)stream;
  const int64_t entries = (int64_t)n_views * max_chunks;
  auto grid = [](int64_t items, int64_t cap) {
    const int64_t g = (items + 255) / 256;
    return dim3((unsigned)(g < 1 ? 1 : (g > cap ? cap : g)));
  };
  hipLaunchKernelGGL(refine_clear_kernel, grid(w.status_words, 256), dim3(256), 0, s, w.status, w.status_words,
                     w.counter);
  hipLaunchKernelGGL(refine_test_kernel, grid(entries, 4096), dim3(256), 0, s, a, w.sizes);
  hipLaunchKernelGGL(refine_scan_kernel, grid(entries / kScanItems, 1024), dim3(256), 0, s, a, w.sizes, w.offs,
                     w.status, w.counter, counts);
  const int64_t batches = (entries + kExpandBatch - 1) / kExpandBatch;
  hipLaunchKernelGGL(refine_expand_kernel, dim3((unsigned)(batches < 2048 ? (batches > 0 ? batches : 1) : 2048)),
                     dim3(256), 0, s, a, blocks->lvl_off, w.sizes, w.offs, record_capacity, gather, view_offsets,
                     counts);
  GS_LAUNCH_CHECK();
  return GS_OK;
}
