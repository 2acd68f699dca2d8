// Tile binning: (tile, depth, record) ordering of the projected Gaussians.
//
// The (tile | depth) key of every (tile, Gaussian) pair is sorted by a stable
// least-significant-digit radix sort.  Its low (depth) digits do not depend on
// the tile, so those passes run once per visible record, before the pairs are
// duplicated; only the tile digits run over the pairs.  Stages:
//   1. hist      digit histograms of the visible records' depth keys, and the
//                pairs (tiles_touched) per top digit
//   2. 4 passes  stable radix sort by the 32-bit depth key (ties keep record order);
//                the first one reads every selected record and keeps the visible
//                ones (compaction), the last one gathers each record's footprint
//                word, writes its tile rectangle (first tile id, extent) and the
//                pair offsets, the exclusive prefix of the tile counts in depth
//                order (its look-back carries both sums)
//   3. emit      one (view*tiles + tile, record) pair per tile of each footprint,
//                reading the rectangles in depth order
//   4. passes    stable radix sort by tile id (ceil(bits / 8) passes)
//   5. ranges    [start, end) of every tile
// The result equals a sort by (tile, depth, record id).
//
// The radix passes are single-pass with decoupled
// look-back: work-groups take tile ids from an atomic counter in launch order,
// publish their local aggregate, then walk back over predecessors' published
// values.  A work-group
// only waits on tiles claimed before its own, so the waits always end; each
// wait is still bounded (kSpinLimit) and raises GS_FLAG_WAIT if it gives up.
// Every device size is read from the counts array, so nothing here needs a
// host synchronisation and the whole stage can be captured in a HIP graph.
#include <mutex>

#include "radix.h"

namespace gs {
namespace {

constexpr int kMaxPasses = 8;
constexpr int kPersistentBlocks = 1024;
constexpr int kBigFootprint = 16;  // records touching more tiles are emitted cooperatively
// emit_kernel's work-groups all finish at about the same time and each adds its
// tile-digit histogram to device memory, so a single copy would take ~2000
// same-address atomics per word in a row.  They add into kTileHistCopies
// partial copies instead (copy blockIdx.x mod kTileHistCopies; copy 0 is the
// histogram the radix passes read), and emit_big_kernel, which runs next, folds
// copies 1.. into copy 0.
constexpr int kTileHistCopies = 8;
constexpr int64_t kTileHistWords = kMaxPasses * kRadix;  // one copy

// ---------------------------------------------------------------------------
// zero fill of the small fixed state (counters, histograms) and of the look-back
// words of the four depth passes, sized by the selected records (the compacting
// first pass runs over all of them; the later ones over the visible ones):
// u32 [radix tiles][4][256] and the last pass's u64 [radix tiles][256]
__global__ void clear_front_kernel(uint32_t* __restrict__ fixed, int64_t fixed_words, const int64_t* counts,
                                   int64_t cap, uint32_t* __restrict__ dstatus, uint64_t* __restrict__ pstatus) {
  const int64_t n = count_clamped(counts, GS_COUNT_RECORDS, cap);
  const int64_t rt = (n + kRadixTile - 1) / kRadixTile;
  const int64_t dwords = rt * 4 * kRadix, pwords = rt * kRadix;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < fixed_words + dwords + pwords; i += stride) {
    if (i < fixed_words) fixed[i] = 0u;
    else if (i < fixed_words + dwords) dstatus[i - fixed_words] = 0u;
    else pstatus[i - fixed_words - dwords] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// 1. histograms of the visible records' depth digits (all four passes) and of
//    their pairs by the top digit; the work-groups finish together, so their
//    device atomics are spread over kDepthHistCopies partial copies (copy 0 is
//    the histogram itself; each pass adds the others to its digit)
// ---------------------------------------------------------------------------
constexpr int kDepthHistCopies = 8;
constexpr int64_t kDepthHistWords = 4 * kRadix;

// Histogram adds of a wave whose lanes often share a digit.  Depth keys are
// float bits and a wave holds neighbouring Gaussians, so the top digit (sign and
// exponent) and the next one take a few values per wave; plain LDS atomics on
// them serialise on one address.  match_add: each lane finds the lanes with its
// digit with eight ballots (a fixed cost whatever the distribution) and the
// lowest of them adds their count.  top_add: one round per distinct top digit
// in the wave (sign and exponent of depths within a wave: one or two values),
// adding the lanes' count and their tiles_touched sum.
__device__ __forceinline__ void match_add(bool valid, uint32_t d, uint32_t* h) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int bit = 0; bit < 8; ++bit) {
    const bool b = (d >> bit) & 1u;
    const uint64_t m = __ballot(b);
    peers &= b ? m : ~m;
  }
  if (valid && lanemask_lt_count(peers) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
}

__device__ __forceinline__ void top_add(bool valid, uint32_t d, uint32_t tt, uint32_t* h, uint64_t* wh) {
  const int lane = threadIdx.x & 63;
  uint64_t left = __ballot(valid);
  while (left) {
    const int leader = (int)__builtin_ctzll(left);
    const uint32_t dl = (uint32_t)__builtin_amdgcn_readlane((int)d, leader);
    const bool mine = valid && d == dl;
    const uint64_t m = __ballot(mine);
    uint64_t v = mine ? (uint64_t)tt : 0ull;  // 64 lanes of tiles_touched may pass 2^32
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == leader) {
      atomicAdd(&h[dl], (uint32_t)__popcll(m));
      atomicAdd((unsigned long long*)&wh[dl], (unsigned long long)v);
    }
    left &= ~m;
  }
}

__global__ void __launch_bounds__(kThreads) depth_hist_kernel(const int32_t* __restrict__ tiles_touched,
                                                              const uint32_t* __restrict__ depth_keys, int64_t cap,
                                                              const int64_t* counts, uint32_t* __restrict__ hist,
                                                              uint32_t* __restrict__ hist_extra,
                                                              uint64_t* __restrict__ whist) {
  __shared__ uint32_t s_hist[4][kRadix];
  __shared__ uint64_t s_whist[kRadix];  // tiles_touched summed by the top depth digit
  const int64_t n = count_clamped(counts, GS_COUNT_RECORDS, cap);
  const int64_t per_block = (int64_t)kThreads * kItems;
  const int64_t nblocks = (n + per_block - 1) / per_block;
  if ((int64_t)blockIdx.x >= nblocks) return;
  for (int i = threadIdx.x; i < 4 * kRadix; i += kThreads) (&s_hist[0][0])[i] = 0u;
  s_whist[threadIdx.x] = 0ull;
  __syncthreads();
  for (int64_t b = blockIdx.x; b < nblocks; b += gridDim.x) {
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      const int64_t idx = b * per_block + (int64_t)k * kThreads + threadIdx.x;  // coalesced
      const int32_t tt = idx < n ? tiles_touched[idx] : 0;
      const bool vis = tt > 0;
      if (__ballot(vis) == 0) continue;  // a wave of culled records (neighbours are culled together)
      const uint32_t key = vis ? depth_keys[idx] : 0u;
      if (vis) {
        atomicAdd(&s_hist[0][key & 255u], 1u);
        atomicAdd(&s_hist[1][(key >> 8) & 255u], 1u);
      }
      match_add(vis, (key >> 16) & 255u, s_hist[2]);
      top_add(vis, key >> 24, vis ? (uint32_t)tt : 0u, s_hist[3], s_whist);
    }
  }
  __syncthreads();
  const int copy = (int)(blockIdx.x % kDepthHistCopies);
  uint32_t* h = copy == 0 ? hist : hist_extra + (int64_t)(copy - 1) * kDepthHistWords;
  for (int i = threadIdx.x; i < 4 * kRadix; i += kThreads) {
    const uint32_t c = (&s_hist[0][0])[i];
    if (c) atomicAdd(&h[i], c);
  }
  const uint64_t wv = s_whist[threadIdx.x];
  if (wv) atomicAdd((unsigned long long*)&whist[copy * kRadix + threadIdx.x], (unsigned long long)wv);
}

// ---------------------------------------------------------------------------
// 3. pair emission
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) emit_kernel(const uint32_t* __restrict__ tile_first,
                                                        const uint32_t* __restrict__ tile_extent,
                                                        const uint32_t* __restrict__ sorted_records,
                                                        const uint32_t* __restrict__ pair_off, int64_t cap,
                                                        const int64_t* counts, int64_t pair_cap, int tw, int th,
                                                        int tiles_x_n, int tiles_per_view,
                                                        uint32_t* __restrict__ out_tiles,
                                                        uint32_t* __restrict__ out_records, int tpasses,
                                                        uint32_t* __restrict__ hist, uint32_t* __restrict__ pstatus,
                                                        uint32_t* __restrict__ ranges, int64_t range_words,
                                                        uint32_t* __restrict__ big_list,
                                                        uint32_t* __restrict__ big_count,
                                                        uint32_t* __restrict__ hist_extra) {
  __shared__ uint32_t s_hist[kMaxPasses][kRadix];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // zero the look-back words of the tile passes (sized by the pair count) and the ranges
  {
    const int64_t m = count_clamped(counts, GS_COUNT_PAIRS, pair_cap);
    const int64_t words = ((m + kRadixTile - 1) / kRadixTile) * (int64_t)tpasses * kRadix;
    for (int64_t i = gtid; i < words; i += stride) pstatus[i] = 0u;
    for (int64_t i = gtid; i < range_words; i += stride) ranges[i] = 0u;
  }
  for (int i = threadIdx.x; i < tpasses * kRadix; i += kThreads) (&s_hist[0][0])[i] = 0u;
  __syncthreads();
  const int64_t n = count_clamped(counts, GS_COUNT_VISIBLE, cap);
  for (int64_t j = gtid; j < n; j += stride) {
    // the record's tile rectangle, written in this (depth) order by the last depth pass
    const uint32_t first = tile_first[j], ext = tile_extent[j];
    const int ntx = (int)(ext & 0xFFFFu), nty = (int)(ext >> 16);
    if (ntx * nty > kBigFootprint) {  // many tiles: left to emit_big_kernel
      big_list[atomicAdd(big_count, 1u)] = (uint32_t)j;
      continue;
    }
    const uint32_t rid = sorted_records[j];
    int64_t o = pair_off[j];
    for (int ty = 0; ty < nty; ++ty)
      for (int tx = 0; tx < ntx; ++tx) {
        if (o < pair_cap) {
          const uint32_t key = first + (uint32_t)(ty * tiles_x_n + tx);
          out_tiles[o] = key;
          out_records[o] = rid;
          for (int p = 0; p < tpasses; ++p) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255u], 1u);
        }
        ++o;
      }
  }
  __syncthreads();
  const int copy = (int)(blockIdx.x % kTileHistCopies);
  uint32_t* h = copy == 0 ? hist : hist_extra + (int64_t)(copy - 1) * kTileHistWords;
  for (int i = threadIdx.x; i < tpasses * kRadix; i += kThreads) {
    const uint32_t c = (&s_hist[0][0])[i];
    if (c) atomicAdd(&h[i], c);
  }
}

// Records whose footprint covers many tiles (a Gaussian close to the camera):
// one work-group per record, its tiles strided over the threads, written to
// the same slots (row-major tile order) the serial loop would use.
__global__ void __launch_bounds__(kThreads) emit_big_kernel(const uint32_t* __restrict__ tile_first,
                                                            const uint32_t* __restrict__ tile_extent,
                                                            const uint32_t* __restrict__ sorted_records,
                                                            const uint32_t* __restrict__ pair_off,
                                                            const uint32_t* __restrict__ big_list,
                                                            const uint32_t* __restrict__ big_count, int64_t pair_cap,
                                                            int tw, int th, int tiles_x_n, int tiles_per_view,
                                                            uint32_t* __restrict__ out_tiles,
                                                            uint32_t* __restrict__ out_records, int tpasses,
                                                            uint32_t* __restrict__ hist,
                                                            const uint32_t* __restrict__ hist_extra) {
  __shared__ uint32_t s_hist[kMaxPasses][kRadix];
  for (int i = threadIdx.x; i < tpasses * kRadix; i += kThreads) (&s_hist[0][0])[i] = 0u;
  // emit_kernel has finished (same stream): its partial histograms are final
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < tpasses * kRadix; i += kThreads) {
      uint32_t part[kTileHistCopies - 1];
#pragma unroll
      for (int c = 0; c < kTileHistCopies - 1; ++c) part[c] = hist_extra[c * kTileHistWords + i];
      uint32_t sum = 0;
#pragma unroll
      for (int c = 0; c < kTileHistCopies - 1; ++c) sum += part[c];
      if (sum) atomicAdd(&hist[i], sum);
    }
  }
  __syncthreads();
  const uint32_t nbig = *big_count;
  for (uint32_t k = blockIdx.x; k < nbig; k += gridDim.x) {
    const uint32_t j = big_list[k];
    const uint32_t rid = sorted_records[j];
    const uint32_t first = tile_first[j], ext = tile_extent[j];
    const int ntx = (int)(ext & 0xFFFFu), nty = (int)(ext >> 16);
    const int64_t o0 = pair_off[j];
    for (int q = threadIdx.x; q < ntx * nty; q += kThreads) {
      const int64_t o = o0 + q;
      if (o < pair_cap) {
        const int ty = q / ntx, tx = q % ntx;
        const uint32_t key = first + (uint32_t)(ty * tiles_x_n + tx);
        out_tiles[o] = key;
        out_records[o] = rid;
        for (int p = 0; p < tpasses; ++p) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255u], 1u);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < tpasses * kRadix; i += kThreads) {
    const uint32_t c = (&s_hist[0][0])[i];
    if (c) atomicAdd(&hist[i], c);
  }
}

// ---------------------------------------------------------------------------
// 5. tile ranges
// ---------------------------------------------------------------------------
__global__ void ranges_kernel(const uint32_t* __restrict__ tiles, const int64_t* counts, int64_t pair_cap,
                              int64_t n_tile_ids, uint32_t* __restrict__ ranges) {
  const int64_t m = count_clamped(counts, GS_COUNT_PAIRS, pair_cap);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
    const uint32_t k = tiles[j];
    if ((int64_t)k >= n_tile_ids) continue;  // never produced by emission; kept off the ranges array
    if (j == 0 || tiles[j - 1] != k) ranges[2 * (int64_t)k] = (uint32_t)j;
    if (j == m - 1 || tiles[j + 1] != k) ranges[2 * (int64_t)k + 1] = (uint32_t)(j + 1);
  }
}

// ---------------------------------------------------------------------------
// 6. work queue for the persistent tile kernels: tiles ordered by decreasing
//    list length, bucketed by floor(log2(length)) (empty tiles last); the order
//    inside a bucket is irrelevant because tiles are independent
// ---------------------------------------------------------------------------
constexpr int kQueueBins = 33;

__device__ __forceinline__ int queue_bin(const uint32_t* ranges, int64_t t) {
  const uint32_t len = ranges[2 * t + 1] - ranges[2 * t];
  return len == 0 ? 32 : __clz(len);  // 0 = longest (bit 31 set) ... 31 = length 1
}

__global__ void queue_hist_kernel(const uint32_t* __restrict__ ranges, int64_t n_tiles, uint32_t* __restrict__ qhist) {
  __shared__ uint32_t s_h[kQueueBins];
  for (int i = threadIdx.x; i < kQueueBins; i += blockDim.x) s_h[i] = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles; t += stride)
    atomicAdd(&s_h[queue_bin(ranges, t)], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < kQueueBins; i += blockDim.x)
    if (s_h[i]) atomicAdd(&qhist[i], s_h[i]);
}

// Each work-group ranks its tiles inside their bins with LDS atomics, then takes
// one range per non-empty bin from the global cursors: one global atomic per
// (work-group, bin) instead of one per tile (same-address atomics serialise).
__global__ void queue_scatter_kernel(const uint32_t* __restrict__ ranges, int64_t n_tiles,
                                     const uint32_t* __restrict__ qhist, uint32_t* __restrict__ qcur,
                                     uint32_t* __restrict__ queue) {
  __shared__ uint32_t s_base[kQueueBins];
  __shared__ uint32_t s_cnt[kQueueBins];
  __shared__ uint32_t s_off[kQueueBins];
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int i = 0; i < kQueueBins; ++i) {
      s_base[i] = acc;
      acc += qhist[i];
    }
    if (blockIdx.x == 0) {
      queue[0] = 0u;  // head counters of the forward and backward tile kernels
      queue[1] = 0u;
    }
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t0 = (int64_t)blockIdx.x * blockDim.x; t0 < n_tiles; t0 += stride) {
    for (int i = threadIdx.x; i < kQueueBins; i += blockDim.x) s_cnt[i] = 0u;
    __syncthreads();
    const int64_t t = t0 + threadIdx.x;
    const int bin = t < n_tiles ? queue_bin(ranges, t) : 0;
    const uint32_t rank = t < n_tiles ? atomicAdd(&s_cnt[bin], 1u) : 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < kQueueBins; i += blockDim.x)
      if (s_cnt[i]) s_off[i] = atomicAdd(&qcur[i], s_cnt[i]);
    __syncthreads();
    if (t < n_tiles) queue[2 + s_base[bin] + s_off[bin] + rank] = (uint32_t)t;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
// tile counters [64], depth + tile digit histograms [2][kMaxPasses][256], queue histogram and cursors
// [2][40], partial tile-digit histograms of emit_kernel [kTileHistCopies - 1][kMaxPasses][256], partial
// depth-digit histograms of depth_hist_kernel [kDepthHistCopies - 1][4][256]
constexpr int64_t kQueueWords = 2 * 40;
constexpr int64_t kTileExtraAt = 64 + 2 * kMaxPasses * kRadix + kQueueWords;
constexpr int64_t kDepthExtraAt = kTileExtraAt + (kTileHistCopies - 1) * kTileHistWords;
// partial histograms of tiles_touched by the top depth digit, u64 [kDepthHistCopies][256] (the last
// depth pass sums the copies)
constexpr int64_t kWhistAt = ((kDepthExtraAt + (kDepthHistCopies - 1) * kDepthHistWords) + 1) & ~(int64_t)1;
constexpr int64_t kFixedWords = kWhistAt + 2 * kDepthHistCopies * kRadix;

struct SortWs {
  uint32_t* dkeys_a;      // [rc]
  uint32_t* dvals_a;      // [rc]
  uint32_t* dkeys_b;      // [rc]
  uint32_t* dvals_b;      // [rc]
  uint32_t* pair_off;     // [rc]
  uint32_t* big_list;     // [rc] visible records with large footprints
  uint32_t* tile_extent;  // [rc] tile columns | rows << 16 per visible record, depth order
                          // (its first tile id goes to dkeys_a, free in the last depth pass)
  uint32_t* ptiles_alt;   // [pc]
  uint32_t* precs_alt;    // [pc]
  uint32_t* fixed;        // counters [64], hist [2][kMaxPasses][256], queue words, partial tile hists
  uint32_t* dstatus;      // [radix tiles][4][256] (tile-major so a prefix covers every pass; slot 3 unused)
  uint64_t* p3status;     // [radix tiles][256]: last depth pass, record count and pair sum per word
  uint32_t* pstatus;      // [ptiles][kMaxPasses][256]
  size_t bytes;
};

inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

SortWs sort_ws_layout(char* base, int64_t rc, int64_t pc) {
  SortWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return p;
  };
  const int64_t drtiles = (rc + kRadixTile - 1) / kRadixTile + 1;  // radix tiles over records
  const int64_t ptiles = (pc + kRadixTile - 1) / kRadixTile + 1;   // radix tiles over pairs
  w.dkeys_a = (uint32_t*)take(4 * (size_t)rc);
  w.dvals_a = (uint32_t*)take(4 * (size_t)rc);
  w.dkeys_b = (uint32_t*)take(4 * (size_t)rc);
  w.dvals_b = (uint32_t*)take(4 * (size_t)rc);
  w.pair_off = (uint32_t*)take(4 * (size_t)rc);
  w.big_list = (uint32_t*)take(4 * (size_t)rc);
  w.tile_extent = (uint32_t*)take(4 * (size_t)rc);
  w.ptiles_alt = (uint32_t*)take(4 * (size_t)pc);
  w.precs_alt = (uint32_t*)take(4 * (size_t)pc);
  w.fixed = (uint32_t*)take(4 * (size_t)kFixedWords);
  w.dstatus = (uint32_t*)take(4 * 4 * (size_t)drtiles * kRadix);
  w.p3status = (uint64_t*)take(8 * (size_t)drtiles * kRadix);
  w.pstatus = (uint32_t*)take(4 * (size_t)kMaxPasses * (size_t)ptiles * kRadix);
  w.bytes = off;
  return w;
}

int tile_bits(int64_t n_ids) {
  int b = 0;
  while (((int64_t)1 << b) < n_ids) ++b;
  return b;
}

}  // namespace

size_t bin_sort_ws_bytes(int64_t rc, int64_t pc) { return sort_ws_layout(nullptr, rc, pc).bytes; }

}  // namespace gs

extern "C" gs_status gs_bin_sort(const void* records, const uint32_t* depth_keys, const int32_t* tiles_touched,
                                 int32_t n_views, int32_t width, int32_t height, const gs_tuning* tuning,
                                 int64_t record_capacity, int64_t pair_capacity, uint32_t* pair_tiles,
                                 uint32_t* pair_records, uint32_t* tile_ranges, uint32_t* tile_queue,
                                 int64_t* counts, void* ws, size_t ws_bytes, void* stream) {
  using namespace gs;
  if (!records || !depth_keys || !tiles_touched || !tuning || !pair_tiles || !pair_records || !tile_ranges ||
      !counts || !ws)
    return GS_ERR_INVALID_ARG;
  if (n_views <= 0 || width <= 0 || height <= 0 || width > 65535 || height > 65535) return GS_ERR_INVALID_ARG;
  if (!tile_shape_supported(tuning->tile_w, tuning->tile_h)) return GS_ERR_UNSUPPORTED;
  if (record_capacity <= 0 || pair_capacity <= 0) return GS_ERR_INVALID_ARG;
  // look-back words carry 30-bit counts
  if (record_capacity >= ((int64_t)1 << 30) || pair_capacity >= ((int64_t)1 << 30)) return GS_ERR_INVALID_ARG;
  const SortWs w = sort_ws_layout((char*)ws, record_capacity, pair_capacity);
  if (ws_bytes < w.bytes) return GS_ERR_WORKSPACE;
  const int tw = tuning->tile_w, th = tuning->tile_h;
  const int tx_n = tiles_x(width, tw), ty_n = tiles_y(height, th);
  const int64_t tiles_per_view = (int64_t)tx_n * ty_n;
  const int64_t n_tile_ids = tiles_per_view * n_views;
  if (n_tile_ids >= ((int64_t)1 << 31)) return GS_ERR_INVALID_ARG;
  const int tbits = tile_bits(n_tile_ids);
  const int tpasses = tbits == 0 ? 0 : (tbits + 7) / 8;
  hipStream_t s = (hipStream_t)stream;
  const dim3 blk(kThreads);
  auto grid_for = [](int64_t items) {
    int64_t g = (items + kThreads - 1) / kThreads;
    return dim3((unsigned)(g < 1 ? 1 : (g > 2048 ? 2048 : g)));
  };
  auto persistent_radix = [](int64_t cap) {
    int64_t g = (cap + kRadixTile - 1) / kRadixTile;
    return dim3((unsigned)(g < 1 ? 1 : (g > kPersistentBlocks ? kPersistentBlocks : g)));
  };
  uint32_t* counters = w.fixed;
  uint32_t* dhist = w.fixed + 64;
  uint32_t* thist = w.fixed + 64 + kMaxPasses * kRadix;
  uint64_t* whist = (uint64_t*)(w.fixed + kWhistAt);
  uint32_t* dhist_extra = w.fixed + kDepthExtraAt;
  // 0. zero the counters, histograms and the depth passes' look-back words
  {
    const int64_t drt = (record_capacity + kRadixTile - 1) / kRadixTile;
    hipLaunchKernelGGL(clear_front_kernel, grid_for(kFixedWords + drt * 5 * kRadix), blk, 0, s, w.fixed,
                       kFixedWords, counts, record_capacity, w.dstatus, w.p3status);
  }
  GS_LAUNCH_CHECK();
  // 1. histograms of the four depth digits and of the pairs by the top digit
  hipLaunchKernelGGL(depth_hist_kernel, grid_for((record_capacity + kItems - 1) / kItems), blk, 0, s, tiles_touched,
                     depth_keys, record_capacity, counts, dhist, dhist_extra, whist);
  GS_LAUNCH_CHECK();
  // 2. depth sort, 4 passes of 8 bits: selected records -> b -> a -> b -> a.  The first pass keeps
  //    the visible records (index order within a digit) and writes counts[GS_COUNT_VISIBLE]; the
  //    last also writes the pair offsets (exclusive prefix of tiles_touched in depth order) and
  //    counts[GS_COUNT_PAIRS].  Each pass adds the partial copies of its digit histogram.
  const int tw_shift = __builtin_ctz((unsigned)tw), th_shift = __builtin_ctz((unsigned)th);  // powers of two
  auto extra = [&](int p, const uint64_t* wh, uint64_t* pst, uint32_t* poff) {
    return PairPass{tiles_touched, (const uint4*)records, tw_shift, th_shift, tx_n, (int)tiles_per_view,
                    w.dkeys_a, w.tile_extent, wh, kDepthHistCopies, pst, poff, pair_capacity,
                    dhist_extra + p * kRadix, kDepthHistCopies - 1, kDepthHistWords};
  };
  hipLaunchKernelGGL((radix_pass_kernel<kPassCompact>), persistent_radix(record_capacity), blk, 0, s, depth_keys,
                     nullptr, w.dkeys_b, w.dvals_b, counts, GS_COUNT_RECORDS, record_capacity, 0, dhist,
                     w.dstatus, (int64_t)4 * kRadix, counters + 1, counts, extra(0, nullptr, nullptr, nullptr));
  hipLaunchKernelGGL((radix_pass_kernel<kPassPlain>), persistent_radix(record_capacity), blk, 0, s, w.dkeys_b,
                     w.dvals_b, w.dkeys_a, w.dvals_a, counts, GS_COUNT_VISIBLE, record_capacity, 8, dhist + kRadix,
                     w.dstatus + kRadix, (int64_t)4 * kRadix, counters + 2, counts, extra(1, nullptr, nullptr, nullptr));
  hipLaunchKernelGGL((radix_pass_kernel<kPassPlain>), persistent_radix(record_capacity), blk, 0, s, w.dkeys_a,
                     w.dvals_a, w.dkeys_b, w.dvals_b, counts, GS_COUNT_VISIBLE, record_capacity, 16,
                     dhist + 2 * kRadix, w.dstatus + 2 * kRadix, (int64_t)4 * kRadix, counters + 3, counts,
                     extra(2, nullptr, nullptr, nullptr));
  hipLaunchKernelGGL((radix_pass_kernel<kPassPairs>), persistent_radix(record_capacity), blk, 0, s, w.dkeys_b,
                     w.dvals_b, w.dkeys_a, w.dvals_a, counts, GS_COUNT_VISIBLE, record_capacity, 24,
                     dhist + 3 * kRadix, nullptr, (int64_t)0, counters + 4, counts,
                     extra(3, whist, w.p3status, w.pair_off));
  GS_LAUNCH_CHECK();
  // 3. emission (+ tile-digit histograms, + zeroing of the tile-pass state and ranges), into the
  //    buffer that the last tile pass will read last
  uint32_t* em_tiles = (tpasses % 2 == 0) ? pair_tiles : w.ptiles_alt;
  uint32_t* em_recs = (tpasses % 2 == 0) ? pair_records : w.precs_alt;
  uint32_t* big_count = counters + 32;
  uint32_t* thist_extra = w.fixed + kTileExtraAt;
  hipLaunchKernelGGL(emit_kernel, grid_for(record_capacity), blk, 0, s, w.dkeys_a, w.tile_extent, w.dvals_a, w.pair_off,
                     record_capacity, counts, pair_capacity, tw, th, tx_n, (int)tiles_per_view, em_tiles, em_recs,
                     tpasses, thist, w.pstatus, tile_ranges, 2 * n_tile_ids, w.big_list, big_count, thist_extra);
  hipLaunchKernelGGL(emit_big_kernel, dim3(256), blk, 0, s, w.dkeys_a, w.tile_extent, w.dvals_a, w.pair_off, w.big_list,
                     big_count, pair_capacity, tw, th, tx_n, (int)tiles_per_view, em_tiles, em_recs, tpasses, thist,
                     thist_extra);
  GS_LAUNCH_CHECK();
  // 4. tile passes
  uint32_t* kin = em_tiles;
  uint32_t* vin = em_recs;
  for (int p = 0; p < tpasses; ++p) {
    uint32_t* kout = (kin == pair_tiles) ? w.ptiles_alt : pair_tiles;
    uint32_t* vout = (vin == pair_records) ? w.precs_alt : pair_records;
    hipLaunchKernelGGL((radix_pass_kernel<kPassPlain>), persistent_radix(pair_capacity), blk, 0, s, kin, vin, kout, vout,
                       counts, GS_COUNT_PAIRS, pair_capacity, 8 * p, thist + p * kRadix, w.pstatus + p * kRadix,
                       (int64_t)tpasses * kRadix, counters + 16 + p, counts, PairPass{});
    GS_LAUNCH_CHECK();
    kin = kout;
    vin = vout;
  }
  // 5. ranges
  hipLaunchKernelGGL(ranges_kernel, dim3(2048), blk, 0, s, pair_tiles, counts, pair_capacity, n_tile_ids,
                     tile_ranges);
  GS_LAUNCH_CHECK();
  // 6. work queue
  if ((tuning->flags & GS_TUNE_WORK_QUEUE) && tile_queue) {
    uint32_t* qhist = w.fixed + 64 + 2 * kMaxPasses * kRadix;
    uint32_t* qcur = qhist + 40;
    hipLaunchKernelGGL(queue_hist_kernel, grid_for(n_tile_ids), blk, 0, s, tile_ranges, n_tile_ids, qhist);
    hipLaunchKernelGGL(queue_scatter_kernel, grid_for(n_tile_ids), blk, 0, s, tile_ranges, n_tile_ids, qhist, qcur,
                       tile_queue);
    GS_LAUNCH_CHECK();
  }
  return GS_OK;
}

// ---------------------------------------------------------------------------
// Variant of gs_bin_sort for callers that cannot allocate: its workspace is a
// file-scope device array.  Host code only ever uses the address that
// hipGetSymbolAddress reports for the current device (the array's own name is
// a host-side stand-in, not a device address).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[GS_STATIC_SCRATCH_BYTES];

namespace gs {
namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per device.
gs_status static_scratch(void** out) {
  int dev = -1;
  GS_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return GS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    GS_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return GS_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}

}  // namespace
}  // namespace gs

extern "C" gs_status gs_bin_sort_static(const void* records, const uint32_t* depth_keys,
                                        const int32_t* tiles_touched, int32_t n_views, int32_t width, int32_t height,
                                        const gs_tuning* tuning, int64_t record_capacity, int64_t pair_capacity,
                                        uint32_t* pair_tiles, uint32_t* pair_records, uint32_t* tile_ranges,
                                        uint32_t* tile_queue, int64_t* counts, void* stream) {
  // the checks gs_bin_sort makes without a workspace come first, so a bad call
  // fails the same way before the scratch array is looked up
  if (!records || !depth_keys || !tiles_touched || !tuning || !pair_tiles || !pair_records || !tile_ranges ||
      !counts)
    return GS_ERR_INVALID_ARG;
  if (record_capacity <= 0 || pair_capacity <= 0) return GS_ERR_INVALID_ARG;
  if (record_capacity >= ((int64_t)1 << 30) || pair_capacity >= ((int64_t)1 << 30)) return GS_ERR_INVALID_ARG;
  if (gs::bin_sort_ws_bytes(record_capacity, pair_capacity) > (size_t)GS_STATIC_SCRATCH_BYTES)
    return GS_ERR_SCRATCH;
  void* ws = nullptr;
  const gs_status st = gs::static_scratch(&ws);
  if (st != GS_OK) return st;
  return gs_bin_sort(records, depth_keys, tiles_touched, n_views, width, height, tuning, record_capacity,
                     pair_capacity, pair_tiles, pair_records, tile_ranges, tile_queue, counts, ws,
                     (size_t)GS_STATIC_SCRATCH_BYTES, stream);
}
