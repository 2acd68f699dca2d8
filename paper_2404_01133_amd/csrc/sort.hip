// Tile binning: (tile, depth, record) ordering of the projected Gaussians.
//
// The (tile | depth) key of every (tile, Gaussian) pair is sorted by a stable
// least-significant-digit radix sort.  Its low (depth) digits do not depend on
// the tile, so those passes run once per visible record, before the pairs are
// duplicated; only the tile digits run over the pairs.  Stages:
//   1. compact   visible records -> (depth bits, record id), record order kept
//                (per-tile counts, one-work-group scan, write: three launches)
//   2. 4 passes  stable radix sort by the 32-bit depth key (ties keep record order)
//   3. scan      pair offsets = exclusive prefix of tiles_touched in depth order
//   4. emit      one (view*tiles + tile, record) pair per tile of each footprint
//   5. passes    stable radix sort by tile id (ceil(bits / 8) passes)
//   6. ranges    [start, end) of every tile
// The result equals a sort by (tile, depth, record id).
//
// The pair-offset scan and the radix passes are single-pass with decoupled
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
// tiles of the two record scans (compaction, pair offsets): 2048 records;
// measured, 4x larger tiles were slower (less parallel work)
constexpr int kScanItems = kItems;
constexpr int kScanTile = kThreads * kScanItems;
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
// zero fill of the small fixed state (counters, histograms); the look-back
// words of the pair-offset scan and the depth passes are cleared by
// compact_write_kernel, sized by the visible count
// ---------------------------------------------------------------------------
__global__ void clear_front_kernel(uint32_t* __restrict__ fixed, int64_t fixed_words) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < fixed_words; i += stride) fixed[i] = 0u;
}

// ---------------------------------------------------------------------------
// 1. compaction of visible records, in three launches (count, scan, write).
//    Each scan tile's work is small and all tiles are in flight at once, so a
//    single pass with decoupled look-back spends most of its time in look-back
//    rounds and in the same-address tile counter; here tile t's offset is the
//    prefix of the tile counts, computed by one work-group.
// ---------------------------------------------------------------------------
constexpr int kDepthHistCopies = 8;  // partial depth-digit histograms of the count launch (folded by the scan)
constexpr int64_t kDepthHistWords = 4 * kRadix;

__device__ __forceinline__ int64_t scan_tiles_of(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

// per tile: number of visible records; depth-digit histograms of their keys
__global__ void __launch_bounds__(kThreads) compact_count_kernel(const int32_t* __restrict__ tiles_touched,
                                                                 const uint32_t* __restrict__ depth_keys, int64_t cap,
                                                                 const int64_t* counts,
                                                                 uint32_t* __restrict__ tile_count,
                                                                 uint32_t* __restrict__ hist,
                                                                 uint32_t* __restrict__ hist_extra) {
  __shared__ uint32_t s_wave[kThreads / 64];
  __shared__ uint32_t s_hist[4][kRadix];
  const int64_t n = count_clamped(counts, GS_COUNT_RECORDS, cap);
  const int64_t ntiles = scan_tiles_of(n);
  if ((int64_t)blockIdx.x >= ntiles) return;
  for (int i = threadIdx.x; i < 4 * kRadix; i += kThreads) (&s_hist[0][0])[i] = 0u;
  __syncthreads();
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t base = t * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t idx = base + k;
      if (idx < n && tiles_touched[idx] > 0) {
        ++mine;
        const uint32_t key = depth_keys[idx];
#pragma unroll
        for (int p = 0; p < 4; ++p) atomicAdd(&s_hist[p][(key >> (8 * p)) & 255u], 1u);
      }
    }
    uint32_t total;
    block_excl_scan(mine, s_wave, &total);
    if (threadIdx.x == 0) tile_count[t] = total;
  }
  __syncthreads();
  // the work-groups finish together: spread their histogram atomics over the copies
  const int copy = (int)(blockIdx.x % kDepthHistCopies);
  uint32_t* h = copy == 0 ? hist : hist_extra + (int64_t)(copy - 1) * kDepthHistWords;
  for (int i = threadIdx.x; i < 4 * kRadix; i += kThreads) {
    const uint32_t c = (&s_hist[0][0])[i];
    if (c) atomicAdd(&h[i], c);
  }
}

// one work-group: exclusive prefix of the tile counts, the visible count, and
// the partial depth histograms folded into the one the radix passes read
__global__ void __launch_bounds__(kThreads) compact_scan_kernel(int64_t cap, int64_t* counts,
                                                                const uint32_t* __restrict__ tile_count,
                                                                uint32_t* __restrict__ tile_off,
                                                                uint32_t* __restrict__ hist,
                                                                const uint32_t* __restrict__ hist_extra) {
  constexpr int kPer = 4;  // consecutive tiles per thread and round
  __shared__ uint32_t s_wave[kThreads / 64];
  const int64_t n = count_clamped(counts, GS_COUNT_RECORDS, cap);
  const int64_t ntiles = scan_tiles_of(n);
  uint32_t carry = 0;
  for (int64_t b = 0; b < ntiles; b += (int64_t)kThreads * kPer) {
    const int64_t t0 = b + (int64_t)threadIdx.x * kPer;
    uint32_t c[kPer], mine = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      c[k] = (t0 + k < ntiles) ? tile_count[t0 + k] : 0u;
      mine += c[k];
    }
    uint32_t tot;
    uint32_t off = carry + block_excl_scan(mine, s_wave, &tot);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      if (t0 + k < ntiles) tile_off[t0 + k] = off;
      off += c[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) counts[GS_COUNT_VISIBLE] = (int64_t)carry;
  // the count launch has finished (same stream): its partial histograms are final
  for (int i = threadIdx.x; i < kDepthHistWords; i += kThreads) {
    uint32_t part[kDepthHistCopies - 1];
#pragma unroll
    for (int k = 0; k < kDepthHistCopies - 1; ++k) part[k] = hist_extra[k * kDepthHistWords + i];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kDepthHistCopies - 1; ++k) sum += part[k];
    hist[i] += sum;
  }
}

// per tile: visible records' (depth key, record index) at the tile's offset, in index order
__global__ void __launch_bounds__(kThreads) compact_write_kernel(const int32_t* __restrict__ tiles_touched,
                                                                 const uint32_t* __restrict__ depth_keys, int64_t cap,
                                                                 const int64_t* counts,
                                                                 const uint32_t* __restrict__ tile_off,
                                                                 uint32_t* __restrict__ keys_out,
                                                                 uint32_t* __restrict__ vals_out,
                                                                 uint32_t* __restrict__ poff_status,
                                                                 uint32_t* __restrict__ dstatus) {
  __shared__ uint32_t s_wave[kThreads / 64];
  const int64_t n = count_clamped(counts, GS_COUNT_RECORDS, cap);
  const int64_t ntiles = scan_tiles_of(n);
  {
    // look-back words of the stages that run over the visible records: the
    // pair-offset scan (one u64 per scan tile, + 1) and the four depth passes
    const int64_t nv = count_clamped(counts, GS_COUNT_VISIBLE, cap);
    const int64_t pwords = 2 * (scan_tiles_of(nv) + 1);
    const int64_t dwords = ((nv + kRadixTile - 1) / kRadixTile) * 4 * kRadix;  // [radix tiles][4 passes][256]
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < pwords + dwords; i += stride) {
      if (i < pwords) poff_status[i] = 0u;
      else dstatus[i - pwords] = 0u;
    }
  }
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t base = t * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const uint32_t tbase = tile_off[t];
    bool f[kScanItems];
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t idx = base + k;
      f[k] = idx < n && tiles_touched[idx] > 0;
      mine += f[k] ? 1u : 0u;
    }
    uint32_t total;
    uint32_t pos = tbase + block_excl_scan(mine, s_wave, &total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      if (f[k]) {
        const int64_t idx = base + k;
        keys_out[pos] = depth_keys[idx];
        vals_out[pos] = (uint32_t)idx;
        ++pos;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 3. pair offsets: exclusive prefix of tiles_touched in depth order
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) pair_offsets_kernel(const uint32_t* __restrict__ sorted_records,
                                                                const int32_t* __restrict__ tiles_touched,
                                                                int64_t cap, uint32_t* __restrict__ pair_off,
                                                                uint64_t* status, uint32_t* tile_counter,
                                                                int64_t* counts, int64_t pair_cap) {
  __shared__ uint32_t s_wave[kThreads / 64];
  __shared__ uint32_t s_tile;
  __shared__ uint64_t s_excl;
  const int64_t n = count_clamped(counts, GS_COUNT_VISIBLE, cap);
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (n == 0 && blockIdx.x == 0 && threadIdx.x == 0) counts[GS_COUNT_PAIRS] = 0;
  if ((int64_t)blockIdx.x >= ntiles) return;
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
    __syncthreads();
    const int64_t t = s_tile;
    if (t >= ntiles) break;
    const int64_t base = t * kScanTile + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t idx = base + k;
      v[k] = idx < n ? (uint32_t)tiles_touched[sorted_records[idx]] : 0u;
      mine += v[k];
    }
    uint32_t total;
    const uint32_t excl_thread = block_excl_scan(mine, s_wave, &total);
    if (threadIdx.x < 64) {
      const uint64_t ex = lookback64_wave(status, t, total, counts);
      if (threadIdx.x == 0) {
        s_excl = ex;
        if (t == ntiles - 1) {
          const int64_t m = (int64_t)(ex + total);
          counts[GS_COUNT_PAIRS] = m;
          if (m > pair_cap) raise_flag(counts, GS_FLAG_PAIRS);
        }
      }
    }
    __syncthreads();
    uint64_t pos = s_excl + excl_thread;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
      const int64_t idx = base + k;
      if (idx < n) pair_off[idx] = (uint32_t)(pos < 0xFFFFFFFFull ? pos : 0xFFFFFFFFull);
      pos += v[k];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 4. pair emission
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) emit_kernel(const Record* __restrict__ records,
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
    const uint32_t rid = sorted_records[j];
    const uint4 w0 = *reinterpret_cast<const uint4*>(&records[rid]);
    const uint32_t view = reinterpret_cast<const uint32_t*>(&records[rid])[11];
    const int i0 = (int)(w0.z & 0xFFFFu), i1 = i0 + (int)(w0.z >> 16);
    const int j0 = (int)(w0.w & 0xFFFFu), j1 = j0 + (int)(w0.w >> 16);
    const int ntx = i1 / tw - i0 / tw + 1, nty = j1 / th - j0 / th + 1;
    if (ntx * nty > kBigFootprint) {  // many tiles: left to emit_big_kernel
      big_list[atomicAdd(big_count, 1u)] = (uint32_t)j;
      continue;
    }
    int64_t o = pair_off[j];
    const uint32_t vbase = view * (uint32_t)tiles_per_view;
    for (int ty = j0 / th; ty <= j1 / th; ++ty)
      for (int tx = i0 / tw; tx <= i1 / tw; ++tx) {
        if (o < pair_cap) {
          const uint32_t key = vbase + (uint32_t)(ty * tiles_x_n + tx);
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
__global__ void __launch_bounds__(kThreads) emit_big_kernel(const Record* __restrict__ records,
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
    const uint4 w0 = *reinterpret_cast<const uint4*>(&records[rid]);
    const uint32_t view = reinterpret_cast<const uint32_t*>(&records[rid])[11];
    const int i0 = (int)(w0.z & 0xFFFFu), i1 = i0 + (int)(w0.z >> 16);
    const int j0 = (int)(w0.w & 0xFFFFu), j1 = j0 + (int)(w0.w >> 16);
    const int tx0 = i0 / tw, ty0 = j0 / th;
    const int ntx = i1 / tw - tx0 + 1, nty = j1 / th - ty0 + 1;
    const int64_t o0 = pair_off[j];
    const uint32_t vbase = view * (uint32_t)tiles_per_view;
    for (int q = threadIdx.x; q < ntx * nty; q += kThreads) {
      const int64_t o = o0 + q;
      if (o < pair_cap) {
        const int ty = ty0 + q / ntx, tx = tx0 + q % ntx;
        const uint32_t key = vbase + (uint32_t)(ty * tiles_x_n + tx);
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
// 6. tile ranges
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
// 7. work queue for the persistent tile kernels: tiles ordered by decreasing
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
// depth-digit histograms of compact_count_kernel [kDepthHistCopies - 1][4][256]
constexpr int64_t kQueueWords = 2 * 40;
constexpr int64_t kTileExtraAt = 64 + 2 * kMaxPasses * kRadix + kQueueWords;
constexpr int64_t kDepthExtraAt = kTileExtraAt + (kTileHistCopies - 1) * kTileHistWords;
constexpr int64_t kFixedWords = kDepthExtraAt + (kDepthHistCopies - 1) * kDepthHistWords;

struct SortWs {
  uint32_t* dkeys_a;      // [rc]
  uint32_t* dvals_a;      // [rc]
  uint32_t* dkeys_b;      // [rc]
  uint32_t* dvals_b;      // [rc]
  uint32_t* pair_off;     // [rc]
  uint32_t* big_list;     // [rc] visible records with large footprints
  uint32_t* ptiles_alt;   // [pc]
  uint32_t* precs_alt;    // [pc]
  uint32_t* fixed;        // counters [64], hist [2][kMaxPasses][256], queue words, partial tile hists
  uint64_t* scan_status;  // [2][rtiles]: compaction tile counts and offsets (u32), pair-offset look-back
  uint32_t* dstatus;      // [radix tiles][4][256] (tile-major so a prefix covers every pass)
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
  const int64_t rtiles = (rc + kTile - 1) / kTile + 1;            // scan tiles
  const int64_t drtiles = (rc + kRadixTile - 1) / kRadixTile + 1;  // radix tiles over records
  const int64_t ptiles = (pc + kRadixTile - 1) / kRadixTile + 1;   // radix tiles over pairs
  w.dkeys_a = (uint32_t*)take(4 * (size_t)rc);
  w.dvals_a = (uint32_t*)take(4 * (size_t)rc);
  w.dkeys_b = (uint32_t*)take(4 * (size_t)rc);
  w.dvals_b = (uint32_t*)take(4 * (size_t)rc);
  w.pair_off = (uint32_t*)take(4 * (size_t)rc);
  w.big_list = (uint32_t*)take(4 * (size_t)rc);
  w.ptiles_alt = (uint32_t*)take(4 * (size_t)pc);
  w.precs_alt = (uint32_t*)take(4 * (size_t)pc);
  w.fixed = (uint32_t*)take(4 * (size_t)kFixedWords);
  // the two scan status arrays are adjacent: [rtiles] then [rtiles]
  w.scan_status = (uint64_t*)take(8 * 2 * (size_t)rtiles);
  w.dstatus = (uint32_t*)take(4 * 4 * (size_t)drtiles * kRadix);
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
  const int64_t rtiles = (record_capacity + kTile - 1) / kTile + 1;
  const dim3 blk(kThreads);
  auto grid_for = [](int64_t items) {
    int64_t g = (items + kThreads - 1) / kThreads;
    return dim3((unsigned)(g < 1 ? 1 : (g > 2048 ? 2048 : g)));
  };
  auto persistent = [](int64_t cap) {
    int64_t g = (cap + kTile - 1) / kTile;
    return dim3((unsigned)(g < 1 ? 1 : (g > kPersistentBlocks ? kPersistentBlocks : g)));
  };
  auto persistent_radix = [](int64_t cap) {
    int64_t g = (cap + kRadixTile - 1) / kRadixTile;
    return dim3((unsigned)(g < 1 ? 1 : (g > kPersistentBlocks ? kPersistentBlocks : g)));
  };
  uint32_t* counters = w.fixed;
  uint32_t* dhist = w.fixed + 64;
  uint32_t* thist = w.fixed + 64 + kMaxPasses * kRadix;
  // 0. zero the counters and histograms
  hipLaunchKernelGGL(clear_front_kernel, grid_for(kFixedWords), blk, 0, s, w.fixed, kFixedWords);
  GS_LAUNCH_CHECK();
  // 1. compaction (+ histograms of the four depth digits)
  {
    uint32_t* tile_count = (uint32_t*)w.scan_status;  // [rtiles], then tile_off [rtiles]
    uint32_t* tile_off = tile_count + rtiles;
    uint32_t* dhist_extra = w.fixed + kDepthExtraAt;
    const dim3 cgrid = grid_for((int64_t)kThreads * ((record_capacity + kScanTile - 1) / kScanTile));
    hipLaunchKernelGGL(compact_count_kernel, cgrid, blk, 0, s, tiles_touched, depth_keys, record_capacity, counts,
                       tile_count, dhist, dhist_extra);
    hipLaunchKernelGGL(compact_scan_kernel, dim3(1), blk, 0, s, record_capacity, counts, tile_count, tile_off, dhist,
                       dhist_extra);
    hipLaunchKernelGGL(compact_write_kernel, cgrid, blk, 0, s, tiles_touched, depth_keys, record_capacity, counts,
                       tile_off, w.dkeys_a, w.dvals_a, (uint32_t*)(w.scan_status + rtiles), w.dstatus);
  }
  GS_LAUNCH_CHECK();
  // 2. depth sort, 4 passes of 8 bits: a -> b -> a -> b -> a
  for (int p = 0; p < 4; ++p) {
    const bool even = (p % 2) == 0;
    hipLaunchKernelGGL(radix_pass_kernel, persistent_radix(record_capacity), blk, 0, s, even ? w.dkeys_a : w.dkeys_b,
                       even ? w.dvals_a : w.dvals_b, even ? w.dkeys_b : w.dkeys_a, even ? w.dvals_b : w.dvals_a,
                       counts, GS_COUNT_VISIBLE, record_capacity, 8 * p, dhist + p * kRadix, w.dstatus + p * kRadix,
                       (int64_t)4 * kRadix, counters + 1 + p, counts);
    GS_LAUNCH_CHECK();
  }
  // 3. pair offsets in depth order
  hipLaunchKernelGGL(pair_offsets_kernel, persistent(record_capacity), blk, 0, s, w.dvals_a, tiles_touched,
                     record_capacity, w.pair_off, w.scan_status + rtiles, counters + 8, counts, pair_capacity);
  GS_LAUNCH_CHECK();
  // 4. emission (+ tile-digit histograms, + zeroing of the tile-pass state and ranges), into the
  //    buffer that the last tile pass will read last
  uint32_t* em_tiles = (tpasses % 2 == 0) ? pair_tiles : w.ptiles_alt;
  uint32_t* em_recs = (tpasses % 2 == 0) ? pair_records : w.precs_alt;
  uint32_t* big_count = counters + 32;
  uint32_t* thist_extra = w.fixed + kTileExtraAt;
  hipLaunchKernelGGL(emit_kernel, grid_for(record_capacity), blk, 0, s, (const Record*)records, w.dvals_a, w.pair_off,
                     record_capacity, counts, pair_capacity, tw, th, tx_n, (int)tiles_per_view, em_tiles, em_recs,
                     tpasses, thist, w.pstatus, tile_ranges, 2 * n_tile_ids, w.big_list, big_count, thist_extra);
  hipLaunchKernelGGL(emit_big_kernel, dim3(256), blk, 0, s, (const Record*)records, w.dvals_a, w.pair_off, w.big_list,
                     big_count, pair_capacity, tw, th, tx_n, (int)tiles_per_view, em_tiles, em_recs, tpasses, thist,
                     thist_extra);
  GS_LAUNCH_CHECK();
  // 5. tile passes
  uint32_t* kin = em_tiles;
  uint32_t* vin = em_recs;
  for (int p = 0; p < tpasses; ++p) {
    uint32_t* kout = (kin == pair_tiles) ? w.ptiles_alt : pair_tiles;
    uint32_t* vout = (vin == pair_records) ? w.precs_alt : pair_records;
    hipLaunchKernelGGL(radix_pass_kernel, persistent_radix(pair_capacity), blk, 0, s, kin, vin, kout, vout, counts,
                       GS_COUNT_PAIRS, pair_capacity, 8 * p, thist + p * kRadix, w.pstatus + p * kRadix,
                       (int64_t)tpasses * kRadix, counters + 16 + p, counts);
    GS_LAUNCH_CHECK();
    kin = kout;
    vin = vout;
  }
  // 6. ranges
  hipLaunchKernelGGL(ranges_kernel, dim3(2048), blk, 0, s, pair_tiles, counts, pair_capacity, n_tile_ids,
                     tile_ranges);
  GS_LAUNCH_CHECK();
  // 7. work queue
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
