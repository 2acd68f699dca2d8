// Stable single-pass LSD radix pass over 8-bit digits (onesweep style), shared
// by the tile binning and the block partition.  Work-groups take tiles of
// kRadixTile keys from an atomic counter in launch order, rank their keys with
// wave64 ballot multisplit, publish per-digit tile counts and walk back over
// the predecessors' published counts (decoupled look-back), then scatter
// through LDS so the global writes of each digit run are contiguous.
#pragma once

#include "scan.h"

namespace gs {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;  // 2048 elements per scan tile
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kThreads * kRadixItems;  // 4096 keys per radix tile
constexpr int kRadix = 256;
constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 2u << 30;
constexpr uint32_t kValMask = (1u << 30) - 1;
constexpr int kLookWindow = 8;  // look-back words read per round by one digit's thread

// ---------------------------------------------------------------------------
// block-level exclusive scan of one u32 per thread (256 threads, 4 waves)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t x, uint32_t* s_wave, uint32_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = x;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) s_wave[wid] = inc;
  __syncthreads();
  uint32_t wave_base = 0, tot = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    const uint32_t s = s_wave[w];
    if (w < wid) wave_base += s;
    tot += s;
  }
  *total = tot;
  __syncthreads();
  return wave_base + inc - x;
}

// saturating u32 sum (values past 2^32 - 1 only ever mean "beyond every capacity")
__device__ __forceinline__ uint32_t sat_add(uint32_t a, uint32_t b) {
  const uint32_t c = a + b;
  return c < a ? 0xFFFFFFFFu : c;
}
__device__ __forceinline__ uint32_t sat_u32(uint64_t v) { return v > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)v; }

// block-level exclusive scan of one u64 per thread (256 threads, 4 waves)
__device__ __forceinline__ uint64_t block_excl_scan64(uint64_t x, uint64_t* s_wave64, uint64_t* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint64_t inc = x;
  for (int off = 1; off < 64; off <<= 1) {
    const uint64_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) s_wave64[wid] = inc;
  __syncthreads();
  uint64_t wave_base = 0, tot = 0;
  for (int w = 0; w < kThreads / 64; ++w) {
    const uint64_t v = s_wave64[w];
    if (w < wid) wave_base += v;
    tot += v;
  }
  *total = tot;
  __syncthreads();
  return wave_base + inc - x;
}

// Variants of a pass (template argument MODE):
//   kPassPlain    sort (key, value) pairs
//   kPassPairs    the most significant depth pass of the binning: besides the
//                 sorted record ids it writes each record's first pair slot, the
//                 exclusive prefix of tiles_touched in the sorted order
//                 (saturating at 2^32 - 1).  Per (radix tile, digit) one 64-bit
//                 look-back word carries both the record count (bits 32..61) and
//                 the pair sum (bits 0..31, saturating).  whist holds `copies`
//                 partial histograms of tiles_touched by this digit (u64).
//                 A record's tile rectangle comes from its footprint word (the
//                 first 16 bytes of its record, gathered once here): the pass
//                 also writes, in the sorted order, its first tile id (view *
//                 tiles per view + row * tiles_x + column) and its extent in
//                 tiles (columns | rows << 16), so the emission reads them in
//                 order instead of gathering every record again.
//   kPassCompact  the least significant depth pass: reads every selected record's
//                 depth key, keeps those with tiles_touched > 0 (values = record
//                 index, in index order) and writes the visible count.
// hist_extra: `hist_copies` further partial copies of the digit histogram
// (stride hist_stride) that the pass adds to `hist` itself.
constexpr int kPassPlain = 0;
constexpr int kPassPairs = 1;
constexpr int kPassCompact = 2;
struct PairPass {
  const int32_t* tiles_touched;  // kPassCompact
  const uint4* rec_words;        // kPassPairs: records as 16-byte words, kRecordWords per record
  int tw_shift, th_shift;        // log2 of the tile shape (every supported shape is a power of two)
  int tiles_x, tiles_per_view;
  uint32_t* tile_first;          // [visible] first tile id, sorted order
  uint32_t* tile_extent;         // [visible] columns | rows << 16, sorted order
  const uint64_t* whist;
  int copies;
  uint64_t* status;  // [radix tiles][256]
  uint32_t* pair_off;
  int64_t pair_cap;
  const uint32_t* hist_extra;
  int hist_copies;
  int64_t hist_stride;
};
constexpr uint64_t kPFlagAgg = 1ull << 62;
constexpr uint64_t kPFlagInc = 2ull << 62;
constexpr uint64_t kPFlagMask = 3ull << 62;

// ---------------------------------------------------------------------------
// one stable LSD pass over 8 bits; the digit histogram of the whole input was
// accumulated by the kernel that produced the keys
// ---------------------------------------------------------------------------
template <int MODE = kPassPlain>
__global__ void __launch_bounds__(kThreads) radix_pass_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const int64_t* counts_in, int count_idx, int64_t cap, int shift,
    const uint32_t* __restrict__ hist, uint32_t* status, int64_t status_stride, uint32_t* tile_counter,
    int64_t* counts, PairPass pp) {
  __shared__ uint32_t s_keys[kRadixTile];
  __shared__ uint32_t s_vals[kRadixTile];
  __shared__ uint32_t s_wave_hist[kThreads / 64][kRadix];
  __shared__ uint32_t s_tile_excl[kRadix];
  __shared__ uint32_t s_digit_base[kRadix];
  __shared__ uint32_t s_wave[kThreads / 64];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_goff[kRadix];
  // kPassPairs only (sized 1 otherwise): tiles_touched, then its exclusive prefix, in LDS
  // order; the first pair slot of each digit's run of this tile; the prefix at each run start
  __shared__ uint32_t s_pfx[MODE == kPassPairs ? kRadixTile : 1];
  __shared__ uint32_t s_pbase[MODE == kPassPairs ? kRadix : 1];
  __shared__ uint32_t s_pfx_start[MODE == kPassPairs ? kRadix : 1];
  __shared__ uint64_t s_wave64[MODE == kPassPairs ? kThreads / 64 : 1];
  __shared__ uint32_t s_ptotal;
  constexpr bool PAIRS = MODE == kPassPairs;
  constexpr bool COMPACT = MODE == kPassCompact;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t n = count_clamped(counts_in, count_idx, cap);
  const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  // this digit's count over the whole input: `hist` plus the partial copies
  uint32_t hist_d = hist[threadIdx.x];
  for (int c = 0; c < pp.hist_copies; ++c) hist_d += pp.hist_extra[c * pp.hist_stride + threadIdx.x];
  if constexpr (COMPACT) {
    // the visible count = the digit histogram's total (taken by the later passes)
    if (blockIdx.x == 0) {
      uint32_t tot;
      block_excl_scan(hist_d, s_wave, &tot);
      if (threadIdx.x == 0) counts[GS_COUNT_VISIBLE] = (int64_t)tot;
    }
  }
  if constexpr (PAIRS) {
    // the pair count M = sum of tiles_touched over the visible records, from the weighted histogram
    if (blockIdx.x == 0) {
      uint64_t w = 0;
      for (int c = 0; c < pp.copies; ++c) w += pp.whist[c * kRadix + threadIdx.x];
      uint64_t tot;
      block_excl_scan64(w, s_wave64, &tot);
      if (threadIdx.x == 0) {
        counts[GS_COUNT_PAIRS] = (int64_t)tot;
        if ((int64_t)tot > pp.pair_cap) raise_flag(counts, GS_FLAG_PAIRS);
      }
    }
  }
  if ((int64_t)blockIdx.x >= ntiles) return;
  {
    uint32_t tot;
    s_goff[threadIdx.x] = block_excl_scan(hist_d, s_wave, &tot);  // global digit offsets
  }
  uint32_t pair_goff = 0;  // PAIRS: pairs of all records with a smaller digit (saturating)
  if constexpr (PAIRS) {
    uint64_t w = 0;
    for (int c = 0; c < pp.copies; ++c) w += pp.whist[c * kRadix + threadIdx.x];
    uint64_t tot;
    pair_goff = sat_u32(block_excl_scan64(w, s_wave64, &tot));
  }
  for (;;) {
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_counter, 1u);
    for (int i = threadIdx.x; i < (kThreads / 64) * kRadix; i += kThreads) (&s_wave_hist[0][0])[i] = 0u;
    __syncthreads();
    const int64_t t = s_tile;
    if (t >= ntiles) break;
    const int64_t tile_base = t * kRadixTile;
    const int tile_n = (int)((n - tile_base) < kRadixTile ? (n - tile_base) : kRadixTile);
    // wave w owns the contiguous slice [w*64*kRadixItems, (w+1)*64*kRadixItems) of the tile;
    // item k of lane l is element k*64 + l of that slice (coalesced loads)
    uint32_t key[kRadixItems], val[kRadixItems], rank[kRadixItems];
    uint32_t ttv[PAIRS ? kRadixItems : 1];
    bool valid[kRadixItems];
    const int slice = wid * 64 * kRadixItems;
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
      const int li = slice + k * 64 + lane;
      if constexpr (COMPACT) {
        // both loads issued together (a culled record's key is read and dropped)
        const bool in_tile = li < tile_n;
        const int32_t tt = in_tile ? pp.tiles_touched[tile_base + li] : 0;
        key[k] = in_tile ? keys_in[tile_base + li] : 0u;
        valid[k] = tt > 0;
        val[k] = (uint32_t)(tile_base + li);
      } else {
        valid[k] = li < tile_n;
        key[k] = valid[k] ? keys_in[tile_base + li] : 0u;
        val[k] = valid[k] ? vals_in[tile_base + li] : 0u;
      }
    }
    uint32_t tfirst[PAIRS ? kRadixItems : 1], textent[PAIRS ? kRadixItems : 1];
    if constexpr (PAIRS) {
#pragma unroll
      for (int k = 0; k < kRadixItems; ++k) {
        uint4 w0 = make_uint4(0u, 0u, 0u, 0u);
        if (valid[k]) w0 = pp.rec_words[(size_t)kRecordWords * val[k]];
        const uint32_t i0 = w0.z & 0xFFFFu, i1 = i0 + (w0.z >> 16);
        const uint32_t j0 = w0.w & 0xFFFFu, j1 = j0 + (w0.w >> 16);
        const uint32_t tx0 = i0 >> pp.tw_shift, ty0 = j0 >> pp.th_shift;
        const uint32_t ntx = (i1 >> pp.tw_shift) - tx0 + 1u, nty = (j1 >> pp.th_shift) - ty0 + 1u;
        ttv[k] = valid[k] ? ntx * nty : 0u;
        tfirst[k] = w0.y * (uint32_t)pp.tiles_per_view + ty0 * (uint32_t)pp.tiles_x + tx0;
        textent[k] = ntx | (nty << 16);
      }
    }
    // stable rank inside the wave: items in order k, lanes in order within an item
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
      const uint32_t d = (key[k] >> shift) & 255u;
      uint64_t peers = __ballot(valid[k]);
      if (peers == 0) {  // no valid item in the wave (the compacting pass: a run of culled records)
        rank[k] = 0;
        continue;
      }
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool b = (d >> bit) & 1u;
        const uint64_t m = __ballot(b);
        peers &= b ? m : ~m;
      }
      uint32_t prev = 0;
      if (valid[k]) prev = s_wave_hist[wid][d];
      const uint32_t below = (uint32_t)lanemask_lt_count(peers);
      rank[k] = prev + below;
      if (valid[k] && below == 0) s_wave_hist[wid][d] = prev + (uint32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: exclusive prefix over waves, tile count, tile-local digit prefix
    const int d = threadIdx.x;
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
      const uint32_t c = s_wave_hist[w][d];
      s_wave_hist[w][d] = run;
      run += c;
    }
    const uint32_t tile_cnt = run;
    uint32_t tile_total;
    const uint32_t tile_excl = block_excl_scan(tile_cnt, s_wave, &tile_total);
    s_tile_excl[d] = tile_excl;
    uint32_t excl = 0;
    if constexpr (PAIRS) {
      // local scatter of tiles_touched into the tile's digit order, then its
      // exclusive prefix there (16 consecutive positions per thread)
      __syncthreads();  // s_tile_excl of every digit
#pragma unroll
      for (int k = 0; k < kRadixItems; ++k) {
        if (valid[k]) {
          const uint32_t dd = (key[k] >> shift) & 255u;
          s_pfx[s_tile_excl[dd] + s_wave_hist[wid][dd] + rank[k]] = ttv[k];
        }
      }
      __syncthreads();
      uint32_t loc[kRadixItems];
      uint64_t mine = 0;
#pragma unroll
      for (int k = 0; k < kRadixItems; ++k) {
        const int i = threadIdx.x * kRadixItems + k;
        loc[k] = i < (int)tile_total ? s_pfx[i] : 0u;
        mine += loc[k];
      }
      uint64_t tsum;
      uint64_t run64 = block_excl_scan64(mine, s_wave64, &tsum);
#pragma unroll
      for (int k = 0; k < kRadixItems; ++k) {
        const int i = threadIdx.x * kRadixItems + k;
        if (i < (int)tile_total) s_pfx[i] = sat_u32(run64);
        run64 += loc[k];
      }
      if (threadIdx.x == 0) s_ptotal = sat_u32(tsum);
      __syncthreads();
      // pairs of this tile's digit-d run; one 64-bit look-back word per digit
      // carries the record count (bits 32..61) and the pair sum (bits 0..31)
      const uint32_t rs = tile_excl, re = tile_excl + tile_cnt;
      const uint32_t ps = rs < tile_total ? s_pfx[rs] : s_ptotal;
      const uint32_t pe = re < tile_total ? s_pfx[re] : s_ptotal;
      const uint32_t tpairs = pe - ps;
      s_pfx_start[d] = ps;
      uint32_t excl_pairs = 0;
      uint64_t* st = pp.status + t * kRadix + d;
      if (t == 0) {
        store_agent(st, kPFlagInc | ((uint64_t)tile_cnt << 32) | tpairs);
      } else {
        store_agent(st, kPFlagAgg | ((uint64_t)tile_cnt << 32) | tpairs);
        int64_t k = t - 1;
        int64_t spins = 0;
        for (;;) {
          uint64_t sv[kLookWindow];
#pragma unroll
          for (int i = 0; i < kLookWindow; ++i)
            sv[i] = (k - i >= 0) ? load_agent(pp.status + (k - i) * kRadix + d) : kPFlagInc;
          int used = 0;
          bool done = false, stalled = false;
#pragma unroll
          for (int i = 0; i < kLookWindow; ++i) {
            if (done || stalled) continue;
            const uint64_t flag = sv[i] & kPFlagMask;
            if (flag == 0) {
              stalled = true;
              continue;
            }
            excl += (uint32_t)(sv[i] >> 32) & kValMask;
            excl_pairs = sat_add(excl_pairs, (uint32_t)sv[i]);
            ++used;
            done = flag == kPFlagInc;
          }
          if (done) break;
          k -= used;
          if (stalled) {
            if (++spins > kSpinLimit) {
              raise_flag(counts, GS_FLAG_WAIT);
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        }
        store_agent(st, kPFlagInc | ((uint64_t)(excl + tile_cnt) << 32) | sat_add(excl_pairs, tpairs));
      }
      s_pbase[d] = sat_add(pair_goff, excl_pairs);
    } else {
    // decoupled look-back for digit d
    uint32_t* st = status + t * status_stride + d;
    if (t == 0) {
      store_agent(st, kFlagInc | tile_cnt);
    } else {
      store_agent(st, kFlagAgg | tile_cnt);
      // the predecessors' words are read kLookWindow at a time (independent
      // loads in flight) and consumed in order up to the first inclusive
      // prefix; positions before tile 0 read as an inclusive prefix of 0
      int64_t k = t - 1;
      int64_t spins = 0;
      for (;;) {
        uint32_t sv[kLookWindow];
#pragma unroll
        for (int i = 0; i < kLookWindow; ++i)
          sv[i] = (k - i >= 0) ? load_agent(status + (k - i) * status_stride + d) : kFlagInc;
        int used = 0;
        bool done = false, stalled = false;
#pragma unroll
        for (int i = 0; i < kLookWindow; ++i) {
          if (done || stalled) continue;
          const uint32_t flag = sv[i] & ~kValMask;
          if (flag == 0) {
            stalled = true;
            continue;
          }
          excl += sv[i] & kValMask;
          ++used;
          done = flag == kFlagInc;
        }
        if (done) break;
        k -= used;
        if (stalled) {
          if (++spins > kSpinLimit) {
            raise_flag(counts, GS_FLAG_WAIT);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      store_agent(st, kFlagInc | (excl + tile_cnt));
    }
    }
    s_digit_base[d] = s_goff[d] + excl;
    __syncthreads();
    if constexpr (PAIRS) {
      // each item's tile rectangle straight to its sorted slot: for one item k, the
      // lanes of a digit land on consecutive slots (and the top depth digit takes
      // few values), so these stores stay close to contiguous
#pragma unroll
      for (int k = 0; k < kRadixItems; ++k) {
        if (valid[k]) {
          const uint32_t dd = (key[k] >> shift) & 255u;
          const uint32_t out = s_digit_base[dd] + s_wave_hist[wid][dd] + rank[k];
          pp.tile_first[out] = tfirst[k];
          pp.tile_extent[out] = textent[k];
        }
      }
    }
    // local scatter by digit, then coalesced write-out
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
      if (valid[k]) {
        const uint32_t dd = (key[k] >> shift) & 255u;
        const uint32_t pos = s_tile_excl[dd] + s_wave_hist[wid][dd] + rank[k];
        s_keys[pos] = key[k];
        s_vals[pos] = val[k];
      }
    }
    __syncthreads();
    // (valid items only: tile_total = tile_n except in the compacting pass)
    for (int i = threadIdx.x; i < (int)tile_total; i += kThreads) {
      const uint32_t kk = s_keys[i];
      const uint32_t dd = (kk >> shift) & 255u;
      const uint32_t out = s_digit_base[dd] + ((uint32_t)i - s_tile_excl[dd]);
      vals_out[out] = s_vals[i];
      if constexpr (PAIRS) {
        pp.pair_off[out] = sat_add(s_pbase[dd], s_pfx[i] - s_pfx_start[dd]);
      } else {
        keys_out[out] = kk;
      }
    }
    __syncthreads();
  }
}

}  // namespace
}  // namespace gs
