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

// ---------------------------------------------------------------------------
// one stable LSD pass over 8 bits; the digit histogram of the whole input was
// accumulated by the kernel that produced the keys
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) radix_pass_kernel(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint32_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, const int64_t* counts_in, int count_idx, int64_t cap, int shift,
    const uint32_t* __restrict__ hist, uint32_t* status, int64_t status_stride, uint32_t* tile_counter,
    int64_t* counts) {
  __shared__ uint32_t s_keys[kRadixTile];
  __shared__ uint32_t s_vals[kRadixTile];
  __shared__ uint32_t s_wave_hist[kThreads / 64][kRadix];
  __shared__ uint32_t s_tile_excl[kRadix];
  __shared__ uint32_t s_digit_base[kRadix];
  __shared__ uint32_t s_wave[kThreads / 64];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_goff[kRadix];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t n = count_clamped(counts_in, count_idx, cap);
  const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  if ((int64_t)blockIdx.x >= ntiles) return;
  {
    uint32_t tot;
    s_goff[threadIdx.x] = block_excl_scan(hist[threadIdx.x], s_wave, &tot);  // global digit offsets
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
    bool valid[kRadixItems];
    const int slice = wid * 64 * kRadixItems;
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
      const int li = slice + k * 64 + lane;
      valid[k] = li < tile_n;
      key[k] = valid[k] ? keys_in[tile_base + li] : 0u;
      val[k] = valid[k] ? vals_in[tile_base + li] : 0u;
    }
    // stable rank inside the wave: items in order k, lanes in order within an item
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
      const uint32_t d = (key[k] >> shift) & 255u;
      uint64_t peers = __ballot(valid[k]);
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
    // decoupled look-back for digit d
    uint32_t excl = 0;
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
    s_digit_base[d] = s_goff[d] + excl;
    __syncthreads();
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
    for (int i = threadIdx.x; i < tile_n; i += kThreads) {
      const uint32_t kk = s_keys[i];
      const uint32_t dd = (kk >> shift) & 255u;
      const uint32_t out = s_digit_base[dd] + ((uint32_t)i - s_tile_excl[dd]);
      keys_out[out] = kk;
      vals_out[out] = s_vals[i];
    }
    __syncthreads();
  }
}

}  // namespace
}  // namespace gs
