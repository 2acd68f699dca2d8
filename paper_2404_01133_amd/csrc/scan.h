// Single-pass scan helpers shared by the kernels that compact data in order:
// device counters with a capacity clamp, the flag word of the counts array,
// and the decoupled look-back over 64-bit status words.
#pragma once

#include "gs_common.h"

namespace gs {

__device__ __forceinline__ int64_t count_clamped(const int64_t* counts, int idx, int64_t cap) {
  int64_t n = counts[idx];
  return n < cap ? n : cap;
}

__device__ __forceinline__ void raise_flag(int64_t* counts, int64_t bit) {
  atomicOr((unsigned long long*)&counts[GS_COUNT_FLAGS], (unsigned long long)bit);
}

// 64-bit status word of one scan tile: 2 flag bits (none / aggregate /
// inclusive prefix) over a 62-bit value.  Zero means "not published yet".
constexpr uint64_t kFlagAgg64 = 1ull << 62;
constexpr uint64_t kFlagInc64 = 2ull << 62;
constexpr uint64_t kValMask64 = (1ull << 62) - 1;

// Decoupled look-back done by one whole wave: lane l inspects predecessor
// t-1-l, so each round of loads covers 64 predecessors.  Positions before
// tile 0 read as an inclusive prefix of 0.  Tile t publishes its aggregate,
// sums the predecessors' values up to the nearest inclusive prefix, then
// publishes its own inclusive prefix.  Tiles must be claimed in order (an
// atomic tile counter) so every wait is on a running or finished tile; the
// wait is still bounded and raises GS_FLAG_WAIT if it gives up.  Must be
// called by all 64 lanes of one wave; returns the exclusive prefix.
__device__ inline uint64_t lookback64_wave(uint64_t* status, int64_t t, uint64_t aggregate, int64_t* counts) {
  const int lane = threadIdx.x & 63;
  if (t == 0) {
    if (lane == 0) store_agent(&status[0], kFlagInc64 | aggregate);
    return 0;
  }
  if (lane == 0) store_agent(&status[t], kFlagAgg64 | aggregate);
  uint64_t excl = 0;
  int64_t base = t - 1;
  int64_t spins = 0;
  for (;;) {
    const int64_t k = base - lane;
    const uint64_t sv = k >= 0 ? load_agent(&status[k]) : kFlagInc64;
    const uint64_t flag = sv & ~kValMask64;
    const uint64_t inc = __ballot(flag == kFlagInc64);
    const uint64_t pending = __ballot(flag == 0);
    // lanes that matter: up to and including the nearest inclusive prefix
    const int last = inc ? __ffsll((unsigned long long)inc) - 1 : 63;
    const uint64_t window = last == 63 ? ~0ull : ((2ull << last) - 1);
    if (pending & window) {
      if (++spins > kSpinLimit) {
        if (lane == 0) raise_flag(counts, GS_FLAG_WAIT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    uint64_t v = (lane <= last) ? (sv & kValMask64) : 0;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    excl += v;
    if (inc) break;
    base -= 64;
  }
  if (lane == 0) store_agent(&status[t], kFlagInc64 | (excl + aggregate));
  return excl;
}

}  // namespace gs
