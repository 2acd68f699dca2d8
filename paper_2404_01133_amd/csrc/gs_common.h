// Internal definitions shared by the HIP translation units of libgs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gs.h"

namespace gs {

// ---------------------------------------------------------------------------
// projected record (48 bytes, three 16-byte words)
//   w0: du            (2D mean minus the centre of the footprint's first pixel,
//                      i.e. u - i0 - 1/2, FP32; the 1/2 shift of the rounded
//                      u - i0 is exact, so a pixel at offset di has dx = di - du
//                      with the same rounding as (di + 1/2) - (u - i0); dv, the
//                      same for v, is the last word of w2)
//       view index (int bits)
//       px = i0 | (i1 - i0) << 16, py = j0 | (j1 - j0) << 16  (footprint, inclusive)
//       (w0 holds everything the binning reads: one 16-byte load per record)
//   w1: ca, cb, cc    (factor of the conic scaled by sqrt(log2(e) / 2): the
//                      Gaussian's value at pixel offset d is
//                      exp2(-((ca dx + cb dy)^2 + (cc dy)^2)))
//       opacity
//   w2: r, g, b       (SH colour, clamped at 0)
//       dv
// ---------------------------------------------------------------------------
struct alignas(16) Record {
  float du;
  uint32_t view;
  uint32_t px, py;
  float ca, cb, cc, opac;
  float r, g, b;
  float dv;
};
static_assert(sizeof(Record) == 48, "record layout");
constexpr int kRecordWords = sizeof(Record) / 16;  // 16-byte words per record; the first is du, view, px, py

constexpr uint32_t kCulledKey = 0xFFFFFFFFu;

// compositing thresholds of the 3DGS blending rule
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1.0e-4f;

struct DevCounts {
  int64_t* p;
};

// Host-side checks --------------------------------------------------------
inline bool tile_shape_supported(int tw, int th) {
  return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 16 && th == 8) || (tw == 32 && th == 8) ||
         (tw == 32 && th == 16);
}
inline int tiles_x(int width, int tw) { return (width + tw - 1) / tw; }
inline int tiles_y(int height, int th) { return (height + th - 1) / th; }

gs_status set_hip_error(hipError_t e);
#define GS_HIP_CHECK(expr)                        \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return set_hip_error(e_); \
  } while (0)
#define GS_LAUNCH_CHECK() GS_HIP_CHECK(hipGetLastError())

// Device helpers -------------------------------------------------------------
__device__ __forceinline__ uint64_t lanemask_lt_count(uint64_t mask) {
  // number of set bits of `mask` below the calling lane
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <class T>
__device__ __forceinline__ T load_agent(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void store_agent(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Upper bound on the number of polls of a device-side wait before it gives up
// and raises GS_FLAG_WAIT (a wait that long means a scheduling fault, never a
// normal run).
constexpr int64_t kSpinLimit = int64_t(1) << 22;

}  // namespace gs
