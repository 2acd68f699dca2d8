// Pieces shared by the per-tile compositing kernels (forward and adjoint):
// evaluation of a record at a pixel, the lane -> pixel map, per-group record
// lists, the tile arguments and the work distribution over tiles.  Included by
// translation units compiled with -ffp-contract=off: evaluate() is the
// operation order both kernels must share.
#pragma once

#include "project.h"

namespace gs {
namespace {

// Value of a projected Gaussian at pixel offset (dx, dy): exp2(-(p1^2 + p2^2)).
struct Eval {
  float dx, dy, p1, p2, G, alpha;
};

__device__ __forceinline__ bool in_footprint(int i, int j, uint32_t px, uint32_t py, int& di, int& dj) {
  di = i - (int)(px & 0xFFFFu);
  dj = j - (int)(py & 0xFFFFu);
  return ((uint32_t)di <= (px >> 16)) && ((uint32_t)dj <= (py >> 16));
}

// Gaussian and alpha at offset (dx, dy) from the projected mean
__device__ __forceinline__ void evaluate_at(const float4& w1, Eval& e) {
  e.p1 = fmaf(w1.x, e.dx, w1.y * e.dy);
  e.p2 = w1.z * e.dy;
  e.G = __builtin_amdgcn_exp2f(-fmaf(e.p1, e.p1, e.p2 * e.p2));
  e.alpha = fminf(kAlphaMax, w1.w * e.G);
}

__device__ __forceinline__ void evaluate(const float4& w0, const float4& w1, const float4& w2, int di, int dj,
                                         Eval& e) {
  e.dx = (float)di - w0.x;  // w0.x = u - i0 - 1/2
  e.dy = (float)dj - w2.w;  // w2.w = v - j0 - 1/2
  evaluate_at(w1, e);
}

// The same with the footprint given as floats f = (i0, j0, i1 - i0, j1 - j0),
// for a pixel (fi, fj) as floats: fi - i0 is exact (integers below 2^24), so dx
// equals the value above bit for bit, and the footprint test is one unsigned
// compare of float bits per axis (a non-negative float's bits grow with its
// value; a negative difference has the sign bit set and fails).
__device__ __forceinline__ bool evaluate_f(float fi, float fj, const float4& f, float du, float dv,
                                           const float4& w1, Eval& e) {
  const float fdi = fi - f.x, fdj = fj - f.y;
  e.dx = fdi - du;
  e.dy = fdj - dv;
  evaluate_at(w1, e);
  return (__float_as_uint(fdi) <= __float_as_uint(f.z)) && (__float_as_uint(fdj) <= __float_as_uint(f.w));
}


// Lane -> pixel map of the tile kernels: the tile is cut into 8x8 pixel
// blocks, one per wave (wave w is block (w mod TW/8, w div TW/8)); each block
// is cut into groups of GW x GH pixels, numbered row-major over the block;
// lanes [g*GW*GH, (g+1)*GW*GH) hold group g and lane l is pixel (r mod GW,
// r div GW) of it (r = l mod GW*GH).  Each group walks its own list of records
// (below), so a small footprint costs one group's step, not the wave's.
template <int TW, int TH, int GW, int GH>
struct LaneMap {
  static_assert(TW % 8 == 0 && TH % 8 == 0, "tiles are whole 8x8 blocks");
  static_assert(8 % GW == 0 && 8 % GH == 0, "groups tile the 8x8 block");
  static constexpr int kGroups = 64 / (GW * GH);
  int i, j;    // this lane's pixel
  int x0, y0;  // first pixel of the wave's block
  int g;       // this lane's group
  __device__ __forceinline__ LaneMap(int txi, int tyi, int wid) {
    const int lane = threadIdx.x & 63;
    x0 = txi * TW + (wid % (TW / 8)) * 8;
    y0 = tyi * TH + (wid / (TW / 8)) * 8;
    g = lane / (GW * GH);
    const int r = lane % (GW * GH);
    i = x0 + (g % (8 / GW)) * GW + r % GW;
    j = y0 + (g / (8 / GW)) * GH + r / GW;
  }
};

// Group list stride: BATCH bytes plus one dword, so the lists a wave reads
// side by side start in different LDS banks.
template <int BATCH>
constexpr int kListStride = BATCH + 4;

// Per-group ballot compaction: list[g][0 .. cnt[g]) receives, in ascending
// (= depth) order, the staged records whose footprint rectangle meets group g
// of the wave's block.  The counts are a struct of named scalars (arrays of
// them end up in scratch memory).
struct Counts4 {
  int c0, c1, c2, c3;
  __device__ __forceinline__ int max() const { return ::max(::max(c0, c1), ::max(c2, c3)); }
  __device__ __forceinline__ int of(int g) const { return g == 0 ? c0 : g == 1 ? c1 : g == 2 ? c2 : c3; }
};
struct Counts8 {
  int c0, c1, c2, c3, c4, c5, c6, c7;
  __device__ __forceinline__ int max() const {
    return ::max(::max(::max(c0, c1), ::max(c2, c3)), ::max(::max(c4, c5), ::max(c6, c7)));
  }
  __device__ __forceinline__ int of(int g) const {
    const int lo = g == 0 ? c0 : g == 1 ? c1 : g == 2 ? c2 : c3;
    const int hi = g == 4 ? c4 : g == 5 ? c5 : g == 6 ? c6 : c7;
    return g < 4 ? lo : hi;
  }
};

template <int BATCH>
__device__ __forceinline__ void append_if(bool h, uint8_t* list, int& c, int k) {
  const uint64_t m = __ballot(h);
  if (h) list[c + (int)lanemask_lt_count(m)] = (uint8_t)k;
  c += (int)__popcll(m);
}

// rectangle of staged record k; past the batch one that meets no pixel (every
// overlap test "i0 <= hi && i1 >= lo" with lo, hi >= 0 fails on it)
__device__ __forceinline__ void staged_rect(const float4* s_w0, int k, int nb, int& i0, int& i1, int& j0, int& j1) {
  i0 = j0 = 1 << 30;
  i1 = j1 = -1;
  if (k < nb) {
    const uint32_t px = __float_as_uint(s_w0[k].z), py = __float_as_uint(s_w0[k].w);
    i0 = (int)(px & 0xFFFFu), i1 = i0 + (int)(px >> 16);
    j0 = (int)(py & 0xFFFFu), j1 = j0 + (int)(py >> 16);
  }
}

// 4x4 quadrants (groups 0..3 row-major over the 8x8 block)
template <int BATCH>
__device__ __forceinline__ Counts4 wave_compact4(const float4* s_w0, int nb, int x0, int y0,
                                                 uint8_t (*list)[kListStride<BATCH>]) {
  static_assert(BATCH <= 256, "record indices are bytes");
  const int lane = threadIdx.x & 63;
  Counts4 c{0, 0, 0, 0};
  for (int base = 0; base < nb; base += 64) {
    const int k = base + lane;
    int i0, i1, j0, j1;
    staged_rect(s_w0, k, nb, i0, i1, j0, j1);
    const bool xa = i0 <= x0 + 3 && i1 >= x0, xb = i0 <= x0 + 7 && i1 >= x0 + 4;
    const bool ya = j0 <= y0 + 3 && j1 >= y0, yb = j0 <= y0 + 7 && j1 >= y0 + 4;
    append_if<BATCH>(xa && ya, list[0], c.c0, k);
    append_if<BATCH>(xb && ya, list[1], c.c1, k);
    append_if<BATCH>(xa && yb, list[2], c.c2, k);
    append_if<BATCH>(xb && yb, list[3], c.c3, k);
  }
  return c;
}

// 4x2 groups (two columns of four pixels, four rows of two; row-major)
template <int BATCH>
__device__ __forceinline__ Counts8 wave_compact8(const float4* s_w0, int nb, int x0, int y0,
                                                 uint8_t (*list)[kListStride<BATCH>]) {
  static_assert(BATCH <= 256, "record indices are bytes");
  const int lane = threadIdx.x & 63;
  Counts8 c{0, 0, 0, 0, 0, 0, 0, 0};
  for (int base = 0; base < nb; base += 64) {
    const int k = base + lane;
    int i0, i1, j0, j1;
    staged_rect(s_w0, k, nb, i0, i1, j0, j1);
    const bool xa = i0 <= x0 + 3 && i1 >= x0, xb = i0 <= x0 + 7 && i1 >= x0 + 4;
    const bool y0r = j0 <= y0 + 1 && j1 >= y0, y1r = j0 <= y0 + 3 && j1 >= y0 + 2;
    const bool y2r = j0 <= y0 + 5 && j1 >= y0 + 4, y3r = j0 <= y0 + 7 && j1 >= y0 + 6;
    append_if<BATCH>(xa && y0r, list[0], c.c0, k);
    append_if<BATCH>(xb && y0r, list[1], c.c1, k);
    append_if<BATCH>(xa && y1r, list[2], c.c2, k);
    append_if<BATCH>(xb && y1r, list[3], c.c3, k);
    append_if<BATCH>(xa && y2r, list[4], c.c4, k);
    append_if<BATCH>(xb && y2r, list[5], c.c5, k);
    append_if<BATCH>(xa && y3r, list[6], c.c6, k);
    append_if<BATCH>(xb && y3r, list[7], c.c7, k);
  }
  return c;
}

struct TileArgs {
  const Record* records;
  const uint32_t* pair_records;
  const uint32_t* ranges;
  int W, H, tiles_x_n, tiles_per_view;
  int64_t n_tiles;
};

// Work distribution shared by the tile kernels: either one work-group per tile
// (queue == nullptr) or persistent work-groups taking tiles from the device
// queue built by bin_sort, longest lists first.
//
// Every work-group ends on exactly one fetch past the end, so those fetches
// return n_tiles .. n_tiles + gridDim.x - 1; the work-group that draws the last
// of them knows no other will read the head again and puts it back to zero.
// A second launch on the same sorted frame (a repeated forward, a second
// backward) therefore walks the whole queue again.
template <class Body>
__device__ __forceinline__ void for_each_tile(const TileArgs& t, uint32_t* queue, int head, Body body) {
  if (queue == nullptr) {
    body((int)blockIdx.x);
    return;
  }
  __shared__ uint32_t s_next;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(&queue[head], 1u);
    __syncthreads();
    const uint32_t k = s_next;
    __syncthreads();
    if ((int64_t)k >= t.n_tiles) {
      if (threadIdx.x == 0 && (int64_t)k == t.n_tiles + (int64_t)gridDim.x - 1) atomicExch(&queue[head], 0u);
      break;
    }
    body((int)queue[2 + k]);
  }
}

// Persistent grid for the queue mode: enough work-groups to fill every CU a few times over.
inline dim3 tile_grid(int64_t n_tiles, bool queued) {
  const int64_t cap = 256 * 8;
  return dim3((unsigned)(queued ? (n_tiles < cap ? (n_tiles > 0 ? n_tiles : 1) : cap) : n_tiles));
}

inline bool batch_supported(int b) { return b == 64 || b == 128 || b == 256; }

}  // namespace
}  // namespace gs
