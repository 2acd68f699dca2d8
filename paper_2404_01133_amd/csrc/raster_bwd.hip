// Adjoint of the per-tile compositing (Sec. 3.1, differentiable rendering) and
// of the projection.
//
// Compositing adjoint: the forward's walk on 4x4 quadrants of 16 lanes, front
// to back, bounded by each pixel's n_last, with the blend state recomputed
// (colour in front is accumulated, colour behind = final colour - accumulated),
// so nothing per (pixel, Gaussian) is stored.  The nine per-Gaussian partial
// gradients of a quadrant are summed with DPP row operations, added into LDS
// across the tile's waves, and flushed with one FP32 atomic per (tile,
// Gaussian, quantity).  Then the projection adjoint chains each record's 2D
// partials back to the Gaussian's parameters.
#include "tile.h"

namespace gs {
namespace {

// ---------------------------------------------------------------------------
// Sums of nine per-lane values over each 16-lane quadrant, all at once.  At
// butterfly level k (partner lane = lane ^ 2^k, k = 0..3) two quantities share
// one register: lanes with bit k clear keep the first, lanes with bit k set the
// second, and each lane adds the partner's copy of the quantity it keeps.  Nine
// registers become one after the four levels; on return lane 16p + r of
// quadrant p holds the quadrant's total of value min(r, 8).
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int PATTERN>
__device__ __forceinline__ float swz(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), PATTERN));
}
__device__ __forceinline__ float pack_add1(bool hi, float a, float b) {  // partner lane ^ 1
  return (hi ? b : a) + dpp_mov<0xB1>(hi ? a : b);                      // quad_perm [1,0,3,2]
}
__device__ __forceinline__ float pack_add2(bool hi, float a, float b) {  // partner lane ^ 2
  return (hi ? b : a) + dpp_mov<0x4E>(hi ? a : b);                      // quad_perm [2,3,0,1]
}

__device__ __forceinline__ float quad_sum9(const float v[9], int lane) {
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4, b3 = lane & 8;
  const float r0 = pack_add1(b0, v[0], v[1]);
  const float r1 = pack_add1(b0, v[2], v[3]);
  const float r2 = pack_add1(b0, v[4], v[5]);
  const float r3 = pack_add1(b0, v[6], v[7]);
  const float r4 = v[8] + dpp_mov<0xB1>(v[8]);
  const float s0 = pack_add2(b1, r0, r1);
  const float s1 = pack_add2(b1, r2, r3);
  const float s2 = r4 + dpp_mov<0x4E>(r4);
  // ds_swizzle bit-mask mode (and 0x1F, xor m) exchanges with lane ^ m inside 32 lanes
  const float u0 = (b2 ? s1 : s0) + swz<0x101F>(b2 ? s0 : s1);
  const float u1 = s2 + swz<0x101F>(s2);
  return (b3 ? u1 : u0) + swz<0x201F>(b3 ? u0 : u1);
}

constexpr int kG = 9;  // partials per Gaussian: r, g, b, opacity, A1, A2, Axx, Axy, Ayy
constexpr int kBwdLdsOffsets = 1024;  // segment offsets staged in LDS by the view-major adjoint up to this many

// DET: each quadrant of the tile stores its sums for the staged records in its
// own slots (grad[quadrant][record][9], plain stores: a quadrant's list holds a
// record at most once); the slots are then summed in quadrant order.
// Otherwise grad[record][9] receives LDS atomic adds.
template <int TW, int TH, int BATCH, bool DET>
struct BwdLds {
  static constexpr int kQuads = DET ? (TW * TH) / 16 : 1;
  float4 w0[BATCH], w1[BATCH], w2[BATCH];
  uint32_t rec[BATCH];
  float grad[kQuads * BATCH * kG];
  uint8_t list[(TW * TH) / 64][4][kListStride<BATCH>];
  int wave_last[(TW * TH) / 64];
};

// Deterministic mode: per-(tile, record) partials are stored at slot
// base[record] + (the tile's row-major index within the record's footprint
// tiles), so a record's partials lie contiguous in ascending tile order and
// are summed in that order afterwards.
struct DetArgs {
  float* partial;        // [slots][kG]
  const uint32_t* base;  // [records]: first slot of each record
  int64_t slots;         // slots the workspace holds
};

template <int TW, int TH>
__device__ __forceinline__ int64_t det_slot(const DetArgs& d, uint32_t rid, uint32_t px, uint32_t py, int txi,
                                            int tyi) {
  const int i0 = (int)(px & 0xFFFFu), i1 = i0 + (int)(px >> 16);
  const int j0 = (int)(py & 0xFFFFu);
  const int tx0 = i0 / TW, ntx = i1 / TW - tx0 + 1, ty0 = j0 / TH;
  return (int64_t)d.base[rid] + (int64_t)(tyi - ty0) * ntx + (txi - tx0);
}

template <int TW, int TH, int BATCH, bool DET>
__device__ __forceinline__ void raster_bwd_tile(const TileArgs& ta, BwdLds<TW, TH, BATCH, DET>& lds, int tile_g,
                                                const float* __restrict__ rgb, const float* __restrict__ T_final,
                                                const int32_t* __restrict__ n_last, const float* __restrict__ d_rgb,
                                                float* __restrict__ grad2d, const DetArgs& det) {
  constexpr int NT = TW * TH;
  constexpr int NW = NT / 64;
  const Record* __restrict__ records = ta.records;
  const uint32_t* __restrict__ pair_records = ta.pair_records;
  const uint32_t* __restrict__ ranges = ta.ranges;
  const int W = ta.W, H = ta.H, tiles_x_n = ta.tiles_x_n, tiles_per_view = ta.tiles_per_view;
  float4* s_w0 = lds.w0;
  float4* s_w1 = lds.w1;
  float4* s_w2 = lds.w2;
  uint32_t* s_rec = lds.rec;
  float* s_grad = lds.grad;
  int* s_wave_last = lds.wave_last;
  const int view = tile_g / tiles_per_view;
  const int tile = tile_g - view * tiles_per_view;
  const int tyi = tile / tiles_x_n, txi = tile - tyi * tiles_x_n;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const LaneMap<TW, TH, 4, 4> qb(txi, tyi, wid);
  const int i = qb.i, j = qb.j;
  const bool inside = (i < W) && (j < H);
  const uint32_t start = ranges[2 * tile_g];
  const int64_t plane = (int64_t)H * W;
  const int64_t pix = (int64_t)j * W + i;
  float g0 = 0.f, g1 = 0.f, g2 = 0.f, out0 = 0.f, out1 = 0.f, out2 = 0.f;
  int last = 0;
  if (inside) {
    const int64_t o = (int64_t)view * 3 * plane + pix;
    g0 = d_rgb[o];
    g1 = d_rgb[o + plane];
    g2 = d_rgb[o + 2 * plane];
    out0 = rgb[o];
    out1 = rgb[o + plane];
    out2 = rgb[o + 2 * plane];
    last = n_last[(int64_t)view * plane + pix];
  }
  // entries this wave / the tile must walk
  int wl = last;
  for (int off = 32; off > 0; off >>= 1) wl = max(wl, __shfl_xor(wl, off, 64));
  if (lane == 0) s_wave_last[wid] = wl;
  __syncthreads();
  int tile_last = 0;
  for (int w = 0; w < NW; ++w) tile_last = max(tile_last, s_wave_last[w]);
  const int wave_last = __builtin_amdgcn_readfirstlane(s_wave_last[wid]);
  uint8_t(*lists)[kListStride<BATCH>] = lds.list[wid];
  const uint8_t* my_list = lists[qb.g];
  const int r = lane & 15;  // lane within the quadrant
  float T = 1.0f, A0 = 0.f, A1c = 0.f, A2c = 0.f;  // transmittance and colour accumulated in front
  for (uint32_t b = start; b < start + (uint32_t)tile_last; b += BATCH) {
    const int nb = (int)min((uint32_t)BATCH, start + (uint32_t)tile_last - b);
    for (int k = threadIdx.x; k < nb; k += NT) {
      const uint32_t rid = pair_records[b + k];
      const float4* rp = reinterpret_cast<const float4*>(&records[rid]);
      s_w0[k] = rp[0];
      s_w1[k] = rp[1];
      s_w2[k] = rp[2];
      s_rec[k] = rid;
    }
    for (int k = threadIdx.x; k < lds.kQuads * BATCH * kG; k += NT) s_grad[k] = 0.0f;
    __syncthreads();
    const int base_idx = (int)(b - start);
    const int kmax = min(nb, wave_last - base_idx);  // entries past every lane's n_last are not needed
    const Counts4 cnt = kmax > 0 ? wave_compact4<BATCH>(s_w0, kmax, qb.x0, qb.y0, lists) : Counts4{0, 0, 0, 0};
    const int max_cnt = cnt.max();
    const int my_cnt = cnt.of(qb.g);
    // one entry of each quadrant's list: the four quadrants step (possibly
    // different) records side by side; partials are summed per quadrant and
    // added into the record's LDS slots (two quadrants on one record add twice)
    auto step = [&](int k, bool valid, const float4& w0, const float4& w1, const float4& w2) {
      int di, dj;
      const bool in_fp = in_footprint(i, j, __float_as_uint(w0.z), __float_as_uint(w0.w), di, dj);
      Eval e;
      evaluate(w0, w1, w2, di, dj, e);
      const bool use = valid && (base_idx + k < last) && in_fp && (e.alpha >= kAlphaMin);
      if (__ballot(use) == 0) return;
      const float aT = e.alpha * T;
      const float nA0 = fmaf(w2.x, aT, A0), nA1 = fmaf(w2.y, aT, A1c), nA2 = fmaf(w2.z, aT, A2c);
      // hardware reciprocal (1 ulp): a correctly rounded division costs ~10 instructions
      // here and the gradient is not bit-compared
      const float inv1ma = __builtin_amdgcn_rcpf(1.0f - e.alpha);
      // dL/dalpha = sum_c g_c (colour_c T - (colour behind)_c / (1 - alpha))
      const float dalpha = g0 * (w2.x * T - (out0 - nA0) * inv1ma) + g1 * (w2.y * T - (out1 - nA1) * inv1ma) +
                           g2 * (w2.z * T - (out2 - nA2) * inv1ma);
      const bool unclamped = use && (w1.w * e.G <= kAlphaMax);
      // dL/dQ with G = exp2(-Q): dG/dQ = -ln2 G
      const float gQ = unclamped ? -0.69314718055994531f * dalpha * w1.w * e.G : 0.0f;
      float c[kG];
      c[0] = use ? aT * g0 : 0.0f;
      c[1] = use ? aT * g1 : 0.0f;
      c[2] = use ? aT * g2 : 0.0f;
      c[3] = unclamped ? dalpha * e.G : 0.0f;
      c[4] = gQ * e.p1;
      c[5] = gQ * e.p2;
      c[6] = gQ * e.dx * e.dx;
      c[7] = gQ * e.dx * e.dy;
      c[8] = gQ * e.dy * e.dy;
      A0 = use ? nA0 : A0;
      A1c = use ? nA1 : A1c;
      A2c = use ? nA2 : A2c;
      T = use ? T * (1.0f - e.alpha) : T;
      const float sum = quad_sum9(c, lane);
      if constexpr (DET) {
        if (valid && r < kG) s_grad[((wid * 4 + qb.g) * BATCH + k) * kG + r] = sum;
      } else {
        if (valid && r < kG && sum != 0.0f) atomicAdd(&s_grad[k * kG + r], sum);
      }
    };
    // two entries of the lane's quadrant list per trip, byte indices in one LDS
    // read (entries past the quadrant's count: stale bytes, masked, not used)
    for (int t = 0; t < max_cnt; t += 2) {
      const uint32_t pk = *reinterpret_cast<const uint16_t*>(&my_list[t]);
      const int ka = (int)(pk & (BATCH - 1)), kb = (int)((pk >> 8) & (BATCH - 1));
      const float4 a0 = s_w0[ka], a1 = s_w1[ka], a2 = s_w2[ka];
      const float4 b0 = s_w0[kb], b1 = s_w1[kb], b2 = s_w2[kb];
      step(ka, t < my_cnt, a0, a1, a2);
      step(kb, t + 1 < my_cnt, b0, b1, b2);
    }
    __syncthreads();
    if constexpr (DET) {
      for (int t = threadIdx.x; t < nb * kG; t += NT) {
        float v = 0.0f;
        for (int q = 0; q < lds.kQuads; ++q) v += s_grad[q * BATCH * kG + t];
        const int k = t / kG;
        const int64_t slot = det_slot<TW, TH>(det, s_rec[k], __float_as_uint(s_w0[k].z),
                                              __float_as_uint(s_w0[k].w), txi, tyi);
        if (slot < det.slots) det.partial[slot * kG + (t - k * kG)] = v;
      }
    } else {
      for (int t = threadIdx.x; t < nb * kG; t += NT) {
        const float v = s_grad[t];
        if (v != 0.0f) unsafeAtomicAdd(&grad2d[(int64_t)s_rec[t / kG] * kG + (t % kG)], v);
      }
    }
    __syncthreads();
  }
  if constexpr (DET) {
    // entries behind every pixel's last one were not walked: their slots get zeros
    const uint32_t len = ranges[2 * tile_g + 1] - start;
    for (uint32_t k = (uint32_t)tile_last + threadIdx.x; k < len; k += NT) {
      const uint32_t rid = pair_records[start + k];
      const uint4 w0 = *reinterpret_cast<const uint4*>(&records[rid]);
      const int64_t slot = det_slot<TW, TH>(det, rid, w0.z, w0.w, txi, tyi);
      if (slot < det.slots)
#pragma unroll
        for (int q = 0; q < kG; ++q) det.partial[slot * kG + q] = 0.0f;
    }
  }
}

template <int TW, int TH, int BATCH, bool DET>
__global__ void __launch_bounds__(TW* TH) raster_bwd_kernel(TileArgs ta, uint32_t* queue,
                                                            const float* __restrict__ rgb,
                                                            const float* __restrict__ T_final,
                                                            const int32_t* __restrict__ n_last,
                                                            const float* __restrict__ d_rgb,
                                                            float* __restrict__ grad2d, DetArgs det) {
  __shared__ BwdLds<TW, TH, BATCH, DET> lds;
  for_each_tile(ta, queue, 1, [&](int tile_g) {
    raster_bwd_tile<TW, TH, BATCH, DET>(ta, lds, tile_g, rgb, T_final, n_last, d_rgb, grad2d, det);
  });
}

// ---------------------------------------------------------------------------
// deterministic mode: slots per record, then per-record sums in tile order
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t det_pairs(const int64_t* counts, int64_t slots) {
  const int64_t m = counts[GS_COUNT_PAIRS];
  return m < slots ? m : slots;
}

// cnt[r] = 0 for every record, and the slot cursor
__global__ void det_clear_kernel(uint32_t* __restrict__ cnt, uint32_t* __restrict__ cursor, const int64_t* counts,
                                 int64_t cap) {
  int64_t n = counts[GS_COUNT_RECORDS];
  if (n > cap) n = cap;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t0 == 0) *cursor = 0u;
  for (int64_t k = t0; k < n; k += stride) cnt[k] = 0u;
}

// cnt[r] = number of (tile, record) pairs of record r (integer adds: exact in any order)
__global__ void det_count_kernel(const uint32_t* __restrict__ pair_records, const int64_t* counts, int64_t slots,
                                 uint32_t* __restrict__ cnt) {
  const int64_t m = det_pairs(counts, slots);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += stride)
    atomicAdd(&cnt[pair_records[p]], 1u);
}

// base[r]: a contiguous run of cnt[r] slots per record.  Where a run lies does
// not change any sum, so work-groups take their ranges with one atomic each.
__global__ void __launch_bounds__(256) det_base_kernel(const uint32_t* __restrict__ cnt, const int64_t* counts,
                                                       int64_t cap, uint32_t* __restrict__ cursor,
                                                       uint32_t* __restrict__ base) {
  __shared__ uint32_t s_wave[4];
  __shared__ uint32_t s_start;
  int64_t n = counts[GS_COUNT_RECORDS];
  if (n > cap) n = cap;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t r0 = (int64_t)blockIdx.x * 256; r0 < n; r0 += (int64_t)gridDim.x * 256) {
    const int64_t r = r0 + threadIdx.x;
    const uint32_t c = r < n ? cnt[r] : 0u;
    uint32_t inc = c;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(inc, off, 64);
      if (lane >= off) inc += y;
    }
    if (lane == 63) s_wave[wid] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int w = 0; w < 4; ++w) {
      before += w < wid ? s_wave[w] : 0u;
      total += s_wave[w];
    }
    if (threadIdx.x == 0) s_start = total ? atomicAdd(cursor, total) : 0u;
    __syncthreads();
    if (r < n) base[r] = s_start + before + inc - c;
    __syncthreads();
  }
}

// grad2d[r] = sum of record r's slots, in ascending tile order
__global__ void det_reduce_kernel(const float* __restrict__ partial, const uint32_t* __restrict__ cnt,
                                  const uint32_t* __restrict__ base, const int64_t* counts, int64_t cap,
                                  int64_t slots, float* __restrict__ grad2d) {
  int64_t n = counts[GS_COUNT_RECORDS];
  if (n > cap) n = cap;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const uint32_t c = cnt[r];
    if (c == 0) continue;
    const int64_t b = base[r];
    if (b + c > slots) continue;  // the workspace holds fewer slots than pairs
    float acc[kG];
#pragma unroll
    for (int q = 0; q < kG; ++q) acc[q] = 0.0f;
    for (uint32_t k = 0; k < c; ++k)
#pragma unroll
      for (int q = 0; q < kG; ++q) acc[q] += partial[(b + k) * kG + q];
#pragma unroll
    for (int q = 0; q < kG; ++q) grad2d[r * kG + q] = acc[q];
  }
}

// ---------------------------------------------------------------------------
// preprocess adjoint: per record, chain the 2D partials back to the parameters
// ---------------------------------------------------------------------------
struct BwdArgs {
  LevelPtrs lv[kMaxLevels];
  gs_gaussian_grads gr[kMaxLevels];
  const int64_t* lvl_off;
  const int64_t* lvl_cnt;
  const int8_t* level;
  const int64_t* offsets;
  const uint32_t* gather;  // point-wise selection: record -> index within its level (packed: see below)
  const gs_camera* cams;
  int64_t capacity;
  int32_t B, L, V, W, H, sh_degree;
  int32_t segs;    // segments per view: B (block-wise), L (point-wise) or 1 (packed)
  int32_t packed;  // gather entries are level << GS_PACKED_INDEX_BITS | index (refined selection)
};

// Destinations of a record's parameter gradients.
//
// AtomicSink adds into the level's gradient arrays with no-return FP32 atomics
// (records of one Gaussian may run concurrently when views share it; with one
// view each address receives one add, so the result is the plain sum).  The
// adds do not wait for memory, so a record's 59 updates are all in flight
// together, where a read-modify-write chain would wait for each load.
struct AtomicSink {
  const gs_gaussian_grads& G;
  int64_t n, gi;
  __device__ __forceinline__ void sh(int idx, float v) const {
    if (v != 0.0f) unsafeAtomicAdd(&G.sh[(int64_t)idx * n + gi], v);
  }
  __device__ __forceinline__ void mean(int k, float v) const { unsafeAtomicAdd(&G.means[k * n + gi], v); }
  __device__ __forceinline__ void scale(int k, float v) const { unsafeAtomicAdd(&G.scales[k * n + gi], v); }
  __device__ __forceinline__ void quat(int k, float v) const { unsafeAtomicAdd(&G.quats[k * n + gi], v); }
  __device__ __forceinline__ void opac(float v) const { unsafeAtomicAdd(&G.opac[gi], v); }
};

// RegisterSink sums the gradients of all records of one Gaussian (a thread
// that owns them, views in order) and adds the totals to memory once.
struct RegisterSink {
  float shv[48], m[3], s[3], q[4], o;
  __device__ __forceinline__ RegisterSink() {
#pragma unroll
    for (int i = 0; i < 48; ++i) shv[i] = 0.0f;
#pragma unroll
    for (int i = 0; i < 3; ++i) m[i] = s[i] = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = 0.0f;
    o = 0.0f;
  }
  __device__ __forceinline__ void sh(int idx, float v) { shv[idx] += v; }
  __device__ __forceinline__ void mean(int k, float v) { m[k] += v; }
  __device__ __forceinline__ void scale(int k, float v) { s[k] += v; }
  __device__ __forceinline__ void quat(int k, float v) { q[k] += v; }
  __device__ __forceinline__ void opac(float v) { o += v; }
  // planes: coefficient planes stored per colour channel ((sh_degree + 1)^2).
  // Every current value is loaded before the first store, so the loads are in
  // flight together (in a += chain each load would wait for the previous store).
  __device__ __forceinline__ void flush(const gs_gaussian_grads& G, int64_t n, int64_t gi, int planes) const {
    float cm[3], cs[3], cq[4], csh[48];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cm[k] = G.means[k * n + gi];
      cs[k] = G.scales[k * n + gi];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) cq[k] = G.quats[k * n + gi];
    const float co = G.opac[gi];
#pragma unroll
    for (int i = 0; i < 48; ++i) csh[i] = i < 3 * planes ? G.sh[(int64_t)i * n + gi] : 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      G.means[k * n + gi] = cm[k] + m[k];
      G.scales[k * n + gi] = cs[k] + s[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) G.quats[k * n + gi] = cq[k] + q[k];
    G.opac[gi] = co + o;
#pragma unroll
    for (int i = 0; i < 48; ++i)
      if (i < 3 * planes) G.sh[(int64_t)i * n + gi] = csh[i] + shv[i];
  }
};

// Adjoint of the SH colour, FP32, one basis term at a time (no basis arrays
// live): dL/df_{k,c} = Y_k g_c and dL/d(direction) += (sum_c g_c f_{k,c}) grad Y_k.
template <bool HALF, class Sink>
__device__ __forceinline__ void sh_adjoint(float x, float y, float z, int deg, const void* __restrict__ sh, int64_t n,
                                           int64_t gi, const float g[3], Sink& sink, float gdir[3]) {
  auto term = [&](int k, float Y, float dx, float dy, float dz) {
    const float f0 = attr<HALF>(sh, (int64_t)(3 * k + 0) * n + gi);
    const float f1 = attr<HALF>(sh, (int64_t)(3 * k + 1) * n + gi);
    const float f2 = attr<HALF>(sh, (int64_t)(3 * k + 2) * n + gi);
    const float w = fmaf(g[0], f0, fmaf(g[1], f1, g[2] * f2));
    gdir[0] = fmaf(w, dx, gdir[0]);
    gdir[1] = fmaf(w, dy, gdir[1]);
    gdir[2] = fmaf(w, dz, gdir[2]);
    sink.sh(3 * k + 0, Y * g[0]);
    sink.sh(3 * k + 1, Y * g[1]);
    sink.sh(3 * k + 2, Y * g[2]);
  };
  const float k1 = (float)kSH1, k2a = (float)kSH2a, k2b = (float)kSH2b, k2c = (float)kSH2c;
  const float k3a = (float)kSH3a, k3b = (float)kSH3b, k3c = (float)kSH3c, k3d = (float)kSH3d, k3e = (float)kSH3e;
  term(0, (float)kSH00, 0.f, 0.f, 0.f);
  if (deg < 1) return;
  term(1, -k1 * y, 0.f, -k1, 0.f);
  term(2, k1 * z, 0.f, 0.f, k1);
  term(3, -k1 * x, -k1, 0.f, 0.f);
  if (deg < 2) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  term(4, k2a * x * y, k2a * y, k2a * x, 0.f);
  term(5, -k2a * y * z, 0.f, -k2a * z, -k2a * y);
  term(6, k2b * (2.f * zz - xx - yy), -2.f * k2b * x, -2.f * k2b * y, 4.f * k2b * z);
  term(7, -k2a * x * z, -k2a * z, 0.f, -k2a * x);
  term(8, k2c * (xx - yy), 2.f * k2c * x, -2.f * k2c * y, 0.f);
  if (deg < 3) return;
  term(9, -k3a * y * (3.f * xx - yy), -6.f * k3a * x * y, -3.f * k3a * (xx - yy), 0.f);
  term(10, k3b * x * y * z, k3b * y * z, k3b * x * z, k3b * x * y);
  term(11, -k3c * y * (4.f * zz - xx - yy), 2.f * k3c * x * y, -k3c * (4.f * zz - xx - 3.f * yy), -8.f * k3c * y * z);
  term(12, k3d * z * (2.f * zz - 3.f * xx - 3.f * yy), -6.f * k3d * x * z, -6.f * k3d * y * z,
       k3d * (6.f * zz - 3.f * xx - 3.f * yy));
  term(13, -k3c * x * (4.f * zz - xx - yy), -k3c * (4.f * zz - 3.f * xx - yy), 2.f * k3c * x * y, -8.f * k3c * x * z);
  term(14, k3e * z * (xx - yy), 2.f * k3e * x * z, -2.f * k3e * y * z, k3e * (xx - yy));
  term(15, -k3a * x * (xx - 3.f * yy), -3.f * k3a * (xx - yy), 6.f * k3a * x * y, 0.f);
}

// Record g's 2D gradient (colour, opacity, conic and mean partials); false if
// it is all zero (a culled record, or one no pixel's loss depends on).
__device__ __forceinline__ bool load_grad2d(const float* __restrict__ grad2d, int64_t g, float (&p2)[kG]) {
  bool any = false;
#pragma unroll
  for (int q = 0; q < kG; ++q) {
    p2[q] = grad2d[g * kG + q];
    any |= p2[q] != 0.0f;
  }
  return any;
}

// One record's adjoint, for a record whose 2D gradient p2 is not all zero.
template <bool HALF, class Sink>
__device__ __forceinline__ void preprocess_bwd_record_t(const BwdArgs& a, const Record* __restrict__ records,
                                                        const float (&p2)[kG], int64_t g, int v, int l, int64_t gi,
                                                        Sink& sink) {
  const LevelPtrs& L = a.lv[l];
  const int64_t n = L.n;
  const gs_camera& cam = a.cams[v];
  // A record with a non-zero 2D gradient was visible in the forward pass, so
  // the projection below (same code, same inputs) takes the same decisions.
  // ---- colour first (FP32): clamped channels (record colour exactly 0) pass no gradient
  double dm_col[3];
  {
    const float4 w2 = reinterpret_cast<const float4*>(&records[g])[2];
    const float grgb[3] = {w2.x > 0.0f ? p2[0] : 0.0f, w2.y > 0.0f ? p2[1] : 0.0f, w2.z > 0.0f ? p2[2] : 0.0f};
    double C[3];
    camera_centre(cam, C);
    const double d0 = (double)L.means[gi] - C[0], d1 = (double)L.means[n + gi] - C[1],
                 d2 = (double)L.means[2 * n + gi] - C[2];
    const double dn = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
    const float dir[3] = {(float)(d0 / dn), (float)(d1 / dn), (float)(d2 / dn)};
    float gdir[3] = {0.0f, 0.0f, 0.0f};
    sh_adjoint<HALF>(dir[0], dir[1], dir[2], a.sh_degree < L.sh_deg ? a.sh_degree : L.sh_deg, L.sh, n, gi, grgb, sink,
                     gdir);
    const float gd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
    for (int k = 0; k < 3; ++k) dm_col[k] = (double)(gdir[k] - dir[k] * gd) / dn;
  }
  // ---- geometry adjoint (FP32); the guard-band clamp is decided in FP64 exactly as in the forward pass
  const double* R64 = cam.R;
  const double m0 = L.means[gi], m1 = L.means[n + gi], m2 = L.means[2 * n + gi];
  const double tx64 = ((R64[0] * m0 + R64[1] * m1) + R64[2] * m2) + cam.t[0];
  const double ty64 = ((R64[3] * m0 + R64[4] * m1) + R64[5] * m2) + cam.t[1];
  const double tz64 = ((R64[6] * m0 + R64[7] * m1) + R64[8] * m2) + cam.t[2];
  const double rz64 = 1.0 / tz64;
  const double ux64 = tx64 * rz64, uy64 = ty64 * rz64;
  const double limx = 1.3 * ((0.5 * a.W) / cam.fx), limy = 1.3 * ((0.5 * a.H) / cam.fy);
  const double uxc64 = dmin_(limx, dmax_(-limx, ux64)), uyc64 = dmin_(limy, dmax_(-limy, uy64));
  const bool clamp_x = uxc64 != ux64, clamp_y = uyc64 != uy64;
  const float tx = (float)tx64, ty = (float)ty64, rz = (float)rz64;
  const float uxc = (float)uxc64, uyc = (float)uyc64;
  const float fx = (float)cam.fx, fy = (float)cam.fy;
  float Rc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) Rc[k] = (float)R64[k];
  // rotation of the normalised quaternion, scales
  const float qa = attr<HALF>(L.quats, gi), qb = attr<HALF>(L.quats, n + gi), qc = attr<HALF>(L.quats, 2 * n + gi),
              qd_ = attr<HALF>(L.quats, 3 * n + gi);
  const float qinv = 1.0f / sqrtf(qa * qa + qb * qb + qc * qc + qd_ * qd_);
  const float w = qa * qinv, x = qb * qinv, y = qc * qinv, z = qd_ * qinv;
  float Rq[3][3];
  Rq[0][0] = 1.f - 2.f * (y * y + z * z);
  Rq[0][1] = 2.f * (x * y - w * z);
  Rq[0][2] = 2.f * (x * z + w * y);
  Rq[1][0] = 2.f * (x * y + w * z);
  Rq[1][1] = 1.f - 2.f * (x * x + z * z);
  Rq[1][2] = 2.f * (y * z - w * x);
  Rq[2][0] = 2.f * (x * z - w * y);
  Rq[2][1] = 2.f * (y * z + w * x);
  Rq[2][2] = 1.f - 2.f * (x * x + y * y);
  const float sc[3] = {attr<HALF>(L.scales, gi), attr<HALF>(L.scales, n + gi), attr<HALF>(L.scales, 2 * n + gi)};
  float WL[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      WL[i][j] = (Rc[3 * i] * Rq[0][j] + Rc[3 * i + 1] * Rq[1][j] + Rc[3 * i + 2] * Rq[2][j]) * sc[j];
  const float J00 = fx * rz, J02 = -(fx * uxc) * rz, J11 = fy * rz, J12 = -(fy * uyc) * rz;
  float M[2][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    M[0][j] = J00 * WL[0][j] + J02 * WL[2][j];
    M[1][j] = J11 * WL[1][j] + J12 * WL[2][j];
  }
  const float n0 = M[0][0] * M[0][0] + M[0][1] * M[0][1] + M[0][2] * M[0][2];
  const float n1 = M[1][0] * M[1][0] + M[1][1] * M[1][1] + M[1][2] * M[1][2];
  const float sb = M[0][0] * M[1][0] + M[0][1] * M[1][1] + M[0][2] * M[1][2];
  const float sa = n0 + 0.3f, sc2 = n1 + 0.3f;
  const float cr0 = M[0][1] * M[1][2] - M[0][2] * M[1][1];
  const float cr1 = M[0][2] * M[1][0] - M[0][0] * M[1][2];
  const float cr2 = M[0][0] * M[1][1] - M[0][1] * M[1][0];
  const float det = cr0 * cr0 + cr1 * cr1 + cr2 * cr2 + 0.3f * (n0 + n1) + 0.09f;
  // ---- 2D mean and conic partials ----
  const float kS = (float)kConicScale, kS2 = (float)kConicScale2;
  const float ca = kS * sqrtf(sc2 / det);
  const float cb = -kS * sb / sqrtf(sc2 * det);
  const float cc = kS / sqrtf(sc2);
  const float gu = -2.0f * ca * p2[4];
  const float gv = -2.0f * (cb * p2[4] + cc * p2[5]);
  const float gA = kS2 * p2[6], gB = 2.0f * kS2 * p2[7], gC = kS2 * p2[8];
  // conic K = Sigma2D^-1;  dL/dSigma = -K Gk K with Gk = [[gA, gB/2], [gB/2, gC]]
  const float KA = sc2 / det, KB = -sb / det, KC = sa / det;
  const float h = 0.5f * gB;
  const float t00 = gA * KA + h * KB, t01 = gA * KB + h * KC;
  const float t10 = h * KA + gC * KB, t11 = h * KB + gC * KC;
  const float S00 = -(KA * t00 + KB * t10);
  const float S01 = -(KA * t01 + KB * t11);
  const float S11 = -(KB * t01 + KC * t11);
  // Sigma2D = M M^T + 0.3 I -> dL/dM = 2 Gs M; M = J WL; WL = R_cam Rq diag(s), one column at a time
  float dJ00 = 0.f, dJ02 = 0.f, dJ11 = 0.f, dJ12 = 0.f;
  float ds[3], dRq[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float dM0 = 2.0f * (S00 * M[0][j] + S01 * M[1][j]);
    const float dM1 = 2.0f * (S01 * M[0][j] + S11 * M[1][j]);
    dJ00 += dM0 * WL[0][j];
    dJ02 += dM0 * WL[2][j];
    dJ11 += dM1 * WL[1][j];
    dJ12 += dM1 * WL[2][j];
    const float dW0 = J00 * dM0, dW1 = J11 * dM1, dW2 = J02 * dM0 + J12 * dM1;
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const float dLm = Rc[i] * dW0 + Rc[3 + i] * dW1 + Rc[6 + i] * dW2;  // (R_cam^T dWL)[i][j]
      acc += Rq[i][j] * dLm;
      dRq[i][j] = sc[j] * dLm;
    }
    ds[j] = acc;
  }
  float dq[4];
  dq[0] = 2.f * (-z * dRq[0][1] + y * dRq[0][2] + z * dRq[1][0] - x * dRq[1][2] - y * dRq[2][0] + x * dRq[2][1]);
  dq[1] = 2.f * (y * dRq[0][1] + z * dRq[0][2] + y * dRq[1][0] - w * dRq[1][2] + z * dRq[2][0] + w * dRq[2][1]) -
          4.f * x * (dRq[1][1] + dRq[2][2]);
  dq[2] = 2.f * (x * dRq[0][1] + w * dRq[0][2] + x * dRq[1][0] + z * dRq[1][2] - w * dRq[2][0] + z * dRq[2][1]) -
          4.f * y * (dRq[0][0] + dRq[2][2]);
  dq[3] = 2.f * (-w * dRq[0][1] + x * dRq[0][2] + w * dRq[1][0] + y * dRq[1][2] + x * dRq[2][0] + y * dRq[2][1]) -
          4.f * z * (dRq[0][0] + dRq[1][1]);
  const float qdot = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
  const float qn[4] = {w, x, y, z};
  float gq[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) gq[k] = (dq[k] - qn[k] * qdot) * qinv;
  // J(t) and (u, v)(t)
  const float rz2 = rz * rz;
  float dt0 = gu * fx * rz, dt1 = gv * fy * rz;
  float dt2 = -gu * fx * tx * rz2 - gv * fy * ty * rz2 - dJ00 * fx * rz2 - dJ11 * fy * rz2;
  if (!clamp_x) {
    dt0 += -dJ02 * fx * rz2;
    dt2 += dJ02 * 2.0f * fx * tx * rz2 * rz;
  } else {
    dt2 += dJ02 * fx * uxc * rz2;
  }
  if (!clamp_y) {
    dt1 += -dJ12 * fy * rz2;
    dt2 += dJ12 * 2.0f * fy * ty * rz2 * rz;
  } else {
    dt2 += dJ12 * fy * uyc * rz2;
  }
  float dm[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) dm[k] = Rc[k] * dt0 + Rc[3 + k] * dt1 + Rc[6 + k] * dt2 + (float)dm_col[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    sink.mean(k, dm[k]);
    sink.scale(k, ds[k]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) sink.quat(k, gq[k]);
  sink.opac(p2[3]);
}

template <bool SINGLE>
__device__ __forceinline__ void preprocess_bwd_record(const BwdArgs& a, const Record* __restrict__ records,
                                                      const float (&p2)[kG], int64_t g, int v, int l, int64_t gi) {
  if constexpr (SINGLE) {
    RegisterSink acc;
    if (a.lv[l].half) preprocess_bwd_record_t<true>(a, records, p2, g, v, l, gi, acc);
    else preprocess_bwd_record_t<false>(a, records, p2, g, v, l, gi, acc);
    acc.flush(a.gr[l], a.lv[l].n, gi, (a.lv[l].sh_deg + 1) * (a.lv[l].sh_deg + 1));
  } else {
    AtomicSink sink{a.gr[l], a.lv[l].n, gi};
    if (a.lv[l].half) preprocess_bwd_record_t<true>(a, records, p2, g, v, l, gi, sink);
    else preprocess_bwd_record_t<false>(a, records, p2, g, v, l, gi, sink);
  }
}

// All records of Gaussian gi (index i in every view's selection), views in
// order, summed in registers and added to memory once.
template <bool HALF>
__device__ __forceinline__ void preprocess_bwd_gaussian(const BwdArgs& a, const Record* __restrict__ records,
                                                        const float* __restrict__ grad2d, int64_t n_rec,
                                                        int64_t n_view, int64_t i, int l, int64_t gi) {
  RegisterSink acc;
  bool any = false;
  for (int v = 0; v < a.V; ++v) {
    const int64_t g = (int64_t)v * n_view + i;
    if (g >= n_rec) break;
    float p2[kG];
    if (!load_grad2d(grad2d, g, p2)) continue;
    preprocess_bwd_record_t<HALF>(a, records, p2, g, v, l, gi, acc);
    any = true;
  }
  if (any) acc.flush(a.gr[l], a.lv[l].n, gi, (a.lv[l].sh_deg + 1) * (a.lv[l].sh_deg + 1));
}

// View-major: records in index order, gradients added with no-return atomics
// (SINGLE: one view, each Gaussian has at most one record: register sums
// flushed with all loads ahead of the stores).
template <bool SINGLE>
__global__ void __launch_bounds__(256) preprocess_bwd_kernel(BwdArgs a, const Record* __restrict__ records,
                                                             const float* __restrict__ grad2d,
                                                             const int64_t* __restrict__ counts) {
  int64_t n_rec = counts[GS_COUNT_RECORDS];
  if (n_rec > a.capacity) n_rec = a.capacity;
  const int nseg = a.V * a.segs;
  // segment offsets staged in LDS when they fit; a record is looked up only
  // once its 2D gradient is known to be non-zero (most selected records were culled)
  __shared__ int64_t s_off[kBwdLdsOffsets];
  const bool lds_off = nseg < kBwdLdsOffsets;
  if (lds_off)
    for (int k = threadIdx.x; k <= nseg; k += blockDim.x) s_off[k] = a.offsets[k];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_rec; g += stride) {
    float p2[kG];
    if (!load_grad2d(grad2d, g, p2)) continue;
    const int p = lds_off ? find_segment(s_off, nseg, g) : find_segment(a.offsets, nseg, g);
    const int v = p / a.segs, b = p - v * a.segs;
    int l;
    int64_t gi;
    if (a.packed) {  // refined selection: the entry names the level and the index
      const uint32_t e = a.gather[g];
      l = (int)(e >> GS_PACKED_INDEX_BITS);
      gi = (int64_t)(e & ((1u << GS_PACKED_INDEX_BITS) - 1u));
      if (l >= a.L || gi >= a.lv[l].n) continue;  // not a stored Gaussian (the forward culled it)
    } else {
      l = a.gather ? b : a.level[p];
      const int64_t seg0 = lds_off ? s_off[p] : a.offsets[p];
      gi = a.gather ? (int64_t)a.gather[g] : a.lvl_off[(int64_t)b * a.L + l] + (g - seg0);
    }
    preprocess_bwd_record<SINGLE>(a, records, p2, g, v, l, gi);
  }
}

// Gaussian-major (every view selected the same records): one thread owns a
// Gaussian's records in all views and sums its gradient in registers.
__global__ void __launch_bounds__(256) preprocess_bwd_shared_kernel(BwdArgs a, const Record* __restrict__ records,
                                                                    const float* __restrict__ grad2d,
                                                                    const int64_t* __restrict__ counts) {
  if (counts[GS_COUNT_FLAGS] & GS_FLAG_SELECTION) return;  // the forward projected nothing
  int64_t n_rec = counts[GS_COUNT_RECORDS];
  if (n_rec > a.capacity) n_rec = a.capacity;
  const int64_t n_view = a.offsets[a.segs];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_view; i += stride) {
    const int b = find_segment(a.offsets, a.segs, i);
    const int l = a.gather ? b : a.level[b];
    const int64_t gi = a.gather ? (int64_t)a.gather[i] : a.lvl_off[(int64_t)b * a.L + l] + (i - a.offsets[b]);
    if (a.lv[l].half) preprocess_bwd_gaussian<true>(a, records, grad2d, n_rec, n_view, i, l, gi);
    else preprocess_bwd_gaussian<false>(a, records, grad2d, n_rec, n_view, i, l, gi);
  }
}

// Deterministic mode with several views that selected different blocks or
// levels (block-wise): one thread per stored Gaussian of every level sums its
// records over the views in view order (record of view v: the view chose the
// Gaussian's block at the Gaussian's level) and adds the total once.
__global__ void __launch_bounds__(256) preprocess_bwd_det_kernel(BwdArgs a, const Record* __restrict__ records,
                                                                 const float* __restrict__ grad2d,
                                                                 const int64_t* __restrict__ counts,
                                                                 int64_t n_stored) {
  int64_t n_rec = counts[GS_COUNT_RECORDS];
  if (n_rec > a.capacity) n_rec = a.capacity;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_stored; t += stride) {
    int l = 0;
    int64_t gi = t;
    while (l < a.L - 1 && gi >= a.lv[l].n) gi -= a.lv[l++].n;
    // block of gi in level l: blocks are stored in block order, so the last block
    // whose first index is <= gi (then checked against its count)
    int lo = 0, hi = a.B - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.lvl_off[(int64_t)mid * a.L + l] <= gi) lo = mid;
      else hi = mid - 1;
    }
    const int b = lo;
    const int64_t first = a.lvl_off[(int64_t)b * a.L + l];
    if (gi < first || gi >= first + a.lvl_cnt[(int64_t)b * a.L + l]) continue;
    RegisterSink acc;
    bool any = false;
    for (int v = 0; v < a.V; ++v) {
      const int64_t p = (int64_t)v * a.B + b;
      if (a.level[p] != l) continue;
      const int64_t g = a.offsets[p] + (gi - first);
      if (g >= n_rec) continue;
      float p2[kG];
      if (!load_grad2d(grad2d, g, p2)) continue;
      if (a.lv[l].half) preprocess_bwd_record_t<true>(a, records, p2, g, v, l, gi, acc);
      else preprocess_bwd_record_t<false>(a, records, p2, g, v, l, gi, acc);
      any = true;
    }
    if (any) acc.flush(a.gr[l], a.lv[l].n, gi, (a.lv[l].sh_deg + 1) * (a.lv[l].sh_deg + 1));
  }
}

__global__ void clear_floats_kernel(float* __restrict__ p, const int64_t* counts, int64_t cap, int per_record) {
  int64_t n = counts[GS_COUNT_RECORDS];
  if (n > cap) n = cap;
  const int64_t words = n * per_record;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < words; k += stride) p[k] = 0.0f;
}

template <int TW, int TH>
void launch_bwd(int batch, bool det, const TileArgs& ta, uint32_t* queue, hipStream_t s, const float* rgb,
                const float* T, const int32_t* nl, const float* drgb, float* g2d, const DetArgs& d) {
  constexpr int NT = TW * TH;
  const dim3 grid = tile_grid(ta.n_tiles, queue != nullptr);
  if (det) {
    // per-quadrant slots: 64 staged records per round (32 for the largest tile), under 40 KB of LDS
    constexpr int DB = TW * TH > 256 ? 32 : 64;
    hipLaunchKernelGGL((raster_bwd_kernel<TW, TH, DB, true>), grid, dim3(NT), 0, s, ta, queue, rgb, T, nl, drgb, g2d,
                       d);
  } else if (batch == 64) {
    hipLaunchKernelGGL((raster_bwd_kernel<TW, TH, 64, false>), grid, dim3(NT), 0, s, ta, queue, rgb, T, nl, drgb,
                       g2d, d);
  } else if (batch == 128) {
    hipLaunchKernelGGL((raster_bwd_kernel<TW, TH, 128, false>), grid, dim3(NT), 0, s, ta, queue, rgb, T, nl, drgb,
                       g2d, d);
  } else {
    hipLaunchKernelGGL((raster_bwd_kernel<TW, TH, 256, false>), grid, dim3(NT), 0, s, ta, queue, rgb, T, nl, drgb,
                       g2d, d);
  }
}

// workspace: grad2d [rc][kG]; deterministic mode adds cnt [rc], base [rc], a
// cursor and partial [slots][kG] with one slot per pair of pair capacity
struct BwdWs {
  float* grad2d;
  uint32_t* cnt;
  uint32_t* base;
  uint32_t* cursor;
  float* partial;
  size_t fixed_bytes;  // everything but the slots
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

BwdWs bwd_ws_layout(char* p, int64_t rc, bool det) {
  BwdWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = p ? p + off : nullptr;
    off = align256(off + bytes);
    return q;
  };
  w.grad2d = (float*)take((size_t)rc * kG * sizeof(float));
  if (det) {
    w.cnt = (uint32_t*)take((size_t)rc * 4);
    w.base = (uint32_t*)take((size_t)rc * 4);
    w.cursor = (uint32_t*)take(4);
    w.partial = (float*)(p ? p + off : nullptr);
  }
  w.fixed_bytes = off;
  return w;
}

}  // namespace

size_t rasterize_bwd_ws_bytes(int64_t rc, int64_t pc, bool det) {
  const size_t fixed = bwd_ws_layout(nullptr, rc, det).fixed_bytes;
  return det ? fixed + (size_t)pc * kG * sizeof(float) : fixed + 256;
}

}  // namespace gs

extern "C" gs_status gs_rasterize_bwd(const void* records, const uint32_t* pair_records, const uint32_t* tile_ranges,
                                      uint32_t* tile_queue, int32_t n_views, int32_t width, int32_t height,
                                      const float* bg,
                                      const gs_tuning* tuning, const float* rgb, const float* T_final,
                                      const int32_t* n_last, const float* d_rgb, const gs_gaussians* levels,
                                      const gs_blocks* blocks, const int8_t* level, const int64_t* offsets,
                                      const uint32_t* gather, const gs_camera* cams, int32_t sh_degree,
                                      int64_t record_capacity,
                                      const int64_t* counts, const gs_gaussian_grads* grads, void* ws,
                                      size_t ws_bytes, void* stream) {
  using namespace gs;
  (void)bg;  // the background enters through the saved forward colour
  if (!records || !pair_records || !tile_ranges || !tuning || !rgb || !T_final || !n_last || !d_rgb || !levels ||
      !blocks || (!level && !gather) || !offsets || !cams || !counts || !grads || !ws)
    return GS_ERR_INVALID_ARG;
  if (n_views <= 0 || width <= 0 || height <= 0 || width > 65535 || height > 65535) return GS_ERR_INVALID_ARG;
  if (sh_degree < 0 || sh_degree > 3 || record_capacity <= 0) return GS_ERR_INVALID_ARG;
  if (blocks->n_levels <= 0 || blocks->n_levels > kMaxLevels) return GS_ERR_INVALID_ARG;
  if (!gather && (blocks->n_blocks <= 0 || !blocks->lvl_off)) return GS_ERR_INVALID_ARG;
  const int tw = tuning->tile_w, th = tuning->tile_h;
  if (!tile_shape_supported(tw, th) || !batch_supported(tuning->batch)) return GS_ERR_UNSUPPORTED;
  const bool packed = (tuning->flags & GS_TUNE_PACKED_SELECTION) != 0;
  if (packed && !gather) return GS_ERR_INVALID_ARG;
  const bool det = (tuning->flags & GS_TUNE_DETERMINISTIC) != 0;
  const bool shared = (tuning->flags & GS_TUNE_SHARED_SELECTION) && n_views > 1;
  // decided before any launch: the Gaussian-major adjoint takes block-wise selections only, and the
  // deterministic adjoint of several different selections needs the block-wise level table
  if (shared && gather) return GS_ERR_UNSUPPORTED;
  if (det && gather && n_views > 1 && !shared) return GS_ERR_UNSUPPORTED;
  if (det && !shared && n_views > 1 && !blocks->lvl_cnt) return GS_ERR_INVALID_ARG;
  if (ws_bytes < rasterize_bwd_ws_bytes(record_capacity, 0, det)) return GS_ERR_WORKSPACE;
  const BwdWs w = bwd_ws_layout((char*)ws, record_capacity, det);
  float* grad2d = w.grad2d;
  DetArgs d{};
  if (det) {
    d.partial = w.partial;
    d.base = w.base;
    d.slots = (int64_t)((ws_bytes - w.fixed_bytes) / (kG * sizeof(float)));
  }
  const int tx = tiles_x(width, tw), ty = tiles_y(height, th);
  const int64_t tpv = (int64_t)tx * ty;
  const int64_t nblocks = tpv * n_views;
  if (nblocks >= ((int64_t)1 << 31)) return GS_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  int64_t cg = (record_capacity * kG + 255) / 256;
  hipLaunchKernelGGL(clear_floats_kernel, dim3((unsigned)(cg < 4096 ? (cg < 1 ? 1 : cg) : 4096)), dim3(256), 0, s,
                     grad2d, counts, record_capacity, kG);
  GS_LAUNCH_CHECK();
  const unsigned rg = (unsigned)(cg < 4096 ? (cg < 1 ? 1 : cg) : 4096);
  if (det) {
    // slots: count each record's pairs, then give each record a run of that many
    hipLaunchKernelGGL(det_clear_kernel, dim3(rg), dim3(256), 0, s, w.cnt, w.cursor, counts, record_capacity);
    hipLaunchKernelGGL(det_count_kernel, dim3(4096), dim3(256), 0, s, pair_records, counts, d.slots, w.cnt);
    hipLaunchKernelGGL(det_base_kernel, dim3(2048), dim3(256), 0, s, w.cnt, counts, record_capacity, w.cursor,
                       w.base);
    GS_LAUNCH_CHECK();
  }
  const Record* rec = (const Record*)records;
  const TileArgs ta{rec, pair_records, tile_ranges, width, height, tx, (int)tpv, nblocks};
  uint32_t* q = ((tuning->flags & GS_TUNE_WORK_QUEUE) && tile_queue) ? tile_queue : nullptr;
  const int b = tuning->batch;
  if (tw == 16 && th == 16) launch_bwd<16, 16>(b, det, ta, q, s, rgb, T_final, n_last, d_rgb, grad2d, d);
  else if (tw == 8 && th == 8) launch_bwd<8, 8>(b, det, ta, q, s, rgb, T_final, n_last, d_rgb, grad2d, d);
  else if (tw == 16 && th == 8) launch_bwd<16, 8>(b, det, ta, q, s, rgb, T_final, n_last, d_rgb, grad2d, d);
  else if (tw == 32 && th == 8) launch_bwd<32, 8>(b, det, ta, q, s, rgb, T_final, n_last, d_rgb, grad2d, d);
  else launch_bwd<32, 16>(b, det, ta, q, s, rgb, T_final, n_last, d_rgb, grad2d, d);
  GS_LAUNCH_CHECK();
  if (det) {
    hipLaunchKernelGGL(det_reduce_kernel, dim3(rg), dim3(256), 0, s, w.partial, w.cnt, w.base, counts,
                       record_capacity, d.slots, grad2d);
    GS_LAUNCH_CHECK();
  }
  BwdArgs a{};
  for (int l = 0; l < blocks->n_levels; ++l) {
    const gs_gaussians& g = levels[l];
    if (g.sh_degree < 0 || g.sh_degree > 3 || (g.attr_half != 0 && g.attr_half != 1)) return GS_ERR_INVALID_ARG;
    a.lv[l] = level_ptrs(g);
    a.gr[l] = grads[l];
    if (g.n > 0 && (!grads[l].means || !grads[l].scales || !grads[l].quats || !grads[l].opac || !grads[l].sh))
      return GS_ERR_INVALID_ARG;
  }
  a.lvl_off = blocks->lvl_off;
  a.lvl_cnt = blocks->lvl_cnt;
  a.level = level;
  a.offsets = offsets;
  a.gather = gather;
  a.segs = packed ? 1 : gather ? blocks->n_levels : blocks->n_blocks;
  a.packed = packed ? 1 : 0;
  a.cams = cams;
  a.capacity = record_capacity;
  a.B = blocks->n_blocks;
  a.L = blocks->n_levels;
  a.V = n_views;
  a.W = width;
  a.H = height;
  a.sh_degree = sh_degree;
  int64_t gb = (record_capacity + 255) / 256;
  const dim3 gbg((unsigned)(gb < 8192 ? (gb < 1 ? 1 : gb) : 8192));
  if ((tuning->flags & GS_TUNE_SHARED_SELECTION) && n_views > 1) {
    if (gather) return GS_ERR_UNSUPPORTED;
    int64_t pv = (record_capacity / n_views + 255) / 256;
    const dim3 gs_grid((unsigned)(pv < 8192 ? (pv < 1 ? 1 : pv) : 8192));
    hipLaunchKernelGGL(preprocess_bwd_shared_kernel, gs_grid, dim3(256), 0, s, a, rec, grad2d, counts);
  } else if (n_views == 1) {
    hipLaunchKernelGGL(preprocess_bwd_kernel<true>, gbg, dim3(256), 0, s, a, rec, grad2d, counts);
  } else if (det) {
    if (!blocks->lvl_cnt) return GS_ERR_INVALID_ARG;
    int64_t n_stored = 0;
    for (int l = 0; l < blocks->n_levels; ++l) n_stored += levels[l].n;
    int64_t sb = (n_stored + 255) / 256;
    const dim3 sg((unsigned)(sb < 8192 ? (sb < 1 ? 1 : sb) : 8192));
    hipLaunchKernelGGL(preprocess_bwd_det_kernel, sg, dim3(256), 0, s, a, rec, grad2d, counts, n_stored);
  } else {
    hipLaunchKernelGGL(preprocess_bwd_kernel<false>, gbg, dim3(256), 0, s, a, rec, grad2d, counts);
  }
  GS_LAUNCH_CHECK();
  return GS_OK;
}
