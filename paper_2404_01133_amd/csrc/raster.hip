// Per-tile alpha compositing (Eq. 1 of the paper), forward.
//
// One work-group per (view, tile); one lane per pixel, each wave64 an 8x8
// pixel block of the tile (a 16x16 tile is four waves), cut into eight 4x2
// pixel groups of 8 lanes.  The tile's Gaussians are staged through LDS in
// batches (coalesced gathers of 48-byte records, one per lane); each group
// keeps its own depth-ordered list of the staged records whose footprint meets
// it, and the groups walk their lists side by side (a lane reads the record of
// its group), so a small footprint occupies one group's step rather than a
// whole wave's.  A lane leaves the loop when its transmittance would drop below
// 1e-4; a wave leaves when all its lanes have, the work-group when all waves
// have (block-wide vote before each batch).
//
// Compiled with -ffp-contract=off: alpha is computed by exactly the same
// operations as in the adjoint (explicit fmaf), so the backward's recomputed
// decisions match the forward's.
#include "tile.h"

namespace gs {
namespace {

// group shapes: the forward blends in 4x2 groups (eight per wave), the
// backward in 4x4 quadrants (its partial sums run over 16 lanes)
constexpr int kFwdGW = 4, kFwdGH = 2;
constexpr int kFwdGroups = 64 / (kFwdGW * kFwdGH);
static_assert(kFwdGroups == 8, "the forward uses wave_compact8");

template <int TW, int TH, int BATCH>
struct FwdLds {
  float4 w0[BATCH], w1[BATCH], w2[BATCH];
  float4 f[BATCH];  // footprint as floats: i0, j0, i1 - i0, j1 - j0
  uint8_t list[(TW * TH) / 64][kFwdGroups][kListStride<BATCH>];
};

template <int TW, int TH, int BATCH>
__device__ __forceinline__ void raster_fwd_tile(const TileArgs& ta, FwdLds<TW, TH, BATCH>& lds, int tile_g,
                                                float bg0, float bg1, float bg2, float* __restrict__ rgb,
                                                float* __restrict__ T_final, int32_t* __restrict__ n_last) {
  constexpr int NT = TW * TH;
  const Record* __restrict__ records = ta.records;
  const uint32_t* __restrict__ pair_records = ta.pair_records;
  const uint32_t* __restrict__ ranges = ta.ranges;
  const int W = ta.W, H = ta.H, tiles_x_n = ta.tiles_x_n, tiles_per_view = ta.tiles_per_view;
  float4* s_w0 = lds.w0;
  float4* s_w1 = lds.w1;
  float4* s_w2 = lds.w2;
  float4* s_f = lds.f;
  const int view = tile_g / tiles_per_view;
  const int tile = tile_g - view * tiles_per_view;
  const int tyi = tile / tiles_x_n, txi = tile - tyi * tiles_x_n;
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const LaneMap<TW, TH, kFwdGW, kFwdGH> qb(txi, tyi, wid);
  const int i = qb.i, j = qb.j;
  const float fi = (float)i, fj = (float)j;
  const bool inside = (i < W) && (j < H);
  const uint32_t start = ranges[2 * tile_g], end = ranges[2 * tile_g + 1];
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  int last = 0;
  bool done = !inside;
  uint8_t(*lists)[kListStride<BATCH>] = lds.list[wid];
  const uint8_t* my_list = lists[qb.g];
  for (uint32_t b = start; b < end; b += BATCH) {
    if (__syncthreads_and(done)) break;
    const int nb = (int)min((uint32_t)BATCH, end - b);
    for (int k = threadIdx.x; k < nb; k += NT) {
      const float4* r = reinterpret_cast<const float4*>(&records[pair_records[b + k]]);
      const float4 a = r[0];
      s_w0[k] = a;
      s_w1[k] = r[1];
      s_w2[k] = r[2];
      const uint32_t px = __float_as_uint(a.z), py = __float_as_uint(a.w);
      s_f[k] = make_float4((float)(px & 0xFFFFu), (float)(py & 0xFFFFu), (float)(px >> 16), (float)(py >> 16));
    }
    // list entries past a group's count read stale indices that may land on
    // unstaged slots: their colour must be finite (it is multiplied by 0)
    for (int k = nb + threadIdx.x; k < BATCH; k += NT) s_w2[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    __syncthreads();
    const Counts8 cnt = wave_compact8<BATCH>(s_w0, nb, qb.x0, qb.y0, lists);
    const int max_cnt = cnt.max();
    const int my_cnt = cnt.of(qb.g);
    const int base_idx = (int)(b - start);
    int last_k = -1;  // 16 x the batch index of the last entry used in this batch
    auto blend = [&](int k, bool valid, float du, const float4& f, const float4& w1, const float4& w2) {
      Eval e;
      const bool in_fp = evaluate_f(fi, fj, f, du, w2.w, w1, e);
      bool use = valid && !done && in_fp && (e.alpha >= kAlphaMin);
      const float Tn = T * (1.0f - e.alpha);
      const bool stop = use && (Tn < kTMin);
      done = done || stop;
      use = use && !stop;
      // an unused entry adds colour * 0 (colours are finite): C is unchanged bit for bit
      const float aT = use ? e.alpha * T : 0.0f;
      C0 = fmaf(w2.x, aT, C0);
      C1 = fmaf(w2.y, aT, C1);
      C2 = fmaf(w2.z, aT, C2);
      T = use ? Tn : T;
      last_k = use ? k : last_k;
    };
    // four entries of the lane's group list per trip: one LDS read for the
    // four byte indices, all records' words in flight together, one vote per
    // trip (entries past the group's count are read from stale list bytes,
    // masked into the staged range and not used)
    for (int t = 0; t < max_cnt; t += 4) {
      if (__ballot(!done && t < my_cnt) == 0) break;
      // byte offsets (index * 16) of the four entries into the staged arrays
      const uint32_t pk = *reinterpret_cast<const uint32_t*>(&my_list[t]);
      const uint32_t o0 = (pk & (BATCH - 1)) << 4, o1 = ((pk >> 8) & (BATCH - 1)) << 4;
      const uint32_t o2 = ((pk >> 16) & (BATCH - 1)) << 4, o3 = ((pk >> 24) & (BATCH - 1)) << 4;
      auto at = [](const float4* a, uint32_t o) {
        return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(a) + o);
      };
      auto at_x = [](const float4* a, uint32_t o) {
        return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(a) + o);
      };
      const float au = at_x(s_w0, o0), bu = at_x(s_w0, o1), cu = at_x(s_w0, o2), du = at_x(s_w0, o3);
      const float4 af = at(s_f, o0), a1 = at(s_w1, o0), a2 = at(s_w2, o0);
      const float4 bf = at(s_f, o1), b1 = at(s_w1, o1), b2 = at(s_w2, o1);
      const float4 cf = at(s_f, o2), c1 = at(s_w1, o2), c2 = at(s_w2, o2);
      const float4 df = at(s_f, o3), d1 = at(s_w1, o3), d2 = at(s_w2, o3);
      blend((int)o0, t < my_cnt, au, af, a1, a2);
      blend((int)o1, t + 1 < my_cnt, bu, bf, b1, b2);
      blend((int)o2, t + 2 < my_cnt, cu, cf, c1, c2);
      blend((int)o3, t + 3 < my_cnt, du, df, d1, d2);
    }
    if (last_k >= 0) last = base_idx + (last_k >> 4) + 1;
    __syncthreads();
  }
  if (inside) {
    const int64_t plane = (int64_t)H * W;
    const int64_t pix = (int64_t)j * W + i;
    float* out = rgb + (int64_t)view * 3 * plane + pix;
    out[0] = fmaf(T, bg0, C0);
    out[plane] = fmaf(T, bg1, C1);
    out[2 * plane] = fmaf(T, bg2, C2);
    T_final[(int64_t)view * plane + pix] = T;
    n_last[(int64_t)view * plane + pix] = last;
  }
}

// Six waves per SIMD for the multi-wave tiles: at 80 registers the compiler
// spills six of them, and the sixth wave is still worth more than the freer
// allocation (one 8-view city call: 0.367 ms at six waves, 0.408 ms at five).
template <int TW, int TH, int BATCH>
__global__ void __launch_bounds__(TW* TH) __attribute__((amdgpu_waves_per_eu(TW * TH >= 128 ? 6 : 1))) raster_fwd_kernel(TileArgs ta, uint32_t* queue, float bg0, float bg1,
                                                            float bg2, float* __restrict__ rgb,
                                                            float* __restrict__ T_final,
                                                            int32_t* __restrict__ n_last) {
  __shared__ FwdLds<TW, TH, BATCH> lds;
  for_each_tile(ta, queue, 0, [&](int tile_g) {
    raster_fwd_tile<TW, TH, BATCH>(ta, lds, tile_g, bg0, bg1, bg2, rgb, T_final, n_last);
  });
}

template <int TW, int TH>
void launch_fwd(int batch, const TileArgs& ta, uint32_t* queue, hipStream_t s, const float* bg, float* rgb, float* T,
                int32_t* nl) {
  constexpr int NT = TW * TH;
  const dim3 grid = tile_grid(ta.n_tiles, queue != nullptr);
  if (batch == 64)
    hipLaunchKernelGGL((raster_fwd_kernel<TW, TH, 64>), grid, dim3(NT), 0, s, ta, queue, bg[0], bg[1], bg[2], rgb, T,
                       nl);
  else if (batch == 128)
    hipLaunchKernelGGL((raster_fwd_kernel<TW, TH, 128>), grid, dim3(NT), 0, s, ta, queue, bg[0], bg[1], bg[2], rgb,
                       T, nl);
  else
    hipLaunchKernelGGL((raster_fwd_kernel<TW, TH, 256>), grid, dim3(NT), 0, s, ta, queue, bg[0], bg[1], bg[2], rgb,
                       T, nl);
}

}  // namespace
}  // namespace gs

extern "C" gs_status gs_rasterize_fwd(const void* records, const uint32_t* pair_records, const uint32_t* tile_ranges,
                                      uint32_t* tile_queue, int32_t n_views, int32_t width, int32_t height,
                                      const float* bg,
                                      const gs_tuning* tuning, float* rgb, float* T_final, int32_t* n_last,
                                      void* stream) {
  using namespace gs;
  if (!records || !pair_records || !tile_ranges || !bg || !tuning || !rgb || !T_final || !n_last)
    return GS_ERR_INVALID_ARG;
  if (n_views <= 0 || width <= 0 || height <= 0 || width > 65535 || height > 65535) return GS_ERR_INVALID_ARG;
  const int tw = tuning->tile_w, th = tuning->tile_h;
  if (!tile_shape_supported(tw, th) || !batch_supported(tuning->batch)) return GS_ERR_UNSUPPORTED;
  const int tx = tiles_x(width, tw), ty = tiles_y(height, th);
  const int64_t tpv = (int64_t)tx * ty;
  const int64_t nblocks = tpv * n_views;
  if (nblocks >= ((int64_t)1 << 31)) return GS_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  const TileArgs ta{(const Record*)records, pair_records, tile_ranges, width, height, tx, (int)tpv, nblocks};
  uint32_t* q = ((tuning->flags & GS_TUNE_WORK_QUEUE) && tile_queue) ? tile_queue : nullptr;
  const int b = tuning->batch;
  if (tw == 16 && th == 16) launch_fwd<16, 16>(b, ta, q, s, bg, rgb, T_final, n_last);
  else if (tw == 8 && th == 8) launch_fwd<8, 8>(b, ta, q, s, bg, rgb, T_final, n_last);
  else if (tw == 16 && th == 8) launch_fwd<16, 8>(b, ta, q, s, bg, rgb, T_final, n_last);
  else if (tw == 32 && th == 8) launch_fwd<32, 8>(b, ta, q, s, bg, rgb, T_final, n_last);
  else launch_fwd<32, 16>(b, ta, q, s, bg, rgb, T_final, n_last);
  GS_LAUNCH_CHECK();
  return GS_OK;
}

