// Per-tile alpha compositing (Eq. 1 of the paper) and its adjoint.
//
// Forward: one work-group per (view, tile); one lane per pixel, so a 16x16
// tile is four wave64s covering 16x4 pixel strips.  The tile's Gaussians are
// staged through LDS in batches (coalesced gathers of 48-byte records, one per
// lane); every lane then reads the same LDS record (a broadcast, no bank
// conflicts).  A lane leaves the loop when its transmittance would drop below
// 1e-4; a wave leaves when all its lanes have, the work-group when all waves
// have (block-wide vote before each batch).
//
// Backward: the same walk, front to back, bounded by each pixel's n_last, with
// the blend state recomputed (colour in front is accumulated, colour behind =
// final colour - accumulated), so nothing per (pixel, Gaussian) is stored.
// The nine per-Gaussian partial gradients of a wave are summed with DPP row
// operations, added into LDS across the tile's waves, and flushed with one
// FP32 atomic per (tile, Gaussian, quantity).
//
// Compiled with -ffp-contract=off: alpha is computed by exactly the same
// operations in both kernels (explicit fmaf), so the backward's recomputed
// decisions match the forward's.
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

__device__ __forceinline__ void evaluate(const float4& w0, const float4& w1, int di, int dj, Eval& e) {
  e.dx = ((float)di + 0.5f) - w0.x;
  e.dy = ((float)dj + 0.5f) - w0.y;
  e.p1 = fmaf(w1.x, e.dx, w1.y * e.dy);
  e.p2 = w1.z * e.dy;
  e.G = __builtin_amdgcn_exp2f(-fmaf(e.p1, e.p1, e.p2 * e.p2));
  e.alpha = fminf(kAlphaMax, w1.w * e.G);
}

// Each wave keeps the indices of the staged records whose footprint rows meet
// its own pixel rows (ballot compaction), so the blend loop never visits a
// record that cannot touch the wave.
template <int TW, int BATCH>
__device__ __forceinline__ int wave_compact_rows(const float4* s_w0, int nb, int row0, int row1, uint16_t* list) {
  const int lane = threadIdx.x & 63;
  int cnt = 0;
  for (int base = 0; base < nb; base += 64) {
    const int k = base + lane;
    bool hit = false;
    if (k < nb) {
      const uint32_t py = __float_as_uint(s_w0[k].w);
      const int j0 = (int)(py & 0xFFFFu), j1 = j0 + (int)(py >> 16);
      hit = !(j1 < row0 || j0 > row1);
    }
    const uint64_t m = __ballot(hit);
    if (hit) list[cnt + (int)lanemask_lt_count(m)] = (uint16_t)k;
    cnt += (int)__popcll(m);
  }
  return cnt;
}

template <int TW, int TH, int BATCH>
__global__ void __launch_bounds__(TW* TH) raster_fwd_kernel(const Record* __restrict__ records,
                                                            const uint32_t* __restrict__ pair_records,
                                                            const uint32_t* __restrict__ ranges, int W, int H,
                                                            int tiles_x_n, int tiles_per_view, float bg0, float bg1,
                                                            float bg2, float* __restrict__ rgb,
                                                            float* __restrict__ T_final,
                                                            int32_t* __restrict__ n_last) {
  constexpr int NT = TW * TH;
  constexpr int NW = NT / 64;
  __shared__ float4 s_w0[BATCH], s_w1[BATCH], s_w2[BATCH];
  __shared__ uint16_t s_list[NW][BATCH];
  const int tile_g = blockIdx.x;
  const int view = tile_g / tiles_per_view;
  const int tile = tile_g - view * tiles_per_view;
  const int tyi = tile / tiles_x_n, txi = tile - tyi * tiles_x_n;
  const int i = txi * TW + (int)(threadIdx.x % TW);
  const int j = tyi * TH + (int)(threadIdx.x / TW);
  const bool inside = (i < W) && (j < H);
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  // rows covered by this wave (a wave is 64 consecutive pixels of the row-major tile)
  const int wave_row0 = tyi * TH + wid * (64 / TW);
  const int wave_row1 = wave_row0 + 64 / TW - 1;
  const uint32_t start = ranges[2 * tile_g], end = ranges[2 * tile_g + 1];
  float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  int last = 0;
  bool done = !inside;
  uint16_t* list = s_list[wid];
  for (uint32_t b = start; b < end; b += BATCH) {
    if (__syncthreads_and(done)) break;
    const int nb = (int)min((uint32_t)BATCH, end - b);
    for (int k = threadIdx.x; k < nb; k += NT) {
      const float4* r = reinterpret_cast<const float4*>(&records[pair_records[b + k]]);
      s_w0[k] = r[0];
      s_w1[k] = r[1];
      s_w2[k] = r[2];
    }
    __syncthreads();
    const int cnt = wave_compact_rows<TW, BATCH>(s_w0, nb, wave_row0, wave_row1, list);
    const int base_idx = (int)(b - start);
    if (cnt > 0 && __ballot(!done) != 0) {
      int k = __builtin_amdgcn_readfirstlane((int)list[0]);
      float4 w0 = s_w0[k], w1 = s_w1[k], w2 = s_w2[k];
      for (int t = 0; t < cnt; ++t) {
        // prefetch the next compacted record while this one is blended
        const int kn = __builtin_amdgcn_readfirstlane((int)list[t + 1 < cnt ? t + 1 : t]);
        const float4 n0 = s_w0[kn], n1 = s_w1[kn], n2 = s_w2[kn];
        int di, dj;
        const bool in_fp = in_footprint(i, j, __float_as_uint(w0.z), __float_as_uint(w0.w), di, dj);
        Eval e;
        evaluate(w0, w1, di, dj, e);
        bool use = !done && in_fp && (e.alpha >= kAlphaMin);
        const float Tn = T * (1.0f - e.alpha);
        const bool stop = use && (Tn < kTMin);
        done = done || stop;
        use = use && !stop;
        const float aT = e.alpha * T;
        C0 = use ? fmaf(w2.x, aT, C0) : C0;
        C1 = use ? fmaf(w2.y, aT, C1) : C1;
        C2 = use ? fmaf(w2.z, aT, C2) : C2;
        T = use ? Tn : T;
        last = use ? base_idx + k + 1 : last;
        if (__ballot(!done) == 0) break;
        k = kn;
        w0 = n0;
        w1 = n1;
        w2 = n2;
      }
    }
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

// ---------------------------------------------------------------------------
// wave64 sum with DPP row operations; the total ends in lane 63
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add(float v) {
  const int moved = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false);
  return v + __int_as_float(moved);
}

__device__ __forceinline__ float wave_sum_to_lane63(float v) {
  v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xF>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xF>(v);  // row_mirror: every lane of a row holds the row sum
  v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

constexpr int kG = 9;  // partials per Gaussian: r, g, b, opacity, A1, A2, Axx, Axy, Ayy

template <int TW, int TH, int BATCH>
__global__ void __launch_bounds__(TW* TH) raster_bwd_kernel(
    const Record* __restrict__ records, const uint32_t* __restrict__ pair_records,
    const uint32_t* __restrict__ ranges, int W, int H, int tiles_x_n, int tiles_per_view,
    const float* __restrict__ rgb, const float* __restrict__ T_final, const int32_t* __restrict__ n_last,
    const float* __restrict__ d_rgb, float* __restrict__ grad2d) {
  constexpr int NT = TW * TH;
  constexpr int NW = NT / 64;
  __shared__ float4 s_w0[BATCH], s_w1[BATCH], s_w2[BATCH];
  __shared__ uint32_t s_rec[BATCH];
  __shared__ float s_grad[BATCH * kG];
  __shared__ uint16_t s_list[NW][BATCH];
  __shared__ int s_wave_last[NW];
  const int tile_g = blockIdx.x;
  const int view = tile_g / tiles_per_view;
  const int tile = tile_g - view * tiles_per_view;
  const int tyi = tile / tiles_x_n, txi = tile - tyi * tiles_x_n;
  const int i = txi * TW + (int)(threadIdx.x % TW);
  const int j = tyi * TH + (int)(threadIdx.x / TW);
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const bool inside = (i < W) && (j < H);
  const int wave_row0 = tyi * TH + wid * (64 / TW);
  const int wave_row1 = wave_row0 + 64 / TW - 1;
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
  uint16_t* list = s_list[wid];
  float T = 1.0f, A0 = 0.f, A1c = 0.f, A2c = 0.f;  // transmittance and colour accumulated in front
  for (uint32_t b = start; b < start + (uint32_t)tile_last; b += BATCH) {
    const int nb = (int)min((uint32_t)BATCH, start + (uint32_t)tile_last - b);
    for (int k = threadIdx.x; k < nb; k += NT) {
      const uint32_t rid = pair_records[b + k];
      const float4* r = reinterpret_cast<const float4*>(&records[rid]);
      s_w0[k] = r[0];
      s_w1[k] = r[1];
      s_w2[k] = r[2];
      s_rec[k] = rid;
    }
    for (int k = threadIdx.x; k < nb * kG; k += NT) s_grad[k] = 0.0f;
    __syncthreads();
    const int base_idx = (int)(b - start);
    const int kmax = min(nb, wave_last - base_idx);  // entries past every lane's n_last are not needed
    const int cnt = kmax > 0 ? wave_compact_rows<TW, BATCH>(s_w0, kmax, wave_row0, wave_row1, list) : 0;
    for (int t = 0; t < cnt; ++t) {
      const int k = __builtin_amdgcn_readfirstlane((int)list[t]);
      const float4 w0 = s_w0[k], w1 = s_w1[k], w2 = s_w2[k];
      int di, dj;
      const bool in_fp = in_footprint(i, j, __float_as_uint(w0.z), __float_as_uint(w0.w), di, dj);
      Eval e;
      evaluate(w0, w1, di, dj, e);
      const bool use = (base_idx + k < last) && in_fp && (e.alpha >= kAlphaMin);
      if (__ballot(use) == 0) continue;
      const float aT = e.alpha * T;
      const float nA0 = fmaf(w2.x, aT, A0), nA1 = fmaf(w2.y, aT, A1c), nA2 = fmaf(w2.z, aT, A2c);
      const float inv1ma = 1.0f / (1.0f - e.alpha);
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
#pragma unroll
      for (int q = 0; q < kG; ++q) {
        const float sum = wave_sum_to_lane63(c[q]);
        if (lane == 63 && sum != 0.0f) atomicAdd(&s_grad[k * kG + q], sum);
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nb * kG; t += NT) {
      const float v = s_grad[t];
      if (v != 0.0f) unsafeAtomicAdd(&grad2d[(int64_t)s_rec[t / kG] * kG + (t % kG)], v);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// preprocess adjoint: per record, chain the 2D partials back to the parameters
// ---------------------------------------------------------------------------
struct BwdArgs {
  LevelPtrs lv[kMaxLevels];
  gs_gaussian_grads gr[kMaxLevels];
  const int64_t* lvl_off;
  const int8_t* level;
  const int64_t* offsets;
  const gs_camera* cams;
  int64_t capacity;
  int32_t B, L, V, W, H, sh_degree;
};

__global__ void __launch_bounds__(256) preprocess_bwd_kernel(BwdArgs a, const float* __restrict__ grad2d,
                                                             const int64_t* __restrict__ counts) {
  int64_t n_rec = counts[GS_COUNT_RECORDS];
  if (n_rec > a.capacity) n_rec = a.capacity;
  const int nseg = a.V * a.B;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_rec; g += stride) {
    float p2[kG];
    bool any = false;
#pragma unroll
    for (int q = 0; q < kG; ++q) {
      p2[q] = grad2d[g * kG + q];
      any |= p2[q] != 0.0f;
    }
    if (!any) continue;
    const int p = find_segment(a.offsets, nseg, g);
    const int v = p / a.B, b = p - v * a.B;
    const int l = a.level[p];
    const LevelPtrs& L = a.lv[l];
    const gs_gaussian_grads& G = a.gr[l];
    const int64_t n = L.n;
    const int64_t gi = a.lvl_off[(int64_t)b * a.L + l] + (g - a.offsets[p]);
    const gs_camera& cam = a.cams[v];
    Geo o;
    if (!project_geo(L, gi, cam, a.W, a.H, o)) continue;
    const double* R = cam.R;
    // ---- 2D mean and conic partials ----
    const double ca = kConicScale * sqrt(o.c / o.det);
    const double cb = -kConicScale * o.b / sqrt(o.c * o.det);
    const double cc = kConicScale / sqrt(o.c);
    const double gu = -2.0 * ca * p2[4];
    const double gv = -2.0 * (cb * p2[4] + cc * p2[5]);
    const double gA = kConicScale2 * p2[6];
    const double gB = 2.0 * kConicScale2 * p2[7];
    const double gC = kConicScale2 * p2[8];
    // conic K = Sigma2D^-1;  dL/dSigma = -K Gk K with Gk = [[gA, gB/2], [gB/2, gC]]
    const double KA = o.c / o.det, KB = -o.b / o.det, KC = o.a / o.det;
    const double h = 0.5 * gB;
    const double t00 = gA * KA + h * KB, t01 = gA * KB + h * KC;  // Gk K
    const double t10 = h * KA + gC * KB, t11 = h * KB + gC * KC;
    const double S00 = -(KA * t00 + KB * t10);
    const double S01 = -(KA * t01 + KB * t11);
    const double S11 = -(KB * t01 + KC * t11);
    // Sigma2D = M M^T + 0.3 I  ->  dL/dM = 2 Gs M, Gs = [[S00, S01], [S01, S11]]
    double dM[2][3];
    for (int jj = 0; jj < 3; ++jj) {
      dM[0][jj] = 2.0 * (S00 * o.M[0][jj] + S01 * o.M[1][jj]);
      dM[1][jj] = 2.0 * (S01 * o.M[0][jj] + S11 * o.M[1][jj]);
    }
    // M = J WL
    const double dJ00 = dM[0][0] * o.WL[0][0] + dM[0][1] * o.WL[0][1] + dM[0][2] * o.WL[0][2];
    const double dJ02 = dM[0][0] * o.WL[2][0] + dM[0][1] * o.WL[2][1] + dM[0][2] * o.WL[2][2];
    const double dJ11 = dM[1][0] * o.WL[1][0] + dM[1][1] * o.WL[1][1] + dM[1][2] * o.WL[1][2];
    const double dJ12 = dM[1][0] * o.WL[2][0] + dM[1][1] * o.WL[2][1] + dM[1][2] * o.WL[2][2];
    double dWL[3][3];
    for (int jj = 0; jj < 3; ++jj) {
      dWL[0][jj] = o.J00 * dM[0][jj];
      dWL[1][jj] = o.J11 * dM[1][jj];
      dWL[2][jj] = o.J02 * dM[0][jj] + o.J12 * dM[1][jj];
    }
    // WL = R_cam Lm,  Lm = Rq diag(s)
    double dLm[3][3];
    for (int ii = 0; ii < 3; ++ii)
      for (int jj = 0; jj < 3; ++jj)
        dLm[ii][jj] = R[ii] * dWL[0][jj] + R[3 + ii] * dWL[1][jj] + R[6 + ii] * dWL[2][jj];
    double ds[3], dRq[3][3];
    for (int jj = 0; jj < 3; ++jj) {
      ds[jj] = o.Rq[0][jj] * dLm[0][jj] + o.Rq[1][jj] * dLm[1][jj] + o.Rq[2][jj] * dLm[2][jj];
      for (int ii = 0; ii < 3; ++ii) dRq[ii][jj] = o.s[jj] * dLm[ii][jj];
    }
    // rotation matrix of the unit quaternion (w, x, y, z)
    const double w = o.q[0], x = o.q[1], y = o.q[2], z = o.q[3];
    double dq[4];
    dq[0] = 2.0 * (-z * dRq[0][1] + y * dRq[0][2] + z * dRq[1][0] - x * dRq[1][2] - y * dRq[2][0] + x * dRq[2][1]);
    dq[1] = 2.0 * (y * dRq[0][1] + z * dRq[0][2] + y * dRq[1][0] - w * dRq[1][2] + z * dRq[2][0] + w * dRq[2][1]) -
            4.0 * x * (dRq[1][1] + dRq[2][2]);
    dq[2] = 2.0 * (x * dRq[0][1] + w * dRq[0][2] + x * dRq[1][0] + z * dRq[1][2] - w * dRq[2][0] + z * dRq[2][1]) -
            4.0 * y * (dRq[0][0] + dRq[2][2]);
    dq[3] = 2.0 * (-w * dRq[0][1] + x * dRq[0][2] + w * dRq[1][0] + y * dRq[1][2] + x * dRq[2][0] + y * dRq[2][1]) -
            4.0 * z * (dRq[0][0] + dRq[1][1]);
    // normalisation q_hat = q / |q|
    const double qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
    double gq[4];
    for (int k = 0; k < 4; ++k) gq[k] = (dq[k] - o.q[k] * qd) * o.qinv;
    // J(t) and (u, v)(t)
    const double fx = cam.fx, fy = cam.fy, rz = o.rz, rz2 = rz * rz;
    double dt0 = gu * fx * rz, dt1 = gv * fy * rz;
    double dt2 = -gu * fx * o.tx * rz2 - gv * fy * o.ty * rz2;
    dt2 += -dJ00 * fx * rz2 - dJ11 * fy * rz2;
    if (!o.clamp_x) {
      dt0 += -dJ02 * fx * rz2;
      dt2 += dJ02 * 2.0 * fx * o.tx * rz2 * rz;
    } else {
      dt2 += dJ02 * fx * o.uxc * rz2;
    }
    if (!o.clamp_y) {
      dt1 += -dJ12 * fy * rz2;
      dt2 += dJ12 * 2.0 * fy * o.ty * rz2 * rz;
    } else {
      dt2 += dJ12 * fy * o.uyc * rz2;
    }
    double dm[3];
    for (int k = 0; k < 3; ++k) dm[k] = R[k] * dt0 + R[3 + k] * dt1 + R[6 + k] * dt2;
    // colour: SH coefficients and the view direction
    double C[3];
    camera_centre(cam, C);
    const double d0 = o.m[0] - C[0], d1 = o.m[1] - C[1], d2 = o.m[2] - C[2];
    const double dn = sqrt((d0 * d0 + d1 * d1) + d2 * d2);
    const double dir[3] = {d0 / dn, d1 / dn, d2 / dn};
    double Y[16], dY[16][3];
    const int nk = sh_basis(dir[0], dir[1], dir[2], a.sh_degree, Y);
    sh_basis_grad(dir[0], dir[1], dir[2], a.sh_degree, dY);
    double col[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < nk; ++k)
      for (int ch = 0; ch < 3; ++ch) col[ch] += Y[k] * (double)L.sh[(int64_t)(3 * k + ch) * n + gi];
    double grgb[3];
    for (int ch = 0; ch < 3; ++ch) grgb[ch] = (col[ch] + 0.5 >= 0.0) ? (double)p2[ch] : 0.0;
    double gdir[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < nk; ++k) {
      double wk = 0.0;
      for (int ch = 0; ch < 3; ++ch) {
        const double f = L.sh[(int64_t)(3 * k + ch) * n + gi];
        wk += grgb[ch] * f;
        const float gsh = (float)(Y[k] * grgb[ch]);
        if (gsh != 0.0f) unsafeAtomicAdd(&G.sh[(int64_t)(3 * k + ch) * n + gi], gsh);
      }
      gdir[0] += wk * dY[k][0];
      gdir[1] += wk * dY[k][1];
      gdir[2] += wk * dY[k][2];
    }
    const double gd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
    for (int k = 0; k < 3; ++k) dm[k] += (gdir[k] - dir[k] * gd) / dn;
    for (int k = 0; k < 3; ++k) {
      unsafeAtomicAdd(&G.means[k * n + gi], (float)dm[k]);
      unsafeAtomicAdd(&G.scales[k * n + gi], (float)ds[k]);
    }
    for (int k = 0; k < 4; ++k) unsafeAtomicAdd(&G.quats[k * n + gi], (float)gq[k]);
    unsafeAtomicAdd(&G.opac[gi], p2[3]);
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
void launch_fwd(int batch, dim3 grid, hipStream_t s, const Record* rec, const uint32_t* pr, const uint32_t* rg, int W,
                int H, int tx, int tpv, const float* bg, float* rgb, float* T, int32_t* nl) {
  constexpr int NT = TW * TH;
  if (batch == 64)
    hipLaunchKernelGGL((raster_fwd_kernel<TW, TH, 64>), grid, dim3(NT), 0, s, rec, pr, rg, W, H, tx, tpv, bg[0], bg[1],
                       bg[2], rgb, T, nl);
  else if (batch == 128)
    hipLaunchKernelGGL((raster_fwd_kernel<TW, TH, 128>), grid, dim3(NT), 0, s, rec, pr, rg, W, H, tx, tpv, bg[0],
                       bg[1], bg[2], rgb, T, nl);
  else
    hipLaunchKernelGGL((raster_fwd_kernel<TW, TH, 256>), grid, dim3(NT), 0, s, rec, pr, rg, W, H, tx, tpv, bg[0],
                       bg[1], bg[2], rgb, T, nl);
}

template <int TW, int TH>
void launch_bwd(int batch, dim3 grid, hipStream_t s, const Record* rec, const uint32_t* pr, const uint32_t* rg, int W,
                int H, int tx, int tpv, const float* rgb, const float* T, const int32_t* nl, const float* drgb,
                float* g2d) {
  constexpr int NT = TW * TH;
  if (batch == 64)
    hipLaunchKernelGGL((raster_bwd_kernel<TW, TH, 64>), grid, dim3(NT), 0, s, rec, pr, rg, W, H, tx, tpv, rgb, T, nl,
                       drgb, g2d);
  else if (batch == 128)
    hipLaunchKernelGGL((raster_bwd_kernel<TW, TH, 128>), grid, dim3(NT), 0, s, rec, pr, rg, W, H, tx, tpv, rgb, T,
                       nl, drgb, g2d);
  else
    hipLaunchKernelGGL((raster_bwd_kernel<TW, TH, 256>), grid, dim3(NT), 0, s, rec, pr, rg, W, H, tx, tpv, rgb, T,
                       nl, drgb, g2d);
}

bool batch_supported(int b) { return b == 64 || b == 128 || b == 256; }

}  // namespace

size_t rasterize_bwd_ws_bytes(int64_t rc) { return (size_t)rc * kG * sizeof(float) + 256; }

}  // namespace gs

extern "C" gs_status gs_rasterize_fwd(const void* records, const uint32_t* pair_records, const uint32_t* tile_ranges,
                                      int32_t n_views, int32_t width, int32_t height, const float* bg,
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
  const dim3 grid((unsigned)nblocks);
  hipStream_t s = (hipStream_t)stream;
  const Record* rec = (const Record*)records;
  const int b = tuning->batch;
  if (tw == 16 && th == 16) launch_fwd<16, 16>(b, grid, s, rec, pair_records, tile_ranges, width, height, tx, (int)tpv, bg, rgb, T_final, n_last);
  else if (tw == 8 && th == 8) launch_fwd<8, 8>(b, grid, s, rec, pair_records, tile_ranges, width, height, tx, (int)tpv, bg, rgb, T_final, n_last);
  else if (tw == 16 && th == 8) launch_fwd<16, 8>(b, grid, s, rec, pair_records, tile_ranges, width, height, tx, (int)tpv, bg, rgb, T_final, n_last);
  else if (tw == 32 && th == 8) launch_fwd<32, 8>(b, grid, s, rec, pair_records, tile_ranges, width, height, tx, (int)tpv, bg, rgb, T_final, n_last);
  else launch_fwd<32, 16>(b, grid, s, rec, pair_records, tile_ranges, width, height, tx, (int)tpv, bg, rgb, T_final, n_last);
  GS_LAUNCH_CHECK();
  return GS_OK;
}

extern "C" gs_status gs_rasterize_bwd(const void* records, const uint32_t* pair_records, const uint32_t* tile_ranges,
                                      int32_t n_views, int32_t width, int32_t height, const float* bg,
                                      const gs_tuning* tuning, const float* rgb, const float* T_final,
                                      const int32_t* n_last, const float* d_rgb, const gs_gaussians* levels,
                                      const gs_blocks* blocks, const int8_t* level, const int64_t* offsets,
                                      const gs_camera* cams, int32_t sh_degree, int64_t record_capacity,
                                      const int64_t* counts, const gs_gaussian_grads* grads, void* ws,
                                      size_t ws_bytes, void* stream) {
  using namespace gs;
  (void)bg;  // the background enters through the saved forward colour
  if (!records || !pair_records || !tile_ranges || !tuning || !rgb || !T_final || !n_last || !d_rgb || !levels ||
      !blocks || !level || !offsets || !cams || !counts || !grads || !ws)
    return GS_ERR_INVALID_ARG;
  if (n_views <= 0 || width <= 0 || height <= 0 || width > 65535 || height > 65535) return GS_ERR_INVALID_ARG;
  if (sh_degree < 0 || sh_degree > 3 || record_capacity <= 0) return GS_ERR_INVALID_ARG;
  if (blocks->n_blocks <= 0 || blocks->n_levels <= 0 || blocks->n_levels > kMaxLevels || !blocks->lvl_off)
    return GS_ERR_INVALID_ARG;
  const int tw = tuning->tile_w, th = tuning->tile_h;
  if (!tile_shape_supported(tw, th) || !batch_supported(tuning->batch)) return GS_ERR_UNSUPPORTED;
  if (ws_bytes < rasterize_bwd_ws_bytes(record_capacity)) return GS_ERR_WORKSPACE;
  float* grad2d = (float*)ws;
  const int tx = tiles_x(width, tw), ty = tiles_y(height, th);
  const int64_t tpv = (int64_t)tx * ty;
  const int64_t nblocks = tpv * n_views;
  if (nblocks >= ((int64_t)1 << 31)) return GS_ERR_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  int64_t cg = (record_capacity * kG + 255) / 256;
  hipLaunchKernelGGL(clear_floats_kernel, dim3((unsigned)(cg < 4096 ? (cg < 1 ? 1 : cg) : 4096)), dim3(256), 0, s,
                     grad2d, counts, record_capacity, kG);
  GS_LAUNCH_CHECK();
  const dim3 grid((unsigned)nblocks);
  const Record* rec = (const Record*)records;
  const int b = tuning->batch;
  if (tw == 16 && th == 16) launch_bwd<16, 16>(b, grid, s, rec, pair_records, tile_ranges, width, height, tx, (int)tpv, rgb, T_final, n_last, d_rgb, grad2d);
  else if (tw == 8 && th == 8) launch_bwd<8, 8>(b, grid, s, rec, pair_records, tile_ranges, width, height, tx, (int)tpv, rgb, T_final, n_last, d_rgb, grad2d);
  else if (tw == 16 && th == 8) launch_bwd<16, 8>(b, grid, s, rec, pair_records, tile_ranges, width, height, tx, (int)tpv, rgb, T_final, n_last, d_rgb, grad2d);
  else if (tw == 32 && th == 8) launch_bwd<32, 8>(b, grid, s, rec, pair_records, tile_ranges, width, height, tx, (int)tpv, rgb, T_final, n_last, d_rgb, grad2d);
  else launch_bwd<32, 16>(b, grid, s, rec, pair_records, tile_ranges, width, height, tx, (int)tpv, rgb, T_final, n_last, d_rgb, grad2d);
  GS_LAUNCH_CHECK();
  BwdArgs a{};
  for (int l = 0; l < blocks->n_levels; ++l) {
    const gs_gaussians& g = levels[l];
    a.lv[l] = LevelPtrs{g.means, g.scales, g.quats, g.opac, g.sh, g.n};
    a.gr[l] = grads[l];
    if (g.n > 0 && (!grads[l].means || !grads[l].scales || !grads[l].quats || !grads[l].opac || !grads[l].sh))
      return GS_ERR_INVALID_ARG;
  }
  a.lvl_off = blocks->lvl_off;
  a.level = level;
  a.offsets = offsets;
  a.cams = cams;
  a.capacity = record_capacity;
  a.B = blocks->n_blocks;
  a.L = blocks->n_levels;
  a.V = n_views;
  a.W = width;
  a.H = height;
  a.sh_degree = sh_degree;
  int64_t gb = (record_capacity + 255) / 256;
  hipLaunchKernelGGL(preprocess_bwd_kernel, dim3((unsigned)(gb < 8192 ? (gb < 1 ? 1 : gb) : 8192)), dim3(256), 0, s, a,
                     grad2d, counts);
  GS_LAUNCH_CHECK();
  return GS_OK;
}
