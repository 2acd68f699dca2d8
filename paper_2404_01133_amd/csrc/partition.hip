// Block partition of a Gaussian cloud (Sec. 3.2.2, Eq. 2): foreground
// normalisation, contraction of unbounded space into the cube (-2, 2)^3, a
// uniform grid over the contracted x and y, and the Gaussians grouped by
// block with their original order kept inside a block.
//
// Stages (all sizes known on the host, nothing synchronises):
//   1. z range of all centres (order-preserving integer min / max)
//   2. per centre: block id in FP64 (fixed operation order; this file is
//      compiled with -ffp-contract=off), (id, index) pairs, digit histograms
//   3. one or two stable 8-bit radix passes by block id (the binning's pass)
//   4. block offsets from the boundaries of the sorted ids
// plus a gather of all attribute arrays into the new order.
#include "radix.h"

namespace gs {
namespace {

struct PartArgs {
  const float* means;  // [3][n]
  int64_t n;
  double xlo, xhi, ylo, yhi;  // foreground x / y extent (lo < hi)
  const uint32_t* zr;         // device: order-mapped z min, z max
  int32_t nx, ny;
};

// float bits -> unsigned integer with the same order (and back)
__device__ __forceinline__ uint32_t order_key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float order_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__global__ void part_clear_kernel(uint32_t* __restrict__ words, int64_t n_words, int64_t* __restrict__ counts,
                                  int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += stride) words[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    words[0] = 0xFFFFFFFFu;  // z min (order-mapped), shrinks
    words[1] = 0u;           // z max (order-mapped), grows
    for (int k = 0; k < GS_COUNT_SLOTS; ++k) counts[k] = 0;
    counts[GS_COUNT_RECORDS] = n;
  }
}

__global__ void __launch_bounds__(256) zrange_kernel(const float* __restrict__ z, int64_t n, uint32_t* __restrict__ zr) {
  uint32_t lo = 0xFFFFFFFFu, hi = 0u;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t k = order_key(z[i]);
    lo = k < lo ? k : lo;
    hi = k > hi ? k : hi;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t a = __shfl_xor(lo, off, 64), b = __shfl_xor(hi, off, 64);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&zr[0], lo);
    atomicMax(&zr[1], hi);
  }
}

// index of the grid cell along one axis: the number of interior boundaries
// -2 + 4k/cells (k = 1 .. cells-1) that are <= c; a NaN coordinate gets 0
__device__ __forceinline__ int grid_index(double c, int cells) {
  if (!(c == c)) return 0;
  double e = (c + 2.0) * (double)cells * 0.25;  // estimate, corrected exactly below
  int k = e < 0.0 ? 0 : (e > (double)(cells - 1) ? cells - 1 : (int)e);
  while (k + 1 <= cells - 1 && (-2.0 + (4.0 * (double)(k + 1)) / (double)cells) <= c) ++k;
  while (k >= 1 && (-2.0 + (4.0 * (double)k) / (double)cells) > c) --k;
  return k;
}

__device__ __forceinline__ uint32_t block_of(const PartArgs& a, double zlo, double zhi, double x, double y,
                                             double z) {
  const double q0 = (2.0 * (x - a.xlo)) / (a.xhi - a.xlo) - 1.0;
  const double q1 = (2.0 * (y - a.ylo)) / (a.yhi - a.ylo) - 1.0;
  const double q2 = (2.0 * (z - zlo)) / (zhi - zlo) - 1.0;
  const double m0 = fabs(q0), m1 = fabs(q1), m2 = fabs(q2);
  const bool nan = !(m0 == m0) || !(m1 == m1) || !(m2 == m2);
  double nrm = m0 > m1 ? m0 : m1;
  nrm = m2 > nrm ? m2 : nrm;
  double c0 = q0, c1 = q1;
  if (!nan && nrm > 1.0) {  // Eq. 2, outer region
    const double s = 2.0 - 1.0 / nrm;
    c0 = s * (q0 / nrm);
    c1 = s * (q1 / nrm);
  }
  return (uint32_t)(grid_index(c1, a.ny) * a.nx + grid_index(c0, a.nx));
}

__global__ void __launch_bounds__(kThreads) part_ids_kernel(PartArgs a, uint32_t* __restrict__ keys,
                                                            uint32_t* __restrict__ vals,
                                                            uint32_t* __restrict__ block_id, int passes,
                                                            uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_hist[2][kRadix];
  for (int k = threadIdx.x; k < 2 * kRadix; k += kThreads) (&s_hist[0][0])[k] = 0u;
  __syncthreads();
  const double zlo = (double)order_value(a.zr[0]), zhi = (double)order_value(a.zr[1]);
  const int64_t n = a.n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const uint32_t b = block_of(a, zlo, zhi, (double)a.means[i], (double)a.means[n + i], (double)a.means[2 * n + i]);
    keys[i] = b;
    vals[i] = (uint32_t)i;
    if (block_id) block_id[i] = b;
    atomicAdd(&s_hist[0][b & 255u], 1u);
    if (passes > 1) atomicAdd(&s_hist[1][(b >> 8) & 255u], 1u);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < passes * kRadix; k += kThreads) {
    const uint32_t c = (&s_hist[0][0])[k];
    if (c) atomicAdd(&hist[k], c);
  }
}

// block_off[b] = first position of the sorted ids holding an id >= b
__global__ void part_offsets_kernel(const uint32_t* __restrict__ ids, int64_t n, int32_t n_blocks,
                                    int64_t* __restrict__ block_off) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += stride) {
    const int64_t cur = ids[j];
    const int64_t prev = j == 0 ? -1 : (int64_t)ids[j - 1];
    for (int64_t b = prev + 1; b <= cur; ++b) block_off[b] = j;
    if (j == n - 1)
      for (int64_t b = cur + 1; b <= n_blocks; ++b) block_off[b] = n;
  }
}

__global__ void part_empty_kernel(int64_t* __restrict__ block_off, int32_t n_blocks) {
  for (int b = threadIdx.x; b <= n_blocks; b += blockDim.x) block_off[b] = 0;
}

// cells of the grid in contracted coordinates (x0, x1, y0, y1): the boundaries
// grid_index compares against, outermost ends open, so a point's cell is its block
__global__ void part_cells_kernel(int32_t nx, int32_t ny, double* __restrict__ cells) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nx * ny) return;
  const int ix = b % nx, iy = b / nx;
  const double inf = __builtin_inf();
  double* c = cells + 4 * (int64_t)b;
  c[0] = ix == 0 ? -inf : -2.0 + (4.0 * (double)ix) / (double)nx;
  c[1] = ix == nx - 1 ? inf : -2.0 + (4.0 * (double)(ix + 1)) / (double)nx;
  c[2] = iy == 0 ? -inf : -2.0 + (4.0 * (double)iy) / (double)ny;
  c[3] = iy == ny - 1 ? inf : -2.0 + (4.0 * (double)(iy + 1)) / (double)ny;
}

// dst[c][k] = src[c][perm[k]] for every component array of a Gaussian set
__global__ void __launch_bounds__(256) gather_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                                     int comps, int64_t n_src, int64_t n,
                                                     const uint32_t* __restrict__ perm) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
    const int64_t s = perm[k];
    for (int c = 0; c < comps; ++c) dst[(int64_t)c * n + k] = src[(int64_t)c * n_src + s];
  }
}

struct PartWs {
  uint32_t* words;  // [0..1] z range, [2..7] tile counters, then hist [2][256]
  uint32_t* hist;
  uint32_t* status; // [2][ntiles][256]
  uint32_t* k0;
  uint32_t* v0;
  uint32_t* k1;
  uint32_t* v1;
  int64_t* counts;
  int64_t n_words;
  size_t bytes;
};

PartWs part_ws_layout(char* base, int64_t n) {
  PartWs w{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  w.n_words = 8 + 2 * kRadix + 2 * ntiles * kRadix;
  w.words = (uint32_t*)take(4 * (size_t)w.n_words);
  w.hist = w.words ? w.words + 8 : nullptr;
  w.status = w.words ? w.words + 8 + 2 * kRadix : nullptr;
  w.counts = (int64_t*)take(8 * GS_COUNT_SLOTS);
  w.k0 = (uint32_t*)take(4 * (size_t)n);
  w.v0 = (uint32_t*)take(4 * (size_t)n);
  w.k1 = (uint32_t*)take(4 * (size_t)n);
  w.v1 = (uint32_t*)take(4 * (size_t)n);
  w.bytes = off;
  return w;
}

unsigned grid_of(int64_t n, int64_t cap) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace
}  // namespace gs

extern "C" size_t gs_partition_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  return gs::part_ws_layout(nullptr, n).bytes;
}

extern "C" gs_status gs_partition(const float* means, int64_t n, const double* xy_box, int32_t nx, int32_t ny,
                                  uint32_t* block_id, uint32_t* perm, int64_t* block_off, double* cells, void* ws,
                                  size_t ws_bytes, void* stream) {
  using namespace gs;
  if (!xy_box || !block_off || n < 0 || (n > 0 && (!means || !perm || !ws))) return GS_ERR_INVALID_ARG;
  if (n >= ((int64_t)1 << 32)) return GS_ERR_INVALID_ARG;
  if (nx <= 0 || ny <= 0 || (int64_t)nx * ny > 65536) return GS_ERR_INVALID_ARG;
  PartArgs a{};
  a.means = means;
  a.n = n;
  a.nx = nx;
  a.ny = ny;
  // ends of each printed interval in either order
  a.xlo = xy_box[0] < xy_box[2] ? xy_box[0] : xy_box[2];
  a.xhi = xy_box[0] < xy_box[2] ? xy_box[2] : xy_box[0];
  a.ylo = xy_box[1] < xy_box[3] ? xy_box[1] : xy_box[3];
  a.yhi = xy_box[1] < xy_box[3] ? xy_box[3] : xy_box[1];
  if (!(a.xhi > a.xlo) || !(a.yhi > a.ylo)) return GS_ERR_INVALID_ARG;
  const int32_t B = nx * ny;
  hipStream_t s = (hipStream_t)stream;
  if (cells) {
    hipLaunchKernelGGL(part_cells_kernel, dim3((B + 255) / 256), dim3(256), 0, s, nx, ny, cells);
    GS_LAUNCH_CHECK();
  }
  if (n == 0) {
    hipLaunchKernelGGL(part_empty_kernel, dim3(1), dim3(256), 0, s, block_off, B);
    GS_LAUNCH_CHECK();
    return GS_OK;
  }
  if (ws_bytes < gs_partition_workspace_bytes(n)) return GS_ERR_WORKSPACE;
  PartWs w = part_ws_layout((char*)ws, n);
  a.zr = w.words;
  const int passes = B > kRadix ? 2 : 1;
  const int64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  hipLaunchKernelGGL(part_clear_kernel, dim3(grid_of(w.n_words, 2048)), dim3(256), 0, s, w.words, w.n_words,
                     w.counts, n);
  hipLaunchKernelGGL(zrange_kernel, dim3(grid_of(n, 1024)), dim3(256), 0, s, means + 2 * n, n, w.words);
  hipLaunchKernelGGL(part_ids_kernel, dim3(grid_of(n, 2048)), dim3(kThreads), 0, s, a, w.k0, w.v0, block_id, passes,
                     w.hist);
  GS_LAUNCH_CHECK();
  const unsigned rgrid = (unsigned)(ntiles < 1024 ? ntiles : 1024);
  const uint32_t* kin = w.k0;
  const uint32_t* vin = w.v0;
  for (int p = 0; p < passes; ++p) {
    const bool last = p == passes - 1;
    uint32_t* kout = (p % 2 == 0) ? w.k1 : w.k0;
    uint32_t* vout = last ? perm : ((p % 2 == 0) ? w.v1 : w.v0);
    hipLaunchKernelGGL((radix_pass_kernel<kPassPlain>), dim3(rgrid), dim3(kThreads), 0, s, kin, vin, kout, vout,
                       (const int64_t*)w.counts, GS_COUNT_RECORDS, n, 8 * p, w.hist + p * kRadix,
                       w.status + (int64_t)p * ntiles * kRadix, (int64_t)kRadix, w.words + 2 + p, w.counts,
                       PairPass{});
    GS_LAUNCH_CHECK();
    kin = kout;
    vin = vout;
  }
  hipLaunchKernelGGL(part_offsets_kernel, dim3(grid_of(n, 4096)), dim3(256), 0, s, kin, n, B, block_off);
  GS_LAUNCH_CHECK();
  return GS_OK;
}

extern "C" gs_status gs_gather_gaussians(const gs_gaussians* src, const uint32_t* perm, int64_t n,
                                         const gs_gaussian_grads* dst, void* stream) {
  using namespace gs;
  if (!src || !dst || n < 0 || (n > 0 && !perm)) return GS_ERR_INVALID_ARG;
  if (n == 0) return GS_OK;
  if (!src->means || !src->scales || !src->quats || !src->opac || !src->sh || !dst->means || !dst->scales ||
      !dst->quats || !dst->opac || !dst->sh)
    return GS_ERR_INVALID_ARG;
  if (src->attr_half != 0) return GS_ERR_UNSUPPORTED;
  if (src->sh_degree < 0 || src->sh_degree > 3) return GS_ERR_INVALID_ARG;
  const int planes = (src->sh_degree + 1) * (src->sh_degree + 1);
  hipStream_t s = (hipStream_t)stream;
  const unsigned g = grid_of(n, 8192);
  const int64_t ns = src->n;
  hipLaunchKernelGGL(gather_kernel, dim3(g), dim3(256), 0, s, src->means, dst->means, 3, ns, n, perm);
  hipLaunchKernelGGL(gather_kernel, dim3(g), dim3(256), 0, s, (const float*)src->scales, dst->scales, 3, ns, n, perm);
  hipLaunchKernelGGL(gather_kernel, dim3(g), dim3(256), 0, s, (const float*)src->quats, dst->quats, 4, ns, n, perm);
  hipLaunchKernelGGL(gather_kernel, dim3(g), dim3(256), 0, s, (const float*)src->opac, dst->opac, 1, ns, n, perm);
  hipLaunchKernelGGL(gather_kernel, dim3(g), dim3(256), 0, s, (const float*)src->sh, dst->sh, 3 * planes, ns, n,
                     perm);
  GS_LAUNCH_CHECK();
  return GS_OK;
}
