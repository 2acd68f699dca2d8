// FP64 projection of one Gaussian (the "proj" operator of Eq. 1, Sec. 3.1,
// following 3DGS), shared by the forward preprocess and its adjoint.  Every
// translation unit that includes this header is compiled with
// -ffp-contract=off: the operation order below is the reproducibility contract
// for culls, footprints and depth keys.
#pragma once

#include "gs_common.h"

namespace gs {

constexpr int kMaxLevels = 8;

struct LevelPtrs {
  const float* means;
  const void* scales;
  const void* quats;
  const void* opac;
  const void* sh;
  int64_t n;
  int sh_deg;  // SH bands stored
  bool half;   // attributes other than the centre are binary16
};

__host__ __forceinline__ LevelPtrs level_ptrs(const gs_gaussians& g) {
  return LevelPtrs{g.means, g.scales, g.quats, g.opac, g.sh, g.n, g.sh_degree, g.attr_half != 0};
}

// attribute i of an array stored as FP32 or binary16 (widening is exact); the
// storage is a template parameter so each record's code has no per-load branch
template <bool HALF>
__device__ __forceinline__ float attr(const void* p, int64_t i) {
  if constexpr (HALF) return (float)reinterpret_cast<const _Float16*>(p)[i];
  else return reinterpret_cast<const float*>(p)[i];
}

__device__ __forceinline__ double dmin_(double a, double b) { return b < a ? b : a; }
__device__ __forceinline__ double dmax_(double a, double b) { return a < b ? b : a; }

// index of the (view, block) segment holding record g: largest p with offsets[p] <= g
__device__ __forceinline__ int find_segment(const int64_t* __restrict__ offsets, int nseg, int64_t g) {
  int lo = 0, hi = nseg;  // invariant: offsets[lo] <= g < offsets[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offsets[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Normalisation constants of the real SH basis up to degree 3 (m = -l..l,
// Condon-Shortley phase kept), evaluated at a unit direction below.
constexpr double kSH00 = 0.28209479177387814;
constexpr double kSH1 = 0.4886025119029199;
constexpr double kSH2a = 1.0925484305920792;
constexpr double kSH2b = 0.31539156525252005;
constexpr double kSH2c = 0.5462742152960396;
constexpr double kSH3a = 0.5900435899266435;
constexpr double kSH3b = 2.890611442640554;
constexpr double kSH3c = 0.4570457994644658;
constexpr double kSH3d = 0.3731763325901154;
constexpr double kSH3e = 1.445305721320277;

// Colour sum_k Y_k f_k (per channel, k ascending) with the basis terms of
// sh_basis computed one at a time, so no basis array is live.
template <bool HALF>
__device__ __forceinline__ void sh_colour(double x, double y, double z, int deg, const void* __restrict__ sh,
                                          int64_t n, int64_t gi, double col[3]) {
  auto term = [&](int k, double Yk) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) col[ch] += Yk * (double)attr<HALF>(sh, (int64_t)(3 * k + ch) * n + gi);
  };
  term(0, kSH00);
  if (deg < 1) return;
  term(1, -kSH1 * y);
  term(2, kSH1 * z);
  term(3, -kSH1 * x);
  if (deg < 2) return;
  const double xx = x * x, yy = y * y, zz = z * z;
  term(4, kSH2a * (x * y));
  term(5, -kSH2a * (y * z));
  term(6, kSH2b * (2.0 * zz - xx - yy));
  term(7, -kSH2a * (x * z));
  term(8, kSH2c * (xx - yy));
  if (deg < 3) return;
  term(9, -kSH3a * (y * (3.0 * xx - yy)));
  term(10, kSH3b * (x * y * z));
  term(11, -kSH3c * (y * (4.0 * zz - xx - yy)));
  term(12, kSH3d * (z * (2.0 * zz - 3.0 * xx - 3.0 * yy)));
  term(13, -kSH3c * (x * (4.0 * zz - xx - yy)));
  term(14, kSH3e * (z * (xx - yy)));
  term(15, -kSH3a * (x * (xx - 3.0 * yy)));
}

// Everything the forward projection computes for one Gaussian.
struct Geo {
  double m[3];         // centre
  double tx, ty, tz;   // camera-space centre
  double rz, ux, uy;   // 1/tz, tx/tz, ty/tz
  bool clamp_x, clamp_y;
  double uxc, uyc;     // guard-band clamped tan values
  double q[4];         // normalised quaternion (w, x, y, z)
  double qinv;         // 1 / |q|
  double s[3];
  double Rq[3][3];
  double Lm[3][3];     // Rq diag(s)
  double WL[3][3];     // R_cam Lm
  double J00, J02, J11, J12;
  double M[2][3];      // J WL
  double n0, n1, a, b, c, det;
  double u, v;
  float depth;
  int i0, i1, j0, j1;
  double opac;
};

// Decides culling and the footprint; returns false if culled.  Two rounds of
// loads: centre, scale and opacity first (28 B), which decide most culls — the
// near plane, the opacity threshold, and a footprint that certainly misses the
// image (below) — and the rotation (16 B) only for the Gaussians left; the SH
// coefficients are read later, by the caller, only for survivors.
//
// Early footprint test: the projected covariance is J W Rq diag(s)^2 Rq^T W^T J^T
// with W and Rq rotations, so its trace is at most |J|_F^2 s_max^2, and the
// larger eigenvalue of the dilated matrix is below that trace + 0.6.  With |J|_F^2
// bounded through the guard-band limits of x/z and y/z, 3 sqrt(bound) + 2 px is
// more than the radius ceil(3 sqrt(lmax)) computed below (the relative slack of
// 1e-6 covers the rounding of both sides), and u, v are computed by the same
// operations as below, so a centre farther than that outside the image is one
// the exact test would cull too.  Non-finite values fail every comparison and
// take the exact path.
template <bool HALF>
__device__ __forceinline__ bool project_geo(const LevelPtrs& L, int64_t gi, const gs_camera& cam, int W, int H,
                                            Geo& o) {
  const int64_t n = L.n;
  const double* R = cam.R;
  o.m[0] = L.means[gi];
  o.m[1] = L.means[n + gi];
  o.m[2] = L.means[2 * n + gi];
  const float op32 = attr<HALF>(L.opac, gi);
  const float s0f = attr<HALF>(L.scales, gi), s1f = attr<HALF>(L.scales, n + gi),
              s2f = attr<HALF>(L.scales, 2 * n + gi);
  o.tx = ((R[0] * o.m[0] + R[1] * o.m[1]) + R[2] * o.m[2]) + cam.t[0];
  o.ty = ((R[3] * o.m[0] + R[4] * o.m[1]) + R[5] * o.m[2]) + cam.t[1];
  o.tz = ((R[6] * o.m[0] + R[7] * o.m[1]) + R[8] * o.m[2]) + cam.t[2];
  if (!(o.tz > cam.znear)) return false;
  o.opac = op32;
  if (!(o.opac >= 1.0 / 255.0)) return false;
  o.depth = (float)o.tz;
  o.rz = 1.0 / o.tz;
  o.ux = o.tx * o.rz;
  o.uy = o.ty * o.rz;
  o.u = cam.fx * o.ux + cam.cx;
  o.v = cam.fy * o.uy + cam.cy;
  const double tanx = (0.5 * W) / cam.fx, tany = (0.5 * H) / cam.fy;
  const double limx = 1.3 * tanx, limy = 1.3 * tany;
  {
    const double smax = dmax_(fabs((double)s0f), dmax_(fabs((double)s1f), fabs((double)s2f)));
    const double jx = cam.fx * o.rz, jy = cam.fy * o.rz;
    const double jf2 = jx * jx * (1.0 + limx * limx) + jy * jy * (1.0 + limy * limy);
    const double rb = 3.0 * sqrt((jf2 * (smax * smax) + 0.6) * (1.0 + 1e-6)) + 2.0;
    if ((o.u + rb) - 0.5 < 0.0 || (o.u - rb) - 0.5 > (double)(W - 1) || (o.v + rb) - 0.5 < 0.0 ||
        (o.v - rb) - 0.5 > (double)(H - 1))
      return false;
  }
  const float q0f = attr<HALF>(L.quats, gi), q1f = attr<HALF>(L.quats, n + gi), q2f = attr<HALF>(L.quats, 2 * n + gi),
              q3f = attr<HALF>(L.quats, 3 * n + gi);
  const double q0 = q0f, q1 = q1f, q2 = q2f, q3 = q3f;
  const double qn2 = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
  if (!(qn2 > 0.0 && qn2 <= 1.0e300)) return false;
  o.qinv = 1.0 / sqrt(qn2);
  const double w = q0 * o.qinv, x = q1 * o.qinv, y = q2 * o.qinv, z = q3 * o.qinv;
  o.q[0] = w; o.q[1] = x; o.q[2] = y; o.q[3] = z;
  o.Rq[0][0] = 1.0 - 2.0 * (y * y + z * z);
  o.Rq[0][1] = 2.0 * (x * y - w * z);
  o.Rq[0][2] = 2.0 * (x * z + w * y);
  o.Rq[1][0] = 2.0 * (x * y + w * z);
  o.Rq[1][1] = 1.0 - 2.0 * (x * x + z * z);
  o.Rq[1][2] = 2.0 * (y * z - w * x);
  o.Rq[2][0] = 2.0 * (x * z - w * y);
  o.Rq[2][1] = 2.0 * (y * z + w * x);
  o.Rq[2][2] = 1.0 - 2.0 * (x * x + y * y);
  o.s[0] = s0f;
  o.s[1] = s1f;
  o.s[2] = s2f;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) o.Lm[i][j] = o.Rq[i][j] * o.s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      o.WL[i][j] = (R[3 * i + 0] * o.Lm[0][j] + R[3 * i + 1] * o.Lm[1][j]) + R[3 * i + 2] * o.Lm[2][j];
  o.uxc = dmin_(limx, dmax_(-limx, o.ux));
  o.uyc = dmin_(limy, dmax_(-limy, o.uy));
  o.clamp_x = o.uxc != o.ux;
  o.clamp_y = o.uyc != o.uy;
  o.J00 = cam.fx * o.rz;
  o.J02 = -(cam.fx * o.uxc) * o.rz;
  o.J11 = cam.fy * o.rz;
  o.J12 = -(cam.fy * o.uyc) * o.rz;
  for (int j = 0; j < 3; ++j) {
    o.M[0][j] = o.J00 * o.WL[0][j] + o.J02 * o.WL[2][j];
    o.M[1][j] = o.J11 * o.WL[1][j] + o.J12 * o.WL[2][j];
  }
  o.n0 = (o.M[0][0] * o.M[0][0] + o.M[0][1] * o.M[0][1]) + o.M[0][2] * o.M[0][2];
  o.n1 = (o.M[1][0] * o.M[1][0] + o.M[1][1] * o.M[1][1]) + o.M[1][2] * o.M[1][2];
  o.b = (o.M[0][0] * o.M[1][0] + o.M[0][1] * o.M[1][1]) + o.M[0][2] * o.M[1][2];
  o.a = o.n0 + 0.3;
  o.c = o.n1 + 0.3;
  const double cr0 = o.M[0][1] * o.M[1][2] - o.M[0][2] * o.M[1][1];
  const double cr1 = o.M[0][2] * o.M[1][0] - o.M[0][0] * o.M[1][2];
  const double cr2 = o.M[0][0] * o.M[1][1] - o.M[0][1] * o.M[1][0];
  o.det = (((cr0 * cr0 + cr1 * cr1) + cr2 * cr2) + 0.3 * (o.n0 + o.n1)) + 0.09;
  if (!(o.det > 0.0 && o.det <= 1.0e300)) return false;
  const double hd = 0.5 * (o.a - o.c);
  const double lmax = 0.5 * (o.a + o.c) + sqrt(hd * hd + o.b * o.b);
  if (!(lmax <= 1.0e300)) return false;
  const double r = ceil(3.0 * sqrt(lmax));
  const double i0 = dmax_(0.0, ceil((o.u - r) - 0.5));
  const double i1 = dmin_((double)(W - 1), floor((o.u + r) - 0.5));
  const double j0 = dmax_(0.0, ceil((o.v - r) - 0.5));
  const double j1 = dmin_((double)(H - 1), floor((o.v + r) - 0.5));
  if (!(i0 <= i1) || !(j0 <= j1)) return false;
  o.i0 = (int)i0;
  o.i1 = (int)i1;
  o.j0 = (int)j0;
  o.j1 = (int)j1;
  return true;
}

// Camera centre C = -R^T t.
__device__ __forceinline__ void camera_centre(const gs_camera& cam, double C[3]) {
  const double* R = cam.R;
  C[0] = -((R[0] * cam.t[0] + R[3] * cam.t[1]) + R[6] * cam.t[2]);
  C[1] = -((R[1] * cam.t[0] + R[4] * cam.t[1]) + R[7] * cam.t[2]);
  C[2] = -((R[2] * cam.t[0] + R[5] * cam.t[1]) + R[8] * cam.t[2]);
}

// sqrt(log2(e) / 2): the conic factor is scaled so the Gaussian is exp2(-Q).
constexpr double kConicScale = 0.84932180028801907;
constexpr double kConicScale2 = 0.72134752044448170;  // log2(e) / 2

}  // namespace gs
