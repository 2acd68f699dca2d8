// CPU oracle for the Gaussian splatting rasterizer: TEST INFRASTRUCTURE ONLY.
//
// Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
// load this library.  It shares no code with the GPU path.
//
// A plain FP64 implementation of what the rendering path computes:
//   * projection of each 3D Gaussian to a 2D Gaussian (the paper's "proj" in
//     Eq. 1, Sec. 3.1, which defers to the 3DGS paper: EWA splatting with the
//     local affine approximation of the perspective map, a 0.3 px^2 low-pass
//     dilation, and a 3-sigma screen footprint),
//   * view-dependent colour from degree-3 real spherical harmonics (Sec. 3.1),
//   * per-pixel front-to-back alpha compositing of Eq. 1 over the Gaussians
//     whose footprint holds the pixel, sorted by (f32 depth bits, index).
//     No tiles are used, except in the separate tiled mode that exists only to
//     show that tiling does not change the result,
//   * the exact FP64 gradient of that image with respect to every Gaussian
//     parameter, decisions (culls, footprints, order, skips, early stop and
//     clamps) held fixed.  The per-pixel part is a hand-written adjoint; the
//     per-Gaussian part uses forward-mode dual numbers, so it is the exact
//     derivative of the projection code below.
//
// Integer-valued results (culls, footprints, depth bits, tile lists) come out of
// FP64 arithmetic done in a fixed operation order: no fused multiply-add (this
// file is compiled with -ffp-contract=off), correctly rounded division and
// square root.  Build: g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -shared -fPIC.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

struct Cam {
  double R[9];
  double t[3];
  double fx, fy, cx, cy, znear;
  int32_t width, height;
};

// ---------------------------------------------------------------------------
// forward-mode dual number: value + one derivative direction
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual(double v_ = 0.0, double d_ = 0.0) : v(v_), d(d_) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual dsqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
inline double dsqrt(double a) { return std::sqrt(a); }
inline double val(double a) { return a; }
inline double val(const Dual& a) { return a.v; }

// ---------------------------------------------------------------------------
// real spherical harmonics up to degree 3, m = -l..l ordering, Condon-Shortley
// phase kept (Y_{l,m>0} = sqrt2 Re Y_l^m, Y_{l,m<0} = sqrt2 Im Y_l^|m| of the
// complex harmonics); valid on the unit sphere.
// ---------------------------------------------------------------------------
template <class S>
void sh_basis(const S& x, const S& y, const S& z, int deg, S* Y) {
  const double k00 = 0.28209479177387814;  // 1 / (2 sqrt(pi))
  const double k1 = 0.4886025119029199;    // sqrt(3 / (4 pi))
  const double k2a = 1.0925484305920792;   // sqrt(15 / pi) / 2
  const double k2b = 0.31539156525252005;  // sqrt(5 / pi) / 4
  const double k2c = 0.5462742152960396;   // sqrt(15 / pi) / 4
  const double k3a = 0.5900435899266435;   // sqrt(70 / pi) / 8
  const double k3b = 2.890611442640554;    // sqrt(105 / pi) / 2
  const double k3c = 0.4570457994644658;   // sqrt(42 / pi) / 8
  const double k3d = 0.3731763325901154;   // sqrt(7 / pi) / 4
  const double k3e = 1.445305721320277;    // sqrt(105 / pi) / 4
  Y[0] = S(k00);
  if (deg < 1) return;
  Y[1] = S(-k1) * y;
  Y[2] = S(k1) * z;
  Y[3] = S(-k1) * x;
  if (deg < 2) return;
  S xx = x * x, yy = y * y, zz = z * z;
  Y[4] = S(k2a) * (x * y);
  Y[5] = S(-k2a) * (y * z);
  Y[6] = S(k2b) * (S(2.0) * zz - xx - yy);
  Y[7] = S(-k2a) * (x * z);
  Y[8] = S(k2c) * (xx - yy);
  if (deg < 3) return;
  Y[9] = S(-k3a) * (y * (S(3.0) * xx - yy));
  Y[10] = S(k3b) * (x * y * z);
  Y[11] = S(-k3c) * (y * (S(4.0) * zz - xx - yy));
  Y[12] = S(k3d) * (z * (S(2.0) * zz - S(3.0) * xx - S(3.0) * yy));
  Y[13] = S(-k3c) * (x * (S(4.0) * zz - xx - yy));
  Y[14] = S(k3e) * (z * (xx - yy));
  Y[15] = S(-k3a) * (x * (xx - S(3.0) * yy));
}

// Decisions taken by the FP64 value pass; the dual pass re-uses them so both
// follow the same branch of every clamp.
struct Decisions {
  bool visible = false;
  bool clamp_x = false, clamp_y = false;  // guard-band clamp active
  double cx_val = 0, cy_val = 0;          // clamped tan values when active
  bool rgb_clamped[3] = {false, false, false};
  int32_t i0 = 0, i1 = -1, j0 = 0, j1 = -1;
  float depth = 0.f;
  double radius = 0;
};

template <class S>
struct Proj {
  S u, v;          // 2D mean, pixels
  S a, b, c;       // dilated 2D covariance
  S A, B, C;       // conic = inverse of (a b; b c)
  S rgb[3];
  S det;
};

// Project one Gaussian.  For S = double this decides culling, footprint and
// clamps (written into `dec`); for S = Dual it reuses `dec`.
template <class S>
bool project_one(const S m[3], const S s[3], const S q[4], const S* sh /*[16][3]*/, int deg,
                 double opac, const Cam& cam, Decisions& dec, Proj<S>& P, bool decide) {
  const double* R = cam.R;
  // view transform (world -> camera)
  S tx = ((S(R[0]) * m[0] + S(R[1]) * m[1]) + S(R[2]) * m[2]) + S(cam.t[0]);
  S ty = ((S(R[3]) * m[0] + S(R[4]) * m[1]) + S(R[5]) * m[2]) + S(cam.t[1]);
  S tz = ((S(R[6]) * m[0] + S(R[7]) * m[1]) + S(R[8]) * m[2]) + S(cam.t[2]);
  if (decide) {
    dec.visible = false;
    if (!(val(tz) > cam.znear)) return false;
    if (!(opac >= 1.0 / 255.0)) return false;
    dec.depth = (float)val(tz);
  }
  // rotation from the normalised quaternion (w, x, y, z), Hamilton convention
  S qn2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
  if (decide && !(val(qn2) > 0.0 && val(qn2) <= 1.0e300)) return false;
  S inv = S(1.0) / dsqrt(qn2);
  S w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
  S Rq[3][3];
  Rq[0][0] = S(1.0) - S(2.0) * (y * y + z * z);
  Rq[0][1] = S(2.0) * (x * y - w * z);
  Rq[0][2] = S(2.0) * (x * z + w * y);
  Rq[1][0] = S(2.0) * (x * y + w * z);
  Rq[1][1] = S(1.0) - S(2.0) * (x * x + z * z);
  Rq[1][2] = S(2.0) * (y * z - w * x);
  Rq[2][0] = S(2.0) * (x * z - w * y);
  Rq[2][1] = S(2.0) * (y * z + w * x);
  Rq[2][2] = S(1.0) - S(2.0) * (x * x + y * y);
  // covariance factor L = Rq diag(s), so Sigma = L L^T; then W L in camera axes
  S Lm[3][3], WL[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Lm[i][j] = Rq[i][j] * s[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      WL[i][j] = (S(R[3 * i + 0]) * Lm[0][j] + S(R[3 * i + 1]) * Lm[1][j]) + S(R[3 * i + 2]) * Lm[2][j];
  // Jacobian of the pinhole map at t, with the 1.3x guard band on x/z and y/z
  S rz = S(1.0) / tz;
  S ux = tx * rz, uy = ty * rz;
  double tanx = (0.5 * cam.width) / cam.fx, tany = (0.5 * cam.height) / cam.fy;
  double limx = 1.3 * tanx, limy = 1.3 * tany;
  S uxc = ux, uyc = uy;
  if (decide) {
    double cxv = std::min(limx, std::max(-limx, val(ux)));
    double cyv = std::min(limy, std::max(-limy, val(uy)));
    dec.clamp_x = (cxv != val(ux));
    dec.clamp_y = (cyv != val(uy));
    dec.cx_val = cxv;
    dec.cy_val = cyv;
  }
  if (dec.clamp_x) uxc = S(dec.cx_val);
  if (dec.clamp_y) uyc = S(dec.cy_val);
  S J00 = S(cam.fx) * rz;
  S J02 = -(S(cam.fx) * uxc) * rz;
  S J11 = S(cam.fy) * rz;
  S J12 = -(S(cam.fy) * uyc) * rz;
  S M[2][3];
  for (int j = 0; j < 3; ++j) {
    M[0][j] = J00 * WL[0][j] + J02 * WL[2][j];
    M[1][j] = J11 * WL[1][j] + J12 * WL[2][j];
  }
  // 2D covariance M M^T + 0.3 I; determinant by the Lagrange identity
  S n0 = (M[0][0] * M[0][0] + M[0][1] * M[0][1]) + M[0][2] * M[0][2];
  S n1 = (M[1][0] * M[1][0] + M[1][1] * M[1][1]) + M[1][2] * M[1][2];
  S b = (M[0][0] * M[1][0] + M[0][1] * M[1][1]) + M[0][2] * M[1][2];
  S a = n0 + S(0.3), c = n1 + S(0.3);
  S cr0 = M[0][1] * M[1][2] - M[0][2] * M[1][1];
  S cr1 = M[0][2] * M[1][0] - M[0][0] * M[1][2];
  S cr2 = M[0][0] * M[1][1] - M[0][1] * M[1][0];
  S det = (((cr0 * cr0 + cr1 * cr1) + cr2 * cr2) + S(0.3) * (n0 + n1)) + S(0.09);
  S u = S(cam.fx) * ux + S(cam.cx);
  S v = S(cam.fy) * uy + S(cam.cy);
  if (decide) {
    double dv = val(det);
    if (!(dv > 0.0 && dv <= 1.0e300)) return false;
    double hd = 0.5 * (val(a) - val(c));
    double lmax = 0.5 * (val(a) + val(c)) + std::sqrt(hd * hd + val(b) * val(b));
    if (!(lmax <= 1.0e300)) return false;
    double r = std::ceil(3.0 * std::sqrt(lmax));
    double uu = val(u), vv = val(v);
    double i0 = std::max(0.0, std::ceil((uu - r) - 0.5));
    double i1 = std::min((double)(cam.width - 1), std::floor((uu + r) - 0.5));
    double j0 = std::max(0.0, std::ceil((vv - r) - 0.5));
    double j1 = std::min((double)(cam.height - 1), std::floor((vv + r) - 0.5));
    if (!(i0 <= i1) || !(j0 <= j1)) return false;
    dec.i0 = (int32_t)i0;
    dec.i1 = (int32_t)i1;
    dec.j0 = (int32_t)j0;
    dec.j1 = (int32_t)j1;
    dec.radius = r;
  }
  P.u = u;
  P.v = v;
  P.a = a;
  P.b = b;
  P.c = c;
  P.det = det;
  P.A = c / det;
  P.B = -b / det;
  P.C = a / det;
  // colour: direction from the camera centre C = -R^T t to the mean
  double Cw[3];
  for (int k = 0; k < 3; ++k)
    Cw[k] = -((R[k] * cam.t[0] + R[3 + k] * cam.t[1]) + R[6 + k] * cam.t[2]);
  S d0 = m[0] - S(Cw[0]), d1 = m[1] - S(Cw[1]), d2 = m[2] - S(Cw[2]);
  S dn = dsqrt((d0 * d0 + d1 * d1) + d2 * d2);
  S dx = d0 / dn, dy = d1 / dn, dz = d2 / dn;
  S Y[16];
  sh_basis(dx, dy, dz, deg, Y);
  int nk = (deg + 1) * (deg + 1);
  for (int ch = 0; ch < 3; ++ch) {
    S acc = S(0.0);
    for (int k = 0; k < nk; ++k) acc = acc + Y[k] * sh[k * 3 + ch];
    acc = acc + S(0.5);
    if (decide) dec.rgb_clamped[ch] = !(val(acc) >= 0.0);
    P.rgb[ch] = dec.rgb_clamped[ch] ? S(0.0) : acc;
  }
  if (decide) dec.visible = true;
  return true;
}

struct Inputs {
  int64_t n;
  const double *means, *scales, *quats, *opac, *sh;
  int deg;
};

// Gather one Gaussian's parameters (the caller promotes FP32 inputs to FP64 exactly).
inline void load_params(const Inputs& in, int64_t g, double m[3], double s[3], double q[4], double sh[48]) {
  for (int k = 0; k < 3; ++k) {
    m[k] = in.means[k * in.n + g];
    s[k] = in.scales[k * in.n + g];
  }
  for (int k = 0; k < 4; ++k) q[k] = in.quats[k * in.n + g];
  for (int k = 0; k < 16; ++k)
    for (int ch = 0; ch < 3; ++ch) sh[k * 3 + ch] = in.sh[(k * 3 + ch) * in.n + g];
}

struct Splat {
  int32_t i0, i1, j0, j1;
  uint32_t depth_bits;
  int64_t index;
  double u, v, A, B, C, o, rgb[3];
};

inline uint32_t float_bits(float f) {
  uint32_t b;
  std::memcpy(&b, &f, 4);
  return b;
}

void project_all(const Inputs& in, const Cam& cam, std::vector<Splat>& out, std::vector<Decisions>* decs) {
  std::vector<Splat> tmp(in.n);
  std::vector<char> vis(in.n, 0);
  if (decs) decs->assign(in.n, Decisions());
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < in.n; ++g) {
    double m[3], s[3], q[4], sh[48];
    load_params(in, g, m, s, q, sh);
    Decisions dec;
    Proj<double> P;
    double o = in.opac[g];
    if (project_one<double>(m, s, q, sh, in.deg, o, cam, dec, P, true)) {
      Splat& sp = tmp[g];
      sp.i0 = dec.i0; sp.i1 = dec.i1; sp.j0 = dec.j0; sp.j1 = dec.j1;
      sp.depth_bits = float_bits(dec.depth);
      sp.index = g;
      sp.u = P.u; sp.v = P.v; sp.A = P.A; sp.B = P.B; sp.C = P.C; sp.o = o;
      for (int ch = 0; ch < 3; ++ch) sp.rgb[ch] = P.rgb[ch];
      vis[g] = 1;
    }
    if (decs) (*decs)[g] = dec;
  }
  out.clear();
  for (int64_t g = 0; g < in.n; ++g)
    if (vis[g]) out.push_back(tmp[g]);
}

inline bool splat_less(const Splat* a, const Splat* b) {
  if (a->depth_bits != b->depth_bits) return a->depth_bits < b->depth_bits;
  return a->index < b->index;
}

// Blending thresholds of the 3DGS compositing rule.
const double kAlphaMin = 1.0 / 255.0;
const double kAlphaMax = 0.99;
const double kTMin = 1.0e-4;
// Relative width of the bands around each threshold inside which FP32 and FP64
// may legitimately decide differently.
const double kBand = 1.0e-5;

struct PixelResult {
  double C[3];
  double T;
  int32_t n_contrib;
  // decisions of the image that fall inside a band: the skip of alpha below
  // 1/255 and the stop before T drops below 1e-4 (either choice is a correct
  // result of the method at that precision)
  int32_t ambiguous;
  // entries whose raw alpha o * G lies inside the band around the 0.99 clamp:
  // the image is continuous there, its gradient with respect to o and the
  // footprint is not
  int32_t grad_ambiguous;
};

// Composite one pixel over a depth-sorted candidate list (entries whose
// footprint does not hold the pixel are skipped).  flip >= 0 takes the other
// branch at the flip-th ambiguous decision (0 = the first), which gives the
// second correct result of a pixel with one such decision.
PixelResult composite(const std::vector<const Splat*>& list, int i, int j, const double bg[3],
                      std::vector<const Splat*>* contrib, std::vector<double>* alphas, std::vector<double>* Ts,
                      int flip = -1, std::vector<const Splat*>* near = nullptr, double near_band = 0.0) {
  PixelResult r;
  r.C[0] = r.C[1] = r.C[2] = 0.0;
  r.T = 1.0;
  r.n_contrib = 0;
  r.ambiguous = 0;
  r.grad_ambiguous = 0;
  double px = i + 0.5, py = j + 0.5;
  for (const Splat* s : list) {
    if (i < s->i0 || i > s->i1 || j < s->j0 || j > s->j1) continue;
    double dx = px - s->u, dy = py - s->v;
    double power = -0.5 * (s->A * dx * dx + s->C * dy * dy) - s->B * dx * dy;
    double raw = s->o * std::exp(power);
    double alpha = std::min(kAlphaMax, raw);
    if (near && std::fabs(alpha - kAlphaMin) <= near_band * kAlphaMin) near->push_back(s);
    bool skip = alpha < kAlphaMin;
    if (std::fabs(alpha - kAlphaMin) <= kBand * kAlphaMin) {
      if (r.ambiguous == flip) skip = !skip;
      r.ambiguous++;
    }
    if (skip) continue;
    double Tn = r.T * (1.0 - alpha);
    if (near && std::fabs(Tn - kTMin) <= near_band * kTMin) near->push_back(s);
    bool stop = Tn < kTMin;
    if (std::fabs(Tn - kTMin) <= kBand * kTMin) {
      if (r.ambiguous == flip) stop = !stop;
      r.ambiguous++;
    }
    if (stop) break;
    if (std::fabs(raw - kAlphaMax) <= kBand * kAlphaMax) r.grad_ambiguous++;
    if (near && std::fabs(raw - kAlphaMax) <= near_band * kAlphaMax) near->push_back(s);
    if (contrib) {
      contrib->push_back(s);
      alphas->push_back(alpha);
      Ts->push_back(r.T);
    }
    for (int ch = 0; ch < 3; ++ch) r.C[ch] += s->rgb[ch] * alpha * r.T;
    r.T = Tn;
    r.n_contrib++;
  }
  for (int ch = 0; ch < 3; ++ch) r.C[ch] += r.T * bg[ch];
  return r;
}

// Per-row candidate lists: every splat whose footprint spans row j, sorted by
// (depth bits, index).  A pixel's list is the row list filtered by column.
void row_lists(const std::vector<Splat>& splats, int H, std::vector<std::vector<const Splat*>>& rows,
               const std::vector<char>* need) {
  rows.assign(H, {});
  for (const Splat& s : splats)
    for (int j = s.j0; j <= s.j1; ++j)
      if (!need || (*need)[j]) rows[j].push_back(&s);
#pragma omp parallel for schedule(dynamic)
  for (int j = 0; j < H; ++j) std::sort(rows[j].begin(), rows[j].end(), splat_less);
}

Cam to_cam(const double* cam_d, const int32_t* cam_i) {
  Cam c;
  for (int k = 0; k < 9; ++k) c.R[k] = cam_d[k];
  for (int k = 0; k < 3; ++k) c.t[k] = cam_d[9 + k];
  c.fx = cam_d[12];
  c.fy = cam_d[13];
  c.cx = cam_d[14];
  c.cy = cam_d[15];
  c.znear = cam_d[16];
  c.width = cam_i[0];
  c.height = cam_i[1];
  return c;
}

}  // namespace

extern "C" {

// Camera encoding: cam_d = R[9] (row-major world->camera), t[3], fx, fy, cx, cy,
// znear (17 doubles); cam_i = width, height.

// Per-Gaussian projection.  Every output pointer may be NULL.
int orc_project(int64_t n, const double* means, const double* scales, const double* quats, const double* opac,
                const double* sh, int deg, const double* cam_d, const int32_t* cam_i, int tile_w, int tile_h,
                int32_t* visible, uint32_t* depth_bits, int32_t* rect, int32_t* tiles_touched, double* uv,
                double* cov2d, double* conic, double* rgb, int32_t* rgb_clamped, double* radius) {
  Cam cam = to_cam(cam_d, cam_i);
  Inputs in{n, means, scales, quats, opac, sh, deg};
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < n; ++g) {
    double m[3], s[3], q[4], shv[48];
    load_params(in, g, m, s, q, shv);
    Decisions dec;
    Proj<double> P;
    bool vis = project_one<double>(m, s, q, shv, deg, opac[g], cam, dec, P, true);
    if (visible) visible[g] = vis ? 1 : 0;
    if (depth_bits) depth_bits[g] = vis ? float_bits(dec.depth) : 0xFFFFFFFFu;
    if (rect) {
      rect[4 * g + 0] = vis ? dec.i0 : 0;
      rect[4 * g + 1] = vis ? dec.i1 : -1;
      rect[4 * g + 2] = vis ? dec.j0 : 0;
      rect[4 * g + 3] = vis ? dec.j1 : -1;
    }
    if (tiles_touched) {
      int32_t tt = 0;
      if (vis) tt = (dec.i1 / tile_w - dec.i0 / tile_w + 1) * (dec.j1 / tile_h - dec.j0 / tile_h + 1);
      tiles_touched[g] = tt;
    }
    if (uv) { uv[2 * g] = vis ? P.u : 0; uv[2 * g + 1] = vis ? P.v : 0; }
    if (cov2d) { cov2d[3 * g] = vis ? P.a : 0; cov2d[3 * g + 1] = vis ? P.b : 0; cov2d[3 * g + 2] = vis ? P.c : 0; }
    if (conic) { conic[3 * g] = vis ? P.A : 0; conic[3 * g + 1] = vis ? P.B : 0; conic[3 * g + 2] = vis ? P.C : 0; }
    if (rgb) for (int ch = 0; ch < 3; ++ch) rgb[3 * g + ch] = vis ? P.rgb[ch] : 0;
    if (rgb_clamped) for (int ch = 0; ch < 3; ++ch) rgb_clamped[3 * g + ch] = vis ? dec.rgb_clamped[ch] : 0;
    if (radius) radius[g] = vis ? dec.radius : 0;
  }
  return 0;
}

// Untiled render.  If pix != NULL only the listed pixels (index j*W + i) are
// rendered and outputs are [3][npix], [npix]; otherwise the whole image.
// ambiguous = number of image decisions inside a threshold band; img_alt and
// T_alt (may be NULL) hold the result with the other branch taken at a pixel's
// only ambiguous decision; grad_ambiguous counts entries whose raw alpha lies
// inside the band of the 0.99 clamp.
int orc_render(int64_t n, const double* means, const double* scales, const double* quats, const double* opac,
               const double* sh, int deg, const double* cam_d, const int32_t* cam_i, const double* bg,
               const int64_t* pix, int64_t npix, double* img, double* T_final, int32_t* n_contrib,
               int32_t* ambiguous, double* img_alt, double* T_alt, int32_t* grad_ambiguous) {
  Cam cam = to_cam(cam_d, cam_i);
  Inputs in{n, means, scales, quats, opac, sh, deg};
  std::vector<Splat> splats;
  project_all(in, cam, splats, nullptr);
  const int W = cam.width, H = cam.height;
  int64_t P = pix ? npix : (int64_t)W * H;
  std::vector<char> need;
  if (pix) {
    need.assign(H, 0);
    for (int64_t k = 0; k < npix; ++k) need[pix[k] / W] = 1;
  }
  std::vector<std::vector<const Splat*>> rows;
  row_lists(splats, H, rows, pix ? &need : nullptr);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t k = 0; k < P; ++k) {
    int64_t p = pix ? pix[k] : k;
    int i = (int)(p % W), j = (int)(p / W);
    PixelResult r = composite(rows[j], i, j, bg, nullptr, nullptr, nullptr);
    for (int ch = 0; ch < 3; ++ch) img[ch * P + k] = r.C[ch];
    if (T_final) T_final[k] = r.T;
    if (n_contrib) n_contrib[k] = r.n_contrib;
    if (ambiguous) ambiguous[k] = r.ambiguous;
    if (grad_ambiguous) grad_ambiguous[k] = r.grad_ambiguous;
    if (img_alt || T_alt) {
      // second correct result of a pixel with exactly one ambiguous decision;
      // elsewhere the alternative equals the primary result
      PixelResult a = r.ambiguous == 1 ? composite(rows[j], i, j, bg, nullptr, nullptr, nullptr, 0) : r;
      if (img_alt)
        for (int ch = 0; ch < 3; ++ch) img_alt[ch * P + k] = a.C[ch];
      if (T_alt) T_alt[k] = a.T;
    }
  }
  return 0;
}

// Tiled render of the whole image: each tile composites the splats whose tile
// rectangle covers it.  Exists only to show tiling does not change the image.
int orc_render_tiled(int64_t n, const double* means, const double* scales, const double* quats, const double* opac,
                     const double* sh, int deg, const double* cam_d, const int32_t* cam_i, const double* bg,
                     int tile_w, int tile_h, double* img, double* T_final, int32_t* n_contrib) {
  Cam cam = to_cam(cam_d, cam_i);
  Inputs in{n, means, scales, quats, opac, sh, deg};
  std::vector<Splat> splats;
  project_all(in, cam, splats, nullptr);
  const int W = cam.width, H = cam.height;
  const int tx_n = (W + tile_w - 1) / tile_w, ty_n = (H + tile_h - 1) / tile_h;
  const int64_t P = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic)
  for (int t = 0; t < tx_n * ty_n; ++t) {
    int tx = t % tx_n, ty = t / tx_n;
    std::vector<const Splat*> list;
    for (const Splat& s : splats)
      if (s.i0 / tile_w <= tx && tx <= s.i1 / tile_w && s.j0 / tile_h <= ty && ty <= s.j1 / tile_h)
        list.push_back(&s);
    std::sort(list.begin(), list.end(), splat_less);
    for (int j = ty * tile_h; j < std::min(H, (ty + 1) * tile_h); ++j)
      for (int i = tx * tile_w; i < std::min(W, (tx + 1) * tile_w); ++i) {
        PixelResult r = composite(list, i, j, bg, nullptr, nullptr, nullptr);
        int64_t p = (int64_t)j * W + i;
        for (int ch = 0; ch < 3; ++ch) img[ch * P + p] = r.C[ch];
        if (T_final) T_final[p] = r.T;
        if (n_contrib) n_contrib[p] = r.n_contrib;
      }
  }
  return 0;
}

// (tile, Gaussian) pairs sorted by (tile, depth bits, index); tile ids are
// row-major over the tile grid.  Returns the pair count (also when it exceeds
// cap, in which case nothing beyond cap is written).
int64_t orc_pairs(int64_t n, const double* means, const double* scales, const double* quats, const double* opac,
                  const double* sh, int deg, const double* cam_d, const int32_t* cam_i, int tile_w, int tile_h,
                  int64_t cap, uint32_t* tile_out, uint32_t* index_out) {
  Cam cam = to_cam(cam_d, cam_i);
  Inputs in{n, means, scales, quats, opac, sh, deg};
  std::vector<Splat> splats;
  project_all(in, cam, splats, nullptr);
  const int tx_n = (cam.width + tile_w - 1) / tile_w;
  struct Pair { uint32_t tile, depth; int64_t index; };
  std::vector<Pair> pairs;
  for (const Splat& s : splats)
    for (int ty = s.j0 / tile_h; ty <= s.j1 / tile_h; ++ty)
      for (int tx = s.i0 / tile_w; tx <= s.i1 / tile_w; ++tx)
        pairs.push_back({(uint32_t)(ty * tx_n + tx), s.depth_bits, s.index});
  std::sort(pairs.begin(), pairs.end(), [](const Pair& a, const Pair& b) {
    if (a.tile != b.tile) return a.tile < b.tile;
    if (a.depth != b.depth) return a.depth < b.depth;
    return a.index < b.index;
  });
  int64_t m = (int64_t)pairs.size();
  for (int64_t k = 0; k < std::min(m, cap); ++k) {
    tile_out[k] = pairs[k].tile;
    index_out[k] = (uint32_t)pairs[k].index;
  }
  return m;
}

// Exact FP64 gradient of sum(dimg * img) with respect to every parameter.
//   dimg: [3][H][W]; g2d (optional): [n][9] = dL/d(u, v, A, B, C, opacity, r, g, b)
//   with (A, B, C) the conic entries; outputs [3][n], [3][n], [4][n], [n], [16][3][n].
//   abs_out (optional, [59][n]: means, scales, quats, opac, sh): the same chain
//   applied to the sums of the magnitudes of the per-pixel terms, a bound on
//   what a gradient entry's summands add up to before they cancel (the scale
//   of the rounding error of any evaluation that sums them in another order).
//   The colour behind an entry counts with the magnitude of the pixel's final
//   colour: an adjoint that walks front to back forms it as the final colour
//   minus the colour in front, a difference of numbers of that size.  Each
//   per-pixel term is weighted by k + mag_offset, k the number of contributors
//   in front of the entry at that pixel: the rounding of its transmittance and
//   of the colour in front grows with k, the rest of a term's rounding does not.
//   near_out (optional, [n], zeroed by the caller): set to 1 for every Gaussian
//   that contributes to a pixel with a decision within a relative near_band of
//   its threshold (alpha vs 1/255, T vs 1e-4, raw alpha vs 0.99), and for the
//   entries at the band.  The gradient is piecewise smooth with jumps at these
//   decisions (one of them changes the transmittance behind it and the colour
//   behind the entries in front), so such a Gaussian's gradient may
//   legitimately take another value at a slightly different precision.
int orc_render_bwd(int64_t n, const double* means, const double* scales, const double* quats, const double* opac,
                   const double* sh, int deg, const double* cam_d, const int32_t* cam_i, const double* bg,
                   const double* dimg, double* g2d_out, double* dmeans, double* dscales, double* dquats,
                   double* dopac, double* dsh, double near_band, int32_t* near_out, double* abs_out,
                   double mag_offset) {
  Cam cam = to_cam(cam_d, cam_i);
  Inputs in{n, means, scales, quats, opac, sh, deg};
  std::vector<Splat> splats;
  std::vector<Decisions> decs;
  project_all(in, cam, splats, &decs);
  const int W = cam.width, H = cam.height;
  const int64_t P = (int64_t)W * H;
  std::vector<std::vector<const Splat*>> rows;
  row_lists(splats, H, rows, nullptr);
  // per-pixel adjoint of Eq. 1, accumulated per Gaussian (per-thread buffers)
  std::vector<double> g2d((size_t)n * 9, 0.0);
  // sums of the magnitudes of the same per-pixel terms (abs_out only)
  std::vector<double> g2d_abs(abs_out ? (size_t)n * 9 : 0, 0.0);
#pragma omp parallel
  {
    std::vector<double> loc((size_t)n * 9, 0.0);
    std::vector<double> loc_abs(abs_out ? (size_t)n * 9 : 0, 0.0);
    std::vector<const Splat*> contrib, near;
    std::vector<char> loc_near(near_out ? (size_t)n : 0, 0);
    std::vector<double> alphas, Ts;
#pragma omp for schedule(dynamic, 64)
    for (int64_t p = 0; p < P; ++p) {
      int i = (int)(p % W), j = (int)(p / W);
      contrib.clear(); alphas.clear(); Ts.clear(); near.clear();
      PixelResult r = composite(rows[j], i, j, bg, &contrib, &alphas, &Ts, -1, near_out ? &near : nullptr,
                                near_band);
      // a decision near its threshold changes the transmittance of every entry
      // behind it and the colour behind every entry in front: all of the
      // pixel's contributors are marked, with the entries at the band
      if (!near.empty()) {
        for (const Splat* s : near) loc_near[(size_t)s->index] = 1;
        for (const Splat* s : contrib) loc_near[(size_t)s->index] = 1;
      }
      double gC[3] = {dimg[p], dimg[P + p], dimg[2 * P + p]};
      // R = colour accumulated behind entry k, including the background
      double Racc[3] = {r.T * bg[0], r.T * bg[1], r.T * bg[2]};
      for (int64_t k = (int64_t)contrib.size() - 1; k >= 0; --k) {
        const Splat* s = contrib[k];
        double a = alphas[k], T = Ts[k];
        double* G = &loc[(size_t)s->index * 9];
        double dalpha = 0.0, dalpha_abs = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
          G[6 + ch] += gC[ch] * a * T;
          dalpha += gC[ch] * (s->rgb[ch] * T - Racc[ch] / (1.0 - a));
          // magnitude of the operands of the colour behind the entry when it is
          // formed as (final colour - colour up to and including the entry), the
          // form a front-to-back adjoint evaluates: both are at most r.C
          dalpha_abs += std::fabs(gC[ch]) * (s->rgb[ch] * T + r.C[ch] / (1.0 - a));
          Racc[ch] += s->rgb[ch] * a * T;
        }
        double dx = (i + 0.5) - s->u, dy = (j + 0.5) - s->v;
        double power = -0.5 * (s->A * dx * dx + s->C * dy * dy) - s->B * dx * dy;
        double Gv = std::exp(power);
        if (abs_out) {
          // weight k + mag_offset: the entry's transmittance and the colour in
          // front are products and sums over the k contributors in front of it
          const double wk = (double)k + mag_offset;
          double* Ga = &loc_abs[(size_t)s->index * 9];
          for (int ch = 0; ch < 3; ++ch) Ga[6 + ch] += wk * std::fabs(gC[ch]) * a * T;
          if (!(s->o * Gv > kAlphaMax)) {
            double pa = wk * dalpha_abs * s->o * Gv;
            Ga[5] += wk * dalpha_abs * Gv;
            Ga[0] += pa * (std::fabs(s->A * dx) + std::fabs(s->B * dy));
            Ga[1] += pa * (std::fabs(s->C * dy) + std::fabs(s->B * dx));
            Ga[2] += pa * 0.5 * dx * dx;
            Ga[3] += pa * std::fabs(dx * dy);
            Ga[4] += pa * 0.5 * dy * dy;
          }
        }
        if (s->o * Gv > kAlphaMax) continue;  // clamped: no gradient to o or the footprint
        G[5] += dalpha * Gv;
        double dpow = dalpha * s->o * Gv;
        G[0] += dpow * (s->A * dx + s->B * dy);   // d power / d u
        G[1] += dpow * (s->C * dy + s->B * dx);   // d power / d v
        G[2] += dpow * (-0.5 * dx * dx);
        G[3] += dpow * (-dx * dy);
        G[4] += dpow * (-0.5 * dy * dy);
      }
    }
#pragma omp critical
    {
      for (size_t k = 0; k < g2d.size(); ++k) g2d[k] += loc[k];
      for (size_t k = 0; k < g2d_abs.size(); ++k) g2d_abs[k] += loc_abs[k];
      if (near_out)
        for (int64_t k = 0; k < n; ++k) near_out[k] |= loc_near[(size_t)k];
    }
  }
  if (g2d_out) std::memcpy(g2d_out, g2d.data(), g2d.size() * sizeof(double));
  // per-Gaussian chain rule, exact via dual numbers over the projection
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t g = 0; g < n; ++g) {
    for (int k = 0; k < 3; ++k) { dmeans[k * n + g] = 0; dscales[k * n + g] = 0; }
    for (int k = 0; k < 4; ++k) dquats[k * n + g] = 0;
    dopac[g] = 0;
    for (int k = 0; k < 48; ++k) dsh[(size_t)k * n + g] = 0;
    // abs_out layout: means [3][n], scales [3][n], quats [4][n], opac [n], sh [48][n]
    double* am = abs_out ? abs_out : nullptr;
    double* as = abs_out ? abs_out + 3 * n : nullptr;
    double* aq = abs_out ? abs_out + 6 * n : nullptr;
    double* ao = abs_out ? abs_out + 10 * n : nullptr;
    double* ash = abs_out ? abs_out + 11 * n : nullptr;
    if (abs_out) {
      for (int k = 0; k < 3; ++k) am[k * n + g] = as[k * n + g] = 0;
      for (int k = 0; k < 4; ++k) aq[k * n + g] = 0;
      ao[g] = 0;
      for (int k = 0; k < 48; ++k) ash[(size_t)k * n + g] = 0;
    }
    const Decisions& dec = decs[g];
    if (!dec.visible) continue;
    const double* G = &g2d[(size_t)g * 9];
    const double* Ga = abs_out ? &g2d_abs[(size_t)g * 9] : nullptr;
    dopac[g] = G[5];
    if (abs_out) ao[g] = Ga[5];
    double m[3], s[3], q[4], shv[48];
    load_params(in, g, m, s, q, shv);
    // SH coefficients enter the colour linearly: d rgb_ch / d f_{k,ch} = Y_k(dir)
    {
      double Cw[3];
      for (int k = 0; k < 3; ++k)
        Cw[k] = -((cam.R[k] * cam.t[0] + cam.R[3 + k] * cam.t[1]) + cam.R[6 + k] * cam.t[2]);
      double e0 = m[0] - Cw[0], e1 = m[1] - Cw[1], e2 = m[2] - Cw[2];
      double en = std::sqrt((e0 * e0 + e1 * e1) + e2 * e2);
      double Y[16];
      sh_basis(e0 / en, e1 / en, e2 / en, deg, Y);
      int nk = (deg + 1) * (deg + 1);
      for (int k = 0; k < nk; ++k)
        for (int ch = 0; ch < 3; ++ch)
          if (!dec.rgb_clamped[ch]) {
            dsh[(size_t)(k * 3 + ch) * n + g] = Y[k] * G[6 + ch];
            if (abs_out) ash[(size_t)(k * 3 + ch) * n + g] = std::fabs(Y[k]) * Ga[6 + ch];
          }
    }
    // geometry parameters: 3 means, 3 scales, 4 quaternion entries
    for (int dir = 0; dir < 10; ++dir) {
      Dual M[3], S[3], Q[4], SH[48];
      for (int k = 0; k < 3; ++k) { M[k] = Dual(m[k], dir == k ? 1.0 : 0.0); S[k] = Dual(s[k], dir == 3 + k ? 1.0 : 0.0); }
      for (int k = 0; k < 4; ++k) Q[k] = Dual(q[k], dir == 6 + k ? 1.0 : 0.0);
      for (int k = 0; k < 48; ++k) SH[k] = Dual(shv[k], 0.0);
      Decisions d2 = dec;
      Proj<Dual> Pd;
      project_one<Dual>(M, S, Q, SH, deg, opac[g], cam, d2, Pd, false);
      double gsum = G[0] * Pd.u.d + G[1] * Pd.v.d + G[2] * Pd.A.d + G[3] * Pd.B.d + G[4] * Pd.C.d +
                    G[6] * Pd.rgb[0].d + G[7] * Pd.rgb[1].d + G[8] * Pd.rgb[2].d;
      if (dir < 3) dmeans[dir * n + g] = gsum;
      else if (dir < 6) dscales[(dir - 3) * n + g] = gsum;
      else dquats[(dir - 6) * n + g] = gsum;
      if (abs_out) {
        double asum = Ga[0] * std::fabs(Pd.u.d) + Ga[1] * std::fabs(Pd.v.d) + Ga[2] * std::fabs(Pd.A.d) +
                      Ga[3] * std::fabs(Pd.B.d) + Ga[4] * std::fabs(Pd.C.d);
        for (int ch = 0; ch < 3; ++ch) asum += Ga[6 + ch] * std::fabs(Pd.rgb[ch].d);
        if (dir < 3) am[dir * n + g] = asum;
        else if (dir < 6) as[(dir - 3) * n + g] = asum;
        else aq[(dir - 6) * n + g] = asum;
      }
    }
  }
  return 0;
}

}  // extern "C"
