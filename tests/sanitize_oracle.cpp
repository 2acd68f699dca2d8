// Host-only driver for the sanitizer test: runs every entry point of the
// oracle (oracle/raster.cpp, linked in) on a small seeded scene with
// degenerate members, under AddressSanitizer and UndefinedBehaviorSanitizer.
// Exit status 0 when every call returned normally.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
int orc_project(int64_t, const double*, const double*, const double*, const double*, const double*, int,
                const double*, const int32_t*, int, int, int32_t*, uint32_t*, int32_t*, int32_t*, double*, double*,
                double*, double*, int32_t*, double*);
int orc_render(int64_t, const double*, const double*, const double*, const double*, const double*, int, const double*,
               const int32_t*, const double*, const int64_t*, int64_t, double*, double*, int32_t*, int32_t*, double*,
               double*, int32_t*);
int orc_render_tiled(int64_t, const double*, const double*, const double*, const double*, const double*, int,
                     const double*, const int32_t*, const double*, int, int, double*, double*, int32_t*);
int64_t orc_pairs(int64_t, const double*, const double*, const double*, const double*, const double*, int,
                  const double*, const int32_t*, int, int, int64_t, uint32_t*, uint32_t*);
int orc_render_bwd(int64_t, const double*, const double*, const double*, const double*, const double*, int,
                   const double*, const int32_t*, const double*, const double*, double*, double*, double*, double*,
                   double*, double*, double, int32_t*, double*, double);
}

static uint64_t state = 12345;
static double uniform() {  // 53-bit uniform from a 64-bit LCG
  state = state * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}

static int run(int64_t n, int W, int H) {
  std::vector<double> means(3 * n), scales(3 * n), quats(4 * n), opac(n), sh(48 * n);
  for (int64_t g = 0; g < n; ++g) {
    for (int k = 0; k < 3; ++k) means[k * n + g] = 2.0 * uniform() - 1.0;
    for (int k = 0; k < 3; ++k) scales[k * n + g] = std::exp(-3.0 + uniform());
    for (int k = 0; k < 4; ++k) quats[k * n + g] = uniform() - 0.5;
    opac[g] = uniform();
    for (int k = 0; k < 48; ++k) sh[k * n + g] = 0.3 * (uniform() - 0.5);
  }
  if (n >= 5) {
    means[0] = NAN;                       // non-finite centre
    for (int k = 0; k < 4; ++k) quats[k * n + 1] = 0.0;  // zero quaternion
    means[2 * n + 2] = -10.0;             // behind the camera
    scales[3] = 1e6;                      // footprint larger than the image
    opac[4] = 1e-4;                       // below 1/255
  }
  const double cam_d[17] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 3, 0.866 * W, 0.866 * W, 0.5 * W, 0.5 * H, 0.2};
  const int32_t cam_i[2] = {W, H};
  const double bg[3] = {0.1, 0.2, 0.3};
  const int64_t P = (int64_t)W * H;
  std::vector<int32_t> vis(n), rect(4 * n), tt(n), clamped(3 * n), nc(P), amb(P), gamb(P), near(n);
  std::vector<uint32_t> depth(n);
  std::vector<double> uv(2 * n), cov(3 * n), conic(3 * n), rgb(3 * n), radius(n), img(3 * P), T(P), img_alt(3 * P),
      T_alt(P);
  orc_project(n, means.data(), scales.data(), quats.data(), opac.data(), sh.data(), 3, cam_d, cam_i, 16, 16,
              vis.data(), depth.data(), rect.data(), tt.data(), uv.data(), cov.data(), conic.data(), rgb.data(),
              clamped.data(), radius.data());
  orc_render(n, means.data(), scales.data(), quats.data(), opac.data(), sh.data(), 3, cam_d, cam_i, bg, nullptr, 0,
             img.data(), T.data(), nc.data(), amb.data(), img_alt.data(), T_alt.data(), gamb.data());
  std::vector<int64_t> pix = {0, P - 1, P / 2};
  std::vector<double> img3(9), T3(3);
  std::vector<int32_t> nc3(3);
  orc_render(n, means.data(), scales.data(), quats.data(), opac.data(), sh.data(), 3, cam_d, cam_i, bg, pix.data(),
             3, img3.data(), T3.data(), nc3.data(), nullptr, nullptr, nullptr, nullptr);
  orc_render_tiled(n, means.data(), scales.data(), quats.data(), opac.data(), sh.data(), 2, cam_d, cam_i, bg, 8, 8,
                   img.data(), T.data(), nc.data());
  const int64_t m = orc_pairs(n, means.data(), scales.data(), quats.data(), opac.data(), sh.data(), 3, cam_d, cam_i,
                              16, 16, 0, nullptr, nullptr);
  std::vector<uint32_t> tiles(m > 0 ? m : 1), idx(m > 0 ? m : 1);
  orc_pairs(n, means.data(), scales.data(), quats.data(), opac.data(), sh.data(), 3, cam_d, cam_i, 16, 16, m,
            tiles.data(), idx.data());
  std::vector<double> dimg(3 * P), g2d(9 * n), dm(3 * n), ds(3 * n), dq(4 * n), dop(n), dsh(48 * n), mag(59 * n);
  for (int64_t p = 0; p < 3 * P; ++p) dimg[p] = uniform() - 0.5;
  orc_render_bwd(n, means.data(), scales.data(), quats.data(), opac.data(), sh.data(), 3, cam_d, cam_i, bg,
                 dimg.data(), g2d.data(), dm.data(), ds.data(), dq.data(), dop.data(), dsh.data(), 1e-4, near.data(),
                 mag.data(), 64.0);
  orc_render_bwd(n, means.data(), scales.data(), quats.data(), opac.data(), sh.data(), 1, cam_d, cam_i, bg,
                 dimg.data(), nullptr, dm.data(), ds.data(), dq.data(), dop.data(), dsh.data(), 0.0, nullptr, nullptr,
                 1.0);
  std::printf("n=%lld %dx%d: pairs %lld\n", (long long)n, W, H, (long long)m);
  return 0;
}

int main() {
  run(300, 64, 48);  // ragged tiles, degenerate members
  run(0, 16, 16);    // empty scene
  run(20, 1, 1);     // one pixel
  return 0;
}
