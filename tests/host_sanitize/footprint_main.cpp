// Host-side exercise of plan construction under AddressSanitizer and
// UndefinedBehaviorSanitizer: pc_plan_footprint runs the whole host layout
// (FP64 phases, fine cells and offsets, band, tile sort, spreading work list,
// w-plane geometry) without touching a device.  Geometries cover a random
// uniform disc, a dense Gaussian core (split hot tiles), a narrow band (no
// wrap), visibilities on cell and tile edges, a single visibility, the
// smallest and largest grids, metres, several accuracies and non-coplanar w;
// bad geometries must fail with their documented status.  Prints "ok".
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "polyclean.h"

namespace {

struct Lcg {  // 64-bit linear congruential generator, uniform in [0, 1)
  uint64_t s;
  double next() {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) * (1.0 / 9007199254740992.0);
  }
};

int failures = 0;

void expect(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (%s)\n", what, pc_last_error());
    ++failures;
  }
}

pc_geometry geo(const std::vector<double>& u, const std::vector<double>& v, int npix, double fov) {
  pc_geometry g{};
  g.nvis = (int64_t)u.size();
  g.u = u.data();
  g.v = v.data();
  g.w = nullptr;
  g.npix = npix;
  g.fov_rad = fov;
  g.uv_units = PC_UV_WAVELENGTHS;
  g.freq_hz = 0;
  g.nufft_eps = 1e-6;
  g.upsamp = 2.0;
  g.precision = PC_PREC_FP32;
  return g;
}

size_t footprint(const pc_geometry& g, pc_status want = PC_OK) {
  size_t b = 0;
  const pc_status st = pc_plan_footprint(&g, &b);
  expect(st == want, "status");
  return b;
}

}  // namespace

int main() {
  Lcg r{12345};
  for (int npix : {16, 64, 256, 1024, 4096}) {
    const double fov = 0.05, dl = fov / npix;
    for (int L : {1, 7, 1000, 20000}) {
      std::vector<double> u(L), v(L), w(L);
      for (int k = 0; k < L; ++k) {  // uniform over the whole periodic grid
        u[k] = (r.next() - 0.5) / dl;
        v[k] = (r.next() - 0.5) / dl;
        w[k] = (r.next() - 0.5) * 2000.0;
      }
      pc_geometry g = geo(u, v, npix, fov);
      expect(footprint(g) > 0, "uniform");
      g.w = w.data();
      expect(footprint(g) > 0, "uniform with w");
      g.w = nullptr;
      for (double eps : {1e-2, 1e-4, 1e-9, 1e-14}) {
        g.nufft_eps = eps;
        expect(footprint(g) > 0, "accuracy");
      }
    }
  }
  {  // dense core: hot tiles split into partials
    const int npix = 512, L = 200000;
    const double fov = 0.05, dl = fov / npix;
    std::vector<double> u(L), v(L);
    for (int k = 0; k < L; ++k) {
      const double a = r.next() * 6.283185307179586, rad = std::sqrt(-2 * std::log(1 - r.next()));
      u[k] = 0.01 * rad * std::cos(a) / dl;
      v[k] = 0.01 * rad * std::sin(a) / dl;
    }
    expect(footprint(geo(u, v, npix, fov)) > 0, "dense core");
  }
  {  // narrow band, visibilities on cell and tile edges
    const int npix = 1024, M = 2 * npix;
    const double fov = 0.05, dl = fov / npix;
    std::vector<double> u, v;
    for (int c = -300; c <= 300; c += 1) {
      u.push_back((double)c / M / dl);
      v.push_back((double)(c / 2) / M / dl);
      u.push_back((32.0 * (c / 32)) / M / dl);
      v.push_back((-32.0 * (c / 32) + 0.5) / M / dl);
    }
    expect(footprint(geo(u, v, npix, fov)) > 0, "edges");
  }
  {  // largest grid, a few visibilities; metres
    std::vector<double> u{1.0, -2.0, 3.5}, v{0.5, 7.0, -1.25};
    expect(footprint(geo(u, v, 8192, 0.05)) > 0, "8192");
    pc_geometry g = geo(u, v, 64, 0.05);
    g.uv_units = PC_UV_METRES;
    g.freq_hz = 150e6;
    expect(footprint(g) > 0, "metres");
    g.precision = PC_PREC_FP64;
    expect(footprint(g) > 0, "fp64");
  }
  {  // refusals
    std::vector<double> u{1.0, 2.0}, v{1.0, NAN}, w{0.0, 5.0};
    footprint(geo(u, v, 64, 0.05), PC_ERR_INVALID_ARG);
    v[1] = 2.0;
    footprint(geo(u, v, 63, 0.05), PC_ERR_INVALID_ARG);
    footprint(geo(u, v, 64, 2.0), PC_ERR_INVALID_ARG);
    pc_geometry g = geo(u, v, 64, 0.05);
    g.upsamp = 1.5;
    footprint(g, PC_ERR_UNSUPPORTED);
    g = geo(u, v, 64, 0.05);
    g.w = w.data();
    g.precision = PC_PREC_FP64;
    footprint(g, PC_ERR_UNSUPPORTED);
    g.nvis = 0;
    footprint(g, PC_ERR_INVALID_ARG);
  }
  if (failures) return 1;
  std::printf("ok\n");
  return 0;
}
