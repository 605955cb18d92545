// PWBF_TUNE_CACHE across two processes. Run with PWBF_TUNE_CACHE set and
// PWBF_DEBUG=1: "store" plans a geometry (default shape), stores a measured
// shape as the tuner does (which writes the cache file); a second process run
// as "load" must plan the same geometry with that shape, read from the file.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pwbf.h"
#include "../../paper_2311_00482_amd/csrc/plan_host.h"

#define CHECK(c)                                                                 \
  do {                                                                           \
    if (!(c)) {                                                                  \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                              \
    }                                                                            \
  } while (0)

int main(int argc, char **argv) {
  CHECK(argc == 2 && std::getenv("PWBF_TUNE_CACHE"));
  std::vector<double> ex(128), th(5), t0(5, 0.0);
  for (int e = 0; e < 128; ++e) ex[e] = (e - 63.5) * 0.3e-3;
  for (int a = 0; a < 5; ++a) th[a] = (-10.0 + 5.0 * a) * M_PI / 180.0;
  pwbf_geometry g;
  std::memset(&g, 0, sizeof g);
  g.abi_version = PWBF_ABI_VERSION;
  g.n_angles = 5;
  g.n_channels = 128;
  g.n_samples = 4096;
  g.elem_x = ex.data();
  g.angle_rad = th.data();
  g.t0 = t0.data();
  g.c = 1540;
  g.fs = 20.8e6;
  g.f0 = 5.2e6;
  g.nx = 512;
  g.nz = 512;
  g.dx = 0.075e-3;
  g.x0 = -0.5 * g.dx * 511;
  g.dz = 0.078e-3;
  g.z0 = 5e-3;
  g.f_number = 1.5;
  g.apod = PWBF_APOD_HANN;
  g.log_floor_db = -60;
  const pwbf_tile tuned = {2, 4, 2, 4, 0};
  pwbf::FramePlan P;
  std::string err;
  CHECK(pwbf::plan_frame(&g, pwbf::kF32, pwbf::kDas, -1, nullptr, &P, &err, 0) == PWBF_OK);
  const bool is_tuned = P.cpw == tuned.cpw && P.lz == tuned.lz && P.wz == tuned.wz &&
                        P.wx == tuned.wx;
  if (std::strcmp(argv[1], "store") == 0) {
    CHECK(!is_tuned);  // the default shape differs from the one stored below
    pwbf::tune_store(pwbf::shape_key(&g, pwbf::kF32, pwbf::kDas, -1, 0), tuned);
    // the plan cache sees the new table at once
    CHECK(pwbf::plan_frame(&g, pwbf::kF32, pwbf::kDas, -1, nullptr, &P, &err, 0) == PWBF_OK);
    CHECK(P.cpw == tuned.cpw && P.lz == tuned.lz && P.wz == tuned.wz && P.wx == tuned.wx);
  } else {
    CHECK(std::strcmp(argv[1], "load") == 0);
    CHECK(is_tuned);
  }
  std::puts("all ok");
  return 0;
}
