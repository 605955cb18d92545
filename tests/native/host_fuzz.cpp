// Host validation, launch planning and the tuning table under random and
// hostile arguments (built with the address and undefined-behaviour
// sanitizers by the test that runs it). Every accepted plan must satisfy the
// invariants the kernels rely on; every rejected one must come with a message;
// nothing may overflow, read out of bounds or crash. Prints "ok <part>" lines
// and exits 1 at the first failed check.
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <random>
#include <string>
#include <vector>

#include "../../include/pwbf.h"
#include "../../paper_2311_00482_amd/csrc/plan_host.h"

#define CHECK(c)                                                                    \
  do {                                                                              \
    if (!(c)) {                                                                     \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c);    \
      std::exit(1);                                                                 \
    }                                                                               \
  } while (0)

namespace {

std::mt19937_64 rng(20231101);

double uni() { return std::uniform_real_distribution<double>(0.0, 1.0)(rng); }
int pick(int n) { return (int)(rng() % (uint64_t)n); }
bool chance(double p) { return uni() < p; }

const double kNaN = std::numeric_limits<double>::quiet_NaN();
const double kInf = std::numeric_limits<double>::infinity();

double hostile_double(double v) {
  static const double s[] = {0.0, -0.0, -1.0, kNaN, kInf, -kInf, 1e300, -1e300, 1e-300, 5e-324};
  return chance(0.5) ? s[pick(10)] : v * std::exp2((double)pick(200) - 100);
}

int32_t hostile_int(int32_t v) {
  static const int32_t s[] = {0, -1, 1, 2, 3, 31, 32, 33, 255, 256, 257, 4096, 4097, 1 << 24,
                              (1 << 24) - 1, INT_MAX, INT_MIN, 65535, 65536};
  return chance(0.6) ? s[pick(19)] : (int32_t)std::max<int64_t>(INT_MIN, std::min<int64_t>(INT_MAX, (int64_t)v + pick(9) - 4));
}

struct Geo {
  pwbf_geometry g;
  std::vector<double> elem_x, angle, t0;
};

// A valid plane-wave geometry: the paper's linear array and grid family with
// random sizes, then zero or more hostile fields.
Geo make_geo(bool mutate) {
  Geo G;
  pwbf_geometry &g = G.g;
  std::memset(&g, 0, sizeof g);
  g.abi_version = PWBF_ABI_VERSION;
  const int na[] = {1, 3, 5, 11, 16, 31, 32};
  const int nc[] = {1, 2, 16, 64, 128, 192, 256};
  const int ns[] = {2, 64, 512, 2048, 4096, 1 << 16};
  g.n_angles = na[pick(7)];
  g.n_channels = nc[pick(7)];
  g.n_samples = ns[pick(6)];
  const double pitch = 0.3e-3 * (0.5 + uni());
  G.elem_x.resize(g.n_channels);
  for (int e = 0; e < g.n_channels; ++e) G.elem_x[e] = (e - (g.n_channels - 1) / 2.0) * pitch;
  G.angle.resize(g.n_angles);
  for (int a = 0; a < g.n_angles; ++a)
    G.angle[a] = g.n_angles == 1 ? 0.0 : (-16.0 + 32.0 * a / (g.n_angles - 1)) * M_PI / 180.0;
  G.t0.assign(g.n_angles, 0.0);
  g.c = 1540.0;
  g.fs = 20.8e6 * (0.5 + uni());
  g.f0 = 5.2e6;
  const int nx[] = {1, 2, 7, 64, 128, 256, 387, 1024};
  const int nz[] = {1, 2, 16, 100, 256, 1024, 1 << 12};
  g.nx = nx[pick(8)];
  g.nz = nz[pick(7)];
  g.dx = pitch * (0.25 + uni());
  g.dz = 0.1e-3 * (0.2 + 4 * uni());
  g.x0 = -0.5 * g.dx * (g.nx - 1);
  g.z0 = 5e-3 * uni();
  g.f_number = 0.5 + 2 * uni();
  g.apod = pick(3);
  g.bandpass = pick(2);
  g.log_floor_db = -60.0;
  g.pdas_p = 1.0 + uni();
  bool t0_null = chance(0.2);  // NULL t0: every angle starts at time 0
  if (mutate) {
    const int n = 1 + pick(3);
    for (int k = 0; k < n; ++k) {
      switch (pick(24)) {
        case 0: g.abi_version = (uint32_t)pick(8); break;
        case 1: g.n_angles = hostile_int(g.n_angles); break;
        case 2: g.n_channels = hostile_int(g.n_channels); break;
        case 3: g.n_samples = hostile_int(g.n_samples); break;
        case 4: g.c = hostile_double(g.c); break;
        case 5: g.fs = hostile_double(g.fs); break;
        case 6: g.f0 = hostile_double(g.f0); break;
        case 7: g.nx = hostile_int(g.nx); break;
        case 8: g.nz = hostile_int(g.nz); break;
        case 9: g.x0 = hostile_double(g.x0); break;
        case 10: g.dx = hostile_double(g.dx); break;
        case 11: g.z0 = hostile_double(g.z0); break;
        case 12: g.dz = hostile_double(g.dz); break;
        case 13: g.f_number = hostile_double(g.f_number); break;
        case 14: g.apod = hostile_int(g.apod); break;
        case 15: g.bandpass = hostile_int(g.bandpass); break;
        case 16: g.log_floor_db = hostile_double(g.log_floor_db); break;
        case 17: g.pdas_p = hostile_double(g.pdas_p); break;
        case 18: if (!G.elem_x.empty()) G.elem_x[pick((int)G.elem_x.size())] = hostile_double(1e-3); break;
        case 19: if (!G.angle.empty()) G.angle[pick((int)G.angle.size())] = hostile_double(0.2); break;
        case 20: if (!G.t0.empty()) G.t0[pick((int)G.t0.size())] = hostile_double(1e-6); break;
        case 21: t0_null = true; break;
        case 22: g.iq_decimation = chance(0.5) ? (1 << pick(4)) : hostile_int(2); break;
        case 23: g.reserved = hostile_int(0); break;
      }
    }
  }
  // the arrays must hold what the counts claim, or the call reads past them:
  // keep them at least that long (hostile counts are capped by validation first)
  const size_t nch = g.n_channels > 0 ? std::min<size_t>(g.n_channels, 4096) : 0;
  const size_t nan_ = g.n_angles > 0 ? std::min<size_t>(g.n_angles, 4096) : 0;
  while (G.elem_x.size() < nch) G.elem_x.push_back(G.elem_x.empty() ? 0.0 : G.elem_x.back() + pitch);
  while (G.angle.size() < nan_) G.angle.push_back(0.0);
  while (G.t0.size() < nan_) G.t0.push_back(0.0);
  g.elem_x = G.elem_x.data();
  g.angle_rad = G.angle.data();
  g.t0 = t0_null ? nullptr : G.t0.data();
  return G;
}

pwbf_tile hostile_tile() {
  pwbf_tile t;
  const int cpw[] = {0, 1, 2, 3, 4, 8, 16, 32, -1};
  t.cpw = cpw[pick(9)];
  t.lz = chance(0.8) ? (1 << pick(7)) : hostile_int(4);
  t.wz = chance(0.8) ? 1 + pick(8) : hostile_int(2);
  t.wx = chance(0.8) ? 1 + pick(8) : hostile_int(2);
  t.chunk = chance(0.7) ? pick(300) : hostile_int(16);
  return t;
}

// What every accepted plan guarantees to the kernels.
void check_plan(const pwbf_geometry &g, const pwbf::FramePlan &P, int mode, int angle, int waves) {
  CHECK(P.cpw >= 1 && P.cpw <= 16 && (P.cpw & (P.cpw - 1)) == 0);
  CHECK(P.lz >= 1 && P.lx >= 1 && P.cpw * P.lz * P.lx == pwbf::kWave);
  CHECK(P.wz >= 1 && P.wx >= 1 && P.wz * P.wx <= pwbf::kMaxWavesPerBlock);
  if (waves) CHECK(P.wz * P.wx == waves);
  CHECK(P.tile_z == P.lz * P.wz && P.tile_x == P.lx * P.wx);
  CHECK(P.tiles_z >= 1 && P.tiles_x >= 1 && P.n_tiles == P.tiles_z * P.tiles_x);
  CHECK((int64_t)P.tiles_z * P.tile_z >= g.nz && (int64_t)(P.tiles_z - 1) * P.tile_z < g.nz);
  CHECK((int64_t)P.tiles_x * P.tile_x >= g.nx && (int64_t)(P.tiles_x - 1) * P.tile_x < g.nx);
  CHECK(P.chunk >= P.cpw && P.chunk % P.cpw == 0);
  CHECK(P.win >= 1 && P.win <= pwbf::max_window(mode));
  CHECK(P.n_angles == (angle < 0 ? g.n_angles : 1));
  CHECK(pwbf::plan_lds_bytes(P) <= (size_t)pwbf::kMaxLdsBytes);
  CHECK(std::isfinite(P.X0) && std::isfinite(P.DX) && std::isfinite(P.Z0) && std::isfinite(P.DZ));
  for (int a = 0; a < P.n_angles; ++a)
    CHECK(std::isfinite(P.sa[a]) && std::isfinite(P.ca[a]) && std::isfinite(P.to[a]));
  const int probe_tiles[] = {0, P.n_tiles / 2, P.n_tiles - 1};
  for (int t : probe_tiles) {
    const double c = pwbf::tile_cost(&g, P, t);
    CHECK(std::isfinite(c) && c >= 0);
    const int ch = pwbf::tile_active_channels(&g, P, t);
    CHECK(ch >= 0 && ch <= g.n_channels);
  }
}

void fuzz_plans(int iters) {
  int accepted_geo = 0, accepted_plan = 0, rejected = 0;
  for (int it = 0; it < iters; ++it) {
    Geo G = make_geo(chance(0.7));
    const pwbf_geometry &g = G.g;
    std::string err;
    const int vg = pwbf::validate_geometry(&g, &err);
    if (vg) {
      CHECK(!err.empty());
      ++rejected;
    } else {
      ++accepted_geo;
      CHECK(g.n_angles >= 1 && g.n_angles <= PWBF_MAX_ANGLES);
      CHECK(g.n_channels >= 1 && g.n_channels <= PWBF_MAX_CHANNELS);
      CHECK((int64_t)g.n_angles * g.n_channels * g.n_samples < (int64_t)1 << 31);
      CHECK(std::isfinite(g.c) && g.c > 0 && std::isfinite(g.fs) && g.fs > 0);
      CHECK(std::isfinite(g.dx) && g.dx > 0 && std::isfinite(g.dz) && g.dz > 0);
    }
    for (int rep = 0; rep < 3; ++rep) {
      const int mode = chance(0.9) ? pick(5) : hostile_int(1);
      const int dtype = chance(0.9) ? pick(4) : hostile_int(1);
      const int angle = chance(0.5) ? -1 : (chance(0.8) ? pick(std::max(1, g.n_angles)) : hostile_int(0));
      const int waves = chance(0.5) ? 0 : 8;
      pwbf_tile t = hostile_tile();
      const pwbf_tile *tp = chance(0.5) ? nullptr : &t;
      pwbf::FramePlan P;
      std::memset(&P, 0, sizeof P);
      err.clear();
      const int rc = pwbf::plan_frame(&g, dtype, mode, angle, tp, &P, &err, waves);
      if (rc) {
        CHECK(!err.empty());
        CHECK(rc == PWBF_E_INVALID || rc == PWBF_E_UNSUPPORTED);
        continue;
      }
      CHECK(vg == 0);  // an invalid geometry never plans
      ++accepted_plan;
      check_plan(g, P, mode, angle, waves);
      // outputs and workspace: fake aligned device addresses, checked on the host only
      float *fake = (float *)(uintptr_t)4096;
      pwbf_outputs o = {fake, chance(0.5) ? fake : nullptr, chance(0.5) ? fake : nullptr,
                        chance(0.5) ? fake : nullptr, chance(0.3) ? fake : nullptr};
      const size_t need = pwbf::workspace_bytes(&g, &o);
      std::vector<unsigned char> ws(std::min<size_t>(need, 1 << 22) + 256);
      void *wsp = (void *)(((uintptr_t)ws.data() + 255) / 256 * 256);
      err.clear();
      const int vo = pwbf::validate_outputs(&g, &o, need ? wsp : nullptr,
                                            need ? std::min<size_t>(need, 1 << 22) : 0, &err, mode);
      if (vo) CHECK(!err.empty());
      if (!vo && pwbf::post_needed(&o) && !pwbf::is_iq_mode(mode)) {
        pwbf::PostPlan Q;
        std::memset(&Q, 0, sizeof Q);
        pwbf::build_post_plan(&g, &o, wsp, &Q);
        CHECK(Q.nx == g.nx && Q.nz == g.nz && (1 << Q.log2nz) == g.nz);
        if (g.bandpass)  // the kept band of bins, or none (-1, -2)
          CHECK((Q.k_lo == -1 && Q.k_hi == -2) ||
                (0 <= Q.k_lo && Q.k_lo <= Q.k_hi && Q.k_hi <= g.nz / 2));
        else
          CHECK(Q.k_lo == 0 && Q.k_hi == 0);
      }
    }
  }
  CHECK(accepted_geo > iters / 10 && accepted_plan > iters / 10 && rejected > iters / 10);
  std::printf("ok plans (%d geometries accepted, %d rejected, %d plans)\n", accepted_geo,
              rejected, accepted_plan);
}

// The tuning table: save and load round trip, and files with damaged or
// hostile lines. A tuned shape that does not fit is never used.
void fuzz_tune(const char *dir) {
  const std::string path = std::string(dir) + "/tune_fuzz.json";
  pwbf::tune_clear();
  Geo G = make_geo(false);
  G.g.n_angles = 5;
  G.g.nx = 128;
  G.g.nz = 256;
  G.g.n_channels = 128;
  G.g.n_samples = 2048;
  G.elem_x.resize(128);
  for (int e = 0; e < 128; ++e) G.elem_x[e] = (e - 63.5) * 0.3e-3;
  G.angle.assign(5, 0.0);
  G.t0.assign(5, 0.0);
  G.g.elem_x = G.elem_x.data();
  G.g.angle_rad = G.angle.data();
  G.g.t0 = G.t0.data();
  G.g.dx = 0.15e-3;
  G.g.dz = 0.15e-3;
  G.g.apod = pwbf::kHann;
  std::string err;
  CHECK(pwbf::validate_geometry(&G.g, &err) == PWBF_OK);
  const std::string key = pwbf::shape_key(&G.g, pwbf::kF16, pwbf::kDas, -1, 0);
  pwbf_tile t = {2, 8, 2, 2, 32};
  pwbf::tune_store(key, t);
  CHECK(pwbf::tune_save(path.c_str(), &err) == PWBF_OK);
  pwbf::tune_clear();
  pwbf_tile u;
  CHECK(!pwbf::tune_lookup(key, &u));
  CHECK(pwbf::tune_load(path.c_str(), &err) == PWBF_OK);
  CHECK(pwbf::tune_lookup(key, &u) && std::memcmp(&u, &t, sizeof t) == 0);
  CHECK(pwbf::tune_load((path + ".missing").c_str(), &err) == PWBF_E_INVALID);
  for (int it = 0; it < 400; ++it) {
    FILE *f = std::fopen(path.c_str(), "w");
    CHECK(f);
    const int lines = pick(6);
    for (int l = 0; l < lines; ++l) {
      switch (pick(5)) {
        case 0: {  // the real key with a hostile tile
          pwbf_tile h = hostile_tile();
          std::fprintf(f, "  \"%s\": [%d, %d, %d, %d, %d],\n", key.c_str(), h.cpw, h.lz, h.wz,
                       h.wx, h.chunk);
          break;
        }
        case 1: {  // a very long line
          std::string s(700 + pick(2000), 'x');
          std::fprintf(f, "\"%s\": [1, 2, 3, 4, 5]\n", s.c_str());
          break;
        }
        case 2: std::fprintf(f, "  \"%s\": [%d, %d\n", key.c_str(), pick(99), pick(99)); break;
        case 3: {  // random bytes
          for (int b = 0; b < 80; ++b) std::fputc(1 + pick(255), f);
          std::fputc('\n', f);
          break;
        }
        default: std::fprintf(f, "  \"%s\": [99999999999, -2147483648, 0, 0, 0]\n", key.c_str());
      }
    }
    std::fclose(f);
    pwbf::tune_clear();
    err.clear();
    CHECK(pwbf::tune_load(path.c_str(), &err) == PWBF_OK);
    pwbf::FramePlan P;
    std::memset(&P, 0, sizeof P);
    // the tuned entry is ignored unless it fits: the default plan still comes out
    CHECK(pwbf::plan_frame(&G.g, pwbf::kF16, pwbf::kDas, -1, nullptr, &P, &err, 0) == PWBF_OK);
    check_plan(G.g, P, pwbf::kDas, -1, 0);
  }
  pwbf::tune_clear();
  std::remove(path.c_str());
  std::puts("ok tune");
}

}  // namespace

// One angle's records start at angle x channels x (the plan's record length)
// entries: n_samples for RF, n_samples / D for IQ records decimated by D.
void check_single_angle_offsets() {
  int checked = 0, decimated = 0;
  for (int it = 0; it < 4000 && checked < 300; ++it) {
    Geo G = make_geo(false);
    pwbf_geometry &g = G.g;
    const bool iq = chance(0.5);
    const int D = iq ? 1 << pick(3) : 1;
    g.iq_decimation = D;
    const int mode = iq ? (chance(0.5) ? pwbf::kIqdas : pwbf::kBbdmas) : pwbf::kDas;
    const int dtype = iq ? pwbf::kC32 : pwbf::kF32;
    const int angle = pick(g.n_angles);
    alignas(16) static float plane[4];
    alignas(16) static char base[16];
    pwbf_outputs o;
    std::memset(&o, 0, sizeof o);
    o.rf = plane;
    pwbf::FramePlan P;
    std::string err;
    if (pwbf::build_plan(&g, base, dtype, mode, angle, nullptr, &o, nullptr, 0, &P, &err) !=
        PWBF_OK)
      continue;
    const int rec = g.n_samples / D;
    CHECK(P.n_samples == rec);
    CHECK((const char *)P.rf == base + (size_t)angle * g.n_channels * rec * (iq ? 8 : 4));
    ++checked;
    decimated += D > 1 && angle > 0;
  }
  CHECK(checked >= 100 && decimated >= 20);
}

int main(int argc, char **argv) {
  const int iters = argc > 1 ? std::atoi(argv[1]) : 20000;
  const char *dir = argc > 2 ? argv[2] : ".";
  fuzz_plans(iters);
  fuzz_tune(dir);
  check_single_angle_offsets();
  std::puts("all ok");
  return 0;
}
