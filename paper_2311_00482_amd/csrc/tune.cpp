// Process-wide tuning table: shape key -> launch shape, with JSON persistence.
//
// A shape key names everything that changes which launch shape is fastest:
// mode, storage type, angle count, channels, samples, grid size and pitches
// (in samples), steering extent, and whether the batch kernel's fixed
// 8-wavefront blocks are required.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "plan_host.h"

namespace pwbf {

namespace {
std::mutex g_mu;
std::map<std::string, pwbf_tile> g_table;
std::atomic<uint32_t> g_generation{0};  // bumped on every change of the table
}  // namespace

uint32_t tune_generation() { return g_generation.load(); }

std::string shape_key(const pwbf_geometry *g, int dtype, int mode, int angle, int waves) {
  double scale = g->fs / g->c;
  double smax = 0;
  for (int a = 0; a < g->n_angles; ++a) smax = std::max(smax, std::fabs(std::sin(g->angle_rad[a])));
  char buf[256];
  snprintf(buf, sizeof buf, "m%d_t%d_a%d_n%d_s%d_x%d_z%d_dx%.4g_dz%.4g_sin%.3g_w%d", mode, dtype,
           angle < 0 ? g->n_angles : 1, g->n_channels, g->n_samples, g->nx, g->nz,
           g->dx * scale, g->dz * scale, smax, waves);
  return buf;
}

bool tune_lookup(const std::string &key, pwbf_tile *t) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(key);
  if (it == g_table.end()) return false;
  *t = it->second;
  return true;
}

void tune_store(const std::string &key, const pwbf_tile &t) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[key] = t;
  ++g_generation;
}

int tune_save(const char *path, std::string *err) {
  std::lock_guard<std::mutex> lk(g_mu);
  FILE *f = fopen(path, "w");
  if (!f) {
    *err = std::string("cannot write ") + path;
    return PWBF_E_INVALID;
  }
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto &kv : g_table) {
    const pwbf_tile &t = kv.second;
    fprintf(f, "  \"%s\": [%d, %d, %d, %d, %d]%s\n", kv.first.c_str(), t.cpw, t.lz, t.wz, t.wx,
            t.chunk, ++i < g_table.size() ? "," : "");
  }
  fprintf(f, "}\n");
  fclose(f);
  return PWBF_OK;
}

// Reads the format written by tune_save: one "key": [5 ints] entry per line.
int tune_load(const char *path, std::string *err) {
  FILE *f = fopen(path, "r");
  if (!f) {
    *err = std::string("cannot read ") + path;
    return PWBF_E_INVALID;
  }
  char line[512];
  std::map<std::string, pwbf_tile> add;
  while (fgets(line, sizeof line, f)) {
    char key[256];
    pwbf_tile t;
    if (sscanf(line, " \"%255[^\"]\": [%d, %d, %d, %d, %d]", key, &t.cpw, &t.lz, &t.wz, &t.wx,
               &t.chunk) == 6)
      add[key] = t;
  }
  fclose(f);
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto &kv : add) g_table[kv.first] = kv.second;
  ++g_generation;
  return PWBF_OK;
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  ++g_generation;
}

}  // namespace pwbf
