// Process-wide tuning table: shape key -> launch shape, with JSON persistence,
// and the library's two environment switches.
//
// A shape key names everything that changes which launch shape is fastest:
// mode, storage type, angle count, channels, samples, grid size and pitches
// (in samples), steering extent, and whether the batch kernel's fixed
// 8-wavefront blocks are required.
//
// PWBF_TUNE_CACHE=<path>: the table starts from that file (when it exists)
// and every shape the tuner measures is written back to it at once, so tuned
// shapes survive the process. PWBF_DEBUG=1: each launch shape the planner picks
// and each error a call returns are printed to stderr.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
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
std::once_flag g_env_once;
std::string g_cache_path;  // PWBF_TUNE_CACHE, empty when unset

int load_locked(const char *path, std::string *err);
int save_locked(const char *path, std::string *err);

void env_init() {
  std::call_once(g_env_once, [] {
    const char *p = std::getenv("PWBF_TUNE_CACHE");
    if (!p || !*p) return;
    g_cache_path = p;
    std::string err;
    std::lock_guard<std::mutex> lk(g_mu);
    if (FILE *f = std::fopen(p, "r")) {  // a missing file is a cache not yet written
      std::fclose(f);
      if (load_locked(p, &err)) debug_log("tune cache %s not read: %s", p, err.c_str());
      else debug_log("tune cache %s: %zu shapes", p, g_table.size());
    }
  });
}
}  // namespace

bool debug_enabled() {
  static const bool on = [] {
    const char *d = std::getenv("PWBF_DEBUG");
    return d && *d && std::strcmp(d, "0") != 0;
  }();
  return on;
}

void debug_log(const char *fmt, ...) {
  if (!debug_enabled()) return;
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "pwbf: %s\n", buf);
}

const std::string &tune_cache_path() {
  env_init();
  return g_cache_path;
}

uint32_t tune_generation() {
  env_init();
  return g_generation.load();
}

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
  env_init();
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_table.find(key);
  if (it == g_table.end()) return false;
  *t = it->second;
  return true;
}

void tune_store(const std::string &key, const pwbf_tile &t) {
  env_init();
  std::lock_guard<std::mutex> lk(g_mu);
  g_table[key] = t;
  ++g_generation;
  if (!g_cache_path.empty()) {
    // written to a side file and renamed, so a reader never sees half a table
    const std::string tmp = g_cache_path + ".tmp";
    std::string err;
    if (save_locked(tmp.c_str(), &err) || std::rename(tmp.c_str(), g_cache_path.c_str()))
      debug_log("tune cache %s not written: %s", g_cache_path.c_str(),
                err.empty() ? "rename failed" : err.c_str());
  }
}

int tune_save(const char *path, std::string *err) {
  env_init();
  std::lock_guard<std::mutex> lk(g_mu);
  return save_locked(path, err);
}

namespace {

int save_locked(const char *path, std::string *err) {
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
int load_locked(const char *path, std::string *err) {
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
  for (const auto &kv : add) g_table[kv.first] = kv.second;
  ++g_generation;
  return PWBF_OK;
}

}  // namespace

int tune_load(const char *path, std::string *err) {
  env_init();
  std::lock_guard<std::mutex> lk(g_mu);
  return load_locked(path, err);
}

void tune_clear() {
  env_init();
  std::lock_guard<std::mutex> lk(g_mu);
  g_table.clear();
  ++g_generation;
}

}  // namespace pwbf
