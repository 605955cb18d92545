// Batches (one persistent, graph-captured launch over uneven frames) and the
// launch-shape tuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pwbf.h"
#include "batch.h"
#include "plan_host.h"

namespace pwbf {
hipError_t launch_beamform(const FramePlan &P, hipStream_t stream);
int api_set_error(int code, const std::string &msg);
void api_clear_error();
}  // namespace pwbf

using pwbf::api_set_error;

struct pwbf_batch {
  int n = 0;
  std::vector<pwbf::FramePlan> plans;  // host copies of the device tables
  std::vector<pwbf::PostPlan> post;
  std::vector<std::string> sig;  // per-frame shape signature (update must match)
  pwbf::FramePlan *d_plans = nullptr;
  pwbf::PostPlan *d_post = nullptr;
  int4 *d_items = nullptr;  // (frame, tile, channel hull lo, hi)
  std::vector<int4> items;  // host copy (the hulls follow the frames' geometry)
  int2 *d_post_cols = nullptr, *d_log_cols = nullptr;
  std::vector<pwbf::BatchClass> classes;  // every branch's class launches, branch by branch
  struct Branch {
    int class_first = 0, class_n = 0;
    int post_first = 0, post_n = 0, log_first = 0, log_n = 0;
    double cost = 0;
  };
  std::vector<Branch> branches;
  std::vector<hipStream_t> fork_streams;  // used only while capturing the graph
  std::vector<hipEvent_t> fork_events;
  unsigned char *d_ws = nullptr;  // per-frame workspaces (envelope maximum, envelope plane)
  std::vector<size_t> ws_off;
  void *h_stage = nullptr;  // pinned staging of the descriptor tables for updates
  hipEvent_t staged = nullptr;
  bool stage_pending = false;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int n_items = 0, n_post_cols = 0, n_log_cols = 0, blocks = 0, blocks_per_cu = 0;
  int lds = 0, max_nz = 0, graph_nodes = 0;
};

namespace {

// Graph branches of a batch: they run side by side only while each has a
// hardware queue of its own, and the process's queues (four by default) also
// serve the launching stream, so the default is three. PWBF_BATCH_BRANCHES
// (1..4) overrides it when the batch is created.
constexpr int kMaxBranches = 4;
int branch_limit() {
  const char *v = getenv("PWBF_BATCH_BRANCHES");
  const int k = v ? atoi(v) : 3;
  return k >= 1 && k <= kMaxBranches ? k : 3;
}

int dev_error(hipError_t e, const char *what) {
  return api_set_error(PWBF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool tile_is_zero(const pwbf_tile &t) { return !t.cpw && !t.lz && !t.wz && !t.wx && !t.chunk; }

// Everything of a frame that a batch's graph and work list depend on.
std::string frame_signature(const pwbf_frame &f, const pwbf::FramePlan &P) {
  char buf[512];
  snprintf(buf, sizeof buf, "%s|a%d|t%d|%d%d%d|tile%d.%d.%d.%d.%d|win%d|bp%d|nz%d",
           pwbf::shape_key(f.geom, f.rf_dtype, f.mode, f.angle, 8).c_str(), f.angle, f.rf_dtype,
           f.out.filtered != nullptr, f.out.env != nullptr, f.out.logimg != nullptr, P.cpw, P.lz,
           P.wz, P.wx, P.chunk, P.win, f.geom->bandpass, f.geom->nz);
  return buf;
}

// Plan one batch frame (8-wavefront tiles) with its pointers and workspace.
int plan_batch_frame(const pwbf_frame &f, unsigned char *ws, pwbf::FramePlan *P,
                     pwbf::PostPlan *Q, std::string *err) {
  if (f.reserved != 0) {
    *err = "pwbf_frame.reserved must be 0";
    return PWBF_E_INVALID;
  }
  const pwbf_tile *t = tile_is_zero(f.tile) ? nullptr : &f.tile;
  if (pwbf::is_iq_mode(f.mode)) {
    *err = "the IQ modes are single-frame only";
    return PWBF_E_UNSUPPORTED;
  }
  int rc = pwbf::plan_frame(f.geom, f.rf_dtype, f.mode, f.angle, t, P, err, pwbf::batch_waves());
  if (rc) return rc;
  if (P->n_angles > pwbf::batch_max_angles()) {
    *err = "batch frames sum at most " + std::to_string(pwbf::batch_max_angles()) + " angles";
    return PWBF_E_UNSUPPORTED;
  }
  if (!f.rf) {
    *err = "frame rf is NULL";
    return PWBF_E_INVALID;
  }
  if ((uintptr_t)f.rf % pwbf::dtype_bytes(f.rf_dtype)) {
    *err = "frame rf not aligned to its element size";
    return PWBF_E_INVALID;
  }
  size_t need = pwbf::workspace_bytes(f.geom, &f.out);
  rc = pwbf::validate_outputs(f.geom, &f.out, need ? ws : nullptr, need, err);
  if (rc) return rc;
  const size_t slab =
      (size_t)f.geom->n_channels * f.geom->n_samples * pwbf::dtype_bytes(f.rf_dtype);
  P->rf = (const char *)f.rf + (size_t)(f.angle < 0 ? 0 : f.angle) * slab;
  P->out = f.out.rf;
  P->ws_max = nullptr;  // cleared by the batch reset kernel instead
  std::memset(Q, 0, sizeof *Q);
  if (pwbf::post_needed(&f.out)) pwbf::build_post_plan(f.geom, &f.out, ws, Q);
  return PWBF_OK;
}

// Release everything a batch holds; errors on the way are not actionable here
// (best-effort teardown), so their codes are dropped explicitly.
void free_batch(pwbf_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (hipStream_t st : b->fork_streams) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : b->fork_events) (void)hipEventDestroy(ev);
  if (b->staged) (void)hipEventDestroy(b->staged);
  if (b->h_stage) (void)hipHostFree(b->h_stage);
  (void)hipFree(b->d_plans);
  (void)hipFree(b->d_post);
  (void)hipFree(b->d_items);
  (void)hipFree(b->d_post_cols);
  (void)hipFree(b->d_log_cols);
  (void)hipFree(b->d_ws);
  delete b;
}

template <class T>
hipError_t upload(T **dst, const std::vector<T> &src) {
  if (src.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void **)dst, src.size() * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
}

}  // namespace

extern "C" {

int pwbf_tune(const pwbf_geometry *g, const void *rf, int32_t rf_dtype, int32_t mode,
              int32_t angle, const pwbf_outputs *out, int32_t waves, void *stream,
              pwbf_tile *best, float *best_ms) {
  pwbf::api_clear_error();
  if (waves != 0 && waves != pwbf::batch_waves())
    return api_set_error(PWBF_E_INVALID, "waves must be 0 or 8");
  if (!out || !out->rf) return api_set_error(PWBF_E_INVALID, "out->rf is required as scratch");
  const pwbf_outputs rf_only = {out->rf, nullptr, nullptr, nullptr, nullptr};
  out = &rf_only;
  pwbf::FramePlan P;
  std::string err;
  // validates geometry, pointers and the default plan before anything runs
  int rc = pwbf::build_plan(g, rf, rf_dtype, mode, angle, nullptr, out, nullptr, 0, &P, &err);
  if (rc) return api_set_error(rc, err);
  hipStream_t s = (hipStream_t)stream;
  // the shape this frame plans with now (it fits, so tuning never fails where
  // planning succeeds), then a fixed grid of lane groupings, lane-group
  // depths from 2 to 32 and wavefront arrangements
  std::vector<pwbf_tile> cands = {{P.cpw, P.lz, P.wz, P.wx, 0}};
  // DMAS and pDAS: only shapes within their delay-offset bound, when the
  // frame's own plan (of the required wavefront count) shows that one is
  bool compact_only = pwbf::root_compact(g, P);
  if (waves) {
    pwbf::FramePlan W;
    std::string e2;
    compact_only = false;
    if (pwbf::plan_frame(g, rf_dtype, mode, angle, nullptr, &W, &e2, waves) == PWBF_OK) {
      cands.insert(cands.begin(), {W.cpw, W.lz, W.wz, W.wx, 0});
      compact_only = pwbf::root_compact(g, W);
    }
  }
  static const int kArr[][2] = {{1, 8}, {2, 4}, {4, 2}, {8, 1}, {1, 4}};
  for (int cpw : {1, 2, 4})
    for (int lz : {2, 4, 8, 16, 32})
      for (const auto &wa : kArr) {
        if (lz > 64 / cpw) continue;
        if (waves && wa[0] * wa[1] != waves) continue;
        cands.push_back({cpw, lz, wa[0], wa[1], 0});
      }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return api_set_error(PWBF_E_DEVICE, "event creation failed");
  float best_t = 1e30f;
  pwbf_tile best_tile = {0, 0, 0, 0, 0};
  for (const pwbf_tile &t : cands) {
    pwbf::FramePlan Q;
    if (pwbf::build_plan(g, rf, rf_dtype, mode, angle, &t, out, nullptr, 0, &Q, &err)) continue;
    if (waves && Q.wz * Q.wx != waves) continue;
    if (compact_only && !pwbf::root_compact(g, Q)) continue;
    hipError_t e = pwbf::launch_beamform(Q, s);  // warm-up
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
      if (k == 0) e = hipEventRecord(e0, s);
      if (e == hipSuccess) e = pwbf::launch_beamform(Q, s);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return dev_error(e, "tuning launch");
    }
    ms /= 3;
    if (ms < best_t) {
      best_t = ms;
      best_tile = {Q.cpw, Q.lz, Q.wz, Q.wx, 0};
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (best_t >= 1e30f) return api_set_error(PWBF_E_UNSUPPORTED, "no launch shape fits");
  pwbf::tune_store(pwbf::shape_key(g, rf_dtype, mode, angle, waves), best_tile);
  if (best) *best = best_tile;
  if (best_ms) *best_ms = best_t;
  return PWBF_OK;
}

int pwbf_tune_save(const char *path) {
  pwbf::api_clear_error();
  if (!path) return api_set_error(PWBF_E_INVALID, "path is NULL");
  std::string err;
  int rc = pwbf::tune_save(path, &err);
  return rc ? api_set_error(rc, err) : PWBF_OK;
}

int pwbf_tune_load(const char *path) {
  pwbf::api_clear_error();
  if (!path) return api_set_error(PWBF_E_INVALID, "path is NULL");
  std::string err;
  int rc = pwbf::tune_load(path, &err);
  return rc ? api_set_error(rc, err) : PWBF_OK;
}

int pwbf_tune_clear(void) {
  pwbf::api_clear_error();
  pwbf::tune_clear();
  return PWBF_OK;
}

int pwbf_batch_create(const pwbf_frame *frames, int32_t n, int32_t flags, void *stream,
                      pwbf_batch **out) {
  pwbf::api_clear_error();
  if (!out) return api_set_error(PWBF_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!frames || n < 1) return api_set_error(PWBF_E_INVALID, "need n >= 1 frames");
  if (flags & ~PWBF_BATCH_TUNE) return api_set_error(PWBF_E_INVALID, "unknown flags");
  std::string err;
  // validate every frame (and its shape) before touching the device
  for (int i = 0; i < n; ++i) {
    pwbf::FramePlan P;
    pwbf::PostPlan Q;
    static unsigned char fake_ws[1] __attribute__((aligned(256)));
    int rc = plan_batch_frame(frames[i], fake_ws, &P, &Q, &err);
    if (rc) return api_set_error(rc, "frame " + std::to_string(i) + ": " + err);
  }
  hipStream_t s = (hipStream_t)stream;
  if (flags & PWBF_BATCH_TUNE) {
    for (int i = 0; i < n; ++i) {
      const pwbf_frame &f = frames[i];
      pwbf_tile t;
      if (!tile_is_zero(f.tile) ||
          pwbf::tune_lookup(pwbf::shape_key(f.geom, f.rf_dtype, f.mode, f.angle, 8), &t))
        continue;
      pwbf_outputs scratch = {f.out.rf, nullptr, nullptr, nullptr, nullptr};
      int rc = pwbf_tune(f.geom, f.rf, f.rf_dtype, f.mode, f.angle, &scratch, 8, stream,
                         nullptr, nullptr);
      if (rc) return rc;
    }
  }
  pwbf_batch *b = new pwbf_batch();
  b->n = n;
  b->plans.resize(n);
  b->post.resize(n);
  b->sig.resize(n);
  b->ws_off.resize(n);
  size_t ws_total = 0;
  for (int i = 0; i < n; ++i) {
    b->ws_off[i] = ws_total;
    ws_total += (pwbf::workspace_bytes(frames[i].geom, &frames[i].out) + 255) / 256 * 256;
  }
  hipError_t e = hipSuccess;
  if (ws_total) e = hipMalloc((void **)&b->d_ws, ws_total);
  if (e != hipSuccess) {
    free_batch(b);
    return api_set_error(PWBF_E_NOMEM, "batch workspace allocation failed");
  }
  // Plan every frame; estimate its cost (the sum of its tiles' costs).
  struct Work {
    double cost;
    int frame, tile;
  };
  std::vector<std::vector<Work>> frame_work(n);
  std::vector<double> frame_cost(n, 0.0);
  std::vector<int> cls(n);
  for (int i = 0; i < n; ++i) {
    const pwbf_frame &f = frames[i];
    unsigned char *ws = b->d_ws ? b->d_ws + b->ws_off[i] : nullptr;
    int rc = plan_batch_frame(f, ws, &b->plans[i], &b->post[i], &err);
    if (rc) {
      free_batch(b);
      return api_set_error(rc, "frame " + std::to_string(i) + ": " + err);
    }
    const pwbf::FramePlan &P = b->plans[i];
    b->sig[i] = frame_signature(f, P);
    b->lds = std::max(b->lds, (int)pwbf::plan_lds_bytes(P));
    cls[i] = pwbf::tile_class(P.mode, P.cpw == 1, P.n_angles);
    for (int t = 0; t < P.n_tiles; ++t) {
      const double c = pwbf::tile_cost(f.geom, P, t);
      frame_work[i].push_back({c, i, t});
      frame_cost[i] += c;
    }
    if (pwbf::post_needed(&f.out)) b->max_nz = std::max(b->max_nz, f.geom->nz);
  }
  // Frames go to up to kMaxBranches graph branches, longest first, each to the
  // branch with the least work so far; branches run side by side, so each
  // branch's post-processing and tail overlap the others' beamforming.
  const int n_br = std::min(n, branch_limit());
  b->branches.assign(n_br, pwbf_batch::Branch());
  std::vector<int> by_cost(n), branch_of(n);
  for (int i = 0; i < n; ++i) by_cost[i] = i;
  std::stable_sort(by_cost.begin(), by_cost.end(),
                   [&frame_cost](int a, int c) { return frame_cost[a] > frame_cost[c]; });
  for (int i : by_cost) {
    int best = 0;
    for (int k = 1; k < n_br; ++k)
      if (b->branches[k].cost < b->branches[best].cost) best = k;
    branch_of[i] = best;
    b->branches[best].cost += frame_cost[i];
  }
  // Per branch: its items grouped by class, the costliest class first and the
  // longest tiles first within a class; then its frames' columns.
  std::vector<int4> items;
  std::vector<int2> post_cols, log_cols;
  for (int k = 0; k < n_br; ++k) {
    pwbf_batch::Branch &br = b->branches[k];
    std::vector<Work> order;
    std::vector<double> class_cost(pwbf::kTileClasses, 0.0);
    for (int i = 0; i < n; ++i)
      if (branch_of[i] == k) {
        order.insert(order.end(), frame_work[i].begin(), frame_work[i].end());
        class_cost[cls[i]] += frame_cost[i];
      }
    std::stable_sort(order.begin(), order.end(), [&](const Work &a, const Work &c) {
      const int ca = cls[a.frame], cc = cls[c.frame];
      if (ca != cc) return class_cost[ca] != class_cost[cc] ? class_cost[ca] > class_cost[cc]
                                                            : ca < cc;
      return a.cost > c.cost;
    });
    br.class_first = (int)b->classes.size();
    for (size_t q = 0; q < order.size(); ++q) {
      const int c = cls[order[q].frame];
      if ((int)b->classes.size() == br.class_first || b->classes.back().cls != c)
        b->classes.push_back({c, (int)items.size(), 0, 0});
      ++b->classes.back().n;
      int lo, hi;
      pwbf::tile_channel_hull(frames[order[q].frame].geom, b->plans[order[q].frame],
                              order[q].tile, &lo, &hi);
      items.push_back(make_int4(order[q].frame, order[q].tile, lo, hi));
    }
    br.class_n = (int)b->classes.size() - br.class_first;
    br.post_first = (int)post_cols.size();
    br.log_first = (int)log_cols.size();
    for (int i = 0; i < n; ++i) {
      const pwbf_frame &f = frames[i];
      if (branch_of[i] != k || !pwbf::post_needed(&f.out)) continue;
      for (int ix = 0; ix < f.geom->nx; ++ix) post_cols.push_back(make_int2(i, ix));
      if (f.out.logimg)
        for (int ix = 0; ix < f.geom->nx; ++ix) log_cols.push_back(make_int2(i, ix));
    }
    br.post_n = (int)post_cols.size() - br.post_first;
    br.log_n = (int)log_cols.size() - br.log_first;
  }
  b->n_items = (int)items.size();
  b->items = items;
  b->n_post_cols = (int)post_cols.size();
  b->n_log_cols = (int)log_cols.size();

  int dev_id = 0, n_cu = 0;
  e = hipGetDevice(&dev_id);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev_id);
  b->blocks = 0;
  b->blocks_per_cu = 0;
  for (pwbf::BatchClass &k : b->classes) {
    int bpc = 0;
    if (e == hipSuccess) e = pwbf::batch_occupancy(k.cls, (size_t)b->lds, &bpc);
    k.blocks = k.n;  // one block per item
    b->blocks += k.blocks;
    b->blocks_per_cu = b->blocks_per_cu ? std::min(b->blocks_per_cu, bpc) : bpc;
  }
  if (e != hipSuccess) {
    free_batch(b);
    return dev_error(e, "device query");
  }

  e = upload(&b->d_plans, b->plans);
  if (e == hipSuccess) e = upload(&b->d_post, b->post);
  if (e == hipSuccess) e = upload(&b->d_items, items);
  if (e == hipSuccess) e = upload(&b->d_post_cols, post_cols);
  if (e == hipSuccess) e = upload(&b->d_log_cols, log_cols);
  if (e == hipSuccess)
    e = hipHostMalloc(&b->h_stage,
                      n * (sizeof(pwbf::FramePlan) + sizeof(pwbf::PostPlan)) +
                          items.size() * sizeof(int4),
                      hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->staged, hipEventDisableTiming);
  if (e != hipSuccess) {
    free_batch(b);
    return api_set_error(PWBF_E_NOMEM, std::string("batch tables: ") + hipGetErrorString(e));
  }
  // capture the launch sequence once: reset, fork into the branches, join
  e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  for (int k = 0; k < n_br + 1 && e == hipSuccess; ++k) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->fork_events.push_back(ev);
  }
  for (int k = 0; k < n_br && e == hipSuccess; ++k) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) b->fork_streams.push_back(st);
  }
  if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = pwbf::launch_batch_reset(b->d_post, n, b->cap);
    if (le == hipSuccess) le = hipEventRecord(b->fork_events[n_br], b->cap);
    std::vector<int> steps(n_br);
    int max_steps = 0;
    for (int k = 0; k < n_br && le == hipSuccess; ++k) {
      const pwbf_batch::Branch &br = b->branches[k];
      steps[k] = pwbf::batch_branch_steps(br.class_n, br.post_n, br.log_n);
      max_steps = std::max(max_steps, steps[k]);
      le = hipStreamWaitEvent(b->fork_streams[k], b->fork_events[n_br], 0);
    }
    // the launches are captured round robin over the branches (step 0 of each,
    // then step 1, ...): the graph enqueues its nodes in about that order, so
    // every branch starts at once instead of after the others' launches
    for (int step = 0; step < max_steps && le == hipSuccess; ++step)
      for (int k = 0; k < n_br && le == hipSuccess; ++k) {
        if (step >= steps[k]) continue;
        const pwbf_batch::Branch &br = b->branches[k];
        le = pwbf::launch_batch_branch_step(b->d_plans, b->d_post, b->d_items,
                                            b->classes.data() + br.class_first, br.class_n,
                                            b->d_post_cols + br.post_first, br.post_n,
                                            b->d_log_cols + br.log_first, br.log_n, b->lds,
                                            b->max_nz, step, b->fork_streams[k]);
      }
    for (int k = 0; k < n_br && le == hipSuccess; ++k) {
      le = hipEventRecord(b->fork_events[k], b->fork_streams[k]);
      if (le == hipSuccess) le = hipStreamWaitEvent(b->cap, b->fork_events[k], 0);
    }
    e = hipStreamEndCapture(b->cap, &b->graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e == hipSuccess) {
    size_t nodes = 0;
    e = hipGraphGetNodes(b->graph, nullptr, &nodes);
    b->graph_nodes = (int)nodes;
  }
  if (e != hipSuccess) {
    free_batch(b);
    return dev_error(e, "batch graph capture");
  }
  (void)s;
  *out = b;
  return PWBF_OK;
}

int pwbf_batch_update(pwbf_batch *b, const pwbf_frame *frames, int32_t n, void *stream) {
  pwbf::api_clear_error();
  if (!b || !frames) return api_set_error(PWBF_E_INVALID, "batch or frames is NULL");
  if (n != b->n) return api_set_error(PWBF_E_INVALID, "frame count differs from the batch");
  std::vector<pwbf::FramePlan> plans(n);
  std::vector<pwbf::PostPlan> post(n);
  std::string err;
  for (int i = 0; i < n; ++i) {
    pwbf_frame f = frames[i];
    // keep the launch shape the batch was built with
    const pwbf::FramePlan &old = b->plans[i];
    f.tile = {old.cpw, old.lz, old.wz, old.wx, old.chunk};
    unsigned char *ws = b->d_ws ? b->d_ws + b->ws_off[i] : nullptr;
    int rc = plan_batch_frame(f, ws, &plans[i], &post[i], &err);
    if (rc) return api_set_error(rc, "frame " + std::to_string(i) + ": " + err);
    if (frame_signature(frames[i], plans[i]) != b->sig[i])
      return api_set_error(PWBF_E_INVALID,
                           "frame " + std::to_string(i) + " differs in shape from the batch");
  }
  // the tiles' channel hulls follow the new geometry (element positions, grid
  // origin and F-number may differ at the same shape)
  std::vector<int4> items = b->items;
  for (int4 &it : items)
    pwbf::tile_channel_hull(frames[it.x].geom, plans[it.x], it.y, &it.z, &it.w);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  if (b->stage_pending) e = hipEventSynchronize(b->staged);  // staging buffer free again
  if (e != hipSuccess) return dev_error(e, "batch update");
  unsigned char *h = (unsigned char *)b->h_stage;
  const size_t pb = n * sizeof(pwbf::FramePlan), qb = n * sizeof(pwbf::PostPlan);
  const size_t ib = items.size() * sizeof(int4);
  std::memcpy(h, plans.data(), pb);
  std::memcpy(h + pb, post.data(), qb);
  if (ib) std::memcpy(h + pb + qb, items.data(), ib);
  e = hipMemcpyAsync(b->d_plans, h, pb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_post, h + pb, qb, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && ib)
    e = hipMemcpyAsync(b->d_items, h + pb + qb, ib, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(b->staged, s);
  if (e != hipSuccess) return dev_error(e, "batch update");
  b->stage_pending = true;
  b->plans = plans;
  b->post = post;
  b->items = items;
  return PWBF_OK;
}

int pwbf_batch_launch(pwbf_batch *b, void *stream) {
  pwbf::api_clear_error();
  if (!b) return api_set_error(PWBF_E_INVALID, "batch is NULL");
  hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
  return e == hipSuccess ? PWBF_OK : dev_error(e, "batch graph launch");
}

int pwbf_batch_describe(const pwbf_batch *b, pwbf_batch_info *info) {
  pwbf::api_clear_error();
  if (!b || !info) return api_set_error(PWBF_E_INVALID, "batch or info is NULL");
  info->n_frames = b->n;
  info->n_items = b->n_items;
  info->n_columns = b->n_post_cols;
  info->blocks = b->blocks;
  info->blocks_per_cu = b->blocks_per_cu;
  info->lds_bytes = b->lds;
  info->graph_nodes = b->graph_nodes;
  info->kernels = (int32_t)b->classes.size();
  info->branches = (int32_t)b->branches.size();
  return PWBF_OK;
}

int pwbf_batch_destroy(pwbf_batch *b) {
  pwbf::api_clear_error();
  if (!b) return PWBF_OK;
  hipError_t e = hipDeviceSynchronize();
  free_batch(b);
  return e == hipSuccess ? PWBF_OK : dev_error(e, "batch destroy");
}

}  // extern "C"
