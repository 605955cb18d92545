// Serving loop: continuous batching of frame requests over probes whose RF ring
// slots and output planes stay resident in HBM.
//
// Threads: callers submit / poll / release (host state only, under the mutex);
// one scheduler thread makes every HIP call; completion callbacks enqueued with
// hipLaunchHostFunc stamp finished requests (host state only). The scheduler
// never holds the mutex while it calls into HIP, so a callback waiting for the
// mutex cannot block a HIP call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/pwbf.h"
#include "frame_max.h"
#include "plan_host.h"
#include "serve.h"

namespace pwbf {
int api_set_error(int code, const std::string &msg);
void api_clear_error();
}  // namespace pwbf

using pwbf::api_set_error;

namespace {

struct GeomCopy {  // a probe's geometry with its own arrays
  pwbf_geometry g;
  std::vector<double> elem_x, angle, t0;
  void set(const pwbf_geometry &src) {
    g = src;
    elem_x.assign(src.elem_x, src.elem_x + src.n_channels);
    angle.assign(src.angle_rad, src.angle_rad + src.n_angles);
    g.elem_x = elem_x.data();
    g.angle_rad = angle.data();
    if (src.t0) {
      t0.assign(src.t0, src.t0 + src.n_angles);
      g.t0 = t0.data();
    }
  }
};

struct Probe {
  GeomCopy geom;
  int mode = 0, angle = -1, want_env = 0, want_log = 0;
  size_t rf_elems = 0, slot_bytes = 0;
  int tiles = 0, cols = 0, log_cols = 0;
  double tile_cost = 0;
  std::deque<uint64_t> queue;
  std::vector<int> free_slots;
};

struct Slot {
  int probe = 0;
  void *rf = nullptr;  // FP16 RF (int16 is uploaded here and converted in place)
  float *out_rf = nullptr, *env = nullptr, *logimg = nullptr;
  unsigned char *ws = nullptr;
  hipEvent_t uploaded = nullptr;
};

enum State { kQueued, kAdmitted, kRunning, kDone };

struct Request {
  uint64_t id;
  int probe, slot = -1;
  const int16_t *host;
  double t_arrival, t_admit = 0, t_launch = 0, t_done = 0;
  State state = kQueued;
};

}  // namespace

struct pwbf_server {
  std::chrono::steady_clock::time_point t0;
  std::vector<Probe> probes;
  std::vector<Slot> slots;
  pwbf::FramePlan *d_plans = nullptr;
  pwbf::PostPlan *d_post = nullptr;
  int *d_counter = nullptr;           // one work counter per tile class
  std::vector<int> plan_class;        // tile class of each slot's plan
  int class_blocks[pwbf::kTileClasses] = {};  // persistent blocks per class
  hipStream_t copy_s = nullptr, comp_s = nullptr;
  int device = 0, lds = 0, max_nz = 0;
  size_t budget = 0, in_use = 0, peak = 0;
  int max_queue = 1024;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  bool stop = false;
  std::thread worker;
  uint64_t next_id = 1;
  std::unordered_map<uint64_t, Request> reqs;
  std::vector<uint64_t> admitted;  // upload enqueued, not yet in a batch
  std::deque<uint64_t> done;       // completed, not yet polled
  int inflight = 0;
  int rr = 0;  // round-robin start for admission
  int64_t submitted = 0, rejected = 0, completed = 0, batches = 0, batched_reqs = 0;
  std::string worker_error;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

struct CallbackArg {
  pwbf_server *s;
  std::vector<uint64_t> ids;
};

void on_batch_done(void *p) {
  std::unique_ptr<CallbackArg> a((CallbackArg *)p);
  pwbf_server *s = a->s;
  const double t = s->now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (uint64_t id : a->ids) {
      Request &r = s->reqs[id];
      r.t_done = t;
      r.state = kDone;
      s->done.push_back(id);
    }
    s->completed += (int64_t)a->ids.size();
    s->inflight -= 1;
  }
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

void fail_worker(pwbf_server *s, const std::string &msg) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->worker_error.empty()) s->worker_error = msg;
  s->stop = true;
  s->cv_done.notify_all();
}

void scheduler(pwbf_server *s) {
  if (hipSetDevice(s->device) != hipSuccess) return fail_worker(s, "hipSetDevice failed");
  while (true) {
    struct Upload {
      uint64_t id;
      int slot;
      const int16_t *host;
    };
    std::vector<Upload> uploads;
    std::vector<std::pair<uint64_t, int>> candidates;  // admitted: (id, slot)
    bool can_launch = false;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      if (s->stop) return;
      // admission: round robin over probes, FIFO within a probe, while a slot
      // is free and the budget ledger allows the slot's bytes
      const int np = (int)s->probes.size();
      bool any = true;
      while (any) {
        any = false;
        for (int k = 0; k < np; ++k) {
          Probe &p = s->probes[(s->rr + k) % np];
          if (p.queue.empty() || p.free_slots.empty()) continue;
          if (s->budget && s->in_use + p.slot_bytes > s->budget) continue;
          const uint64_t id = p.queue.front();
          p.queue.pop_front();
          const int slot = p.free_slots.back();
          p.free_slots.pop_back();
          s->in_use += p.slot_bytes;
          s->peak = std::max(s->peak, s->in_use);
          Request &r = s->reqs[id];
          r.slot = slot;
          r.t_admit = s->now();
          r.state = kAdmitted;
          uploads.push_back({id, slot, r.host});
          any = true;
        }
      }
      s->rr = (s->rr + 1) % std::max(1, np);
      for (const Upload &u : uploads) s->admitted.push_back(u.id);
      can_launch = s->inflight < 2 && !s->admitted.empty();
      if (can_launch)
        for (uint64_t id : s->admitted) candidates.push_back({id, s->reqs[id].slot});
      if (uploads.empty() && !can_launch) {
        s->cv_work.wait_for(lk, std::chrono::microseconds(200));
        continue;
      }
    }
    // uploads: int16 host RF into the slot, converted to FP16 in place
    for (const Upload &u : uploads) {
      Slot &sl = s->slots[u.slot];
      const Probe &p = s->probes[sl.probe];
      hipError_t e = hipMemcpyAsync(sl.rf, u.host, p.rf_elems * sizeof(int16_t),
                                    hipMemcpyHostToDevice, s->copy_s);
      if (e == hipSuccess) e = pwbf::launch_i16_to_f16(sl.rf, p.rf_elems, s->copy_s);
      if (e == hipSuccess) e = hipEventRecord(sl.uploaded, s->copy_s);
      if (e != hipSuccess) return fail_worker(s, std::string("upload: ") + hipGetErrorString(e));
    }
    if (!can_launch) continue;
    // continuous batching: every admitted request whose upload has finished
    // joins this batch; with nothing on the GPU, the oldest one starts a batch
    // even if its upload is still running (the stream waits for it)
    std::vector<std::pair<uint64_t, int>> ready;
    for (const auto &c : candidates) {
      if ((int)ready.size() >= pwbf::kServeMaxActive) break;
      if (hipEventQuery(s->slots[c.second].uploaded) == hipSuccess) ready.push_back(c);
    }
    int inflight_now;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      inflight_now = s->inflight;
    }
    if (ready.empty() && inflight_now == 0 && !candidates.empty()) ready.push_back(candidates[0]);
    if (ready.empty()) {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait_for(lk, std::chrono::microseconds(50));
      continue;
    }
    // slots with the costliest tiles first
    std::stable_sort(ready.begin(), ready.end(), [&](const auto &a, const auto &b) {
      return s->probes[s->slots[a.second].probe].tile_cost >
             s->probes[s->slots[b.second].probe].tile_cost;
    });
    pwbf::ActiveList al;
    std::memset(&al, 0, sizeof al);
    al.n = (int)ready.size();
    for (int k = 0; k < al.n; ++k) {
      const Probe &p = s->probes[s->slots[ready[k].second].probe];
      al.plan[k] = ready[k].second;
      al.tile0[k + 1] = al.tile0[k] + p.tiles;
      al.col0[k + 1] = al.col0[k] + p.cols;
      al.log0[k + 1] = al.log0[k] + p.log_cols;
    }
    auto *arg = new CallbackArg{s, {}};
    for (const auto &r : ready) arg->ids.push_back(r.first);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      const double t = s->now();
      for (uint64_t id : arg->ids) {
        Request &r = s->reqs[id];
        r.t_launch = t;
        r.state = kRunning;
      }
      auto &adm = s->admitted;
      adm.erase(std::remove_if(adm.begin(), adm.end(),
                               [&](uint64_t id) { return s->reqs[id].state == kRunning; }),
                adm.end());
      s->inflight += 1;
      s->batches += 1;
      s->batched_reqs += al.n;
    }
    hipError_t e = hipSuccess;
    for (const auto &r : ready)
      if (e == hipSuccess) e = hipStreamWaitEvent(s->comp_s, s->slots[r.second].uploaded, 0);
    if (e == hipSuccess)
      e = pwbf::launch_serve(s->d_plans, s->d_post, al, s->plan_class.data(), s->class_blocks,
                             s->d_counter, s->lds, s->max_nz, s->comp_s);
    if (e == hipSuccess) e = hipLaunchHostFunc(s->comp_s, on_batch_done, arg);
    if (e != hipSuccess) {
      delete arg;
      return fail_worker(s, std::string("batch launch: ") + hipGetErrorString(e));
    }
  }
}

// device bytes of one ring slot: FP16 RF, the output planes, the frame maximum's slots
size_t slot_bytes(const pwbf_probe &p) {
  const pwbf_geometry &g = *p.geom;
  const size_t plane = (size_t)g.nx * g.nz * sizeof(float);
  const int planes = 1 + ((p.want_env || p.want_log) ? 1 : 0) + (p.want_log ? 1 : 0);
  return (size_t)g.n_angles * g.n_channels * g.n_samples * 2 + planes * plane +
         pwbf::kMaxSlotBytes;
}

void free_server(pwbf_server *s) {
  if (!s) return;
  for (Slot &sl : s->slots) {
    (void)hipFree(sl.rf);
    (void)hipFree(sl.out_rf);
    (void)hipFree(sl.env);
    (void)hipFree(sl.logimg);
    (void)hipFree(sl.ws);
    if (sl.uploaded) (void)hipEventDestroy(sl.uploaded);
  }
  (void)hipFree(s->d_plans);
  (void)hipFree(s->d_post);
  (void)hipFree(s->d_counter);
  if (s->copy_s) (void)hipStreamDestroy(s->copy_s);
  if (s->comp_s) (void)hipStreamDestroy(s->comp_s);
  delete s;
}

}  // namespace

extern "C" {

int pwbf_server_create(const pwbf_probe *probes, int32_t n, size_t hbm_budget_bytes,
                       int32_t max_queue, pwbf_server **out) {
  pwbf::api_clear_error();
  if (!out) return api_set_error(PWBF_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!probes || n < 1) return api_set_error(PWBF_E_INVALID, "need n >= 1 probes");
  if (max_queue < 0) return api_set_error(PWBF_E_INVALID, "max_queue must be >= 0");
  std::string err;
  // validate every probe on the host first
  for (int i = 0; i < n; ++i) {
    const pwbf_probe &p = probes[i];
    if (p.reserved || p.slots < 0 || p.slots > 64 || (p.want_env != 0 && p.want_env != 1) ||
        (p.want_log != 0 && p.want_log != 1))
      return api_set_error(PWBF_E_INVALID, "probe " + std::to_string(i) +
                                               ": slots 0..64, want_* 0/1, reserved 0");
    if (pwbf::is_iq_mode(p.mode))
      return api_set_error(PWBF_E_UNSUPPORTED,
                           "probe " + std::to_string(i) + ": the IQ modes are single-frame only");
    pwbf::FramePlan P;
    int rc = pwbf::plan_frame(p.geom, pwbf::kF16, p.mode, p.angle, nullptr, &P, &err,
                              pwbf::serve_waves());
    if (rc) return api_set_error(rc, "probe " + std::to_string(i) + ": " + err);
    if (P.n_angles > pwbf::serve_max_angles())
      return api_set_error(PWBF_E_UNSUPPORTED, "probe " + std::to_string(i) + ": at most " +
                                                   std::to_string(pwbf::serve_max_angles()) +
                                                   " angles are summed per frame");
    if ((p.want_env || p.want_log || p.geom->bandpass)) {
      pwbf_outputs o = {(float *)256, nullptr, (float *)256, p.want_log ? (float *)256 : nullptr,
                        nullptr};
      static unsigned char fake_ws[pwbf::kMaxSlotBytes] __attribute__((aligned(256)));
      rc = pwbf::validate_outputs(p.geom, &o, fake_ws, sizeof fake_ws, &err);
      if (rc) return api_set_error(rc, "probe " + std::to_string(i) + ": " + err);
    }
  }
  for (int i = 0; i < n; ++i)
    if (hbm_budget_bytes && slot_bytes(probes[i]) > hbm_budget_bytes)
      return api_set_error(PWBF_E_INVALID, "probe " + std::to_string(i) + ": one slot needs " +
                                               std::to_string(slot_bytes(probes[i])) +
                                               " bytes, more than the HBM budget");
  pwbf_server *s = new pwbf_server();
  s->t0 = std::chrono::steady_clock::now();
  s->budget = hbm_budget_bytes;
  s->max_queue = max_queue ? max_queue : 1024;
  s->probes.resize(n);
  std::vector<pwbf::FramePlan> plans;
  std::vector<pwbf::PostPlan> post;
  hipError_t e = hipSuccess;
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    const pwbf_probe &pp = probes[i];
    Probe &p = s->probes[i];
    p.geom.set(*pp.geom);
    p.mode = pp.mode;
    p.angle = pp.angle;
    p.want_log = pp.want_log;
    p.want_env = pp.want_env || pp.want_log;
    const pwbf_geometry &g = p.geom.g;
    p.rf_elems = (size_t)g.n_angles * g.n_channels * g.n_samples;
    const size_t plane = (size_t)g.nx * g.nz * sizeof(float);
    const int nslots = pp.slots ? pp.slots : 4;
    p.slot_bytes = slot_bytes(pp);
    for (int k = 0; k < nslots && e == hipSuccess; ++k) {
      const int idx = (int)s->slots.size();
      s->slots.emplace_back();  // owned by the server from here, freed on any failure
      Slot &sl = s->slots.back();
      sl.probe = i;
      e = hipMalloc(&sl.rf, p.rf_elems * 2);
      if (e == hipSuccess) e = hipMalloc((void **)&sl.out_rf, plane);
      if (e == hipSuccess && p.want_env) e = hipMalloc((void **)&sl.env, plane);
      if (e == hipSuccess && p.want_log) e = hipMalloc((void **)&sl.logimg, plane);
      // the frame maximum's slots (the envelope is a slot plane)
      if (e == hipSuccess) e = hipMalloc((void **)&sl.ws, pwbf::kMaxSlotBytes);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.uploaded, hipEventDisableTiming);
      if (e != hipSuccess) break;
      const pwbf_outputs o = {sl.out_rf, nullptr, sl.env, sl.logimg, nullptr};
      pwbf::FramePlan P;
      pwbf::PostPlan Q;
      std::memset(&Q, 0, sizeof Q);
      int rc = pwbf::plan_frame(&g, pwbf::kF16, pp.mode, pp.angle, nullptr, &P, &err,
                                pwbf::serve_waves());
      if (rc) {
        free_server(s);
        return api_set_error(rc, err);
      }
      const size_t slab = (size_t)g.n_channels * g.n_samples * 2;
      P.rf = (const char *)sl.rf + (size_t)(pp.angle < 0 ? 0 : pp.angle) * slab;
      P.out = sl.out_rf;
      P.ws_max = nullptr;
      if (pwbf::post_needed(&o)) pwbf::build_post_plan(&g, &o, sl.ws, &Q);
      p.tiles = P.n_tiles;
      p.cols = pwbf::post_needed(&o) ? g.nx : 0;
      p.log_cols = p.want_log ? g.nx : 0;
      if (k == 0)  // its deepest (first-run) tile row holds the costliest tiles
        for (int t = 0; t < P.n_tiles; ++t) p.tile_cost = std::max(p.tile_cost, pwbf::tile_cost(&g, P, t));
      s->lds = std::max(s->lds, (int)pwbf::plan_lds_bytes(P));
      if (pwbf::post_needed(&o)) s->max_nz = std::max(s->max_nz, g.nz);
      p.free_slots.insert(p.free_slots.begin(), idx);
      plans.push_back(P);
      post.push_back(Q);
    }
  }
  int n_cu = 0;
  if (e == hipSuccess) e = hipGetDevice(&s->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, s->device);
  for (const pwbf::FramePlan &P : plans) {
    const int c = pwbf::tile_class(P.mode, P.cpw == 1, P.n_angles);
    s->plan_class.push_back(c);
    int bpc = 0;
    if (e == hipSuccess && !s->class_blocks[c]) {
      e = pwbf::serve_occupancy(c, (size_t)s->lds, &bpc);
      s->class_blocks[c] = std::max(1, bpc) * std::max(1, n_cu);
    }
  }
  if (e == hipSuccess) e = hipMalloc((void **)&s->d_plans, plans.size() * sizeof(pwbf::FramePlan));
  if (e == hipSuccess) e = hipMalloc((void **)&s->d_post, post.size() * sizeof(pwbf::PostPlan));
  if (e == hipSuccess) e = hipMalloc((void **)&s->d_counter, sizeof(int) * pwbf::kTileClasses);
  if (e == hipSuccess)
    e = hipMemcpy(s->d_plans, plans.data(), plans.size() * sizeof(pwbf::FramePlan),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(s->d_post, post.data(), post.size() * sizeof(pwbf::PostPlan),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->copy_s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->comp_s, hipStreamNonBlocking);
  if (e != hipSuccess) {
    free_server(s);
    return api_set_error(PWBF_E_NOMEM, std::string("server allocation: ") + hipGetErrorString(e));
  }
  s->worker = std::thread(scheduler, s);
  *out = s;
  return PWBF_OK;
}

int pwbf_server_submit(pwbf_server *s, int32_t probe, const int16_t *host_rf, double t_arrival,
                       uint64_t *id) {
  pwbf::api_clear_error();
  if (!s || !host_rf) return api_set_error(PWBF_E_INVALID, "server or host_rf is NULL");
  uint64_t rid;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->worker_error.empty()) return api_set_error(PWBF_E_DEVICE, s->worker_error);
    if (probe < 0 || probe >= (int)s->probes.size())
      return api_set_error(PWBF_E_INVALID, "probe index out of range");
    Probe &p = s->probes[probe];
    s->submitted += 1;
    if ((int)p.queue.size() >= s->max_queue) {
      s->rejected += 1;
      return api_set_error(PWBF_E_BUSY, "probe queue full");
    }
    rid = s->next_id++;
    Request r;
    r.id = rid;
    r.probe = probe;
    r.host = host_rf;
    r.t_arrival = t_arrival < 0 ? s->now() : t_arrival;
    s->reqs.emplace(rid, r);
    p.queue.push_back(rid);
  }
  s->cv_work.notify_one();
  if (id) *id = rid;
  return PWBF_OK;
}

int pwbf_server_poll(pwbf_server *s, pwbf_result *results, int32_t max, int32_t *n,
                     int32_t wait_ms) {
  pwbf::api_clear_error();
  if (!s || !results || !n || max < 1) return api_set_error(PWBF_E_INVALID, "bad poll arguments");
  *n = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms),
                        [&] { return !s->done.empty() || !s->worker_error.empty(); });
  if (!s->worker_error.empty() && s->done.empty())
    return api_set_error(PWBF_E_DEVICE, s->worker_error);
  while (!s->done.empty() && *n < max) {
    const Request &r = s->reqs[s->done.front()];
    s->done.pop_front();
    const Slot &sl = s->slots[r.slot];
    pwbf_result &o = results[(*n)++];
    o.id = r.id;
    o.probe = r.probe;
    o.slot = r.slot;
    o.t_arrival = r.t_arrival;
    o.t_admit = r.t_admit;
    o.t_launch = r.t_launch;
    o.t_done = r.t_done;
    o.rf = sl.out_rf;
    o.env = sl.env;
    o.logimg = sl.logimg;
  }
  return PWBF_OK;
}

int pwbf_server_release(pwbf_server *s, uint64_t id) {
  pwbf::api_clear_error();
  if (!s) return api_set_error(PWBF_E_INVALID, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || it->second.state != kDone)
      return api_set_error(PWBF_E_INVALID, "no completed request with that id");
    Probe &p = s->probes[it->second.probe];
    p.free_slots.push_back(it->second.slot);
    s->in_use -= p.slot_bytes;
    s->reqs.erase(it);
  }
  s->cv_work.notify_one();
  return PWBF_OK;
}

int pwbf_server_stats_get(pwbf_server *s, pwbf_server_stats *st) {
  pwbf::api_clear_error();
  if (!s || !st) return api_set_error(PWBF_E_INVALID, "server or stats is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  st->submitted = s->submitted;
  st->rejected = s->rejected;
  st->completed = s->completed;
  st->batches = s->batches;
  int64_t q = 0;
  for (const Probe &p : s->probes) q += (int64_t)p.queue.size();
  st->queued = q;
  st->in_flight = (int64_t)s->reqs.size() - q - (int64_t)s->done.size();
  st->mean_batch = s->batches ? (double)s->batched_reqs / s->batches : 0.0;
  st->budget_bytes = s->budget;
  st->budget_in_use = s->in_use;
  st->budget_peak = s->peak;
  return PWBF_OK;
}

double pwbf_server_now(const pwbf_server *s) { return s ? s->now() : 0.0; }

int pwbf_server_destroy(pwbf_server *s) {
  pwbf::api_clear_error();
  if (!s) return PWBF_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  hipError_t e = hipStreamSynchronize(s->comp_s);
  if (e == hipSuccess) e = hipStreamSynchronize(s->copy_s);
  {
    // completion callbacks touch the server: wait until the last one has run
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait_for(lk, std::chrono::seconds(10), [&] { return s->inflight == 0; });
  }
  free_server(s);
  return e == hipSuccess ? PWBF_OK : api_set_error(PWBF_E_DEVICE, "server teardown");
}

}  // extern "C"
