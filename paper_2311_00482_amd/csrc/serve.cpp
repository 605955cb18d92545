// Serving loop: continuous batching of frame requests over probes whose RF ring
// slots and output planes stay resident in HBM.
//
// The decisions (request ledger, HBM budget, admission, deadlines, batching)
// live in serve::Core, which makes no device call; this file gives it a HIP
// launcher and the server clock. Threads: callers submit / poll / release
// (host state only); one scheduler thread steps the core and makes every HIP
// call; completion callbacks enqueued with hipLaunchHostFunc hand finished
// batches back to the core (host state only). The core never holds its mutex
// while the launcher calls into HIP, so a callback waiting for the mutex cannot
// block a HIP call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pwbf.h"
#include "frame_max.h"
#include "metrics.h"
#include "plan_host.h"
#include "serve.h"
#include "serve_core.h"

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
  int want_env = 0, want_log = 0, want_quality = 0;
  size_t rf_elems = 0;
  int tiles = 0, cols = 0, log_cols = 0;
};

struct Slot {
  int probe = 0;
  void *rf = nullptr;  // FP16 RF (int16 is uploaded here and converted in place)
  float *out_rf = nullptr, *env = nullptr, *logimg = nullptr;
  unsigned char *ws = nullptr;
  hipEvent_t uploaded = nullptr;
  int copy_stream = -1;     // stream of the last upload
  bool upload_pending = false;
};

class ServerClock : public pwbf::serve::Clock {
 public:
  ServerClock() : t0_(std::chrono::steady_clock::now()) {}
  double now() const override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
  }

 private:
  std::chrono::steady_clock::time_point t0_;
};

constexpr int kCopyStreams = 2;
constexpr int kQualityBlocksPerSlot = 2 * pwbf::kQualityMaxChunks;
constexpr int kInflight = pwbf::serve::Core::kMaxInflight;  // device regions: the most

// Batches on the device at once, four by default: with two, a request whose
// upload finished while two batches ran waited for one of them before its
// launch; with four it launches and waits in the device queue instead, so the
// upload leg stays the shorter part of a request's latency up to the rates
// where the device itself saturates. PWBF_SERVE_INFLIGHT (1..4) overrides it
// when a server is created.
int serve_inflight() {
  const char *v = getenv("PWBF_SERVE_INFLIGHT");
  const int k = v ? atoi(v) : kInflight;
  return k >= 1 && k <= kInflight ? k : kInflight;
}
static_assert(pwbf::serve::Core::kMaxBatch <= pwbf::kServeMaxActive, "a batch fits the list");
static_assert(pwbf::serve::Core::kMaxBatch <= pwbf::kQualityMax, "a batch fits the list");

}  // namespace

struct pwbf_server;

namespace {

class HipLauncher : public pwbf::serve::Launcher {
 public:
  explicit HipLauncher(pwbf_server *s) : s_(s) {}
  int upload(int slot, const void *host, std::string *err) override;
  bool upload_done(int slot) override;
  int launch(const pwbf::serve::Batch &batch, std::string *err) override;

 private:
  pwbf_server *s_;
  int batch_no_ = 0;
};

}  // namespace

struct pwbf_server {
  ServerClock clock;
  std::vector<Probe> probes;
  std::vector<Slot> slots;
  pwbf::FramePlan *d_plans = nullptr;
  pwbf::PostPlan *d_post = nullptr;
  pwbf::QualityPlan *d_quality = nullptr;  // per slot (unused entries zero)
  std::vector<pwbf::QualityPlan> quality;  // host copy (chunk counts per slot)
  pwbf::QualityOut *d_qout = nullptr;      // kInflight regions of kMaxBatch
  pwbf::QualityOut *h_qout = nullptr;      // pinned copies of those regions
  float4 *d_qpart = nullptr;               // kInflight regions of the checks' partials
  int *d_qcount = nullptr;                 // kInflight regions of kMaxBatch counters (zero)
  int *d_counter = nullptr;                // one work counter per tile class
  std::vector<int> plan_class;             // tile class of each slot's plan
  int class_blocks[pwbf::kTileClasses] = {};  // persistent blocks per class
  hipStream_t copy_s[kCopyStreams] = {}, comp_s = nullptr;
  int device = 0, lds = 0, max_nz = 0;
  std::unique_ptr<pwbf::serve::Core> core;
  std::unique_ptr<HipLauncher> launcher;
  std::thread worker;
};

namespace {

// The uploads of int16 frames go to the copy stream with fewer bytes still in
// flight, so a large frame does not hold back a small one behind it.
int HipLauncher::upload(int slot, const void *host, std::string *err) {
  Slot &sl = s_->slots[slot];
  const Probe &p = s_->probes[sl.probe];
  size_t pending[kCopyStreams] = {};
  for (Slot &o : s_->slots) {
    if (!o.upload_pending) continue;
    if (hipEventQuery(o.uploaded) == hipSuccess)
      o.upload_pending = false;
    else
      pending[o.copy_stream] += s_->probes[o.probe].rf_elems * sizeof(int16_t);
  }
  int cs = 0;
  for (int k = 1; k < kCopyStreams; ++k)
    if (pending[k] < pending[cs]) cs = k;
  hipStream_t st = s_->copy_s[cs];
  hipError_t e = hipMemcpyAsync(sl.rf, host, p.rf_elems * sizeof(int16_t), hipMemcpyHostToDevice,
                                st);
  if (e == hipSuccess) e = pwbf::launch_i16_to_f16(sl.rf, p.rf_elems, st);
  if (e == hipSuccess) e = hipEventRecord(sl.uploaded, st);
  if (e != hipSuccess) {
    *err = hipGetErrorString(e);
    return PWBF_E_DEVICE;
  }
  sl.copy_stream = cs;
  sl.upload_pending = true;
  return PWBF_OK;
}

bool HipLauncher::upload_done(int slot) {
  return hipEventQuery(s_->slots[slot].uploaded) == hipSuccess;
}

struct CallbackArg {
  pwbf_server *s;
  std::vector<uint64_t> ids;
  std::vector<int> qpos;  // position of each request's check in the region, or -1
  int region;
};

void on_batch_done(void *p) {
  std::unique_ptr<CallbackArg> a((CallbackArg *)p);
  // the stream ran the copy of the checks into pinned memory before this call
  std::vector<pwbf::serve::Quality> q(a->ids.size());
  const pwbf::QualityOut *h = a->s->h_qout + (size_t)a->region * pwbf::serve::Core::kMaxBatch;
  for (size_t k = 0; k < a->ids.size(); ++k) {
    if (a->qpos[k] < 0) continue;
    const pwbf::QualityOut &r = h[a->qpos[k]];
    q[k].frame_max = r.frame_max;
    q[k].cr_db = r.cr_db;
    q[k].cnr = r.cnr;
    q[k].ok = r.ok;
  }
  a->s->core->complete(a->ids, &q);
}

int HipLauncher::launch(const pwbf::serve::Batch &batch, std::string *err) {
  pwbf::ActiveList al;
  std::memset(&al, 0, sizeof al);
  pwbf::QualityList ql;
  ql.n = 0;
  ql.block0[0] = 0;
  auto arg = std::make_unique<CallbackArg>();
  arg->s = s_;
  // at most kInflight batches are on the device and they finish in order, so
  // the region of the batch kInflight launches back is free again
  arg->region = batch_no_++ % kInflight;
  al.n = (int)batch.size();
  for (int k = 0; k < al.n; ++k) {
    const int slot = batch[k].second;
    const Probe &p = s_->probes[s_->slots[slot].probe];
    al.plan[k] = slot;
    al.tile0[k + 1] = al.tile0[k] + p.tiles;
    al.col0[k + 1] = al.col0[k] + p.cols;
    al.log0[k + 1] = al.log0[k] + p.log_cols;
    arg->ids.push_back(batch[k].first);
    if (p.want_quality) {
      const pwbf::QualityPlan &qp = s_->quality[slot];
      arg->qpos.push_back(ql.n);
      ql.plan[ql.n] = slot;
      ql.block0[ql.n + 1] = ql.block0[ql.n] + qp.chunks_in + qp.chunks_out;
      ++ql.n;
    } else {
      arg->qpos.push_back(-1);
    }
  }
  hipError_t e = hipSuccess;
  for (const auto &r : batch)
    if (e == hipSuccess) e = hipStreamWaitEvent(s_->comp_s, s_->slots[r.second].uploaded, 0);
  if (e == hipSuccess)
    e = pwbf::launch_serve(s_->d_plans, s_->d_post, al, s_->plan_class.data(), s_->class_blocks,
                           s_->d_counter, s_->lds, s_->max_nz, s_->comp_s);
  if (e == hipSuccess && ql.n > 0) {
    const size_t off = (size_t)arg->region * pwbf::serve::Core::kMaxBatch;
    e = pwbf::launch_quality(s_->d_quality, ql, s_->d_qout + off,
                             s_->d_qpart + off * kQualityBlocksPerSlot, s_->d_qcount + off,
                             s_->comp_s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(s_->h_qout + off, s_->d_qout + off, ql.n * sizeof(pwbf::QualityOut),
                         hipMemcpyDeviceToHost, s_->comp_s);
  }
  if (e == hipSuccess) e = hipLaunchHostFunc(s_->comp_s, on_batch_done, arg.get());
  if (e != hipSuccess) {
    *err = hipGetErrorString(e);
    return PWBF_E_DEVICE;
  }
  arg.release();  // owned by the callback now
  return PWBF_OK;
}

void scheduler(pwbf_server *s) {
  if (hipSetDevice(s->device) != hipSuccess) return s->core->fail("hipSetDevice failed");
  while (!s->core->stopped()) {
    const auto r = s->core->step(*s->launcher);
    if (r == pwbf::serve::Core::kIdle)
      s->core->wait_for_work(200);
    else if (r == pwbf::serve::Core::kUploading)
      s->core->wait_for_work(50);
  }
}

bool wants_env(const pwbf_probe &p) { return p.want_env || p.want_log || p.want_quality; }

// device bytes of one ring slot: FP16 RF, the output planes, the frame maximum's slots
size_t slot_bytes(const pwbf_probe &p) {
  const pwbf_geometry &g = *p.geom;
  const size_t plane = (size_t)g.nx * g.nz * sizeof(float);
  const int planes = 1 + (wants_env(p) ? 1 : 0) + (p.want_log ? 1 : 0);
  return (size_t)g.n_angles * g.n_channels * g.n_samples * 2 + planes * plane +
         pwbf::kMaxSlotBytes;
}

bool finite_disc(const pwbf_disc &d) {
  return std::isfinite(d.x) && std::isfinite(d.z) && std::isfinite(d.r) && d.r > 0;
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
  (void)hipFree(s->d_quality);
  (void)hipFree(s->d_qout);
  (void)hipFree(s->d_qpart);
  (void)hipFree(s->d_qcount);
  if (s->h_qout) (void)hipHostFree(s->h_qout);
  (void)hipFree(s->d_counter);
  for (hipStream_t &c : s->copy_s)
    if (c) (void)hipStreamDestroy(c);
  if (s->comp_s) (void)hipStreamDestroy(s->comp_s);
  delete s;
}

int validate_probe(const pwbf_probe &p, int i, std::string *err) {
  auto bad = [&](int rc, const std::string &m) {
    *err = "probe " + std::to_string(i) + ": " + m;
    return rc;
  };
  auto flag = [](int32_t v) { return v == 0 || v == 1; };
  if (p.slots < 0 || p.slots > 64 || !flag(p.want_env) || !flag(p.want_log) ||
      !flag(p.want_quality))
    return bad(PWBF_E_INVALID, "slots 0..64, want_* 0/1");
  if (p.want_quality && (!finite_disc(p.quality_region.in) || !finite_disc(p.quality_region.out) ||
                         std::isnan(p.quality_max_cr_db)))
    return bad(PWBF_E_INVALID, "the quality check needs two finite discs (r > 0) and a bound");
  if (pwbf::is_iq_mode(p.mode))
    return bad(PWBF_E_UNSUPPORTED, "the IQ modes are single-frame only");
  pwbf::FramePlan P;
  int rc = pwbf::plan_frame(p.geom, pwbf::kF16, p.mode, p.angle, nullptr, &P, err,
                            pwbf::serve_waves());
  if (rc) return bad(rc, *err);
  if (P.n_angles > pwbf::serve_max_angles())
    return bad(PWBF_E_UNSUPPORTED, "at most " + std::to_string(pwbf::serve_max_angles()) +
                                       " angles are summed per frame");
  if (wants_env(p) || p.geom->bandpass) {
    pwbf_outputs o = {(float *)256, nullptr, (float *)256, p.want_log ? (float *)256 : nullptr,
                      nullptr};
    static unsigned char fake_ws[pwbf::kMaxSlotBytes] __attribute__((aligned(256)));
    rc = pwbf::validate_outputs(p.geom, &o, fake_ws, sizeof fake_ws, err);
    if (rc) return bad(rc, *err);
  }
  return PWBF_OK;
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
    const int rc = validate_probe(probes[i], i, &err);
    if (rc) return api_set_error(rc, err);
  }
  for (int i = 0; i < n; ++i)
    if (hbm_budget_bytes && slot_bytes(probes[i]) > hbm_budget_bytes)
      return api_set_error(PWBF_E_INVALID, "probe " + std::to_string(i) + ": one slot needs " +
                                               std::to_string(slot_bytes(probes[i])) +
                                               " bytes, more than the HBM budget");
  pwbf_server *s = new pwbf_server();
  s->probes.resize(n);
  std::vector<pwbf::serve::ProbeInfo> info(n);
  std::vector<pwbf::FramePlan> plans;
  std::vector<pwbf::PostPlan> post;
  std::vector<pwbf::QualityPlan> quality;
  hipError_t e = hipSuccess;
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    const pwbf_probe &pp = probes[i];
    Probe &p = s->probes[i];
    p.geom.set(*pp.geom);
    p.want_log = pp.want_log;
    p.want_env = wants_env(pp);
    p.want_quality = pp.want_quality;
    const pwbf_geometry &g = p.geom.g;
    p.rf_elems = (size_t)g.n_angles * g.n_channels * g.n_samples;
    const size_t plane = (size_t)g.nx * g.nz * sizeof(float);
    const int nslots = pp.slots ? pp.slots : 4;
    info[i].slot_bytes = slot_bytes(pp);
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
      // the quality check reads the frame maximum that post-processing folds
      if (p.want_quality) Q.ws_max = (uint32_t *)sl.ws;
      pwbf::QualityPlan qp;
      std::memset(&qp, 0, sizeof qp);
      if (p.want_quality) {
        qp.env = sl.env;
        qp.ws_max = (const uint32_t *)sl.ws;
        qp.nz = g.nz;
        qp.max_cr_db = (float)pp.quality_max_cr_db;
        qp.in = pwbf::disc_to_pixels(&g, pp.quality_region.in);
        qp.out = pwbf::disc_to_pixels(&g, pp.quality_region.out);
        pwbf::quality_chunks(qp.in, &qp.chunks_in, &qp.cols_in);
        pwbf::quality_chunks(qp.out, &qp.chunks_out, &qp.cols_out);
      }
      p.tiles = P.n_tiles;
      p.cols = pwbf::post_needed(&o) ? g.nx : 0;
      p.log_cols = p.want_log ? g.nx : 0;
      if (k == 0)  // its deepest (first-run) tile row holds the costliest tiles
        for (int t = 0; t < P.n_tiles; ++t)
          info[i].tile_cost = std::max(info[i].tile_cost, pwbf::tile_cost(&g, P, t));
      s->lds = std::max(s->lds, (int)pwbf::plan_lds_bytes(P));
      if (pwbf::post_needed(&o)) s->max_nz = std::max(s->max_nz, g.nz);
      info[i].slots.push_back(idx);
      plans.push_back(P);
      post.push_back(Q);
      quality.push_back(qp);
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
  const size_t qregion = (size_t)kInflight * pwbf::serve::Core::kMaxBatch;
  if (e == hipSuccess) e = hipMalloc((void **)&s->d_plans, plans.size() * sizeof(pwbf::FramePlan));
  if (e == hipSuccess) e = hipMalloc((void **)&s->d_post, post.size() * sizeof(pwbf::PostPlan));
  if (e == hipSuccess)
    e = hipMalloc((void **)&s->d_quality, quality.size() * sizeof(pwbf::QualityPlan));
  if (e == hipSuccess) e = hipMalloc((void **)&s->d_qout, qregion * sizeof(pwbf::QualityOut));
  if (e == hipSuccess) e = hipHostMalloc((void **)&s->h_qout, qregion * sizeof(pwbf::QualityOut));
  if (e == hipSuccess)
    e = hipMalloc((void **)&s->d_qpart, qregion * kQualityBlocksPerSlot * sizeof(float4));
  if (e == hipSuccess) e = hipMalloc((void **)&s->d_qcount, qregion * sizeof(int));
  if (e == hipSuccess) e = hipMemset(s->d_qcount, 0, qregion * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void **)&s->d_counter, sizeof(int) * pwbf::kTileClasses);
  if (e == hipSuccess)
    e = hipMemcpy(s->d_plans, plans.data(), plans.size() * sizeof(pwbf::FramePlan),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(s->d_post, post.data(), post.size() * sizeof(pwbf::PostPlan),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(s->d_quality, quality.data(), quality.size() * sizeof(pwbf::QualityPlan),
                  hipMemcpyHostToDevice);
  s->quality = quality;
  for (hipStream_t &c : s->copy_s)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->comp_s, hipStreamNonBlocking);
  if (e != hipSuccess) {
    free_server(s);
    return api_set_error(PWBF_E_NOMEM, std::string("server allocation: ") + hipGetErrorString(e));
  }
  s->core = std::make_unique<pwbf::serve::Core>(std::move(info), hbm_budget_bytes,
                                                max_queue ? max_queue : 1024, &s->clock,
                                                serve_inflight());
  s->launcher = std::make_unique<HipLauncher>(s);
  s->worker = std::thread(scheduler, s);
  *out = s;
  return PWBF_OK;
}

int pwbf_server_submit_ex(pwbf_server *s, int32_t probe, const int16_t *host_rf,
                          double t_arrival, double deadline, uint64_t *id) {
  pwbf::api_clear_error();
  if (!s || !host_rf) return api_set_error(PWBF_E_INVALID, "server or host_rf is NULL");
  if (std::isnan(deadline) || std::isnan(t_arrival))
    return api_set_error(PWBF_E_INVALID, "t_arrival and deadline must be numbers");
  std::string err;
  const int rc = s->core->submit(probe, host_rf, t_arrival, deadline, id, &err);
  return rc ? api_set_error(rc, err) : PWBF_OK;
}

int pwbf_server_submit(pwbf_server *s, int32_t probe, const int16_t *host_rf, double t_arrival,
                       uint64_t *id) {
  return pwbf_server_submit_ex(s, probe, host_rf, t_arrival, -1.0, id);
}

int pwbf_server_poll(pwbf_server *s, pwbf_result *results, int32_t max, int32_t *n,
                     int32_t wait_ms) {
  pwbf::api_clear_error();
  if (!s || !results || !n || max < 1) return api_set_error(PWBF_E_INVALID, "bad poll arguments");
  *n = 0;
  std::vector<pwbf::serve::Request> got;
  std::string err;
  const int rc = s->core->poll(&got, max, wait_ms, &err);
  if (rc) return api_set_error(rc, err);
  for (const pwbf::serve::Request &r : got) {
    pwbf_result &o = results[(*n)++];
    std::memset(&o, 0, sizeof o);
    o.id = r.id;
    o.probe = r.probe;
    o.t_arrival = r.t_arrival;
    o.t_admit = r.t_admit;
    o.t_launch = r.t_launch;
    o.t_done = r.t_done;
    if (r.state == pwbf::serve::kExpired) {
      o.slot = -1;
      o.status = PWBF_E_TIMEOUT;
      continue;
    }
    const Slot &sl = s->slots[r.slot];
    o.slot = r.slot;
    o.status = PWBF_OK;
    o.rf = sl.out_rf;
    o.env = sl.env;
    o.logimg = sl.logimg;
    o.quality_ok = r.quality.ok;
    o.frame_max = r.quality.frame_max;
    o.cr_db = r.quality.cr_db;
    o.cnr = r.quality.cnr;
  }
  return PWBF_OK;
}

int pwbf_server_release(pwbf_server *s, uint64_t id) {
  pwbf::api_clear_error();
  if (!s) return api_set_error(PWBF_E_INVALID, "server is NULL");
  std::string err;
  const int rc = s->core->release(id, &err);
  return rc ? api_set_error(rc, err) : PWBF_OK;
}

int pwbf_server_stats_get(pwbf_server *s, pwbf_server_stats *st) {
  pwbf::api_clear_error();
  if (!s || !st) return api_set_error(PWBF_E_INVALID, "server or stats is NULL");
  const pwbf::serve::Stats c = s->core->stats();
  st->submitted = c.submitted;
  st->rejected = c.rejected;
  st->completed = c.completed;
  st->batches = c.batches;
  st->queued = c.queued;
  st->in_flight = c.in_flight;
  st->mean_batch = c.mean_batch;
  st->budget_bytes = c.budget;
  st->budget_in_use = c.in_use;
  st->budget_peak = c.peak;
  st->expired = c.expired;
  return PWBF_OK;
}

double pwbf_server_now(const pwbf_server *s) { return s ? s->clock.now() : 0.0; }

int pwbf_server_destroy(pwbf_server *s) {
  pwbf::api_clear_error();
  if (!s) return PWBF_OK;
  s->core->stop();
  if (s->worker.joinable()) s->worker.join();
  hipError_t e = hipStreamSynchronize(s->comp_s);
  for (hipStream_t c : s->copy_s)
    if (e == hipSuccess) e = hipStreamSynchronize(c);
  // completion callbacks touch the server: wait until the last one has run
  for (int k = 0; k < 10000 && s->core->inflight() > 0; ++k)
    std::this_thread::sleep_for(std::chrono::milliseconds(1));
  free_server(s);
  return e == hipSuccess ? PWBF_OK : api_set_error(PWBF_E_DEVICE, "server teardown");
}

}  // extern "C"
