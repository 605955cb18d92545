// The serving loop's decisions (serve_core.h), free of any device call.
#include "serve_core.h"

#include <algorithm>
#include <chrono>

#include "../../include/pwbf.h"

namespace pwbf {
namespace serve {

Core::Core(std::vector<ProbeInfo> probes, size_t budget, int max_queue, const Clock *clock,
           int max_inflight)
    : probes_(std::move(probes)), budget_(budget), max_queue_(max_queue), clock_(clock),
      max_inflight_(std::min(std::max(max_inflight, 1), kMaxInflight)) {
  int n_slots = 0;
  for (const ProbeInfo &p : probes_)
    for (int s : p.slots) n_slots = std::max(n_slots, s + 1);
  slot_probe_.assign(n_slots, -1);
  queue_.resize(probes_.size());
  free_.resize(probes_.size());
  for (size_t i = 0; i < probes_.size(); ++i) {
    for (int s : probes_[i].slots) slot_probe_[s] = (int)i;
    // slots are handed out last-in first-out: the first listed is used first
    free_[i].assign(probes_[i].slots.rbegin(), probes_[i].slots.rend());
  }
}

int Core::submit(int probe, const void *host, double t_arrival, double deadline, uint64_t *id,
                 std::string *err) {
  std::unique_lock<std::mutex> lk(mu_);
  if (!failure_.empty()) {
    *err = failure_;
    return PWBF_E_DEVICE;
  }
  if (probe < 0 || probe >= (int)probes_.size()) {
    *err = "probe index out of range";
    return PWBF_E_INVALID;
  }
  submitted_ += 1;
  if ((int)queue_[probe].size() >= max_queue_) {
    rejected_ += 1;
    *err = "probe queue full";
    return PWBF_E_BUSY;
  }
  Request r;
  r.id = next_id_++;
  r.probe = probe;
  r.host = host;
  r.t_arrival = t_arrival < 0 ? clock_->now() : t_arrival;
  r.deadline = deadline;
  reqs_.emplace(r.id, r);
  queue_[probe].push_back(r.id);
  if (id) *id = r.id;
  lk.unlock();
  cv_work_.notify_one();
  return PWBF_OK;
}

int Core::poll(std::vector<Request> *out, int max, int wait_ms, std::string *err) {
  std::unique_lock<std::mutex> lk(mu_);
  if (done_.empty() && wait_ms > 0)
    cv_done_.wait_for(lk, std::chrono::milliseconds(wait_ms),
                      [&] { return !done_.empty() || !failure_.empty(); });
  if (!failure_.empty() && done_.empty()) {
    *err = failure_;
    return PWBF_E_DEVICE;
  }
  while (!done_.empty() && (int)out->size() < max) {
    out->push_back(reqs_.at(done_.front()));
    done_.pop_front();
  }
  return PWBF_OK;
}

int Core::release(uint64_t id, std::string *err) {
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = reqs_.find(id);
    if (it == reqs_.end() || (it->second.state != kDone && it->second.state != kExpired)) {
      *err = "no finished request with that id";
      return PWBF_E_INVALID;
    }
    if (it->second.state == kDone) {
      const int p = it->second.probe;
      free_[p].push_back(it->second.slot);
      in_use_ -= probes_[p].slot_bytes;
    }
    // released before it was polled: poll no longer returns it
    done_.erase(std::remove(done_.begin(), done_.end(), id), done_.end());
    reqs_.erase(it);
  }
  cv_work_.notify_one();
  return PWBF_OK;
}

Stats Core::stats() {
  std::lock_guard<std::mutex> lk(mu_);
  Stats st;
  st.submitted = submitted_;
  st.rejected = rejected_;
  st.completed = completed_;
  st.expired = expired_;
  st.batches = batches_;
  for (const auto &q : queue_) st.queued += (int64_t)q.size();
  int64_t finished = 0;
  for (const auto &kv : reqs_)
    if (kv.second.state == kDone || kv.second.state == kExpired) ++finished;
  st.in_flight = (int64_t)reqs_.size() - st.queued - finished;
  st.mean_batch = batches_ ? (double)batched_reqs_ / batches_ : 0.0;
  st.budget = budget_;
  st.in_use = in_use_;
  st.peak = peak_;
  return st;
}

std::string Core::failure() {
  std::lock_guard<std::mutex> lk(mu_);
  return failure_;
}

Core::StepResult Core::step(Launcher &launcher) {
  struct Upload {
    int slot;
    const void *host;
  };
  std::vector<Upload> uploads;
  Batch candidates;
  bool can_launch = false, expired_any = false;
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (stop_ || !failure_.empty()) return kIdle;
    const double now = clock_->now();
    // requests still queued past their deadline are dropped
    for (auto &q : queue_) {
      for (auto it = q.begin(); it != q.end();) {
        Request &r = reqs_[*it];
        if (r.deadline >= 0 && now > r.deadline) {
          r.state = kExpired;
          r.t_done = now;
          done_.push_back(r.id);
          expired_ += 1;
          expired_any = true;
          it = q.erase(it);
        } else {
          ++it;
        }
      }
    }
    // admission: round robin over probes, FIFO within a probe, while a slot
    // is free and the budget ledger allows the slot's bytes
    const int np = (int)probes_.size();
    bool any = true;
    while (any) {
      any = false;
      for (int k = 0; k < np; ++k) {
        const int p = (rr_ + k) % np;
        if (queue_[p].empty() || free_[p].empty()) continue;
        if (budget_ && in_use_ + probes_[p].slot_bytes > budget_) continue;
        const uint64_t id = queue_[p].front();
        queue_[p].pop_front();
        const int slot = free_[p].back();
        free_[p].pop_back();
        in_use_ += probes_[p].slot_bytes;
        peak_ = std::max(peak_, in_use_);
        Request &r = reqs_[id];
        r.slot = slot;
        r.t_admit = now;
        r.state = kAdmitted;
        uploads.push_back({slot, r.host});
        admitted_.push_back(id);
        any = true;
      }
    }
    rr_ = (rr_ + 1) % std::max(1, np);
    can_launch = inflight_ < max_inflight_ && !admitted_.empty();
    if (can_launch)
      for (uint64_t id : admitted_) candidates.push_back({id, reqs_[id].slot});
  }
  if (expired_any) cv_done_.notify_all();
  for (const Upload &u : uploads) {
    std::string err;
    const int rc = launcher.upload(u.slot, u.host, &err);
    if (rc) {
      fail("upload: " + err);
      return kIdle;
    }
  }
  if (!can_launch) return uploads.empty() ? kIdle : kWorked;
  // continuous batching: every admitted request whose upload has finished
  // joins this batch; with nothing on the device, the oldest one starts a batch
  // even if its upload is still running (the launch waits for it)
  Batch ready;
  for (const auto &c : candidates) {
    if ((int)ready.size() >= kMaxBatch) break;
    if (launcher.upload_done(c.second)) ready.push_back(c);
  }
  if (ready.empty() && inflight() == 0 && !candidates.empty()) ready.push_back(candidates[0]);
  if (ready.empty()) return kUploading;
  // slots with the costliest tiles first
  std::stable_sort(ready.begin(), ready.end(), [&](const auto &a, const auto &b) {
    return probes_[slot_probe_[a.second]].tile_cost > probes_[slot_probe_[b.second]].tile_cost;
  });
  {
    std::lock_guard<std::mutex> lk(mu_);
    const double t = clock_->now();
    for (const auto &r : ready) {
      Request &q = reqs_[r.first];
      q.t_launch = t;
      q.state = kRunning;
    }
    admitted_.erase(std::remove_if(admitted_.begin(), admitted_.end(),
                                   [&](uint64_t id) { return reqs_[id].state == kRunning; }),
                    admitted_.end());
    inflight_ += 1;
    batches_ += 1;
    batched_reqs_ += (int64_t)ready.size();
  }
  std::string err;
  const int rc = launcher.launch(ready, &err);
  if (rc) {
    fail("batch launch: " + err);
    return kIdle;
  }
  return kWorked;
}

void Core::wait_for_work(int max_us) {
  std::unique_lock<std::mutex> lk(mu_);
  if (stop_) return;
  cv_work_.wait_for(lk, std::chrono::microseconds(max_us));
}

void Core::stop() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_work_.notify_all();
  cv_done_.notify_all();
}

bool Core::stopped() {
  std::lock_guard<std::mutex> lk(mu_);
  return stop_;
}

void Core::complete(const std::vector<uint64_t> &ids, const std::vector<Quality> *quality) {
  {
    std::lock_guard<std::mutex> lk(mu_);
    const double t = clock_->now();
    for (size_t k = 0; k < ids.size(); ++k) {
      Request &r = reqs_[ids[k]];
      r.t_done = t;
      r.state = kDone;
      if (quality && k < quality->size()) r.quality = (*quality)[k];
      done_.push_back(r.id);
    }
    completed_ += (int64_t)ids.size();
    inflight_ -= 1;
  }
  cv_done_.notify_all();
  cv_work_.notify_all();
}

void Core::fail(const std::string &msg) {
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (failure_.empty()) failure_ = msg;
  }
  cv_done_.notify_all();
  cv_work_.notify_all();
}

int Core::inflight() {
  std::lock_guard<std::mutex> lk(mu_);
  return inflight_;
}

}  // namespace serve
}  // namespace pwbf
