// The serving loop's decisions without the device: the request ledger, queue
// limits, admission by HBM budget, deadlines, continuous batching, completion
// and release. The HIP side (serve.cpp) supplies a Launcher that uploads a
// request's RF into its slot and launches a batch of slots; tests supply a
// mock launcher and a fake clock, so every decision runs on the CPU.
#pragma once

#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <functional>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

namespace pwbf {
namespace serve {

struct ProbeInfo {
  size_t slot_bytes = 0;          // device bytes a slot holds while in use
  std::vector<int> slots;         // global indices of the probe's ring slots
  double tile_cost = 0;           // its costliest tile (batch ordering)
};

enum ReqState { kQueued, kAdmitted, kRunning, kDone, kExpired };

struct Quality {
  float frame_max = 0, cr_db = 0, cnr = 0;
  int ok = 0;
};

struct Request {
  uint64_t id = 0;
  int probe = 0, slot = -1;
  const void *host = nullptr;
  double t_arrival = 0, deadline = -1, t_admit = 0, t_launch = 0, t_done = 0;
  ReqState state = kQueued;
  Quality quality;
};

struct Stats {
  int64_t submitted = 0, rejected = 0, completed = 0, expired = 0, batches = 0;
  int64_t queued = 0, in_flight = 0;
  double mean_batch = 0;
  size_t budget = 0, in_use = 0, peak = 0;
};

// One batch handed to the launcher: (request id, slot) pairs, costliest first.
using Batch = std::vector<std::pair<uint64_t, int>>;

class Launcher {
 public:
  virtual ~Launcher() = default;
  // enqueue the upload of host RF into the slot; 0 or a PWBF_E_* code
  virtual int upload(int slot, const void *host, std::string *err) = 0;
  // whether the slot's last upload has finished
  virtual bool upload_done(int slot) = 0;
  // enqueue the batch; the launcher calls Core::complete(ids, ...) when it is done
  virtual int launch(const Batch &batch, std::string *err) = 0;
};

class Clock {
 public:
  virtual ~Clock() = default;
  virtual double now() const = 0;  // seconds
};

class Core {
 public:
  static constexpr int kMaxBatch = 64;
  static constexpr int kMaxInflight = 4;  // the most batches on the device at once

  // max_inflight: batches on the device at once, 1..kMaxInflight (clamped;
  // the server passes PWBF_SERVE_INFLIGHT, by default kMaxInflight)
  Core(std::vector<ProbeInfo> probes, size_t budget, int max_queue, const Clock *clock,
       int max_inflight = 2);

  // ---- callers (thread-safe)
  // queue a request; deadline < 0: none, else the server time by which it must
  // be admitted. PWBF_OK, PWBF_E_INVALID, PWBF_E_BUSY (queue full) or
  // PWBF_E_DEVICE (the loop has failed; *err holds why)
  int submit(int probe, const void *host, double t_arrival, double deadline, uint64_t *id,
             std::string *err);
  // move up to max finished requests (completed or expired) into out
  int poll(std::vector<Request> *out, int max, int wait_ms, std::string *err);
  // free the slot of a finished request
  int release(uint64_t id, std::string *err);
  Stats stats();
  // the scheduler's failure, if any ("" while healthy)
  std::string failure();

  // ---- the scheduler (one thread)
  // one round: expire late requests, admit, upload, launch a batch if a device
  // slot is free. Returns kWorked, kIdle (nothing to do: wait for work) or
  // kUploading (admitted requests wait for their uploads: poll again soon)
  enum StepResult { kWorked, kIdle, kUploading };
  StepResult step(Launcher &launcher);
  // block up to max_us for new work or a completion
  void wait_for_work(int max_us);
  void stop();
  bool stopped();
  // completion of a launched batch (from the launcher's callback)
  void complete(const std::vector<uint64_t> &ids, const std::vector<Quality> *quality);
  void fail(const std::string &msg);
  int inflight();

 private:
  std::vector<ProbeInfo> probes_;
  std::vector<int> slot_probe_;
  std::vector<std::deque<uint64_t>> queue_;
  std::vector<std::vector<int>> free_;
  size_t budget_, in_use_ = 0, peak_ = 0;
  int max_queue_;
  const Clock *clock_;

  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  bool stop_ = false;
  uint64_t next_id_ = 1;
  std::unordered_map<uint64_t, Request> reqs_;
  std::vector<uint64_t> admitted_;  // upload enqueued, not yet launched (oldest first)
  std::deque<uint64_t> done_;       // finished, not yet polled
  int max_inflight_ = 2;
  int inflight_ = 0, rr_ = 0;
  int64_t submitted_ = 0, rejected_ = 0, completed_ = 0, expired_ = 0, batches_ = 0,
          batched_reqs_ = 0;
  std::string failure_;
};

}  // namespace serve
}  // namespace pwbf
