// The serving loop's decisions on the CPU: serve::Core driven by a fake clock
// and a mock launcher (no device). Each case prints "ok <name>"; the first
// failed check prints where and exits with status 1.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pwbf.h"
#include "../../paper_2311_00482_amd/csrc/serve_core.h"

using namespace pwbf::serve;

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #c); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

namespace {

struct FakeClock : Clock {
  double t = 0;
  double now() const override { return t; }
};

struct MockLauncher : Launcher {
  std::vector<std::pair<int, const void *>> uploads;
  std::set<int> done;          // slots whose upload has finished
  bool all_done = true;        // every upload finishes at once
  std::vector<Batch> batches;  // launched batches
  int fail_upload = 0, fail_launch = 0;
  int upload(int slot, const void *host, std::string *err) override {
    if (fail_upload) {
      *err = "mock upload failure";
      return fail_upload;
    }
    uploads.push_back({slot, host});
    done.erase(slot);
    return PWBF_OK;
  }
  bool upload_done(int slot) override { return all_done || done.count(slot) > 0; }
  int launch(const Batch &b, std::string *err) override {
    if (fail_launch) {
      *err = "mock launch failure";
      return fail_launch;
    }
    batches.push_back(b);
    return PWBF_OK;
  }
};

ProbeInfo probe(size_t bytes, std::vector<int> slots, double cost = 1.0) {
  ProbeInfo p;
  p.slot_bytes = bytes;
  p.slots = std::move(slots);
  p.tile_cost = cost;
  return p;
}

const int16_t kHost[4] = {1, 2, 3, 4};

uint64_t submit_ok(Core &c, int probe, double deadline = -1) {
  uint64_t id = 0;
  std::string err;
  CHECK(c.submit(probe, kHost, -1, deadline, &id, &err) == PWBF_OK);
  CHECK(id != 0);
  return id;
}

std::vector<Request> poll_all(Core &c) {
  std::vector<Request> out;
  std::string err;
  CHECK(c.poll(&out, 1000, 0, &err) == PWBF_OK);
  return out;
}

std::vector<uint64_t> ids_of(const Batch &b) {
  std::vector<uint64_t> v;
  for (const auto &x : b) v.push_back(x.first);
  return v;
}

void test_budget_admission_and_release() {
  FakeClock clk;
  // probe 0: two slots of 100 bytes; probe 1: one slot of 100 bytes, costlier tiles
  Core c({probe(100, {0, 1}, 1.0), probe(100, {2}, 5.0)}, 200, 16, &clk);
  MockLauncher m;
  const uint64_t a = submit_ok(c, 0), b = submit_ok(c, 0), d = submit_ok(c, 0);
  const uint64_t e = submit_ok(c, 1);
  CHECK(c.step(m) == Core::kWorked);
  // round robin: one of probe 0, one of probe 1, then the budget is spent
  CHECK(m.uploads.size() == 2);
  Stats st = c.stats();
  CHECK(st.in_use == 200 && st.peak == 200 && st.queued == 2 && st.in_flight == 2);
  CHECK(m.batches.size() == 1 && m.batches[0].size() == 2);
  // the costlier probe's slot first
  CHECK(m.batches[0][0].first == e && m.batches[0][0].second == 2);
  CHECK(m.batches[0][1].first == a && m.batches[0][1].second == 0);
  // nothing fits the budget until a slot is released
  CHECK(c.step(m) == Core::kIdle);
  CHECK(m.uploads.size() == 2);
  c.complete(ids_of(m.batches[0]), nullptr);
  std::vector<Request> got = poll_all(c);
  CHECK(got.size() == 2 && got[0].state == kDone && got[1].state == kDone);
  CHECK(c.stats().completed == 2 && c.stats().in_use == 200);
  std::string err;
  CHECK(c.release(e, &err) == PWBF_OK);
  CHECK(c.stats().in_use == 100);
  CHECK(c.step(m) == Core::kWorked);
  CHECK(m.uploads.size() == 3 && m.uploads[2].second == kHost);
  // probe 0's second slot goes to its oldest waiting request
  CHECK(m.batches.size() == 2 && m.batches[1].size() == 1 && m.batches[1][0].first == b &&
        m.batches[1][0].second == 1);
  CHECK(c.stats().queued == 1);  // d still waits for the budget
  (void)d;
  std::puts("ok budget_admission_and_release");
}

void test_queue_limit_and_bad_probe() {
  FakeClock clk;
  Core c({probe(10, {0})}, 0, 2, &clk);
  std::string err;
  uint64_t id;
  CHECK(c.submit(0, kHost, -1, -1, &id, &err) == PWBF_OK);
  CHECK(c.submit(0, kHost, -1, -1, &id, &err) == PWBF_OK);
  CHECK(c.submit(0, kHost, -1, -1, &id, &err) == PWBF_E_BUSY);
  CHECK(err.find("queue full") != std::string::npos);
  CHECK(c.submit(1, kHost, -1, -1, &id, &err) == PWBF_E_INVALID);
  CHECK(c.submit(-1, kHost, -1, -1, &id, &err) == PWBF_E_INVALID);
  Stats st = c.stats();
  CHECK(st.submitted == 3 && st.rejected == 1 && st.queued == 2);
  std::puts("ok queue_limit_and_bad_probe");
}

void test_deadline_expiry() {
  FakeClock clk;
  Core c({probe(50, {0})}, 0, 16, &clk);
  MockLauncher m;
  const uint64_t a = submit_ok(c, 0);
  const uint64_t b = submit_ok(c, 0, 1.0);   // waits for the one slot
  const uint64_t f = submit_ok(c, 0, 10.0);  // admitted in time later
  CHECK(c.step(m) == Core::kWorked);
  CHECK(m.batches.size() == 1 && m.batches[0].size() == 1 && m.batches[0][0].first == a);
  clk.t = 0.5;
  CHECK(c.step(m) == Core::kIdle);
  CHECK(poll_all(c).empty());
  clk.t = 1.5;
  c.step(m);
  std::vector<Request> got = poll_all(c);
  CHECK(got.size() == 1 && got[0].id == b && got[0].state == kExpired && got[0].slot == -1);
  CHECK(got[0].t_done == 1.5);
  Stats st = c.stats();
  CHECK(st.expired == 1 && st.in_use == 50 && st.queued == 1);
  std::string err;
  CHECK(c.release(b, &err) == PWBF_OK);  // frees nothing
  CHECK(c.stats().in_use == 50);
  CHECK(c.release(b, &err) == PWBF_E_INVALID);
  // the slot comes back; f (deadline 10) is admitted at t = 2
  c.complete({a}, nullptr);
  CHECK(c.release(a, &err) == PWBF_OK);
  clk.t = 2.0;
  CHECK(c.step(m) == Core::kWorked);
  CHECK(m.batches.size() == 2 && m.batches[1][0].first == f);
  c.complete({f}, nullptr);
  got = poll_all(c);  // a was released before it was polled: only f comes back
  CHECK(got.size() == 1 && got[0].id == f && got[0].state == kDone && got[0].t_admit == 2.0);
  std::puts("ok deadline_expiry");
}

void test_upload_failure_propagates() {
  FakeClock clk;
  Core c({probe(10, {0, 1})}, 0, 16, &clk);
  MockLauncher m;
  m.fail_upload = PWBF_E_DEVICE;
  submit_ok(c, 0);
  CHECK(c.step(m) == Core::kIdle);
  CHECK(c.failure().find("upload: mock upload failure") != std::string::npos);
  std::string err;
  uint64_t id;
  CHECK(c.submit(0, kHost, -1, -1, &id, &err) == PWBF_E_DEVICE);
  CHECK(err.find("mock upload failure") != std::string::npos);
  std::vector<Request> out;
  CHECK(c.poll(&out, 4, 0, &err) == PWBF_E_DEVICE);
  CHECK(c.step(m) == Core::kIdle && m.batches.empty());  // the loop does nothing more
  std::puts("ok upload_failure_propagates");
}

void test_launch_failure_propagates() {
  FakeClock clk;
  Core c({probe(10, {0})}, 0, 16, &clk);
  MockLauncher m;
  m.fail_launch = PWBF_E_DEVICE;
  submit_ok(c, 0);
  c.step(m);
  CHECK(c.failure().find("batch launch: mock launch failure") != std::string::npos);
  std::vector<Request> out;
  std::string err;
  // a waiting poller wakes up with the failure instead of timing out
  const auto t0 = std::chrono::steady_clock::now();
  CHECK(c.poll(&out, 4, 5000, &err) == PWBF_E_DEVICE);
  CHECK(std::chrono::steady_clock::now() - t0 < std::chrono::seconds(2));
  std::puts("ok launch_failure_propagates");
}

void test_release_errors() {
  FakeClock clk;
  Core c({probe(10, {0})}, 0, 16, &clk);
  MockLauncher m;
  std::string err;
  CHECK(c.release(12345, &err) == PWBF_E_INVALID);
  const uint64_t a = submit_ok(c, 0);
  CHECK(c.release(a, &err) == PWBF_E_INVALID);  // queued
  c.step(m);
  CHECK(c.release(a, &err) == PWBF_E_INVALID);  // running
  c.complete({a}, nullptr);
  CHECK(c.release(a, &err) == PWBF_OK);
  CHECK(c.release(a, &err) == PWBF_E_INVALID);  // twice
  std::puts("ok release_errors");
}

void test_continuous_batching() {
  FakeClock clk;
  Core c({probe(10, {0, 1, 2, 3, 4})}, 0, 64, &clk);
  MockLauncher m;
  m.all_done = false;
  const uint64_t a = submit_ok(c, 0);
  // nothing on the device: the oldest request starts a batch before its upload ends
  CHECK(c.step(m) == Core::kWorked);
  CHECK(m.batches.size() == 1 && m.batches[0].size() == 1 && m.batches[0][0].first == a);
  const uint64_t b = submit_ok(c, 0), d = submit_ok(c, 0), e = submit_ok(c, 0);
  // one batch runs: requests join the next batch only once uploaded
  CHECK(c.step(m) == Core::kUploading);
  CHECK(m.batches.size() == 1 && m.uploads.size() == 4);
  m.done.insert(m.uploads[1].first);
  m.done.insert(m.uploads[2].first);
  CHECK(c.step(m) == Core::kWorked);
  CHECK(m.batches.size() == 2 && m.batches[1].size() == 2);
  CHECK(m.batches[1][0].first == b && m.batches[1][1].first == d);
  // two batches on the device: no third launch, even with e uploaded
  m.done.insert(m.uploads[3].first);
  CHECK(c.step(m) == Core::kIdle);
  CHECK(m.batches.size() == 2);
  c.complete({a}, nullptr);
  CHECK(c.step(m) == Core::kWorked);
  CHECK(m.batches.size() == 3 && m.batches[2].size() == 1 && m.batches[2][0].first == e);
  Stats st = c.stats();
  CHECK(st.batches == 3 && st.mean_batch == 4.0 / 3.0);
  std::puts("ok continuous_batching");
}

void test_inflight_limit() {
  // the limit given to the core (the server's PWBF_SERVE_INFLIGHT): four
  // batches may run at once and a fifth waits; out-of-range limits clamp
  for (int limit : {4, 9, 0}) {
    const int want = limit < 1 ? 1 : (limit > Core::kMaxInflight ? Core::kMaxInflight : limit);
    FakeClock clk;
    Core c({probe(10, {0, 1, 2, 3, 4, 5})}, 0, 64, &clk, limit);
    MockLauncher m;
    std::vector<uint64_t> ids;
    for (int k = 0; k < 6; ++k) {
      ids.push_back(submit_ok(c, 0));
      c.step(m);  // each request uploads at once and starts its own batch while a slot is free
    }
    CHECK((int)m.batches.size() == want);
    CHECK(c.inflight() == want);
    c.complete({ids[0]}, nullptr);
    CHECK(c.step(m) == Core::kWorked);
    CHECK((int)m.batches.size() == want + 1);
  }
  std::puts("ok inflight_limit");
}

void test_round_robin_and_fifo() {
  FakeClock clk;
  Core c({probe(1, {0, 1, 2}), probe(1, {3, 4, 5})}, 0, 64, &clk);
  MockLauncher m;
  std::vector<uint64_t> p0, p1;
  for (int k = 0; k < 3; ++k) p0.push_back(submit_ok(c, 0));
  for (int k = 0; k < 3; ++k) p1.push_back(submit_ok(c, 1));
  c.step(m);
  CHECK(m.uploads.size() == 6 && m.batches.size() == 1 && m.batches[0].size() == 6);
  // alternate probes, each in arrival order, on the probe's slots in listed order
  const std::vector<int> slots = {0, 3, 1, 4, 2, 5};
  for (int k = 0; k < 6; ++k) CHECK(m.uploads[k].first == slots[k]);
  std::map<uint64_t, int> slot_of;
  for (const auto &x : m.batches[0]) slot_of[x.first] = x.second;
  CHECK(slot_of[p0[0]] == 0 && slot_of[p0[1]] == 1 && slot_of[p0[2]] == 2);
  CHECK(slot_of[p1[0]] == 3 && slot_of[p1[1]] == 4 && slot_of[p1[2]] == 5);
  std::puts("ok round_robin_and_fifo");
}

void test_poll_limit_quality_and_times() {
  FakeClock clk;
  Core c({probe(1, {0, 1, 2})}, 0, 64, &clk);
  MockLauncher m;
  clk.t = 3.0;
  std::string err;
  uint64_t a, b, d;
  CHECK(c.submit(0, kHost, 2.5, -1, &a, &err) == PWBF_OK);  // the caller's arrival time
  CHECK(c.submit(0, kHost, -1, -1, &b, &err) == PWBF_OK);   // the clock's
  CHECK(c.submit(0, kHost, -1, -1, &d, &err) == PWBF_OK);
  clk.t = 4.0;
  c.step(m);
  clk.t = 5.0;
  std::vector<Quality> q(3);
  q[1].frame_max = 7.f;
  q[1].cr_db = -20.f;
  q[1].cnr = -1.5f;
  q[1].ok = 1;
  c.complete(ids_of(m.batches[0]), &q);
  std::vector<Request> out;
  CHECK(c.poll(&out, 2, 0, &err) == PWBF_OK && out.size() == 2);
  CHECK(c.poll(&out, 3, 0, &err) == PWBF_OK && out.size() == 3);
  CHECK(out[0].t_arrival == 2.5 && out[1].t_arrival == 3.0);
  for (const Request &r : out) CHECK(r.t_admit == 4.0 && r.t_launch == 4.0 && r.t_done == 5.0);
  CHECK(out[1].quality.ok == 1 && out[1].quality.frame_max == 7.f && out[1].quality.cr_db == -20.f);
  CHECK(out[0].quality.ok == 0 && out[2].quality.ok == 0);
  std::puts("ok poll_limit_quality_and_times");
}

void test_stop() {
  FakeClock clk;
  Core c({probe(1, {0})}, 0, 4, &clk);
  MockLauncher m;
  submit_ok(c, 0);
  c.stop();
  CHECK(c.stopped());
  CHECK(c.step(m) == Core::kIdle && m.uploads.empty());
  c.wait_for_work(1000000);  // returns at once once stopped
  std::puts("ok stop");
}

// A scheduler thread, a completion thread standing in for the device, two
// producers and a consumer that releases: every request completes once, the
// ledger returns to zero and never exceeds the budget.
struct AsyncLauncher : Launcher {
  Core *core = nullptr;
  std::mutex mu;
  std::vector<std::vector<uint64_t>> pending;
  int upload(int, const void *, std::string *) override { return PWBF_OK; }
  bool upload_done(int) override { return true; }
  int launch(const Batch &b, std::string *) override {
    std::lock_guard<std::mutex> lk(mu);
    pending.push_back(ids_of(b));
    return PWBF_OK;
  }
};

struct RealClock : Clock {
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double now() const override {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

void test_threads() {
  RealClock clk;
  Core c({probe(100, {0, 1, 2}), probe(300, {3, 4})}, 500, 1 << 20, &clk);
  AsyncLauncher L;
  L.core = &c;
  std::atomic<bool> quit{false};
  std::thread sched([&] {
    while (!c.stopped()) {
      if (c.step(L) != Core::kWorked) c.wait_for_work(100);
    }
  });
  std::thread device([&] {
    while (!quit) {
      std::vector<std::vector<uint64_t>> todo;
      {
        std::lock_guard<std::mutex> lk(L.mu);
        todo.swap(L.pending);
      }
      for (auto &ids : todo) c.complete(ids, nullptr);
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
  });
  const int per = 400;
  std::vector<std::thread> prod;
  for (int p = 0; p < 2; ++p)
    prod.emplace_back([&, p] {
      for (int k = 0; k < per; ++k) submit_ok(c, p);
    });
  int got = 0;
  size_t peak = 0;
  std::set<uint64_t> seen;
  const auto t0 = std::chrono::steady_clock::now();
  while (got < 2 * per) {
    std::vector<Request> out;
    std::string err;
    CHECK(c.poll(&out, 64, 10, &err) == PWBF_OK);
    for (const Request &r : out) {
      CHECK(r.state == kDone && seen.insert(r.id).second);
      CHECK(c.release(r.id, &err) == PWBF_OK);
      ++got;
    }
    peak = std::max(peak, c.stats().peak);
    CHECK(std::chrono::steady_clock::now() - t0 < std::chrono::seconds(60));
  }
  for (auto &t : prod) t.join();
  c.stop();
  sched.join();
  quit = true;
  device.join();
  Stats st = c.stats();
  CHECK(st.completed == 2 * per && st.in_use == 0 && st.queued == 0 && st.in_flight == 0);
  CHECK(st.peak <= 500 && peak <= 500);
  std::puts("ok threads");
}

}  // namespace

int main() {
  test_budget_admission_and_release();
  test_queue_limit_and_bad_probe();
  test_deadline_expiry();
  test_upload_failure_propagates();
  test_launch_failure_propagates();
  test_release_errors();
  test_continuous_batching();
  test_inflight_limit();
  test_round_robin_and_fifo();
  test_poll_limit_quality_and_times();
  test_stop();
  test_threads();
  std::puts("all ok");
  return 0;
}
