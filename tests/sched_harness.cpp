// CPU harness of the serving scheduler (paper_1803_00005_amd/csrc/sched.hpp)
// with a fake executor: a simulated device whose jobs finish after a given
// number of polls, can be held back (a slow device), can fail to launch or
// finish with an error.  Each scenario checks the scheduler's invariants and
// exits non-zero on the first violation.
//
//   g++ -std=c++17 -O1 -I<repo> tests/sched_harness.cpp -o sched_harness
//   ./sched_harness <scenario>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "paper_1803_00005_amd/csrc/sched.hpp"

using hgf::sched::Job;
using hgf::sched::Scheduler;

namespace {

int g_failures = 0;

#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "CHECK failed at line %d: %s\n", __LINE__, #cond); \
      ++g_failures;                                                        \
    }                                                                      \
  } while (0)

struct Payload {
  int tag = 0;
};

// Simulated device: a launched job runs for `steps` polls once the device is
// not held; launches and completions are logged for the checks.
struct FakeExec {
  std::map<int64_t, int> left;          // polls until done, per running job
  std::map<int64_t, hgf_status> result; // completion status per job
  std::set<int64_t> fail_launch;        // jobs whose launch fails
  std::map<int64_t, hgf_status> fail_run;  // jobs that finish with an error
  std::vector<int64_t> launched;        // launch order
  std::vector<std::pair<size_t, size_t>> live;  // arena ranges of running jobs
  std::map<int64_t, std::pair<size_t, size_t>> range;
  int steps = 2;
  bool held = false;                    // a held device finishes nothing
  int released = 0;
  size_t arena = 0;

  hgf_status launch(Job<Payload>& j) {
    if (fail_launch.count(j.id)) return HGF_E_DEVICE;
    // the job's range lies in the arena and overlaps no running job's range
    const size_t a = j.off, b = j.off + hgf::sched::arena_align(j.bytes);
    CHECK(b <= arena);
    for (auto& kv : range) CHECK(b <= kv.second.first || a >= kv.second.second);
    range[j.id] = {a, b};
    launched.push_back(j.id);
    left[j.id] = steps;
    return HGF_OK;
  }
  int query(Job<Payload>& j, bool wait, hgf_completion* c) {
    auto it = left.find(j.id);
    CHECK(it != left.end());
    if (held && !wait) return 0;
    if (!wait && --it->second > 0) return 0;
    c->status = fail_run.count(j.id) ? fail_run[j.id] : HGF_OK;
    c->start_ms = 1.0;
    c->end_ms = 2.0;
    left.erase(it);
    range.erase(j.id);
    return 1;
  }
  void release(Job<Payload>& j) {
    (void)j;
    ++released;
  }
};

Job<Payload> job(size_t bytes, double work = 1.0, int tag = 0) {
  Job<Payload> j;
  j.bytes = bytes;
  j.work = work;
  j.payload.tag = tag;
  return j;
}

std::vector<hgf_completion> poll_all(Scheduler<Payload>& s, FakeExec& ex, hgf_status* st = nullptr) {
  std::vector<hgf_completion> out(64);
  int n = 0;
  const hgf_status r = s.poll(ex, out.data(), 64, &n);
  if (st != nullptr) *st = r;
  out.resize(n);
  return out;
}

// Strict FIFO admission within the arena budget; every job completes once.
void scenario_fifo() {
  FakeExec ex;
  ex.arena = 1024;
  Scheduler<Payload> s(1024, 3, 16);
  std::vector<int64_t> ids;
  for (int k = 0; k < 6; ++k) {
    int64_t id = -1;
    CHECK(s.submit(job(400), &id) == HGF_OK);
    ids.push_back(id);
  }
  CHECK(s.admit(ex) == HGF_OK);
  // two 400-byte jobs fit 1024 bytes, the third waits
  CHECK(s.running().size() == 2);
  CHECK(s.pending().size() == 4);
  std::vector<int64_t> done;
  for (int it = 0; it < 100 && s.completed() < 6; ++it)
    for (auto& c : poll_all(s, ex)) {
      CHECK(c.status == HGF_OK);
      done.push_back(c.id);
    }
  CHECK(done.size() == 6);
  CHECK(ex.launched == ids);  // admitted in submission order
  CHECK(s.arena().used() == 0);
  CHECK(s.arena().peak() <= 1024);
  CHECK(s.arena().free_ranges() == 1);  // freed ranges coalesce back to one
  CHECK(ex.released == 6);
}

// A job larger than the arena is refused at submit (nothing queued); a large
// job at the head of the queue holds back smaller later ones (no overtaking,
// so it cannot starve) until the arena has room for it.
void scenario_alloc_failure() {
  FakeExec ex;
  ex.arena = 1024;
  Scheduler<Payload> s(1024, 2, 16);
  int64_t id = -1;
  CHECK(s.submit(job(2048), &id) == HGF_E_NOMEM);
  CHECK(s.pending().empty());
  int64_t a, big, small;
  CHECK(s.submit(job(512), &a) == HGF_OK);
  CHECK(s.submit(job(1024), &big) == HGF_OK);
  CHECK(s.submit(job(256), &small) == HGF_OK);
  CHECK(s.admit(ex) == HGF_OK);
  // `big` does not fit next to `a`; `small` would, but must wait behind it
  CHECK(s.running().size() == 1);
  CHECK(ex.launched.size() == 1 && ex.launched[0] == a);
  for (int it = 0; it < 100 && s.completed() < 3; ++it) poll_all(s, ex);
  CHECK(s.completed() == 3);
  CHECK((ex.launched == std::vector<int64_t>{a, big, small}));
}

// A slow device: nothing finishes while it is held, the bounded queue fills
// and refuses further jobs with HGF_E_BUSY; once the device runs again,
// drain completes everything.
void scenario_slow_device() {
  FakeExec ex;
  ex.arena = 1000;
  ex.held = true;
  Scheduler<Payload> s(1000, 2, 3);
  int64_t id;
  CHECK(s.submit(job(600), &id) == HGF_OK);
  CHECK(s.admit(ex) == HGF_OK);
  CHECK(s.running().size() == 1);
  for (int k = 0; k < 3; ++k) CHECK(s.submit(job(600), &id) == HGF_OK);
  CHECK(s.submit(job(600), &id) == HGF_E_BUSY);
  for (int it = 0; it < 20; ++it) poll_all(s, ex);
  CHECK(s.completed() == 0);
  CHECK(s.pending().size() == 3);
  ex.held = false;
  CHECK(s.drain(ex) == HGF_OK);
  CHECK(s.completed() == 4);
  CHECK(s.pending().empty() && s.running().empty());
  CHECK(s.submit(job(600), &id) == HGF_OK);  // room again
}

// A launch that fails completes its job with the error, releases its range
// and lets the queue move on; a job that fails on the device is reported in
// its completion record.
void scenario_failures() {
  FakeExec ex;
  ex.arena = 4096;
  Scheduler<Payload> s(4096, 2, 16);
  std::vector<int64_t> ids(5);
  for (int k = 0; k < 5; ++k) CHECK(s.submit(job(1000), &ids[k]) == HGF_OK);
  ex.fail_launch.insert(ids[1]);
  ex.fail_run[ids[3]] = HGF_E_DEVICE;
  const hgf_status st = s.admit(ex);
  CHECK(st == HGF_E_DEVICE);  // the failed launch is reported
  std::map<int64_t, int> status;
  for (int it = 0; it < 100 && s.completed() < 5; ++it)
    for (auto& c : poll_all(s, ex)) status[c.id] = c.status;
  CHECK(s.completed() == 5);
  CHECK(status.size() == 5);
  CHECK(status[ids[0]] == HGF_OK);
  CHECK(status[ids[1]] == HGF_E_DEVICE);
  CHECK(status[ids[2]] == HGF_OK);
  CHECK(status[ids[3]] == HGF_E_DEVICE);
  CHECK(status[ids[4]] == HGF_OK);
  CHECK(s.arena().used() == 0);
  CHECK(ex.released == 5);
}

// Slot choice: each admitted job goes to the slot with the least running work.
void scenario_slots() {
  FakeExec ex;
  ex.arena = 1 << 20;
  ex.held = true;
  Scheduler<Payload> s(1 << 20, 3, 16);
  int64_t id;
  CHECK(s.submit(job(100, 10.0), &id) == HGF_OK);
  CHECK(s.submit(job(100, 1.0), &id) == HGF_OK);
  CHECK(s.submit(job(100, 1.0), &id) == HGF_OK);
  CHECK(s.submit(job(100, 1.0), &id) == HGF_OK);
  CHECK(s.admit(ex) == HGF_OK);
  std::vector<int> slot_of;
  for (auto& j : s.running()) slot_of.push_back(j.slot);
  // 10 -> slot 0, 1 -> slot 1, 1 -> slot 2, then the least-loaded (slot 1)
  CHECK((slot_of == std::vector<int>{0, 1, 2, 1}));
  ex.held = false;
  CHECK(s.drain(ex) == HGF_OK);
}

// A long randomised stream: jobs of random size (some larger than the arena),
// random launch failures and device errors, a device that is held now and
// then.  Every queued job completes exactly once with the expected status,
// launches follow submission order, ranges never overlap (checked by the
// executor), the queue bound holds and the arena drains back to one range.
void scenario_random() {
  uint64_t state = 0x9e3779b97f4a7c15ull;
  auto rnd = [&](uint64_t m) {
    state = state * 6364136223846793005ull + 1442695040888963407ull;
    return static_cast<size_t>((state >> 33) % m);
  };
  FakeExec ex;
  ex.arena = 1 << 16;
  constexpr int kMaxQueue = 8;
  Scheduler<Payload> s(ex.arena, 4, kMaxQueue);
  std::vector<int64_t> queued;
  std::map<int64_t, hgf_status> expect;
  std::map<int64_t, int> seen;
  std::map<int64_t, int> status;
  auto collect = [&](const std::vector<hgf_completion>& cs) {
    for (const auto& c : cs) {
      ++seen[c.id];
      status[c.id] = c.status;
    }
  };
  for (int it = 0; it < 4000; ++it) {
    ex.held = rnd(8) == 0;
    if (rnd(3) != 0) {
      const size_t bytes = 1 + rnd(ex.arena + ex.arena / 8);
      const size_t pending_before = s.pending().size();
      int64_t id = -1;
      const hgf_status r = s.submit(job(bytes, 1.0 + static_cast<double>(rnd(5))), &id);
      if (r == HGF_OK) {
        queued.push_back(id);
        expect[id] = HGF_OK;
        const size_t f = rnd(20);
        if (f == 0) {
          ex.fail_launch.insert(id);
          expect[id] = HGF_E_DEVICE;
        } else if (f == 1) {
          ex.fail_run[id] = HGF_E_DEVICE;
          expect[id] = HGF_E_DEVICE;
        }
      } else if (r == HGF_E_BUSY) {
        CHECK(static_cast<int>(pending_before) >= kMaxQueue);
      } else {
        CHECK(r == HGF_E_NOMEM);
        CHECK(hgf::sched::arena_align(bytes) > ex.arena);
      }
    }
    CHECK(static_cast<int>(s.pending().size()) <= kMaxQueue);
    CHECK(s.arena().used() <= ex.arena);
    collect(poll_all(s, ex));
  }
  ex.held = false;
  (void)s.drain(ex);
  for (int it = 0; it < 1000 && s.done_count() > 0; ++it) collect(poll_all(s, ex));
  CHECK(s.pending().empty() && s.running().empty());
  CHECK(queued.size() > 100);
  for (int64_t id : queued) {
    CHECK(seen[id] == 1);
    CHECK(status[id] == expect[id]);
  }
  CHECK(seen.size() == queued.size());
  // launches (failed ones excluded) in submission order
  std::vector<int64_t> ok_launch;
  for (int64_t id : queued)
    if (!ex.fail_launch.count(id)) ok_launch.push_back(id);
  CHECK(ex.launched == ok_launch);
  CHECK(ex.released == static_cast<int>(queued.size()));
  CHECK(s.arena().used() == 0);
  CHECK(s.arena().free_ranges() == 1);
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 2) {
    std::fprintf(stderr, "usage: %s fifo|alloc_failure|slow_device|failures|slots|random\n", argv[0]);
    return 2;
  }
  const std::string sc = argv[1];
  if (sc == "fifo") scenario_fifo();
  else if (sc == "alloc_failure") scenario_alloc_failure();
  else if (sc == "slow_device") scenario_slow_device();
  else if (sc == "failures") scenario_failures();
  else if (sc == "slots") scenario_slots();
  else if (sc == "random") scenario_random();
  else {
    std::fprintf(stderr, "unknown scenario %s\n", sc.c_str());
    return 2;
  }
  if (g_failures != 0) return 1;
  std::printf("ok %s\n", sc.c_str());
  return 0;
}
