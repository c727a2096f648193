// Host-only scheduler of the serving form: admission by device-memory budget,
// a bounded strict-FIFO queue, least-loaded slot choice and retirement.  It
// holds no device state and includes no HIP header: the device work is done
// by an executor, a template parameter (the HIP one in serve.hip; the tests
// drive it with a fake executor on the CPU).
//
// Executor interface, for jobs Job<P>:
//   hgf_status launch(Job<P>& j)   start j on slot j.slot with its arena range
//                                  at j.off; on failure nothing of j may
//                                  remain queued on the device
//   int query(Job<P>& j, bool wait, hgf_completion* c)
//                                  1 when j has finished (c->status and the
//                                  device-clock times filled in), 0 if not
//                                  yet; wait = block until finished
//   void release(Job<P>& j)        drop the job's executor resources (after
//                                  query returned 1, or after a failed launch)
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <vector>

#include "../../include/hgf.h"

namespace hgf {
namespace sched {

constexpr size_t kArenaAlign = 256;
inline size_t arena_align(size_t v) { return (v + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// First-fit allocator over [0, size) with coalescing of freed ranges.
class Arena {
 public:
  explicit Arena(size_t size = 0) : size_(size) {
    if (size > 0) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = arena_align(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t next = it->first + bytes;
      free_.erase(it);
      if (rest > 0) free_[next] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = arena_align(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t size() const { return size_; }
  size_t free_ranges() const { return free_.size(); }

 private:
  size_t size_;
  size_t used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

template <class P>
struct Job {
  int64_t id = 0;
  size_t bytes = 0;  // arena bytes the job holds while it runs
  double work = 0.0; // load weight for the slot choice
  size_t off = 0;
  int slot = -1;
  P payload{};
};

template <class P>
class Scheduler {
 public:
  Scheduler(size_t arena_bytes, int slots, int max_queue)
      : arena_(arena_align(arena_bytes)), slot_work_(slots, 0.0), max_queue_(max_queue) {}

  // Queue a job.  HGF_E_BUSY: max_queue jobs already wait; HGF_E_NOMEM: it
  // can never fit in the arena.  Nothing is queued on failure.
  hgf_status submit(Job<P> j, int64_t* id) {
    if (static_cast<int>(pending_.size()) >= max_queue_) return HGF_E_BUSY;
    if (arena_align(j.bytes) > arena_.size()) return HGF_E_NOMEM;
    j.id = next_id_++;
    *id = j.id;
    pending_.push_back(std::move(j));
    return HGF_OK;
  }

  // Launch the jobs at the head of the queue while their arena ranges fit
  // (strict FIFO: a job that does not fit holds back every later one, so no
  // job starves).  A failed launch completes its job with the error and
  // releases its range; the error is returned after the queue moved on.
  template <class E>
  hgf_status admit(E& ex) {
    hgf_status first = HGF_OK;
    while (!pending_.empty()) {
      Job<P>& q = pending_.front();
      size_t off = 0;
      if (!arena_.alloc(q.bytes, &off)) break;
      Job<P> j = std::move(q);
      pending_.pop_front();
      j.off = off;
      j.slot = static_cast<int>(std::min_element(slot_work_.begin(), slot_work_.end()) -
                                slot_work_.begin());
      const hgf_status st = ex.launch(j);
      if (st != HGF_OK) {
        arena_.release(j.off, j.bytes);
        ex.release(j);
        done_.push_back(hgf_completion{j.id, st, j.slot, 0.0, 0.0});
        ++completed_;
        if (first == HGF_OK) first = st;
        continue;
      }
      slot_work_[j.slot] += j.work;
      running_.push_back(std::move(j));
    }
    return first;
  }

  // Retire finished jobs (wait: until every running job has finished).
  // Returns the first error status among the retired jobs.
  template <class E>
  hgf_status retire(E& ex, bool wait) {
    hgf_status first = HGF_OK;
    for (size_t i = 0; i < running_.size();) {
      Job<P>& r = running_[i];
      hgf_completion c{r.id, HGF_OK, r.slot, 0.0, 0.0};
      if (ex.query(r, wait, &c) == 0) {
        ++i;
        continue;
      }
      c.id = r.id;
      c.slot = r.slot;
      if (c.status != HGF_OK && first == HGF_OK) first = static_cast<hgf_status>(c.status);
      done_.push_back(c);
      ++completed_;
      arena_.release(r.off, r.bytes);
      slot_work_[r.slot] -= r.work;
      ex.release(r);
      running_[i] = std::move(running_.back());
      running_.pop_back();
    }
    return first;
  }

  // Retire, admit and hand out up to max_done completion records, oldest first.
  template <class E>
  hgf_status poll(E& ex, hgf_completion* out, int max_done, int* count) {
    hgf_status st = retire(ex, false);
    const hgf_status st2 = admit(ex);
    if (st == HGF_OK) st = st2;
    *count = 0;
    while (out != nullptr && *count < max_done && !done_.empty()) {
      out[(*count)++] = done_.front();
      done_.pop_front();
    }
    return st;
  }

  // Until every submitted job has completed.
  template <class E>
  hgf_status drain(E& ex) {
    hgf_status st = HGF_OK;
    while (!running_.empty() || !pending_.empty()) {
      const hgf_status a = retire(ex, true);
      const hgf_status b = admit(ex);
      if (st == HGF_OK) st = a != HGF_OK ? a : b;
      // a pending job that cannot fit an empty arena cannot exist (submit
      // refuses it), so an empty running set means the queue drained
      if (running_.empty() && !pending_.empty() && arena_.used() == 0) break;
    }
    return st;
  }

  const std::deque<Job<P>>& pending() const { return pending_; }
  const std::vector<Job<P>>& running() const { return running_; }
  size_t done_count() const { return done_.size(); }
  int64_t completed() const { return completed_; }
  const Arena& arena() const { return arena_; }

 private:
  Arena arena_;
  std::vector<double> slot_work_;
  int max_queue_;
  int64_t next_id_ = 0;
  int64_t completed_ = 0;
  std::deque<Job<P>> pending_;
  std::vector<Job<P>> running_;
  std::deque<hgf_completion> done_;
};

}  // namespace sched
}  // namespace hgf
