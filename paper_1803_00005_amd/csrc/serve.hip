// Serving form: requests of mixed size, label count and cost dtype arrive one
// at a time and are filtered as soon as device memory allows.
//
// Admission is by HBM budget: every request's workspace (its resident
// guidance statistics, its coefficient workspace and its WTA keys) is carved
// out of one device arena with a first-fit allocator; a request that does
// not fit waits in a bounded FIFO queue (strict order, so no request starves)
// and is admitted when earlier ones retire.  Admitted requests run the whole
// path on one of a few slot streams (the least-loaded one), so requests join
// and leave the running set one by one and overlap on the device (continuous
// batching: no batch barrier).  Completion is detected with events; each
// completion record carries the device-clock start and end times relative to
// the server's epoch, from which the caller derives latency percentiles.
//
// A request computes exactly what hgf_filter computes for the same
// parameters and tuning table: results do not depend on the mix it ran in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <map>
#include <vector>

#include "runtime.hpp"

using namespace hgf;

namespace {

// First-fit allocator over [0, size) with coalescing of freed ranges.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at_ = it->first + bytes;
      free_.erase(it);
      if (rest > 0) free_[at_] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes);
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

 private:
  size_t size_;
  size_t used_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;
};

struct Request {
  int64_t id = 0;
  hgf_params params{};
  Plan plan;
  const float* guide = nullptr;
  const void* cost = nullptr;
  float* out = nullptr;
  int32_t* labels = nullptr;
  hipEvent_t ready = nullptr;  // inputs ready on the submitting stream
  hipEvent_t start = nullptr, done = nullptr;
  size_t off = 0;
  int slot = -1;
  double work = 0.0;
};

}  // namespace

struct hgf_server {
  hgf_context* ctx = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<double> slot_work;
  void* base = nullptr;
  Arena arena{0};
  int max_queue = 0;
  hipEvent_t epoch = nullptr;
  hipStream_t clock = nullptr;  // holds no work: events on it complete at once
  int64_t next_id = 0;
  int64_t completed = 0;
  std::deque<Request> pending;
  std::vector<Request> running;
  std::deque<hgf_completion> done;
  std::vector<hipEvent_t> spare;
};

namespace {

hgf_status take_event(hgf_server* s, bool timed, hipEvent_t* e) {
  if (timed && !s->spare.empty()) {
    *e = s->spare.back();
    s->spare.pop_back();
    return HGF_OK;
  }
  HGF_TRY(hipEventCreateWithFlags(e, timed ? hipEventDefault : hipEventDisableTiming),
          "hipEventCreate");
  return HGF_OK;
}

// Launch every admissible request at the head of the queue.
hgf_status admit(hgf_server* s) {
  while (!s->pending.empty()) {
    Request& q = s->pending.front();
    size_t off = 0;
    if (!s->arena.alloc(q.plan.total, &off)) break;  // strict FIFO
    Request r = q;
    s->pending.pop_front();
    r.off = off;
    r.slot = static_cast<int>(std::min_element(s->slot_work.begin(), s->slot_work.end()) -
                              s->slot_work.begin());
    hipStream_t st = s->streams[r.slot];
    hgf_status status = take_event(s, true, &r.start);
    if (status == HGF_OK) status = take_event(s, true, &r.done);
    if (status == HGF_OK && hipStreamWaitEvent(st, r.ready, 0) != hipSuccess)
      status = fail(HGF_E_DEVICE, "hipStreamWaitEvent");
    if (status == HGF_OK && hipEventRecord(r.start, st) != hipSuccess)
      status = fail(HGF_E_DEVICE, "hipEventRecord");
    if (status == HGF_OK) {
      const int cost_ld = r.params.cost_ld ? r.params.cost_ld : r.params.num_labels;
      const int out_ld = r.params.out_ld ? r.params.out_ld : r.params.num_labels;
      status = run_filter(s->ctx, r.plan, r.guide, r.cost, cost_ld, r.out, out_ld, r.labels,
                          static_cast<char*>(s->base) + off, st);
    }
    if (status == HGF_OK && hipEventRecord(r.done, st) != hipSuccess)
      status = fail(HGF_E_DEVICE, "hipEventRecord");
    if (status != HGF_OK) {
      // nothing of this request is left queued except what already launched;
      // wait for it so the arena range can be reused safely
      (void)hipStreamSynchronize(st);
      s->arena.release(off, r.plan.total);
      hgf_completion c{r.id, status, r.slot, 0.0, 0.0};
      s->done.push_back(c);
      if (r.start) s->spare.push_back(r.start);
      if (r.done) s->spare.push_back(r.done);
      (void)hipEventDestroy(r.ready);
      ++s->completed;
      return status;
    }
    s->slot_work[r.slot] += r.work;
    s->running.push_back(r);
  }
  return HGF_OK;
}

// Retire finished requests; `wait` blocks until every running one is done.
hgf_status retire(hgf_server* s, bool wait) {
  hgf_status first = HGF_OK;
  for (size_t i = 0; i < s->running.size();) {
    Request& r = s->running[i];
    hipError_t e = wait ? hipEventSynchronize(r.done) : hipEventQuery(r.done);
    if (e == hipErrorNotReady) {
      ++i;
      continue;
    }
    hgf_completion c{r.id, HGF_OK, r.slot, 0.0, 0.0};
    if (e != hipSuccess) {
      c.status = device_fail(e, "request");
      if (first == HGF_OK) first = static_cast<hgf_status>(c.status);
    } else {
      float a = 0.f, b = 0.f;
      (void)hipEventElapsedTime(&a, s->epoch, r.start);
      (void)hipEventElapsedTime(&b, s->epoch, r.done);
      c.start_ms = a;
      c.end_ms = b;
    }
    s->done.push_back(c);
    ++s->completed;
    s->arena.release(r.off, r.plan.total);
    s->slot_work[r.slot] -= r.work;
    s->spare.push_back(r.start);
    s->spare.push_back(r.done);
    (void)hipEventDestroy(r.ready);
    s->running[i] = s->running.back();
    s->running.pop_back();
  }
  return first;
}

}  // namespace

extern "C" {

hgf_status hgf_server_create(hgf_context* ctx, int32_t slots, size_t arena_bytes,
                             int32_t max_queue, hgf_server** out) {
  if (ctx == nullptr || out == nullptr) return fail(HGF_E_INVALID, "context or out is NULL");
  if (slots < 1 || slots > 16) return fail(HGF_E_INVALID, "slots must be in [1, 16]");
  if (max_queue < 1) return fail(HGF_E_INVALID, "max_queue must be >= 1");
  if (arena_bytes < kAlign) return fail(HGF_E_INVALID, "arena_bytes too small");
  *out = nullptr;
  auto* s = new hgf_server();
  s->ctx = ctx;
  s->max_queue = max_queue;
  arena_bytes = align_up(arena_bytes);
  hgf_status st = ctx_alloc(ctx, arena_bytes, &s->base);
  if (st != HGF_OK) {
    delete s;
    return st;
  }
  s->arena = Arena(arena_bytes);
  for (int i = 0; i < slots; ++i) {
    hipStream_t h = nullptr;
    if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess) {
      st = fail(HGF_E_DEVICE, "hipStreamCreate");
      break;
    }
    s->streams.push_back(h);
    s->slot_work.push_back(0.0);
  }
  if (st == HGF_OK && hipStreamCreateWithFlags(&s->clock, hipStreamNonBlocking) != hipSuccess)
    st = fail(HGF_E_DEVICE, "hipStreamCreate");
  if (st == HGF_OK && (hipEventCreate(&s->epoch) != hipSuccess ||
                       hipEventRecord(s->epoch, s->clock) != hipSuccess ||
                       hipEventSynchronize(s->epoch) != hipSuccess))
    st = fail(HGF_E_DEVICE, "epoch event");
  if (st != HGF_OK) {
    hgf_server_destroy(s);
    return st;
  }
  *out = s;
  return HGF_OK;
}

void hgf_server_destroy(hgf_server* s) {
  if (s == nullptr) return;
  for (hipStream_t h : s->streams) (void)hipStreamSynchronize(h);
  for (Request& r : s->running) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.done);
    (void)hipEventDestroy(r.ready);
  }
  for (Request& r : s->pending) (void)hipEventDestroy(r.ready);
  for (hipEvent_t e : s->spare) (void)hipEventDestroy(e);
  if (s->epoch != nullptr) (void)hipEventDestroy(s->epoch);
  for (hipStream_t h : s->streams) (void)hipStreamDestroy(h);
  if (s->clock != nullptr) (void)hipStreamDestroy(s->clock);
  ctx_free(s->ctx, s->base, s->arena.size());
  delete s;
}

hgf_status hgf_server_submit(hgf_server* s, const hgf_params* params, const float* guide,
                             const void* cost, float* out, int32_t* labels, void* hip_stream,
                             int64_t* id) {
  if (s == nullptr || id == nullptr) return fail(HGF_E_INVALID, "server or id is NULL");
  MonoTable t;
  hgf_status st = validate(params, &t);
  if (st != HGF_OK) return st;
  if (guide == nullptr || cost == nullptr) return fail(HGF_E_INVALID, "guide or cost is NULL");
  if (out == nullptr && labels == nullptr) return fail(HGF_E_INVALID, "nothing to compute");
  if (static_cast<int>(s->pending.size()) >= s->max_queue)
    return fail(HGF_E_BUSY, "request queue is full");
  Request r;
  r.params = *params;
  r.plan = make_plan(params, t, (params->num_labels + 63) / 64);
  if (align_up(r.plan.total) > s->arena.size())
    return fail(HGF_E_NOMEM, "request workspace (" + std::to_string(r.plan.total) +
                                 " B) exceeds the serving arena");
  r.guide = guide;
  r.cost = cost;
  r.out = out;
  r.labels = labels;
  r.work = static_cast<double>(r.plan.P) * r.plan.L * (r.plan.n + 1);
  st = take_event(s, false, &r.ready);
  if (st != HGF_OK) return st;
  if (hipEventRecord(r.ready, static_cast<hipStream_t>(hip_stream)) != hipSuccess) {
    (void)hipEventDestroy(r.ready);
    return fail(HGF_E_DEVICE, "hipEventRecord");
  }
  r.id = s->next_id++;
  *id = r.id;
  s->pending.push_back(r);
  (void)retire(s, false);
  return admit(s);
}

hgf_status hgf_server_poll(hgf_server* s, hgf_completion* done, int32_t max_done,
                           int32_t* count) {
  if (s == nullptr || count == nullptr) return fail(HGF_E_INVALID, "server or count is NULL");
  *count = 0;
  hgf_status st = retire(s, false);
  const hgf_status st2 = admit(s);
  if (st == HGF_OK) st = st2;
  while (done != nullptr && *count < max_done && !s->done.empty()) {
    done[(*count)++] = s->done.front();
    s->done.pop_front();
  }
  return st;
}

hgf_status hgf_server_drain(hgf_server* s) {
  if (s == nullptr) return fail(HGF_E_INVALID, "server is NULL");
  hgf_status st = HGF_OK;
  while (!s->running.empty() || !s->pending.empty()) {
    hgf_status a = retire(s, true);
    hgf_status b = admit(s);
    if (st == HGF_OK) st = a != HGF_OK ? a : b;
    if (b != HGF_OK && s->running.empty()) break;
  }
  return st;
}

hgf_status hgf_server_now(hgf_server* s, double* ms) {
  if (s == nullptr || ms == nullptr) return fail(HGF_E_INVALID, "server or ms is NULL");
  hipEvent_t e = nullptr;
  hgf_status st = take_event(s, true, &e);
  if (st != HGF_OK) return st;
  float t = 0.f;
  if (hipEventRecord(e, s->clock) != hipSuccess || hipEventSynchronize(e) != hipSuccess ||
      hipEventElapsedTime(&t, s->epoch, e) != hipSuccess)
    st = fail(HGF_E_DEVICE, "clock event");
  s->spare.push_back(e);
  *ms = t;
  return st;
}

hgf_status hgf_server_stats(const hgf_server* s, hgf_server_info* out) {
  if (s == nullptr || out == nullptr) return fail(HGF_E_INVALID, "server or out is NULL");
  out->pending = static_cast<int32_t>(s->pending.size());
  out->running = static_cast<int32_t>(s->running.size());
  out->completed = s->completed;
  out->arena_bytes = s->arena.size();
  out->arena_in_use = s->arena.used();
  out->arena_peak = s->arena.peak();
  return HGF_OK;
}

}  // extern "C"
