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
// The queue, the arena and the slot choice are the host-only scheduler of
// sched.hpp; this unit is its HIP executor.  A request computes exactly what
// hgf_filter computes for the same parameters and tuning table: results do
// not depend on the mix it ran in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "runtime.hpp"
#include "sched.hpp"

using namespace hgf;

namespace {

// What the HIP executor keeps per request.
struct Request {
  hgf_params params{};
  Plan plan;
  const float* guide = nullptr;
  const void* cost = nullptr;
  float* out = nullptr;
  int32_t* labels = nullptr;
  hipEvent_t ready = nullptr;  // inputs ready on the submitting stream
  hipEvent_t start = nullptr, done = nullptr;
};

using Job = sched::Job<Request>;

}  // namespace

struct hgf_server;

namespace {

// The executor of the scheduler: runs a request's whole path on its slot
// stream in its arena range, bracketed by timing events.
struct HipExec {
  hgf_server* s;
  hgf_status launch(Job& j);
  int query(Job& j, bool wait, hgf_completion* c);
  void release(Job& j);
};

}  // namespace

struct hgf_server {
  hgf_context* ctx = nullptr;
  std::vector<hipStream_t> streams;
  void* base = nullptr;
  size_t arena_bytes = 0;
  sched::Scheduler<Request>* sch = nullptr;
  hipEvent_t epoch = nullptr;
  hipStream_t clock = nullptr;  // holds no work: events on it complete at once
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

hgf_status HipExec::launch(Job& j) {
  Request& r = j.payload;
  hipStream_t st = s->streams[j.slot];
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
                        static_cast<char*>(s->base) + j.off, st);
  }
  if (status == HGF_OK && hipEventRecord(r.done, st) != hipSuccess)
    status = fail(HGF_E_DEVICE, "hipEventRecord");
  // on failure, what already launched must finish before the arena range is
  // reused
  if (status != HGF_OK) (void)hipStreamSynchronize(st);
  return status;
}

int HipExec::query(Job& j, bool wait, hgf_completion* c) {
  Request& r = j.payload;
  const hipError_t e = wait ? hipEventSynchronize(r.done) : hipEventQuery(r.done);
  if (e == hipErrorNotReady) return 0;
  if (e != hipSuccess) {
    c->status = device_fail(e, "request");
    return 1;
  }
  float a = 0.f, b = 0.f;
  (void)hipEventElapsedTime(&a, s->epoch, r.start);
  (void)hipEventElapsedTime(&b, s->epoch, r.done);
  c->status = HGF_OK;
  c->start_ms = a;
  c->end_ms = b;
  return 1;
}

void HipExec::release(Job& j) {
  Request& r = j.payload;
  if (r.start != nullptr) s->spare.push_back(r.start);
  if (r.done != nullptr) s->spare.push_back(r.done);
  if (r.ready != nullptr) (void)hipEventDestroy(r.ready);
  r.start = r.done = r.ready = nullptr;
}

hgf_context* ctx_of(const hgf_server* s) { return s != nullptr ? s->ctx : nullptr; }

void destroy_server(hgf_server* s) {
  for (hipStream_t h : s->streams) (void)hipStreamSynchronize(h);
  if (s->sch != nullptr) {
    HipExec ex{s};
    for (const Job& j : s->sch->running()) {
      Job k = j;
      ex.release(k);
    }
    for (const Job& j : s->sch->pending()) {
      Job k = j;
      ex.release(k);
    }
    delete s->sch;
  }
  for (hipEvent_t e : s->spare) (void)hipEventDestroy(e);
  if (s->epoch != nullptr) (void)hipEventDestroy(s->epoch);
  for (hipStream_t h : s->streams) (void)hipStreamDestroy(h);
  if (s->clock != nullptr) (void)hipStreamDestroy(s->clock);
  ctx_free(s->ctx, s->base, s->arena_bytes);
  delete s;
}

}  // namespace

extern "C" {

hgf_status hgf_server_create(hgf_context* ctx, int32_t slots, size_t arena_bytes,
                             int32_t max_queue, hgf_server** out) {
  return guarded(ctx, [&]() -> hgf_status {
    if (ctx == nullptr || out == nullptr) return fail(HGF_E_INVALID, "context or out is NULL");
    if (slots < 1 || slots > 16) return fail(HGF_E_INVALID, "slots must be in [1, 16]");
    if (max_queue < 1) return fail(HGF_E_INVALID, "max_queue must be >= 1");
    if (arena_bytes < kAlign) return fail(HGF_E_INVALID, "arena_bytes too small");
    *out = nullptr;
    hgf_server* s = new (std::nothrow) hgf_server();
    if (s == nullptr) return fail(HGF_E_NOMEM, "host allocation");
    s->ctx = ctx;
    s->arena_bytes = align_up(arena_bytes);
    hgf_status st = ctx_alloc(ctx, s->arena_bytes, &s->base);
    if (st != HGF_OK) {
      s->arena_bytes = 0;
      destroy_server(s);
      return st;
    }
    s->sch = new (std::nothrow) sched::Scheduler<Request>(s->arena_bytes, slots, max_queue);
    if (s->sch == nullptr) st = fail(HGF_E_NOMEM, "host allocation");
    for (int i = 0; i < slots && st == HGF_OK; ++i) {
      hipStream_t h = nullptr;
      if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess) {
        st = fail(HGF_E_DEVICE, "hipStreamCreate");
        break;
      }
      s->streams.push_back(h);
    }
    if (st == HGF_OK && hipStreamCreateWithFlags(&s->clock, hipStreamNonBlocking) != hipSuccess)
      st = fail(HGF_E_DEVICE, "hipStreamCreate");
    if (st == HGF_OK && (hipEventCreate(&s->epoch) != hipSuccess ||
                         hipEventRecord(s->epoch, s->clock) != hipSuccess ||
                         hipEventSynchronize(s->epoch) != hipSuccess))
      st = fail(HGF_E_DEVICE, "epoch event");
    if (st != HGF_OK) {
      destroy_server(s);
      return st;
    }
    *out = s;
    return HGF_OK;
  });
}

void hgf_server_destroy(hgf_server* s) {
  if (s == nullptr) return;
  try {
    destroy_server(s);
  } catch (...) {
  }
}

hgf_status hgf_server_submit(hgf_server* s, const hgf_params* params, const float* guide,
                             const void* cost, float* out, int32_t* labels, void* hip_stream,
                             int64_t* id) {
  return guarded(ctx_of(s), [&]() -> hgf_status {
    if (s == nullptr || id == nullptr) return fail(HGF_E_INVALID, "server or id is NULL");
    MonoTable t;
    hgf_status st = validate(params, &t);
    if (st != HGF_OK) return st;
    if (guide == nullptr || cost == nullptr) return fail(HGF_E_INVALID, "guide or cost is NULL");
    if (out == nullptr && labels == nullptr) return fail(HGF_E_INVALID, "nothing to compute");
    Job j;
    Request& r = j.payload;
    r.params = *params;
    r.plan = make_plan(params, t, (params->num_labels + 63) / 64, s->ctx->group_bytes);
    r.guide = guide;
    r.cost = cost;
    r.out = out;
    r.labels = labels;
    j.bytes = r.plan.total;
    j.work = static_cast<double>(r.plan.P) * r.plan.L * (r.plan.n + 1);
    st = take_event(s, false, &r.ready);
    if (st != HGF_OK) return st;
    if (hipEventRecord(r.ready, static_cast<hipStream_t>(hip_stream)) != hipSuccess) {
      (void)hipEventDestroy(r.ready);
      return fail(HGF_E_DEVICE, "hipEventRecord");
    }
    const hipEvent_t ready = r.ready;
    const size_t need = r.plan.total;
    st = s->sch->submit(std::move(j), id);
    if (st != HGF_OK) {
      (void)hipEventDestroy(ready);
      if (st == HGF_E_BUSY) return fail(st, "request queue is full");
      return fail(st, "request workspace (%zu B) exceeds the serving arena (%zu B)", need,
                  s->arena_bytes);
    }
    HipExec ex{s};
    (void)s->sch->retire(ex, false);
    return s->sch->admit(ex);
  });
}

hgf_status hgf_server_poll(hgf_server* s, hgf_completion* done, int32_t max_done,
                           int32_t* count) {
  return guarded(ctx_of(s), [&]() -> hgf_status {
    if (s == nullptr || count == nullptr) return fail(HGF_E_INVALID, "server or count is NULL");
    HipExec ex{s};
    int c = 0;
    const hgf_status st = s->sch->poll(ex, done, max_done, &c);
    *count = c;
    return st;
  });
}

hgf_status hgf_server_drain(hgf_server* s) {
  return guarded(ctx_of(s), [&]() -> hgf_status {
    if (s == nullptr) return fail(HGF_E_INVALID, "server is NULL");
    HipExec ex{s};
    return s->sch->drain(ex);
  });
}

hgf_status hgf_server_now(hgf_server* s, double* ms) {
  return guarded(ctx_of(s), [&]() -> hgf_status {
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
  });
}

hgf_status hgf_server_stats(const hgf_server* s, hgf_server_info* out) {
  return guarded(ctx_of(s), [&]() -> hgf_status {
    if (s == nullptr || out == nullptr) return fail(HGF_E_INVALID, "server or out is NULL");
    out->pending = static_cast<int32_t>(s->sch->pending().size());
    out->running = static_cast<int32_t>(s->sch->running().size());
    out->completed = s->sch->completed();
    out->arena_bytes = s->arena_bytes;
    out->arena_in_use = s->sch->arena().used();
    out->arena_peak = s->sch->arena().peak();
    return HGF_OK;
  });
}

}  // extern "C"
