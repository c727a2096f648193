// Batched form: many images of uneven size and label count filtered by one
// replay of a hipGraph.
//
// The batch is spread over a few worker streams (largest images first, each
// to the least-loaded stream).  Each image runs the whole hot path on its
// stream in the context's worker workspace; images on different streams
// overlap on the device.  The sequence is captured once (fork from the
// caller's stream, join back) and the instantiated graph is cached with the
// batch's signature (parameters, buffers, tuning); a call with the same
// signature replays it with one hipGraphLaunch.  Every node is a kernel
// launch (no memset nodes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "runtime.hpp"

namespace hgf {
namespace {

constexpr int kBatchStreams = 4;

template <typename T>
void append(std::vector<unsigned char>& v, const T& x) {
  const auto* p = reinterpret_cast<const unsigned char*>(&x);
  v.insert(v.end(), p, p + sizeof(T));
}

hgf_status ensure_workers(hgf_context* ctx, int nstreams, const std::vector<size_t>& need) {
  if (ctx->capture == nullptr)
    HGF_TRY(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking), "hipStreamCreate");
  while (static_cast<int>(ctx->workers.size()) < nstreams) {
    hipStream_t st = nullptr;
    HGF_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "hipStreamCreate");
    ctx->workers.push_back(st);
    ctx->worker_ws.push_back(nullptr);
    ctx->worker_ws_bytes.push_back(0);
  }
  for (int k = 0; k < nstreams; ++k) {
    if (ctx->worker_ws_bytes[k] >= need[k]) continue;
    // the old buffer may be in use by the last graph launch
    wait_used(ctx->batch_done);
    ctx->graph.reset();             // a cached graph refers to the old buffer
    ctx_free(ctx, ctx->worker_ws[k], ctx->worker_ws_bytes[k]);
    ctx->worker_ws[k] = nullptr;
    ctx->worker_ws_bytes[k] = 0;
    void* p = nullptr;
    const hgf_status st = ctx_alloc(ctx, need[k], &p);
    if (st != HGF_OK) return st;
    ctx->worker_ws[k] = p;
    ctx->worker_ws_bytes[k] = need[k];
  }
  return HGF_OK;
}

}  // namespace
}  // namespace hgf

using namespace hgf;

void hgf_release_batch_resources(hgf_context* ctx) {
  ctx->graph.reset();
  for (size_t k = 0; k < ctx->workers.size(); ++k) {
    ctx_free(ctx, ctx->worker_ws[k], ctx->worker_ws_bytes[k]);
    (void)hipStreamDestroy(ctx->workers[k]);
  }
  if (ctx->capture != nullptr) (void)hipStreamDestroy(ctx->capture);
  ctx->capture = nullptr;
  ctx->workers.clear();
  ctx->worker_ws.clear();
  ctx->worker_ws_bytes.clear();
}

static hgf_status filter_batch(hgf_context* ctx, int32_t count, const hgf_params* params,
                               const float* const* guides, const void* const* costs,
                               float* const* outs, int32_t* const* labels, void* hip_stream) {
  if (ctx == nullptr) return fail(HGF_E_INVALID, "context is NULL");
  if (count < 0) return fail(HGF_E_INVALID, "count < 0");
  if (count == 0) return HGF_OK;
  if (params == nullptr || guides == nullptr || costs == nullptr)
    return fail(HGF_E_INVALID, "params, guides or costs is NULL");
  std::vector<Plan> plans(count);
  for (int i = 0; i < count; ++i) {
    MonoTable t;
    const hgf_status st = validate(&params[i], &t);
    if (st != HGF_OK) {
      char detail[400];
      std::snprintf(detail, sizeof(detail), "%s", thread_error());
      return fail(st, "image %d: %s", i, detail);
    }
    if (guides[i] == nullptr || costs[i] == nullptr)
      return fail(HGF_E_INVALID, "image %d: guide or cost is NULL", i);
    float* o = outs != nullptr ? outs[i] : nullptr;
    int32_t* l = labels != nullptr ? labels[i] : nullptr;
    if (o == nullptr && l == nullptr)
      return fail(HGF_E_INVALID, "image %d: nothing to compute", i);
    plans[i] = make_plan(&params[i], t, (params[i].num_labels + 63) / 64, ctx->group_bytes);
  }
  // largest-first assignment of images to worker streams
  const int nstreams = std::min<int>(kBatchStreams, count);
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  auto work = [&](int i) {
    return static_cast<double>(plans[i].P) * plans[i].L * (plans[i].n + 1);
  };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
  std::vector<int> stream_of(count, 0);
  std::vector<double> load(nstreams, 0.0);
  std::vector<size_t> need(nstreams, 0);
  for (int i : order) {
    const int k = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
    stream_of[i] = k;
    load[k] += work(i);
    need[k] = std::max(need[k], plans[i].total);
  }
  hgf_status st = ensure_workers(ctx, nstreams, need);
  if (st != HGF_OK) return st;

  std::vector<unsigned char> sig;
  append(sig, count);
  for (int i = 0; i < count; ++i) {
    append(sig, params[i]);
    append(sig, guides[i]);
    append(sig, costs[i]);
    append(sig, outs != nullptr ? outs[i] : nullptr);
    append(sig, labels != nullptr ? labels[i] : nullptr);
    append(sig, stream_of[i]);
    append(sig, tuned_target(ctx, kTuneCoef, plans[i]));
    append(sig, tuned_target(ctx, kTuneOut, plans[i]));
  }
  for (int k = 0; k < nstreams; ++k) append(sig, ctx->worker_ws[k]);

  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (ctx->graph == nullptr || ctx->graph->signature != sig) {
    // the previous graph may still be replaying on some stream
    if (ctx->graph != nullptr) wait_used(ctx->batch_done);
    ctx->graph.reset();
    auto g = std::make_unique<hgf_batch_graph>();
    g->signature = sig;
    g->events.resize(nstreams + 1, nullptr);
    for (auto& e : g->events)
      HGF_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    // Captured from the context's own origin stream (the caller's may be the
    // null stream, which cannot be captured); launched on the caller's.
    hipStream_t origin = ctx->capture;
    const bool timing = ctx->timing;
    ctx->timing = false;  // no timing events inside the captured graph
    HGF_TRY(hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal),
            "hipStreamBeginCapture");
    hgf_status cst = HGF_OK;
    if (hipEventRecord(g->events[nstreams], origin) != hipSuccess)
      cst = fail(HGF_E_DEVICE, "fork event");
    for (int k = 0; k < nstreams && cst == HGF_OK; ++k)
      if (hipStreamWaitEvent(ctx->workers[k], g->events[nstreams], 0) != hipSuccess)
        cst = fail(HGF_E_DEVICE, "fork wait");
    for (int i : order) {
      if (cst != HGF_OK) break;
      const Plan& pl = plans[i];
      const int k = stream_of[i];
      const int cost_ld = params[i].cost_ld ? params[i].cost_ld : params[i].num_labels;
      const int out_ld = params[i].out_ld ? params[i].out_ld : params[i].num_labels;
      cst = run_filter(ctx, pl, guides[i], costs[i], cost_ld, outs != nullptr ? outs[i] : nullptr,
                       out_ld, labels != nullptr ? labels[i] : nullptr, ctx->worker_ws[k],
                       ctx->workers[k]);
    }
    for (int k = 0; k < nstreams && cst == HGF_OK; ++k) {
      if (hipEventRecord(g->events[k], ctx->workers[k]) != hipSuccess ||
          hipStreamWaitEvent(origin, g->events[k], 0) != hipSuccess)
        cst = fail(HGF_E_DEVICE, "join");
    }
    const hipError_t ec = hipStreamEndCapture(origin, &g->graph);
    ctx->timing = timing;
    if (cst != HGF_OK) return cst;
    if (ec != hipSuccess) return device_fail(ec, "hipStreamEndCapture");
    HGF_TRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    ctx->graph = std::move(g);
  }
  HGF_TRY(hipGraphLaunch(ctx->graph->exec, s), "hipGraphLaunch");
  return mark_used(&ctx->batch_done, s);
}

extern "C" hgf_status hgf_filter_batch(hgf_context* ctx, int32_t count, const hgf_params* params,
                                       const float* const* guides, const void* const* costs,
                                       float* const* outs, int32_t* const* labels,
                                       void* hip_stream) {
  return guarded(ctx, [&] {
    return filter_batch(ctx, count, params, guides, costs, outs, labels, hip_stream);
  });
}
