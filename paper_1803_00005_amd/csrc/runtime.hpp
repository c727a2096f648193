// Host runtime shared by the C ABI translation units: argument validation,
// workspace plans, the context (device memory, stage timing, tuning table,
// cached batch graphs) and the launch sequences of the hot path.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/hgf.h"
#include "hgf_launch.hpp"

namespace hgf {

// ---------------------------------------------------------------------------
// errors: a thread-local detail string (printf-style, no allocation), copied
// into the context by the entry points (hgf_last_error)
// ---------------------------------------------------------------------------
hgf_status fail(hgf_status st, const char* fmt, ...) noexcept
    __attribute__((format(printf, 2, 3)));
hgf_status device_fail(hipError_t e, const char* where) noexcept;
const char* thread_error() noexcept;

#define HGF_TRY(expr, where)                                \
  do {                                                      \
    hipError_t e_ = (expr);                                 \
    if (e_ != hipSuccess) return ::hgf::device_fail(e_, where); \
  } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

template <typename T>
T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

int num_channels_impl(int m, int d, int basis);
bool build_table(int m, int d, int basis, MonoTable* t);

// ---------------------------------------------------------------------------
// workspace plan of one image
// ---------------------------------------------------------------------------
struct Plan {
  int n = 0, D = 0, PD = 0, K = 0, P = 0, H = 0, W = 0, R = 0, L = 0, reg = 0;
  int cost_type = 0;   // CostType
  int mode = 0;        // SolveMode
  double eps = 0.0;
  // label chunks of 64: of the whole volume (fixes the band partition), and
  // per launch group (bounded by the group size)
  int chunks_total = 0, chunks_per_launch = 0;
  size_t off_shift = 0, off_g64 = 0, off_g32 = 0, off_mu = 0, off_minv = 0;
  size_t off_x = 0, off_keys = 0, total = 0;
  size_t ws_chunk_bytes = 0;
  MonoTable table{};
  const float* g32(void* ws) const { return at<float>(ws, off_g32) + kGPad; }
};

hgf_status validate(const hgf_params* p, MonoTable* table);
// chunks_ws: label chunks the coefficient workspace must hold at most (the
// launch group is the smaller of that and group_bytes' worth).
constexpr size_t kDefaultGroupBytes = size_t(12) << 30;
Plan make_plan(const hgf_params* p, const MonoTable& table, int chunks_ws,
               size_t group_bytes = kDefaultGroupBytes);

// ---------------------------------------------------------------------------
// tuning: target block counts of the strip kernels, chosen by the autotuner
// per (kernel, n, radius, solve mode, cost dtype, image size class)
// ---------------------------------------------------------------------------
enum TuneKernel { kTuneCoef = 0, kTuneOut = 1, kTuneMoments = 2 };
using TuneKey = std::tuple<int, int, int, int, int, int>;
TuneKey tune_key(int kernel, const Plan& pl);
int size_class(int P);
constexpr int kDefaultTarget = 512;
// candidate values the autotuner times
const std::vector<int>& tune_candidates();

}  // namespace hgf

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
// A captured and instantiated batch, cached with the signature it was built
// for (parameters, buffers, stream assignment, tuning).
struct hgf_batch_graph {
  std::vector<unsigned char> signature;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<hipEvent_t> events;
  hgf_batch_graph() = default;
  hgf_batch_graph(const hgf_batch_graph&) = delete;
  hgf_batch_graph& operator=(const hgf_batch_graph&) = delete;
  ~hgf_batch_graph() {
    if (exec != nullptr) (void)hipGraphExecDestroy(exec);
    if (graph != nullptr) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : events)
      if (e != nullptr) (void)hipEventDestroy(e);
  }
};

struct hgf_context {
  int device = 0;
  size_t budget = 0;
  size_t allocated = 0;
  size_t group_bytes = hgf::kDefaultGroupBytes;
  char err[512] = {0};            // detail of the last failed call (hgf_last_error)
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  hipEvent_t scratch_used = nullptr;  // recorded after the last call that used scratch
  // stage timing (hgf_set_stage_timing)
  bool timing = false;
  struct Rec {
    int stage;
    hipEvent_t start, stop;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> spare;
  // tuning table (kernel config -> target blocks)
  std::map<hgf::TuneKey, int> tune;
  // batched form: worker streams, their workspaces and the cached graph
  hipStream_t capture = nullptr;  // origin stream of graph capture (never the null stream)
  std::vector<hipStream_t> workers;
  std::vector<void*> worker_ws;
  std::vector<size_t> worker_ws_bytes;
  std::unique_ptr<hgf_batch_graph> graph;
  hipEvent_t batch_done = nullptr;  // recorded after the last graph launch
};

struct hgf_guide {
  hgf_context* ctx = nullptr;
  hgf_params params{};
  hgf::Plan plan;
  void* base = nullptr;  // one plan-sized buffer: g32, mu, minv stay resident
  size_t bytes = 0;
  bool owns = true;      // false when the buffer belongs to a serving arena
  hipEvent_t used = nullptr;  // recorded after the last call that used the buffer
};

namespace hgf {

hgf_status ctx_alloc(hgf_context* ctx, size_t bytes, void** out);
void ctx_free(hgf_context* ctx, void* p, size_t bytes);
hgf_status ctx_scratch(hgf_context* ctx, size_t bytes, void** out);
// Record `*ev` (created on first use) on stream s: the point after which the
// memory used by work queued so far on s may be freed.
hgf_status mark_used(hipEvent_t* ev, hipStream_t s);
// Wait for the last mark of `ev` (nothing if it was never recorded).
void wait_used(hipEvent_t ev);

// Runs an entry point's body: no C++ exception leaves it (a failed host
// allocation becomes HGF_E_NOMEM), and a failure's detail string is kept in
// the context for hgf_last_error.
template <class F>
hgf_status guarded(hgf_context* ctx, F&& body) noexcept {
  hgf_status st;
  try {
    st = body();
  } catch (const std::bad_alloc&) {
    st = fail(HGF_E_NOMEM, "host memory allocation failed");
  } catch (...) {
    st = fail(HGF_E_DEVICE, "unexpected host exception");
  }
  if (st != HGF_OK && ctx != nullptr) {
    const char* e = thread_error();
    size_t i = 0;
    for (; i + 1 < sizeof(ctx->err) && e[i] != 0; ++i) ctx->err[i] = e[i];
    ctx->err[i] = 0;
  }
  return st;
}

int tuned_target(hgf_context* ctx, int kernel, const Plan& pl);

// The launch sequences (stream-ordered; every kernel on stream s).
hgf_status run_guide(hgf_context* ctx, const Plan& pl, const float* guide, void* ws,
                     hipStream_t s);
hgf_status run_labels(hgf_context* ctx, const Plan& pl, const void* cost, int cost_ld, float* out,
                      int out_ld, unsigned long long* keys, int32_t* labels, int label_base,
                      int count,
                      const float* g32, const void* minv, float* wsbuf,
                      hipStream_t s);
// Whole image: guide + labels + winner-takes-all into `labels`.
hgf_status run_filter(hgf_context* ctx, const Plan& pl, const float* guide, const void* cost,
                      int cost_ld, float* out, int out_ld, int32_t* labels, void* ws,
                      hipStream_t s);

}  // namespace hgf
