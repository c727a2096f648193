// C ABI of the HGF library (include/hgf.h): argument validation, workspace
// planning, device memory, stage timing and the launch sequence of the hot
// path.  The batched form, the autotuner and the server live in batch.hip,
// tune.hip and serve.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "runtime.hpp"

namespace hgf {
// Strips of (sin - 2R) output columns, label chunks, and as many bands as fit
// in target_blocks with every chunk of the volume in one launch (never more:
// a grid slightly larger than a multiple of the resident workgroup slots
// leaves a nearly empty last round).  Each band restarts the vertical running
// sums (2R + 1 rows of set-up), which the tuned targets keep in proportion
// for large images; small images take bands down to one row, so that their
// latency-bound strips run as more, shorter blocks.  At most kMaxBand rows
// bound the float32 drift of the running sums.
constexpr int kMinBand = 1;
constexpr int kMaxBand = 64;

StripGrid strip_grid_w(int H, int W, int R, int sin, int chunks, int chunks_total,
                       int target_blocks) {
  StripGrid g;
  const int sout = sin - 2 * R;
  g.strips = (W + sout - 1) / sout;
  g.chunks = chunks;
  const int per_band = std::max(1, g.strips * chunks_total);
  const int bands = std::max(1, target_blocks / per_band);
  int band_h = (H + bands - 1) / bands;
  band_h = std::min(kMaxBand, std::max(kMinBand, band_h));
  g.band_h = band_h;
  g.bands = (H + band_h - 1) / band_h;
  return g;
}

StripGrid strip_grid(int H, int W, int R, int chunks, int target_blocks) {
  return strip_grid_w(H, W, R, kStrip, chunks, chunks, target_blocks);
}

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local char g_last_error[512];

hgf_status fail(hgf_status st, const char* fmt, ...) noexcept {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return st;
}

hgf_status device_fail(hipError_t e, const char* where) noexcept {
  if (e == hipErrorNotSupported)
    return fail(HGF_E_UNSUPPORTED, "%s: configuration not compiled in", where);
  return fail(HGF_E_DEVICE, "%s: %s", where, hipGetErrorString(e));
}

const char* thread_error() noexcept { return g_last_error; }

// ---------------------------------------------------------------------------
// guidance basis (Sec. 4.2)
// ---------------------------------------------------------------------------
static int64_t binom(int a, int b) {
  int64_t r = 1;
  for (int i = 1; i <= b; ++i) r = r * (a - b + i) / i;
  return r;
}

int num_channels_impl(int m, int d, int basis) {
  if (m < 1 || m > 3 || d < 1 || d > 16) return -1;
  if (basis == HGF_BASIS_POWER) return m * d;
  if (basis == HGF_BASIS_MONOMIAL) return static_cast<int>(binom(m + d, d) - 1);
  return -1;
}

// Exponents of the guidance channels, in the order the header documents:
// power basis channel-major; monomials graded, lexicographic within a degree.
bool build_table(int m, int d, int basis, MonoTable* t) {
  std::memset(t, 0, sizeof(*t));
  const int n = num_channels_impl(m, d, basis);
  if (n < 1 || n > kMaxN) return false;
  t->n = n;
  t->m = m;
  int k = 0;
  if (basis == HGF_BASIS_POWER) {
    for (int i = 0; i < m; ++i)
      for (int j = 1; j <= d; ++j) t->e[k++][i] = static_cast<int8_t>(j);
    return true;
  }
  for (int deg = 1; deg <= d; ++deg) {
    // non-decreasing index sequences of length deg over m channels
    std::vector<int> idx(deg, 0);
    while (true) {
      for (int c : idx) t->e[k][c] += 1;
      ++k;
      int pos = deg - 1;
      while (pos >= 0 && idx[pos] == m - 1) --pos;
      if (pos < 0) break;
      const int v = idx[pos] + 1;
      for (int q = pos; q < deg; ++q) idx[q] = v;
    }
  }
  return k == n;
}

// ---------------------------------------------------------------------------
// validation and workspace plan
// ---------------------------------------------------------------------------
hgf_status validate(const hgf_params* p, MonoTable* table) {
  if (p == nullptr) return fail(HGF_E_INVALID, "params is NULL");
  if (p->height < 1 || p->width < 1) return fail(HGF_E_INVALID, "height and width must be >= 1");
  if (static_cast<int64_t>(p->height) * p->width > (int64_t(1) << 30))
    return fail(HGF_E_INVALID, "image too large");
  if (p->guide_channels < 1 || p->guide_channels > 3)
    return fail(HGF_E_INVALID, "guide_channels must be 1, 2 or 3");
  if (p->degree < 1) return fail(HGF_E_INVALID, "degree must be >= 1");
  if (p->basis != HGF_BASIS_MONOMIAL && p->basis != HGF_BASIS_POWER)
    return fail(HGF_E_INVALID, "unknown basis");
  if (p->reg != HGF_REG_COVARIANCE && p->reg != HGF_REG_RIDGE)
    return fail(HGF_E_INVALID, "unknown regularisation");
  if (p->radius < 0) return fail(HGF_E_INVALID, "radius must be >= 0");
  if (p->num_labels < 1) return fail(HGF_E_INVALID, "num_labels must be >= 1");
  if (!(p->eps > 0.0) || !std::isfinite(p->eps))
    return fail(HGF_E_INVALID, "eps must be finite and > 0 (Prop. 1 divides by it)");
  if (p->cost_dtype != HGF_F32 && p->cost_dtype != HGF_BF16 && p->cost_dtype != HGF_F16)
    return fail(HGF_E_INVALID, "cost_dtype must be HGF_F32, HGF_BF16 or HGF_F16");
  if (p->stats_dtype != HGF_F32 && p->stats_dtype != HGF_F64)
    return fail(HGF_E_INVALID, "stats_dtype must be HGF_F32 or HGF_F64");
  if (p->cost_ld != 0 && p->cost_ld < p->num_labels)
    return fail(HGF_E_INVALID, "cost_ld must be 0 or >= num_labels");
  if (p->out_ld != 0 && p->out_ld < p->num_labels)
    return fail(HGF_E_INVALID, "out_ld must be 0 or >= num_labels");
  const int n = num_channels_impl(p->guide_channels, p->degree, p->basis);
  if (n < 1) return fail(HGF_E_INVALID, "invalid guide_channels/degree/basis");
  if (!config_supported(n, p->radius))
    return fail(HGF_E_UNSUPPORTED, "n=%d radius=%d not compiled in (n 1..%d, radius %d..%d)",
                n, p->radius, kMaxN, kMinRadius, kMaxRadius);
  if (p->reg == HGF_REG_RIDGE && p->cost_dtype != HGF_F32)
    return fail(HGF_E_UNSUPPORTED, "ridge form is compiled for float32 costs only");
  if (!build_table(p->guide_channels, p->degree, p->basis, table))
    return fail(HGF_E_UNSUPPORTED, "guidance table");
  return HGF_OK;
}

Plan make_plan(const hgf_params* p, const MonoTable& table, int chunks_ws, size_t group_bytes) {
  Plan pl;
  pl.table = table;
  pl.n = table.n;
  pl.reg = p->reg;
  pl.cost_type = p->cost_dtype;
  pl.mode = p->reg == HGF_REG_RIDGE ? kSolveRidge
                                    : (p->stats_dtype == HGF_F64 ? kSolveCov64 : kSolveCov32);
  pl.eps = p->eps;
  pl.D = p->reg == HGF_REG_RIDGE ? pl.n + 1 : pl.n;
  pl.PD = pl.D * (pl.D + 1) / 2;
  pl.K = pl.n + pl.n * (pl.n + 1) / 2;
  pl.H = p->height;
  pl.W = p->width;
  pl.P = pl.H * pl.W;
  pl.R = p->radius;
  pl.L = p->num_labels;
  pl.chunks_total = (pl.L + 63) / 64;
  pl.ws_chunk_bytes = static_cast<size_t>(pl.P) * (pl.n + 1) * 64 * sizeof(float);
  pl.chunks_per_launch = static_cast<int>(std::max<size_t>(
      1, std::min<size_t>(std::min(chunks_ws, pl.chunks_total), group_bytes / pl.ws_chunk_bytes)));
  size_t off = 0;
  pl.off_shift = off;
  off = align_up(off + sizeof(double) * kMaxD);
  pl.off_g64 = off;
  off = align_up(off + sizeof(double) * static_cast<size_t>(pl.P) * pl.n);
  pl.off_g32 = off;
  off = align_up(off + sizeof(float) * (static_cast<size_t>(pl.P) * (pl.n + 1) + 2 * kGPad));
  pl.off_mu = off;
  off = align_up(off + sizeof(double) * static_cast<size_t>(pl.P) * pl.n);
  pl.off_minv = off;
  off = align_up(off + static_cast<size_t>(minv_elem_bytes(pl.mode)) * pl.P *
                           minv_stride(pl.mode, pl.n));
  pl.off_x = off;
  const size_t s_bytes = sizeof(double) * static_cast<size_t>(pl.P) * pl.K;
  const size_t ws_bytes = pl.ws_chunk_bytes * pl.chunks_per_launch;
  off = align_up(off + std::max(s_bytes, ws_bytes));
  pl.off_keys = off;
  off = align_up(off + sizeof(unsigned long long) * static_cast<size_t>(pl.P));
  pl.total = off;
  return pl;
}

// ---------------------------------------------------------------------------
// tuning table
// ---------------------------------------------------------------------------
int size_class(int P) {
  int c = 0;
  while (c < 30 && (1 << (c + 1)) <= P) ++c;
  return c;  // floor(log2 P)
}

TuneKey tune_key(int kernel, const Plan& pl) {
  return TuneKey(kernel, pl.n, pl.R, pl.mode, pl.cost_type, size_class(pl.P));
}

const std::vector<int>& tune_candidates() {
  static const std::vector<int> c = {128, 256, 384, 512, 768, 1024, 2048};
  return c;
}

int tuned_target(hgf_context* ctx, int kernel, const Plan& pl) {
  if (ctx != nullptr) {
    auto it = ctx->tune.find(tune_key(kernel, pl));
    if (it != ctx->tune.end()) return it->second;
  }
  // untuned: output blocks of fewer than eight waves (few channels) need
  // more blocks to keep enough loads in flight
  if (kernel == kTuneOut) {
    const int cpw = out_channels_per_wave(pl.n);
    if ((pl.n + 1 + cpw - 1) / cpw < 8) return 2 * kDefaultTarget;
  }
  return kDefaultTarget;
}

// ---------------------------------------------------------------------------
// device memory owned by the context
// ---------------------------------------------------------------------------
hgf_status ctx_alloc(hgf_context* ctx, size_t bytes, void** out) {
  if (ctx->budget != 0 && ctx->allocated + bytes > ctx->budget)
    return fail(HGF_E_NOMEM, "device memory budget exceeded");
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return fail(HGF_E_DEVICE, "hipGetDevice");
  if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
    return fail(HGF_E_DEVICE, "hipSetDevice");
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, bytes);
  if (cur != ctx->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(HGF_E_NOMEM, "hipMalloc of %zu bytes: %s", bytes, hipGetErrorString(e));
  }
  ctx->allocated += bytes;
  *out = p;
  return HGF_OK;
}

void ctx_free(hgf_context* ctx, void* p, size_t bytes) {
  if (p == nullptr) return;
  (void)hipFree(p);
  ctx->allocated -= std::min(ctx->allocated, bytes);
}

hgf_status mark_used(hipEvent_t* ev, hipStream_t s) {
  if (*ev == nullptr)
    HGF_TRY(hipEventCreateWithFlags(ev, hipEventDisableTiming), "hipEventCreate");
  HGF_TRY(hipEventRecord(*ev, s), "hipEventRecord");
  return HGF_OK;
}

void wait_used(hipEvent_t ev) {
  if (ev != nullptr) (void)hipEventSynchronize(ev);
}

hgf_status ctx_scratch(hgf_context* ctx, size_t bytes, void** out) {
  if (ctx->scratch_bytes >= bytes) {
    *out = ctx->scratch;
    return HGF_OK;
  }
  // the previous scratch may still be in use by the last call that took it
  wait_used(ctx->scratch_used);
  ctx_free(ctx, ctx->scratch, ctx->scratch_bytes);
  ctx->scratch = nullptr;
  ctx->scratch_bytes = 0;
  void* p = nullptr;
  const hgf_status st = ctx_alloc(ctx, bytes, &p);
  if (st != HGF_OK) return st;
  ctx->scratch = p;
  ctx->scratch_bytes = bytes;
  *out = p;
  return HGF_OK;
}

// ---------------------------------------------------------------------------
// stage timing: an event pair around each launch while enabled
// ---------------------------------------------------------------------------
static hipEvent_t take_event(hgf_context* ctx) {
  if (!ctx->spare.empty()) {
    hipEvent_t e = ctx->spare.back();
    ctx->spare.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

namespace {
class Stage {
 public:
  Stage(hgf_context* ctx, int stage, hipStream_t s) : ctx_(ctx), stage_(stage), s_(s) {
    if (ctx_ != nullptr && ctx_->timing) {
      a_ = take_event(ctx_);
      if (a_ != nullptr && hipEventRecord(a_, s_) != hipSuccess) {
        ctx_->spare.push_back(a_);
        a_ = nullptr;
      }
    }
  }
  ~Stage() {
    if (a_ == nullptr) return;
    hipEvent_t b = take_event(ctx_);
    if (b == nullptr || hipEventRecord(b, s_) != hipSuccess) {
      ctx_->spare.push_back(a_);
      if (b != nullptr) ctx_->spare.push_back(b);
      return;
    }
    ctx_->recs.push_back({stage_, a_, b});
  }
  Stage(const Stage&) = delete;
  Stage& operator=(const Stage&) = delete;

 private:
  hgf_context* ctx_;
  int stage_;
  hipStream_t s_;
  hipEvent_t a_ = nullptr;
};
}  // namespace

// ---------------------------------------------------------------------------
// launch sequences
// ---------------------------------------------------------------------------
hgf_status run_guide(hgf_context* ctx, const Plan& pl, const float* guide, void* ws,
                     hipStream_t s) {
  {
    Stage st(ctx, 0, s);
    HGF_TRY(launch_guide_mean(guide, pl.H, pl.W, pl.table, at<double>(ws, pl.off_shift),
                              pl.reg == HGF_REG_COVARIANCE, s),
            "guide_mean");
  }
  {
    Stage st(ctx, 1, s);
    HGF_TRY(launch_guide_synth(guide, pl.H, pl.W, pl.table, at<double>(ws, pl.off_shift),
                               at<float>(ws, pl.off_g32) + kGPad, at<double>(ws, pl.off_g64), s),
            "guide_synth");
  }
  int fused = 0;
  {
    Stage st(ctx, 2, s);
    HGF_TRY(launch_moments(at<double>(ws, pl.off_g64), pl.n, pl.H, pl.W, pl.R,
                           tuned_target(ctx, kTuneMoments, pl), at<double>(ws, pl.off_x),
                           pl.eps, pl.mode, at<double>(ws, pl.off_mu), at<char>(ws, pl.off_minv),
                           &fused, s),
            "moments");
  }
  if (!fused) {
    Stage st(ctx, 3, s);
    HGF_TRY(launch_invert(at<double>(ws, pl.off_x), pl.n, pl.H, pl.W, pl.R, pl.eps, pl.mode,
                          at<double>(ws, pl.off_mu), at<char>(ws, pl.off_minv), s),
            "invert");
  }
  return HGF_OK;
}

hgf_status run_labels(hgf_context* ctx, const Plan& pl, const void* cost, int cost_ld, float* out,
                      int out_ld, unsigned long long* keys, int32_t* labels, int label_base,
                      int count,
                      const float* g32, const void* minv, float* wsbuf,
                      hipStream_t s) {
  const size_t esz = pl.cost_type == kCostF32 ? 4 : 2;
  if (pl.L == 1 && count == 1) {
    // a one-label filter: lanes as pixels (the label-lane kernels would idle
    // 63 lanes).  Only for filters of one label, so that a one-label chunk of
    // a larger filter takes the same kernels as the whole filter.
    SingleLaunch sa;
    sa.cost = cost;
    sa.cost_type = pl.cost_type;
    sa.cost_ld = cost_ld;
    sa.g32 = g32;
    sa.minv = minv;
    sa.ws = wsbuf;
    sa.out = out;
    sa.out_ld = out_ld;
    sa.keys = keys;
    sa.labels = labels;
    sa.label = label_base;
    sa.n = pl.n;
    sa.H = pl.H;
    sa.W = pl.W;
    sa.R = pl.R;
    sa.mode = pl.mode;
    Stage st(ctx, 4, s);
    HGF_TRY(launch_single(sa, s), "single-slice filter");
    return HGF_OK;
  }
  const int coef_target = tuned_target(ctx, kTuneCoef, pl);
  const int out_target = tuned_target(ctx, kTuneOut, pl);
  for (int l0 = 0; l0 < count; l0 += pl.chunks_per_launch * 64) {
    const int lc = std::min(count - l0, pl.chunks_per_launch * 64);
    const int chunks = (lc + 63) / 64;
    CoefLaunch ca;
    ca.cost = static_cast<const char*>(cost) + esz * l0;
    ca.cost_type = pl.cost_type;
    ca.cost_ld = cost_ld;
    ca.g32 = g32;
    ca.minv = minv;
    ca.ws = wsbuf;
    ca.n = pl.n;
    ca.H = pl.H;
    ca.W = pl.W;
    ca.R = pl.R;
    ca.mode = pl.mode;
    ca.label_count = lc;
    ca.grid = strip_grid_w(pl.H, pl.W, pl.R, coef_strip_width(pl.n, pl.R), chunks, pl.chunks_total,
                           coef_target);
    {
      Stage st(ctx, 4, s);
      HGF_TRY(launch_coef(ca, s), "coef");
    }
    OutLaunch oa;
    oa.ws = wsbuf;
    oa.g32 = g32;
    oa.out = out != nullptr ? out + l0 : nullptr;
    oa.out_ld = out_ld;
    oa.keys = keys;
    oa.labels = labels;
    oa.label_base = label_base + l0;
    oa.n = pl.n;
    oa.H = pl.H;
    oa.W = pl.W;
    oa.R = pl.R;
    oa.label_count = lc;
    oa.grid = strip_grid_w(pl.H, pl.W, pl.R, out_strip_width(pl.n, pl.R), chunks, pl.chunks_total,
                           out_target);
    {
      Stage st(ctx, 5, s);
      HGF_TRY(launch_out(oa, s), "out");
    }
  }
  return HGF_OK;
}

hgf_status run_filter(hgf_context* ctx, const Plan& pl, const float* guide, const void* cost,
                      int cost_ld, float* out, int out_ld, int32_t* labels, void* ws,
                      hipStream_t s) {
  hgf_status st = run_guide(ctx, pl, guide, ws, s);
  if (st != HGF_OK) return st;
  // With every label in one chunk of one launch the output kernel writes the
  // final labels itself; otherwise the chunks merge per-pixel keys.
  const bool direct = labels != nullptr && pl.L <= 64;
  unsigned long long* keys =
      (labels != nullptr && !direct) ? at<unsigned long long>(ws, pl.off_keys) : nullptr;
  if (keys != nullptr) {
    Stage sk(ctx, 6, s);
    HGF_TRY(launch_key_fill(keys, pl.P, s), "key_fill");
  }
  st = run_labels(ctx, pl, cost, cost_ld, out, out_ld, keys, direct ? labels : nullptr, 0, pl.L,
                  pl.g32(ws),
                  at<char>(ws, pl.off_minv), at<float>(ws, pl.off_x),
                  s);
  if (st != HGF_OK) return st;
  if (keys != nullptr) {
    Stage sk(ctx, 6, s);
    HGF_TRY(launch_key_finalize(keys, pl.P, nullptr, labels, 0, s), "key_finalize");
  }
  return HGF_OK;
}

}  // namespace hgf

using namespace hgf;

// ===========================================================================
// extern "C"
// ===========================================================================
void hgf_release_batch_resources(hgf_context* ctx);  // batch.hip

namespace {

hgf_status check_workspace(const Plan& pl, void* ws, size_t bytes) {
  if (bytes < pl.total)
    return fail(HGF_E_INVALID, "workspace of %zu bytes is smaller than the %zu this call needs",
                bytes, pl.total);
  if (reinterpret_cast<uintptr_t>(ws) % kAlign != 0)
    return fail(HGF_E_INVALID, "workspace must be 256-byte aligned");
  return HGF_OK;
}

}  // namespace

extern "C" {

int32_t hgf_num_channels(int32_t m, int32_t d, int32_t basis) {
  return num_channels_impl(m, d, basis);
}

int32_t hgf_is_supported(int32_t n, int32_t radius, int32_t reg) {
  return (reg == HGF_REG_COVARIANCE || reg == HGF_REG_RIDGE) && config_supported(n, radius) ? 1
                                                                                           : 0;
}

hgf_status hgf_create(int32_t device, size_t hbm_budget_bytes, hgf_context** out) {
  return guarded(nullptr, [&]() -> hgf_status {
    if (out == nullptr) return fail(HGF_E_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    const hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0) return fail(HGF_E_DEVICE, "no HIP device");
    if (device < 0 || device >= count) return fail(HGF_E_INVALID, "device index out of range");
    hgf_context* ctx = new (std::nothrow) hgf_context();
    if (ctx == nullptr) return fail(HGF_E_NOMEM, "host allocation");
    ctx->device = device;
    ctx->budget = hbm_budget_bytes;
    *out = ctx;
    return HGF_OK;
  });
}

void hgf_destroy(hgf_context* ctx) {
  if (ctx == nullptr) return;
  try {
    // work that still uses context-owned memory: the last call that took the
    // scratch buffer, the last batch graph launch and the batch worker streams
    wait_used(ctx->scratch_used);
    wait_used(ctx->batch_done);
    for (hipStream_t st : ctx->workers) (void)hipStreamSynchronize(st);
    hgf_release_batch_resources(ctx);
    for (auto& r : ctx->recs) {
      ctx->spare.push_back(r.start);
      ctx->spare.push_back(r.stop);
    }
    for (hipEvent_t e : ctx->spare) (void)hipEventDestroy(e);
    if (ctx->scratch_used != nullptr) (void)hipEventDestroy(ctx->scratch_used);
    if (ctx->batch_done != nullptr) (void)hipEventDestroy(ctx->batch_done);
    ctx_free(ctx, ctx->scratch, ctx->scratch_bytes);
  } catch (...) {
  }
  delete ctx;
}

hgf_status hgf_workspace_size(const hgf_params* params, size_t* bytes) {
  return guarded(nullptr, [&]() -> hgf_status {
    if (bytes == nullptr) return fail(HGF_E_INVALID, "bytes is NULL");
    MonoTable t;
    const hgf_status st = validate(params, &t);
    if (st != HGF_OK) return st;
    *bytes = make_plan(params, t, (params->num_labels + 63) / 64).total;
    return HGF_OK;
  });
}

hgf_status hgf_set_group_bytes(hgf_context* ctx, size_t bytes) {
  return guarded(ctx, [&]() -> hgf_status {
    if (ctx == nullptr) return fail(HGF_E_INVALID, "context is NULL");
    ctx->group_bytes = bytes == 0 ? kDefaultGroupBytes : bytes;
    return HGF_OK;
  });
}

hgf_status hgf_filter(hgf_context* ctx, const hgf_params* params, const float* guide,
                      const void* cost, float* out, int32_t* labels, void* workspace,
                      size_t workspace_bytes, void* hip_stream) {
  return guarded(ctx, [&]() -> hgf_status {
    if (ctx == nullptr) return fail(HGF_E_INVALID, "context is NULL");
    MonoTable t;
    hgf_status st = validate(params, &t);
    if (st != HGF_OK) return st;
    if (guide == nullptr || cost == nullptr) return fail(HGF_E_INVALID, "guide or cost is NULL");
    if (out == nullptr && labels == nullptr)
      return fail(HGF_E_INVALID, "out and labels are both NULL: nothing to compute");
    const Plan pl = make_plan(params, t, (params->num_labels + 63) / 64, ctx->group_bytes);
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    void* ws = workspace;
    if (ws == nullptr) {
      st = ctx_scratch(ctx, pl.total, &ws);
      if (st != HGF_OK) return st;
    } else {
      st = check_workspace(pl, ws, workspace_bytes);
      if (st != HGF_OK) return st;
    }
    const int cost_ld = params->cost_ld ? params->cost_ld : params->num_labels;
    const int out_ld = params->out_ld ? params->out_ld : params->num_labels;
    st = run_filter(ctx, pl, guide, cost, cost_ld, out, out_ld, labels, ws, s);
    if (workspace == nullptr) {
      const hgf_status m = mark_used(&ctx->scratch_used, s);
      if (st == HGF_OK) st = m;
    }
    return st;
  });
}

hgf_status hgf_guide_create(hgf_context* ctx, const hgf_params* params, const float* guide,
                            void* hip_stream, hgf_guide** out) {
  return guarded(ctx, [&]() -> hgf_status {
    if (ctx == nullptr || out == nullptr) return fail(HGF_E_INVALID, "context or out is NULL");
    *out = nullptr;
    MonoTable t;
    hgf_status st = validate(params, &t);
    if (st != HGF_OK) return st;
    if (guide == nullptr) return fail(HGF_E_INVALID, "guide is NULL");
    hgf_guide* g = new (std::nothrow) hgf_guide();
    if (g == nullptr) return fail(HGF_E_NOMEM, "host allocation");
    g->ctx = ctx;
    g->params = *params;
    // coefficient workspace for one chunk of 64 labels: a filter call runs
    // its chunks one launch group after another
    g->plan = make_plan(params, t, 1, ctx->group_bytes);
    g->bytes = g->plan.total;
    st = ctx_alloc(ctx, g->bytes, &g->base);
    if (st != HGF_OK) {
      delete g;
      return st;
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    st = run_guide(ctx, g->plan, guide, g->base, s);
    if (st == HGF_OK) st = mark_used(&g->used, s);
    if (st != HGF_OK) {
      (void)hipStreamSynchronize(s);
      ctx_free(ctx, g->base, g->bytes);
      if (g->used != nullptr) (void)hipEventDestroy(g->used);
      delete g;
      return st;
    }
    *out = g;
    return HGF_OK;
  });
}

hgf_status hgf_guide_filter(hgf_context* ctx, hgf_guide* g, const void* cost_chunk,
                            int32_t label_begin, int32_t label_count, int32_t ld,
                            float* out_chunk, float* best_cost, int32_t* labels,
                            void* hip_stream) {
  return guarded(ctx, [&]() -> hgf_status {
    if (ctx == nullptr || g == nullptr) return fail(HGF_E_INVALID, "context or guide is NULL");
    if (cost_chunk == nullptr) return fail(HGF_E_INVALID, "cost_chunk is NULL");
    if (label_count < 1 || label_begin < 0 ||
        static_cast<int64_t>(label_begin) + label_count > g->params.num_labels)
      return fail(HGF_E_INVALID, "label range outside [0, num_labels)");
    if (ld != 0 && ld < label_count) return fail(HGF_E_INVALID, "ld must be 0 or >= label_count");
    if ((best_cost == nullptr) != (labels == nullptr))
      return fail(HGF_E_INVALID, "best_cost and labels must both be given or both be NULL");
    if (out_chunk == nullptr && labels == nullptr)
      return fail(HGF_E_INVALID, "out_chunk and labels are both NULL: nothing to compute");
    const Plan& pl = g->plan;
    const int ldv = ld ? ld : label_count;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    void* base = g->base;
    unsigned long long* keys =
        labels != nullptr ? at<unsigned long long>(base, pl.off_keys) : nullptr;
    if (keys != nullptr) {
      Stage sk(ctx, 6, s);
      HGF_TRY(launch_key_fill(keys, pl.P, s), "key_fill");
    }
    hgf_status st = run_labels(ctx, pl, cost_chunk, ldv, out_chunk, ldv, keys, nullptr,
                               label_begin, label_count, pl.g32(base),
                               at<char>(base, pl.off_minv), at<float>(base, pl.off_x), s);
    if (st == HGF_OK && keys != nullptr) {
      Stage sk(ctx, 6, s);
      HGF_TRY(launch_key_finalize(keys, pl.P, best_cost, labels, label_begin > 0 ? 1 : 0, s),
              "key_finalize");
    }
    const hgf_status m = mark_used(&g->used, s);
    return st != HGF_OK ? st : m;
  });
}

size_t hgf_guide_bytes(const hgf_guide* g) { return g != nullptr ? g->bytes : 0; }

void hgf_guide_destroy(hgf_guide* g) {
  if (g == nullptr) return;
  try {
    // only the work that used this guide's buffer, not the whole device
    wait_used(g->used);
    if (g->used != nullptr) (void)hipEventDestroy(g->used);
    if (g->owns) ctx_free(g->ctx, g->base, g->bytes);
  } catch (...) {
  }
  delete g;
}

hgf_status hgf_guide_export(const hgf_guide* g, double* mu, void* minv, double* shift,
                            void* hip_stream) {
  return guarded(g != nullptr ? g->ctx : nullptr, [&]() -> hgf_status {
    if (g == nullptr) return fail(HGF_E_INVALID, "guide is NULL");
    const Plan& pl = g->plan;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (mu != nullptr)
      HGF_TRY(hipMemcpyAsync(mu, at<char>(g->base, pl.off_mu),
                             sizeof(double) * static_cast<size_t>(pl.P) * pl.n,
                             hipMemcpyDeviceToDevice, s),
              "export mu");
    if (minv != nullptr) {
      // the packed triangle of each pixel, out of its stored record
      const size_t eb = static_cast<size_t>(minv_elem_bytes(pl.mode));
      const size_t skip = pl.mode == kSolveRidge ? 0 : static_cast<size_t>(pl.n);
      HGF_TRY(hipMemcpy2DAsync(minv, eb * pl.PD, at<char>(g->base, pl.off_minv) + eb * skip,
                               eb * minv_stride(pl.mode, pl.n), eb * pl.PD,
                               static_cast<size_t>(pl.P), hipMemcpyDeviceToDevice, s),
              "export minv");
    }
    if (shift != nullptr)
      HGF_TRY(hipMemcpyAsync(shift, at<char>(g->base, pl.off_shift), sizeof(double) * pl.n,
                             hipMemcpyDeviceToDevice, s),
              "export shift");
    return HGF_OK;
  });
}

hgf_status hgf_box_sum(const float* in, float* out, int32_t channels, int32_t height,
                       int32_t width, int32_t radius, void* hip_stream) {
  return guarded(nullptr, [&]() -> hgf_status {
    if (in == nullptr || out == nullptr) return fail(HGF_E_INVALID, "in or out is NULL");
    if (channels < 1 || height < 1 || width < 1 || radius < 0)
      return fail(HGF_E_INVALID, "channels, height, width must be >= 1 and radius >= 0");
    if (radius > kBoxMaxRadius) return fail(HGF_E_UNSUPPORTED, "radius above %d", kBoxMaxRadius);
    const size_t bytes = sizeof(float) * static_cast<size_t>(channels) * height * width;
    const char* a = reinterpret_cast<const char*>(in);
    const char* b = reinterpret_cast<const char*>(out);
    if (a < b + bytes && b < a + bytes) return fail(HGF_E_INVALID, "in and out must not overlap");
    HGF_TRY(launch_box_sum(in, out, channels, height, width, radius,
                           static_cast<hipStream_t>(hip_stream)),
            "box_sum");
    return HGF_OK;
  });
}

hgf_status hgf_spd_inverse(const double* a, double* minv, int32_t dim, int32_t count,
                           void* hip_stream) {
  return guarded(nullptr, [&]() -> hgf_status {
    if (a == nullptr || minv == nullptr) return fail(HGF_E_INVALID, "a or minv is NULL");
    if (dim < 1 || dim > kMaxD) return fail(HGF_E_INVALID, "dim must be in [1, 20]");
    if (count < 0) return fail(HGF_E_INVALID, "count < 0");
    if (count == 0) return HGF_OK;
    HGF_TRY(launch_spd_inverse(a, minv, dim, count, static_cast<hipStream_t>(hip_stream)),
            "spd_inverse");
    return HGF_OK;
  });
}

hgf_status hgf_set_stage_timing(hgf_context* ctx, int32_t enable) {
  return guarded(ctx, [&]() -> hgf_status {
    if (ctx == nullptr) return fail(HGF_E_INVALID, "context is NULL");
    ctx->timing = enable != 0;
    return HGF_OK;
  });
}

hgf_status hgf_stage_times(hgf_context* ctx, double* ms, int32_t* launches, int32_t max_stages) {
  return guarded(ctx, [&]() -> hgf_status {
    if (ctx == nullptr) return fail(HGF_E_INVALID, "context is NULL");
    if (max_stages < 0) return fail(HGF_E_INVALID, "max_stages < 0");
    for (int i = 0; i < max_stages; ++i) {
      if (ms != nullptr) ms[i] = 0.0;
      if (launches != nullptr) launches[i] = 0;
    }
    hgf_status st = HGF_OK;
    for (auto& r : ctx->recs) {
      float t = 0.f;
      if (hipEventSynchronize(r.stop) != hipSuccess ||
          hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess)
        st = fail(HGF_E_DEVICE, "stage event timing");
      if (r.stage < max_stages) {
        if (ms != nullptr) ms[r.stage] += t;
        if (launches != nullptr) launches[r.stage] += 1;
      }
      ctx->spare.push_back(r.start);
      ctx->spare.push_back(r.stop);
    }
    ctx->recs.clear();
    return st;
  });
}

const char* hgf_status_string(hgf_status status) {
  switch (status) {
    case HGF_OK: return "HGF_OK";
    case HGF_E_INVALID: return "HGF_E_INVALID";
    case HGF_E_NOMEM: return "HGF_E_NOMEM";
    case HGF_E_DEVICE: return "HGF_E_DEVICE";
    case HGF_E_UNSUPPORTED: return "HGF_E_UNSUPPORTED";
    case HGF_E_BUSY: return "HGF_E_BUSY";
  }
  return "unknown hgf_status";
}

const char* hgf_last_error(const hgf_context* ctx) {
  return ctx != nullptr ? ctx->err : thread_error();
}

}  // extern "C"
