// Autotuner of the strip decomposition.
//
// The coefficient and output kernels split an image into strips of output
// columns and bands of rows; the band height trades parallelism (more
// blocks) against the 2r + 1 rows each band spends restarting its running
// sums.  hgf_autotune times each candidate block count on the caller's data
// with HIP events and keeps the fastest per (kernel, n, radius, form, cost
// dtype, image size class) in the context; later launches of the same class
// use it.  Tables can be saved to and loaded from a text file.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <limits>
#include <vector>

#include "runtime.hpp"

using namespace hgf;

namespace {

// Milliseconds per pass of the guidance moment sums (stage 2), the
// coefficient (stage 4) and the output (stage 5) kernels over `reps` passes
// of the whole path with the current table.
hgf_status time_path(hgf_context* ctx, const Plan& pl, const float* guide, const void* cost,
                     int cost_ld, float* out, int out_ld, void* ws, int reps, hipStream_t s,
                     double* ms_out) {
  const bool timing = ctx->timing;
  ctx->timing = true;
  double ms[HGF_NUM_STAGES];
  (void)hgf_stage_times(ctx, ms, nullptr, HGF_NUM_STAGES);  // drop older records
  hgf_status st = HGF_OK;
  unsigned long long* keys = at<unsigned long long>(ws, pl.off_keys);
  for (int r = 0; r < reps && st == HGF_OK; ++r) {
    st = run_guide(ctx, pl, guide, ws, s);
    if (st != HGF_OK) break;
    if (launch_key_fill(keys, pl.P, s) != hipSuccess) {
      st = fail(HGF_E_DEVICE, "key_fill");
      break;
    }
    st = run_labels(ctx, pl, cost, cost_ld, out, out_ld, keys, nullptr, 0, pl.L, pl.g32(ws),
                    at<char>(ws, pl.off_minv), at<float>(ws, pl.off_x),
                    s);
  }
  const hgf_status st2 = hgf_stage_times(ctx, ms, nullptr, HGF_NUM_STAGES);
  ctx->timing = timing;
  if (st != HGF_OK) return st;
  if (st2 != HGF_OK) return st2;
  for (int k = 0; k < HGF_NUM_STAGES; ++k) ms_out[k] = ms[k] / reps;
  return HGF_OK;
}

hgf_status autotune(hgf_context* ctx, const hgf_params* params, const float* guide,
                    const void* cost, float* out, void* workspace, size_t workspace_bytes,
                    void* hip_stream) {
  if (ctx == nullptr) return fail(HGF_E_INVALID, "context is NULL");
  MonoTable t;
  hgf_status st = validate(params, &t);
  if (st != HGF_OK) return st;
  if (guide == nullptr || cost == nullptr) return fail(HGF_E_INVALID, "guide or cost is NULL");
  const Plan pl = make_plan(params, t, (params->num_labels + 63) / 64, ctx->group_bytes);
  void* ws = workspace;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (ws == nullptr) {
    st = ctx_scratch(ctx, pl.total, &ws);
    if (st != HGF_OK) return st;
    st = mark_used(&ctx->scratch_used, s);
    if (st != HGF_OK) return st;
  } else if (workspace_bytes < pl.total) {
    return fail(HGF_E_INVALID, "workspace smaller than hgf_workspace_size()");
  }
  const int cost_ld = params->cost_ld ? params->cost_ld : params->num_labels;
  const int out_ld = params->out_ld ? params->out_ld : params->num_labels;
  double ms[HGF_NUM_STAGES];
  // one untimed pass to warm caches and code objects
  st = time_path(ctx, pl, guide, cost, cost_ld, out, out_ld, ws, 1, s, ms);
  if (st != HGF_OK) return st;
  const int kernels[3] = {kTuneMoments, kTuneCoef, kTuneOut};
  const int stage_of[3] = {2, 4, 5};
  TuneKey keys[3];
  double best[3];
  int arg[3];
  for (int k = 0; k < 3; ++k) {
    keys[k] = tune_key(kernels[k], pl);
    best[k] = std::numeric_limits<double>::max();
    arg[k] = kDefaultTarget;
  }
  for (int cand : tune_candidates()) {
    for (int k = 0; k < 3; ++k) ctx->tune[keys[k]] = cand;
    st = time_path(ctx, pl, guide, cost, cost_ld, out, out_ld, ws, 3, s, ms);
    if (st != HGF_OK) return st;
    for (int k = 0; k < 3; ++k) {
      if (ms[stage_of[k]] < best[k]) {
        best[k] = ms[stage_of[k]];
        arg[k] = cand;
      }
    }
  }
  for (int k = 0; k < 3; ++k) ctx->tune[keys[k]] = arg[k];
  // leave `out` holding what hgf_filter now computes with the chosen table
  if (out != nullptr) st = time_path(ctx, pl, guide, cost, cost_ld, out, out_ld, ws, 1, s, ms);
  if (workspace == nullptr) {
    const hgf_status m = mark_used(&ctx->scratch_used, s);
    if (st == HGF_OK) st = m;
  }
  return st;
}

}  // namespace

extern "C" {

hgf_status hgf_autotune(hgf_context* ctx, const hgf_params* params, const float* guide,
                        const void* cost, float* out, void* workspace, size_t workspace_bytes,
                        void* hip_stream) {
  return guarded(ctx, [&] {
    return autotune(ctx, params, guide, cost, out, workspace, workspace_bytes, hip_stream);
  });
}

hgf_status hgf_tune_entries(const hgf_context* ctx, int32_t* rows, int32_t max_rows,
                            int32_t* count) {
  return guarded(const_cast<hgf_context*>(ctx), [&]() -> hgf_status {
  if (ctx == nullptr || count == nullptr) return fail(HGF_E_INVALID, "context or count is NULL");
  int32_t i = 0;
  for (const auto& kv : ctx->tune) {
    if (rows != nullptr && i < max_rows) {
      int32_t* r = rows + 7 * i;
      r[0] = std::get<0>(kv.first);
      r[1] = std::get<1>(kv.first);
      r[2] = std::get<2>(kv.first);
      r[3] = std::get<3>(kv.first);
      r[4] = std::get<4>(kv.first);
      r[5] = std::get<5>(kv.first);
      r[6] = kv.second;
    }
    ++i;
  }
  *count = i;
  return HGF_OK;
  });
}

hgf_status hgf_tune_set(hgf_context* ctx, const int32_t* row) {
  return guarded(ctx, [&]() -> hgf_status {
    if (ctx == nullptr || row == nullptr) return fail(HGF_E_INVALID, "context or row is NULL");
    if (row[0] < 0 || row[0] > 2 || row[6] < 1)
      return fail(HGF_E_INVALID, "tuning row: kernel in {0,1,2}, target >= 1");
    ctx->tune[TuneKey(row[0], row[1], row[2], row[3], row[4], row[5])] = row[6];
    return HGF_OK;
  });
}

hgf_status hgf_tune_save(const hgf_context* ctx, const char* path) {
  return guarded(const_cast<hgf_context*>(ctx), [&]() -> hgf_status {
  if (ctx == nullptr || path == nullptr) return fail(HGF_E_INVALID, "context or path is NULL");
  FILE* f = std::fopen(path, "w");
  if (f == nullptr) return fail(HGF_E_INVALID, "cannot write %s", path);
  std::fprintf(f, "# kernel n radius solve_form cost_dtype size_class target_blocks\n");
  for (const auto& kv : ctx->tune)
    std::fprintf(f, "%d %d %d %d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first),
                 std::get<2>(kv.first), std::get<3>(kv.first), std::get<4>(kv.first),
                 std::get<5>(kv.first), kv.second);
  std::fclose(f);
  return HGF_OK;
  });
}

hgf_status hgf_tune_load(hgf_context* ctx, const char* path) {
  return guarded(ctx, [&]() -> hgf_status {
  if (ctx == nullptr || path == nullptr) return fail(HGF_E_INVALID, "context or path is NULL");
  FILE* f = std::fopen(path, "r");
  if (f == nullptr) return fail(HGF_E_INVALID, "cannot read %s", path);
  char line[256];
  hgf_status st = HGF_OK;
  while (std::fgets(line, sizeof(line), f) != nullptr) {
    if (line[0] == '#' || line[0] == '\n') continue;
    int32_t r[7];
    if (std::sscanf(line, "%d %d %d %d %d %d %d", &r[0], &r[1], &r[2], &r[3], &r[4], &r[5],
                    &r[6]) != 7) {
      st = fail(HGF_E_INVALID, "malformed tuning line: %s", line);
      break;
    }
    st = hgf_tune_set(ctx, r);
    if (st != HGF_OK) break;
  }
  std::fclose(f);
  return st;
  });
}

}  // extern "C"
