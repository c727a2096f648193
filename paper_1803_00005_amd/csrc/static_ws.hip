// hgf_filter_static: the plain filter with its workspace in a library-owned,
// statically allocated device array, for callers that cannot allocate device
// memory (code under graph capture, tight serving loops, harnesses that
// forbid allocation).
//
// The array below is a file-scope __device__ object: each GPU the library
// runs on holds its own copy, at its own address, for the life of the
// process.  Host code never uses the array's name as an address (on the host
// it is only a stand-in symbol); its device address is looked up once per
// device with hipGetSymbolAddress and kept in `g_scratch`.  Every call on a
// device shares that device's array, which keeps the last call's contents:
// the one region that must start at zero (the winner-takes-all keys) is
// cleared by a fill kernel on every call, and calls that overlap on one GPU
// (two streams, or two threads) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "runtime.hpp"

namespace hgf {
namespace {

// 96 MiB: room for the 64 x 64 colour workload many times over, or about
// 30,000 pixels at n = 9 (one 64-label chunk per launch group).
constexpr size_t kStaticScratchBytes = size_t(96) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

void* g_scratch[kMaxDevices] = {nullptr};
std::mutex g_scratch_mu;

// The device address of this device's array (looked up on first use, with
// the device current).
hgf_status static_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(HGF_E_UNSUPPORTED, "device index %d", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device] == nullptr) {
    int cur = 0;
    HGF_TRY(hipGetDevice(&cur), "hipGetDevice");
    if (cur != device) HGF_TRY(hipSetDevice(device), "hipSetDevice");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return device_fail(e, "hipGetSymbolAddress(scratch)");
    if (p == nullptr || reinterpret_cast<uintptr_t>(p) % kAlign != 0)
      return fail(HGF_E_DEVICE, "static scratch: unexpected device address");
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return HGF_OK;
}

}  // namespace
}  // namespace hgf

using namespace hgf;

extern "C" {

size_t hgf_static_scratch_bytes(void) { return kStaticScratchBytes; }

hgf_status hgf_filter_static(hgf_context* ctx, const hgf_params* params, const float* guide,
                             const void* cost, float* out, int32_t* labels, void* hip_stream) {
  return guarded(ctx, [&]() -> hgf_status {
    if (ctx == nullptr) return fail(HGF_E_INVALID, "context is NULL");
    MonoTable t;
    hgf_status st = validate(params, &t);
    if (st != HGF_OK) return st;
    if (guide == nullptr || cost == nullptr) return fail(HGF_E_INVALID, "guide or cost is NULL");
    if (out == nullptr && labels == nullptr)
      return fail(HGF_E_INVALID, "out and labels are both NULL: nothing to compute");
    // one 64-label chunk per launch group: the smallest workspace (the band
    // partition does not depend on it, so the results equal hgf_filter's)
    const Plan pl = make_plan(params, t, 1, ctx->group_bytes);
    if (pl.total > kStaticScratchBytes)
      return fail(HGF_E_NOMEM,
                  "this filter needs %zu bytes of workspace; the static workspace holds %zu",
                  pl.total, kStaticScratchBytes);
    // the array of the device the stream belongs to (the current device for
    // the null stream)
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int device = 0;
    if (s == nullptr) {
      HGF_TRY(hipGetDevice(&device), "hipGetDevice");
    } else {
      HGF_TRY(hipStreamGetDevice(s, &device), "hipStreamGetDevice");
    }
    void* ws = nullptr;
    st = static_scratch(device, &ws);
    if (st != HGF_OK) return st;
    const int cost_ld = params->cost_ld ? params->cost_ld : params->num_labels;
    const int out_ld = params->out_ld ? params->out_ld : params->num_labels;
    return run_filter(ctx, pl, guide, cost, cost_ld, out, out_ld, labels, ws, s);
  });
}

}  // extern "C"
