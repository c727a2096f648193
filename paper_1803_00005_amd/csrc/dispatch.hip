// Dispatch of the per-(n, radius) kernel instantiations.
//
// The strip kernels are templates over the channel count n and the radius
// (their per-wave running sums live in registers indexed at compile time).
// Their instantiations are compiled in separate generated units (one per
// (n, radius) for the coefficient kernel, one per n for the rest) so that the
// build runs in parallel; this unit only maps a runtime (n, radius) to them.
#include <array>
#include <utility>

#include "hgf_launch.hpp"

namespace hgf {

template <int NG, int R>
hipError_t coef_launch_nr(const CoefLaunch& a, hipStream_t s);
template <int NG>
hipError_t out_launch_n(const OutLaunch& a, hipStream_t s);
template <int NG>
hipError_t moments_n(const double* g64, int H, int W, int R, int target, double* S, double eps,
                     int mode, double* mu, void* minv, int* fused, hipStream_t s);
template <int NG>
hipError_t invert_n(const double* S, int H, int W, int R, double eps, int mode, double* mu,
                    void* minv, hipStream_t s);
template <int NG>
hipError_t single_launch_n(const SingleLaunch& a, hipStream_t s);

namespace {

constexpr int kNumR = kMaxRadius - kMinRadius + 1;
using CoefFn = hipError_t (*)(const CoefLaunch&, hipStream_t);

template <int NG, int... Rs>
constexpr std::array<CoefFn, kNumR> coef_row(std::integer_sequence<int, Rs...>) {
  return {&coef_launch_nr<NG, kMinRadius + Rs>...};
}

template <int... Ns>
constexpr std::array<std::array<CoefFn, kNumR>, kMaxN> coef_table(
    std::integer_sequence<int, Ns...>) {
  return {coef_row<Ns + 1>(std::make_integer_sequence<int, kNumR>())...};
}

template <typename Fn, template <int> class Pick, int... Ns>
constexpr std::array<Fn, kMaxN> per_n(std::integer_sequence<int, Ns...>) {
  return {Pick<Ns + 1>::fn...};
}

template <int NG> struct PickOut { static constexpr auto fn = &out_launch_n<NG>; };
template <int NG> struct PickMoments { static constexpr auto fn = &moments_n<NG>; };
template <int NG> struct PickInvert { static constexpr auto fn = &invert_n<NG>; };
template <int NG> struct PickSingle { static constexpr auto fn = &single_launch_n<NG>; };

using OutFn = decltype(&out_launch_n<1>);
using MomentsFn = decltype(&moments_n<1>);
using InvertFn = decltype(&invert_n<1>);
using SingleFn = decltype(&single_launch_n<1>);

const auto kCoef = coef_table(std::make_integer_sequence<int, kMaxN>());
const auto kOut = per_n<OutFn, PickOut>(std::make_integer_sequence<int, kMaxN>());
const auto kMoments = per_n<MomentsFn, PickMoments>(std::make_integer_sequence<int, kMaxN>());
const auto kInvert = per_n<InvertFn, PickInvert>(std::make_integer_sequence<int, kMaxN>());
const auto kSingle = per_n<SingleFn, PickSingle>(std::make_integer_sequence<int, kMaxN>());

bool n_ok(int n) { return n >= 1 && n <= kMaxN; }

}  // namespace

bool radius_supported(int R) { return R >= kMinRadius && R <= kMaxRadius; }

bool config_supported(int n, int R) { return n_ok(n) && radius_supported(R); }

hipError_t launch_coef(const CoefLaunch& a, hipStream_t s) {
  if (!config_supported(a.n, a.R)) return hipErrorNotSupported;
  return kCoef[a.n - 1][a.R - kMinRadius](a, s);
}

hipError_t launch_out(const OutLaunch& a, hipStream_t s) {
  if (!config_supported(a.n, a.R)) return hipErrorNotSupported;
  return kOut[a.n - 1](a, s);
}

hipError_t launch_moments(const double* g64, int n, int H, int W, int R, int target, double* S,
                          double eps, int mode, double* mu, void* minv, int* fused,
                          hipStream_t s) {
  *fused = 0;
  if (!config_supported(n, R)) return hipErrorNotSupported;
  return kMoments[n - 1](g64, H, W, R, target, S, eps, mode, mu, minv, fused, s);
}

hipError_t launch_invert(const double* S, int n, int H, int W, int R, double eps, int mode,
                         double* mu, void* minv, hipStream_t s) {
  if (!n_ok(n)) return hipErrorNotSupported;
  return kInvert[n - 1](S, H, W, R, eps, mode, mu, minv, s);
}

hipError_t launch_single(const SingleLaunch& a, hipStream_t s) {
  if (!config_supported(a.n, a.R)) return hipErrorNotSupported;
  return kSingle[a.n - 1](a, s);
}

}  // namespace hgf
