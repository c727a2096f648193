// Coefficient kernels for n = 2 guidance channels (all compiled radii, both
// regularisation forms, float32 and bfloat16 cost).
#include "coef.hpp"

namespace hgf {
hipError_t launch_coef_n2(const CoefLaunch& a, hipStream_t s) { return coef_launch_n<2>(a, s); }
}  // namespace hgf
