// Coefficient kernels for n = 6 guidance channels (all compiled radii, both
// regularisation forms, float32 and bfloat16 cost).
#include "coef.hpp"

namespace hgf {
hipError_t launch_coef_n6(const CoefLaunch& a, hipStream_t s) { return coef_launch_n<6>(a, s); }
}  // namespace hgf
