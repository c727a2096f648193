// Output kernels for n = 6 guidance channels (all compiled radii).
#include "out.hpp"

namespace hgf {
hipError_t launch_out_n6(const OutLaunch& a, hipStream_t s) { return out_launch_n<6>(a, s); }
}  // namespace hgf
