// Output kernels for n = 2 guidance channels (all compiled radii).
#include "out.hpp"

namespace hgf {
hipError_t launch_out_n2(const OutLaunch& a, hipStream_t s) { return out_launch_n<2>(a, s); }
}  // namespace hgf
