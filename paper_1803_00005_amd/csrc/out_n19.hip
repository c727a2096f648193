// Output kernels for n = 19 guidance channels (all compiled radii).
#include "out.hpp"

namespace hgf {
hipError_t launch_out_n19(const OutLaunch& a, hipStream_t s) { return out_launch_n<19>(a, s); }
}  // namespace hgf
