// Output kernels for n = 7 guidance channels (all compiled radii).
#include "out.hpp"

namespace hgf {
hipError_t launch_out_n7(const OutLaunch& a, hipStream_t s) { return out_launch_n<7>(a, s); }
}  // namespace hgf
