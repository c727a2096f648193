// Output kernels for n = 8 guidance channels (all compiled radii).
#include "out.hpp"

namespace hgf {
hipError_t launch_out_n8(const OutLaunch& a, hipStream_t s) { return out_launch_n<8>(a, s); }
}  // namespace hgf
