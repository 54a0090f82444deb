// Axis-2 passes of the FP64 evaluation, every length class and radix order (see
// kernels.hpp).
#include "kernels.hpp"

namespace vdwnl {

hipError_t launch_y_f64(int kind, int lc, int var, const LaunchArgs &a) {
    VDWNL_LC_VARIANTS(launch_y_lc, double, kind, lc, var, a)
}

}  // namespace vdwnl
