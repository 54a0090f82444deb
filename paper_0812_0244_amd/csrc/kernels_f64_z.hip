// Axis-1 passes (the fused contraction pass, the gradient and divergence multipliers, the spectra probes) of the FP64 evaluation, every length class and radix order (see
// kernels.hpp).
#include "kernels.hpp"

namespace vdwnl {

hipError_t launch_z_f64(int kind, int lc, int var, const LaunchArgs &a) {
    VDWNL_LC_VARIANTS(launch_z_lc, double, kind, lc, var, a)
}

}  // namespace vdwnl
