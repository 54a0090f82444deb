// The passes without a transform (finite-difference stencils, the theta
// probe), the FP64 energy reduction, and the dispatch of every launch by
// precision and family (see kernels.hpp).
#include "kernels.hpp"

namespace vdwnl {

// E_k = (Omega/2) sum of the axis-1 partials; Delta E = dOmega sum of the
// theta partials; E_x, E_c^LDA = dOmega sums of the semilocal partials (zero
// unless the semilocal terms are on).  One workgroup per grid, fixed
// summation order; E[4 g + 0..3].
__global__ void __launch_bounds__(kThreads) k_reduce(const InstDev *insts, double *E) {
    const InstDev &I = insts[blockIdx.x];
    double a = 0.0, b = 0.0, x = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < I.n_ek; i += kThreads) a += I.part_ek[i];
    for (int i = threadIdx.x; i < I.n_de; i += kThreads) {
        b += I.part_de[i];
        x += I.part_sl[2 * i];
        c += I.part_sl[2 * i + 1];
    }
    a = block_sum(a);
    b = block_sum(b);
    x = block_sum(x);
    c = block_sum(c);
    if (threadIdx.x == 0) {
        // a density the theta pass flagged: every energy of the grid NaN
        const double nan = __builtin_nan("");
        const bool bad = gld(I.bad)[0] != 0;
        E[4 * blockIdx.x] = bad ? nan : 0.5 * I.omega * a;
        E[4 * blockIdx.x + 1] = bad ? nan : I.dvol * b;
        E[4 * blockIdx.x + 2] = bad ? nan : I.dvol * x;
        E[4 * blockIdx.x + 3] = bad ? nan : I.dvol * c;
    }
}

template <typename T>
static hipError_t launch_plain(int kind, const LaunchArgs &a) {
    if (a.ntiles == 0) return hipSuccess;    // (no LDS to raise)
    const dim3 grid(a.ntiles), block(kThreads);
    switch (kind) {
        case KF_GRAD: hipLaunchKernelGGL(k_fd_grad<T>, grid, block, 0, a.stream, a.insts, a.tiles); break;
        case KF_DIV: hipLaunchKernelGGL(k_fd_div<T>, grid, block, 0, a.stream, a.insts, a.tiles); break;
        case KP_THETA:
            hipLaunchKernelGGL(k_probe_theta<T>, grid, block, 0, a.stream, a.insts, a.tiles, a.cst, a.dst, a.target);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_kind(int kind, int lc, int precision, const LaunchArgs &a) {
    if (a.ntiles < 0) return hipErrorInvalidValue;
    const bool dp = precision == 64;
    switch (kind) {
        case KF_GRAD: case KF_DIV: case KP_THETA:
            return dp ? launch_plain<double>(kind, a) : launch_plain<float>(kind, a);
        case KG_X: case KD_X: case KX_THETA: case KX_ASSEMBLE: case KP_U:
            return dp ? launch_x_f64(kind, lc, a.var, a) : launch_x_f32(kind, lc, a.var, a);
        case KG_Y: case KD_Y: case KY_20F: case KY_20I:
            return dp ? launch_y_f64(kind, lc, a.var, a) : launch_y_f32(kind, lc, a.var, a);
        case KG_Z: case KD_Z: case KZ_MAIN: case KP_THETA_K: case KP_U_K:
            return dp ? launch_z_f64(kind, lc, a.var, a) : launch_z_f32(kind, lc, a.var, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_probe(int probe, int lc, int precision, const LaunchArgs &a, void *dst, int target) {
    static const int kinds[4] = {KP_THETA, KP_THETA_K, KP_U_K, KP_U};
    if (probe < 0 || probe > 3) return hipErrorInvalidValue;
    LaunchArgs b = a;
    b.dst = dst;
    b.target = target;
    return launch_kind(kinds[probe], lc, precision, b);
}

hipError_t launch_reduce(const InstDev *insts, int ninst, double *E, hipStream_t stream) {
    hipLaunchKernelGGL(k_reduce, dim3(ninst), dim3(kThreads), 0, stream, insts, E);
    return hipGetLastError();
}

}  // namespace vdwnl
