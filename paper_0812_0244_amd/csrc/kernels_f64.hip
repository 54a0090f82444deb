// The kernels of the FP64 evaluation (see kernels.hpp), the FP64 energy
// reduction both precisions share, and the dispatch by precision.
#include "kernels.hpp"

namespace vdwnl {

hipError_t launch_kind_f32(int kind, int lc, const LaunchArgs &a);
hipError_t launch_probe_f32(int probe, int lc, const LaunchArgs &a, void *dst, int target);

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
        E[4 * blockIdx.x] = 0.5 * I.omega * a;
        E[4 * blockIdx.x + 1] = I.dvol * b;
        E[4 * blockIdx.x + 2] = I.dvol * x;
        E[4 * blockIdx.x + 3] = I.dvol * c;
    }
}

hipError_t launch_kind(int kind, int lc, int precision, const LaunchArgs &a) {
    return precision == 64 ? launch_kind_t<double>(kind, lc, a) : launch_kind_f32(kind, lc, a);
}

hipError_t launch_probe(int probe, int lc, int precision, const LaunchArgs &a, void *dst, int target) {
    return precision == 64 ? launch_probe_t<double>(probe, lc, a, dst, target) : launch_probe_f32(probe, lc, a, dst, target);
}

hipError_t launch_reduce(const InstDev *insts, int ninst, double *E, hipStream_t stream) {
    hipLaunchKernelGGL(k_reduce, dim3(ninst), dim3(kThreads), 0, stream, insts, E);
    return hipGetLastError();
}

}  // namespace vdwnl
