// Shared host/device definitions of libvdwnl.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace vdwnl {

constexpr int kNQ = 20;                          // interpolation points q_a (compile-time)
constexpr int kNPair = kNQ * (kNQ + 1) / 2;      // distinct phi_ab (a <= b) per |G| shell
constexpr int kTabRow = kNQ * kNQ;               // shell table entries per shell (full matrix)
constexpr int kTabPacked = kNQ * (kNQ + 1) / 2;  // the same, packed upper triangle (some general-cell tables)
constexpr size_t kFullRowCacheBytes = (size_t)256 << 20;   // a general-cell table this small keeps full rows
constexpr int kThreads = 256;                    // threads per workgroup, every kernel
constexpr int kTileCap = 4096;                   // complex elements of one LDS FFT tile
constexpr int kLdsCap = 65536;                   // bytes of LDS one workgroup may take
constexpr int kMaxStages = 16;
constexpr int kMaxCols = 16;                     // (k2, k3) columns per fused axis-1 tile
constexpr int kMaxMc = 64;                       // largest m_c of Eq. (Sat)
constexpr int kMaxFd = 4;                        // largest finite-difference half-width
constexpr int kMaxN1 = 204;                      // 20 N1 <= kTileCap (fused axis-1 pass)
constexpr int kMaxN3 = 340;                      // 12 N3 complex doubles <= kLdsCap

// One 1-D FFT length: radix sequence (each 2, 3, 4, 5 or 8) and the offset of
// its twiddles W_n^k = exp(-2 pi i k / n), k < n, in the twiddle table.
struct FftPlan {
    int n;
    int nstage;
    int radix[kMaxStages];
    int tw;
};

// Per-grid state seen by the kernels.  Field layouts (C order):
//   n, v, vloc      [N1][N2][N3] real
//   grad            [3][N1][N2][N3] real  (grad n, Cartesian components, after the
//                   gradient passes (general cells: d_3 n, d_2 n in slots 2, 1
//                   between them); overwritten in place by the assembly with the
//                   lattice components q_c = sum_x W[c][x] w_x of its vector field)
//   spec            [N1][N2][N3h][kNQ] complex  (20 theta / u spectra, component fastest)
//   shellmap        [N1/2+1][N2/2+1][N3h] int   (|G| shell of (|m1|, |m2|, m3)); in a
//                   general (non-orthogonal) cell [N1][N2][N3h] over the whole half spectrum
//   shelltab        [nshell][kNQ][kNQ] real     (phi_ab(|G_s|), the full symmetric matrix:
//                   row a of a shell is contiguous for the lane that forms u_a), or
//                   [nshell][kNQ (kNQ + 1) / 2] (packed upper triangle; some general-cell tables)
struct InstDev {
    int n1, n2, n3, n3h, h1, h2;
    FftPlan p1, p2, p3;
    double inv_n;            // 1 / (N1 N2 N3)
    double B[3][3];          // reciprocal vectors b_c (rows, Cartesian): G = sum_c m_c b_c
    int general;             // non-orthogonal cell: shells over the whole half spectrum
    double omega, dvol;
    int fdm;                 // finite-difference half-width m (0: spectral gradient)
    double fdc[kMaxFd];      // weights c_s of the central formula (unit spacing)
    double fdW[3][3];        // W[c][x] = N_c b_c,x / (2 pi): grad n = sum_c W[c] d_c n
    void *grad, *vloc, *spec;
    const int *shellmap;
    const void *shelltab;
    double *part_ek;         // one partial per fused axis-1 tile
    double *part_de;         // one partial per theta tile
    double *part_sl;         // two per theta tile: E_x and E_c^LDA partials
    int *bad;                // set when a density value is negative, NaN or infinite
    int n_ek, n_de;
    int semilocal;           // add the semilocal terms of Eq. (Exc) (per call)
    const void *n;           // per call
    void *v;                 // per call
};

// Method constants (copied into LDS by the kernels that need them).
struct Consts {
    double qc;
    double iqc;              // 1 / q_c
    double cs;               // C_s
    double nmin;
    int mc;
    int nq;
    double q[kNQ];           // q mesh
    double M[kNQ * kNQ];     // M[j][a]: second derivative at q_j of the cardinal spline p_a
    double invm[kMaxMc + 1]; // 1/m, m <= m_c (coefficients of the saturation series)
};

// One workgroup's work item; the meaning of a, b, c depends on the pass.
struct Tile {
    int inst;
    int a, b, c;
    int slot;                // partial-sum slot within the grid (or -1)
};

enum KernelKind {
    // spectral gradient: one pass per grid axis (one-axis FFTs in FP64)
    KG_X = 0,      // axis 3: d_3 n
    KG_Y,          // axis 2: d_2 n
    KG_Z,          // axis 1: d_1 n, grad n complete (Cartesian components)
    KX_THETA,      // theta_a from n and the stored grad n, R2C theta along axis 3
    KY_20F,        // axis-2 forward, 20 components
    KZ_MAIN,       // axis 1 forward, u = phi c, energy, axis 1 inverse
    KY_20I,        // axis-2 inverse, 20 components
    KX_ASSEMBLE,   // C2R u_a, v_loc, the lattice components q_c of w in place of grad n
    // spectral divergence: v = v_loc - sum_c d_c q_c, one pass per axis
    KD_X,          // axis 3: v = v_loc - d_3 q_3
    KD_Y,          // axis 2: v -= d_2 q_2
    KD_Z,          // axis 1: v -= d_1 q_1
    // finite-difference gradient mode: the stencils replace the per-axis passes
    KF_GRAD,       // grad n by central differences
    KF_DIV,        // v = v_loc - sum_c D_c q_c
    KIND_COUNT
};

// Arguments of one pass launch.  ntiles == 0: no launch, only raise the
// kernel's dynamic LDS limit to lds (done when the launches are planned).
struct LaunchArgs {
    const InstDev *insts;
    const Tile *tiles;
    int ntiles;
    size_t lds;
    const Consts *cst;
    const void *tw;          // twiddles in the working precision
    const void *twd;         // FP64 twiddles (gradient and divergence chains)
    hipStream_t stream;
    const int2 *cols;        // (k2, k3) columns of the fused axis-1 tiles
    int general;             // the launch's grids have non-orthogonal cells (packed shell rows)
    int mfma = 0;            // FP32 orthorhombic fused axis-1 pass: contraction on the matrix cores
    int var = 0;             // radix order of the pass's transform length (0 .. its variants - 1)
    int packed = 0;          // (general cells) the launch's shell tables hold packed upper triangles
    void *dst = nullptr;     // (stage probes) the probe's output
    int target = 0;          // (stage probes) the grid whose tiles run
};

// Parity probes of the stages (the stage values of vdwnl_debug_stage): the
// launch args of the pass the probe replaces (the theta pass for THETA, the
// fused axis-1 pass for THETA_K and U_K, the assembly pass for U); dst the
// probe's output (THETA, U), target the grid whose tiles run.
enum ProbeKind { PROBE_THETA = 0, PROBE_THETA_K = 1, PROBE_U_K = 2, PROBE_U = 3 };
// the probes as launch kinds of their families
enum ProbeLaunch { KP_THETA = KIND_COUNT + 1, KP_THETA_K, KP_U_K, KP_U };

hipError_t launch_kind(int kind, int len_class, int precision, const LaunchArgs &a);
hipError_t launch_probe(int probe, int len_class, int precision, const LaunchArgs &a, void *dst, int target);
// family launchers (kernels_f32_x.hip ...): kind, length class, radix order
hipError_t launch_x_f32(int kind, int lc, int var, const LaunchArgs &a);
hipError_t launch_y_f32(int kind, int lc, int var, const LaunchArgs &a);
hipError_t launch_z_f32(int kind, int lc, int var, const LaunchArgs &a);
hipError_t launch_x_f64(int kind, int lc, int var, const LaunchArgs &a);
hipError_t launch_y_f64(int kind, int lc, int var, const LaunchArgs &a);
hipError_t launch_z_f64(int kind, int lc, int var, const LaunchArgs &a);
hipError_t launch_reduce(const InstDev *insts, int ninst, double *E, hipStream_t stream);

}  // namespace vdwnl
