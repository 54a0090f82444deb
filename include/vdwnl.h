/*
 * vdwnl.h -- C ABI of libvdwnl: the nonlocal correlation energy E_c^nl and
 * potential v_nl of the van der Waals density functional, evaluated with the
 * factorised kernel and FFTs of Roman-Perez and Soler (arXiv:0812.0244) on
 * AMD Instinct MI355X (gfx950).
 *
 * Following the paper's statement of the problem (the paragraph after
 * Eq. (epsofk)), the library accepts the density n(r_i) on a uniform periodic
 * real-space grid and returns E_c^nl and v_nl(r_i) on the same grid (or, with
 * vdwnl_set_functional, the whole E_xc of Eq. (Exc) and v_xc).
 *
 * Conventions
 *  - Hartree atomic units (bohr, Hartree).
 *  - vdwnl_set_grid(s) take orthorhombic cells (lengths L1, L2, L3 along the
 *    three axes), vdwnl_set_grids_lattice cells of any shape (three cell
 *    vectors); arrays are C order [N1][N2][N3] (N3 fastest); r_i =
 *    (i1/N1) a_1 + (i2/N2) a_2 + (i3/N3) a_3 for cell vectors a_c.
 *  - Precision 32 or 64 selects the arithmetic of every device array and
 *    kernel (float / double); global reductions are always FP64.
 *  - Every function returns VDWNL_OK (0) or a negative error code; nothing
 *    throws across the ABI.  vdwnl_strerror() names a code and
 *    vdwnl_last_error() gives the context's last message.
 *  - A context is not thread safe: use it from one host thread and one stream
 *    at a time.  Device pointers passed in are owned by the caller; the
 *    library owns its context and all workspace.
 */
#ifndef VDWNL_H
#define VDWNL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VDWNL_OK = 0,
    VDWNL_E_ARG = -1,               /* null pointer, bad enum, non-positive size */
    VDWNL_E_UNSUPPORTED_SIZE = -2,  /* grid edge with a prime factor > 5, or outside the limits
                                       (edges >= 4; at most 715827882 points) */
    VDWNL_E_NOMEM = -3,             /* device or host allocation failed */
    VDWNL_E_TABLE = -4,             /* kernel table invalid (mesh, symmetry, size) */
    VDWNL_E_KRANGE = -5,            /* radial table does not reach max |G| of a grid */
    VDWNL_E_STATE = -6,             /* grid or table missing, or no device */
    VDWNL_E_HIP = -7,               /* a HIP runtime call failed */
    VDWNL_E_BAD_DENSITY = -8        /* a density value is negative, NaN or infinite (the method
                                       is defined for n >= 0); E and v of that grid are not valid */
};

typedef struct vdwnl_ctx vdwnl_ctx;

/* Create a context on HIP device `device`.  device < 0 creates a host-only
 * context: every validation and planning step runs, nothing touches a GPU,
 * and the evaluation calls return VDWNL_E_STATE. */
int vdwnl_create(vdwnl_ctx **out, int device);

/* Free the context and all its device memory. */
int vdwnl_destroy(vdwnl_ctx *ctx);

const char *vdwnl_strerror(int code);
const char *vdwnl_last_error(const vdwnl_ctx *ctx);

/* Plan one grid (replaces any previous plan).
 *   shape[3]   N1, N2, N3 >= 4, each a product of 2, 3 and 5;
 *              N1 <= 204, N3 <= 408, N2 <= 4096 (one line of each axis must
 *              fit an LDS tile; a device with less LDS may refuse smaller
 *              grids), N1 N2 even
 *   cell[3]    orthorhombic cell lengths, bohr, > 0
 *   grad_mode  0: grad n by spectral differentiation, the Nyquist multiplier
 *              set to zero.  m = 1..4: the paper's choice, finite differences
 *              on the same grid (the potential section, around Eq. (Vi)):
 *              the central formula with m points on each side along every
 *              axis (order 2m), periodic; its weights d(grad n_j)/dn_i give
 *              the gradient term of Eq. (Vi) as minus the same stencil's
 *              divergence.  An edge shorter than 2m + 1 folds coinciding
 *              neighbours' weights together.
 *   precision  32 or 64
 * Device workspace is allocated at the first evaluation after planning
 * (one block, kept across later plans of the context while it is large
 * enough; vdwnl_destroy hands it to the library's per-device pool, from
 * which later contexts take blocks before they allocate, and the pool is
 * held until the process ends); later evaluations allocate nothing.  Tile
 * shapes follow one LDS budget per
 * pass group: a budget set tuned by vdwnl_autotune for the same grid list,
 * precision, gradient mode and device architecture is reused (from this
 * process, or from the tuning file of an earlier one; see vdwnl_autotune),
 * else 64 KB each. */
int vdwnl_set_grid(vdwnl_ctx *ctx, const int32_t shape[3], const double cell[3],
                   int32_t grad_mode, int32_t precision);

/* Plan a batch of nb independent grids evaluated together (same rules as
 * vdwnl_set_grid for each; shapes[nb][3], cells[nb][3]). */
int vdwnl_set_grids(vdwnl_ctx *ctx, int32_t nb, const int32_t *shapes, const double *cells,
                    int32_t grad_mode, int32_t precision);

/* Plan a batch of grids in cells of any shape: lattices[nb][3][3], host,
 * row c = the cell vector a_c in Cartesian bohr (any orientation; a diagonal
 * matrix is the orthorhombic case of vdwnl_set_grids, with identical
 * results).  Grid point i sits at sum_c (i_c / N_c) a_c; the grid is the
 * uniform real-space grid on which the paper's method takes n and returns
 * E and v (paragraph after Eq. (epsofk)).  Wave vectors G = sum_c m_c b_c
 * with the reciprocal vectors a_i . b_j = 2 pi delta_ij; the volume is
 * |det|.  Where the cell is not orthorhombic, |G| at a Nyquist index (which
 * stands for both +-N_c/2) is the mean of |G|^2 over the two (the cross
 * terms of that axis dropped), the kernel table holds one row per distinct
 * |G| over the whole half spectrum (up to about half the grid's points:
 * larger tables and a slower fused axis-1 pass than an orthorhombic cell),
 * and finite differences run along the cell axes, combined into Cartesian
 * components with (N_c / 2 pi) b_c.  Other rules as vdwnl_set_grid.
 * Errors: VDWNL_E_ARG (null pointer, non-finite entry, cell vectors that
 * span no volume), as vdwnl_set_grid otherwise. */
int vdwnl_set_grids_lattice(vdwnl_ctx *ctx, int32_t nb, const int32_t *shapes, const double *lattices,
                            int32_t grad_mode, int32_t precision);

/* The kernel of the factorisation, Eq. (phi), in k space (the radial table
 * described after Eq. (Eoffk)), and the parameters of q0:
 *   nq        number of interpolation points q_a (20 is the supported value)
 *   qmesh     [nq] strictly increasing, qmesh[nq-1] == q_c (host pointer)
 *   q_c, m_c  saturation of Eq. (Sat)
 *   nk, dk    radial mesh k_j = j dk, j < nk
 *   phi       [nq][nq][nk] host array, phi_ab(k_j), symmetric in (a, b)
 *   c_soft    C_s of the local correction, Eqs. (DEnl)/(Depsnl):
 *             Delta E = Int n^2 C_s / q0^3
 * The arrays are copied; the caller keeps ownership.  phi_ab(|G|) is taken
 * from the natural cubic spline through phi_ab(k_j). */
int vdwnl_set_kernel_table(vdwnl_ctx *ctx, int32_t nq, const double *qmesh, double q_c,
                           int32_t m_c, int32_t nk, double dk, const double *phi,
                           double c_soft);

/* E_c^nl and v_nl of one density (the planned grid).
 *   n_dev   device array [N1][N2][N3] of the planned precision (read only)
 *   v_dev   device array of the same shape, receives v_nl (Hartree)
 *   E_out   host double[2]: E_k (the FFT part, Eq. Eoffk) and Delta E (the
 *           local correction, Eq. DEnl); E_c^nl = E_out[0] + E_out[1]
 *   stream  hipStream_t to run on (0: the null stream); the call returns
 *           after the stream has finished the evaluation.
 * The theta pass checks every density value as it reads it (no extra pass):
 * a negative, NaN or infinite value makes both energies NaN and the call
 * return VDWNL_E_BAD_DENSITY (v is then not valid either); the next
 * evaluation starts clean.  The batched calls do the same per grid (the
 * other grids' results stay valid; the asynchronous call reports it only
 * through the NaN energies in E_dev). */
int vdwnl_energy_potential(vdwnl_ctx *ctx, const void *n_dev, void *v_dev, double *E_out,
                           void *stream);

/* As vdwnl_energy_potential, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation): this call allocates nothing, neither device nor host memory,
 * and calls no allocating library routine.  Every device structure of the
 * evaluation (the per-grid fields and spectra, tile lists, twiddles, kernel
 * rows, partial sums, instance table and energies) lives in one buffer of
 * 64 MiB, a static device array of the library, one per GPU the library runs
 * on (each held from the library's first use of that GPU until the process
 * ends; its address is taken when a context is created).  A plan fits when
 * its whole image does: about 64^3 points in FP32 or 48^3 in FP64 for cubic
 * grids in orthorhombic cells, about 48^3 in FP32 in general cells (whose
 * kernel rows, one set per k point, are then kept as packed upper
 * triangles); larger plans return VDWNL_E_UNSUPPORTED_SIZE with the bytes
 * they need in vdwnl_last_error.  Every call on a GPU shares that GPU's buffer and
 * it keeps the last call's contents: nothing in it must start at zero (each
 * evaluation writes every value before reading it), the tables of the plan
 * are copied in when the buffer holds another plan's, and calls that overlap
 * on one GPU (from other threads or on other streams) race.  The context must
 * hold a single grid (vdwnl_set_grid); E_out is a host double[2] as in
 * vdwnl_energy_potential; the passes are launched one by one on `stream` and
 * the call returns after the stream has finished.  The semilocal energies of
 * the whole functional are not kept (vdwnl_semilocal_energies returns
 * VDWNL_E_STATE after this call).  Errors: VDWNL_E_ARG (null pointer),
 * VDWNL_E_STATE (no grid or table, a batch plan, a host-only context,
 * per-pass timing on), VDWNL_E_UNSUPPORTED_SIZE (the plan exceeds the
 * buffer), VDWNL_E_KRANGE, VDWNL_E_HIP, VDWNL_E_BAD_DENSITY (as
 * vdwnl_energy_potential). */
int vdwnl_energy_potential_noalloc(vdwnl_ctx *ctx, const void *n_dev, void *v_dev, double *E_out,
                                   void *stream);

/* The planned batch: n_ptrs[nb], v_ptrs[nb] device pointers, E_out[nb][2].
 * The first evaluation after planning captures the whole evaluation (every
 * pass of every grid, the reduction and the copy of the energies) into a HIP
 * graph on a private stream; later calls replay it on `stream`.  The graph
 * reads the density and potential pointers of each call from pinned host
 * memory when it runs, so any buffers may be passed. */
int vdwnl_energy_potential_batched(vdwnl_ctx *ctx, int32_t nb, const void *const *n_ptrs,
                                   void *const *v_ptrs, double *E_out, void *stream);

/* As vdwnl_energy_potential_batched, without waiting for the result: the
 * call returns once the evaluation is enqueued on `stream`, and E_dev, a
 * device array double[nb][2], receives (E_k, Delta E) of every grid on that
 * stream (the paper's E as a device value, for callers that keep the
 * evaluation inside their own stream-ordered work).  The density and
 * potential buffers must stay valid until the stream has passed the
 * evaluation.  The next call on the context (any evaluation, re-planning,
 * vdwnl_semilocal_energies, vdwnl_debug_field, destroy) first waits on the
 * host until this evaluation has finished, since it reads the context's
 * pinned instance table.  VDWNL_E_ARG for a null E_dev; VDWNL_E_STATE while per-pass timing
 * is on; otherwise the errors of the synchronous call. */
int vdwnl_energy_potential_batched_async(vdwnl_ctx *ctx, int32_t nb, const void *const *n_ptrs,
                                         void *const *v_ptrs, double *E_dev, void *stream);

/* Which functional an evaluation computes (Eq. (Exc) of the paper:
 * E_xc = E_x^GGA + E_c^LDA + E_c^nl).
 *   VDWNL_FUNCTIONAL_NONLOCAL (the default): v = v_nl, E_c^nl only.
 *   VDWNL_FUNCTIONAL_VDW_DF: the whole functional.  v receives v_xc =
 *     v_nl + v_x + v_c^LDA, where the semilocal terms are the revPBE GGA
 *     exchange of Zhang and Yang (the PBE enhancement factor
 *     F_x = 1 + kappa - kappa / (1 + mu s^2 / kappa), kappa = 1.245,
 *     mu = 0.066725 pi^2 / 3) and the Perdew-Wang 1992 LDA correlation (the
 *     LDA inside q0); their gradient parts go through the same adjoint of the
 *     gradient as the nonlocal term (the paper's Sec. on the potential,
 *     around Eq. (Vi)).  E_out still holds (E_k, Delta E); the semilocal
 *     energies come from vdwnl_semilocal_energies.
 * The setting applies from the next evaluation on (no re-planning; a
 * captured graph reads it from the instance table).  VDWNL_E_ARG for any
 * other value. */
enum { VDWNL_FUNCTIONAL_NONLOCAL = 0, VDWNL_FUNCTIONAL_VDW_DF = 1 };
int vdwnl_set_functional(vdwnl_ctx *ctx, int32_t functional);

/* E_out[nb][2] (host): E_x^GGA and E_c^LDA (Hartree, FP64 sums) of every grid
 * of the last evaluation, which must have run with VDWNL_FUNCTIONAL_VDW_DF
 * (else VDWNL_E_STATE; also before any evaluation and after re-planning).
 * nb must equal the planned number of grids (VDWNL_E_ARG). */
int vdwnl_semilocal_energies(const vdwnl_ctx *ctx, int32_t nb, double *E_out);

/* Copy an internal per-grid field of the last evaluation of grid `inst` to
 * the device buffer dst (for parity probes): which = 0: the components
 * q_c = sum_x W[c][x] w_x (W[c][x] = N_c b_c,x / (2 pi), N_c / L_c on the
 * diagonal of an orthorhombic cell) of the vector field
 * w = sum_a u_a dtheta_a/dgrad n + de/dgrad n of Eq. (Vi), [3][N] (they
 * overwrite grad n in place; grad n itself: vdwnl_debug_stage with
 * VDWNL_STAGE_GRAD); 1: v_loc [N] (the local
 * part of v, before the gradient term; with the whole functional it includes
 * the semilocal terms' local parts).  Arrays in the planned precision. */
int vdwnl_debug_field(vdwnl_ctx *ctx, int32_t inst, int32_t which, void *dst, void *stream);

/* Parity probe of one stage of the method for grid `inst` (0-based) of the
 * planned batch.  The passes of the last evaluation run again, launched one
 * by one on `stream`, up to the stage, with the same density buffers (they
 * must still hold the density of that evaluation; the potential buffers are
 * not written), and the stage's values are written to the caller's device
 * buffer dst (planned precision, C order):
 *   VDWNL_STAGE_THETA    theta_a(r_i) = n_i p_a(q0_i), the weighted densities
 *                        of the factorised kernel (the text after
 *                        Eq. (Eoffk)); real [20][N1][N2][N3]
 *   VDWNL_STAGE_THETA_K  their transforms c_a(G) = FFT(theta_a)(G) / N
 *                        (Eq. (Eoffk)) on the half spectrum m_3 = 0..N3/2;
 *                        complex [N1][N2][N3/2+1][20] (re, im pairs; the 20
 *                        components of a wave vector contiguous); index k_c
 *                        of axes 1, 2 in FFT order (frequency k_c, or
 *                        k_c - N_c above N_c/2)
 *   VDWNL_STAGE_U_K      u_a(G) = sum_b phi_ab(|G|) c_b(G), the per-k
 *                        contraction of Eqs. (epsofk); same layout
 *   VDWNL_STAGE_U        u_a(r_i) = sum_G u_a(G) exp(i G . r_i)
 *                        (Eq. (epsilon): u_ai = dOmega^-1 dE_k/dtheta_ai);
 *                        real [20][N1][N2][N3]
 *   VDWNL_STAGE_GRAD     grad n as the theta pass takes it (the gradient of
 *                        q0's argument, Eq. (q0)), Cartesian components;
 *                        real [3][N1][N2][N3]
 * Returns after the stream has finished.  The workspace is left as the probe
 * left it; the next evaluation recomputes everything.  VDWNL_E_ARG for a null
 * pointer or an unknown stage; VDWNL_E_STATE before the first evaluation of
 * the plan or for an index outside the batch. */
enum { VDWNL_STAGE_THETA = 0, VDWNL_STAGE_THETA_K = 1, VDWNL_STAGE_U_K = 2, VDWNL_STAGE_U = 3, VDWNL_STAGE_GRAD = 4 };
int vdwnl_debug_stage(vdwnl_ctx *ctx, int32_t inst, int32_t stage, void *dst, void *stream);

/* The logarithmic mesh of interpolation points of the factorisation (the
 * paragraph before Eq. (qsat)): q_1 = q1, q_nq = q_c, and increments that grow
 * by the factor lambda, (q_{a+1} - q_a) = lambda (q_a - q_{a-1}).  Host only
 * (no device, no context).  q_out: host array [nq].  VDWNL_E_ARG unless
 * 2 <= nq <= 4096, 0 < q1 < q_c, lambda >= 1 (1: a uniform mesh) and
 * lambda^(nq-2) finite. */
int vdwnl_log_qmesh(int32_t nq, double q1, double q_c, double lambda, double *q_out);

/* Per-pass timing.  vdwnl_set_timing(ctx, 1) clears the counters and makes
 * every later evaluation record a HIP event after each of its passes (on the
 * evaluation's stream); vdwnl_pass_times copies the accumulated milliseconds
 * of every pass kind (indexed by kind, the FP64 energy reduction last; kinds
 * the planned gradient mode does not launch stay 0) into ms[], the number of
 * timed evaluations into *calls, and returns the number of entries.
 * vdwnl_pass_name(k) names kind k ("" outside the range); vdwnl_pass_order
 * writes the kinds the planned mode launches, in launch order, into kinds[]
 * (at most max_passes) and returns their number.  Timed evaluations launch
 * their passes one by one (no graph). */
int vdwnl_set_timing(vdwnl_ctx *ctx, int32_t on);
int vdwnl_pass_times(const vdwnl_ctx *ctx, int32_t max_passes, double *ms, int64_t *calls);
const char *vdwnl_pass_name(int32_t i);
int vdwnl_pass_order(const vdwnl_ctx *ctx, int32_t max_passes, int32_t *kinds);

/* Graph replay on (default, on != 0) or off (every evaluation launches its
 * passes one by one; results are identical). */
int vdwnl_set_graph(vdwnl_ctx *ctx, int32_t on);

/* Schedule tuning for the planned grids: evaluates the batch (n_ptrs[nb],
 * v_ptrs[nb] as for vdwnl_energy_potential_batched; v is overwritten) once
 * plus `reps` timed times (1..100) for each candidate LDS budget (and, for
 * FP32 orthorhombic grids, each contraction unit) at radix order 0, the first
 * candidate after some 300 ms of untimed evaluations so that the device's
 * clocks have risen before any timing, keeps
 * the unit of the fused axis-1 pass with the least time over that pass, then
 * times every candidate budget at every radix order (0..5) with that unit and
 * picks per pass group the (budget, order) pair with the least time over the
 * group's passes, plans with the choices and remembers them, keyed by the device
 * architecture, its LDS size,
 * the precision, the gradient mode and the exact grid list: for the rest of
 * the process, and in the tuning file for later processes.  The file is a
 * JSON object with one entry per line, "<arch>/<key hash>": [five budgets,
 * the contraction unit, five radix orders],
 * at $VDWNL_TUNE_CACHE (an empty value: no file), else
 * $XDG_CACHE_HOME/vdwnl/tuning.json or $HOME/.cache/vdwnl/tuning.json; a file
 * that cannot be read or written is ignored.  Results do not depend on the
 * tile shapes beyond rounding order.  Returns an error code as the
 * evaluation does. */
int vdwnl_autotune(vdwnl_ctx *ctx, int32_t nb, const void *const *n_ptrs, void *const *v_ptrs,
                   int32_t reps, void *stream);

/* Schedule choices of the evaluation (they change no result beyond the order
 * of FP32 additions):
 *   VDWNL_SCHEDULE_CONTRACTION  the unit that forms the per-k contraction
 *     u_a(k) = sum_b phi_ab(|k|) c_b(k) of Eqs. (Eoffk)/(epsofk) in the fused
 *     axis-1 pass of FP32 grids in orthorhombic cells:
 *     VDWNL_CONTRACTION_VECTOR (the vector ALU, a lane per output component)
 *     or VDWNL_CONTRACTION_MATRIX (the matrix cores: 16-block 4 x 4 x 1 FP32
 *     outer products, 15 blocks per instruction for the 20 x 20 matrices of
 *     three k-point groups); FP64 and general cells always use the vector ALU.
 *   VDWNL_SCHEDULE_RADIX_*  the radix order of a pass group's transforms.
 * vdwnl_autotune chooses the contraction unit together with the LDS budgets,
 * then the radix orders (and a plan reuses tuned choices as it does the
 * budgets); untuned, the matrix cores and order 0.  Setting a choice
 * re-plans the launches (the workspace is rebuilt at the next evaluation).
 * VDWNL_E_ARG for an unknown choice or value; VDWNL_E_STATE without a planned
 * grid. */
enum {
    VDWNL_SCHEDULE_CONTRACTION = 0,
    /* radix order of the transforms of each pass group (0..5): every axis-3
     * transform, the axis-2 transforms of the 20 spectra, the other axis-2
     * transforms, the fused axis-1 pass, the other axis-1 passes.  Each length
     * with a compile-time plan has one to six orders (vdwnl_radix_order),
     * and a larger value takes its last; other lengths have one. */
    VDWNL_SCHEDULE_RADIX_X = 1,
    VDWNL_SCHEDULE_RADIX_Y20 = 2,
    VDWNL_SCHEDULE_RADIX_YAUX = 3,
    VDWNL_SCHEDULE_RADIX_Z = 4,
    VDWNL_SCHEDULE_RADIX_ZAUX = 5
};
enum { VDWNL_CONTRACTION_VECTOR = 0, VDWNL_CONTRACTION_MATRIX = 1 };
int vdwnl_set_schedule(vdwnl_ctx *ctx, int32_t what, int32_t value);
int vdwnl_get_schedule(const vdwnl_ctx *ctx, int32_t what, int32_t *value);

/* The radix passes (each 2, 3, 4, 5, 8 or 16, in order) of the transform of
 * length n in radix order `order` (0..5; a larger order than the length has
 * takes its last): up to max_radices values into radices[] (host array).
 * Returns their number, VDWNL_E_ARG for bad arguments, or
 * VDWNL_E_UNSUPPORTED_SIZE for a length with a prime factor above 5.  Host
 * only (no context, no device). */
int vdwnl_radix_order(int32_t n, int32_t order, int32_t max_radices, int32_t *radices);

/* LDS budget (bytes) of each pass group in the current plan, in the order
 * axis-3 (theta, assembly), axis-2 over the 20 spectra, axis-2 over the
 * gradient / divergence spectra, axis-1 with the contraction, axis-1 of the
 * gradient / divergence; copies up to max_groups values and returns the
 * number of groups (5). */
int vdwnl_get_tiling(const vdwnl_ctx *ctx, int32_t max_groups, int64_t *lds_budget);

/* Set the five LDS budgets (bytes, same order, each in [4096, the device's
 * LDS per workgroup]) and re-plan the tiles of the planned grids (the
 * workspace is rebuilt at the next evaluation). */
int vdwnl_set_tiling(vdwnl_ctx *ctx, int32_t ngroups, const int64_t *lds_budget);

/* Build the kernel table that vdwnl_set_kernel_table takes, on GPU `device`
 * (the step before the evaluation; it depends only on the q mesh and the
 * soft-kernel parameters, so it is computed once):
 *   phi_ab(k_j) = 4 pi Int r^2 j0(k_j r) phi_s(q_a r, q_b r) dr,  k_j = j dk,
 * with phi the kernel of Eq. (Enl) (Dion et al. form: a double integral over
 * plane-wave variables) softened below D = sqrt(d1^2 + d2^2) = d_s as in
 * Eq. (PhiSoft) (phi_s = phi0 + phi2 D^2 + phi4 D^4, value and slope matched
 * at d_s on each ray d2/d1 = q_b/q_a), and
 *   C_s = 1/2 Int_0^{d_s/sqrt2} 4 pi d^2 [phi(d,d) - phi_s(d,d)] dd
 * of Eq. (Depsnl).  qmesh[nq] increasing (host); phi_out host array
 * [nq][nq][nk] (caller-owned, filled symmetric); *c_soft_out host double.
 * Takes a few seconds on an MI355X.  Errors: VDWNL_E_ARG, VDWNL_E_TABLE (q
 * mesh not increasing), VDWNL_E_STATE (device < 0), VDWNL_E_HIP. */
int vdwnl_build_kernel_table(int device, int32_t nq, const double *qmesh, double d_s, double phi0,
                             int32_t nk, double dk, double *phi_out, double *c_soft_out);

/* The kernel phi(d1, d2) of Eq. (Enl) itself, by the generator's double
 * integral, on GPU `device`: out[i] = phi(d1[i], d2[i]) (Hartree), host
 * arrays of n values, 0 < d1, d2 <= 460.  E_ARG for other arguments. */
int vdwnl_kernel_phi(int device, int32_t n, const double *d1, const double *d2, double *out);

/* Number of planned grids and the bytes of device workspace held. */
int vdwnl_info(const vdwnl_ctx *ctx, int32_t *n_grids, int64_t *workspace_bytes);

#ifdef __cplusplus
}
#endif

#endif /* VDWNL_H */
