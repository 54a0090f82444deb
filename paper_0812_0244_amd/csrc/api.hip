// Host side of libvdwnl: contexts, argument checks, planning and the C ABI.
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vdwnl.h"
#include "common.hpp"
#include "fft_fast.hpp"

namespace vdwnl {

// ---------------------------------------------------------------- planning helpers

static bool radix_plan(int n, FftPlan &p) {
    p.n = n;
    p.nstage = 0;
    int m = n;
    // radix-8 passes first, then 4 / 2, then 3 and 5
    while (m % 8 == 0 && m > 1) { p.radix[p.nstage++] = 8; m /= 8; }
    while (m % 4 == 0) { p.radix[p.nstage++] = 4; m /= 4; }
    while (m % 2 == 0) { p.radix[p.nstage++] = 2; m /= 2; }
    while (m % 5 == 0) { p.radix[p.nstage++] = 5; m /= 5; }
    while (m % 3 == 0) { p.radix[p.nstage++] = 3; m /= 3; }
    return m == 1 && p.nstage <= kMaxStages;
}

// Second derivatives of the natural cubic spline through y[j] on the nodes
// x[j] (Thomas algorithm for the tridiagonal continuity equations).
static void natural_spline_d2(const double *x, const double *y, int n, double *d2) {
    std::vector<double> c(n, 0.0), r(n, 0.0);
    d2[0] = d2[n - 1] = 0.0;
    if (n < 3) { for (int i = 0; i < n; ++i) d2[i] = 0.0; return; }
    // rows 1..n-2: h_{j-1} M_{j-1} + 2 (h_{j-1} + h_j) M_j + h_j M_{j+1} = rhs_j
    double cprev = 0.0, rprev = 0.0;
    for (int j = 1; j < n - 1; ++j) {
        const double hl = x[j] - x[j - 1], hr = x[j + 1] - x[j];
        const double rhs = 6.0 * ((y[j + 1] - y[j]) / hr - (y[j] - y[j - 1]) / hl);
        const double diag = 2.0 * (hl + hr) - hl * cprev;
        c[j] = hr / diag;
        r[j] = (rhs - hl * rprev) / diag;
        cprev = c[j];
        rprev = r[j];
    }
    d2[n - 2] = r[n - 2];
    for (int j = n - 3; j >= 1; --j) d2[j] = r[j] - c[j] * d2[j + 1];
}

struct Shells {
    std::vector<int> map;       // [h1][h2][n3h] (orthorhombic) or [N1][N2][n3h] (general cell)
    std::vector<double> gmod;   // |G| per shell
    double gmax = 0.0;
    bool general = false;       // non-orthogonal cell: one k point per shell
    bool packed = false;        // table rows as the packed upper triangle (else the full matrix)
};

static Shells shells_from_keys(const std::vector<double> &key) {
    Shells sh;
    std::vector<double> u(key);
    std::sort(u.begin(), u.end());
    u.erase(std::unique(u.begin(), u.end()), u.end());
    sh.map.resize(key.size());
    for (size_t i = 0; i < key.size(); ++i)
        sh.map[i] = (int)(std::lower_bound(u.begin(), u.end(), key[i]) - u.begin());
    sh.gmod.resize(u.size());
    for (size_t i = 0; i < u.size(); ++i) sh.gmod[i] = std::sqrt(std::max(u[i], 0.0));
    sh.gmax = sh.gmod.back();
    return sh;
}

// General cell: |G|^2 = sum_cd m_c m_d (b_c . b_d) at every point of the half
// spectrum (m_1, m_2 in FFT order, Nyquist -N/2; m_3 = k3).  A Nyquist index
// stands for both signs +-N_c/2, whose |G| differ when the cell is not
// orthogonal: |G|^2 there is the mean over the two (the cross terms of that
// axis dropped), so G and -G always meet the same value.
static Shells build_shells_general(const int s[3], const double B[3][3]) {
    double M[3][3];
    for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) M[c][d] = B[c][0] * B[d][0] + B[c][1] * B[d][1] + B[c][2] * B[d][2];
    const int n3h = s[2] / 2 + 1;
    std::vector<double> key((size_t)s[0] * s[1] * n3h);
    for (int k1 = 0; k1 < s[0]; ++k1)
        for (int k2 = 0; k2 < s[1]; ++k2)
            for (int k3 = 0; k3 < n3h; ++k3) {
                const int k[3] = {k1, k2, k3};
                double m[3];
                bool nyq[3];
                for (int c = 0; c < 3; ++c) {
                    const int n = s[c];
                    const int mc = (c < 2 && k[c] >= (n + 1) / 2) ? k[c] - n : k[c];
                    m[c] = (double)mc;
                    nyq[c] = (n % 2 == 0) && (mc == n / 2 || mc == -n / 2);
                }
                double g2 = M[0][0] * m[0] * m[0] + M[1][1] * m[1] * m[1] + M[2][2] * m[2] * m[2];
                for (int c = 0; c < 3; ++c)
                    for (int d = c + 1; d < 3; ++d)
                        if (!nyq[c] && !nyq[d]) g2 += 2.0 * M[c][d] * m[c] * m[d];
                key[((size_t)k1 * s[1] + k2) * n3h + k3] = g2;
            }
    return shells_from_keys(key);
}

static Shells build_shells(const int s[3], const double cell[3]) {
    Shells sh;
    const int h1 = s[0] / 2 + 1, h2 = s[1] / 2 + 1, n3h = s[2] / 2 + 1;
    const double g1 = 2.0 * M_PI / cell[0], g2 = 2.0 * M_PI / cell[1], g3 = 2.0 * M_PI / cell[2];
    std::vector<double> key((size_t)h1 * h2 * n3h);
    for (int a = 0; a < h1; ++a)
        for (int b = 0; b < h2; ++b)
            for (int c = 0; c < n3h; ++c) {
                const double x = g1 * a, y = g2 * b, z = g3 * c;
                key[((size_t)a * h2 + b) * n3h + c] = x * x + y * y + z * z;
            }
    (void)sh;
    return shells_from_keys(key);
}

// Contraction unit of a plan with no tuned choice.
constexpr int kDefaultContraction = VDWNL_CONTRACTION_MATRIX;

// Pass groups whose tile shapes follow one LDS budget each.
enum TileGroup { TG_X = 0, TG_Y20, TG_YAUX, TG_Z, TG_ZAUX, TG_COUNT };

// The pass group whose radix order a pass takes: every axis-3 transform, the
// axis-2 transforms of the 20 spectra, the other axis-2 transforms (the
// gradient and divergence), the fused axis-1 pass, the other axis-1 passes.
static int variant_group(int kind) {
    switch (kind) {
        case KY_20F: case KY_20I: return TG_Y20;
        case KG_Y: case KD_Y: return TG_YAUX;
        case KZ_MAIN: return TG_Z;
        case KG_Z: case KD_Z: return TG_ZAUX;
        default: return TG_X;
    }
}

struct Grid {
    int s[3];
    double A[3][3];          // cell vectors a_c (rows, bohr)
    double B[3][3];          // reciprocal vectors b_c (rows): a_i . b_j = 2 pi delta_ij
    bool general;            // a_c not all along the axes: full-spectrum shells, no column pairing
    double cell[3];          // |a_c| (the orthorhombic lengths when !general)
    FftPlan p1, p2, p3;
    int bmain;               // rows per theta / assemble tile
    int bnf;                 // rows per axis-3 derivative tile (and stencil tile; even)
    int k3main;              // k3 per fused axis-1 tile (20 comps)
    int wy20;                // axis-2 tile width of the 20 spectra
    int wdy, wdz;            // i3 per axis-2 / axis-1 derivative tile
    int shell_key;           // index into Ctx::shells
    size_t off_grad, off_vloc, off_spec, off_map, off_tab, off_ek, off_de, off_sl, off_bad;
    int n_ek, n_de;
    size_t npts() const { return (size_t)s[0] * s[1] * s[2]; }
    size_t nhalf() const { return (size_t)s[0] * s[1] * (s[2] / 2 + 1); }
};

// Host image of the device state of a plan: the layout of one device buffer
// (per-grid fields, shell maps and kernel rows, then the tile list, the
// columns of the fused axis-1 tiles, twiddles, method constants, the
// instance table and the energies), the contents of its tables and the
// launches of every pass.  Host work only (no HIP call); the kernel rows are
// kept only when asked (they are recomputed at upload time otherwise).
struct Image {
    std::vector<Tile> tiles;
    std::vector<int2> cols;
    std::vector<double> twd;                  // FP64 twiddles, (re, im) pairs
    std::vector<float> tw32;                  // the same in FP32 (FP32 plans)
    std::vector<std::vector<char>> tabs;      // kernel rows per shells entry (working precision), if kept
    size_t ws = 0;                            // per-grid fields, shell maps and rows
    size_t off_tiles = 0, off_cols = 0, off_tw = 0, off_twd = 0, off_consts = 0, off_inst = 0, off_E = 0;
    size_t total = 0;
};

// Device pointers into one buffer that holds an image.
struct DevPtrs {
    char *base = nullptr;
    InstDev *inst = nullptr;
    Tile *tiles = nullptr;
    Consts *consts = nullptr;
    void *tw = nullptr, *twd = nullptr;     // twiddles in the working precision, FP64 twiddles
    int2 *cols = nullptr;                   // (k2, k3) columns of the fused axis-1 tiles
    double *E = nullptr;
};

}  // namespace vdwnl

using namespace vdwnl;

struct vdwnl_ctx {
    int device = -1;
    size_t lds_cap = kLdsCap;             // LDS bytes one workgroup may take on this device
    int precision = 32;
    int grad_mode = 0;
    int functional = VDWNL_FUNCTIONAL_NONLOCAL;
    int last_functional = -1;             // of the last finished evaluation (-1: none)
    // an evaluation enqueued by the asynchronous call and not yet waited for
    hipEvent_t done_ev = nullptr;
    bool pending = false;
    int pending_functional = -1;
    std::string err;
    size_t pref[TG_COUNT] = {kLdsCap, kLdsCap, kLdsCap, kLdsCap, kLdsCap};   // LDS budget per pass group
    int contraction = VDWNL_CONTRACTION_VECTOR;   // unit of the per-k contraction (FP32, orthorhombic)
    int variant[TG_COUNT] = {0, 0, 0, 0, 0};        // radix order per pass group
    std::string plan_key;                 // identifies the batch for the tuned-budget cache
    std::string arch = "host";            // device architecture (gcnArchName)
    // plan
    std::vector<Grid> grids;
    std::vector<Shells> shells;
    std::vector<std::pair<std::vector<double>, int>> shell_keys;   // (shape, cell) -> shells index
    bool have_grid = false;
    // table
    bool have_table = false;
    int nq = 0, mc = 0, nk = 0;
    double qc = 0, dk = 0, cs = 0;
    std::vector<double> qmesh, phi, d2;   // phi, d2 packed [pair][nk]
    Consts consts;
    // device state
    bool device_ready = false;            // tables built for the current (grid, table)
    bool evaluated = false;               // an evaluation has run on the current workspace
    void *work = nullptr;
    size_t work_bytes = 0;
    size_t work_cap = 0;                  // bytes of the allocation at work (kept across re-plans)
    std::vector<size_t> tab_off;          // per shells entry: offset of map and table
    std::vector<size_t> map_off;
    DevPtrs dp;                           // the image in the context's own buffer (work)
    InstDev *h_inst = nullptr;            // pinned
    // the host image of the plan, kept for the no-allocation entry point
    // when the plan fits its scratch buffer (with the kernel rows)
    Image img;
    bool img_valid = false;
    size_t img_need = 0;                  // bytes of the plan's image (0: no plan)
    uint64_t plan_stamp = 0;              // changes whenever the image does
    std::vector<InstDev> na_inst;         // instance table of the no-allocation entry point
    std::vector<double> na_E;             // its energies (host)
    struct Launch {
        int kind, lc, off, cnt;
        size_t lds;
        int group;
        int general;          // grids of the group in non-orthogonal cells
        int mfma;             // (fused axis-1 pass) the contraction on the matrix cores
        int var;              // radix order of the transform (its length class's variant)
        int packed;           // (general cells) shell tables of packed upper triangles
    };
    // per pass: one launch per group of grids (grids whose three axes fall in
    // the same FFT length classes); the groups' chains of passes are
    // independent of each other
    std::vector<Launch> launches[KIND_COUNT];
    int ngroups = 0;
    std::vector<hipStream_t> chain_streams;   // one per group (graph capture)
    std::vector<hipEvent_t> chain_events;     // fork (index 0) and one join per group
    double *h_E = nullptr;                // pinned
    std::map<int, int> tw_off;            // length -> offset
    // the evaluation captured as a HIP graph (replayed on the caller's stream)
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // per-pass timing (pass_ms by kind, the reduction last; events by launch position)
    bool timing = false;
    hipEvent_t ev[KIND_COUNT + 2] = {};
    bool ev_made = false;
    double pass_ms[KIND_COUNT + 1] = {0};
    int64_t timed_calls = 0;
};

namespace vdwnl {

static int fail(vdwnl_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

static int check_krange(vdwnl_ctx *c);

// The theta pass flags a grid whose density holds a negative, NaN or
// infinite value; the reduction then makes all its energies NaN.
static int check_density_flags(vdwnl_ctx *c, const double *E4, int nb) {
    for (int i = 0; i < nb; ++i)
        if (E4[4 * i] != E4[4 * i])
            return fail(c, VDWNL_E_BAD_DENSITY,
                        "grid " + std::to_string(i) + ": a density value is negative, NaN or infinite");
    return VDWNL_OK;
}
static void refresh_image(vdwnl_ctx *c);

static int hipfail(vdwnl_ctx *c, hipError_t e, const char *what) {
    return fail(c, VDWNL_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Wait (on the host) for the evaluation the asynchronous call left in
// flight: it reads the pinned instance table and writes the pinned energies.
static int wait_pending(vdwnl_ctx *c) {
    if (!c->pending) return VDWNL_OK;
    c->pending = false;
    const hipError_t e = hipEventSynchronize(c->done_ev);
    if (e != hipSuccess) return hipfail(c, e, "wait for the previous evaluation");
    c->last_functional = c->pending_functional;
    return VDWNL_OK;
}

static void drop_graph(vdwnl_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
}

// Workspace allocations of the process, per device: device memory that the
// kernels of a captured graph had used was not returned to the device when
// freed on this runtime (measured: one workspace lost per re-plan or per
// destroyed context with graph replay), so workspaces are never freed.  A
// context keeps its allocation across re-plans while it is large enough;
// a destroyed context (or one that needs a larger block) hands it to this
// pool, and a context takes the smallest pooled block that is large enough
// before it allocates.  Memory held: the peak of the workspaces in use at
// once (plus the blocks' slack).
struct WorkBlock {
    int device;
    void *ptr;
    size_t bytes;
};
static std::mutex g_pool_mu;
static std::vector<WorkBlock> g_pool;

static void pool_put(int device, void *ptr, size_t bytes) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool.push_back({device, ptr, bytes});
}

// free every pooled block of this device (the allocation's last resort:
// blocks that no graph used do come back)
static void pool_release(int device) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    std::vector<WorkBlock> keep;
    for (auto &b : g_pool) {
        if (b.device == device) (void)hipFree(b.ptr);
        else keep.push_back(b);
    }
    g_pool.swap(keep);
}

// the smallest pooled block of this device with at least `need` bytes, or null
static void *pool_take(int device, size_t need, size_t *bytes) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    size_t best = g_pool.size();
    for (size_t i = 0; i < g_pool.size(); ++i)
        if (g_pool[i].device == device && g_pool[i].bytes >= need &&
            (best == g_pool.size() || g_pool[i].bytes < g_pool[best].bytes))
            best = i;
    if (best == g_pool.size()) return nullptr;
    void *p = g_pool[best].ptr;
    *bytes = g_pool[best].bytes;
    g_pool.erase(g_pool.begin() + (long)best);
    return p;
}

// Drop the device state of the plan.  The workspace allocation is kept for
// the next plan of the context; release_work (context destruction) hands it
// to the process's pool.
static void free_device(vdwnl_ctx *c, bool release_work = false) {
    if (c->device >= 0) (void)hipSetDevice(c->device);
    (void)wait_pending(c);
    c->last_functional = -1;
    if (c->device < 0) return;
    if (c->done_ev) (void)hipEventDestroy(c->done_ev);
    c->done_ev = nullptr;
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    c->cap_stream = nullptr;
    for (auto s : c->chain_streams) (void)hipStreamDestroy(s);
    c->chain_streams.clear();
    for (auto ev : c->chain_events) (void)hipEventDestroy(ev);
    c->chain_events.clear();
    if (c->ev_made) {
        for (auto &e : c->ev) (void)hipEventDestroy(e);
        c->ev_made = false;
    }
    if (release_work && c->work) {
        pool_put(c->device, c->work, c->work_cap);
        c->work = nullptr;
        c->work_cap = 0;
    }
    if (c->h_inst) (void)hipHostFree(c->h_inst);
    if (c->h_E) (void)hipHostFree(c->h_E);
    c->h_inst = nullptr; c->h_E = nullptr;
    c->dp = DevPtrs();
    c->work_bytes = 0;
    c->device_ready = false;
    c->evaluated = false;
}

static bool smooth235(int n) {
    if (n < 1) return false;
    for (int p : {2, 3, 5}) while (n % p == 0) n /= p;
    return n == 1;
}

// LDS of one theta / assembly tile of b rows: the 20 fields' pair lines,
// twiddles and method constants.
static size_t xpass_lds(size_t b, size_t N3, size_t rs) {
    const size_t cs = 2 * rs;
    return b * (N3 + 1) * (kNQ / 2) * cs + N3 * cs + (kNQ + kNQ * kNQ) * rs + (kMaxMc + 1) * 8;
}

// LDS of one derivative tile of a one-axis pass: twiddles and np lines of
// length L, complex elements of ce bytes (16: the gradient's FP64, or the
// working precision's for the divergence); lines at pitch L | 1 along axes
// 2 and 1, at pitch N3 + 1 along axis 3 (the rows).
static size_t deriv_lds(size_t L, size_t np, size_t ce) { return (L + np * (L | 1)) * ce; }
static size_t drow_lds(size_t N3, size_t np, size_t ce) { return (N3 + np * (N3 + 1)) * ce; }

// lattice: 9 values, rows a_1, a_2, a_3 (bohr)
static int check_grid(vdwnl_ctx *c, const int32_t *shape, const double *lattice, int precision, Grid &g) {
    const size_t cs = precision == 64 ? 16 : 8, rs = precision == 64 ? 8 : 4;
    g.general = false;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            g.A[i][j] = lattice[3 * i + j];
            if (!std::isfinite(g.A[i][j])) return fail(c, VDWNL_E_ARG, "cell vectors must be finite");
            if (i != j && g.A[i][j] != 0.0) g.general = true;
        }
    for (int i = 0; i < 3; ++i) {
        g.cell[i] = std::sqrt(g.A[i][0] * g.A[i][0] + g.A[i][1] * g.A[i][1] + g.A[i][2] * g.A[i][2]);
        if (!g.general && !(g.A[i][i] > 0.0)) return fail(c, VDWNL_E_ARG, "cell lengths must be positive and finite");
        if (shape[i] < 4 || !smooth235(shape[i]))
            return fail(c, VDWNL_E_UNSUPPORTED_SIZE, "grid edges must be >= 4 and products of 2, 3 and 5");
        g.s[i] = shape[i];
    }
    // reciprocal vectors: b_c = 2 pi (a_(c+1) x a_(c+2)) / det A
    const double(*A)[3] = g.A;
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (!(std::fabs(det) > 1e-9 * g.cell[0] * g.cell[1] * g.cell[2]))
        return fail(c, VDWNL_E_ARG, "cell vectors must span a volume");
    if (!g.general) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) g.B[i][j] = i == j ? 2.0 * M_PI / g.A[i][i] : 0.0;
    } else {
        for (int cidx = 0; cidx < 3; ++cidx) {
            const double *u = A[(cidx + 1) % 3], *v = A[(cidx + 2) % 3];
            const double x[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
            for (int j = 0; j < 3; ++j) g.B[cidx][j] = 2.0 * M_PI * x[j] / det;
        }
    }
    const size_t N1 = g.s[0], N2 = g.s[1], N3 = g.s[2];
    if ((N1 * N2) % 2 != 0)
        return fail(c, VDWNL_E_UNSUPPORTED_SIZE, "N1 * N2 must be even (rows are transformed in pairs)");
    if (3 * N1 * N2 * N3 >= ((size_t)1 << 31))   // (element offsets of three fields in 32 bits)
        return fail(c, VDWNL_E_UNSUPPORTED_SIZE, "more than 715827882 grid points");
    // LDS of each pass as a function of its tile size (twiddles staged in LDS too)
    auto zmain = [&](size_t k3) { return (N1 + kNQ * k3 * (N1 | 1)) * cs + 16 + (N1 / 2 + 1) * k3 * sizeof(int); };
    auto xmain = [&](size_t b) { return xpass_lds(b, N3, rs); };
    auto ypass = [&](size_t w, size_t c2) { return (N2 + (N2 | 1) * w) * c2; };
    const size_t cap = c->lds_cap;
    if (N1 > (size_t)kMaxN1 || zmain(1) > cap || deriv_lds(N1, 1, 16) > cap)
        return fail(c, VDWNL_E_UNSUPPORTED_SIZE, "N1 too large for the fused axis-1 pass");
    if (N2 > (size_t)kTileCap || ypass(1, cs) > cap || deriv_lds(N2, 1, 16) > cap)
        return fail(c, VDWNL_E_UNSUPPORTED_SIZE, "N2 too large");
    if ((size_t)kNQ / 2 * N3 > (size_t)kTileCap || xmain(1) > cap)
        return fail(c, VDWNL_E_UNSUPPORTED_SIZE, "N3 too large for the axis-3 pass");
    if (!radix_plan((int)N1, g.p1) || !radix_plan((int)N2, g.p2) || !radix_plan((int)N3, g.p3))
        return fail(c, VDWNL_E_UNSUPPORTED_SIZE, "no radix plan");
    return VDWNL_OK;
}

// Tile shapes of grid g from the LDS budget of each pass group: each tile as
// large as the FFT tile cap and its group's budget allow (at least one unit).
static void size_tiles(const vdwnl_ctx *c, Grid &g) {
    const size_t cs = c->precision == 64 ? 16 : 8, rs = c->precision == 64 ? 8 : 4;
    const size_t N1 = g.s[0], N2 = g.s[1], N3 = g.s[2];
    auto zmain = [&](size_t k3) { return (N1 + kNQ * k3 * (N1 | 1)) * cs + 16 + (N1 / 2 + 1) * k3 * sizeof(int); };
    auto xmain = [&](size_t b) { return xpass_lds(b, N3, rs); };
    auto ypass = [&](size_t w, size_t c2) { return (N2 + (N2 | 1) * w) * c2; };
    // complex elements per LDS FFT tile: bounded for the runtime-radix FFT
    // (its per-thread register arrays), not for the compile-time plans
    auto cap = [](size_t n) { return len_class((int)n) == kLenGeneric ? (size_t)kTileCap : (size_t)1 << 30; };
    // axis-3 tiles of the theta / assembly passes: at most one grid point
    // per thread (two measured slower: the local chain needs the VGPRs);
    // of the derivative passes (FP64 lines, one per row pair): about 4096
    // points, enough lines to occupy every lane
    g.bmain = 1;
    while ((size_t)(g.bmain + 1) * N3 <= (size_t)kThreads && (kNQ / 2) * (g.bmain + 1) * N3 <= cap(N3) &&
           xmain(g.bmain + 1) <= c->pref[TG_X])
        ++g.bmain;
    g.bnf = 2;
    while ((size_t)(g.bnf + 2) * N3 <= 4096 && (size_t)(g.bnf / 2 + 1) * N3 <= cap(N3) &&
           drow_lds(N3, g.bnf / 2 + 1, 16) <= kLdsCap)
        g.bnf += 2;
    g.k3main = 1;
    while (g.k3main < kMaxCols && (size_t)kNQ * (g.k3main + 1) * N1 <= cap(N1) && zmain(g.k3main + 1) <= c->pref[TG_Z])
        ++g.k3main;
    g.wy20 = 1;
    while ((size_t)(g.wy20 + 1) * N2 <= cap(N2) && ypass(g.wy20 + 1, cs) <= c->pref[TG_Y20]) ++g.wy20;
    if (g.wy20 > 1) g.wy20 &= ~1;   // even widths: 16-byte aligned FP32 rows
    // derivative tiles along axes 2 and 1: i3 columns in pairs (one FP64
    // line each), within the group's budget
    // (a width short of the whole row: a multiple of 32 once it reaches 32,
    // so that the runs of i3 start and end on 128-byte boundaries)
    auto dwidth = [&](size_t L, size_t budget) {
        int w = 2;
        while ((size_t)(w + 2) <= N3 && (size_t)(w / 2 + 1) * L <= cap(L) && deriv_lds(L, w / 2 + 1, 16) <= budget)
            w += 2;
        w = std::min<int>(w, (int)N3);
        if (w < (int)N3 && w >= 32) w &= ~31;
        return w;
    };
    g.wdy = dwidth(N2, c->pref[TG_YAUX]);
    g.wdz = dwidth(N1, c->pref[TG_ZAUX]);
}

// Tuned LDS budgets, keyed by the device architecture, LDS size, precision,
// gradient mode and the exact list of grid shapes and cells: a map for the
// process, backed by a file so that later processes reuse them.  The file is
// a JSON object with one entry per line,
//   "<arch>/<hash of the rest of the key>": [x, y20, yaux, z, zaux, contraction,
//                                              five radix orders in the same group order],
// at $VDWNL_TUNE_CACHE (empty: no file), else $XDG_CACHE_HOME/vdwnl/tuning.json
// or $HOME/.cache/vdwnl/tuning.json.  A file that cannot be read or written
// is ignored (the process map still works).
static std::mutex g_tuned_mu;
static std::map<std::string, std::vector<size_t>> g_tuned;
constexpr int kTuneVals = 2 * TG_COUNT + 1;   // the five budgets, the contraction unit, five radix orders

static std::string plan_key(const vdwnl_ctx *c) {
    std::string k = std::to_string(c->precision) + "/" + std::to_string(c->grad_mode) + "/" + std::to_string(c->lds_cap);
    char buf[128];
    for (const Grid &g : c->grids) {
        std::snprintf(buf, sizeof(buf), ";%dx%dx%d@", g.s[0], g.s[1], g.s[2]);
        k += buf;
        for (int i = 0; i < 9; ++i) {
            std::snprintf(buf, sizeof(buf), "%.17g,", g.A[i / 3][i % 3]);
            k += buf;
        }
    }
    // FNV-1a of the whole key, behind the readable part
    uint64_t h = 1469598103934665603ull;
    for (unsigned char ch : k) { h ^= ch; h *= 1099511628211ull; }
    std::snprintf(buf, sizeof(buf), "%s/p%d/g%d/l%zu/n%zu/%016llx", c->arch.c_str(), c->precision, c->grad_mode,
                  c->lds_cap, c->grids.size(), (unsigned long long)h);
    return buf;
}

static std::string tune_cache_path() {
    if (const char *p = std::getenv("VDWNL_TUNE_CACHE")) return p;
    if (const char *x = std::getenv("XDG_CACHE_HOME"); x && *x) return std::string(x) + "/vdwnl/tuning.json";
    if (const char *h = std::getenv("HOME"); h && *h) return std::string(h) + "/.cache/vdwnl/tuning.json";
    return "";
}

// Entries of the file: lines  "key": [n, n, n, n, n]  (anything else skipped).
static std::map<std::string, std::vector<size_t>> read_tune_file(const std::string &path) {
    std::map<std::string, std::vector<size_t>> out;
    if (path.empty()) return out;
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return out;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        const char *q0 = std::strchr(line, '"');
        const char *q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
        const char *br = q1 ? std::strchr(q1, '[') : nullptr;
        if (!br) continue;
        std::vector<size_t> v;
        const char *p = br + 1;
        while (v.size() < (size_t)kTuneVals) {
            char *end = nullptr;
            const unsigned long long x = std::strtoull(p, &end, 10);
            if (end == p) break;
            v.push_back((size_t)x);
            p = end;
            while (*p == ',' || *p == ' ') ++p;
        }
        if (v.size() == (size_t)kTuneVals) out[std::string(q0 + 1, q1)] = v;
    }
    std::fclose(f);
    return out;
}

static void write_tune_file(const std::string &path, const std::map<std::string, std::vector<size_t>> &m) {
    if (path.empty()) return;
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos && slash > 0) {
        // (create the directory and its parents; errors show up at fopen)
        std::string dir = path.substr(0, slash);
        for (size_t i = 1; i <= dir.size(); ++i)
            if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
    }
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto &kv : m) {
        std::fprintf(f, "  \"%s\": [", kv.first.c_str());
        for (int g = 0; g < kTuneVals; ++g) std::fprintf(f, g ? ", %zu" : "%zu", kv.second[g]);
        std::fprintf(f, "]%s\n", ++i < m.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    if (ok) (void)std::rename(tmp.c_str(), path.c_str());
    else (void)std::remove(tmp.c_str());
}

static bool tuned_lookup(const std::string &key, size_t *pref, int *contraction, int *variant, size_t cap) {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    auto it = g_tuned.find(key);
    if (it == g_tuned.end()) {
        auto file = read_tune_file(tune_cache_path());
        auto ft = file.find(key);
        if (ft == file.end()) return false;
        for (int i = 0; i < TG_COUNT; ++i)
            if (ft->second[i] < 4096 || ft->second[i] > cap) return false;   // (not a budget this device accepts)
        if (ft->second[TG_COUNT] > 1) return false;
        for (int i = 0; i < TG_COUNT; ++i)
            if (ft->second[TG_COUNT + 1 + i] >= (size_t)kMaxVariants) return false;
        it = g_tuned.insert(*ft).first;
    }
    for (int i = 0; i < TG_COUNT; ++i) pref[i] = it->second[i];
    *contraction = (int)it->second[TG_COUNT];
    for (int i = 0; i < TG_COUNT; ++i) variant[i] = (int)it->second[TG_COUNT + 1 + i];
    return true;
}

static void tuned_store(const std::string &key, const size_t *pref, int contraction, const int *variant) {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    std::vector<size_t> v(pref, pref + TG_COUNT);
    v.push_back((size_t)contraction);
    for (int i = 0; i < TG_COUNT; ++i) v.push_back((size_t)variant[i]);
    g_tuned[key] = v;
    const std::string path = tune_cache_path();
    auto file = read_tune_file(path);
    file[key] = g_tuned[key];
    write_tune_file(path, file);
}

// cells: nb x 9 values (rows a_1, a_2, a_3 of each grid's cell)
static int plan_grids(vdwnl_ctx *c, int nb, const int32_t *shapes, const double *cells, int grad_mode,
                      int precision) {
    if (!c || !shapes || !cells || nb <= 0) return fail(c, VDWNL_E_ARG, "null argument or empty batch");
    if (grad_mode < 0 || grad_mode > kMaxFd)
        return fail(c, VDWNL_E_ARG, "grad_mode must be 0 (spectral) or 1..4 (central differences)");
    if (precision != 32 && precision != 64) return fail(c, VDWNL_E_ARG, "precision must be 32 or 64");
    std::vector<Grid> gs(nb);
    for (int i = 0; i < nb; ++i) {
        int rc = check_grid(c, shapes + 3 * i, cells + 9 * i, precision, gs[i]);
        if (rc != VDWNL_OK) return rc;
    }
    free_device(c);
    c->grids = gs;
    c->precision = precision;
    c->grad_mode = grad_mode;
    // tile budgets: a tuned set for this exact batch if one exists, else defaults
    c->plan_key = plan_key(c);
    if (!tuned_lookup(c->plan_key, c->pref, &c->contraction, c->variant, c->lds_cap)) {
        for (auto &p : c->pref) p = std::min<size_t>(c->lds_cap, kLdsCap);
        c->contraction = kDefaultContraction;
        for (auto &v : c->variant) v = 0;
    }
    for (auto &g : c->grids) size_tiles(c, g);
    c->shells.clear();
    c->shell_keys.clear();
    for (auto &g : c->grids) {
        std::vector<double> key = {(double)g.s[0], (double)g.s[1], (double)g.s[2]};
        for (int i = 0; i < 9; ++i) key.push_back(g.A[i / 3][i % 3]);
        int found = -1;
        for (auto &kv : c->shell_keys)
            if (kv.first == key) found = kv.second;
        if (found < 0) {
            found = (int)c->shells.size();
            double diag[3] = {g.A[0][0], g.A[1][1], g.A[2][2]};
            c->shells.push_back(g.general ? build_shells_general(g.s, g.B) : build_shells(g.s, diag));
            c->shells.back().general = g.general;
            c->shell_keys.push_back({key, found});
        }
        g.shell_key = found;
    }
    // Row layout of each shell table.  Orthorhombic cells: the full matrix
    // (row a contiguous for the lane that forms u_a).  General cells, where
    // every k point has a shell of its own: the full matrix too when two or
    // more grids share the table (a tile's rows, loaded into its XCD's L2,
    // then serve the same tile of the other grids) or when it fits in the
    // Infinity Cache; else the packed upper triangle, half the bytes.
    {
        const size_t rs = precision == 64 ? 8 : 4;
        std::vector<int> users(c->shells.size(), 0);
        for (auto &g : c->grids) ++users[g.shell_key];
        for (size_t i = 0; i < c->shells.size(); ++i) {
            Shells &sh = c->shells[i];
            sh.packed = sh.general && users[i] < 2 && sh.gmod.size() * kTabRow * rs > kFullRowCacheBytes;
        }
    }
    c->have_grid = true;
    const int rc = check_krange(c);
    refresh_image(c);
    return rc;
}

// spline of the radial table at |G| for every pair: phi_ab(|G_s|), FP64,
// stored as the full symmetric matrix of each shell or as its packed upper
// triangle, pair p = (r, q), r <= q, in row order (Shells::packed)
static void shell_table(const vdwnl_ctx *c, const Shells &sh, std::vector<double> &out) {
    const size_t row = sh.packed ? kTabPacked : kTabRow;
    out.assign(sh.gmod.size() * row, 0.0);
    for (size_t s = 0; s < sh.gmod.size(); ++s) {
        const double k = sh.gmod[s];
        int j = (int)std::floor(k / c->dk);
        if (j > c->nk - 2) j = c->nk - 2;
        if (j < 0) j = 0;
        const double t = k / c->dk - j, a = 1.0 - t, b = t;
        const double w = c->dk * c->dk / 6.0;
        int p = 0;
        for (int r = 0; r < kNQ; ++r)
            for (int q = r; q < kNQ; ++q, ++p) {
                const double *f = c->phi.data() + (size_t)p * c->nk;
                const double *m = c->d2.data() + (size_t)p * c->nk;
                const double v = a * f[j] + b * f[j + 1] + ((a * a * a - a) * m[j] + (b * b * b - b) * m[j + 1]) * w;
                if (sh.packed) {
                    out[s * row + p] = v;
                } else {
                    out[s * row + r * kNQ + q] = v;
                    out[s * row + q * kNQ + r] = v;
                }
            }
    }
}

// Every grid's largest |G| must lie on the radial kernel mesh.
static int check_krange(vdwnl_ctx *c) {
    if (!c->have_grid || !c->have_table) return VDWNL_OK;
    for (auto &sh : c->shells)
        if (sh.gmax > (c->nk - 1) * c->dk * (1.0 + 1e-12))
            return fail(c, VDWNL_E_KRANGE, "radial kernel table does not reach max |G| of a grid");
    return VDWNL_OK;
}

// Launch order of the passes of one evaluation (the final reduction follows):
// spectral gradient (eleven passes: one per axis for the gradient and for
// the divergence) or finite differences (seven).
static const int kOrderSpectral[] = {KG_X, KG_Y, KG_Z, KX_THETA, KY_20F, KZ_MAIN, KY_20I, KX_ASSEMBLE,
                                     KD_X, KD_Y, KD_Z};
static const int kOrderFd[] = {KF_GRAD, KX_THETA, KY_20F, KZ_MAIN, KY_20I, KX_ASSEMBLE, KF_DIV};
static const char *kPassName[KIND_COUNT + 1] = {
    "x_deriv", "y_deriv", "z_deriv", "x_theta", "y_20f", "z_main", "y_20i", "x_assemble", "x_div", "y_div",
    "z_div", "fd_grad", "fd_div", "reduce"};

static int pass_order(int grad_mode, const int **order) {
    if (grad_mode == 0) {
        *order = kOrderSpectral;
        return (int)(sizeof(kOrderSpectral) / sizeof(int));
    }
    *order = kOrderFd;
    return (int)(sizeof(kOrderFd) / sizeof(int));
}

// Weights c_s, s = 1..m, of the central first-derivative formula of order 2m
// on a unit grid: c_s = (-1)^(s+1) (m!)^2 / (s (m - s)! (m + s)!).
static void central_weights(int m, double *c) {
    auto fact = [](int k) { double f = 1.0; for (int i = 2; i <= k; ++i) f *= i; return f; };
    for (int s = 1; s <= m; ++s)
        c[s - 1] = ((s % 2) ? 1.0 : -1.0) * fact(m) * fact(m) / (s * fact(m - s) * fact(m + s));
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Launch order for XCD locality: workgroups go round-robin to the 8 XCDs, so
// tile i of a launch runs on XCD i % 8.  Reorder a list of tiles so that each
// XCD receives a contiguous block of it (neighbouring tiles share cache lines
// at their edges and, in the fused pass, kernel rows): position 8 r + x
// holds the r-th tile of block x.
static void xcd_blocks(std::vector<Tile> &t) {
    const size_t n = t.size();
    if (n < 16) return;
    // block sizes differ by at most one, the larger first, so that every
    // full round of 8 positions takes one tile from each block
    const size_t base = n / 8, rem = n % 8;
    std::vector<size_t> start(9, 0);
    for (size_t x = 0; x < 8; ++x) start[x + 1] = start[x] + base + (x < rem ? 1 : 0);
    std::vector<Tile> out;
    out.reserve(n);
    for (size_t r = 0; r <= base; ++r)
        for (size_t x = 0; x < 8; ++x)
            if (start[x] + r < start[x + 1]) out.push_back(t[start[x] + r]);
    t.swap(out);
}

static int build_image(vdwnl_ctx *c, Image &im, bool keep_tables) {
    const bool dp = c->precision == 64;
    const size_t rs = dp ? 8 : 4, cs = 2 * rs;

    // workspace layout
    size_t off = 0;
    c->map_off.assign(c->shells.size(), 0);
    c->tab_off.assign(c->shells.size(), 0);
    for (size_t i = 0; i < c->shells.size(); ++i) {
        c->map_off[i] = off;
        off = align_up(off + c->shells[i].map.size() * sizeof(int));
        c->tab_off[i] = off;
        off = align_up(off + c->shells[i].gmod.size() * (c->shells[i].packed ? kTabPacked : kTabRow) * rs);
    }
    std::vector<Tile> tiles[KIND_COUNT];
    std::vector<int2> zcols;              // columns of the fused axis-1 tiles
    for (size_t gi = 0; gi < c->grids.size(); ++gi) {
        Grid &g = c->grids[gi];
        const int N1 = g.s[0], N2 = g.s[1], N3 = g.s[2], N3h = N3 / 2 + 1;
        const int rows = N1 * N2;
        const int inst = (int)gi;
        size_t first_tile[KIND_COUNT];
        for (int k = 0; k < KIND_COUNT; ++k) first_tile[k] = tiles[k].size();
        // axis-3 tiles (and the stencil passes' runs of lines)
        const bool fd = c->grad_mode > 0;
        for (int r = 0; r < rows; r += g.bnf) {
            const int b = std::min(g.bnf, rows - r);   // even: rows and bnf are
            tiles[fd ? KF_GRAD : KG_X].push_back({inst, r, b, 0, -1});
            tiles[fd ? KF_DIV : KD_X].push_back({inst, r, b, 0, -1});
        }
        int slot = 0;
        for (int r = 0; r < rows; r += g.bmain) {
            const int b = std::min(g.bmain, rows - r);
            tiles[KX_THETA].push_back({inst, r, b, 0, slot++});
            tiles[KX_ASSEMBLE].push_back({inst, r, b, 0, -1});
        }
        g.n_de = slot;
        // axis-2 tiles of the 20 spectra
        for (int i1 = 0; i1 < N1; ++i1)
            for (int f = 0; f < N3h * kNQ; f += g.wy20) {
                tiles[KY_20F].push_back({inst, i1, f, std::min(g.wy20, N3h * kNQ - f), -1});
                tiles[KY_20I].push_back({inst, i1, f, std::min(g.wy20, N3h * kNQ - f), -1});
            }
        // derivative tiles along axes 2 (a = i1) and 1 (a = i2): runs of i3
        if (!fd) {
            for (int i1 = 0; i1 < N1; ++i1)
                for (int i3 = 0; i3 < N3; i3 += g.wdy) {
                    tiles[KG_Y].push_back({inst, i1, i3, std::min(g.wdy, N3 - i3), -1});
                    tiles[KD_Y].push_back({inst, i1, i3, std::min(g.wdy, N3 - i3), -1});
                }
            for (int i2 = 0; i2 < N2; ++i2)
                for (int i3 = 0; i3 < N3; i3 += g.wdz) {
                    tiles[KG_Z].push_back({inst, i2, i3, std::min(g.wdz, N3 - i3), -1});
                    tiles[KD_Z].push_back({inst, i2, i3, std::min(g.wdz, N3 - i3), -1});
                }
        }
        // Fused axis-1 tiles: the columns k2 and N2 - k2 (the same |m2|, so
        // the same |G| shell at every (|m1|, k3)) over a run of consecutive
        // k3; one kernel row (loaded per lane) then serves four k points.  Columns
        // k2 = 0 and N2/2 stand alone.
        {
            const int K = std::min(g.k3main, kMaxCols);
            std::vector<Tile> zt;
            // (a budget of one column per tile: k2 and N2 - k2 in tiles of their own)
            // (general cells: every column alone, k2 over the whole axis)
            for (int k2 = 0; k2 <= (g.general ? N2 - 1 : N2 / 2); ++k2) {
                const int k2b = g.general ? k2 : (N2 - k2) % N2;
                const bool pair = k2b != k2 && K >= 2;
                for (int side = 0; side < ((k2b != k2 && !pair) ? 2 : 1); ++side) {
                    const int ka = side == 0 ? k2 : k2b;
                    const int cp = pair ? 2 : 1;                  // columns per pair
                    const int P = std::max(1, K / cp);            // pairs per tile (P cp <= K)
                    for (int k3 = 0; k3 < N3h; k3 += P) {
                        const int np = std::min(P, N3h - k3);
                        zt.push_back({inst, (int)zcols.size(), np, cp, -1});
                        for (int i = 0; i < np; ++i) {
                            zcols.push_back({ka, k3 + i});
                            if (pair) zcols.push_back({k2b, k3 + i});
                        }
                    }
                }
            }
            slot = 0;
            for (Tile &tl : zt) {
                tl.slot = slot++;
                tiles[KZ_MAIN].push_back(tl);
            }
        }
        g.n_ek = slot;
        // XCD-contiguous order for this grid's tiles of the other passes
        for (int k = 0; k < KIND_COUNT; ++k) {
            if (k == KZ_MAIN) continue;
            std::vector<Tile> mine(tiles[k].begin() + first_tile[k], tiles[k].end());
            xcd_blocks(mine);
            std::copy(mine.begin(), mine.end(), tiles[k].begin() + first_tile[k]);
        }
        // fields
        g.off_grad = off; off = align_up(off + 3 * g.npts() * rs);
        g.off_vloc = off; off = align_up(off + g.npts() * rs);
        g.off_spec = off; off = align_up(off + g.nhalf() * kNQ * cs);
        g.off_ek = off; off = align_up(off + g.n_ek * sizeof(double));
        g.off_de = off; off = align_up(off + g.n_de * sizeof(double));
        g.off_sl = off; off = align_up(off + 2 * g.n_de * sizeof(double));
        g.off_bad = off; off = align_up(off + sizeof(int));
    }
    // LDS of one tile of each pass for grid g
    auto lds_of = [&](int k, const Grid &g) -> size_t {
        const size_t N1 = g.s[0], N2 = g.s[1], N3 = g.s[2];
        switch (k) {
            // the gradient's derivatives in FP64, the divergence's in the working precision
            case KG_X: return drow_lds(N3, g.bnf / 2, 16);
            case KD_X: return drow_lds(N3, g.bnf / 2, cs);
            case KG_Y: return deriv_lds(N2, (g.wdy + 1) / 2, 16);
            case KD_Y: return deriv_lds(N2, (g.wdy + 1) / 2, cs);
            case KG_Z: return deriv_lds(N1, (g.wdz + 1) / 2, 16);
            case KD_Z: return deriv_lds(N1, (g.wdz + 1) / 2, cs);
            case KF_GRAD: case KF_DIV: return 0;
            case KX_THETA: case KX_ASSEMBLE: return xpass_lds(g.bmain, N3, rs);
            case KY_20F: case KY_20I: return (N2 + (N2 | 1) * g.wy20) * cs;
            default: {   // KZ_MAIN
                const size_t K = std::min(g.k3main, kMaxCols);
                return (N1 + (size_t)kNQ * K * (N1 | 1)) * cs + 16 + (g.general ? N1 : N1 / 2 + 1) * K * sizeof(int);
            }
        }
    };
    // the axis whose FFT a pass performs: 3 for the axis-3 passes, 2, 1
    auto axis_len = [&](int k, const Grid &g) -> int {
        switch (k) {
            case KG_X: case KD_X: case KX_THETA: case KX_ASSEMBLE: return g.s[2];
            case KG_Y: case KD_Y: case KY_20F: case KY_20I: return g.s[1];
            default: return g.s[0];
        }
    };
    // groups: grids with the same length classes on all three axes (every
    // pass of a group is then one launch).  (Dealing a group with a large
    // share of the points into sub-groups measured no faster.)
    std::vector<int> group_of(c->grids.size());
    {
        std::vector<int> keys;
        for (size_t gi = 0; gi < c->grids.size(); ++gi) {
            const Grid &g = c->grids[gi];
            // (and the cell kind and kernel-row layout: general cells take the
            // fused pass's general variant, full or packed rows)
            const int key = ((len_class(g.s[0]) * kNumLenClasses + len_class(g.s[1])) * kNumLenClasses +
                             len_class(g.s[2])) * 4 + (g.general ? 1 : 0) + (c->shells[g.shell_key].packed ? 2 : 0);
            auto it = std::find(keys.begin(), keys.end(), key);
            group_of[gi] = (int)(it - keys.begin());
            if (it == keys.end()) keys.push_back(key);
        }
        c->ngroups = (int)keys.size();
    }
    // The fused axis-1 pass: grids that share a kernel-row table (the same
    // shape and cell, so the same tiles) take turns, tile j of each such grid
    // one after another, and the XCD blocks are cut from that order: the rows
    // one tile loads into its XCD's L2 serve the same tile of the other grids.
    {
        std::vector<std::vector<Tile>> per(c->grids.size());
        for (const Tile &tl : tiles[KZ_MAIN]) per[tl.inst].push_back(tl);
        std::vector<Tile> out;
        for (int grp = 0; grp < c->ngroups; ++grp) {
            std::vector<Tile> mine;
            std::vector<bool> done(c->grids.size(), false);
            for (size_t gi = 0; gi < c->grids.size(); ++gi) {
                if (group_of[gi] != grp || done[gi]) continue;
                std::vector<size_t> share;
                for (size_t gj = gi; gj < c->grids.size(); ++gj)
                    if (group_of[gj] == grp && !done[gj] && c->grids[gj].shell_key == c->grids[gi].shell_key &&
                        per[gj].size() == per[gi].size()) {
                        share.push_back(gj);
                        done[gj] = true;
                    }
                for (size_t j = 0; j < per[gi].size(); ++j)
                    for (size_t gj : share) mine.push_back(per[gj][j]);
            }
            xcd_blocks(mine);
            out.insert(out.end(), mine.begin(), mine.end());
        }
        tiles[KZ_MAIN].swap(out);
    }
    std::vector<Tile> all;
    for (int k = 0; k < KIND_COUNT; ++k) {
        c->launches[k].clear();
        for (int grp = 0; grp < c->ngroups; ++grp) {
            vdwnl_ctx::Launch L{k, 0, (int)all.size(), 0, 0, grp, 0, 0, 0, 0};
            for (const Tile &tl : tiles[k]) {
                if (group_of[tl.inst] != grp) continue;
                const Grid &g = c->grids[tl.inst];
                L.general = g.general ? 1 : 0;
                L.packed = c->shells[g.shell_key].packed ? 1 : 0;
                L.mfma = (k == KZ_MAIN && c->precision == 32 && !g.general && c->contraction == VDWNL_CONTRACTION_MATRIX)
                             ? 1 : 0;
                // the stencil passes transform nothing (class 0 for any grid)
                L.lc = (k == KF_GRAD || k == KF_DIV) ? 0 : len_class(axis_len(k, g));
                L.var = (k == KF_GRAD || k == KF_DIV) ? 0 : std::min(c->variant[variant_group(k)], kNumVariants[L.lc] - 1);
                all.push_back(tl);
                L.lds = std::max(L.lds, lds_of(k, g));
            }
            L.cnt = (int)all.size() - L.off;
            if (L.cnt > 0) c->launches[k].push_back(L);
        }
    }
    // twiddles
    c->tw_off.clear();
    std::vector<double> twd;
    for (auto &g : c->grids)
        for (FftPlan *p : {&g.p1, &g.p2, &g.p3}) {
            auto it = c->tw_off.find(p->n);
            if (it == c->tw_off.end()) {
                const int o = (int)(twd.size() / 2);
                c->tw_off[p->n] = o;
                for (int m = 0; m < p->n; ++m) {
                    // exp(-2 pi i m / n)
                    const double ang = 2.0 * M_PI * (double)m / (double)p->n;
                    twd.push_back(std::cos(ang));
                    twd.push_back(-std::sin(ang));
                }
                p->tw = o;
            } else {
                p->tw = it->second;
            }
        }
    // the rest of the buffer
    im.ws = off;
    im.tiles.swap(all);
    im.cols.swap(zcols);
    im.twd.swap(twd);
    im.tw32.assign(im.twd.begin(), im.twd.end());
    const size_t ng = c->grids.size();
    im.off_tiles = align_up(off);
    im.off_cols = align_up(im.off_tiles + std::max<size_t>(im.tiles.size(), 1) * sizeof(Tile));
    im.off_tw = align_up(im.off_cols + std::max<size_t>(im.cols.size(), 1) * sizeof(int2));
    im.off_twd = align_up(im.off_tw + std::max<size_t>(im.twd.size() / 2 * cs, 16));
    im.off_consts = align_up(im.off_twd + std::max<size_t>(im.twd.size() / 2 * 16, 16));
    im.off_inst = align_up(im.off_consts + sizeof(Consts));
    im.off_E = align_up(im.off_inst + ng * sizeof(InstDev));
    im.total = align_up(im.off_E + ng * 4 * sizeof(double));   // four energies per grid: E_k, Delta E, E_x, E_c^LDA
    im.tabs.clear();
    if (keep_tables)
        for (const Shells &sh : c->shells) {
            std::vector<double> tab;
            shell_table(c, sh, tab);
            std::vector<char> bytes(tab.size() * rs);
            if (dp) {
                std::memcpy(bytes.data(), tab.data(), bytes.size());
            } else {
                std::vector<float> tf(tab.begin(), tab.end());
                std::memcpy(bytes.data(), tf.data(), bytes.size());
            }
            im.tabs.push_back(std::move(bytes));
        }
    return VDWNL_OK;
}

// Kernels whose tiles take more than 64 KB of LDS opt in to it (at planning:
// launches may be captured into a graph).
static int lds_optin(vdwnl_ctx *c) {
    hipError_t e;
    for (int k = 0; k < KIND_COUNT; ++k)
        for (const auto &L : c->launches[k]) {
            LaunchArgs a{nullptr, nullptr, 0, L.lds, nullptr, nullptr, nullptr, nullptr, nullptr, L.general, L.mfma, L.var, L.packed};
            if ((e = launch_kind(k, L.lc, c->precision, a)) != hipSuccess) return hipfail(c, e, "kernel LDS limit");
            // (and the stage probes that stand in for the pass)
            for (int pr : {PROBE_THETA_K, PROBE_U_K, PROBE_U}) {
                const int pk = pr == PROBE_U ? KX_ASSEMBLE : KZ_MAIN;
                if (k == pk && (e = launch_probe(pr, L.lc, c->precision, a, nullptr, 0)) != hipSuccess)
                    return hipfail(c, e, "kernel LDS limit");
            }
        }
    return VDWNL_OK;
}

// Device pointers of an image placed at base.
static DevPtrs place(const Image &im, char *base) {
    DevPtrs P;
    P.base = base;
    P.tiles = (Tile *)(base + im.off_tiles);
    P.cols = (int2 *)(base + im.off_cols);
    P.tw = base + im.off_tw;
    P.twd = base + im.off_twd;
    P.consts = (Consts *)(base + im.off_consts);
    P.inst = (InstDev *)(base + im.off_inst);
    P.E = (double *)(base + im.off_E);
    return P;
}

// Copy an image's tables to the buffer at P.base (stream-ordered on st;
// pageable host sources).  Kernel rows not kept in the image are computed
// here, one shells entry at a time, and copied synchronously.
static int upload_image(vdwnl_ctx *c, const Image &im, const DevPtrs &P, hipStream_t st) {
    hipError_t e;
    const bool dp = c->precision == 64;
    const size_t rs = dp ? 8 : 4, cs = 2 * rs;
    char *w = P.base;
    for (size_t i = 0; i < c->shells.size(); ++i) {
        const Shells &sh = c->shells[i];
        if ((e = hipMemcpyAsync(w + c->map_off[i], sh.map.data(), sh.map.size() * sizeof(int), hipMemcpyHostToDevice,
                                st)) != hipSuccess)
            return hipfail(c, e, "upload shell map");
        if (i < im.tabs.size()) {
            e = hipMemcpyAsync(w + c->tab_off[i], im.tabs[i].data(), im.tabs[i].size(), hipMemcpyHostToDevice, st);
        } else {
            std::vector<double> tab;
            shell_table(c, sh, tab);
            if (dp) {
                e = hipMemcpy(w + c->tab_off[i], tab.data(), tab.size() * 8, hipMemcpyHostToDevice);
            } else {
                std::vector<float> tf(tab.begin(), tab.end());
                e = hipMemcpy(w + c->tab_off[i], tf.data(), tf.size() * 4, hipMemcpyHostToDevice);
            }
        }
        if (e != hipSuccess) return hipfail(c, e, "upload shell table");
    }
    const size_t twn = im.twd.size() / 2;
    if (dp) {
        e = hipMemcpyAsync(P.tw, im.twd.data(), twn * cs, hipMemcpyHostToDevice, st);
    } else {
        e = hipMemcpyAsync(P.tw, im.tw32.data(), twn * cs, hipMemcpyHostToDevice, st);
    }
    if (e != hipSuccess) return hipfail(c, e, "upload twiddles");
    if ((e = hipMemcpyAsync(P.twd, im.twd.data(), twn * 16, hipMemcpyHostToDevice, st)) != hipSuccess)
        return hipfail(c, e, "upload twiddles");
    if (!im.tiles.empty() &&
        (e = hipMemcpyAsync(P.tiles, im.tiles.data(), im.tiles.size() * sizeof(Tile), hipMemcpyHostToDevice, st)) !=
            hipSuccess)
        return hipfail(c, e, "upload tiles");
    if (!im.cols.empty() &&
        (e = hipMemcpyAsync(P.cols, im.cols.data(), im.cols.size() * sizeof(int2), hipMemcpyHostToDevice, st)) !=
            hipSuccess)
        return hipfail(c, e, "upload columns");
    if ((e = hipMemcpyAsync(P.consts, &c->consts, sizeof(Consts), hipMemcpyHostToDevice, st)) != hipSuccess)
        return hipfail(c, e, "upload consts");
    return VDWNL_OK;
}

// The per-grid entries of the instance table for a buffer at base (the
// density and potential pointers and the functional switch are kept).
static void fill_insts(vdwnl_ctx *c, char *w, InstDev *out) {
    const size_t ng = c->grids.size();
    for (size_t gi = 0; gi < ng; ++gi) {
        const Grid &g = c->grids[gi];
        InstDev &I = out[gi];
        const void *n_keep = I.n;
        void *v_keep = I.v;
        const int sl_keep = I.semilocal;
        std::memset(&I, 0, sizeof(I));
        I.n = n_keep;
        I.v = v_keep;
        I.semilocal = sl_keep;
        I.n1 = g.s[0]; I.n2 = g.s[1]; I.n3 = g.s[2]; I.n3h = g.s[2] / 2 + 1;
        I.h1 = g.s[0] / 2 + 1; I.h2 = g.s[1] / 2 + 1;
        I.p1 = g.p1; I.p2 = g.p2; I.p3 = g.p3;
        I.inv_n = 1.0 / (double)g.npts();
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) I.B[i][j] = g.B[i][j];
        I.general = g.general ? 1 : 0;
        {
            const double(*A)[3] = g.A;
            I.omega = g.general ? std::fabs(A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                                            A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                                            A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]))
                                : A[0][0] * A[1][1] * A[2][2];
        }
        I.dvol = I.omega / (double)g.npts();
        I.fdm = c->grad_mode;
        if (c->grad_mode > 0) central_weights(c->grad_mode, I.fdc);
        // W[c][x] = N_c b_c,x / (2 pi) (orthorhombic: N_c / L_c on the diagonal):
        // grad n = sum_c W[c] d_c n, the chain rule from grid index to Cartesian
        for (int cc = 0; cc < 3; ++cc)
            for (int x = 0; x < 3; ++x)
                I.fdW[cc][x] = g.general ? (double)g.s[cc] * g.B[cc][x] / (2.0 * M_PI)
                                         : (cc == x ? (double)g.s[cc] / g.A[cc][cc] : 0.0);
        I.grad = w + g.off_grad; I.vloc = w + g.off_vloc; I.spec = w + g.off_spec;
        I.shellmap = (const int *)(w + c->map_off[g.shell_key]);
        I.shelltab = w + c->tab_off[g.shell_key];
        I.part_ek = (double *)(w + g.off_ek); I.part_de = (double *)(w + g.off_de);
        I.part_sl = (double *)(w + g.off_sl);
        I.bad = (int *)(w + g.off_bad);
        I.n_ek = g.n_ek; I.n_de = g.n_de;
    }
}

// Build every device structure for the current grids and table in the
// context's own allocation.
static int prepare_device(vdwnl_ctx *c) {
    if (c->device_ready) return VDWNL_OK;
    if (!c->have_grid || !c->have_table) return fail(c, VDWNL_E_STATE, "grid and kernel table must both be set");
    int krc = check_krange(c);
    if (krc != VDWNL_OK) return krc;
    if (c->device < 0) return fail(c, VDWNL_E_STATE, "host-only context");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hipfail(c, e, "hipSetDevice");
    free_device(c);
    Image tmp;
    const Image *im = &c->img;
    if (!c->img_valid) {
        int rc = build_image(c, tmp, false);
        if (rc != VDWNL_OK) return rc;
        im = &tmp;
    }
    int rc = lds_optin(c);
    if (rc != VDWNL_OK) return rc;
    const size_t ng = c->grids.size();
    c->work_bytes = im->total;
    // (blocks rounded up, 4 MiB or 64 MiB above 512 MiB, so that plans that
    // differ a little, such as tuning candidates, fit the same block)
    const size_t gran = im->total > ((size_t)512 << 20) ? ((size_t)64 << 20) : ((size_t)4 << 20);
    const size_t need = (std::max<size_t>(im->total, 256) + gran - 1) / gran * gran;
    if (c->work && c->work_cap < need) {
        pool_put(c->device, c->work, c->work_cap);
        c->work = nullptr;
        c->work_cap = 0;
    }
    if (!c->work) {
        size_t got = 0;
        if ((c->work = pool_take(c->device, need, &got)) != nullptr) {
            c->work_cap = got;
        } else {
            if ((e = hipMalloc(&c->work, need)) != hipSuccess) {
                (void)hipGetLastError();
                pool_release(c->device);
                if ((e = hipMalloc(&c->work, need)) != hipSuccess) {
                    c->work = nullptr;
                    return hipfail(c, e, "hipMalloc workspace");
                }
            }
            c->work_cap = need;
        }
    }
    if ((e = hipHostMalloc((void **)&c->h_inst, ng * sizeof(InstDev), hipHostMallocDefault)) != hipSuccess) {
        c->h_inst = nullptr;
        return hipfail(c, e, "hipHostMalloc insts");
    }
    if ((e = hipHostMalloc((void **)&c->h_E, ng * 4 * sizeof(double), hipHostMallocDefault)) != hipSuccess) {
        c->h_E = nullptr;
        return hipfail(c, e, "hipHostMalloc E");
    }
    c->dp = place(*im, (char *)c->work);
    if ((rc = upload_image(c, *im, c->dp, 0)) != VDWNL_OK) return rc;
    if ((e = hipStreamSynchronize(0)) != hipSuccess) return hipfail(c, e, "upload");
    std::memset(c->h_inst, 0, ng * sizeof(InstDev));
    fill_insts(c, (char *)c->work, c->h_inst);
    c->device_ready = true;
    return VDWNL_OK;
}

// Enqueue one evaluation on st: the instance table (device pointers of this
// call's n and v), the passes of the gradient mode, the reduction and the copy of the
// energies to pinned host memory.  With timing on, events bracket each pass.
// With chains (graph capture of a batch of several groups) each group's
// passes go to a stream of its own, forked from st and joined back before
// the reduction: the groups' chains are independent, so a pass of one group
// can run beside a pass of another.  Otherwise the passes go in order on st.
static int enqueue(vdwnl_ctx *c, const DevPtrs &P, const InstDev *hinst, double *hE, int nb, hipStream_t st,
                   bool chains = false) {
    hipError_t e;
    if ((e = hipMemcpyAsync(P.inst, hinst, nb * sizeof(InstDev), hipMemcpyHostToDevice, st)) != hipSuccess)
        return hipfail(c, e, "upload instance table");
    if (c->timing) (void)hipEventRecord(c->ev[0], st);
    const int *order;
    const int npass = pass_order(c->grad_mode, &order);
    auto launch = [&](const vdwnl_ctx::Launch &L, hipStream_t s) -> int {
        LaunchArgs a{P.inst, P.tiles + L.off, L.cnt, L.lds, P.consts, P.tw, P.twd, s, P.cols, L.general, L.mfma, L.var, L.packed};
        const hipError_t le = launch_kind(L.kind, L.lc, c->precision, a);
        return le == hipSuccess ? VDWNL_OK : hipfail(c, le, "kernel launch");
    };
    if (chains) {
        if ((e = hipEventRecord(c->chain_events[0], st)) != hipSuccess) return hipfail(c, e, "fork event");
        for (int grp = 0; grp < c->ngroups; ++grp) {
            hipStream_t cs = c->chain_streams[grp];
            if ((e = hipStreamWaitEvent(cs, c->chain_events[0], 0)) != hipSuccess) return hipfail(c, e, "fork wait");
            for (int i = 0; i < npass; ++i)
                for (const auto &L : c->launches[order[i]])
                    if (L.group == grp) {
                        const int rc = launch(L, cs);
                        if (rc != VDWNL_OK) return rc;
                    }
            if ((e = hipEventRecord(c->chain_events[1 + grp], cs)) != hipSuccess) return hipfail(c, e, "join event");
            if ((e = hipStreamWaitEvent(st, c->chain_events[1 + grp], 0)) != hipSuccess) return hipfail(c, e, "join wait");
        }
    } else {
        for (int i = 0; i < npass; ++i) {
            for (const auto &L : c->launches[order[i]]) {
                const int rc = launch(L, st);
                if (rc != VDWNL_OK) return rc;
            }
            if (c->timing) (void)hipEventRecord(c->ev[i + 1], st);
        }
    }
    if ((e = launch_reduce(P.inst, nb, P.E, st)) != hipSuccess) return hipfail(c, e, "reduce launch");
    if (c->timing) (void)hipEventRecord(c->ev[npass + 1], st);
    if ((e = hipMemcpyAsync(hE, P.E, nb * 4 * sizeof(double), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return hipfail(c, e, "copy energies");
    return VDWNL_OK;
}

// Capture enqueue() once into a graph (on a private stream: the caller's may
// be the null stream, which cannot be captured).  The graph reads the pinned
// instance table when it runs, so one graph serves every call.
static int capture(vdwnl_ctx *c, int nb) {
    hipError_t e;
    if (!c->cap_stream && (e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess) {
        c->cap_stream = nullptr;
        return hipfail(c, e, "hipStreamCreate");
    }
    // streams and events of the groups' chains (created once; default priority)
    const bool chains = c->ngroups > 1;
    while (chains && (int)c->chain_streams.size() < c->ngroups) {
        hipStream_t s = nullptr;
        if ((e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) != hipSuccess) return hipfail(c, e, "hipStreamCreate");
        c->chain_streams.push_back(s);
    }
    while (chains && (int)c->chain_events.size() < c->ngroups + 1) {
        hipEvent_t ev = nullptr;
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return hipfail(c, e, "hipEventCreate");
        c->chain_events.push_back(ev);
    }
    if ((e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess)
        return hipfail(c, e, "hipStreamBeginCapture");
    const int rc = enqueue(c, c->dp, c->h_inst, c->h_E, nb, c->cap_stream, chains);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->cap_stream, &g);
    if (rc != VDWNL_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hipfail(c, e, "hipStreamEndCapture");
    c->graph = g;
    if ((e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0)) != hipSuccess) {
        c->gexec = nullptr;
        drop_graph(c);
        return hipfail(c, e, "hipGraphInstantiate");
    }
    return VDWNL_OK;
}

// One evaluation of the planned batch on `stream`.  Synchronous (E_dev null):
// returns after the stream has finished, energies in E_out (host).
// Asynchronous (E_dev set): returns once the work is enqueued; (E_k, Delta E)
// of each grid land in E_dev (device) on the stream.
static int run(vdwnl_ctx *c, int nb, const void *const *n_ptrs, void *const *v_ptrs, double *E_out, void *stream,
               double *E_dev = nullptr) {
    if (!c) return VDWNL_E_ARG;
    if (!n_ptrs || !v_ptrs || (!E_out && !E_dev)) return fail(c, VDWNL_E_ARG, "null pointer");
    if (E_dev && c->timing) return fail(c, VDWNL_E_STATE, "per-pass timing needs the synchronous calls");
    if (!c->have_grid || !c->have_table) return fail(c, VDWNL_E_STATE, "grid and kernel table must both be set");
    if (nb != (int)c->grids.size()) return fail(c, VDWNL_E_ARG, "batch size differs from the planned grids");
    for (int i = 0; i < nb; ++i)
        if (!n_ptrs[i] || !v_ptrs[i]) return fail(c, VDWNL_E_ARG, "null density or potential pointer");
    if (c->device < 0) return fail(c, VDWNL_E_STATE, "host-only context");
    int rc = prepare_device(c);
    if (rc != VDWNL_OK) return rc;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hipfail(c, e, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    // the pinned table is free to update once the previous evaluation is done
    if ((rc = wait_pending(c)) != VDWNL_OK) return rc;
    for (int i = 0; i < nb; ++i) {
        c->h_inst[i].n = n_ptrs[i];
        c->h_inst[i].v = v_ptrs[i];
        c->h_inst[i].semilocal = c->functional == VDWNL_FUNCTIONAL_VDW_DF;
    }
    c->last_functional = -1;
    if (c->timing && !c->ev_made) {
        for (auto &ev : c->ev)
            if ((e = hipEventCreate(&ev)) != hipSuccess) return hipfail(c, e, "hipEventCreate");
        c->ev_made = true;
    }
    if (c->use_graph && !c->timing) {
        if (!c->gexec && (rc = capture(c, nb)) != VDWNL_OK) return rc;
        if ((e = hipGraphLaunch(c->gexec, st)) != hipSuccess) return hipfail(c, e, "hipGraphLaunch");
    } else {
        // per-pass timing: eager launches bracketed by events
        if ((rc = enqueue(c, c->dp, c->h_inst, c->h_E, nb, st)) != VDWNL_OK) return rc;
    }
    c->evaluated = true;
    if (E_dev) {
        // (E_k, Delta E) of each grid: the first two of its four energies
        if ((e = hipMemcpy2DAsync(E_dev, 2 * sizeof(double), c->dp.E, 4 * sizeof(double), 2 * sizeof(double), nb,
                                  hipMemcpyDeviceToDevice, st)) != hipSuccess)
            return hipfail(c, e, "copy energies to the device buffer");
        if (!c->done_ev && (e = hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming)) != hipSuccess)
            return hipfail(c, e, "hipEventCreate");
        if ((e = hipEventRecord(c->done_ev, st)) != hipSuccess) return hipfail(c, e, "hipEventRecord");
        c->pending = true;
        c->pending_functional = c->functional;
        return VDWNL_OK;
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hipfail(c, e, "stream synchronize");
    for (int i = 0; i < nb; ++i) {
        E_out[2 * i] = c->h_E[4 * i];
        E_out[2 * i + 1] = c->h_E[4 * i + 1];
    }
    c->last_functional = c->functional;
    if (c->timing) {
        const int *order;
        const int npass = pass_order(c->grad_mode, &order);
        for (int i = 0; i <= npass; ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]) == hipSuccess)
                c->pass_ms[i < npass ? order[i] : KIND_COUNT] += ms;
        }
        c->timed_calls++;
    }
    return check_density_flags(c, c->h_E, nb);
}

// Parity probe of one stage of grid `target`: the passes of the last
// evaluation (its instance table: the same density buffers) up to the stage,
// launched one by one on st, then the probe in place of the pass that holds
// the stage (theta: the theta pass; the spectra c and u = phi c: the fused
// axis-1 pass; u(r): the assembly pass).  Nothing after the probe runs: the
// caller's potential buffers are not written.
static int probe_stage(vdwnl_ctx *c, int stage, int target, void *dst, hipStream_t st) {
    hipError_t e;
    const int nb = (int)c->grids.size();
    if ((e = hipMemcpyAsync(c->dp.inst, c->h_inst, nb * sizeof(InstDev), hipMemcpyHostToDevice, st)) != hipSuccess)
        return hipfail(c, e, "upload instance table");
    const int *order;
    const int npass = pass_order(c->grad_mode, &order);
    int stop;
    switch (stage) {
        case VDWNL_STAGE_GRAD: case VDWNL_STAGE_THETA: stop = KX_THETA; break;
        case VDWNL_STAGE_THETA_K: case VDWNL_STAGE_U_K: stop = KZ_MAIN; break;
        default: stop = KX_ASSEMBLE; break;
    }
    auto args = [&](const vdwnl_ctx::Launch &L) {
        return LaunchArgs{c->dp.inst, c->dp.tiles + L.off, L.cnt, L.lds, c->dp.consts, c->dp.tw, c->dp.twd, st, c->dp.cols,
                          L.general, L.mfma, L.var, L.packed};
    };
    for (int i = 0; i < npass && order[i] != stop; ++i)
        for (const auto &L : c->launches[order[i]])
            if ((e = launch_kind(L.kind, L.lc, c->precision, args(L))) != hipSuccess) return hipfail(c, e, "kernel launch");
    if (stage == VDWNL_STAGE_GRAD) {
        // grad n as the theta pass takes it: the gradient passes' result
        const Grid &g = c->grids[target];
        const size_t rs = c->precision == 64 ? 8 : 4;
        if ((e = hipMemcpyAsync(dst, (char *)c->work + g.off_grad, 3 * g.npts() * rs, hipMemcpyDeviceToDevice, st)) !=
            hipSuccess)
            return hipfail(c, e, "probe copy");
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return hipfail(c, e, "stream synchronize");
        return VDWNL_OK;
    }
    const int probe = stage == VDWNL_STAGE_THETA ? PROBE_THETA
                      : stage == VDWNL_STAGE_THETA_K ? PROBE_THETA_K
                      : stage == VDWNL_STAGE_U_K ? PROBE_U_K : PROBE_U;
    for (const auto &L : c->launches[stop])
        if ((e = launch_probe(probe, L.lc, c->precision, args(L), dst, target)) != hipSuccess)
            return hipfail(c, e, "probe launch");
    if (stage == VDWNL_STAGE_THETA_K || stage == VDWNL_STAGE_U_K) {
        const Grid &g = c->grids[target];
        const size_t cs = c->precision == 64 ? 16 : 8;
        if ((e = hipMemcpyAsync(dst, (char *)c->work + g.off_spec, g.nhalf() * kNQ * cs, hipMemcpyDeviceToDevice, st)) !=
            hipSuccess)
            return hipfail(c, e, "probe copy");
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hipfail(c, e, "stream synchronize");
    return VDWNL_OK;
}

// ---------------------------------------------------------------- evaluation without allocation

// The device buffer of vdwnl_energy_potential_noalloc: one per GPU the
// library runs on (each device holds its own copy of this array, at its own
// address, from the library's first use of the device until the process
// ends).  Host code never uses the array's name as an address: the pointer
// comes from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
struct ScratchSlot {
    char *ptr = nullptr;       // the device's address of scratch
    uint64_t owner = 0;        // plan stamp of the image it holds (0: none)
    uint64_t optin = 0;        // plan stamp whose kernels have their LDS limits raised
};
static std::mutex g_scratch_mu;
static ScratchSlot g_scratch[kMaxDevices];
static std::mutex g_stamp_mu;
static uint64_t g_stamp = 0;

// Set-up: the address of scratch on `device` (made current for the call;
// the caller's current device is restored).
static hipError_t scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device].ptr) return hipSuccess;
    int prev = -1;
    (void)hipGetDevice(&prev);
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess) g_scratch[device].ptr = (char *)p;
    }
    if (prev >= 0) (void)hipSetDevice(prev);
    return e;
}

// The plan's host image for the entry point without allocation, rebuilt by
// every set-up call that changes the plan, the table or the tiles; kept
// (with its kernel rows) only when the whole image fits the scratch buffer.
static void refresh_image(vdwnl_ctx *c) {
    c->img = Image();
    c->img_valid = false;
    c->img_need = 0;
    {
        std::lock_guard<std::mutex> lk(g_stamp_mu);
        c->plan_stamp = ++g_stamp;
    }
    if (!c->have_grid || !c->have_table) return;
    for (auto &sh : c->shells)
        if (sh.gmax > (c->nk - 1) * c->dk * (1.0 + 1e-12)) return;
    Image probe;
    if (build_image(c, probe, false) != VDWNL_OK) return;
    // a lone grid in a general cell whose full kernel matrices keep the
    // image beyond the scratch array: its table packed (half the row
    // bytes) when that fits, for both entry points
    if (probe.total > kScratchBytes && c->grids.size() == 1) {
        Shells &sh = c->shells[c->grids[0].shell_key];
        if (sh.general && !sh.packed) {
            sh.packed = true;
            Image packed;
            if (build_image(c, packed, false) == VDWNL_OK && packed.total <= kScratchBytes) {
                probe = packed;
            } else {
                sh.packed = false;
                if (build_image(c, probe, false) != VDWNL_OK) return;
            }
        }
    }
    c->img_need = probe.total;
    if (probe.total > kScratchBytes) return;
    if (build_image(c, c->img, true) != VDWNL_OK) return;
    c->na_inst.assign(c->grids.size(), InstDev());
    c->na_E.assign(4 * c->grids.size(), 0.0);
    c->img_valid = true;
}

// One evaluation of a single planned grid with every device structure in
// this device's scratch: the image is copied in when the scratch holds
// another one, then the instance table, the passes launched one by one, the
// reduction and the energies, all on st; returns after st has finished.
static int run_noalloc(vdwnl_ctx *c, const void *n_dev, void *v_dev, double *E_out, hipStream_t st) {
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hipfail(c, e, "hipSetDevice");
    if ((e = scratch_setup(c->device)) != hipSuccess) return hipfail(c, e, "hipGetSymbolAddress(scratch)");
    ScratchSlot &slot = g_scratch[c->device];
    const DevPtrs P = place(c->img, slot.ptr);
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (slot.optin != c->plan_stamp) {
            const int rc = lds_optin(c);
            if (rc != VDWNL_OK) return rc;
            slot.optin = c->plan_stamp;
        }
        if (slot.owner != c->plan_stamp) {
            slot.owner = 0;
            const int rc = upload_image(c, c->img, P, st);
            if (rc != VDWNL_OK) return rc;
            slot.owner = c->plan_stamp;
        }
    }
    InstDev *hi = c->na_inst.data();
    fill_insts(c, slot.ptr, hi);
    hi[0].n = n_dev;
    hi[0].v = v_dev;
    hi[0].semilocal = c->functional == VDWNL_FUNCTIONAL_VDW_DF;
    const int rc = enqueue(c, P, hi, c->na_E.data(), 1, st);
    if (rc != VDWNL_OK) return rc;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hipfail(c, e, "stream synchronize");
    E_out[0] = c->na_E[0];
    E_out[1] = c->na_E[1];
    return check_density_flags(c, c->na_E.data(), 1);
}

// Logarithmic q mesh of the interpolation: q_1 = q1, q_nq = q_c, increments
// growing by the factor lambda, (q_{a+1} - q_a) = lambda (q_a - q_{a-1}).
static void log_qmesh(int nq, double q1, double qc, double lambda, double *q) {
    std::vector<double> d(nq - 1);
    double p = 1.0, tot = 0.0;
    for (int i = 0; i < nq - 1; ++i) { d[i] = p; tot += p; p *= lambda; }
    double acc = 0.0;
    q[0] = q1;
    for (int i = 1; i < nq - 1; ++i) {
        acc += d[i - 1];
        q[i] = q1 + (qc - q1) * (acc / tot);
    }
    q[nq - 1] = qc;
}

}  // namespace vdwnl

// ---------------------------------------------------------------- C ABI

extern "C" {

const char *vdwnl_strerror(int code) {
    switch (code) {
        case VDWNL_OK: return "ok";
        case VDWNL_E_ARG: return "invalid argument";
        case VDWNL_E_UNSUPPORTED_SIZE: return "unsupported grid size";
        case VDWNL_E_NOMEM: return "out of memory";
        case VDWNL_E_TABLE: return "invalid kernel table";
        case VDWNL_E_KRANGE: return "kernel table does not cover the grid's wave vectors";
        case VDWNL_E_STATE: return "grid or kernel table missing, or no device";
        case VDWNL_E_HIP: return "HIP runtime error";
        case VDWNL_E_BAD_DENSITY: return "invalid density (negative, NaN or infinite)";
        default: return "unknown error";
    }
}

static thread_local std::string g_create_err = "no error";

const char *vdwnl_last_error(const vdwnl_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

int vdwnl_create(vdwnl_ctx **out, int device) {
    if (!out) return VDWNL_E_ARG;
    *out = nullptr;
    if (device >= 0) {
        int count = 0;
        const hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess) {
            g_create_err = std::string("hipGetDeviceCount: ") + hipGetErrorString(e);
            return VDWNL_E_HIP;
        }
        if (device >= count) {
            g_create_err = "device " + std::to_string(device) + " not present (" + std::to_string(count) + " visible)";
            return VDWNL_E_STATE;
        }
    }
    vdwnl_ctx *c = new (std::nothrow) vdwnl_ctx();
    if (!c) return VDWNL_E_NOMEM;
    c->device = device;
    if (device >= 0) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
            if (prop.sharedMemPerBlock > 0) c->lds_cap = std::min<size_t>(prop.sharedMemPerBlock, 160 * 1024);
            c->arch = prop.gcnArchName;
        }
    }
    std::memset(&c->consts, 0, sizeof(Consts));
    if (device >= 0) {
        // set-up of the no-allocation entry point's buffer on this device
        const hipError_t e = scratch_setup(device);
        if (e != hipSuccess) {
            g_create_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            delete c;
            return VDWNL_E_HIP;
        }
    }
    *out = c;
    return VDWNL_OK;
}

int vdwnl_destroy(vdwnl_ctx *ctx) {
    if (!ctx) return VDWNL_E_ARG;
    free_device(ctx, true);
    delete ctx;
    return VDWNL_OK;
}

// three orthorhombic lengths per grid -> the diagonal cell matrices
static std::vector<double> diagonal_cells(int nb, const double *cells) {
    std::vector<double> lat((size_t)9 * std::max(nb, 0), 0.0);
    for (int i = 0; i < nb; ++i)
        for (int c = 0; c < 3; ++c) lat[9 * i + 4 * c] = cells[3 * i + c];
    return lat;
}

int vdwnl_set_grid(vdwnl_ctx *ctx, const int32_t shape[3], const double cell[3], int32_t grad_mode,
                   int32_t precision) {
    if (!ctx) return VDWNL_E_ARG;
    if (!shape || !cell) return fail(ctx, VDWNL_E_ARG, "null argument or empty batch");
    const std::vector<double> lat = diagonal_cells(1, cell);
    return plan_grids(ctx, 1, shape, lat.data(), grad_mode, precision);
}

int vdwnl_set_grids(vdwnl_ctx *ctx, int32_t nb, const int32_t *shapes, const double *cells, int32_t grad_mode,
                    int32_t precision) {
    if (!ctx) return VDWNL_E_ARG;
    if (!shapes || !cells || nb <= 0) return fail(ctx, VDWNL_E_ARG, "null argument or empty batch");
    const std::vector<double> lat = diagonal_cells(nb, cells);
    return plan_grids(ctx, nb, shapes, lat.data(), grad_mode, precision);
}

int vdwnl_set_grids_lattice(vdwnl_ctx *ctx, int32_t nb, const int32_t *shapes, const double *lattices,
                            int32_t grad_mode, int32_t precision) {
    if (!ctx) return VDWNL_E_ARG;
    return plan_grids(ctx, nb, shapes, lattices, grad_mode, precision);
}

int vdwnl_set_kernel_table(vdwnl_ctx *ctx, int32_t nq, const double *qmesh, double q_c, int32_t m_c, int32_t nk,
                           double dk, const double *phi, double c_soft) {
    if (!ctx) return VDWNL_E_ARG;
    if (!qmesh || !phi) return fail(ctx, VDWNL_E_ARG, "null table pointer");
    if (nq != kNQ) return fail(ctx, VDWNL_E_TABLE, "nq must be 20");
    if (m_c < 1 || m_c > kMaxMc) return fail(ctx, VDWNL_E_TABLE, "m_c must be in 1..64");
    if (nk < 4 || !(dk > 0.0) || !std::isfinite(dk)) return fail(ctx, VDWNL_E_TABLE, "bad radial mesh");
    if (!(q_c > 0.0) || !std::isfinite(c_soft)) return fail(ctx, VDWNL_E_TABLE, "bad q_c or C_s");
    for (int i = 0; i < nq; ++i) {
        if (!std::isfinite(qmesh[i]) || qmesh[i] <= 0.0) return fail(ctx, VDWNL_E_TABLE, "q mesh must be positive");
        if (i > 0 && !(qmesh[i] > qmesh[i - 1])) return fail(ctx, VDWNL_E_TABLE, "q mesh must increase strictly");
    }
    if (qmesh[nq - 1] != q_c) return fail(ctx, VDWNL_E_TABLE, "last q mesh point must equal q_c");
    const size_t n2 = (size_t)nq * nq;
    for (int a = 0; a < nq; ++a)
        for (int b = a + 1; b < nq; ++b) {
            const double *x = phi + ((size_t)a * nq + b) * nk, *y = phi + ((size_t)b * nq + a) * nk;
            for (int j = 0; j < nk; ++j)
                if (x[j] != y[j]) return fail(ctx, VDWNL_E_TABLE, "phi table must be symmetric in (a, b)");
        }
    for (size_t i = 0; i < n2 * nk; ++i)
        if (!std::isfinite(phi[i])) return fail(ctx, VDWNL_E_TABLE, "phi table has a non-finite value");
    ctx->nq = nq; ctx->mc = m_c; ctx->nk = nk; ctx->qc = q_c; ctx->dk = dk; ctx->cs = c_soft;
    ctx->qmesh.assign(qmesh, qmesh + nq);
    ctx->phi.assign((size_t)kNPair * nk, 0.0);
    ctx->d2.assign((size_t)kNPair * nk, 0.0);
    std::vector<double> kx(nk);
    for (int j = 0; j < nk; ++j) kx[j] = j * dk;
    int p = 0;
    for (int a = 0; a < nq; ++a)
        for (int b = a; b < nq; ++b, ++p) {
            std::memcpy(ctx->phi.data() + (size_t)p * nk, phi + ((size_t)a * nq + b) * nk, nk * sizeof(double));
            natural_spline_d2(kx.data(), ctx->phi.data() + (size_t)p * nk, nk, ctx->d2.data() + (size_t)p * nk);
        }
    // cardinal splines p_a: M[j][a] = second derivative at q_j of the spline through e_a
    Consts &k = ctx->consts;
    std::memset(&k, 0, sizeof(k));
    k.qc = q_c; k.iqc = 1.0 / q_c; k.cs = c_soft; k.nmin = 1e-30; k.mc = m_c; k.nq = nq;
    std::vector<double> e(nq), d2(nq);
    for (int a = 0; a < nq; ++a) {
        std::fill(e.begin(), e.end(), 0.0);
        e[a] = 1.0;
        natural_spline_d2(qmesh, e.data(), nq, d2.data());
        for (int j = 0; j < nq; ++j) k.M[j * kNQ + a] = d2[j];
    }
    for (int j = 0; j < nq; ++j) k.q[j] = qmesh[j];
    for (int m = 1; m <= kMaxMc; ++m) k.invm[m] = 1.0 / (double)m;
    ctx->have_table = true;
    free_device(ctx);
    const int rc = check_krange(ctx);
    refresh_image(ctx);
    return rc;
}

int vdwnl_energy_potential(vdwnl_ctx *ctx, const void *n_dev, void *v_dev, double *E_out, void *stream) {
    if (!ctx) return VDWNL_E_ARG;
    if (ctx->have_grid && ctx->grids.size() != 1) return fail(ctx, VDWNL_E_STATE, "context holds a batch plan");
    const void *np[1] = {n_dev};
    void *vp[1] = {v_dev};
    return run(ctx, 1, np, vp, E_out, stream);
}

int vdwnl_energy_potential_noalloc(vdwnl_ctx *ctx, const void *n_dev, void *v_dev, double *E_out, void *stream) {
    if (!ctx) return VDWNL_E_ARG;
    if (!n_dev || !v_dev || !E_out) return fail(ctx, VDWNL_E_ARG, "null pointer");
    if (!ctx->have_grid || !ctx->have_table) return fail(ctx, VDWNL_E_STATE, "grid and kernel table must both be set");
    if (ctx->grids.size() != 1) return fail(ctx, VDWNL_E_STATE, "context holds a batch plan");
    if (ctx->device < 0) return fail(ctx, VDWNL_E_STATE, "host-only context");
    if (ctx->timing) return fail(ctx, VDWNL_E_STATE, "per-pass timing needs vdwnl_energy_potential");
    const int krc = check_krange(ctx);
    if (krc != VDWNL_OK) return krc;
    if (!ctx->img_valid) {
        char msg[200];
        std::snprintf(msg, sizeof(msg),
                      "the plan needs %zu bytes of device scratch; vdwnl_energy_potential_noalloc has %zu",
                      ctx->img_need, kScratchBytes);
        return fail(ctx, VDWNL_E_UNSUPPORTED_SIZE, msg);
    }
    const int rc = run_noalloc(ctx, n_dev, v_dev, E_out, (hipStream_t)stream);
    ctx->last_functional = -1;   // (its semilocal energies are not kept)
    return rc;
}

int vdwnl_energy_potential_batched(vdwnl_ctx *ctx, int32_t nb, const void *const *n_ptrs, void *const *v_ptrs,
                                   double *E_out, void *stream) {
    if (!ctx) return VDWNL_E_ARG;
    return run(ctx, nb, n_ptrs, v_ptrs, E_out, stream);
}

int vdwnl_energy_potential_batched_async(vdwnl_ctx *ctx, int32_t nb, const void *const *n_ptrs,
                                         void *const *v_ptrs, double *E_dev, void *stream) {
    if (!ctx) return VDWNL_E_ARG;
    if (!E_dev) return fail(ctx, VDWNL_E_ARG, "null energy buffer");
    return run(ctx, nb, n_ptrs, v_ptrs, nullptr, stream, E_dev);
}

int vdwnl_debug_field(vdwnl_ctx *ctx, int32_t inst, int32_t which, void *dst, void *stream) {
    if (!ctx || !dst) return VDWNL_E_ARG;
    if (!ctx->device_ready || inst < 0 || inst >= (int32_t)ctx->grids.size())
        return fail(ctx, VDWNL_E_STATE, "no evaluation of that grid yet");
    const int rc = wait_pending(ctx);     // (the copy reads what that evaluation writes)
    if (rc != VDWNL_OK) return rc;
    const Grid &g = ctx->grids[inst];
    const size_t rs = ctx->precision == 64 ? 8 : 4;
    size_t off, bytes;
    if (which == 0) { off = g.off_grad; bytes = 3 * g.npts() * rs; }
    else if (which == 1) { off = g.off_vloc; bytes = g.npts() * rs; }
    else return fail(ctx, VDWNL_E_ARG, "which must be 0 or 1");
    hipError_t e = hipMemcpyAsync(dst, (char *)ctx->work + off, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    return e == hipSuccess ? VDWNL_OK : hipfail(ctx, e, "debug copy");
}

int vdwnl_debug_stage(vdwnl_ctx *ctx, int32_t inst, int32_t stage, void *dst, void *stream) {
    if (!ctx || !dst) return VDWNL_E_ARG;
    if (stage < VDWNL_STAGE_THETA || stage > VDWNL_STAGE_GRAD) return fail(ctx, VDWNL_E_ARG, "unknown stage");
    int rc = wait_pending(ctx);
    if (rc != VDWNL_OK) return rc;
    if (!ctx->device_ready || !ctx->evaluated || inst < 0 || inst >= (int32_t)ctx->grids.size())
        return fail(ctx, VDWNL_E_STATE, "no evaluation of that grid yet");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hipfail(ctx, e, "hipSetDevice");
    return probe_stage(ctx, stage, inst, dst, (hipStream_t)stream);
}

int vdwnl_log_qmesh(int32_t nq, double q1, double q_c, double lambda, double *q_out) {
    if (!q_out || nq < 2 || nq > 4096) return VDWNL_E_ARG;
    if (!(q1 > 0.0) || !(q_c > q1) || !std::isfinite(q_c) || !(lambda >= 1.0) || !std::isfinite(lambda))
        return VDWNL_E_ARG;
    // (lambda^(nq-2) must stay finite)
    if ((nq - 2) * std::log(lambda) > 700.0) return VDWNL_E_ARG;
    log_qmesh(nq, q1, q_c, lambda, q_out);
    return VDWNL_OK;
}

int vdwnl_set_graph(vdwnl_ctx *ctx, int32_t on) {
    if (!ctx) return VDWNL_E_ARG;
    ctx->use_graph = on != 0;
    return VDWNL_OK;
}

int vdwnl_set_functional(vdwnl_ctx *ctx, int32_t functional) {
    if (!ctx) return VDWNL_E_ARG;
    if (functional != VDWNL_FUNCTIONAL_NONLOCAL && functional != VDWNL_FUNCTIONAL_VDW_DF)
        return fail(ctx, VDWNL_E_ARG, "functional must be VDWNL_FUNCTIONAL_NONLOCAL or VDWNL_FUNCTIONAL_VDW_DF");
    ctx->functional = functional;
    return VDWNL_OK;
}

int vdwnl_semilocal_energies(const vdwnl_ctx *ctx, int32_t nb, double *E_out) {
    if (!ctx || !E_out) return VDWNL_E_ARG;
    // (an asynchronous evaluation in flight is waited for: its energies are
    // the last evaluation's)
    const int rc = wait_pending(const_cast<vdwnl_ctx *>(ctx));
    if (rc != VDWNL_OK) return rc;
    if (ctx->last_functional != VDWNL_FUNCTIONAL_VDW_DF || !ctx->h_E)
        return VDWNL_E_STATE;
    if (nb != (int32_t)ctx->grids.size()) return VDWNL_E_ARG;
    for (int i = 0; i < nb; ++i) {
        E_out[2 * i] = ctx->h_E[4 * i + 2];
        E_out[2 * i + 1] = ctx->h_E[4 * i + 3];
    }
    return VDWNL_OK;
}

int vdwnl_autotune(vdwnl_ctx *ctx, int32_t nb, const void *const *n_ptrs, void *const *v_ptrs, int32_t reps,
                   void *stream) {
    if (!ctx) return VDWNL_E_ARG;
    if (!ctx->have_grid || !ctx->have_table) return fail(ctx, VDWNL_E_STATE, "grid and kernel table must both be set");
    if (reps < 1 || reps > 100) return fail(ctx, VDWNL_E_ARG, "reps must be in 1..100");
    // candidate budgets; the tile sizing keeps at least one unit per tile, so
    // a budget below some pass's minimum simply gives that pass its minimum
    std::vector<size_t> cand;
    for (size_t b : {16384, 24576, 32768, 49152, 65536, 98304, 131072})
        if (b <= ctx->lds_cap) cand.push_back(b);
    const bool timing0 = ctx->timing;
    ctx->img_valid = false;     // (the candidates' tiles differ from the image's)
    for (auto &x : ctx->variant) x = 0;   // (the budgets are tuned with the first radix orders)
    // contraction units to try: the vector ALU, and the matrix cores where
    // some grid takes them (FP32, orthorhombic cell)
    std::vector<int> units = {VDWNL_CONTRACTION_VECTOR};
    bool any_orth = false;
    for (const auto &g : ctx->grids) any_orth = any_orth || !g.general;
    if (ctx->precision == 32 && any_orth) units.push_back(VDWNL_CONTRACTION_MATRIX);
    // t[unit][candidate][pass kind]
    std::vector<std::vector<std::vector<double>>> t(
        units.size(), std::vector<std::vector<double>>(cand.size(), std::vector<double>(KIND_COUNT, 0.0)));
    int rc = VDWNL_OK;
    std::vector<double> E((size_t)nb * 2);
    for (size_t ui = 0; ui < units.size() && rc == VDWNL_OK; ++ui)
        for (size_t ci = 0; ci < cand.size() && rc == VDWNL_OK; ++ci) {
            ctx->contraction = units[ui];
            for (auto &p : ctx->pref) p = cand[ci];
            for (auto &g : ctx->grids) size_tiles(ctx, g);
            free_device(ctx);
            ctx->timing = false;
            rc = run(ctx, nb, n_ptrs, v_ptrs, E.data(), stream);   // plans and warms up
            // the first candidate: untimed evaluations for a few hundred
            // milliseconds more (an idle device's clocks rise over its first
            // work, which would favour the candidates timed later)
            for (auto w0 = std::chrono::steady_clock::now();
                 ui == 0 && ci == 0 && rc == VDWNL_OK &&
                 std::chrono::steady_clock::now() - w0 < std::chrono::milliseconds(300);)
                rc = run(ctx, nb, n_ptrs, v_ptrs, E.data(), stream);
            if (rc != VDWNL_OK) break;
            vdwnl_set_timing(ctx, 1);
            for (int r = 0; r < reps && rc == VDWNL_OK; ++r) rc = run(ctx, nb, n_ptrs, v_ptrs, E.data(), stream);
            for (int k = 0; k < KIND_COUNT; ++k) t[ui][ci][k] = ctx->pass_ms[k];
        }
    // per group, the budget with the least time over the group's passes (a
    // group with no pass in this gradient mode keeps the default); for the
    // fused axis-1 group, the budget and the contraction unit together
    const std::vector<std::vector<int>> groups = {{KX_THETA, KX_ASSEMBLE},
                                                  {KY_20F, KY_20I},
                                                  {KG_Y, KD_Y},
                                                  {KZ_MAIN},
                                                  {KG_Z, KD_Z}};
    size_t best[TG_COUNT];
    int best_unit = VDWNL_CONTRACTION_VECTOR;
    for (int gi = 0; gi < TG_COUNT; ++gi) {
        double bt = 1e300;
        best[gi] = std::min<size_t>(ctx->lds_cap, kLdsCap);
        for (size_t ui = 0; ui < (gi == TG_Z ? units.size() : 1); ++ui)
            for (size_t ci = 0; rc == VDWNL_OK && ci < cand.size(); ++ci) {
                double sum = 0.0;
                for (int k : groups[gi]) sum += t[ui][ci][k];
                if (sum > 0.0 && sum < bt) {
                    bt = sum;
                    best[gi] = cand[ci];
                    if (gi == TG_Z) best_unit = units[ui];
                }
            }
    }
    ctx->contraction = best_unit;
    for (int gi = 0; gi < TG_COUNT; ++gi) ctx->pref[gi] = best[gi];
    // budgets and radix orders together, with the chosen unit: every group at
    // budget b and order v (each length class clamps v to its last variant)
    // for v = 0 .. kMaxVariants - 1 and every candidate b (order 0 timed
    // again, so that the pairs compared come from one stretch of runs), and
    // per group the pair with the least time over the group's passes (a
    // radix order changes the lanes per line, so the best tile width can
    // move with it)
    {
        // tv[v][candidate][pass kind]
        std::vector<std::vector<std::vector<double>>> tv(
            kMaxVariants, std::vector<std::vector<double>>(cand.size(), std::vector<double>(KIND_COUNT, 0.0)));
        for (int v = 0; v < kMaxVariants && rc == VDWNL_OK; ++v)
            for (size_t ci = 0; ci < cand.size() && rc == VDWNL_OK; ++ci) {
                for (auto &x : ctx->variant) x = v;
                for (auto &p : ctx->pref) p = cand[ci];
                for (auto &g : ctx->grids) size_tiles(ctx, g);
                free_device(ctx);
                ctx->timing = false;
                rc = run(ctx, nb, n_ptrs, v_ptrs, E.data(), stream);
                if (rc != VDWNL_OK) break;
                vdwnl_set_timing(ctx, 1);
                for (int r = 0; r < reps && rc == VDWNL_OK; ++r) rc = run(ctx, nb, n_ptrs, v_ptrs, E.data(), stream);
                for (int k = 0; k < KIND_COUNT; ++k) tv[v][ci][k] = ctx->pass_ms[k];
            }
        for (int gi = 0; gi < TG_COUNT; ++gi) {
            double bt = 1e300;
            int bv = 0;
            size_t bb = best[gi];
            for (int v = 0; rc == VDWNL_OK && v < kMaxVariants; ++v)
                for (size_t ci = 0; ci < cand.size(); ++ci) {
                    // (every pass whose transforms take the group's order: the
                    // axis-3 group's FP64 derivative passes too)
                    double sum = 0.0;
                    for (int k = 0; k < KIND_COUNT; ++k)
                        if (k != KF_GRAD && k != KF_DIV && variant_group(k) == gi) sum += tv[v][ci][k];
                    if (sum > 0.0 && sum < bt) {
                        bt = sum;
                        bv = v;
                        bb = cand[ci];
                    }
                }
            ctx->variant[gi] = bv;
            ctx->pref[gi] = bb;
        }
    }
    for (auto &g : ctx->grids) size_tiles(ctx, g);
    free_device(ctx);
    refresh_image(ctx);
    vdwnl_set_timing(ctx, timing0 ? 1 : 0);
    if (rc != VDWNL_OK) return rc;
    tuned_store(ctx->plan_key, ctx->pref, ctx->contraction, ctx->variant);
    return VDWNL_OK;
}

int vdwnl_set_tiling(vdwnl_ctx *ctx, int32_t ngroups, const int64_t *lds_budget) {
    if (!ctx || !lds_budget) return VDWNL_E_ARG;
    if (ngroups != TG_COUNT) return fail(ctx, VDWNL_E_ARG, "expected one budget per pass group (5)");
    if (!ctx->have_grid) return fail(ctx, VDWNL_E_STATE, "no grid planned");
    for (int i = 0; i < TG_COUNT; ++i)
        if (lds_budget[i] < 4096 || (size_t)lds_budget[i] > ctx->lds_cap)
            return fail(ctx, VDWNL_E_ARG, "LDS budget outside [4096, device LDS per workgroup]");
    for (int i = 0; i < TG_COUNT; ++i) ctx->pref[i] = (size_t)lds_budget[i];
    for (auto &g : ctx->grids) size_tiles(ctx, g);
    free_device(ctx);
    refresh_image(ctx);
    return VDWNL_OK;
}

int vdwnl_set_schedule(vdwnl_ctx *ctx, int32_t what, int32_t value) {
    if (!ctx) return VDWNL_E_ARG;
    if (what == VDWNL_SCHEDULE_CONTRACTION) {
        if (value != VDWNL_CONTRACTION_VECTOR && value != VDWNL_CONTRACTION_MATRIX)
            return fail(ctx, VDWNL_E_ARG, "contraction must be VDWNL_CONTRACTION_VECTOR or VDWNL_CONTRACTION_MATRIX");
    } else if (what >= VDWNL_SCHEDULE_RADIX_X && what <= VDWNL_SCHEDULE_RADIX_ZAUX) {
        if (value < 0 || value >= kMaxVariants) return fail(ctx, VDWNL_E_ARG, "radix order must be 0..5");
    } else {
        return fail(ctx, VDWNL_E_ARG, "unknown schedule choice");
    }
    if (!ctx->have_grid) return fail(ctx, VDWNL_E_STATE, "no grid planned");
    if (what == VDWNL_SCHEDULE_CONTRACTION) ctx->contraction = value;
    else ctx->variant[what - VDWNL_SCHEDULE_RADIX_X] = value;
    free_device(ctx);
    refresh_image(ctx);
    return VDWNL_OK;
}

int vdwnl_get_schedule(const vdwnl_ctx *ctx, int32_t what, int32_t *value) {
    if (!ctx || !value) return VDWNL_E_ARG;
    if (what == VDWNL_SCHEDULE_CONTRACTION) *value = ctx->contraction;
    else if (what >= VDWNL_SCHEDULE_RADIX_X && what <= VDWNL_SCHEDULE_RADIX_ZAUX) *value = ctx->variant[what - VDWNL_SCHEDULE_RADIX_X];
    else return VDWNL_E_ARG;
    return VDWNL_OK;
}

int vdwnl_radix_order(int32_t n, int32_t order, int32_t max_radices, int32_t *radices) {
    if (max_radices < 0 || (max_radices > 0 && !radices) || order < 0 || order >= kMaxVariants) return VDWNL_E_ARG;
    const int lc = len_class(n);
    int r[kMaxStages], nr = 0;
    if (lc == kLenGeneric) {
        FftPlan p;
        if (n < 1 || !radix_plan(n, p)) return VDWNL_E_UNSUPPORTED_SIZE;
        for (int i = 0; i < p.nstage; ++i) r[nr++] = p.radix[i];
    } else {
        nr = radix_order_of(lc, std::min<int>(order, kNumVariants[lc] - 1), r);
    }
    for (int i = 0; i < std::min<int>(nr, max_radices); ++i) radices[i] = r[i];
    return nr;
}

int vdwnl_get_tiling(const vdwnl_ctx *ctx, int32_t max_groups, int64_t *lds_budget) {
    if (!ctx || (max_groups > 0 && !lds_budget)) return VDWNL_E_ARG;
    for (int i = 0; i < std::min<int>(max_groups, TG_COUNT); ++i) lds_budget[i] = (int64_t)ctx->pref[i];
    return TG_COUNT;
}

int vdwnl_set_timing(vdwnl_ctx *ctx, int32_t on) {
    if (!ctx) return VDWNL_E_ARG;
    ctx->timing = on != 0;
    for (auto &m : ctx->pass_ms) m = 0.0;
    ctx->timed_calls = 0;
    return VDWNL_OK;
}

int vdwnl_pass_times(const vdwnl_ctx *ctx, int32_t max_passes, double *ms, int64_t *calls) {
    if (!ctx || (max_passes > 0 && !ms)) return VDWNL_E_ARG;
    const int n = std::min<int>(max_passes, KIND_COUNT + 1);
    for (int i = 0; i < n; ++i) ms[i] = ctx->pass_ms[i];
    if (calls) *calls = ctx->timed_calls;
    return KIND_COUNT + 1;
}

const char *vdwnl_pass_name(int32_t i) { return (i >= 0 && i <= KIND_COUNT) ? kPassName[i] : ""; }

int vdwnl_pass_order(const vdwnl_ctx *ctx, int32_t max_passes, int32_t *kinds) {
    if (!ctx || (max_passes > 0 && !kinds)) return VDWNL_E_ARG;
    const int *order;
    const int npass = pass_order(ctx->grad_mode, &order);
    for (int i = 0; i < std::min<int>(max_passes, npass); ++i) kinds[i] = order[i];
    return npass;
}

int vdwnl_info(const vdwnl_ctx *ctx, int32_t *n_grids, int64_t *workspace_bytes) {
    if (!ctx) return VDWNL_E_ARG;
    if (n_grids) *n_grids = (int32_t)ctx->grids.size();
    if (workspace_bytes) *workspace_bytes = (int64_t)ctx->work_bytes;
    return VDWNL_OK;
}

}  // extern "C"
