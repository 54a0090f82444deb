// Host-only exercise of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (test infrastructure): a
// context on device -1 plans grids, batches and lattices, takes kernel
// tables, re-plans tiles and schedules, reads a tuning file with malformed
// lines, and hits every argument check; nothing touches a GPU.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/vdwnl.h"

static int fails = 0;
#define EXPECT(cond)                                                       \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::fprintf(stderr, "line %d: expected %s\n", __LINE__, #cond); \
            ++fails;                                                       \
        }                                                                  \
    } while (0)

static std::vector<double> table(int nq, int nk, double qc, std::vector<double> &q) {
    q.assign(nq, 0.0);
    vdwnl_log_qmesh(nq, 0.05, qc, 1.17, q.data());
    std::vector<double> phi((size_t)nq * nq * nk);
    for (int a = 0; a < nq; ++a)
        for (int b = 0; b < nq; ++b)
            for (int j = 0; j < nk; ++j)
                phi[((size_t)a * nq + b) * nk + j] = std::exp(-0.01 * j) / (1.0 + a + b);
    return phi;
}

int main() {
    // strings of every code
    for (int c = 1; c >= -9; --c) EXPECT(vdwnl_strerror(c) != nullptr);
    for (int i = -2; i < 40; ++i) EXPECT(vdwnl_pass_name(i) != nullptr);
    // radix orders of many lengths
    int r[16];
    for (int n = 1; n <= 420; ++n)
        for (int v = 0; v < 6; ++v) {
            const int k = vdwnl_radix_order(n, v, 16, r);
            if (k > 0) {
                long p = 1;
                for (int i = 0; i < k && i < 16; ++i) p *= r[i];
                EXPECT(p == n);
            }
        }
    EXPECT(vdwnl_radix_order(128, 9, 16, r) == VDWNL_E_ARG);
    EXPECT(vdwnl_radix_order(128, 0, 4, nullptr) == VDWNL_E_ARG);
    double qm[32];
    EXPECT(vdwnl_log_qmesh(20, 0.05, 5.0, 1.17, qm) == VDWNL_OK);
    EXPECT(vdwnl_log_qmesh(1, 0.05, 5.0, 1.17, qm) != VDWNL_OK);

    for (int round = 0; round < 3; ++round) {
        vdwnl_ctx *h = nullptr;
        EXPECT(vdwnl_create(&h, -1) == VDWNL_OK);
        EXPECT(vdwnl_last_error(h) != nullptr);
        // grids: valid, ragged, unsupported, bad arguments
        const int32_t good[][3] = {{24, 24, 24}, {12, 30, 50}, {96, 96, 96}, {160, 160, 320}, {8, 6, 10}};
        const double cell[3] = {10.0, 11.0, 12.0};
        for (auto &s : good)
            for (int gm = 0; gm <= 4; ++gm)
                for (int prec : {32, 64}) EXPECT(vdwnl_set_grid(h, s, cell, gm, prec) == VDWNL_OK);
        const int32_t bad[][3] = {{14, 24, 24}, {24, 24, 3}, {256, 24, 24}, {24, 24, 512}, {15, 15, 16}, {0, 4, 4}};
        for (auto &s : bad) EXPECT(vdwnl_set_grid(h, s, cell, 0, 32) != VDWNL_OK);
        const double negcell[3] = {10.0, -1.0, 10.0};
        EXPECT(vdwnl_set_grid(h, good[0], negcell, 0, 32) == VDWNL_E_ARG);
        EXPECT(vdwnl_set_grid(h, good[0], cell, 7, 32) == VDWNL_E_ARG);
        EXPECT(vdwnl_set_grid(h, good[0], cell, 0, 16) == VDWNL_E_ARG);
        // batches of uneven grids
        std::vector<int32_t> shapes;
        std::vector<double> cells, lat;
        const int sizes[] = {32, 48, 64, 24, 96, 16, 40};
        for (int i = 0; i < 7; ++i) {
            for (int c = 0; c < 3; ++c) {
                shapes.push_back(sizes[i]);
                cells.push_back(0.2 * sizes[i]);
            }
            const double a = 0.2 * sizes[i];
            const double L[9] = {a, 0, 0, 0.1 * a, a, 0, 0.05 * a, -0.1 * a, a};
            lat.insert(lat.end(), L, L + 9);
        }
        for (int gm : {0, 3}) {
            EXPECT(vdwnl_set_grids(h, 7, shapes.data(), cells.data(), gm, 32) == VDWNL_OK);
            EXPECT(vdwnl_set_grids_lattice(h, 7, shapes.data(), lat.data(), gm, 64) == VDWNL_OK);
        }
        std::vector<double> flat(lat);
        for (int i = 0; i < 9; ++i) flat[i] = 0.0;   // no volume
        EXPECT(vdwnl_set_grids_lattice(h, 7, shapes.data(), flat.data(), 0, 32) == VDWNL_E_ARG);
        flat = lat;
        flat[4] = NAN;
        EXPECT(vdwnl_set_grids_lattice(h, 7, shapes.data(), flat.data(), 0, 32) == VDWNL_E_ARG);
        EXPECT(vdwnl_set_grids(h, 0, shapes.data(), cells.data(), 0, 32) == VDWNL_E_ARG);
        // kernel tables: valid, asymmetric, short range
        EXPECT(vdwnl_set_grids(h, 7, shapes.data(), cells.data(), 0, 32) == VDWNL_OK);
        std::vector<double> q;
        std::vector<double> phi = table(20, 1200, 5.0, q);
        EXPECT(vdwnl_set_kernel_table(h, 20, q.data(), 5.0, 12, 1200, 0.05, phi.data(), 0.04) == VDWNL_OK);
        std::vector<double> asym(phi);
        asym[1 * 1200 + 3] += 1.0;
        EXPECT(vdwnl_set_kernel_table(h, 20, q.data(), 5.0, 12, 1200, 0.05, asym.data(), 0.04) == VDWNL_E_TABLE);
        std::vector<double> qs;
        std::vector<double> shortphi = table(20, 40, 5.0, qs);   // reaches k = 1.95 only
        EXPECT(vdwnl_set_kernel_table(h, 20, qs.data(), 5.0, 12, 40, 0.05, shortphi.data(), 0.04) == VDWNL_E_KRANGE);
        EXPECT(vdwnl_set_kernel_table(h, 20, q.data(), 5.0, 0, 1200, 0.05, phi.data(), 0.04) == VDWNL_E_TABLE);
        // tiles, schedules, functional, timing, info
        const int64_t b[5] = {32768, 32768, 16384, 49152, 24576};
        EXPECT(vdwnl_set_tiling(h, 5, b) == VDWNL_OK);
        int64_t out[8];
        EXPECT(vdwnl_get_tiling(h, 8, out) == 5);
        const int64_t tiny[5] = {32768, 32768, 1024, 49152, 24576};
        EXPECT(vdwnl_set_tiling(h, 5, tiny) == VDWNL_E_ARG);
        for (int what = 0; what <= 5; ++what) {
            int32_t v = -1;
            EXPECT(vdwnl_set_schedule(h, what, what == 0 ? 1 : 5) == VDWNL_OK);
            EXPECT(vdwnl_get_schedule(h, what, &v) == VDWNL_OK);
        }
        EXPECT(vdwnl_set_schedule(h, 9, 0) == VDWNL_E_ARG);
        EXPECT(vdwnl_set_functional(h, 1) == VDWNL_OK);
        EXPECT(vdwnl_set_functional(h, 5) == VDWNL_E_ARG);
        int32_t kinds[32];
        EXPECT(vdwnl_pass_order(h, 32, kinds) > 0);
        int32_t ng = 0;
        int64_t ws = 0;
        EXPECT(vdwnl_info(h, &ng, &ws) == VDWNL_OK && ng == 7);
        // evaluations on a host-only context: state errors, no device work
        double E[16];
        const void *np[7] = {};
        void *vp[7] = {};
        EXPECT(vdwnl_energy_potential_batched(h, 7, np, vp, E, nullptr) == VDWNL_E_ARG);
        int dummy;
        for (auto &p : np) p = &dummy;
        for (auto &p : vp) p = &dummy;
        EXPECT(vdwnl_energy_potential_batched(h, 7, np, vp, E, nullptr) == VDWNL_E_STATE);
        EXPECT(vdwnl_energy_potential(h, &dummy, &dummy, E, nullptr) != VDWNL_OK);
        EXPECT(vdwnl_energy_potential_noalloc(h, &dummy, &dummy, E, nullptr) != VDWNL_OK);
        EXPECT(vdwnl_debug_stage(h, 0, 0, &dummy, nullptr) != VDWNL_OK);
        EXPECT(vdwnl_semilocal_energies(h, 7, E) != VDWNL_OK);
        EXPECT(vdwnl_destroy(h) == VDWNL_OK);
    }
    EXPECT(vdwnl_create(nullptr, -1) == VDWNL_E_ARG);
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("host driver ok\n");
    return 0;
}
