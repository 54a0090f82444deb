// Kernel-table generation on the GPU: the radial table phi_ab(k_j) that
// Eq. (Eoffk) needs, and the constant C_s of Eqs. (DEnl)/(Depsnl).
//
// 1. phi(d1, d2), the kernel of Eq. (Enl) (Dion et al. form), is a double
//    integral over the plane-wave variables a, b of a^2 b^2 W(a,b) T(...).
//    k_phi evaluates it for a list of (d1, d2): one workgroup per point, the
//    (a_i, a_j) plane swept in 256 x 256 tiles held in LDS, i <= j only.
// 2. On each ray d2/d1 = q_b/q_a the soft form of Eq. (PhiSoft) replaces phi
//    below D = |(d1, d2)| = d_s (value and slope matched at d_s).
// 3. k_radial integrates 4 pi D^2 j0(kappa D) phi_s(D) exactly for the
//    piecewise-quadratic interpolant of g(D) = D phi_s(D) on the sample mesh
//    (Filon: the linear interpolant plus, per interval, g''/2 (D - a)(D - b)
//    with g'' from the samples), so the result is stable for every kappa on
//    the table and the O(h^2) bias of a linear interpolant is removed;
//    beyond the last sample the r^-6 asymptote
//    -C/(d1^2 d2^2 (d1^2 + d2^2)) continues on a geometric mesh.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/vdwnl.h"
#include "common.hpp"

namespace vdwnl {
namespace tablegen {

constexpr double kPi = 3.14159265358979323846;
constexpr double kGamma = 4.0 * kPi / 9.0;
constexpr double kCasym = 12.0 * kGamma * kGamma * kGamma;
constexpr int kTile = 256;

// (sin x - x cos x) / x^3, with its Taylor series below 0.5
__host__ __device__ inline double f3(double x) {
    if (x < 0.5) {
        const double x2 = x * x;
        // 1/3 - x^2/30 + x^4/840 - x^6/45360 + x^8/3991680 - x^10/518918400
        return 1.0 / 3.0 + x2 * (-1.0 / 30.0 + x2 * (1.0 / 840.0 + x2 * (-1.0 / 45360.0 +
               x2 * (1.0 / 3991680.0 + x2 * (-1.0 / 518918400.0)))));
    }
    return (sin(x) - x * cos(x)) / (x * x * x);
}

__device__ inline double nu(double a, double d) {
    if (d <= 0.0) return 0.5 * a * a;
    if (a == 0.0) return d * d / (2.0 * kGamma);
    const double t = a / d;
    return a * a / (-2.0 * expm1(-kGamma * t * t));
}

// 1/x: the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r), within an ulp or so of 1/x for normal x (a few
// instructions against the division's fifteen-odd)
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// mesh: node a, weight w_i a_i^2 (times the smooth cutoff), S = sin a / a, F = f3(a)
struct MeshDev {
    const double *a, *wa, *S, *F;
    int na;
};

__global__ void __launch_bounds__(kTile) k_phi(const double *d1, const double *d2, const int *band,
                                              const MeshDev *meshes, double *out, int npts) {
    const int p = blockIdx.x;
    if (p >= npts) return;
    const MeshDev m = meshes[band[p]];
    const double x1 = d1[p], x2 = d2[p];
    __shared__ double jn1[kTile], jn2[kTile], jw[kTile], jS[kTile], jF[kTile], js[kTile];
    __shared__ double red[kTile / 64];
    const int nt = (m.na + kTile - 1) / kTile;
    double acc = 0.0;
    for (int ti = 0; ti < nt; ++ti) {
        const int i = ti * kTile + threadIdx.x;
        const bool iv = i < m.na;
        const double ai = iv ? m.a[i] : 1.0;
        const double n1i = nu(ai, x1), n2i = nu(ai, x2);
        const double wi = iv ? m.wa[i] : 0.0, Si = iv ? m.S[i] : 0.0, Fi = iv ? m.F[i] : 0.0;
        const double sii = rcp_nr(n1i + n2i);
        for (int tj = ti; tj < nt; ++tj) {
            __syncthreads();
            const int j = tj * kTile + threadIdx.x;
            if (j < m.na) {
                const double aj = m.a[j];
                const double n1j = nu(aj, x1), n2j = nu(aj, x2);
                jn1[threadIdx.x] = n1j;
                jn2[threadIdx.x] = n2j;
                js[threadIdx.x] = rcp_nr(n1j + n2j);
                jw[threadIdx.x] = m.wa[j];
                jS[threadIdx.x] = m.S[j];
                jF[threadIdx.x] = m.F[j];
            } else {
                jn1[threadIdx.x] = 1.0;
                jn2[threadIdx.x] = 1.0;
                js[threadIdx.x] = 0.5;
                jw[threadIdx.x] = 0.0;
                jS[threadIdx.x] = 0.0;
                jF[threadIdx.x] = 0.0;
            }
            __syncthreads();
            double row = 0.0;
            const int j0 = (tj == ti) ? threadIdx.x : 0;   // upper triangle of the diagonal tile
            for (int jj = j0; jj < kTile; ++jj) {
                const double x = jn1[jj], z = jn2[jj];
                const double W = 2.0 * (Si * jF[jj] + Fi * jS[jj] - 3.0 * Fi * jF[jj]);
                // T = (1/2) [1/(w+x) + 1/(y+z)] [1/((w+y)(x+z)) + 1/((w+z)(y+x))]
                // with w, y = nu(a_i) at d1, d2 and x, z = nu(a_j) at d1, d2:
                // the first bracket as one quotient, 1/(x+z) per j from LDS
                const double p1 = n1i + x, p2 = n2i + z;
                const double T = 0.5 * (p1 + p2) * rcp_nr(p1 * p2) *
                                 (sii * js[jj] + rcp_nr((n1i + z) * (n2i + x)));
                const double term = jw[jj] * W * T;
                row += (tj == ti && jj == (int)threadIdx.x) ? term : 2.0 * term;   // (i,j) and (j,i)
            }
            acc += wi * row;
        }
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kTile / 64; ++w) s += red[w];
        out[p] = 2.0 / (kPi * kPi) * s;
    }
}

// One thread per (ray, kappa): Psi(kappa) / (4 pi) = Int D^2 j0(kappa D) phi_s dD
// = (1/kappa) Int g(D) sin(kappa D) dD with g = D phi_s, between the samples
// D_n (ray r: samples [off[r], off[r+1]) of D and g) the linear interpolant
// plus cv_n (D - D_n)(D - D_{n+1}), cv_n = g''/2 on the interval.
__global__ void k_radial(const double *D, const double *g, const double *cv, const int *off, const double *Qr,
                         int nrays, int nk, double dk, double *out) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)nrays * nk) return;
    const int r = (int)(idx / nk), jk = (int)(idx % nk);
    const double kap = jk * dk / Qr[r];
    const int n0 = off[r], n1 = off[r + 1];
    double s = 0.0;
    if (jk == 0) {
        // Int g D dD, exact for linear g on each interval
        for (int n = n0; n + 1 < n1; ++n) {
            const double a = D[n], b = D[n + 1], h = b - a, ga = g[n], sl = (g[n + 1] - g[n]) / h;
            // Int (D - a)(D - b) D dD = -h^3 (a + b) / 12
            s += ga * (b * b - a * a) * 0.5 + sl * (h * h * (2.0 * b + a) / 6.0) - cv[n] * h * h * h * (a + b) / 12.0;
        }
        out[idx] = s;
        return;
    }
    // Int_a^b (g_a + sl (D - a)) sin(kD) dD with c = k (a+b)/2, e = k h / 2:
    //   g_a (2/k) sin c sin e + sl (2/k^2) [cos c e^3 f3(e) + e sin c sin e]
    for (int n = n0; n + 1 < n1; ++n) {
        const double a = D[n], b = D[n + 1], h = b - a;
        const double e = 0.5 * kap * h, c = 0.5 * kap * (a + b);
        double sc, cc, se, ce;
        sincos(c, &sc, &cc);
        sincos(e, &se, &ce);
        const double sl = (g[n + 1] - g[n]) / h;
        // Int (D - a)(D - b) sin(kD) dD = -4 (h/2)^3 f3(e) sin c
        const double hh = 0.5 * h;
        s += g[n] * (2.0 / kap) * sc * se + sl * (2.0 / (kap * kap)) * (cc * e * e * e * f3(e) + e * sc * se) -
             cv[n] * 4.0 * hh * hh * hh * f3(e) * sc;
    }
    out[idx] = s / kap;
}

}  // namespace tablegen
}  // namespace vdwnl

using namespace vdwnl::tablegen;

namespace {

struct HostMesh {
    std::vector<double> a, wa, S, F;
};

// Composite 8-point Gauss-Legendre: geometric panels (ratio 1.5) from 1e-5 up
// to 2 pi, panels of width pi/3 up to A, and a C-infinity cutoff
// 1 - s(t), s(t) = E(t) / (E(t) + E(1-t)), E(t) = exp(-1/t), from 0.3 A to A.
HostMesh make_mesh(double A) {
    static const double xg[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290, -0.1834346424956498,
                                 0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
    static const double wg[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873, 0.3626837833783620,
                                 0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    std::vector<double> edges = {0.0};
    for (double e = 1e-5; e < 2.0 * kPi; e *= 1.5) edges.push_back(e);
    edges.push_back(2.0 * kPi);
    while (edges.back() < A - 1e-12) edges.push_back(std::min(A, edges.back() + kPi / 3.0));
    HostMesh m;
    const double a1 = 0.3 * A;
    auto E = [](double t) { return t > 0.0 ? std::exp(-1.0 / t) : 0.0; };
    for (size_t p = 0; p + 1 < edges.size(); ++p) {
        const double lo = edges[p], hi = edges[p + 1];
        for (int q = 0; q < 8; ++q) {
            const double a = 0.5 * (hi - lo) * xg[q] + 0.5 * (hi + lo);
            double w = 0.5 * (hi - lo) * wg[q];
            if (a > a1) {
                const double t = (a - a1) / (A - a1);
                w *= 1.0 - E(t) / (E(t) + E(1.0 - t));
            }
            m.a.push_back(a);
            m.wa.push_back(w * a * a);
            m.S.push_back(a == 0.0 ? 1.0 : std::sin(a) / a);
            m.F.push_back(f3(a));
        }
    }
    return m;
}

// upper limits A of the a integration: the smallest with A >= 16 max(d1, d2),
// at least 192.  The truncation error of the tapered integral grows with d
// (the integrand varies on the scale a ~ d) and falls with A: about 1e-8
// relative at A = 16 d and A >= 192, while A = 96 leaves 1e-6..1e-5 at
// d ~ 7..12.  Beyond d = 144 the last band (|phi| < 1e-8 there).
const double kBandA[] = {192.0, 384.0, 768.0, 1536.0, 2304.0};
constexpr int kNBand = 5;

int band_of(double d1, double d2) {
    const double m = std::max(d1, d2);
    for (int b = 0; b < kNBand; ++b)
        if (kBandA[b] >= 16.0 * m) return b;
    return kNBand - 1;
}

struct Ray {
    double c, s, Q;       // cos, sin of the ray, |(q_a, q_b)|
    double X;             // last sampled D (asymptote beyond)
    std::vector<double> D;
    size_t first;         // index of D[0] in the point list (D >= d_s samples)
    size_t slope_first;   // 4 extra points at d_s -+ h, -+ 2h
    double phi2 = 0, phi4 = 0;
};

// phi(P1[i], P2[i]) on the current device, one workgroup per point.
int eval_phi(const std::vector<double> &P1, const std::vector<double> &P2, const std::vector<int> &PB,
             std::vector<double> &phi) {
    std::vector<HostMesh> hm;
    for (int b = 0; b < kNBand; ++b) hm.push_back(make_mesh(kBandA[b]));
    const int npts = (int)P1.size();
    phi.assign(npts, 0.0);
    if (npts == 0) return VDWNL_OK;
    {
        size_t tot = 0;
        for (auto &m : hm) tot += m.a.size();
        double *dmesh = nullptr, *dP1 = nullptr, *dP2 = nullptr, *dout = nullptr;
        int *dPB = nullptr;
        MeshDev *dmd = nullptr;
        bool ok = hipMalloc(&dmesh, 4 * tot * sizeof(double)) == hipSuccess &&
                  hipMalloc(&dP1, npts * sizeof(double)) == hipSuccess &&
                  hipMalloc(&dP2, npts * sizeof(double)) == hipSuccess &&
                  hipMalloc(&dout, npts * sizeof(double)) == hipSuccess &&
                  hipMalloc(&dPB, npts * sizeof(int)) == hipSuccess &&
                  hipMalloc(&dmd, kNBand * sizeof(MeshDev)) == hipSuccess;
        if (ok) {
            std::vector<double> flat(4 * tot);
            std::vector<MeshDev> md(kNBand);
            size_t o = 0;
            for (int b = 0; b < kNBand; ++b) {
                const size_t n = hm[b].a.size();
                std::memcpy(&flat[o], hm[b].a.data(), n * 8);
                std::memcpy(&flat[o + n], hm[b].wa.data(), n * 8);
                std::memcpy(&flat[o + 2 * n], hm[b].S.data(), n * 8);
                std::memcpy(&flat[o + 3 * n], hm[b].F.data(), n * 8);
                md[b] = MeshDev{dmesh + o, dmesh + o + n, dmesh + o + 2 * n, dmesh + o + 3 * n, (int)n};
                o += 4 * n;
            }
            ok = hipMemcpy(dmesh, flat.data(), flat.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(dmd, md.data(), md.size() * sizeof(MeshDev), hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(dP1, P1.data(), npts * 8, hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(dP2, P2.data(), npts * 8, hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(dPB, PB.data(), npts * 4, hipMemcpyHostToDevice) == hipSuccess;
        }
        if (ok) {
            hipLaunchKernelGGL(k_phi, dim3(npts), dim3(kTile), 0, 0, dP1, dP2, dPB, dmd, dout, npts);
            ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess &&
                 hipMemcpy(phi.data(), dout, npts * 8, hipMemcpyDeviceToHost) == hipSuccess;
        }
        for (void *p : {(void *)dmesh, (void *)dP1, (void *)dP2, (void *)dout, (void *)dPB, (void *)dmd})
            if (p) (void)hipFree(p);
        if (!ok) return VDWNL_E_HIP;
    }

    return VDWNL_OK;
}

}  // namespace

extern "C" int vdwnl_build_kernel_table(int device, int32_t nq, const double *qmesh, double d_s, double phi0,
                                        int32_t nk, double dk, double *phi_out, double *c_soft_out) {
    if (!qmesh || !phi_out || !c_soft_out || nq < 2 || nk < 2 || !(dk > 0.0) || !(d_s > 0.0))
        return VDWNL_E_ARG;
    for (int i = 0; i < nq; ++i)
        if (!(qmesh[i] > 0.0) || (i > 0 && !(qmesh[i] > qmesh[i - 1]))) return VDWNL_E_TABLE;
    if (device < 0) return VDWNL_E_STATE;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return VDWNL_E_HIP;

    // ---- points where phi is needed
    std::vector<double> P1, P2;
    std::vector<int> PB;
    auto add = [&](double x1, double x2) {
        P1.push_back(x1);
        P2.push_back(x2);
        PB.push_back(band_of(x1, x2));
    };
    const double h1 = d_s / 200.0;     // D step on [d_s, 10]
    std::vector<Ray> rays;
    for (int a = 0; a < nq; ++a)
        for (int b = a; b < nq; ++b) {
            Ray r;
            r.Q = std::hypot(qmesh[a], qmesh[b]);
            r.c = qmesh[a] / r.Q;
            r.s = qmesh[b] / r.Q;
            // the r^-6 asymptote needs both d1 and d2 large: samples reach
            // min(d1, d2) = 24 (phi/asymptote is 1.04 at min(d) = 4, 1.00000
            // from 12 on; D up to 2400 on the most skewed rays)
            r.X = std::min(24.0 / std::min(r.c, r.s), 2400.0);
            for (int i = 0; d_s + i * h1 < 10.0 - 1e-9; ++i) r.D.push_back(d_s + i * h1);
            for (int i = 0; 10.0 + i * 0.02 < std::min(40.0, r.X) - 1e-9; ++i) r.D.push_back(10.0 + i * 0.02);
            for (double D = 40.0; D < r.X - 1e-9; D *= 1.004) r.D.push_back(D);
            r.D.push_back(r.X);
            r.first = P1.size();
            for (double D : r.D) add(D * r.c, D * r.s);
            r.slope_first = P1.size();
            const double hh = 2e-3 * d_s;
            for (double D : {d_s - 2 * hh, d_s - hh, d_s + hh, d_s + 2 * hh}) add(D * r.c, D * r.s);
            rays.push_back(r);
        }
    // diagonal d1 = d2 = d on (0, d_s/sqrt 2) for C_s: 8-point Gauss-Legendre on geometric panels
    static const double xg[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290, -0.1834346424956498,
                                 0.1834346424956498, 0.5255324099163290, 0.7966664774136267, 0.9602898564975363};
    static const double wg[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873, 0.3626837833783620,
                                 0.3626837833783620, 0.3137066458778873, 0.2223810344533745, 0.1012285362903763};
    const size_t cs_first = P1.size();
    std::vector<double> cs_d, cs_w;
    {
        const double top = d_s / std::sqrt(2.0);
        std::vector<double> edges = {0.0};
        for (double x = 1e-7; x < top; x *= 1.6) edges.push_back(x);
        edges.push_back(top);
        for (size_t p = 0; p + 1 < edges.size(); ++p)
            for (int q = 0; q < 8; ++q) {
                const double lo = edges[p], hi = edges[p + 1];
                cs_d.push_back(0.5 * (hi - lo) * xg[q] + 0.5 * (hi + lo));
                cs_w.push_back(0.5 * (hi - lo) * wg[q]);
                add(cs_d.back(), cs_d.back());
            }
    }

    // ---- the phi kernel at every point
    std::vector<double> phi;
    {
        const int rc = eval_phi(P1, P2, PB, phi);
        if (rc != VDWNL_OK) return rc;
    }

    // ---- soft form per ray, samples of g = D phi_s on [0, X] and the asymptote beyond
    std::vector<double> Dall, gall, cvall, Qr;
    std::vector<int> off = {0};
    const double hh = 2e-3 * d_s;
    // g''/2 per interval.  Nodes carry g'' from their own piece (soft
    // polynomial and asymptote: analytic; sampled kernel: divided differences,
    // one-sided at the ends of the piece, as phi_s is only C^1 at d_s); an
    // interval takes the mean of its nodes, or the piece its interior lies in.
    auto curvatures = [&](size_t b, const std::vector<int> &seg, const std::vector<double> &d2) {
        const size_t n = Dall.size() - b;
        for (size_t i = 0; i < n; ++i) {
            double c = 0.0;
            if (i + 1 < n) {
                if (seg[i] == seg[i + 1]) c = 0.25 * (d2[i] + d2[i + 1]);
                else c = 0.5 * (seg[i + 1] == 2 ? d2[i + 1] : d2[i]);
            }
            cvall.push_back(c);
        }
    };
    for (auto &r : rays) {
        const size_t base = Dall.size();
        std::vector<int> seg;        // 0 soft polynomial, 1 sampled kernel, 2 asymptote
        std::vector<double> d2;      // g'' at the node
        const double *ps = &phi[r.slope_first];
        const double f = phi[r.first];                                      // phi(d_s) on the ray
        const double fp = (ps[0] - 8.0 * ps[1] + 8.0 * ps[2] - ps[3]) / (12.0 * hh);   // d phi / dD at d_s
        // phi0 + phi2 ds^2 + phi4 ds^4 = f,  2 phi2 ds + 4 phi4 ds^3 = fp
        r.phi4 = (0.5 * fp * d_s - (f - phi0)) / (d_s * d_s * d_s * d_s);
        r.phi2 = (f - phi0 - r.phi4 * d_s * d_s * d_s * d_s) / (d_s * d_s);
        for (int i = 0; i < 200; ++i) {
            const double D = i * h1, D2 = D * D;
            Dall.push_back(D);
            gall.push_back(D * (phi0 + r.phi2 * D2 + r.phi4 * D2 * D2));
            seg.push_back(0);
            d2.push_back(6.0 * r.phi2 * D + 20.0 * r.phi4 * D2 * D);   // (D phi_s)''
        }
        const size_t e0 = Dall.size();
        for (size_t i = 0; i < r.D.size(); ++i) {
            Dall.push_back(r.D[i]);
            gall.push_back(r.D[i] * phi[r.first + i]);
            seg.push_back(1);
            d2.push_back(0.0);
        }
        const size_t ne = Dall.size() - e0;
        for (size_t i = 0; i < ne && ne >= 3; ++i) {
            const size_t m = std::min(std::max<size_t>(i, 1), ne - 2) + e0;   // centre of the 3-point stencil
            const double x0 = Dall[m - 1], x1 = Dall[m], x2 = Dall[m + 1];
            const double y0 = gall[m - 1], y1 = gall[m], y2 = gall[m + 1];
            d2[e0 - base + i] = 2.0 * ((y2 - y1) / (x2 - x1) - (y1 - y0) / (x1 - x0)) / (x2 - x0);
        }
        const double coef = kCasym / (r.c * r.c * r.s * r.s);   // phi -> -coef / D^6
        for (double D = r.X * 1.005; D < 200.0 * r.X; D *= 1.005) {
            Dall.push_back(D);
            gall.push_back(-coef / (D * D * D * D * D));
            seg.push_back(2);
            const double D2 = D * D;
            d2.push_back(-30.0 * coef / (D2 * D2 * D2 * D));
        }
        curvatures(base, seg, d2);
        off.push_back((int)Dall.size());
        Qr.push_back(r.Q);
    }

    // ---- radial transforms
    const int nrays = (int)rays.size();
    std::vector<double> psi((size_t)nrays * nk);
    {
        double *dD = nullptr, *dg = nullptr, *dcv = nullptr, *dQ = nullptr, *dout = nullptr;
        int *doff = nullptr;
        bool ok = hipMalloc(&dD, Dall.size() * 8) == hipSuccess && hipMalloc(&dg, gall.size() * 8) == hipSuccess &&
                  hipMalloc(&dcv, cvall.size() * 8) == hipSuccess &&
                  hipMalloc(&dQ, Qr.size() * 8) == hipSuccess && hipMalloc(&doff, off.size() * 4) == hipSuccess &&
                  hipMalloc(&dout, psi.size() * 8) == hipSuccess;
        if (ok)
            ok = hipMemcpy(dD, Dall.data(), Dall.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(dg, gall.data(), gall.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(dcv, cvall.data(), cvall.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(dQ, Qr.data(), Qr.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(doff, off.data(), off.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
        if (ok) {
            const long tot = (long)nrays * nk;
            hipLaunchKernelGGL(k_radial, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, 0, dD, dg, dcv, doff, dQ, nrays,
                               nk, dk, dout);
            ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess &&
                 hipMemcpy(psi.data(), dout, psi.size() * 8, hipMemcpyDeviceToHost) == hipSuccess;
        }
        for (void *p : {(void *)dD, (void *)dg, (void *)dcv, (void *)dQ, (void *)dout, (void *)doff})
            if (p) (void)hipFree(p);
        if (!ok) return VDWNL_E_HIP;
    }
    int ray = 0;
    for (int a = 0; a < nq; ++a)
        for (int b = a; b < nq; ++b, ++ray) {
            const double Q3 = rays[ray].Q * rays[ray].Q * rays[ray].Q;
            for (int j = 0; j < nk; ++j) {
                const double v = 4.0 * kPi * psi[(size_t)ray * nk + j] / Q3;
                phi_out[((size_t)a * nq + b) * nk + j] = v;
                phi_out[((size_t)b * nq + a) * nk + j] = v;
            }
        }

    // ---- C_s = 1/2 Int_0^{d_s/sqrt2} 4 pi d^2 [phi(d,d) - phi_s(d,d)] dd on the diagonal ray
    {
        const Ray *dr = &rays[0];   // pair (0, 0): the diagonal ray, cos = sin
        double acc = 0.0;
        for (size_t i = 0; i < cs_d.size(); ++i) {
            const double d = cs_d[i], D2 = 2.0 * d * d;
            const double soft = phi0 + dr->phi2 * D2 + dr->phi4 * D2 * D2;
            acc += cs_w[i] * 4.0 * kPi * d * d * (phi[cs_first + i] - soft);
        }
        *c_soft_out = 0.5 * acc;
    }
    return VDWNL_OK;
}

extern "C" int vdwnl_kernel_phi(int device, int32_t n, const double *d1, const double *d2, double *out) {
    if (n < 0 || (n > 0 && (!d1 || !d2 || !out))) return VDWNL_E_ARG;
    for (int i = 0; i < n; ++i)
        if (!(d1[i] > 0.0) || !(d2[i] > 0.0) || !std::isfinite(d1[i]) || !std::isfinite(d2[i]) ||
            std::max(d1[i], d2[i]) > kBandA[kNBand - 1] / 5.0)
            return VDWNL_E_ARG;
    if (device < 0) return VDWNL_E_STATE;
    if (hipSetDevice(device) != hipSuccess) return VDWNL_E_HIP;
    std::vector<double> P1(d1, d1 + n), P2(d2, d2 + n), phi;
    std::vector<int> PB(n);
    for (int i = 0; i < n; ++i) PB[i] = band_of(d1[i], d2[i]);
    const int rc = eval_phi(P1, P2, PB, phi);
    if (rc != VDWNL_OK) return rc;
    std::memcpy(out, phi.data(), (size_t)n * sizeof(double));
    return VDWNL_OK;
}
