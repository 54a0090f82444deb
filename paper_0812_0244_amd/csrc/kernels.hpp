// HIP kernels of libvdwnl (gfx950), as templates in the working precision T;
// kernels_f32_{x,y,z}.hip and kernels_f64_{x,y,z}.hip instantiate them per pass
// family (compiled in parallel).  One evaluation of E_c^nl and v_nl is eleven
// passes over the grid with the spectral gradient (its gradient and
// divergence one pass per grid axis each), seven with finite differences;
// each pass is one launch per FFT length class that covers every grid of the
// batch (a workgroup reads its work item from a tile list).
//
// The 20 theta / u fields (the bulk of the traffic), the local chain and the
// divergence of w are computed in the working precision T (float or double).
// The spectral gradient of n always transforms in FP64: the gradient term of
// v_nl multiplies grad n by a factor that grows as 1/n, so FP32 rounding of a
// spectral grad n in the low-density regions would dominate the error of v.
//
// Fields are transformed with three 1-D FFT passes: along axis 3 (the
// contiguous one, real-to-complex by pairing two real lines into one complex
// line), axis 2 and axis 1.  Spectra keep all components of one k point
// together ([N1][N2][N3/2+1][V] complex), so the axis-1 pass of the 20 theta
// spectra holds every component of its k points in LDS and can apply the
// per-k kernel matrix between its forward and inverse FFTs.
#pragma once

#include "common.hpp"
#include "fft_fast.hpp"
#include "tile_io.hpp"

namespace vdwnl {

// ---------------------------------------------------------------- helpers

// Elementary functions of the local chain.  FP64: the device library.  FP32
// (arguments positive and normal there): built on the hardware base-2
// logarithm and exponential (v_log_f32, v_exp_f32), square root and
// reciprocal, each within about an ulp, in a few instructions where the
// library's general versions (special values, denormals, extra-precise
// arithmetic) take tens to a hundred.
__device__ __forceinline__ float hw_log(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ __forceinline__ float hw_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
template <typename T> __device__ __forceinline__ T dev_cbrt(T x);
template <> __device__ __forceinline__ float dev_cbrt(float x) {
    // 2^(log2(x)/3), then one Newton step for r^3 = x
    const float r = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(x) * (1.0f / 3.0f));
    return r + (x * __builtin_amdgcn_rcpf(r * r) - r) * (1.0f / 3.0f);
}
template <> __device__ __forceinline__ double dev_cbrt(double x) { return cbrt(x); }
template <typename T> __device__ __forceinline__ T dev_sqrt(T x);
template <> __device__ __forceinline__ float dev_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double dev_sqrt(double x) { return sqrt(x); }
// 1/x: the hardware reciprocal in FP32 (within 1 ulp), a division in FP64
template <typename T> __device__ __forceinline__ T rcp(T x);
template <> __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
// FP64: the hardware estimate refined by two Newton-Raphson steps
// r <- r + r (1 - x r) (each doubles the correct bits; within an ulp or so
// of 1/x for normal x, against about fifteen instructions for a division)
template <> __device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}
template <typename T> __device__ __forceinline__ T dev_log1p(T x);
template <> __device__ __forceinline__ float dev_log1p(float x) {
    // log(u) x / (u - 1) with u = 1 + x as rounded: the quotient restores what
    // the rounding of 1 + x lost (Goldberg 1991, Theorem 4); x itself when u = 1
    const float u = 1.0f + x, d = u - 1.0f;
    return d == 0.0f ? x : hw_log(u) * (x * __builtin_amdgcn_rcpf(d));
}
template <> __device__ __forceinline__ double dev_log1p(double x) { return log1p(x); }
template <typename T> __device__ __forceinline__ T dev_exp(T x);
template <> __device__ __forceinline__ float dev_exp(float x) { return hw_exp(x); }
template <> __device__ __forceinline__ double dev_exp(double x) { return exp(x); }
template <typename T> __device__ __forceinline__ T dev_expm1(T x);
template <> __device__ __forceinline__ float dev_expm1(float x) {
    // |x| < 1/2: x (1 + x/2! + ... + x^8/9!) (Taylor; the rest is below 1e-9
    // relative); elsewhere exp(x) - 1, where no cancellation can hurt
    float p = 1.0f / 362880.0f;
    p = p * x + 1.0f / 40320.0f;
    p = p * x + 1.0f / 5040.0f;
    p = p * x + 1.0f / 720.0f;
    p = p * x + 1.0f / 120.0f;
    p = p * x + 1.0f / 24.0f;
    p = p * x + 1.0f / 6.0f;
    p = p * x + 0.5f;
    p = p * x + 1.0f;
    return fabsf(x) < 0.5f ? x * p : hw_exp(x) - 1.0f;
}
template <> __device__ __forceinline__ double dev_expm1(double x) { return expm1(x); }

// signed frequency index of position k on an axis of N points, 0 at Nyquist
__device__ __forceinline__ int freq_nz(int k, int N) {
    int m = (k <= N / 2) ? k : k - N;
    if ((N & 1) == 0 && k == N / 2) m = 0;
    return m;
}
__device__ __forceinline__ int freq_abs(int k, int N) { return k <= N - k ? k : N - k; }

// Cartesian components of G = m1 b_1 + m2 b_2 + m3 b_3 (the frequencies with
// Nyquist taken as zero); in an orthorhombic cell the off-diagonal b_c,x are
// zero and each component is the single product m_c b_c,c exactly.
template <typename T>
__device__ __forceinline__ void cart_g(const InstDev &I, double m1, double m2, double m3, T &gx, T &gy, T &gz) {
    gx = (T)(m1 * I.B[0][0] + m2 * I.B[1][0] + m3 * I.B[2][0]);
    gy = (T)(m1 * I.B[0][1] + m2 * I.B[1][1] + m3 * I.B[2][1]);
    gz = (T)(m1 * I.B[0][2] + m2 * I.B[1][2] + m3 * I.B[2][2]);
}

// Sum over the workgroup in a fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[kThreads / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kThreads / 64; ++w) s += red[w];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------- q0 and the spline basis

// q0(n, |grad n|^2) before saturation and its partials (Dion et al. form,
// Perdew-Wang 1992 correlation), then the saturation of Eq. (Sat).
template <typename T, bool DERIV>
struct LocalQ {
    T q0, Q, dqdn, ndqds;    // ndqds = n dq0/dsigma (dq0/dsigma alone overflows FP32 at small n)
    T kf, eps, deps_dn;      // k_F, the LDA eps_c and (DERIV) d eps_c/dn

    __device__ __forceinline__ void eval(T n, T sigma, double qc, double iqc, int mc, const T *invm) {
        const T pi = (T)3.14159265358979323846;
        const T A = (T)0.031091, a1 = (T)0.21370;
        const T b1 = (T)7.5957, b2 = (T)3.5876, b3 = (T)1.6382, b4 = (T)0.49294;
        const T zg = (T)(0.8491 / 36.0);   // -Z_ab / 36
        // k_F = (3 pi^2 n)^(1/3), r_s = (3 / (4 pi n))^(1/3): one cube root
        const T cn = dev_cbrt<T>(n), icn = rcp<T>(cn), in = rcp<T>(n);
        kf = (T)3.0936677262801355 * cn;                  // (3 pi^2)^(1/3)
        const T rs = (T)0.6203504908994001 * icn;         // (3 / (4 pi))^(1/3)
        const T srs = dev_sqrt<T>(rs);
        const T P = b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs;
        const T iP2A = rcp<T>((T)2 * A * P);
        const T L = dev_log1p<T>(iP2A);
        eps = (T)-2 * A * ((T)1 + a1 * rs) * L;
        // sigma / (k_F n^2) as ((sigma / n) / n) / k_F: finite in FP32 wherever
        // |grad n| / n is, down to n_min (1 / (k_F n^2) alone is not below 1e-17)
        const T ikf = rcp<T>(kf);
        const T grad_term = zg * ((sigma * in) * in) * ikf;
        const T qraw = kf - ((T)4 * pi / (T)3) * eps + grad_term;
        if (DERIV) {
            const T dP = (T)0.5 * b1 * rcp<T>(srs) + b2 + (T)1.5 * b3 * srs + (T)2 * b4 * rs;
            const T deps_drs = (T)-2 * A * a1 * L + (T)2 * A * ((T)1 + a1 * rs) * dP * rcp<T>(P * ((T)2 * A * P + (T)1));
            deps_dn = deps_drs * (-rs * in * ((T)1 / (T)3));
            dqdn = kf * in * ((T)1 / (T)3) - ((T)4 * pi / (T)3) * deps_dn - ((T)7 / (T)3) * grad_term * in;
            ndqds = zg * ikf * in;
        }
        // h(x, x_c) = x_c (1 - exp(-S)), S = sum_{m<=m_c} (x/x_c)^m / m (Horner),
        // dh/dx = exp(-S) sum_{m<m_c} (x/x_c)^m.  1 - exp(-S) as -expm1(-S)
        // keeps its relative accuracy for small S.  S from 80 up (exp(-S) <
        // 2e-35), or overflowing, saturates: h = x_c, dh/dx = 0.  Below that
        // the derivative series stays under 80 m_c^2: no overflow in FP32.
        const T y = qraw * (T)iqc;
        T S = (T)0;
        for (int m = mc; m >= 1; --m) S = S * y + invm[m];
        S *= y;
        if (!(S < (T)80)) {
            q0 = (T)qc;
            Q = (T)0;
            if (DERIV) { dqdn = (T)0; ndqds = (T)0; }   // (their products with Q vanish)
        } else {
            q0 = (T)(-qc) * dev_expm1<T>(-S);
            if (DERIV) {
                T D = (T)0;
                for (int m = mc - 1; m >= 0; --m) D = D * y + (T)1;
                Q = dev_exp<T>(-S) * D;
            } else {
                Q = (T)0;
            }
        }
    }
};

// Largest finite value of T.
template <typename T>
__device__ __forceinline__ constexpr T finite_max() {
    if constexpr (sizeof(T) == 4) return __FLT_MAX__;
    else return __DBL_MAX__;
}

// The semilocal terms of Eq. (Exc) at one point, from n, sigma = |grad n|^2
// and the k_F, eps_c (and d eps_c/dn) of LocalQ.  Exchange: the revPBE GGA,
// e_x = e_u F_x(s) with e_u = -3 k_F n / (4 pi), s^2 = sigma / (4 k_F^2 n^2),
// F_x = 1 + kappa - kappa / (1 + mu s^2 / kappa), kappa = 1.245,
// mu = 0.066725 pi^2 / 3; correlation: the LDA e_c = n eps_c.
template <typename T>
struct Semilocal {
    T ex, ec;                // energies per volume
    T dn, ds;                // d(e_x + e_c)/dn, d e_x/dsigma (DERIV)
    template <bool DERIV>
    __device__ __forceinline__ void eval(T n, T sigma, const LocalQ<T, DERIV> &lq) {
        const T kappa = (T)1.245, mu = (T)(0.066725 * 3.14159265358979323846 * 3.14159265358979323846 / 3.0);
        const T in = rcp<T>(n), ikf = rcp<T>(lq.kf);
        const T eu = (T)(-3.0 / (4.0 * 3.14159265358979323846)) * lq.kf * n;
        // s^2 = sigma / (4 k_F^2 n^2), ordered to stay finite at small n; where
        // it still overflows (or is huge) F_x has reached 1 + kappa
        const T s2 = ((sigma * in) * in) * ((T)0.25 * ikf * ikf);
        const bool flat = !(s2 < (T)1e30);
        const T iden = flat ? (T)0 : rcp<T>((T)1 + (mu / kappa) * s2);
        const T fx = (T)1 + kappa - kappa * iden;
        ex = eu * fx;
        ec = n * lq.eps;
        if (DERIV) {
            const T dfx = mu * iden * iden;                  // dF_x / ds^2
            const T dfx_s2 = flat ? (T)0 : dfx * s2;
            // d e_u/dn = (4/3) e_u / n, d s^2/dn = -(8/3) s^2 / n;
            // d e_x/dsigma = e_u F_x' / (4 k_F^2 n^2) = -3 F_x' / (16 pi k_F n)
            dn = ((T)(4.0 / 3.0) * fx - (T)(8.0 / 3.0) * dfx_s2) * eu * in + lq.eps + n * lq.deps_dn;
            ds = (T)(-3.0 / (16.0 * 3.14159265358979323846)) * dfx * rcp<T>(lq.kf * n);
        }
    }
};

// Natural cubic cardinal splines p_a(q) on the q mesh (Eq. fofx and the text
// after it), M[j][a] (second derivative at q_j of p_a) in LDS.  On the
// interval j (a = (q_{j+1} - q)/h, b = 1 - a)
//   p_a  = a d_aj + b d_a,j+1 + ((a^3 - a) M[j][a] + (b^3 - b) M[j+1][a]) h^2/6
//   p_a' = (d_a,j+1 - d_aj)/h + ((1 - 3a^2) M[j][a] + (3b^2 - 1) M[j+1][a]) h/6
// and below q_1 the linear continuation p_a(q_1) + (q - q_1) p_a'(q_1).  Both
// are written p_a = A0 d_aj + A1 d_a,j+1 + C0 M[j][a] + C1 M[j+1][a] and
// p_a' = B0 d_aj + B1 d_a,j+1 + D0 M[j][a] + D1 M[j+1][a] with per-point
// scalars, so sums over a reduce to two dot products with rows of M.
template <typename T>
struct SplineW {
    int j;
    T A0, A1, C0, C1;
    T B0, B1, D0, D1;

    __device__ __forceinline__ void locate(T q0, const T *qm, int nq) {
        // one path for every case (the struct then stays in registers)
        const bool below = q0 < qm[0];
        int lo = 0, hi = nq - 1;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (qm[mid] <= q0) lo = mid; else hi = mid;
        }
        j = lo;
        const T ql = qm[lo], qh = qm[lo + 1];
        const T h = qh - ql, ih = rcp<T>(h), h6 = h * (T)(1.0 / 6.0);
        const T a = below ? (T)1 : (qh - q0) * ih;
        const T b = (T)1 - a;
        const T dq = below ? q0 - ql : (T)0;
        B0 = -ih;
        B1 = ih;
        D0 = ((T)1 - (T)3 * a * a) * h6;
        D1 = ((T)3 * b * b - (T)1) * h6;
        A0 = a + dq * B0;
        A1 = b + dq * B1;
        C0 = (a * a * a - a) * h * h6 + dq * D0;
        C1 = (b * b * b - b) * h * h6 + dq * D1;
    }
};

// q mesh, spline second derivatives and 1/m into LDS (in T); all loads are
// issued before any store (indices clamped, the stores guarded)
template <typename T>
__device__ __forceinline__ void load_consts(const Consts *cst, T *qm, T *Mm, T *invm) {
    static_assert(kNQ * kNQ <= 2 * kThreads && kNQ <= kThreads && kMaxMc < kThreads, "one or two steps each");
    const int i = threadIdx.x, i2 = threadIdx.x + kThreads;
    const gptr<const double> q = gld(cst->q), M = gld(cst->M), im = gld(cst->invm);
    const double a = q[min(i, kNQ - 1)], b = M[min(i, kNQ * kNQ - 1)], b2 = M[min(i2, kNQ * kNQ - 1)];
    const double c = im[min(i, kMaxMc)];
    if (i < kNQ) qm[i] = (T)a;
    if (i < kNQ * kNQ) Mm[i] = (T)b;
    if (i2 < kNQ * kNQ) Mm[i2] = (T)b2;
    if (i <= kMaxMc) invm[i] = (T)c;
}

// ---------------------------------------------------------------- axis-3 passes

// theta_a = n p_a(q0) from n and the stored grad n, Delta E partials, R2C of
// the 20 theta rows.  tile: a = first row, b = rows, slot = partial.
template <typename T, int LC, int V>
__global__ void __launch_bounds__(kThreads) k_x_theta(const InstDev *insts, const Tile *tiles,
                                                      const Consts *cst, const void *twv) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile t = tiles[blockIdx.x];
    const InstDev &I = insts[t.inst];
    const int N3 = axis_len<LC>(I.n3), N3h = N3 / 2 + 1, row0 = t.a, B = t.b, ls = N3 + 1;
    const size_t N = (size_t)I.n1 * I.n2 * I.n3;
    C2<T> *r2 = reinterpret_cast<C2<T> *>(smem);              // 10 lines per row: theta pairs
    C2<T> *tw = r2 + kNQ / 2 * B * ls;                       // twiddles in T
    T *qm = reinterpret_cast<T *>(tw + N3);
    T *Mm = qm + kNQ;
    T *invm = Mm + kNQ * kNQ;
    // density and grad n of this thread's first point, fetched first (used
    // after the constants arrive); unconditional loads, clamped to the tile: a
    // load under a branch would be waited for where the branch joins
    const int npt = B * N3;
    const size_t p0 = (size_t)row0 * N3;
    const gptr<const T> nin = gld(reinterpret_cast<const T *>(I.n) + p0);
    const gptr<const T> gin = gld(reinterpret_cast<const T *>(I.grad) + p0);
    const int i_first = min((int)threadIdx.x, npt - 1);
    const T n_first = nin[i_first], gx_f = gin[i_first], gy_f = gin[N + i_first], gz_f = gin[2 * N + i_first];
    load_consts<T>(cst, qm, Mm, invm);
    load_twiddles<T>(tw, I.p3, reinterpret_cast<const C2<T> *>(twv));
    __syncthreads();

    const double c_qc = cst->qc, c_iqc = cst->iqc, c_cs = cst->cs, c_nmin = cst->nmin;
    const int c_mc = cst->mc;
    const bool semilocal = I.semilocal != 0;
    double de = 0.0, dex = 0.0, dec = 0.0;
    for (int idx = threadIdx.x; idx < npt; idx += kThreads) {
        const int rb = idx / N3, k = idx - rb * N3;
        const bool first = idx == (int)threadIdx.x;
        const T nv = first ? n_first : nin[idx];
        const C2<T> g01 = mk<T>(first ? gx_f : gin[idx], first ? gy_f : gin[N + idx]);
        const C2<T> g2 = mk<T>(first ? gz_f : gin[2 * N + idx], (T)0);
        T *th = reinterpret_cast<T *>(r2 + (size_t)(kNQ / 2 * rb) * ls);   // pair line m at th + 2 m ls
        // a density the method is not defined for (negative, NaN, infinite):
        // flag the grid (its energies come out NaN, the call reports it)
        if (!(nv >= (T)0 && nv <= finite_max<T>())) gst(I.bad)[0] = 1;
        if (nv >= (T)c_nmin) {
            LocalQ<T, false> lq;
            const T sigma = g01.x * g01.x + g01.y * g01.y + g2.x * g2.x;
            lq.eval(nv, sigma, c_qc, c_iqc, c_mc, invm);
            if (semilocal) {
                Semilocal<T> sl;
                sl.eval(nv, sigma, lq);
                dex += (double)sl.ex;
                dec += (double)sl.ec;
            }
            SplineW<T> sw;
            sw.locate(lq.q0, qm, kNQ);
            const T *Mj = Mm + sw.j * kNQ;
            const T nC0 = nv * sw.C0, nC1 = nv * sw.C1;
            // pair m = (theta_2m, theta_2m+1) as one 8- or 16-byte store: lanes
            // (consecutive k) then touch consecutive LDS words
            C2<T> *thc = reinterpret_cast<C2<T> *>(th) + k;   // pair line m at thc[m ls]
#pragma unroll
            for (int m = 0; m < kNQ / 2; ++m)
                thc[m * ls] = mk<T>(nC0 * Mj[2 * m] + nC1 * Mj[kNQ + 2 * m], nC0 * Mj[2 * m + 1] + nC1 * Mj[kNQ + 2 * m + 1]);
            // the interpolating parts A0 d_aj + A1 d_a,j+1 touch components j and
            // j + 1: rewrite the pair (j even) or the two pairs (j odd) that hold
            // them (same thread, so after the loop's stores)
            const int j0 = sw.j, m0 = j0 >> 1;
            const bool odd = (j0 & 1) != 0;
            const T nA0 = nv * sw.A0, nA1 = nv * sw.A1;
            const T *M0 = Mj + 2 * m0, *M1 = Mj + kNQ + 2 * m0;
            thc[m0 * ls] = mk<T>(nC0 * M0[0] + nC1 * M1[0] + (odd ? (T)0 : nA0), nC0 * M0[1] + nC1 * M1[1] + (odd ? nA0 : nA1));
            if (odd) thc[(m0 + 1) * ls] = mk<T>(nC0 * M0[2] + nC1 * M1[2] + nA1, nC0 * M0[3] + nC1 * M1[3]);
            const T iq = rcp<T>(lq.q0);
            de += (double)((T)c_cs * nv * nv * iq * iq * iq);
        } else {
            C2<T> *thc = reinterpret_cast<C2<T> *>(th) + k;
#pragma unroll
            for (int m = 0; m < kNQ / 2; ++m) thc[m * ls] = mk<T>((T)0, (T)0);
        }
    }
    __syncthreads();
    fft_lc<T, -1, LC, V>(r2, I.p3, kNQ / 2 * B, 1, ls, tw);

    // pair line m of row rb holds theta_{2m} + i theta_{2m+1}: its values at
    // k and N3 - k give both spectra at k, written together (item idx =
    // (rb N3h + k) 10 + m lands at spectrum element 2 idx)
    C2<T> *out = reinterpret_cast<C2<T> *>(I.spec) + (size_t)row0 * N3h * kNQ;
    Cursor3 cur(threadIdx.x, kNQ / 2, N3h);
    for (int idx = threadIdx.x; idx < B * N3h * (kNQ / 2); idx += kThreads, cur.step()) {
        const int m = cur.m, k = cur.k, rb = cur.r;
        const C2<T> *Z = r2 + (kNQ / 2 * rb + m) * ls;
        const C2<T> z = Z[k], zc = cconj(Z[k == 0 ? 0 : N3 - k]);
        const T ex = (z.x + zc.x) * (T)0.5, ey = (z.y + zc.y) * (T)0.5;
        const T ox = (z.y - zc.y) * (T)0.5, oy = -(z.x - zc.x) * (T)0.5;
        C2<T> *o = out + 2 * (size_t)idx;
        if constexpr (sizeof(T) == 4) gst(reinterpret_cast<float4 *>(o))[0] = make_float4(ex, ey, ox, oy);
        else { gst(o)[0] = mk<T>(ex, ey); gst(o)[1] = mk<T>(ox, oy); }
    }
    const double s = block_sum(de);
    double sx = 0.0, sc = 0.0;
    if (semilocal) {                 // (uniform over the workgroup)
        sx = block_sum(dex);
        sc = block_sum(dec);
    }
    if (threadIdx.x == 0) {
        I.part_de[t.slot] = s;
        I.part_sl[2 * t.slot] = sx;
        I.part_sl[2 * t.slot + 1] = sc;
    }
}

// The u spectra of B rows (axis 3 half spectra, [B][N3h][kNQ] complex at sp)
// into LDS pair lines ready for the inverse axis-3 FFT: u_{2m} + i u_{2m+1}
// on pair line m of row rb (at r2 + (10 rb + m) ls), from the spectra at k
// (< N3/2 + 1) both the value at k and, by Hermitian symmetry, at N3 - k.
// Item idx = (rb N3h + k) 10 + m reads spectrum elements 2 idx, 2 idx + 1;
// about five steps per thread for every length class: batches of six.
template <typename T>
__device__ __forceinline__ void u_lines_in(C2<T> *r2, int ls, const C2<T> *sp, int B, int N3, int N3h) {
    constexpr int U = 6;
    const int total = B * N3h * (kNQ / 2);
    Cursor3 cur(threadIdx.x, kNQ / 2, N3h);
    const gptr<const C2<T>> g = gld(sp);
    for (int base = threadIdx.x; base < total; base += U * kThreads) {
        C2<T> ya[U], yb[U];
        int lo[U], kk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int idx = base + u * kThreads;
            const bool on = idx < total;
            const size_t e = on ? 2 * (size_t)idx : 0;   // (unconditional loads)
            ya[u] = g[e];
            yb[u] = g[e + 1];
            lo[u] = on ? (kNQ / 2 * cur.r + cur.m) * ls : -1;
            kk[u] = cur.k;
            cur.step();
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (lo[u] < 0) continue;
            C2<T> *line = r2 + lo[u];
            const int k = kk[u];
            const C2<T> a = ya[u], b = yb[u];
            line[k] = mk<T>(a.x - b.y, a.y + b.x);
            if (k != 0 && 2 * k != N3) line[N3 - k] = mk<T>(a.x + b.y, -a.y + b.x);   // conj(a) + i conj(b)
        }
    }
}

// C2R of the 20 u_a rows; v_loc = sum_a u_a dtheta_a/dn + de/dn;
// w = g grad n with g = sum_a u_a 2 n p'_a Q dq/dsigma + de/dsigma-part,
// stored in place of grad n as its lattice components q_c (the divergence
// passes take them).  tile: a = first row, b = rows.
template <typename T, int LC, int V>
__global__ void __launch_bounds__(kThreads) k_x_assemble(const InstDev *insts, const Tile *tiles,
                                                         const Consts *cst, const void *twv) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile t = tiles[blockIdx.x];
    const InstDev &I = insts[t.inst];
    const int N3 = axis_len<LC>(I.n3), N3h = N3 / 2 + 1, row0 = t.a, B = t.b, ls = N3 + 1;
    const size_t N = (size_t)I.n1 * I.n2 * I.n3;
    C2<T> *r2 = reinterpret_cast<C2<T> *>(smem);              // 10 lines per row: u pairs
    C2<T> *tw = r2 + kNQ / 2 * B * ls;                       // twiddles in T
    T *qm = reinterpret_cast<T *>(tw + N3);
    T *Mm = qm + kNQ;
    T *invm = Mm + kNQ * kNQ;
    // n and grad n of this thread's first point, fetched first (used after the FFT)
    const int npt = B * N3;
    const size_t p0 = (size_t)row0 * N3;
    const gptr<const T> nin = gld(reinterpret_cast<const T *>(I.n) + p0);
    const gptr<const T> grad = gld(reinterpret_cast<const T *>(I.grad) + p0);
    // (unconditional loads, clamped to the tile: a load under a branch would
    // be waited for where the branch joins)
    const int i_first = min((int)threadIdx.x, npt - 1);
    const T n_f = nin[i_first], gx_f = grad[i_first], gy_f = grad[N + i_first], gz_f = grad[2 * N + i_first];
    u_lines_in<T>(r2, ls, reinterpret_cast<const C2<T> *>(I.spec) + (size_t)row0 * N3h * kNQ, B, N3, N3h);
    load_consts<T>(cst, qm, Mm, invm);
    load_twiddles<T>(tw, I.p3, reinterpret_cast<const C2<T> *>(twv));
    __syncthreads();
    fft_lc<T, 1, LC, V>(r2, I.p3, kNQ / 2 * B, 1, ls, tw);

    const double c_qc = cst->qc, c_iqc = cst->iqc, c_cs = cst->cs, c_nmin = cst->nmin;
    const int c_mc = cst->mc;
    const bool semilocal = I.semilocal != 0;
    const gptr<T> vloc = gst(reinterpret_cast<T *>(I.vloc) + p0);
    for (int idx = threadIdx.x; idx < npt; idx += kThreads) {
        const int rb = idx / N3, k = idx - rb * N3;
        const bool first = idx == (int)threadIdx.x;
        const T nv = first ? n_f : nin[idx];
        const T gx = first ? gx_f : grad[idx], gy = first ? gy_f : grad[N + idx], gz = first ? gz_f : grad[2 * N + idx];
        T vl = (T)0, gs = (T)0;
        if (nv >= (T)c_nmin) {
            LocalQ<T, true> lq;
            const T sigma = gx * gx + gy * gy + gz * gz;
            lq.eval(nv, sigma, c_qc, c_iqc, c_mc, invm);
            SplineW<T> sw;
            sw.locate(lq.q0, qm, kNQ);
            const T *u = reinterpret_cast<const T *>(r2 + (size_t)(kNQ / 2 * rb) * ls);
            const T cn = nv * lq.Q * lq.dqdn;
            // sum_a u_a p_a and sum_a u_a p_a' through S0 = sum_a u_a M[j][a], S1 = sum_a u_a M[j+1][a]
            const T *Mj = Mm + sw.j * kNQ;
            T S0 = (T)0, S1 = (T)0;
            // pair m = (u_2m, u_2m+1) as one 8- or 16-byte load (lanes on
            // consecutive k read consecutive LDS words)
            const C2<T> *uc = reinterpret_cast<const C2<T> *>(u) + k;
#pragma unroll
            for (int m = 0; m < kNQ / 2; ++m) {
                const C2<T> up = uc[m * ls];
                S0 += up.x * Mj[2 * m] + up.y * Mj[2 * m + 1];
                S1 += up.x * Mj[kNQ + 2 * m] + up.y * Mj[kNQ + 2 * m + 1];
            }
            const int j0 = sw.j, j1 = sw.j + 1;
            const T uj = u[2 * ((j0 >> 1) * ls + k) + (j0 & 1)], uj1 = u[2 * ((j1 >> 1) * ls + k) + (j1 & 1)];
            const T su = sw.A0 * uj + sw.A1 * uj1 + sw.C0 * S0 + sw.C1 * S1;
            const T sdu = sw.B0 * uj + sw.B1 * uj1 + sw.D0 * S0 + sw.D1 * S1;
            // dtheta_a/dn = p_a + n p'_a Q dq/dn ; dtheta_a/dgrad n = 2 n p'_a Q dq/dsigma grad n
            const T q0 = lq.q0, cs = (T)c_cs;
            const T iq = rcp<T>(q0), iq3 = iq * iq * iq, iq4 = iq3 * iq;
            vl = su + cn * sdu + (T)2 * cs * nv * iq3 - (T)3 * cs * nv * nv * iq4 * lq.Q * lq.dqdn;
            gs = (T)2 * lq.Q * lq.ndqds * sdu - (T)6 * cs * nv * iq4 * lq.Q * lq.ndqds;
            if (semilocal) {
                // the semilocal terms: de/dgrad n = 2 de/dsigma grad n
                Semilocal<T> sl;
                sl.eval(nv, sigma, lq);
                vl += sl.dn;
                gs += (T)2 * sl.ds;
            }
        }
        vloc[idx] = vl;
        // the lattice components q_c = sum_x W[c][x] w_x of w in place of
        // grad n (each point is read and written by its own thread)
        const double gsd = (double)gs;
        const double wx = gsd * (double)gx, wy = gsd * (double)gy, wz = gsd * (double)gz;
        const gptr<T> wout = gst(reinterpret_cast<T *>(I.grad) + p0);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            wout[c * N + idx] = (T)(I.fdW[c][0] * wx + I.fdW[c][1] * wy + I.fdW[c][2] * wz);
    }
}

// ---------------------------------------------------------------- finite-difference passes

// Central differences on the periodic grid in the working precision:
// d_c f_i = sum_s c_s (f_{i + s e_c} - f_{i - s e_c}), s = 1..M, along the grid
// (lattice) axis c; grad n = sum_c W[c] d_c n with W[c][x] = N_c b_c,x / (2 pi).
// Neighbour indices wrap once (M <= 4 <= every edge).  Tiles are runs of
// whole axis-3 lines: a = first row (i1 N2 + i2), b = rows.  Offsets are
// 32-bit (a grid and its three fields stay below 2^31 elements).

// offset of the neighbour s steps up (down) an axis of n points with element
// stride st from index i (one wrap at most)
__device__ __forceinline__ int fd_up(int i, int s, int n, int st) { return i + s < n ? s * st : (s - n) * st; }
__device__ __forceinline__ int fd_dn(int i, int s, int n, int st) { return i >= s ? -s * st : (n - s) * st; }

template <typename T, int M>
__device__ __forceinline__ T fd_diff(gptr<const T> f, int i, int n, int st, const T *c) {
    T acc = (T)0;
#pragma unroll
    for (int s = 1; s <= M; ++s) acc += c[s - 1] * (f[fd_up(i, s, n, st)] - f[fd_dn(i, s, n, st)]);
    return acc;
}

template <typename T, int M>
__device__ __forceinline__ void fd_grad_tile(const InstDev &I, int row0, int B) {
    const int N1 = I.n1, N2 = I.n2, N3 = I.n3;
    const int plane = N2 * N3, N = N1 * plane;
    const gptr<const T> n = gld(reinterpret_cast<const T *>(I.n));
    const gptr<T> g = gst(reinterpret_cast<T *>(I.grad));
    T c[M];
#pragma unroll
    for (int s = 0; s < M; ++s) c[s] = (T)I.fdc[s];
    T Wm[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int x = 0; x < 3; ++x) Wm[a][x] = (T)I.fdW[a][x];
    const int npt = B * N3;
    const int drow = kThreads / N3, dk = kThreads - drow * N3;
    int idx = threadIdx.x;
    if (idx >= npt) return;
    int rb = idx / N3, i3 = idx - rb * N3, row = row0 + rb;
    int i1 = row / N2, i2 = row - i1 * N2;
    for (; idx < npt; idx += kThreads) {
        const int p = row * N3 + i3;
        const gptr<const T> f = n + p;
        const T d1 = fd_diff<T, M>(f, i1, N1, plane, c);
        const T d2 = fd_diff<T, M>(f, i2, N2, N3, c);
        const T d3 = fd_diff<T, M>(f, i3, N3, 1, c);
#pragma unroll
        for (int a = 0; a < 3; ++a) g[a * N + p] = Wm[0][a] * d1 + Wm[1][a] * d2 + Wm[2][a] * d3;
        // next point: kThreads = drow N3 + dk further on
        i3 += dk;
        row += drow;
        i2 += drow;
        if (i3 >= N3) { i3 -= N3; ++row; ++i2; }
        while (i2 >= N2) { i2 -= N2; ++i1; }
    }
}

// v = v_loc - sum_c d_c q_c, q_c = sum_x W[c][x] w_x in the grad n buffer
// (Eq. (Vi): the sum over j of w_j . d(grad n_j)/dn_i is the transpose of the
// gradient operator applied to w, minus the same stencils since they are
// antisymmetric).
template <typename T, int M>
__device__ __forceinline__ void fd_div_tile(const InstDev &I, int row0, int B) {
    const int N1 = I.n1, N2 = I.n2, N3 = I.n3;
    const int plane = N2 * N3, N = N1 * plane;
    const gptr<const T> w = gld(reinterpret_cast<const T *>(I.grad));
    const gptr<const T> vloc = gld(reinterpret_cast<const T *>(I.vloc));
    const gptr<T> v = gst(reinterpret_cast<T *>(I.v));
    T c[M];
#pragma unroll
    for (int s = 0; s < M; ++s) c[s] = (T)I.fdc[s];
    const int npt = B * N3;
    const int drow = kThreads / N3, dk = kThreads - drow * N3;
    int idx = threadIdx.x;
    if (idx >= npt) return;
    int rb = idx / N3, i3 = idx - rb * N3, row = row0 + rb;
    int i1 = row / N2, i2 = row - i1 * N2;
    for (; idx < npt; idx += kThreads) {
        const int p = row * N3 + i3;
        const T d1 = fd_diff<T, M>(w + p, i1, N1, plane, c);
        const T d2 = fd_diff<T, M>(w + N + p, i2, N2, N3, c);
        const T d3 = fd_diff<T, M>(w + 2 * N + p, i3, N3, 1, c);
        v[p] = vloc[p] - (d1 + d2 + d3);
        i3 += dk;
        row += drow;
        i2 += drow;
        if (i3 >= N3) { i3 -= N3; ++row; ++i2; }
        while (i2 >= N2) { i2 -= N2; ++i1; }
    }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_fd_grad(const InstDev *insts, const Tile *tiles) {
    const Tile t = tiles[blockIdx.x];
    const InstDev &I = insts[t.inst];
    // (the grid's first pass: clear its bad-density flag before the theta pass)
    if (t.a == 0 && threadIdx.x == 0) gst(I.bad)[0] = 0;
    switch (I.fdm) {
        case 1: fd_grad_tile<T, 1>(I, t.a, t.b); break;
        case 2: fd_grad_tile<T, 2>(I, t.a, t.b); break;
        case 3: fd_grad_tile<T, 3>(I, t.a, t.b); break;
        case 4: fd_grad_tile<T, 4>(I, t.a, t.b); break;
        default: break;
    }
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_fd_div(const InstDev *insts, const Tile *tiles) {
    const Tile t = tiles[blockIdx.x];
    const InstDev &I = insts[t.inst];
    switch (I.fdm) {
        case 1: fd_div_tile<T, 1>(I, t.a, t.b); break;
        case 2: fd_div_tile<T, 2>(I, t.a, t.b); break;
        case 3: fd_div_tile<T, 3>(I, t.a, t.b); break;
        case 4: fd_div_tile<T, 4>(I, t.a, t.b); break;
        default: break;
    }
}

// ---------------------------------------------------------------- per-axis spectral derivatives

// The spectral gradient of Eq. (Vi) multiplies the transform of n by i G_x,
// G = sum_c m_c b_c with the Nyquist index m_c = N_c/2 taken as zero: a sum
// of one-axis multipliers, so grad n = sum_c W[c] d_c n exactly, with d_c n
// = F_c^-1[i (2 pi m_c / N_c) F_c n] the derivative along grid axis c alone
// (in grid-index units; W[c][x] = N_c b_c,x / (2 pi)) and F_c the 1-D DFT
// along that axis; the divergence of the gradient term of v is likewise
// sum_c d_c q_c with q_c = sum_x W[c][x] w_x.  One pass per axis: pairs of
// real lines as one complex line (the one-axis operator is real), forward
// DFT, i kappa_m (Nyquist zero; the inverse's 1/N folded in), inverse DFT.
// MODE 0 (gradient, FP64 lines): n -> d_c n; MODE 1 (divergence, lines in
// the working precision): q_c -> the potential, v = v_loc - sum_c d_c q_c.

// spectra of nl lines (length L, pitch ls) times i s 2 pi m / L^2
template <typename C>
__device__ __forceinline__ void deriv_multiply(C2<C> *buf, int nl, int L, int ls, double s) {
    const double k0 = 2.0 * 3.14159265358979323846 / ((double)L * (double)L) * s;
    for (int idx = threadIdx.x; idx < nl * L; idx += kThreads) {
        const int l = idx / L, m0 = idx - l * L;
        const int m = 2 * m0 == L ? 0 : (2 * m0 < L ? m0 : m0 - L);
        const C kap = (C)(k0 * (double)m);
        C2<C> &z = buf[l * ls + m0];
        z = mk<C>(-kap * z.y, kap * z.x);
    }
    __syncthreads();
}

// Axis 3 (rows, contiguous).  tile: a = first row (i1 N2 + i2), b = rows
// (even: rows 2p, 2p+1 form line p).  MODE 0: grad[2] = W[2][2] d_3 n
// (orthorhombic) or d_3 n (general cells: the axis-1 pass combines); the
// grid's first pass, it also clears the bad-density flag.  MODE 1: v =
// v_loc - d_3 q_3 (q_3 in grad[2]).
template <typename T, typename C, int LC, int V, int MODE>
__global__ void __launch_bounds__(kThreads) k_drow(const InstDev *insts, const Tile *tiles, const void *twv) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile t = tiles[blockIdx.x];
    const InstDev &I = insts[t.inst];
    const int N3 = axis_len<LC>(I.n3), row0 = t.a, B = t.b, np = B / 2, ls = N3 + 1;
    const size_t N = (size_t)I.n1 * I.n2 * I.n3;
    if (MODE == 0 && row0 == 0 && threadIdx.x == 0) gst(I.bad)[0] = 0;
    C2<C> *tw = reinterpret_cast<C2<C> *>(smem);
    C2<C> *buf = tw + N3;
    const T *f = MODE == 0 ? reinterpret_cast<const T *>(I.n) + (size_t)row0 * N3
                           : reinterpret_cast<const T *>(I.grad) + 2 * N + (size_t)row0 * N3;
    batched<4>(np * N3, [&](int idx) {
        const int pr = idx / N3, k = idx - pr * N3;
        return mk<C>((C)gld(f)[(2 * pr) * N3 + k], (C)gld(f)[(2 * pr + 1) * N3 + k]);
    }, [&](int idx, C2<C> z) {
        const int pr = idx / N3, k = idx - pr * N3;
        buf[pr * ls + k] = z;
    });
    load_twiddles<C>(tw, I.p3, reinterpret_cast<const C2<C> *>(twv));
    __syncthreads();
    fft_lc<C, -1, LC, V>(buf, I.p3, np, 1, ls, tw);
    deriv_multiply<C>(buf, np, N3, ls, (MODE == 0 && !I.general) ? I.fdW[2][2] : 1.0);
    fft_lc<C, 1, LC, V>(buf, I.p3, np, 1, ls, tw);
    const int npt = B * N3;
    if constexpr (MODE == 0) {
        const gptr<T> g = gst(reinterpret_cast<T *>(I.grad) + 2 * N + (size_t)row0 * N3);
        for (int idx = threadIdx.x; idx < npt; idx += kThreads) {
            const int rb = idx / N3, k = idx - rb * N3;
            const C2<C> z = buf[(rb >> 1) * ls + k];
            g[idx] = (T)((rb & 1) ? z.y : z.x);
        }
    } else {
        const gptr<const T> vl = gld(reinterpret_cast<const T *>(I.vloc) + (size_t)row0 * N3);
        const gptr<T> v = gst(reinterpret_cast<T *>(I.v) + (size_t)row0 * N3);
        batched<4>(npt, [&](int idx) { return vl[idx]; }, [&](int idx, T x) {
            const int rb = idx / N3, k = idx - rb * N3;
            const C2<C> z = buf[(rb >> 1) * ls + k];
            v[idx] = x - (T)((rb & 1) ? z.y : z.x);
        });
    }
}

// Axes 2 (AX = 2: lines along i2, element stride N3) and 1 (AX = 1: along
// i1, stride N2 N3).  tile: a = the other outer index (i1, or i2), b = first
// i3, c = number W of consecutive i3 (pairs form one complex line; an odd
// W's last line has a zero imaginary part).  MODE 0, AX = 2: grad[1] =
// W[1][1] d_2 n (orthorhombic) or d_2 n (general).  MODE 0, AX = 1 (the last
// gradient pass): grad[0] = W[0][0] d_1 n (orthorhombic); general cells: grad n
// = sum_c W[c] d_c n from d_1 n and the stored d_2 n, d_3 n, all three
// Cartesian components written.  MODE 1: v -= d_c q_c (q_c in grad[AX-1]).
template <typename T, typename C, int LC, int V, int MODE, int AX>
__global__ void __launch_bounds__(kThreads) k_dcol(const InstDev *insts, const Tile *tiles, const void *twv) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile t = tiles[blockIdx.x];
    const InstDev &I = insts[t.inst];
    constexpr int c = AX - 1;                                  // lattice axis (0-based)
    const int L = axis_len<LC>(AX == 2 ? I.n2 : I.n1), lp = L | 1, Wc = t.c, np = (Wc + 1) / 2;
    const size_t N = (size_t)I.n1 * I.n2 * I.n3;
    const int stride = AX == 2 ? I.n3 : I.n2 * I.n3;           // (32-bit offsets: 3 N < 2^31)
    const size_t base = (AX == 2 ? (size_t)t.a * I.n2 * I.n3 : (size_t)t.a * I.n3) + t.b;
    C2<C> *tw = reinterpret_cast<C2<C> *>(smem);
    C2<C> *buf = tw + L;
    C *bc = reinterpret_cast<C *>(buf);                        // (re, im) of element e of line j / 2 at 2 ((j/2) lp + e) + j % 2
    const gptr<const T> f = gld(MODE == 0 ? reinterpret_cast<const T *>(I.n) + base
                                          : reinterpret_cast<const T *>(I.grad) + c * N + base);
    // element e of tile column j at f[e stride + j], flat index e Wc + j
    // (positions advanced without divisions: Wc is a runtime width); eight
    // unconditional loads in flight per lane
    const int total = L * Wc;
    {
        RowCursor cur(threadIdx.x, Wc);
        for (int base = threadIdx.x; base < total; base += 8 * kThreads) {
            C r[8];
            int o[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool on = base + u * kThreads < total;
                r[u] = (C)f[on ? cur.l * stride + cur.w : 0];
                o[u] = on ? 2 * ((cur.w >> 1) * lp + cur.l) + (cur.w & 1) : -1;
                cur.step();
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (o[u] >= 0) bc[o[u]] = r[u];
        }
    }
    if (Wc & 1)
        for (int e = threadIdx.x; e < L; e += kThreads) bc[2 * ((np - 1) * lp + e) + 1] = (C)0;
    load_twiddles<C>(tw, AX == 2 ? I.p2 : I.p1, reinterpret_cast<const C2<C> *>(twv));
    __syncthreads();
    fft_lc<C, -1, LC, V>(buf, AX == 2 ? I.p2 : I.p1, np, 1, lp, tw);
    deriv_multiply<C>(buf, np, L, lp, (MODE == 0 && !I.general) ? I.fdW[c][c] : 1.0);
    fft_lc<C, 1, LC, V>(buf, AX == 2 ? I.p2 : I.p1, np, 1, lp, tw);
    T *gbase = reinterpret_cast<T *>(I.grad) + base;
    if constexpr (MODE == 0) {
        const bool combine = AX == 1 && I.general;
        RowCursor cur(threadIdx.x, Wc);
        for (int idx = threadIdx.x; idx < total; idx += kThreads, cur.step()) {
            const int e = cur.l, j = cur.w;
            const size_t o = (size_t)e * stride + j;
            const C d = bc[2 * ((j >> 1) * lp + e) + (j & 1)];
            if (!combine) {
                gst(gbase)[c * N + o] = (T)d;
            } else {
                const double d1 = (double)d, d2 = (double)gld(gbase)[N + o], d3 = (double)gld(gbase)[2 * N + o];
#pragma unroll
                for (int x = 0; x < 3; ++x)
                    gst(gbase)[x * N + o] = (T)(I.fdW[0][x] * d1 + I.fdW[1][x] * d2 + I.fdW[2][x] * d3);
            }
        }
    } else {
        const gptr<T> v = gst(reinterpret_cast<T *>(I.v) + base);
        RowCursor cur(threadIdx.x, Wc);
        for (int b0 = threadIdx.x; b0 < total; b0 += 4 * kThreads) {
            T r[4];
            int go[4], lo[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool on = b0 + u * kThreads < total;
                go[u] = on ? cur.l * stride + cur.w : -1;
                lo[u] = 2 * ((cur.w >> 1) * lp + cur.l) + (cur.w & 1);
                r[u] = v[on ? go[u] : 0];
                cur.step();
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (go[u] >= 0) v[go[u]] = r[u] - (T)bc[lo[u]];
        }
    }
}

// ---------------------------------------------------------------- axis-2 pass

// The 20 spectra along axis 2.  tile: a = i1, b = first flattened (k3,
// component) index, c = width
template <typename T, int S, int LC, int V>
__global__ void __launch_bounds__(kThreads) k_y(const InstDev *insts, const Tile *tiles, const void *twv) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile t = tiles[blockIdx.x];
    const InstDev &I = insts[t.inst];
    const int N2 = axis_len<LC>(I.n2), W = t.c, lp = N2 | 1;   // lines contiguous, odd pitch
    C2<T> *tw = reinterpret_cast<C2<T> *>(smem);
    C2<T> *buf = tw + N2;
    const size_t rowlen = (size_t)I.n3h * kNQ;
    C2<T> *g = reinterpret_cast<C2<T> *>(I.spec) + (size_t)t.a * N2 * rowlen + t.b;
    rows_in_t(buf, lp, g, rowlen, N2, W);
    load_twiddles<T>(tw, I.p2, reinterpret_cast<const C2<T> *>(twv));
    __syncthreads();
    fft_lc<T, S, LC, V>(buf, I.p2, W, 1, lp, tw);
    rows_out_t(g, rowlen, buf, lp, N2, W);
}

// ---------------------------------------------------------------- axis-1 passes

// Forward axis-1 FFT of the 20 theta spectra, u_a(G) = sum_b phi_ab(|G|) c_b(G)
// with c = Theta / N (Eq. Eoffk, Eq. epsofk), the energy sum
// sum_G w_G sum_a Re(c_a^* u_a), inverse axis-1 FFT.
// tile: a = first entry in the column list, b = number of column pairs P,
// c = columns per pair (2: k2 and N2 - k2, which meet the same |G| shell at
// every (|m1|, k3); 1: k2 = 0 or N2/2).  Pair i has k3 = k3_0 + i; the list
// holds the columns pair by pair.
//
// Contraction layout: lanes form groups of kNQ (three per wave).  A group
// takes one item, a |m1| and a pair; lane a loads row a of that shell's
// kernel matrix (kNQ contiguous values, 16-byte loads) into registers and
// forms u_a at the pair's points (+-m1 of each column).  The rows of the
// group's next item are loaded meanwhile (two register sets in turn).
// GEN (grids in non-orthogonal cells): every item is one k point with its
// own shell; lane a loads row a of its full matrix, or (PK: the launch's
// tables hold packed upper triangles) gathers the row from it through
// offsets fixed per lane.
// PROBE (parity probes of the stages, never in an evaluation): 1 writes the
// forward spectra c = FFT(theta)/N back in place of the tile (no contraction,
// no inverse); 2 writes u = phi c (no inverse); 0 is the evaluation.
// MF (FP32, orthorhombic cells): the contraction on the matrix cores (see the
// item loop below) instead of the vector ALU; the same items, the same
// results up to the order of the FP32 additions.
template <typename T, int LC, int V, bool GEN, int PROBE, bool MF, bool PK>
__global__ void __launch_bounds__(kThreads) k_z_main(const InstDev *insts, const Tile *tiles, const int2 *cols,
                                                     const void *twv) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int kGroups = (kThreads / 64) * (64 / kNQ);   // lane groups per workgroup
    constexpr int kEpc = 16 / (int)sizeof(C2<T>);             // complex values per 16-byte chunk
    const Tile t = tiles[blockIdx.x];
    const InstDev &I = insts[t.inst];
    const int N1 = axis_len<LC>(I.n1), N2 = I.n2, N3 = I.n3, N3h = I.n3h, P = t.b, CP = t.c, K = P * CP;
    const int W = K * kNQ, lp = N1 | 1;                      // W lines, contiguous, odd pitch
    const int cstride = kNQ * lp;                             // LDS elements per column
    __shared__ int colbase[kMaxCols];                         // offset of each column in a k1 plane
    C2<T> *twall = reinterpret_cast<C2<T> *>(smem);
    C2<T> *buf = twall + N1;
    int *sidx = reinterpret_cast<int *>(buf + W * lp);        // shell of every item
    {
        const int2 cw = cols[t.a + min((int)threadIdx.x, K - 1)];   // unconditional (clamped) load
        if ((int)threadIdx.x < K) colbase[threadIdx.x] = (cw.x * N3h + cw.y) * kNQ;
    }
    const int2 c0 = cols[t.a];
    __syncthreads();
    const size_t plane = (size_t)N2 * N3h * kNQ;
    C2<T> *spec = reinterpret_cast<C2<T> *>(I.spec);
    // 16-byte chunks (l, w, e): plane l, column w, chunk e of the column's 20
    // values.  Each thread keeps one chunk column (w, e) and steps through the
    // planes; the loads of U planes are issued before their LDS writes (U at
    // least the planes per lane where that is at most 12: one batch).
    constexpr int kCpc = kNQ / kEpc;                          // chunks per column
    auto io_batch = [&](bool in, int C, int rps, auto Uc) {
        constexpr int U = decltype(Uc)::value;
        const int r0 = threadIdx.x / C, c = threadIdx.x - r0 * C, w = c / kCpc, e = c - w * kCpc;
        C2<T> *lb = buf + (w * kNQ + e * kEpc) * lp;
        // this lane's chunk column; planes l = r0 + s rps, s = j U + u
        char *cb = reinterpret_cast<char *>(spec + colbase[w] + e * kEpc);
        const size_t plane_bytes = plane * sizeof(C2<T>);
        for (int l0 = r0; l0 < N1; l0 += U * rps) {
            T ra[U], rb[U], rc[U], rd[U];
            if (in) {
                // unconditional loads (a plane past N1 re-reads plane r0, valid here)
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int l = l0 + u * rps;
                    const char *src = cb + (size_t)(uint32_t)(l < N1 ? l : r0) * plane_bytes;
                    if constexpr (kEpc == 2) {
                        const float4 v = gld(reinterpret_cast<const float4 *>(src))[0];
                        ra[u] = v.x; rb[u] = v.y; rc[u] = v.z; rd[u] = v.w;
                    } else {
                        const C2<T> v = gld(reinterpret_cast<const C2<T> *>(src))[0];
                        ra[u] = v.x; rb[u] = v.y;
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int l = l0 + u * rps;
                if (l >= N1) continue;
                char *dst = cb + (size_t)(uint32_t)l * plane_bytes;
                if (in) {
                    lb[l] = mk<T>(ra[u], rb[u]);
                    if constexpr (kEpc == 2) lb[lp + l] = mk<T>(rc[u], rd[u]);
                } else if constexpr (kEpc == 2) {
                    const C2<T> p0 = lb[l], p1 = lb[lp + l];
                    gst(reinterpret_cast<float4 *>(dst))[0] = make_float4(p0.x, p0.y, p1.x, p1.y);
                } else {
                    gst(reinterpret_cast<C2<T> *>(dst))[0] = lb[l];
                }
            }
        }
    };
    auto io = [&](bool in) {
        const int C = K * kCpc;                               // chunks per plane
        if (C > kThreads) {                                   // (only tiny N1 with many columns)
            const int total = N1 * C;
            for (int i = threadIdx.x; i < total; i += kThreads) {
                const int l = i / C, c = i - l * C, w = c / kCpc, e = c - w * kCpc;
                C2<T> *lb = buf + (w * kNQ + e * kEpc) * lp + l;
                C2<T> *gb = spec + (size_t)l * plane + colbase[w] + e * kEpc;
#pragma unroll
                for (int q = 0; q < kEpc; ++q) {
                    if (in) lb[q * lp] = gld(gb)[q];
                    else gst(gb)[q] = lb[q * lp];
                }
            }
            return;
        }
        const int rps = kThreads / C;                         // planes per step
        if ((int)threadIdx.x >= rps * C) return;
        const int steps = (N1 + rps - 1) / rps;               // planes per lane
        if (steps > kUnroll && steps <= 12) io_batch(in, C, rps, std::integral_constant<int, 12>{});
        else io_batch(in, C, rps, std::integral_constant<int, kUnroll>{});
    };
    const T *tab = reinterpret_cast<const T *>(I.shelltab);
    // orthorhombic cell: item = |m1| P + pair, the +-m1 points share a shell;
    // general cell: item = k1 P + pair over the whole axis, a shell each
    constexpr bool general = GEN;
    const int k30 = c0.y;
    const int m2 = general ? c0.x : freq_abs(c0.x, N2);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / kNQ, al = lane - grp * kNQ;
    const bool lane_on = grp < 64 / kNQ;
    const int gid = wave * (64 / kNQ) + grp;
    const int nitems = (general ? N1 : N1 / 2 + 1) * P;
    // shell of every item, into LDS; the thread's first item is loaded
    // before the tile (unconditionally, index clamped), so that its latency
    // overlaps the tile's loads
    const gptr<const int> smap = gld(I.shellmap + (size_t)m2 * N3h + k30);
    const size_t smap_m1 = (size_t)(general ? N2 : I.h2) * N3h;
    auto smap_at = [&](int i) {
        const int m1 = i / P;
        return smap[m1 * smap_m1 + (i - m1 * P)];
    };
    const int sh_first = smap_at(min((int)threadIdx.x, nitems - 1));
    io(true);
    load_twiddles<T>(twall, I.p1, reinterpret_cast<const C2<T> *>(twv));
    if ((int)threadIdx.x < nitems) sidx[threadIdx.x] = sh_first;
    for (int i = threadIdx.x + kThreads; i < nitems; i += kThreads) sidx[i] = smap_at(i);
    // (packed rows: entry (r, q), r <= q, at r kNQ - r (r - 1)/2 + q - r)
    int poff[GEN && PK ? kNQ : 1];
    if constexpr (GEN && PK) {
#pragma unroll
        for (int b = 0; b < kNQ; ++b) {
            const int r = min(al, b), q = max(al, b);
            poff[b] = r * kNQ - ((r * (r - 1)) >> 1) + q - r;
        }
    }
    static_assert(!MF || (sizeof(T) == 4 && !GEN), "matrix-core contraction: FP32, orthorhombic cells");
    // the kernel-matrix row this lane holds: a of its group (vector ALU), or
    // 4 rb + (lane % 4) of its block (matrix cores, below)
    const int mf_blk = lane >> 2, mf_q = lane & 3;
    const bool mf_on = mf_blk < 15;
    const int mf_g = mf_on ? mf_blk / 5 : 2;
    const int mf_rb = mf_on ? mf_blk - (mf_blk / 5) * 5 : 0;
    const int row = MF ? 4 * mf_rb + mf_q : al;
    // row `row` of the shell matrix of an item (index clamped to the last
    // item: the loads stay unconditional)
    auto fetch = [&](int item, T *f) {
        const int sh = sidx[min(item, nitems - 1)];
        if constexpr (GEN && PK) {
            const gptr<const T> src = gld(tab + (size_t)sh * kTabPacked);
#pragma unroll
            for (int b = 0; b < kNQ; ++b) f[b] = src[poff[b]];
            return;
        }
        const gptr<const T> src = gld(tab + (size_t)sh * kTabRow + row * kNQ);
        if constexpr (sizeof(T) == 4) {
            const gptr<const float4> s4 = (gptr<const float4>)src;
#pragma unroll
            for (int q = 0; q < kNQ / 4; ++q) {
                const float4 v = s4[q];
                f[4 * q] = v.x; f[4 * q + 1] = v.y; f[4 * q + 2] = v.z; f[4 * q + 3] = v.w;
            }
        } else {
            const gptr<const double2> s2 = (gptr<const double2>)src;
#pragma unroll
            for (int q = 0; q < kNQ / 2; ++q) {
                const double2 v = s2[q];
                f[2 * q] = v.x; f[2 * q + 1] = v.y;
            }
        }
    };
    __syncthreads();
    // kernel rows in flight: one item (vector ALU) or round (matrix cores)
    // ahead, the first before the forward FFT
    T fa[kNQ], fb[kNQ];
    const int it0 = MF ? wave * (64 / kNQ) + mf_g : gid;
    if (PROBE != 1 && (MF || lane_on)) fetch(it0, fa);
    fft_lc<T, -1, LC, V>(buf, I.p1, W, 1, lp, twall);
    if constexpr (PROBE == 1) {
        const T inv_n = (T)I.inv_n;
        for (int i = threadIdx.x; i < W * lp; i += kThreads) buf[i] = cscale(buf[i], inv_n);
        __syncthreads();
        io(false);
        if (threadIdx.x == 0) I.part_ek[t.slot] = 0.0;
        return;
    }

    const T inv_n = (T)I.inv_n;
    const double wn = (double)inv_n * (double)inv_n;
    double e = 0.0;
    // item it = m1 P + pr, stepped by kGroups without divisions
    const int dm = kGroups / P, dr = kGroups - dm * P;
    int m1 = gid / P, pr = gid - m1 * P;
    // u at the points of the current item with the kernel row f; a group's
    // lanes share one wave, so reads of theta and writes of u need wave-level
    // ordering only
    auto process = [&](const T *f) {
        // the points +-m1 of each column of the item (lq = l for k1 = 0, the
        // Nyquist plane and general cells: the second point is the first
        // again, its energy masked and its u the same value written twice)
        const int l = m1;
        int lq = N1 - m1;
        const bool two = !(general || m1 == 0 || lq == m1);
        if (!two) lq = l;
        const T mask2 = two ? (T)1 : (T)0;
        const int w0 = __mul24(pr, CP);
        const int k3 = k30 + pr;                               // the item's columns share k3
        const bool edge = (k3 == 0) || ((N3 & 1) == 0 && 2 * k3 == N3);
        const double wgt = edge ? wn : 2.0 * wn;
        m1 += dm;
        pr += dr;
        if (pr >= P) { pr -= P; ++m1; }
        auto column = [&](int w) {
            C2<T> u1 = mk<T>((T)0, (T)0), u2 = u1;
            C2<T> *xc = buf + __mul24(w, cstride);
            C2<T> *x1 = xc + l;                                   // component b at x1[b lp]
            C2<T> *x2 = xc + lq;
#pragma unroll
            for (int b = 0; b < kNQ; ++b) {
                const C2<T> t1 = x1[b * lp], t2 = x2[b * lp];
                u1.x += f[b] * t1.x;
                u1.y += f[b] * t1.y;
                u2.x += f[b] * t2.x;
                u2.y += f[b] * t2.y;
            }
            const C2<T> own1 = x1[al * lp], own2 = x2[al * lp];
            e += wgt * (double)(own1.x * u1.x + own1.y * u1.y + mask2 * (own2.x * u2.x + own2.y * u2.y));
            // every lane of the group has read theta at these points before
            // any lane overwrites its component with u; the next column or
            // item reads other points (each k point belongs to one item), so
            // no ordering is needed after the writes
            wave_sync();
            x1[al * lp] = cscale(u1, inv_n);
            x2[al * lp] = cscale(u2, inv_n);
        };
        column(w0);
        if (CP == 2) column(w0 + 1);
    };
    if constexpr (MF) {
        // Matrix cores: v_mfma_f32_4x4x1_16b_f32 forms 16 independent 4 x 4
        // outer products per instruction (A 4 x 1 and B 1 x 4 per block,
        // accumulated over K).  A wave takes the three items its three lane
        // groups take on the vector path.  Block k = lane / 4 (15 of the 16
        // in use): item g = k / 5 of the three, rows 4 rb .. 4 rb + 3 of its
        // kernel matrix (rb = k % 5).  Lane 4 k + i feeds A = row 4 rb + i of
        // the matrix (20 values in registers, one per K step b) and B =
        // column i of the item's four real columns: theta_b at point i / 2
        // (+m1 or -m1) and part i % 2 (re, im); it receives in its four
        // accumulators u_{4 rb + r} at that point and part, r = 0..3.  Items
        // of a column pair (two columns sharing every shell) instead use
        // B column i = theta_b at column i % 2 and point i / 2, both parts
        // from one 8-byte LDS read, in two chains (real and imaginary parts:
        // the kernel is real); the accumulators hold u_{4 rb + r} at that
        // column and point.  The lanes of a wave read theta before any of
        // them writes u (wave-level ordering), as on the vector path.
        typedef float v4f __attribute__((ext_vector_type(4)));
        const int g0 = wave * (64 / kNQ);
        int it = g0 + mf_g;
        int mg = it / P, pg = it - mg * P;
        const float fin = (float)I.inv_n;
        auto process_mf = [&](const T *f) {
            const bool valid = mf_on && it < nitems;
            const int l = valid ? mg : 0;                 // (an item past the end reads point 0)
            int lq = N1 - l;
            const bool two = !(l == 0 || lq == l);
            if (!two) lq = l;
            const int w0 = __mul24(pg, CP);
            const int k3 = k30 + pg;
            const bool edge = (k3 == 0) || ((N3 & 1) == 0 && 2 * k3 == N3);
            const double wgt = (valid && (mf_q < 2 || two)) ? (edge ? wn : 2.0 * wn) : 0.0;
            it += kGroups;
            mg += dm;
            pg += dr;
            if (pg >= P) { pg -= P; ++mg; }
            if (CP == 2) {
                // lane column: column mf_q % 2 of the pair, point +m1 (mf_q < 2) or -m1
                C2<T> *xc = buf + __mul24(w0 + (mf_q & 1), cstride) + (mf_q < 2 ? l : lq);
                C2<T> *oc = xc + 4 * mf_rb * lp;
                // every LDS read of the round before the first product (one
                // wait instead of one per K step)
                C2<T> th[kNQ], own[4];
#pragma unroll
                for (int b = 0; b < kNQ; ++b) th[b] = xc[b * lp];
#pragma unroll
                for (int r = 0; r < 4; ++r) own[r] = oc[r * lp];
                __builtin_amdgcn_sched_barrier(0);
                v4f are = {0.f, 0.f, 0.f, 0.f}, aim = are;
#pragma unroll
                for (int b = 0; b < kNQ; ++b) {
                    are = __builtin_amdgcn_mfma_f32_4x4x1f32(f[b], th[b].x, are, 0, 0, 0);
                    aim = __builtin_amdgcn_mfma_f32_4x4x1f32(f[b], th[b].y, aim, 0, 0, 0);
                }
                float es = 0.f;
#pragma unroll
                for (int r = 0; r < 4; ++r) es += own[r].x * are[r] + own[r].y * aim[r];
                e += wgt * (double)es;
                wave_sync();
                if (valid) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) oc[r * lp] = mk<T>(are[r] * fin, aim[r] * fin);
                }
            } else {
                const int pt = mf_q < 2 ? l : lq;
                float *x0 = reinterpret_cast<float *>(buf + __mul24(w0, cstride) + pt) + (mf_q & 1);
                float *o0 = x0 + 2 * 4 * mf_rb * lp;
                v4f a0 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int b = 0; b < kNQ; ++b) a0 = __builtin_amdgcn_mfma_f32_4x4x1f32(f[b], x0[2 * b * lp], a0, 0, 0, 0);
                e += wgt * (double)(o0[0] * a0[0] + o0[2 * lp] * a0[1] + o0[4 * lp] * a0[2] + o0[6 * lp] * a0[3]);
                wave_sync();
                if (valid) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) o0[2 * r * lp] = a0[r] * fin;
                }
            }
        };
        // rounds of three items per wave, the loop bound uniform over the wave
        for (int base = g0; base < nitems; base += 2 * kGroups) {
            fetch(it + kGroups, fb);               // the next round's row (clamped past the end)
            process_mf(fa);
            if (base + kGroups >= nitems) break;
            fetch(it + kGroups, fa);
            process_mf(fb);
        }
    } else {
        for (int it = gid; lane_on && it < nitems;) {
            fetch(it + kGroups, fb);               // the next item's row (clamped past the end)
            process(fa);
            it += kGroups;
            if (it >= nitems) break;
            fetch(it + kGroups, fa);
            process(fb);
            it += kGroups;
        }
    }
    __syncthreads();
    if constexpr (PROBE == 0) fft_lc<T, 1, LC, V>(buf, I.p1, W, 1, lp, twall);
    io(false);
    const double sum = block_sum(e);
    if (threadIdx.x == 0) I.part_ek[t.slot] = sum;
}

// ---------------------------------------------------------------- stage probes

// Parity probes (never part of an evaluation): the launches cover the tiles of
// a whole pass, and every workgroup whose tile belongs to another grid than
// `target` returns at once (uniformly).

// theta_a(r_i) = n_i p_a(q0_i) (the text after Eq. (Eoffk)) of the tile's
// points into dst [kNQ][N] (working precision), from n and the stored grad n,
// as the theta pass forms them.  tile: a = first row, b = rows.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_probe_theta(const InstDev *insts, const Tile *tiles,
                                                          const Consts *cst, void *dstv, int target) {
    __shared__ T qm[kNQ], Mm[kNQ * kNQ], invm[kMaxMc + 1];
    const Tile t = tiles[blockIdx.x];
    if (t.inst != target) return;
    const InstDev &I = insts[t.inst];
    load_consts<T>(cst, qm, Mm, invm);
    __syncthreads();
    const int N3 = I.n3;
    const size_t N = (size_t)I.n1 * I.n2 * I.n3, p0 = (size_t)t.a * N3;
    const T *nin = reinterpret_cast<const T *>(I.n) + p0;
    const T *gin = reinterpret_cast<const T *>(I.grad) + p0;
    T *dst = reinterpret_cast<T *>(dstv) + p0;
    for (int idx = threadIdx.x; idx < t.b * N3; idx += kThreads) {
        const T nv = nin[idx];
        T th[kNQ];
#pragma unroll
        for (int a = 0; a < kNQ; ++a) th[a] = (T)0;
        if (nv >= (T)cst->nmin) {
            const T gx = gin[idx], gy = gin[N + idx], gz = gin[2 * N + idx];
            LocalQ<T, false> lq;
            lq.eval(nv, gx * gx + gy * gy + gz * gz, cst->qc, cst->iqc, cst->mc, invm);
            SplineW<T> sw;
            sw.locate(lq.q0, qm, kNQ);
            const T *Mj = Mm + sw.j * kNQ;
#pragma unroll
            for (int a = 0; a < kNQ; ++a) {
                T v = nv * sw.C0 * Mj[a] + nv * sw.C1 * Mj[kNQ + a];
                if (a == sw.j) v += nv * sw.A0;
                if (a == sw.j + 1) v += nv * sw.A1;
                th[a] = v;
            }
        }
#pragma unroll
        for (int a = 0; a < kNQ; ++a) dst[a * N + idx] = th[a];
    }
}

// u_a(r_i) = sum_G u_a(G) exp(i G.r_i) (Eq. (epsilon)): the inverse axis-3
// transform of the u spectra, as the assembly pass forms it, into dst
// [kNQ][N] (working precision).  tile: a = first row, b = rows.
template <typename T, int LC, int V>
__global__ void __launch_bounds__(kThreads) k_probe_u(const InstDev *insts, const Tile *tiles, const void *twv,
                                                      void *dstv, int target) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile t = tiles[blockIdx.x];
    if (t.inst != target) return;
    const InstDev &I = insts[t.inst];
    const int N3 = axis_len<LC>(I.n3), N3h = N3 / 2 + 1, row0 = t.a, B = t.b, ls = N3 + 1;
    const size_t N = (size_t)I.n1 * I.n2 * I.n3;
    C2<T> *r2 = reinterpret_cast<C2<T> *>(smem);
    C2<T> *tw = r2 + kNQ / 2 * B * ls;
    u_lines_in<T>(r2, ls, reinterpret_cast<const C2<T> *>(I.spec) + (size_t)row0 * N3h * kNQ, B, N3, N3h);
    load_twiddles<T>(tw, I.p3, reinterpret_cast<const C2<T> *>(twv));
    __syncthreads();
    fft_lc<T, 1, LC, V>(r2, I.p3, kNQ / 2 * B, 1, ls, tw);
    T *dst = reinterpret_cast<T *>(dstv) + (size_t)row0 * N3;
    for (int idx = threadIdx.x; idx < (kNQ / 2) * B * N3; idx += kThreads) {
        const int m = idx / (B * N3), rest = idx - m * B * N3, rb = rest / N3, k = rest - rb * N3;
        const C2<T> z = r2[(kNQ / 2 * rb + m) * ls + k];
        dst[(size_t)(2 * m) * N + rest] = z.x;
        dst[(size_t)(2 * m + 1) * N + rest] = z.y;
    }
}

// ---------------------------------------------------------------- launchers

// The passes launch by family (the axis they transform): axis 3 (x), axis 2
// (y), axis 1 (z); each family's launcher is compiled in a translation unit
// of its own per precision (kernels_f32_x.hip ...), so the build runs them in
// parallel.  A launch with ntiles == 0 only raises the kernel's LDS limit
// (done once when the launches are planned, never while a stream is being
// captured).

// Kernels that take more than 64 KB of LDS opt in to the device's limit.
template <typename K>
static void allow_lds(K kernel, size_t bytes) {
    if (bytes > 65536) (void)hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

#define VDWNL_LAUNCH(kern, ...)                                                                      \
    do {                                                                                             \
        if (a.ntiles == 0) allow_lds(kern, a.lds);                                                   \
        else hipLaunchKernelGGL(kern, dim3(a.ntiles), dim3(kThreads), a.lds, a.stream, a.insts, a.tiles, \
                                __VA_ARGS__);                                                        \
    } while (0)

template <typename T, int LC, int V>
hipError_t launch_x_lc(int kind, const LaunchArgs &a) {
    switch (kind) {
        // (the gradient's one-axis transforms in FP64, the divergence's in T)
        case KG_X: VDWNL_LAUNCH((k_drow<T, double, LC, V, 0>), a.twd); break;
        case KD_X: VDWNL_LAUNCH((k_drow<T, T, LC, V, 1>), a.tw); break;
        case KX_THETA: VDWNL_LAUNCH((k_x_theta<T, LC, V>), a.cst, a.tw); break;
        case KX_ASSEMBLE: VDWNL_LAUNCH((k_x_assemble<T, LC, V>), a.cst, a.tw); break;
        case KP_U: VDWNL_LAUNCH((k_probe_u<T, LC, V>), a.tw, a.dst, a.target); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int LC, int V>
hipError_t launch_y_lc(int kind, const LaunchArgs &a) {
    switch (kind) {
        case KG_Y: VDWNL_LAUNCH((k_dcol<T, double, LC, V, 0, 2>), a.twd); break;
        case KD_Y: VDWNL_LAUNCH((k_dcol<T, T, LC, V, 1, 2>), a.tw); break;
        case KY_20F: VDWNL_LAUNCH((k_y<T, -1, LC, V>), a.tw); break;
        case KY_20I: VDWNL_LAUNCH((k_y<T, 1, LC, V>), a.tw); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int LC, int V>
hipError_t launch_z_lc(int kind, const LaunchArgs &a) {
    constexpr bool F32 = sizeof(T) == 4;
    switch (kind) {
        case KG_Z: VDWNL_LAUNCH((k_dcol<T, double, LC, V, 0, 1>), a.twd); break;
        case KD_Z: VDWNL_LAUNCH((k_dcol<T, T, LC, V, 1, 1>), a.tw); break;
        case KZ_MAIN:
            if (a.general && a.packed) VDWNL_LAUNCH((k_z_main<T, LC, V, true, 0, false, true>), a.cols, a.tw);
            else if (a.general) VDWNL_LAUNCH((k_z_main<T, LC, V, true, 0, false, false>), a.cols, a.tw);
            else if (F32 && a.mfma) VDWNL_LAUNCH((k_z_main<T, LC, V, false, 0, F32, false>), a.cols, a.tw);
            else VDWNL_LAUNCH((k_z_main<T, LC, V, false, 0, false, false>), a.cols, a.tw);
            break;
        case KP_THETA_K:
            // (the forward spectra alone: no kernel rows read)
            if (a.general) VDWNL_LAUNCH((k_z_main<T, LC, V, true, 1, false, false>), a.cols, a.tw);
            else VDWNL_LAUNCH((k_z_main<T, LC, V, false, 1, false, false>), a.cols, a.tw);
            break;
        case KP_U_K:
            if (a.general && a.packed) VDWNL_LAUNCH((k_z_main<T, LC, V, true, 2, false, true>), a.cols, a.tw);
            else if (a.general) VDWNL_LAUNCH((k_z_main<T, LC, V, true, 2, false, false>), a.cols, a.tw);
            else if (F32 && a.mfma) VDWNL_LAUNCH((k_z_main<T, LC, V, false, 2, F32, false>), a.cols, a.tw);
            else VDWNL_LAUNCH((k_z_main<T, LC, V, false, 2, false, false>), a.cols, a.tw);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#undef VDWNL_LAUNCH

// (length class, radix order) at run time -> the compiled instance; an order
// beyond the class's variants takes its last one
#define VDWNL_LC_VARIANTS(FN, T, kind, lc, var, a)                                                        \
    switch (lc) {                                                                                         \
        case 0: return FN<T, 0, 0>(kind, a);                                                              \
        case 1: return (var) >= 1 ? FN<T, 1, 1>(kind, a) : FN<T, 1, 0>(kind, a);                          \
        case 2: return (var) >= 1 ? FN<T, 2, 1>(kind, a) : FN<T, 2, 0>(kind, a);                          \
        case 3:                                                                                           \
            return (var) >= 3 ? FN<T, 3, 3>(kind, a)                                                      \
                   : (var) == 2 ? FN<T, 3, 2>(kind, a)                                                    \
                   : (var) == 1 ? FN<T, 3, 1>(kind, a) : FN<T, 3, 0>(kind, a);                            \
        case 4: return (var) >= 2 ? FN<T, 4, 2>(kind, a) : (var) == 1 ? FN<T, 4, 1>(kind, a) : FN<T, 4, 0>(kind, a); \
        case 5:                                                                                           \
            return (var) >= 5 ? FN<T, 5, 5>(kind, a)                                                      \
                   : (var) == 4 ? FN<T, 5, 4>(kind, a)                                                    \
                   : (var) == 3 ? FN<T, 5, 3>(kind, a)                                                    \
                   : (var) == 2 ? FN<T, 5, 2>(kind, a)                                                    \
                   : (var) == 1 ? FN<T, 5, 1>(kind, a) : FN<T, 5, 0>(kind, a);                            \
        case 6: return (var) >= 1 ? FN<T, 6, 1>(kind, a) : FN<T, 6, 0>(kind, a);                          \
        case 7: return (var) >= 1 ? FN<T, 7, 1>(kind, a) : FN<T, 7, 0>(kind, a);                          \
        default: return FN<T, kLenGeneric, 0>(kind, a);                                                   \
    }

}  // namespace vdwnl
