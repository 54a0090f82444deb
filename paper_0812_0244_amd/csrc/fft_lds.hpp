// Batched complex FFTs of lines held in LDS: self-sorting (Stockham) radix
// 2/3/4/5/8 passes, one __syncthreads-bounded read/compute/write round per
// pass, 256 threads per workgroup.  Twiddles come from a per-length table
// W_L^m = exp(-2 pi i m / L) computed on the host in FP64.
#pragma once

#include "common.hpp"

namespace vdwnl {

template <typename T> struct CT;
template <> struct CT<float> { using type = float2; };
template <> struct CT<double> { using type = double2; };
template <typename T> using C2 = typename CT<T>::type;

template <typename T> __device__ __forceinline__ C2<T> mk(T x, T y) { C2<T> r; r.x = x; r.y = y; return r; }

// complex helpers, overloaded for float2 / double2 (s * i * z for s = +1 or -1 in crot)
#define VDWNL_CPLX_OPS(C, T)                                                                    \
    __device__ __forceinline__ C cadd(C a, C b) { return mk<T>(a.x + b.x, a.y + b.y); }          \
    __device__ __forceinline__ C csub(C a, C b) { return mk<T>(a.x - b.x, a.y - b.y); }          \
    __device__ __forceinline__ C cscale(C a, T s) { return mk<T>(a.x * s, a.y * s); }            \
    __device__ __forceinline__ C cmul(C a, C b) {                                                \
        return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);                              \
    }                                                                                            \
    __device__ __forceinline__ C cconj(C a) { return mk<T>(a.x, -a.y); }                         \
    __device__ __forceinline__ C crot(C z, T s) { return mk<T>(-s * z.y, s * z.x); }
VDWNL_CPLX_OPS(float2, float)
VDWNL_CPLX_OPS(double2, double)
#undef VDWNL_CPLX_OPS

// In-register DFT of R points, X_q = sum_r a_r exp(s 2 pi i r q / R).
template <typename T>
__device__ __forceinline__ void dft2(C2<T> *v) {
    C2<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T>
__device__ __forceinline__ void dft4(C2<T> &v0, C2<T> &v1, C2<T> &v2, C2<T> &v3, T s) {
    C2<T> t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = crot(csub(v1, v3), s);
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, t3);
    v3 = csub(t1, t3);
}

template <typename T>
__device__ __forceinline__ void dft3(C2<T> *v, T s) {
    const T h = (T)0.86602540378443864676;  // sqrt(3)/2
    C2<T> t1 = cadd(v[1], v[2]);
    C2<T> t2 = cscale(crot(csub(v[1], v[2]), s), h);
    C2<T> m = csub(v[0], cscale(t1, (T)0.5));
    v[0] = cadd(v[0], t1);
    v[1] = cadd(m, t2);
    v[2] = csub(m, t2);
}

template <typename T>
__device__ __forceinline__ void dft5(C2<T> *v, T s) {
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    C2<T> b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
    C2<T> d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    C2<T> A = cadd(v[0], cadd(cscale(b1, c1), cscale(b2, c2)));
    C2<T> B = cadd(v[0], cadd(cscale(b1, c2), cscale(b2, c1)));
    C2<T> P = crot(cadd(cscale(d1, s1), cscale(d2, s2)), s);
    C2<T> Q = crot(csub(cscale(d1, s2), cscale(d2, s1)), s);
    v[0] = cadd(v[0], cadd(b1, b2));
    v[1] = cadd(A, P);
    v[4] = csub(A, P);
    v[2] = cadd(B, Q);
    v[3] = csub(B, Q);
}

template <typename T>
__device__ __forceinline__ void dft8(C2<T> *v, T s) {
    const T r = (T)0.70710678118654752440;
    C2<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    C2<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<T>(e0, e1, e2, e3, s);
    dft4<T>(o0, o1, o2, o3, s);
    o1 = mk<T>((o1.x - s * o1.y) * r, (o1.y + s * o1.x) * r);   // * (1 + s i)/sqrt2
    o2 = crot(o2, s);                                            // * s i
    o3 = mk<T>((-o3.x - s * o3.y) * r, (s * o3.x - o3.y) * r);  // * (-1 + s i)/sqrt2
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

template <typename T, int R>
__device__ __forceinline__ void dft(C2<T> *v, T s) {
    if constexpr (R == 2) dft2<T>(v);
    else if constexpr (R == 3) dft3<T>(v, s);
    else if constexpr (R == 4) dft4<T>(v[0], v[1], v[2], v[3], s);
    else if constexpr (R == 5) dft5<T>(v, s);
    else dft8<T>(v, s);
}

// One Stockham pass of radix R over nl lines of length L.  Element e of line
// l lives at buf[l * ls + e * es].  Ns = product of the radices already done.
// Butterfly j of a line reads e = j + r L/R and writes
// e = (j - j%Ns) R + j%Ns + r Ns after the twiddle W_{Ns R}^{r (j%Ns)}.
template <typename T, int R>
__device__ __forceinline__ void fft_pass(C2<T> *buf, int L, int nl, int es, int ls, int Ns,
                                         const C2<T> *__restrict__ tw, T s) {
    constexpr int KMAX = (kTileCap / R + kThreads - 1) / kThreads;
    const int nj = L / R;
    const int nb = nl * nj;
    const int step = L / (Ns * R);
    C2<T> v[KMAX][R];
    int out[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int b = threadIdx.x + k * kThreads;
        if (b < nb) {
            int line, j;
            if (es == 1) { line = b / nj; j = b - line * nj; }
            else { j = b / nl; line = b - j * nl; }
            const C2<T> *src = buf + line * ls;
            const int kk = j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                C2<T> a = src[(j + r * nj) * es];
                if (r > 0 && kk > 0) {
                    C2<T> w = tw[r * kk * step];
                    w.y *= -s;  // table holds exp(-2 pi i m/L); s = -1 forward
                    a = cmul(a, w);
                }
                v[k][r] = a;
            }
            dft<T, R>(v[k], s);
            out[k] = line * ls + ((j - kk) * R + kk) * es;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int b = threadIdx.x + k * kThreads;
        if (b < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[out[k] + r * Ns * es] = v[k][r];
        }
    }
    __syncthreads();
}

// Copy the twiddles W_L^m, m < L, of plan p from the global table to LDS.
// The caller synchronises before the first fft_lines that reads them.
template <typename T>
__device__ __forceinline__ void load_twiddles(C2<T> *dst, const FftPlan &p, const C2<T> *__restrict__ twall) {
    // the first step's load is unconditional (clamped) and stored last, so it
    // is not waited for at a branch
    const int n = p.n;
    const C2<T> v0 = twall[p.tw + min((int)threadIdx.x, n - 1)];
    for (int i = threadIdx.x + kThreads; i < n; i += kThreads) dst[i] = twall[p.tw + i];
    if ((int)threadIdx.x < n) dst[threadIdx.x] = v0;
}

// Unnormalised DFT of every line: sign -1 forward, +1 inverse; tw holds
// W_L^m, m < L (in LDS).  The caller has synchronised after filling buf; on
// return buf is synchronised again.
template <typename T>
__device__ void fft_lines(C2<T> *buf, const FftPlan &p, int nl, int es, int ls,
                          const C2<T> *__restrict__ tw, int sign) {
    const T s = (T)sign;
    int Ns = 1;
    for (int st = 0; st < p.nstage; ++st) {
        const int R = p.radix[st];
        switch (R) {
            case 2: fft_pass<T, 2>(buf, p.n, nl, es, ls, Ns, tw, s); break;
            case 3: fft_pass<T, 3>(buf, p.n, nl, es, ls, Ns, tw, s); break;
            case 4: fft_pass<T, 4>(buf, p.n, nl, es, ls, Ns, tw, s); break;
            case 5: fft_pass<T, 5>(buf, p.n, nl, es, ls, Ns, tw, s); break;
            default: fft_pass<T, 8>(buf, p.n, nl, es, ls, Ns, tw, s); break;
        }
        Ns *= R;
    }
}

}  // namespace vdwnl
