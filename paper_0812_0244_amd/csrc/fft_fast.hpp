// Compile-time specialised FFTs of lines held in LDS for the transform lengths
// the workloads use.  A length L = R_1 R_2 ... is done as Stockham passes of
// radix R_i (up to 20); each line is owned by a group of TPL lanes inside one
// wave (TPL = gcd of L / R_i, so every lane has whole butterflies in every
// pass), so the passes are separated by wave-level ordering only.  The
// in-register DFTs of composite radix are Cooley-Tukey splits with
// compile-time twiddles.  Lengths without a specialisation use fft_lines.
#pragma once

#include <utility>

#include "fft_lds.hpp"

namespace vdwnl {

// ---------------------------------------------------------------- compile-time trigonometry

namespace ct {
constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double sin_poly(double x) {   // |x| <= pi/4
    double x2 = x * x, term = x, sum = x;
    for (int n = 1; n < 14; ++n) {
        term *= -x2 / ((2.0 * n) * (2.0 * n + 1.0));
        sum += term;
    }
    return sum;
}
constexpr double cos_poly(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int n = 1; n < 14; ++n) {
        term *= -x2 / ((2.0 * n - 1.0) * (2.0 * n));
        sum += term;
    }
    return sum;
}
// cos and sin of 2 pi m / n (m, n integers), exact to double rounding
constexpr double cos2pi(int m, int n) {
    m %= n;
    if (m < 0) m += n;
    // quadrant q with angle = q pi/2 + r, |r| <= pi/4
    const int q = (4 * m + n / 2) / n;                 // nearest multiple of n/4
    const double r = 2.0 * kPi * ((double)m / n - (double)q / 4.0);
    switch (q & 3) {
        case 0: return cos_poly(r);
        case 1: return -sin_poly(r);
        case 2: return -cos_poly(r);
        default: return sin_poly(r);
    }
}
constexpr double sin2pi(int m, int n) {
    m %= n;
    if (m < 0) m += n;
    const int q = (4 * m + n / 2) / n;
    const double r = 2.0 * kPi * ((double)m / n - (double)q / 4.0);
    switch (q & 3) {
        case 0: return sin_poly(r);
        case 1: return cos_poly(r);
        case 2: return -sin_poly(r);
        default: return -cos_poly(r);
    }
}
constexpr int gcd(int a, int b) { return b == 0 ? a : gcd(b, a % b); }
}  // namespace ct

// ---------------------------------------------------------------- in-register DFTs

// X_q = sum_r v_r exp(S 2 pi i r q / R), in place
template <typename T, int R, int S>
struct Dft {
    // R = P Q, P the first base radix dividing R
    static constexpr int P = (R % 4 == 0) ? 4 : (R % 2 == 0) ? 2 : (R % 5 == 0) ? 5 : 3;
    static constexpr int Q = R / P;
    __device__ __forceinline__ static void run(C2<T> *v) {
        C2<T> y[R];
#pragma unroll
        for (int n2 = 0; n2 < Q; ++n2) {
            C2<T> a[P];
#pragma unroll
            for (int n1 = 0; n1 < P; ++n1) a[n1] = v[Q * n1 + n2];
            Dft<T, P, S>::run(a);
#pragma unroll
            for (int k1 = 0; k1 < P; ++k1) {
                const int e = n2 * k1;
                if (e % R == 0) {
                    y[n2 * P + k1] = a[k1];
                } else {
                    const T c = (T)ct::cos2pi(e, R), s = (T)(S * ct::sin2pi(e, R));
                    y[n2 * P + k1] = mk<T>(a[k1].x * c - a[k1].y * s, a[k1].x * s + a[k1].y * c);
                }
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) {
            C2<T> b[Q];
#pragma unroll
            for (int n2 = 0; n2 < Q; ++n2) b[n2] = y[n2 * P + k1];
            Dft<T, Q, S>::run(b);
#pragma unroll
            for (int k2 = 0; k2 < Q; ++k2) v[k1 + P * k2] = b[k2];
        }
    }
};
template <typename T, int S> struct Dft<T, 1, S> { __device__ __forceinline__ static void run(C2<T> *) {} };
template <typename T, int S> struct Dft<T, 2, S> { __device__ __forceinline__ static void run(C2<T> *v) { dft2<T>(v); } };
template <typename T, int S> struct Dft<T, 3, S> { __device__ __forceinline__ static void run(C2<T> *v) { dft3<T>(v, (T)S); } };
template <typename T, int S> struct Dft<T, 4, S> {
    __device__ __forceinline__ static void run(C2<T> *v) { dft4<T>(v[0], v[1], v[2], v[3], (T)S); }
};
template <typename T, int S> struct Dft<T, 5, S> { __device__ __forceinline__ static void run(C2<T> *v) { dft5<T>(v, (T)S); } };
template <typename T, int S> struct Dft<T, 8, S> { __device__ __forceinline__ static void run(C2<T> *v) { dft8<T>(v, (T)S); } };

// ---------------------------------------------------------------- passes

// Order the wave's LDS accesses: every lane of a line's group is in one wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int L, int... RS>
struct FastPlan {
    static constexpr int gcd_all() {
        int g = 0;
        for (int r : {RS...}) g = ct::gcd(g, L / r);
        return g;
    }
    static constexpr int TPL = gcd_all();
};

// Twiddles a lane applies in the passes from the one after NS combined
// points on (the first pass, NS = 1, needs none): NB (R - 1) per pass.
template <int L, int TPL, int NS, int... RS>
struct TwCount {
    static constexpr int value = 0;
};
template <int L, int TPL, int NS, int R, int... RS>
struct TwCount<L, TPL, NS, R, RS...> {
    static constexpr int value = (NS > 1 ? (L / R / TPL) * (R - 1) : 0) + TwCount<L, TPL, NS * R, RS...>::value;
};

// The lane's twiddles of every pass, in pass order, (m, r) within a pass:
// W_{NS R}^{r (j % NS)} for butterfly j = t + m TPL, r = 1 .. R-1 (forward
// sign; the inverse conjugates them where they are applied).
template <typename T, int L, int TPL, int NS, int R, int... RS>
__device__ __forceinline__ void tw_gather(C2<T> *w, const C2<T> *__restrict__ tw, int t) {
    constexpr int NB = L / R / TPL;
    if constexpr (NS > 1) {
#pragma unroll
        for (int m = 0; m < NB; ++m) {
            const int kk = (t + m * TPL) % NS;
#pragma unroll
            for (int r = 1; r < R; ++r) w[m * (R - 1) + r - 1] = tw[r * kk * (L / (NS * R))];
        }
    }
    if constexpr (sizeof...(RS) > 0) tw_gather<T, L, TPL, NS * R, RS...>(w + (NS > 1 ? NB * (R - 1) : 0), tw, t);
}

// Element slots of the passes' intermediate results (between the first
// pass's reads and the last pass's writes, which keep the line in natural
// order) for the lengths 64 and 128: element e at e ^ ((e / 16) % 8), a
// permutation within aligned groups of 8.  The writes of the early passes
// go at stride R or in runs of NS < 16; the XOR moves the 16-element (128
// byte) blocks they share onto different LDS banks.
template <int L>
struct PassSwizzle {
    static constexpr bool on = (L == 64 || L == 128);
};
__device__ __forceinline__ int swizzle16(int e) { return e ^ ((e >> 4) & 7); }

// Pass of radix R after NS points have been combined; lane t of the group
// owns butterflies j = t + m TPL.  Reads e = j + r L/R, twiddles by
// W_{NS R}^{r (j % NS)}, writes e = (j - j%NS) R + j%NS + r NS (at their
// swizzled slots between passes).  The twiddles come from the lane's
// registers (wr, tw_gather's order) when REG, else from the LDS table.
template <typename T, int L, int S, int TPL, bool REG, int NS, int R, int... RS>
__device__ __forceinline__ void fast_passes(C2<T> *line, int es, const C2<T> *__restrict__ tw, const C2<T> *wr,
                                            int t) {
    constexpr int NB = L / R / TPL;
    constexpr bool SWZ_IN = PassSwizzle<L>::on && NS > 1;                 // not the first pass
    constexpr bool SWZ_OUT = PassSwizzle<L>::on && sizeof...(RS) > 0;     // not the last pass
    C2<T> v[NB][R];
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        const int j = t + m * TPL;
        const int kk = j % NS;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = j + r * (L / R);
            C2<T> a = line[(SWZ_IN ? swizzle16(e) : e) * es];
            if (NS > 1 && r > 0) {
                C2<T> w;
                if constexpr (REG) w = wr[m * (R - 1) + r - 1];
                else w = tw[r * kk * (L / (NS * R))];
                if (S > 0) w.y = -w.y;
                a = cmul(a, w);
            }
            v[m][r] = a;
        }
        Dft<T, R, S>::run(v[m]);
    }
    wave_sync();
#pragma unroll
    for (int m = 0; m < NB; ++m) {
        const int j = t + m * TPL;
        const int kk = j % NS;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = (j - kk) * R + kk + r * NS;
            line[(SWZ_OUT ? swizzle16(e) : e) * es] = v[m][r];
        }
    }
    wave_sync();
    if constexpr (sizeof...(RS) > 0)
        fast_passes<T, L, S, TPL, REG, NS * R, RS...>(line, es, tw, wr + (NS > 1 ? NB * (R - 1) : 0), t);
}

template <typename T, int S, int L, int... RS>
__device__ __forceinline__ void fft_fast(C2<T> *buf, int nl, int es, int ls, const C2<T> *__restrict__ tw) {
    constexpr int TPL = FastPlan<L, RS...>::TPL;
    static_assert(64 % TPL == 0, "a line's lanes must sit in one wave");
    constexpr int G = kThreads / TPL;
    const int grp = threadIdx.x / TPL, t = threadIdx.x - grp * TPL;
    // the lane's twiddles are the same for every line it transforms: read
    // once into registers when they take at most 64 VGPRs
    constexpr int NTW = TwCount<L, TPL, 1, RS...>::value;
    constexpr bool REG = NTW > 0 && NTW * (int)sizeof(C2<T>) <= 64 * 4;
    C2<T> wr[REG ? NTW : 1];
    if constexpr (REG) tw_gather<T, L, TPL, 1, RS...>(wr, tw, t);
    for (int l0 = 0; l0 < nl; l0 += G) {
        const int line = l0 + grp;
        if (line < nl) fast_passes<T, L, S, TPL, REG, 1, RS...>(buf + line * ls, es, tw, wr, t);
    }
    __syncthreads();
}

// Transform lengths with a specialised plan; a pass kernel is compiled once
// per length class (index into this list, or kLenGeneric for any other length).
constexpr int kFastLens[] = {24, 32, 48, 64, 96, 128, 160, 320};
constexpr int kNumLenClasses = 9;
constexpr int kLenGeneric = 8;

__host__ __device__ constexpr int len_class(int n) {
    for (int i = 0; i < kLenGeneric; ++i)
        if (kFastLens[i] == n) return i;
    return kLenGeneric;
}

// Radix orders of each length class, variant V (chosen per pass group by
// the autotuner): the passes' order and number change the LDS access
// strides, the LDS round trips and the twiddle pattern, not the result
// beyond rounding.  Lanes per line =
// gcd(L / R_i) (within one wave), elements per lane <= 20.  Entries end at
// the first zero; the last class (other lengths) uses the runtime plan.
constexpr int kMaxVariants = 6;
constexpr int kRadixOrders[kNumLenClasses][kMaxVariants][5] = {
    {{4, 3, 2}},                                          // 24: 2 lanes, 12 each
    {{8, 4}, {4, 8}},                                     // 32: 4 lanes, 8 each
    {{4, 4, 3}, {3, 4, 4}},                               // 48: 4 lanes, 12 each
    {{8, 8}, {4, 4, 4}, {16, 4}, {4, 16}},                // 64: 8 lanes, 8 each; 16 lanes, 4 each; 4 lanes, 16 each
    {{4, 4, 2, 3}, {2, 4, 4, 3}, {3, 4, 4, 2}},          // 96: 8 lanes, 12 each
    {{8, 4, 4}, {4, 4, 8}, {2, 8, 8}, {4, 8, 4},         // 128: 16 lanes, 8 each
     {16, 8}, {8, 16}},                                   //      8 lanes, 16 each (two passes)
    {{4, 4, 2, 5}, {5, 4, 4, 2}},                         // 160: 8 lanes, 20 each
    {{4, 4, 4, 5}, {5, 4, 4, 4}},                         // 320: 16 lanes, 20 each
    {},
};

__host__ __device__ constexpr int num_radices(int lc, int v) {
    int n = 0;
    while (n < 5 && kRadixOrders[lc][v][n] != 0) ++n;
    return n;
}

__host__ __device__ constexpr int num_variants(int lc) {
    int v = 0;
    while (v < kMaxVariants && num_radices(lc, v) > 0) ++v;
    return v;
}

constexpr int kNumVariants[kNumLenClasses] = {num_variants(0), num_variants(1), num_variants(2), num_variants(3),
                                              num_variants(4), num_variants(5), num_variants(6), num_variants(7),
                                              1};

template <typename T, int S, int LC, int V, int... I>
__device__ __forceinline__ void fft_ordered(C2<T> *buf, int nl, int es, int ls, const C2<T> *__restrict__ tw,
                                            std::integer_sequence<int, I...>) {
    fft_fast<T, S, kFastLens[LC], kRadixOrders[LC][V][I]...>(buf, nl, es, ls, tw);
}

// Unnormalised DFT (sign S) of nl lines of length p.n, for a length of class
// LC, radix order V.
template <typename T, int S, int LC, int V>
__device__ __forceinline__ void fft_lc(C2<T> *buf, const FftPlan &p, int nl, int es, int ls,
                                       const C2<T> *__restrict__ tw) {
    static_assert(V < kNumVariants[LC], "radix order out of range");
    if constexpr (LC == kLenGeneric) fft_lines<T>(buf, p, nl, es, ls, tw, S);
    else fft_ordered<T, S, LC, V>(buf, nl, es, ls, tw, std::make_integer_sequence<int, num_radices(LC, V)>{});
}

// The radix sequence of class lc, order v (host side), into r[]; its length.
inline int radix_order_of(int lc, int v, int *r) {
    const int n = num_radices(lc, v);
    for (int i = 0; i < n; ++i) r[i] = kRadixOrders[lc][v][i];
    return n;
}

}  // namespace vdwnl
