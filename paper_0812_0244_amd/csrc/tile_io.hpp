// Copies between global memory and LDS tiles.  Each thread issues a batch of
// U independent loads before it writes any of them to LDS, so a wave keeps
// U requests per lane in flight instead of waiting on each one; row/column
// indices advance incrementally (no integer division per element).  The
// loads of a batch are unconditional (a load under a branch, even a
// wave-uniform one, is waited for where the branch joins, so the batch would
// go out one load at a time): a step past the end of the tile re-reads the
// tile's first element and its value is dropped.
#pragma once

#include "fft_fast.hpp"

namespace vdwnl {

constexpr int kUnroll = 8;

// The kernels reach global memory through pointers held in memory (the
// per-grid descriptors), which the compiler would access with flat
// instructions; those also count as LDS operations, so every LDS wait would
// also wait for outstanding global loads.  These casts make the accesses
// global ones.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using gptr = __attribute__((address_space(1))) T *;
#else   // the host pass only parses device code
template <typename T>
using gptr = T *;
#endif
template <typename T>
__device__ __forceinline__ gptr<const T> gld(const T *p) { return (gptr<const T>)p; }
template <typename T>
__device__ __forceinline__ gptr<T> gst(T *p) { return (gptr<T>)p; }

// Position (row l, column w) of flat element index i in rows of W columns,
// advanced by kThreads per step.
struct RowCursor {
    int l, w, dl, dw, W;
    __device__ __forceinline__ RowCursor(int i, int W_) : W(W_) {
        l = i / W_;
        w = i - l * W_;
        dl = kThreads / W_;
        dw = kThreads - dl * W_;
    }
    __device__ __forceinline__ void step() {
        w += dw;
        l += dl;
        if (w >= W) { w -= W; ++l; }
    }
};

// Position (r, k, m) of flat index i = (r K + k) M + m, advanced by kThreads
// per step (k < K, m < M).
struct Cursor3 {
    int m, k, r, M, K, dm, dk, dr;
    __device__ __forceinline__ Cursor3(int i, int M_, int K_) : M(M_), K(K_) {
        const int rest = i / M_;
        m = i - rest * M_;
        r = rest / K_;
        k = rest - r * K_;
        const int q = kThreads / M_;
        dm = kThreads - q * M_;
        dr = q / K_;
        dk = q - dr * K_;
    }
    __device__ __forceinline__ void step() {
        m += dm;
        const int c = m >= M ? 1 : 0;
        m -= c * M;
        k += dk + c;
        r += dr;
        if (k >= K) { k -= K; ++r; }
    }
};

// lds[l * lstr + w] = g[l * gstr + w], l < nrows, w < W (E: float2 or double2).
template <typename E, int U = kUnroll>
__device__ __forceinline__ void rows_in(E *lds, int lstr, const E *__restrict__ g, size_t gstr, int nrows, int W) {
    using S = decltype(E{}.x);   // held as scalar components: arrays of vector
                                 // types would be placed in scratch memory
    const int total = nrows * W;
    RowCursor cur(threadIdx.x, W);
    for (int base = threadIdx.x; base < total; base += U * kThreads) {
        S rx[U], ry[U];
        int o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool on = base + u * kThreads < total;
            const E v = gld(g)[on ? (size_t)cur.l * gstr + cur.w : 0];
            rx[u] = v.x;
            ry[u] = v.y;
            o[u] = on ? cur.l * lstr + cur.w : -1;
            cur.step();
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (o[u] >= 0) lds[o[u]] = mk<S>(rx[u], ry[u]);
    }
}

// g[l * gstr + w] = lds[l * lstr + w].
template <typename E, int U = kUnroll>
__device__ __forceinline__ void rows_out(E *__restrict__ g, size_t gstr, const E *lds, int lstr, int nrows, int W) {
    const int total = nrows * W;
    RowCursor cur(threadIdx.x, W);
    for (int base = threadIdx.x; base < total; base += U * kThreads) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + u * kThreads < total) gst(g)[(size_t)cur.l * gstr + cur.w] = lds[cur.l * lstr + cur.w];
            cur.step();
        }
    }
}

// FP32 complex rows moved as 16-byte pairs when the row width, the global row
// stride and the global base allow it (W even, gstr even, g 16-byte aligned);
// LDS rows keep any stride (the pair is written as two 8-byte elements).
__device__ __forceinline__ bool pairable(const void *g, size_t gstr, int W) {
    return ((W | (int)(gstr & 1)) & 1) == 0 && (reinterpret_cast<uintptr_t>(g) & 15) == 0;
}

template <int U = kUnroll>
__device__ __forceinline__ void rows_in_c(float2 *lds, int lstr, const float2 *__restrict__ g, size_t gstr, int nrows,
                                          int W) {
    if (!pairable(g, gstr, W)) { rows_in<float2, U>(lds, lstr, g, gstr, nrows, W); return; }
    const int Wp = W / 2, total = nrows * Wp;
    const float4 *gp = reinterpret_cast<const float4 *>(g);
    const size_t gp_str = gstr / 2;
    RowCursor cur(threadIdx.x, Wp);
    for (int base = threadIdx.x; base < total; base += U * kThreads) {
        float4 r[U];
        int o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool on = base + u * kThreads < total;
            r[u] = gld(gp)[on ? (size_t)cur.l * gp_str + cur.w : 0];
            o[u] = on ? cur.l * lstr + 2 * cur.w : -1;
            cur.step();
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (o[u] >= 0) {
                lds[o[u]] = make_float2(r[u].x, r[u].y);
                lds[o[u] + 1] = make_float2(r[u].z, r[u].w);
            }
    }
}

template <int U = kUnroll>
__device__ __forceinline__ void rows_out_c(float2 *__restrict__ g, size_t gstr, const float2 *lds, int lstr, int nrows,
                                           int W) {
    if (!pairable(g, gstr, W)) { rows_out<float2, U>(g, gstr, lds, lstr, nrows, W); return; }
    const int Wp = W / 2, total = nrows * Wp;
    float4 *gp = reinterpret_cast<float4 *>(g);
    const size_t gp_str = gstr / 2;
    RowCursor cur(threadIdx.x, Wp);
    for (int base = threadIdx.x; base < total; base += U * kThreads) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + u * kThreads < total) {
                const float2 a = lds[cur.l * lstr + 2 * cur.w], b = lds[cur.l * lstr + 2 * cur.w + 1];
                gst(gp)[(size_t)cur.l * gp_str + cur.w] = make_float4(a.x, a.y, b.x, b.y);
            }
            cur.step();
        }
    }
}

// Transposed copies: global rows l < nrows of W contiguous elements go to
// LDS lines w < W with element l at lds[w * lpitch + l] (lines contiguous, for
// FFTs along l with unit element stride).
template <int U = kUnroll>
__device__ __forceinline__ void rows_in_t(float2 *lds, int lpitch, const float2 *__restrict__ g, size_t gstr,
                                          int nrows, int W) {
    if (!pairable(g, gstr, W)) {
        const int total = nrows * W;
        RowCursor cur(threadIdx.x, W);
        for (int base = threadIdx.x; base < total; base += U * kThreads) {
            float rx[U], ry[U];
            int o[U];
    #pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool on = base + u * kThreads < total;
                const float2 v = gld(g)[on ? (size_t)cur.l * gstr + cur.w : 0];
                rx[u] = v.x;
                ry[u] = v.y;
                o[u] = on ? cur.w * lpitch + cur.l : -1;
                cur.step();
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (o[u] >= 0) lds[o[u]] = make_float2(rx[u], ry[u]);
        }
        return;
    }
    const int Wp = W / 2, total = nrows * Wp;
    const float4 *gp = reinterpret_cast<const float4 *>(g);
    const size_t gp_str = gstr / 2;
    RowCursor cur(threadIdx.x, Wp);
    for (int base = threadIdx.x; base < total; base += U * kThreads) {
        float4 r[U];
        int o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool on = base + u * kThreads < total;
            r[u] = gld(gp)[on ? (size_t)cur.l * gp_str + cur.w : 0];
            o[u] = on ? 2 * cur.w * lpitch + cur.l : -1;
            cur.step();
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (o[u] >= 0) {
                lds[o[u]] = make_float2(r[u].x, r[u].y);
                lds[o[u] + lpitch] = make_float2(r[u].z, r[u].w);
            }
    }
}

template <int U = kUnroll>
__device__ __forceinline__ void rows_out_t(float2 *__restrict__ g, size_t gstr, const float2 *lds, int lpitch,
                                           int nrows, int W) {
    if (!pairable(g, gstr, W)) {
        const int total = nrows * W;
        RowCursor cur(threadIdx.x, W);
        for (int base = threadIdx.x; base < total; base += U * kThreads) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (base + u * kThreads < total) gst(g)[(size_t)cur.l * gstr + cur.w] = lds[cur.w * lpitch + cur.l];
                cur.step();
            }
        }
        return;
    }
    const int Wp = W / 2, total = nrows * Wp;
    float4 *gp = reinterpret_cast<float4 *>(g);
    const size_t gp_str = gstr / 2;
    RowCursor cur(threadIdx.x, Wp);
    for (int base = threadIdx.x; base < total; base += U * kThreads) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + u * kThreads < total) {
                const float2 a = lds[2 * cur.w * lpitch + cur.l], b = lds[(2 * cur.w + 1) * lpitch + cur.l];
                gst(gp)[(size_t)cur.l * gp_str + cur.w] = make_float4(a.x, a.y, b.x, b.y);
            }
            cur.step();
        }
    }
}

template <int U = kUnroll>
__device__ __forceinline__ void rows_in_t(double2 *lds, int lpitch, const double2 *__restrict__ g, size_t gstr,
                                          int nrows, int W) {
    const int total = nrows * W;
    RowCursor cur(threadIdx.x, W);
    for (int base = threadIdx.x; base < total; base += U * kThreads) {
        double rx[U], ry[U];
        int o[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool on = base + u * kThreads < total;
            const double2 v = gld(g)[on ? (size_t)cur.l * gstr + cur.w : 0];
            rx[u] = v.x;
            ry[u] = v.y;
            o[u] = on ? cur.w * lpitch + cur.l : -1;
            cur.step();
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (o[u] >= 0) lds[o[u]] = make_double2(rx[u], ry[u]);
    }
}

template <int U = kUnroll>
__device__ __forceinline__ void rows_out_t(double2 *__restrict__ g, size_t gstr, const double2 *lds, int lpitch,
                                           int nrows, int W) {
    const int total = nrows * W;
    RowCursor cur(threadIdx.x, W);
    for (int base = threadIdx.x; base < total; base += U * kThreads) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (base + u * kThreads < total) gst(g)[(size_t)cur.l * gstr + cur.w] = lds[cur.w * lpitch + cur.l];
            cur.step();
        }
    }
}

// Complex rows of either precision (FP64 complex is already 16 bytes).
__device__ __forceinline__ void crows_in(float2 *lds, int lstr, const float2 *g, size_t gstr, int nrows, int W) {
    rows_in_c(lds, lstr, g, gstr, nrows, W);
}
__device__ __forceinline__ void crows_in(double2 *lds, int lstr, const double2 *g, size_t gstr, int nrows, int W) {
    rows_in<double2>(lds, lstr, g, gstr, nrows, W);
}
__device__ __forceinline__ void crows_out(float2 *g, size_t gstr, const float2 *lds, int lstr, int nrows, int W) {
    rows_out_c(g, gstr, lds, lstr, nrows, W);
}
__device__ __forceinline__ void crows_out(double2 *g, size_t gstr, const double2 *lds, int lstr, int nrows, int W) {
    rows_out<double2>(g, gstr, lds, lstr, nrows, W);
}

// Generic batched loop: for i < total (i = threadIdx.x + k kThreads), the
// loads of U consecutive iterations (ld(i) -> value) are issued before any
// of their consumers (st(i, value)) run.  ld is called for every step, past
// the end with i = total - 1 (it must be a pure load).
template <int U, typename LD, typename ST>
__device__ __forceinline__ void batched(int total, LD ld, ST st) {
    using R = decltype(ld(0));
    for (int base = threadIdx.x; base < total; base += U * kThreads) {
        R r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = ld(min(base + u * kThreads, total - 1));
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (base + u * kThreads < total) st(base + u * kThreads, r[u]);
    }
}

// Length of the axis a pass transforms: a compile-time constant for the
// specialised length classes (so divisions by it are cheap), else runtime.
template <int LC>
__device__ __forceinline__ int axis_len(int n) {
    if constexpr (LC < kLenGeneric) return kFastLens[LC];
    else return n;
}

}  // namespace vdwnl
