// In-register complex arithmetic and small DFT butterflies (radix 2, 4, 8, 16) for gfx950.
//
// dft<R, S>(x) replaces x[0..R-1] by X[k] = sum_n x[n] exp(S * 2 pi i n k / R), natural order,
// S = +1 (inverse sign) or -1 (forward sign).  Each radix is built from radix-4/2 stages with
// constant twiddles, so it costs only adds/subs plus a few constant multiplies.
#pragma once

#include <hip/hip_runtime.h>

namespace hs {

template <typename T> struct scalar_of;
template <> struct scalar_of<float2> { using type = float; };
template <> struct scalar_of<double2> { using type = double; };

template <typename T> __device__ __forceinline__ T cadd(T a, T b) { return T{a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ T csub(T a, T b) { return T{a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ T cmul(T a, T b) {
    return T{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ T cmulc(T a, T b) {
    return T{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T> __device__ __forceinline__ T cconj(T a) { return T{a.x, -a.y}; }
// a * (S i)
template <int S, typename T> __device__ __forceinline__ T mul_si(T a) {
    if constexpr (S > 0) return T{-a.y, a.x};
    else return T{a.y, -a.x};
}
// a * exp(S i theta) for a compile-time (c, s) = (cos theta, sin theta)
template <int S, typename T>
__device__ __forceinline__ T rot(T a, typename scalar_of<T>::type c, typename scalar_of<T>::type s) {
    return cmul(a, T{c, S > 0 ? s : -s});
}

template <int S, typename T> __device__ __forceinline__ void dft2(T *x) {
    T a = x[0];
    x[0] = cadd(a, x[1]);
    x[1] = csub(a, x[1]);
}

template <int S, typename T> __device__ __forceinline__ void dft4(T *x) {
    T t0 = cadd(x[0], x[2]);
    T t1 = csub(x[0], x[2]);
    T t2 = cadd(x[1], x[3]);
    T t3 = mul_si<S>(csub(x[1], x[3]));
    x[0] = cadd(t0, t2);
    x[1] = cadd(t1, t3);
    x[2] = csub(t0, t2);
    x[3] = csub(t1, t3);
}

template <int S, typename T> __device__ __forceinline__ void dft8(T *x) {
    using R = typename scalar_of<T>::type;
    const R h = R(0.70710678118654752440084436210485);
    // n = n1 + 2 n2 (n1 < 2, n2 < 4), k = k2 + 4 k1
    T a[4] = {x[0], x[2], x[4], x[6]};
    T b[4] = {x[1], x[3], x[5], x[7]};
    dft4<S>(a);
    dft4<S>(b);
    b[1] = rot<S>(b[1], h, h);            // W8^1
    b[2] = mul_si<S>(b[2]);               // W8^2
    b[3] = rot<S>(b[3], -h, h);           // W8^3
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[k] = cadd(a[k], b[k]);
        x[k + 4] = csub(a[k], b[k]);
    }
}

template <int S, typename T> __device__ __forceinline__ void dft16(T *x) {
    using R = typename scalar_of<T>::type;
    const R c1 = R(0.92387953251128675612818318939679);  // cos(pi/8)
    const R s1 = R(0.38268343236508977172845998403040);  // sin(pi/8)
    const R h = R(0.70710678118654752440084436210485);
    // n = n1 + 4 n2, k = k2 + 4 k1
    T y[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) y[n1][n2] = x[n1 + 4 * n2];
        dft4<S>(y[n1]);
    }
    // twiddles W16^(n1 k2)
    y[1][1] = rot<S>(y[1][1], c1, s1);
    y[1][2] = rot<S>(y[1][2], h, h);
    y[1][3] = rot<S>(y[1][3], s1, c1);
    y[2][1] = rot<S>(y[2][1], h, h);
    y[2][2] = mul_si<S>(y[2][2]);
    y[2][3] = rot<S>(y[2][3], -h, h);
    y[3][1] = rot<S>(y[3][1], s1, c1);
    y[3][2] = rot<S>(y[3][2], -h, h);
    y[3][3] = rot<S>(y[3][3], -c1, -s1);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
        T z[4] = {y[0][k2], y[1][k2], y[2][k2], y[3][k2]};
        dft4<S>(z);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) x[k2 + 4 * k1] = z[k1];
    }
}

template <int R, int S, typename T> __device__ __forceinline__ void dft(T *x) {
    if constexpr (R == 2) dft2<S>(x);
    else if constexpr (R == 4) dft4<S>(x);
    else if constexpr (R == 8) dft8<S>(x);
    else if constexpr (R == 16) dft16<S>(x);
    else static_assert(R == 2 || R == 4 || R == 8 || R == 16, "unsupported radix");
}

}  // namespace hs
