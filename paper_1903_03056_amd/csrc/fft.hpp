// In-register mixed-radix (2/3/4) FFTs for gfx950, fully unrolled at compile time.
//
// A length-N transform lives in a thread's registers as cx<T> x[N].  All data
// movement inside the transform is register renaming; twiddle factors are
// compile-time constants computed in double precision by `twiddle` below (an exact
// octant reduction of 2 pi k / n followed by Taylor series on [0, pi/4]), then
// rounded to T.
//
// Sign convention: SIGN = -1 is the forward DFT  X_k = sum_n x_n e^{-2 pi i k n / N},
// SIGN = +1 the unnormalised inverse               x_n = sum_k X_k e^{+2 pi i k n / N}.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

namespace dgfs {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cmake(T a, T b) { return cx<T>{a, b}; }
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return {s * a.x, s * a.y}; }
// a += b * c
template <typename T>
__device__ __forceinline__ void cmac(cx<T>& a, cx<T> b, cx<T> c) {
    a.x = fma(b.x, c.x, fma(-b.y, c.y, a.x));
    a.y = fma(b.x, c.y, fma(b.y, c.x, a.y));
}

// ---------------------------------------------------------------- constexpr trig
namespace ct {
constexpr double kPi = 3.14159265358979323846264338327950288;

// Taylor series, |x| <= pi/4: 12 terms are below 1e-19.
constexpr double sin_small(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / double((2 * k) * (2 * k + 1));
        sum += term;
    }
    return sum;
}
constexpr double cos_small(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int k = 1; k < 14; ++k) {
        term *= -x2 / double((2 * k - 1) * (2 * k));
        sum += term;
    }
    return sum;
}

struct cd {
    double c, s;
};

// (cos, sin) of 2 pi k / n for integers k, n > 0.
constexpr cd twiddle(long k, long n) {
    long r = k % n;
    if (r < 0) r += n;
    // octant o = floor(8 r / n); angle inside the octant = 2 pi (8 r - o n) / (8 n)
    long o = (8 * r) / n;
    long rem = 8 * r - o * n;                       // in [0, n)
    double t = 2.0 * kPi * double(rem) / double(8 * n);  // in [0, pi/4)
    double c = cos_small(t), s = sin_small(t);
    // angle = o pi/4 + t
    switch (o) {
        case 0: return {c, s};
        case 1: {  // pi/4 + t = pi/2 - (pi/4 - t)
            double u = kPi / 4 - t;
            return {sin_small(u), cos_small(u)};
        }
        case 2: return {-s, c};
        case 3: {
            double u = kPi / 4 - t;  // 3pi/4 + t = pi - (pi/4 - t)
            return {-cos_small(u), sin_small(u)};
        }
        case 4: return {-c, -s};
        case 5: {
            double u = kPi / 4 - t;  // 5pi/4 + t = 3pi/2 - (pi/4 - t)
            return {-sin_small(u), -cos_small(u)};
        }
        case 6: return {s, -c};
        default: {
            double u = kPi / 4 - t;  // 7pi/4 + t = 2pi - (pi/4 - t)
            return {cos_small(u), -sin_small(u)};
        }
    }
}
}  // namespace ct

// Compile-time loop: f(std::integral_constant<int, I>{}) for I in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// x * e^{SIGN 2 pi i K / N} with the trivial cases folded.
template <int SIGN, long K, long N, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> x) {
    constexpr long r = ((K % N) + N) % N;
    if constexpr (r == 0) {
        return x;
    } else if constexpr (4 * r == N) {          // SIGN * i
        return SIGN > 0 ? cx<T>{-x.y, x.x} : cx<T>{x.y, -x.x};
    } else if constexpr (2 * r == N) {
        return cx<T>{-x.x, -x.y};
    } else if constexpr (4 * r == 3 * N) {      // -SIGN * i
        return SIGN > 0 ? cx<T>{x.y, -x.x} : cx<T>{-x.y, x.x};
    } else {
        constexpr ct::cd w = ct::twiddle(r, N);
        constexpr T c = T(w.c);
        constexpr T s = T(SIGN * w.s);
        return cx<T>{x.x * c - x.y * s, x.x * s + x.y * c};
    }
}

// Small DFTs on R values held in t[0..R-1], in place, natural order.
template <int SIGN, typename T>
__device__ __forceinline__ void dft2(cx<T>* t) {
    cx<T> a = t[0], b = t[1];
    t[0] = a + b;
    t[1] = a - b;
}

template <int SIGN, typename T>
__device__ __forceinline__ void dft4(cx<T>* t) {
    cx<T> a = t[0] + t[2], b = t[0] - t[2];
    cx<T> c = t[1] + t[3], d = t[1] - t[3];
    // d * (SIGN i)
    cx<T> e = SIGN > 0 ? cx<T>{-d.y, d.x} : cx<T>{d.y, -d.x};
    t[0] = a + c;
    t[2] = a - c;
    t[1] = b + e;
    t[3] = b - e;
}

template <int SIGN, typename T>
__device__ __forceinline__ void dft3(cx<T>* t) {
    constexpr T h = T(0.5);
    constexpr T r3 = T(SIGN * 0.86602540378443864676372317075293618);  // SIGN sqrt(3)/2
    cx<T> a = t[0], s = t[1] + t[2], d = t[1] - t[2];
    cx<T> m = cx<T>{a.x - h * s.x, a.y - h * s.y};
    cx<T> e = cx<T>{-r3 * d.y, r3 * d.x};  // (SIGN i sqrt3/2) d
    t[0] = a + s;
    t[1] = m + e;
    t[2] = m - e;
}

template <int N>
constexpr int first_radix() {
    return (N % 4 == 0 && N != 8) ? 4 : (N % 2 == 0 ? 2 : 3);
}

// In-place DFT of x[0..N-1] (decimation in time, natural-order output).
template <int N, int SIGN, typename T>
__device__ __forceinline__ void fft(cx<T>* x) {
    static_assert(N >= 1, "bad length");
    if constexpr (N == 1) {
        return;
    } else if constexpr (N == 2) {
        dft2<SIGN>(x);
    } else if constexpr (N == 3) {
        dft3<SIGN>(x);
    } else if constexpr (N == 4) {
        dft4<SIGN>(x);
    } else {
        constexpr int R = first_radix<N>();
        constexpr int Mlen = N / R;
        static_assert(R * Mlen == N, "N must factor into 2, 3, 4");
        cx<T> y[R][Mlen];
        static_for<0, R>([&](auto r) {
            static_for<0, Mlen>([&](auto m) { y[r][m] = x[R * m + r]; });
        });
        static_for<0, R>([&](auto r) { fft<Mlen, SIGN>(y[r]); });
        static_for<1, R>([&](auto r) {
            static_for<1, Mlen>([&](auto k1) {
                y[r][k1] = rot<SIGN, long(decltype(r)::value) * long(decltype(k1)::value), long(N)>(y[r][k1]);
            });
        });
        static_for<0, Mlen>([&](auto k1) {
            cx<T> t[R];
            static_for<0, R>([&](auto r) { t[r] = y[r][k1]; });
            if constexpr (R == 2) dft2<SIGN>(t);
            else if constexpr (R == 3) dft3<SIGN>(t);
            else dft4<SIGN>(t);
            static_for<0, R>([&](auto k2) { x[k1 + Mlen * k2] = t[k2]; });
        });
    }
}

}  // namespace dgfs
