// Complex arithmetic and compile-time roots of unity for the FFT kernels.
//
// Roots of unity w = exp(2 pi i e / R) are evaluated at compile time from an
// exact octant reduction of the rational angle e / R followed by Taylor
// series of cos and sin on [0, pi/4] (terms to x^27, error far below one
// double ulp), so every in-register butterfly uses literal constants and the
// multiples of pi/4 collapse to swaps and sign flips.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include <utility>

namespace ups {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * conj(b)
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
// multiply by +i (sgn > 0) or -i (sgn < 0)
template <int SGN, typename T>
__host__ __device__ __forceinline__ cx<T> mul_i(cx<T> a) {
  if constexpr (SGN > 0) return {-a.im, a.re};
  else return {a.im, -a.re};
}

// ---- compile-time trigonometry ---------------------------------------------
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double taylor_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int n = 1; n <= 14; ++n) {
    term *= -x2 / double((2 * n - 1) * (2 * n));
    sum += term;
  }
  return sum;
}
constexpr double taylor_sin(double x) {
  double x2 = x * x, term = x, sum = x;
  for (int n = 1; n <= 14; ++n) {
    term *= -x2 / double((2 * n) * (2 * n + 1));
    sum += term;
  }
  return sum;
}

struct cs_pair {
  double c, s;
};

// (cos, sin) of 2 pi num / den, exact reduction to an octant.
constexpr cs_pair unit_root(long long num, long long den) {
  num %= den;
  if (num < 0) num += den;
  const long long n8 = 8 * num;
  const int oct = int(n8 / den);
  const long long rem = n8 - (long long)oct * den;  // angle = (pi/4) (oct + rem/den)
  double c = 0, s = 0;
  if ((oct & 1) == 0) {
    const double phi = (kPi / 4.0) * double(rem) / double(den);
    const double cp = taylor_cos(phi), sp = taylor_sin(phi);
    switch (oct / 2) {  // theta = j pi/2 + phi
      case 0: c = cp; s = sp; break;
      case 1: c = -sp; s = cp; break;
      case 2: c = -cp; s = -sp; break;
      default: c = sp; s = -cp; break;
    }
  } else {
    const double phi = (kPi / 4.0) * double(den - rem) / double(den);
    const double cp = taylor_cos(phi), sp = taylor_sin(phi);
    switch ((oct + 1) / 2) {  // theta = j pi/2 - phi
      case 1: c = sp; s = cp; break;
      case 2: c = -cp; s = sp; break;
      case 3: c = -sp; s = -cp; break;
      default: c = cp; s = -sp; break;
    }
  }
  return {c, s};
}

// z * exp(DIR * 2 pi i E / R), DIR = -1 (forward) or +1 (inverse).
template <long long E, long long R, int DIR, typename T>
__device__ __forceinline__ cx<T> twiddle_c(cx<T> z) {
  constexpr long long e = ((E % R) + R) % R;
  if constexpr (e == 0) {
    return z;
  } else if constexpr ((8 * e) % R == 0) {
    constexpr int o = int((8 * e) / R);             // multiple of pi/4
    constexpr int od = DIR > 0 ? o : (8 - o) % 8;   // angle = od * pi/4
    constexpr T h = T(0.70710678118654752440084436210484903928);
    if constexpr (od == 2) return mul_i<+1>(z);
    else if constexpr (od == 4) return {-z.re, -z.im};
    else if constexpr (od == 6) return mul_i<-1>(z);
    else if constexpr (od == 1) return {(z.re - z.im) * h, (z.re + z.im) * h};
    else if constexpr (od == 3) return {(-z.re - z.im) * h, (z.re - z.im) * h};
    else if constexpr (od == 5) return {(z.im - z.re) * h, (-z.re - z.im) * h};
    else return {(z.re + z.im) * h, (z.im - z.re) * h};  // od == 7
  } else {
    constexpr cs_pair w = unit_root(DIR * e, R);
    constexpr T c = T(w.c), s = T(w.s);
    return {z.re * c - z.im * s, z.re * s + z.im * c};
  }
}

// Class of the constant exp(DIR 2 pi i E / R): 0 one, 1 a multiple of pi/2
// other than 0 (a swap and sign flips), 2 an odd multiple of pi/4, 3 general.
template <long long E, long long R>
constexpr int twiddle_class() {
  constexpr long long e = ((E % R) + R) % R;
  if constexpr (e == 0) return 0;
  else if constexpr ((4 * e) % R == 0) return 1;
  else if constexpr ((8 * e) % R == 0) return 2;
  else return 3;
}

template <typename T>
__device__ __forceinline__ T fma_t(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

// u + z exp(DIR 2 pi i E / R) with the product folded into fused
// multiply-adds: 4 operations for a general or pi/4-odd constant, instead
// of 4 (twiddle) + 2 (add).
template <long long E, long long R, int DIR, typename T>
__device__ __forceinline__ cx<T> cmadd_c(cx<T> u, cx<T> z) {
  constexpr int cls = twiddle_class<E, R>();
  if constexpr (cls < 2) {
    return u + twiddle_c<E, R, DIR>(z);
  } else if constexpr (cls == 2) {
    constexpr long long e = ((E % R) + R) % R;
    constexpr int o = int((8 * e) / R);
    constexpr int od = DIR > 0 ? o : (8 - o) % 8;  // angle = od * pi/4, od odd
    constexpr T h = T(0.70710678118654752440084436210484903928);
    if constexpr (od == 1) return {fma_t(h, z.re - z.im, u.re), fma_t(h, z.re + z.im, u.im)};
    else if constexpr (od == 3) return {fma_t(-h, z.re + z.im, u.re), fma_t(h, z.re - z.im, u.im)};
    else if constexpr (od == 5) return {fma_t(h, z.im - z.re, u.re), fma_t(-h, z.re + z.im, u.im)};
    else return {fma_t(h, z.re + z.im, u.re), fma_t(h, z.im - z.re, u.im)};
  } else {
    constexpr cs_pair w = unit_root(DIR * (((E % R) + R) % R), R);
    constexpr T c = T(w.c), sn = T(w.s);
    return {fma_t(c, z.re, fma_t(-sn, z.im, u.re)),
            fma_t(sn, z.re, fma_t(c, z.im, u.im))};
  }
}

// ---- compile-time loops -----------------------------------------------------
template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

}  // namespace ups
