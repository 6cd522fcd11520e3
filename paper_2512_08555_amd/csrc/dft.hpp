// In-register DFTs of compile-time length R (a product of 2, 3, 5 and 7),
// fully unrolled so that every index is a constant and every twiddle a
// literal.  Natural order in and out, unnormalised:
//   X[k] = sum_n x[n] exp(DIR 2 pi i n k / R),  DIR = -1 forward, +1 inverse.
//
// Mixed-radix decimation in time: R = r m, x_s[n'] = x[r n' + s],
//   X[k + m t] = sum_s exp(DIR 2 pi i s t / r) (exp(DIR 2 pi i s k / R) X_s[k]).
// Radix 4 is preferred, then 2, 3, 5, 7.  Odd radices use the symmetric
// real-coefficient form of the small DFT.
#pragma once
#include "cplx.hpp"

namespace ups {

template <int R>
constexpr int pick_radix() {
  if constexpr (R % 4 == 0) return 4;
  else if constexpr (R % 2 == 0) return 2;
  else if constexpr (R % 3 == 0) return 3;
  else if constexpr (R % 5 == 0) return 5;
  else if constexpr (R % 7 == 0) return 7;
  else return R;
}

template <int R>
constexpr bool is_smooth7() {
  int r = R;
  for (int p : {2, 3, 5, 7})
    while (r % p == 0) r /= p;
  return r == 1 && R >= 1;
}

// odd-length small DFT, r in {3, 5, 7}
template <int R, int DIR, typename T>
__device__ __forceinline__ void small_dft_odd(cx<T>* y) {
  constexpr int H = (R - 1) / 2;
  cx<T> sp[H + 1], sm[H + 1];
  static_for<1, H + 1>([&](auto ss) {
    constexpr int s = decltype(ss)::value;
    sp[s] = y[s] + y[R - s];
    sm[s] = y[s] - y[R - s];
  });
  cx<T> x0 = y[0];
  static_for<1, H + 1>([&](auto ss) { x0 = x0 + sp[decltype(ss)::value]; });
  cx<T> out[R];
  out[0] = x0;
  static_for<1, H + 1>([&](auto tt) {
    constexpr int t = decltype(tt)::value;
    cx<T> a = y[0], b = {T(0), T(0)};
    static_for<1, H + 1>([&](auto ss) {
      constexpr int s = decltype(ss)::value;
      constexpr cs_pair w = unit_root((long long)s * t, R);
      constexpr T c = T(w.c), sn = T(w.s);
      a = a + scale(sp[s], c);
      b = b + scale(sm[s], sn);
    });
    // X_t = a + DIR i b, X_{R-t} = a - DIR i b
    cx<T> ib = mul_i<DIR>(b);
    out[t] = a + ib;
    out[R - t] = a - ib;
  });
  static_for<0, R>([&](auto kk) { y[decltype(kk)::value] = out[decltype(kk)::value]; });
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void butterfly(cx<T>* y) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    cx<T> a = y[0], b = y[1];
    y[0] = a + b;
    y[1] = a - b;
  } else if constexpr (R == 4) {
    cx<T> a = y[0] + y[2], b = y[0] - y[2];
    cx<T> c = y[1] + y[3], e = mul_i<DIR>(y[1] - y[3]);
    y[0] = a + c;
    y[2] = a - c;
    y[1] = b + e;
    y[3] = b - e;
  } else {
    small_dft_odd<R, DIR>(y);
  }
}

// a = x + w z, b = x - w z for the constant w = exp(DIR 2 pi i E / R): by
// fused multiply-adds and b = 2 x - a when w is not trivial.
template <long long E, long long R, int DIR, typename T>
__device__ __forceinline__ void pm_pair(cx<T> x, cx<T> z, cx<T>& a, cx<T>& b) {
  if constexpr (twiddle_class<E, R>() < 2) {
    const cx<T> y = twiddle_c<E, R, DIR>(z);
    a = x + y;
    b = x - y;
  } else {
    a = cmadd_c<E, R, DIR>(x, z);
    b = cx<T>{fma_t(T(2), x.re, -a.re), fma_t(T(2), x.im, -a.im)};
  }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cx<T>* v) {
  static_assert(is_smooth7<R>(), "DFT length must be 7-smooth");
  if constexpr (R == 1 || R == 2 || R == 3 || R == 4 || R == 5 || R == 7) {
    butterfly<R, DIR>(v);
  } else {
    constexpr int r = pick_radix<R>();
    constexpr int m = R / r;
    cx<T> sub[r][m];
    static_for<0, r>([&](auto ss) {
      constexpr int s = decltype(ss)::value;
      static_for<0, m>([&](auto nn) {
        constexpr int n = decltype(nn)::value;
        sub[s][n] = v[r * n + s];
      });
      dft<m, DIR>(sub[s]);
    });
    static_for<0, m>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      if constexpr (r == 4) {
        // radix-4 combine; a pair x +- w x' whose w is not trivial is formed
        // as a = x + w x' by fused multiply-adds and b = 2 x - a
        const cx<T> x0 = sub[0][k];
        const cx<T> t1 = twiddle_c<(long long)k, R, DIR>(sub[1][k]);
        cx<T> a, b, c, d;
        pm_pair<(long long)2 * k, R, DIR>(x0, sub[2][k], a, b);
        pm_pair<(long long)3 * k, R, DIR>(t1, sub[3][k], c, d);
        const cx<T> e = mul_i<DIR>(d);
        v[k] = a + c;
        v[k + m] = b + e;
        v[k + 2 * m] = a - c;
        v[k + 3 * m] = b - e;
      } else if constexpr (r == 2) {
        cx<T> a, b;
        pm_pair<(long long)k, R, DIR>(sub[0][k], sub[1][k], a, b);
        v[k] = a;
        v[k + m] = b;
      } else {
        cx<T> y[r];
        static_for<0, r>([&](auto ss) {
          constexpr int s = decltype(ss)::value;
          y[s] = twiddle_c<(long long)s * k, R, DIR>(sub[s][k]);
        });
        butterfly<r, DIR>(y);
        static_for<0, r>([&](auto tt) {
          constexpr int t = decltype(tt)::value;
          v[k + m * t] = y[t];
        });
      }
    });
  }
}

// DFT of length R (even) whose upper half v[R/2 .. R) is zero.  Reads
// v[0 .. R/2), writes all R outputs in natural order.
//
// When R = 4 m with m even, the decimation in time of dft() keeps the zeros
// where they are: sub-DFT s takes x[4 n + s], which is zero exactly for
// n >= m/2, so every sub-DFT is again half-zero (a length-4 one with two
// zero inputs is four additions), followed by dft()'s radix-4 combine.
// Otherwise one decimation-in-frequency stage with a zero partner is a copy
// and a twiddle,
//   X[2j]   = DFT_{R/2}(x[n])[j],  X[2j+1] = DFT_{R/2}(x[n] w_R^n)[j].
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_half_in(cx<T>* v) {
  static_assert(R % 2 == 0, "half-zero input needs an even length");
  constexpr int H = R / 2;
  if constexpr (R == 2) {
    v[1] = v[0];
  } else if constexpr (R == 4) {
    const cx<T> y0 = v[0], y1 = v[1];
    const cx<T> e = mul_i<DIR>(y1);
    v[0] = y0 + y1;
    v[2] = y0 - y1;
    v[1] = y0 + e;
    v[3] = y0 - e;
  } else if constexpr (R % 8 == 0) {
    constexpr int m = R / 4;
    cx<T> sub[4][m];
    static_for<0, 4>([&](auto ss) {
      constexpr int s = decltype(ss)::value;
      static_for<0, m / 2>([&](auto nn) {
        constexpr int n = decltype(nn)::value;
        sub[s][n] = v[4 * n + s];
      });
      dft_half_in<m, DIR>(sub[s]);
    });
    static_for<0, m>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      const cx<T> x0 = sub[0][k];
      const cx<T> t1 = twiddle_c<(long long)k, R, DIR>(sub[1][k]);
      cx<T> a, b, c, d;
      pm_pair<(long long)2 * k, R, DIR>(x0, sub[2][k], a, b);
      pm_pair<(long long)3 * k, R, DIR>(t1, sub[3][k], c, d);
      const cx<T> e = mul_i<DIR>(d);
      v[k] = a + c;
      v[k + m] = b + e;
      v[k + 2 * m] = a - c;
      v[k + 3 * m] = b - e;
    });
  } else {
    cx<T> a[H], b[H];
    static_for<0, H>([&](auto nn) {
      constexpr int n = decltype(nn)::value;
      a[n] = v[n];
      b[n] = twiddle_c<n, R, DIR>(v[n]);
    });
    dft<H, DIR>(a);
    dft<H, DIR>(b);
    static_for<0, H>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      v[2 * j] = a[j];
      v[2 * j + 1] = b[j];
    });
  }
}

// DFT of length R (even) of which only outputs X[0 .. R/2) are needed:
// decimation in time, keeping the '+' half of the last combine.
// Writes v[0 .. R/2); v[R/2 .. R) is left unspecified.
template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_half_out(cx<T>* v) {
  static_assert(R % 2 == 0, "half output needs an even length");
  constexpr int H = R / 2;
  cx<T> e[H], o[H];
  static_for<0, H>([&](auto nn) {
    constexpr int n = decltype(nn)::value;
    e[n] = v[2 * n];
    o[n] = v[2 * n + 1];
  });
  dft<H, DIR>(e);
  dft<H, DIR>(o);
  static_for<0, H>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    v[k] = cmadd_c<k, R, DIR>(e[k], o[k]);
  });
}

}  // namespace ups
