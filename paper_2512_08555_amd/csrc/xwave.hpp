// Pass 5 with one wavefront per row: complex-to-real untangle of the half
// spectrum X[0..L] (L = mx/2 = 64 E), inverse DFT of length L on the wave,
// keep x < nx.
//
//   Z[k] = (X[k] + conj X[L-k]) + i conj(w_2L^k) (X[k] - conj X[L-k]),  k < L,
//
// and the inverse DFT of Z gives u[2m] + i u[2m+1] (unnormalised).  Lane l,
// register r A + m2 loads k = l + 64 r + E^2 m2 straight from the row (both
// X[k] and X[L-k] are contiguous across the wave), which is the layout the
// inverse stages of the z pass take; those stages leave output pair
// m = l + 64 f (f < E/2) in register f, and only m < L/2 is kept (nx <= L).
// No tile staging and no barrier: the row is contiguous in W.  The "_m"
// variants load each X[k] once and take X[L-k] from the wave's LDS area.
//
// Pass 1 the same way: the real row packed as z[m] = f[2m] + i f[2m+1]
// (m < nx/2 <= L/2, the zero padding is the upper half), the forward stages
// of the z pass, then the untangle
//
//   X[k] = (Z[k] + conj Z[L-k])/2 - i w_2L^k (Z[k] - conj Z[L-k])/2,  k <= L
//
// with Z[L-k] read back from the wave's LDS area (the whole Z goes there).
#pragma once
#include "zwave.hpp"

namespace ups {

// LDS area of one wave in the inverse x pass: the exchanges, or (ML) the
// whole half spectrum X[0..L].
template <int E, bool ML>
constexpr int xwinv_slot() {
  constexpr int a = (ZWave<E>::xfloats + 1) / 2, b = 64 * E + 1;
  return ML && b > a ? b : a;
}

// ML: load each X[k] once and take the mirrored X[L-k] from the wave's LDS
// area, instead of loading it a second time from the row.
template <typename T, int E, int RW, bool ML>
__device__ __forceinline__ void xwinv_body(const cx<T>* __restrict__ W, T* __restrict__ u, const PassArgs& a,
                                           unsigned bx, unsigned by) {
  using Z = ZWave<E>;
  constexpr int L = Z::M, A = Z::A, E2 = Z::E2;
  constexpr int NR = 31 - __builtin_clz(E > A ? E : A);
  constexpr bool LT = zwave_lds_twiddles<E>();
  constexpr int XS = xwinv_slot<E, ML>();  // complex elements of one wave's LDS area
  __shared__ cx<T> xs[RW * XS];
  __shared__ cx<T> twl[LT ? NR * 64 : 1];
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_x);  // table of length 2L
  // w_L^(2^j x) = w_2L^(2^(j+1) x): row 2^(j+1) of the x table's product block
  auto trow = [&](int j, int x) { return LT ? twl[64 * j + x] : tw_row(tw, 2 * L, 2u << j)[x]; };
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  if constexpr (LT) {
    for (int i = t; i < NR * 64; i += 64 * RW) twl[i] = tw_row(tw, 2 * L, 2u << (i / 64))[i % 64];
    __syncthreads();
  }
  const long long row = (long long)bx * RW + wv;
  if (row >= (long long)a.ny * a.nz) return;  // no barrier below
  const int comp = int(by);
  const int y = int(row % a.ny), z = int(row / a.ny);
  const cx<T>* src = W + comp * a.comp_w + z * a.plane + (long long)y * a.px;
  T* dst = u + comp * a.comp_f + row * a.nx;
  T* xf = reinterpret_cast<T*>(xs + wv * XS);

  // untangle; conj w_2L^k = conj w_2L^lane * conj w_2L^base
  const cx<T> wl = tw_at(tw, unsigned(lane));
  cx<T> v[E];
  if constexpr (ML) {
    cx<T>* zs = reinterpret_cast<cx<T>*>(xf);
    static_for<0, E>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      v[i] = ld_cx<nt_load<kNtXinvWaveBit>()>(src + (lane + 64 * (i / A) + E2 * (i % A)));
    });
    cx<T> xl = zero_c<T>();
    if (a.nyq) {  // column 0 carries X[0] + i X[L], both real
      if (lane == 0) {
        xl = cx<T>{v[0].im, T(0)};
        v[0] = cx<T>{v[0].re, T(0)};
      }
    } else if (lane == 0) {
      xl = ld_cx<nt_load<kNtXinvWaveBit>()>(src + L);
    }
    wave_fence();
    static_for<0, E>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      zs[lane + 64 * (i / A) + E2 * (i % A)] = v[i];
    });
    if (lane == 0) zs[L] = xl;
    wave_fence();
    static_for<0, E>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      constexpr int base = 64 * (i / A) + E2 * (i % A);
      const cx<T> xk = v[i];
      const cx<T> xm = conj(zs[L - (lane + base)]);
      v[i] = (xk + xm) + mul_i<+1>(twiddle_c<base, 2 * L, +1>(cmulc(xk - xm, wl)));
    });
    wave_fence();
  } else {
    static_for<0, E>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      constexpr int base = 64 * (i / A) + E2 * (i % A);
      const int k = lane + base;  // k < L, so L - k is in 1 .. L
      cx<T> xk = ld_cx<nt_load<4>()>(src + k);
      cx<T> xm;
      if (a.nyq && k == 0) {  // column 0 carries X[0] + i X[L], both real
        xm = cx<T>{xk.im, T(0)};
        xk = cx<T>{xk.re, T(0)};
      } else {
        xm = conj(ld_cx<nt_load<4>()>(src + (L - k)));
      }
      v[i] = (xk + xm) + mul_i<+1>(twiddle_c<base, 2 * L, +1>(cmulc(xk - xm, wl)));
    });
  }
  zw_inverse<T, E, 0>(v, xf, lane, trow, static_cast<const cx<T>*>(nullptr));

  const int nx = a.nx;
  if (nx == L) {  // every pair m < L/2 is inside the row
    static_for<0, E / 2>([&](auto ff) {
      constexpr int f = decltype(ff)::value;
      st_cx<nt_store<kNtXinvWaveBit>()>(reinterpret_cast<cx<T>*>(dst + 2 * (lane + 64 * f)), v[f]);
    });
  } else {
    static_for<0, E / 2>([&](auto ff) {
      constexpr int f = decltype(ff)::value;
      const int m = lane + 64 * f;
      if (2 * m < nx) st_r<nt_store<kNtXinvWaveBit>()>(dst + 2 * m, v[f].re);
      if (2 * m + 1 < nx) st_r<nt_store<kNtXinvWaveBit>()>(dst + 2 * m + 1, v[f].im);
    });
  }
}

// LDS area of one wave in the forward x pass: the exchanges, or the whole
// spectrum Z (L complex) for the untangle.
template <int E>
constexpr int xwfwd_slot() {
  constexpr int a = (ZWave<E>::xfloats + 1) / 2, b = 64 * E;
  return a > b ? a : b;
}

// FILL: the x direction is even or odd (a.fill_x = +1 or -1, nx = L): the
// packed line's second half holds the mirror image, Z[m] = fill_x times the
// swapped pair of Z[L - 1 - m] (x[2 L - 1 - 2 m] + i x[2 L - 2 - 2 m]), loaded
// from the row again in reversed order, and the first stage is full.
template <typename T, int E, int RW, bool FILL = false>
__device__ __forceinline__ void xwfwd_body(const T* __restrict__ f, cx<T>* __restrict__ W, const PassArgs& a,
                                           unsigned bx, unsigned by) {
  using Z = ZWave<E>;
  constexpr int L = Z::M, A = Z::A, E2 = Z::E2;
  constexpr int NR = 31 - __builtin_clz(E > A ? E : A);
  constexpr bool LT = zwave_lds_twiddles<E>();
  constexpr int XS = xwfwd_slot<E>();
  __shared__ cx<T> xs[RW * XS];
  __shared__ cx<T> twl[LT ? NR * 64 : 1];
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_x);  // table of length 2L
  auto trow = [&](int j, int x) { return LT ? twl[64 * j + x] : tw_row(tw, 2 * L, 2u << j)[x]; };
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  if constexpr (LT) {
    for (int i = t; i < NR * 64; i += 64 * RW) twl[i] = tw_row(tw, 2 * L, 2u << (i / 64))[i % 64];
    __syncthreads();
  }
  const long long row = (long long)bx * RW + wv;
  if (row >= (long long)a.ny * a.nz) return;  // no barrier below
  const int comp = int(by);
  const int y = int(row % a.ny), z = int(row / a.ny);
  const T* src = f + comp * a.comp_f + row * a.nx;
  cx<T>* dst = W + comp * a.comp_w + z * a.plane + (long long)y * a.px;
  cx<T>* zs = xs + wv * XS;
  T* xf = reinterpret_cast<T*>(zs);

  // packed row: register j < E/2 takes m = lane + 64 j
  const int nx = a.nx;
  cx<T> v[E];
  if (nx == L) {
    static_for<0, E / 2>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      v[j] = ld_cx<nt_load<0>()>(reinterpret_cast<const cx<T>*>(src + 2 * (lane + 64 * j)));
    });
  } else {
    const bool even_nx = (nx & 1) == 0;
    static_for<0, E / 2>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      const int m = lane + 64 * j;
      cx<T> val = zero_c<T>();
      if (even_nx) {
        if (2 * m < nx) val = ld_cx<nt_load<0>()>(reinterpret_cast<const cx<T>*>(src + 2 * m));
      } else {
        if (2 * m < nx) val.re = ld_r<nt_load<0>()>(src + 2 * m);
        if (2 * m + 1 < nx) val.im = ld_r<nt_load<0>()>(src + 2 * m + 1);
      }
      v[j] = val;
    });
  }
  if constexpr (FILL) {
    // m = lane + 64 j (j >= E/2) mirrors m' = L - 1 - m = (63 - lane) + 64 (E - 1 - j)
    const T fs = T(a.fill_x);
    static_for<E / 2, E>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      const int mr = (63 - lane) + 64 * (E - 1 - j);
      const cx<T> p = ld_cx<nt_load<0>()>(reinterpret_cast<const cx<T>*>(src + 2 * mr));
      v[j] = cx<T>{fs * p.im, fs * p.re};
    });
  }
  zw_forward<T, E, 0, FILL>(v, xf, lane, trow, static_cast<const cx<T>*>(nullptr));
  // register i holds Z[k], k = lane + base(i); the whole Z into LDS at k
  wave_fence();
  static_for<0, E>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    zs[lane + 64 * (i / A) + E2 * (i % A)] = v[i];
  });
  wave_fence();
  const cx<T> wl = tw_at(tw, unsigned(lane));  // w_2L^lane
  static_for<0, E>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    constexpr int base = 64 * (i / A) + E2 * (i % A);
    const int k = lane + base;
    const cx<T> zk = v[i];
    const cx<T> zm = conj(zs[k == 0 ? 0 : L - k]);
    const cx<T> e = scale(zk + zm, T(0.5));
    const cx<T> o = scale(mul_i<-1>(zk - zm), T(0.5));
    cx<T> xk = e + cmul(o, twiddle_c<base, 2 * L, -1>(wl));
    // X[0] = Re Z[0] + Im Z[0], X[L] = Re Z[0] - Im Z[0] (Z[L] = Z[0],
    // w_2L^L = -1); with nyq both go to column 0
    if (a.nyq && k == 0) xk = cx<T>{zk.re + zk.im, zk.re - zk.im};
    st_cx<nt_store<0>()>(dst + k, xk);
  });
  if (lane == 0 && !a.nyq) {
    const cx<T> z0 = zs[0];
    st_cx<nt_store<0>()>(dst + L, cx<T>{z0.re - z0.im, T(0)});
  }
}

template <typename T, int E, int RW, bool FILL = false>
__global__ void __launch_bounds__(64 * RW) k_xwfwd(const T* __restrict__ f, cx<T>* __restrict__ W, PassArgs a) {
  xwfwd_body<T, E, RW, FILL>(f, W, a, blockIdx.x, blockIdx.y);
}
template <typename T, int E, int RW, bool FILL = false>
__global__ void __launch_bounds__(64 * RW) k_xwfwd_g(GroupArgs g) {
  unsigned lin;
  bool live;
  const GroupEntry& e = group_entry(g, &lin, &live);
  if (!live) return;  // uniform over the workgroup, before any barrier
  const unsigned gx = unsigned(cdiv((long long)e.a.ny * e.a.nz, RW));
  xwfwd_body<T, E, RW, FILL>(static_cast<const T*>(group_in(g, e)), static_cast<cx<T>*>(group_out(g, e)), e.a,
                             lin % gx, lin / gx);
}
template <typename T, int E, int RW, bool FILL = false>
void launch_xwfwd(const PassArgs& a, const void* in, void* out, hipStream_t s) {
  dim3 grid(cdiv((long long)a.ny * a.nz, RW), a.ncomp);
  hipLaunchKernelGGL((k_xwfwd<T, E, RW, FILL>), grid, dim3(64 * RW), 0, s, static_cast<const T*>(in),
                     static_cast<cx<T>*>(out), a);
}
template <typename T, int E, int RW, bool FILL = false>
void launchg_xwfwd(const GroupArgs& g, unsigned nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_xwfwd_g<T, E, RW, FILL>), dim3(nblocks), dim3(64 * RW), 0, s, g);
}

template <typename T, int E, int RW, bool ML>
__global__ void __launch_bounds__(64 * RW) k_xwinv(const cx<T>* __restrict__ W, T* __restrict__ u, PassArgs a) {
  xwinv_body<T, E, RW, ML>(W, u, a, blockIdx.x, blockIdx.y);
}
template <typename T, int E, int RW, bool ML>
__global__ void __launch_bounds__(64 * RW) k_xwinv_g(GroupArgs g) {
  unsigned lin;
  bool live;
  const GroupEntry& e = group_entry(g, &lin, &live);
  if (!live) return;  // uniform over the workgroup, before any barrier
  const unsigned gx = unsigned(cdiv((long long)e.a.ny * e.a.nz, RW));
  xwinv_body<T, E, RW, ML>(static_cast<const cx<T>*>(group_in(g, e)), static_cast<T*>(group_out(g, e)), e.a,
                           lin % gx, lin / gx);
}
template <typename T, int E, int RW, bool ML>
void launch_xwinv(const PassArgs& a, const void* in, void* out, hipStream_t s) {
  dim3 grid(cdiv((long long)a.ny * a.nz, RW), a.ncomp);
  hipLaunchKernelGGL((k_xwinv<T, E, RW, ML>), grid, dim3(64 * RW), 0, s, static_cast<const cx<T>*>(in),
                     static_cast<T*>(out), a);
}
template <typename T, int E, int RW, bool ML>
void launchg_xwinv(const GroupArgs& g, unsigned nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_xwinv_g<T, E, RW, ML>), dim3(nblocks), dim3(64 * RW), 0, s, g);
}
template <typename T, int E, int RW>
constexpr int xwfwd_lds_bytes() {
  constexpr int A = 64 / E;
  constexpr int NR = 31 - __builtin_clz(E > A ? E : A);
  return int(sizeof(cx<T>)) * (RW * xwfwd_slot<E>() + (zwave_lds_twiddles<E>() ? NR * 64 : 1));
}
template <typename T, int E, int RW, bool ML>
constexpr int xwave_lds_bytes() {
  constexpr int A = 64 / E;
  constexpr int NR = 31 - __builtin_clz(E > A ? E : A);
  return int(sizeof(cx<T>)) * (RW * xwinv_slot<E, ML>() + (zwave_lds_twiddles<E>() ? NR * 64 : 1));
}

// mx = 128 E; P = E, Q = 64 (half length 64 E), tile = RW rows (one wave
// each), nch = 0 marks the wave-per-line family.
#define XFW(T, E, RW)                                                                             \
  PassVariant{PASS_XFWD, is64<T>(), 128 * E, E, 64, RW, 0, 64 * RW,                               \
              xwfwd_lds_bytes<T, E, RW>(),                                                        \
              "xfwd_" #T "_w" #E "_r" #RW, &launch_xwfwd<T, E, RW>, &launchg_xwfwd<T, E, RW>}
// the x forward pass along an even or odd direction (mirrored fill, suffix "_e")
#define XFWE(T, E, RW)                                                                            \
  PassVariant{PASS_XFWD, is64<T>(), 128 * E, E, 64, RW, 0, 64 * RW,                               \
              xwfwd_lds_bytes<T, E, RW>(), "xfwd_" #T "_w" #E "_r" #RW "_e",                      \
              &launch_xwfwd<T, E, RW, true>, &launchg_xwfwd<T, E, RW, true>, 1}
#define XIWV(T, E, RW, SUF, ML)                                                                   \
  PassVariant{PASS_XINV, is64<T>(), 128 * E, E, 64, RW, 0, 64 * RW, xwave_lds_bytes<T, E, RW, ML>(), \
              "xinv_" #T "_w" #E "_r" #RW SUF, &launch_xwinv<T, E, RW, ML>, &launchg_xwinv<T, E, RW, ML>}
#define XIW(T, E, RW) XIWV(T, E, RW, "", false)
#define XIWM(T, E, RW) XIWV(T, E, RW, "_m", true)

}  // namespace ups
