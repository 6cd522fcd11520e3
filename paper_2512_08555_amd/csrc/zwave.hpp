// Pass 3, one wavefront per z line: forward DFT along z (rows z < nz live),
// times G_hat, inverse DFT, keep z < nz.
//
// A line of length M = 64 E lives in one wavefront, E values per lane, so
// every exchange between FFT stages is wave-local: LDS traffic ordered by
// the wave's own instruction stream, no workgroup barrier.  With 2E floats
// of line data per lane the kernel needs far fewer registers than the
// four-step column kernels, and more waves per SIMD hide the memory latency.
//
// Forward transform, n = l + 64 j (lane l, register j), k = k1 + E k2:
//   stage 1  DFT_E over j (inputs j >= E/2 are the zero padding), times
//            w_M^(l k1);
//   the remaining DFT_64 over l, with l = l1 + A l2 (A = 64/E) and
//   k2 = m1 + E m2, splits into
//   stage 2  DFT_E over l2 on lane (k1, l1), times w_64^(l1 m1);
//   stage 3  DFT_A over l1,
// leaving lane L, register (r, m2) with X[L + 64 r + E^2 m2], r < E/A: for a
// fixed register the lanes hold 64 consecutive frequencies, so the G_hat
// loads of a wave are contiguous.  The inverse runs the mirrored steps with
// n = n0 + A n', a = L + 64 r = b + E c, n' = e + E f:
//   stage A  DFT_A over m2 (inverse), times conj w_M^(n0 a);
//   stage B  DFT_E over c on lane (b, n0), times conj w_M^(A e b);
//   stage C  DFT_E over b on lane (n0, e), only f < E/2 (rows n < M/2),
// leaving lane L' = n0 + A e with rows L' + 64 f.
//
// A workgroup holds CW adjacent columns of one line (ky, component): it
// stages the input tile (nz rows x CW columns) through LDS with coalesced
// loads, each wave transforms one column using that column's LDS slot for
// its exchanges, and the tile goes back through LDS to coalesced stores.
// Exchanges move real parts, then imaginary parts, through the slot.  A run
// of twiddles w^(k x), k < E, takes log2 E loads from the 64 x 64 product
// block of the z table (rows k = 1, 2, 4, ...) and builds the other powers
// as products.
#pragma once
#include "passes_impl.hpp"
#include "ztab.hpp"

namespace ups {

template <int E>
struct ZWave {
  static_assert(E >= 8 && 64 % E == 0, "lines of 64 E points, E in {8, 16, 32, 64}");
  static constexpr int M = 64 * E;
  static constexpr int A = 64 / E;     // stage-3 radix
  static constexpr int E2 = E * E;
  static constexpr int R3 = E / A;     // frequency groups per lane after stage 3
  // LDS maps (floats), chosen so that the 32 lanes of each half-wave hit 32
  // different banks:
  //   exchange 1:  [k1][l], row stride S1 = 64 + 32/E
  //   exchange 2 and inverse exchange 1:  [l1 or n0][a], row stride P2 >= E^2,
  //                P2 = E (mod 32)
  //   inverse exchange 2:  [e][E n0 + (b ^ swz(n0))], row stride 65,
  //                swz(n0) = (E/2) [n0 >= A/2]
  static constexpr int S1 = 64 + 32 / E;
  static constexpr int P2 = E2 + ((E % 32) - (E2 % 32) + 32) % 32;
  static constexpr int S4 = 65;
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int xfloats = cmax(cmax(E * S1, A * P2), (E - 1) * S4 + 64);
};

// Twiddles of the later stages from the tables of ztab.hpp, which the
// workgroup copies into LDS from behind the axis's twiddle table: one load
// per twiddle instead of products.  Table loads are issued in groups of
// kTabGroup between compiler fences, so that the compiler does not hoist all
// of a stage's loads (and their registers) ahead of the arithmetic.
constexpr int kTabGroup = 2;
// Complex elements per LDS column slot: room for the nz <= M/2 tile rows and
// for one exchange (floats), with slot stride = 16 / CW (mod 16) so that the
// 64-bit tile accesses of the CW columns fall in different banks.
template <int E, int CW>
constexpr int zwave_slot() {
  int need = ZWave<E>::cmax(32 * E, (ZWave<E>::xfloats + 1) / 2);
  const int r = (16 / CW) % 16;
  while (need % 16 != r) ++need;
  return need;
}

// Twiddle rows staged in LDS once per workgroup (short lines: measured
// faster at E = 8) or read from the table where used (E = 16: fewer registers).
// (Loading every twiddle from the table instead of forming powers by
// products takes about 30 more registers per lane and measured 30% slower.)
template <int E>
constexpr bool zwave_lds_twiddles() { return E <= 8; }

// LDS of one workgroup: CW column slots plus the staged twiddle rows, plus
// the later-stage twiddle tables if TB.
template <typename T, int E, int CW, bool TB = false>
constexpr int zwave_lds_bytes() {
  constexpr int A = 64 / E;
  constexpr int NR = 31 - __builtin_clz(E > A ? E : A);
  return int(sizeof(cx<T>)) * (CW * zwave_slot<E, CW>() + (zwave_lds_twiddles<E>() ? NR * 64 : 1) +
                               (TB ? ZTab<E>::total : 1));
}

__device__ __forceinline__ void wave_fence() { asm volatile("" ::: "memory"); }

template <typename T, int E, typename WA, typename RA>
__device__ __forceinline__ void wave_exchange(cx<T> (&v)[E], T* xf, WA waddr, RA raddr) {
  T o[E];
  wave_fence();
  static_for<0, E>([&](auto ii) { constexpr int i = decltype(ii)::value; xf[waddr(i)] = v[i].re; });
  wave_fence();
  static_for<0, E>([&](auto ii) { constexpr int i = decltype(ii)::value; o[i] = xf[raddr(i)]; });
  wave_fence();
  static_for<0, E>([&](auto ii) { constexpr int i = decltype(ii)::value; xf[waddr(i)] = v[i].im; });
  wave_fence();
  static_for<0, E>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    v[i].re = o[i];
    v[i].im = xf[raddr(i)];
  });
  wave_fence();
}

// Copy the ZTab tables of length M = 64 E into LDS: they follow the M
// entries and the 64 x 64 product block of the axis table tw.
template <typename T, int E>
__device__ __forceinline__ void zw_fill_tables(cx<T>* tab, const cx<T>* tw, int t, int nthreads) {
  const cx<T>* src = tw + ZTab<E>::M + kTw2Row * kTw2Row;
  for (int i = t; i < ZTab<E>::total; i += nthreads) tab[i] = src[i];
}

// Forward transform of one line held by a wave: on entry v[j] (j < E/2)
// holds row lane + 64 j (rows M/2 .. M-1 are the zero padding; FULL: every
// v[j] holds its row, the first stage is a full DFT_E); on exit register
// r A + m2 holds X[lane + 64 r + E^2 m2].  xf: the wave's LDS exchange area;
// trow(j, x) = w_M^(2^j x).
// TB: stage-2 twiddles from the ZTab tables at tab (LDS), else by products
// of table rows.
template <typename T, int E, bool TB, bool FULL = false, typename TR>
__device__ __forceinline__ void zw_forward(cx<T> (&v)[E], T* xf, int lane, TR trow, const cx<T>* tab) {
  using Z = ZWave<E>;
  constexpr int A = Z::A, R3 = Z::R3, S1 = Z::S1, P2 = Z::P2;
  // stage 1: DFT_E over j, times w_M^(l k1) = T[k1][l]
  if constexpr (FULL) dft<E, -1>(v);
  else dft_half_in<E, -1>(v);
  twiddle_run<E, false>(v, [&](int j) { return trow(j, lane); });
  // exchange 1: (l, k1) at k1 S1 + l; lane (k1, l1) reads l2 at k1 S1 + l1 + A l2
  {
    const int k1 = lane % E, l1 = lane / E;
    const int rb = k1 * S1 + l1;
    wave_exchange<T, E>(v, xf, [&](int i) { return lane + i * S1; }, [&](int i) { return rb + A * i; });
  }
  // stage 2: DFT_E over l2, times w_64^(l1 m1) = T[E l1][m1]
  dft<E, -1>(v);
  if constexpr (TB) {
    const cx<T>* r2 = tab + ZTab<E>::o2 + (E + 1) * (lane / E);
    static_for<1, E>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      if constexpr (k % kTabGroup == 0) wave_fence();  // loads stay near their use
      v[k] = cmul(v[k], r2[k]);
    });
  } else {
    const int el1 = E * (lane / E);
    twiddle_run<E, false>(v, [&](int j) { return trow(j, el1); });
  }
  // exchange 2: (a = k1 + E m1, l1) at l1 P2 + a; lane L reads register
  // r A + l1 (a = L + 64 r)
  {
    const int wb = (lane / E) * P2 + lane % E;
    wave_exchange<T, E>(v, xf, [&](int i) { return wb + E * i; },
                        [&](int i) { return lane + (i % A) * P2 + 64 * (i / A); });
  }
  // stage 3: lane L, register r A + m2 holds k = L + 64 r + E^2 m2
  static_for<0, R3>([&](auto rr) {
    constexpr int r = decltype(rr)::value;
    dft<A, -1>(&v[r * A]);
  });
}

// Inverse transform, first half of the outputs: on entry register r A + m2
// holds X[lane + 64 r + E^2 m2] (the layout zw_forward leaves); on exit v[f]
// (f < E/2) holds the unnormalised inverse DFT at row lane + 64 f.
// TB: twiddles of stages A and B from the ZTab tables at tab (LDS), else
// from table rows and products.
template <typename T, int E, bool TB, typename TR>
__device__ __forceinline__ void zw_inverse(cx<T> (&v)[E], T* xf, int lane, TR trow, const cx<T>* tab) {
  using Z = ZWave<E>;
  constexpr int M = Z::M, A = Z::A, R3 = Z::R3, P2 = Z::P2, S4 = Z::S4;
  // inverse stage A: DFT_A over m2, times conj w_M^(n0 a), a = L + 64 r:
  // w_M^(n0 L) = T[n0][L] and the constant w_M^(64 n0 r)
  if constexpr (TB) {
    const cx<T>* ra = tab + ZTab<E>::oa + lane;
    static_for<0, R3>([&](auto rr) {
      constexpr int r = decltype(rr)::value;
      dft<A, +1>(&v[r * A]);
      static_for<1, A>([&](auto nn) {
        constexpr int n0 = decltype(nn)::value;
        if constexpr ((r * A + n0) % kTabGroup == 0) wave_fence();
        v[r * A + n0] = cmulc(v[r * A + n0], ra[(n0 - 1) * (M / A) + 64 * r]);
      });
    });
  } else {
    // w_M^(n0 L) for n0 < A, shared by the R3 groups
    cx<T> q[A];
    static_for<1, A>([&](auto nn) {
      constexpr int n0 = decltype(nn)::value;
      constexpr int hb = 1 << (31 - __builtin_clz(n0));
      if constexpr (hb == n0) q[n0] = trow(31 - __builtin_clz(n0), lane);
      else q[n0] = cmul(q[hb], q[n0 - hb]);
    });
    static_for<0, R3>([&](auto rr) {
      constexpr int r = decltype(rr)::value;
      dft<A, +1>(&v[r * A]);
      static_for<1, A>([&](auto nn) {
        constexpr int n0 = decltype(nn)::value;
        v[r * A + n0] = twiddle_c<(long long)64 * r * n0, M, +1>(cmulc(v[r * A + n0], q[n0]));
      });
    });
  }
  // inverse exchange 1: (a, n0) at n0 P2 + a; lane (b, n0) reads c at
  // n0 P2 + b + E c
  {
    const int rb = (lane / E) * P2 + lane % E;
    wave_exchange<T, E>(v, xf, [&](int i) { return lane + (i % A) * P2 + 64 * (i / A); },
                        [&](int i) { return rb + E * i; });
  }
  // inverse stage B: DFT_E over c, times conj w_M^(A e b) = T[A e][b]
  dft<E, +1>(v);
  if constexpr (TB) {
    const cx<T>* rb = tab + ZTab<E>::ob + (E + 1) * (lane % E);
    static_for<1, E>([&](auto kk) {
      constexpr int k = decltype(kk)::value;
      if constexpr (k % kTabGroup == 0) wave_fence();
      v[k] = cmulc(v[k], rb[k]);
    });
  } else {
    const int ab = A * (lane % E);
    twiddle_run<E, true>(v, [&](int j) { return trow(j, ab); });
  }
  // inverse exchange 2: (b, n0, e) at e S4 + E n0 + (b ^ swz(n0)); lane
  // (n0, e) = n0 + A e reads b
  {
    constexpr int HE = E / 2;
    const int b = lane % E, n0 = lane / E;
    const int wb = E * n0 + (b ^ (n0 >= A / 2 ? HE : 0));
    const int n0r = lane % A, er = lane / A;
    const int sw = n0r >= A / 2 ? HE : 0;
    const int rlo = er * S4 + E * n0r + sw;   // b < E/2: b ^ sw = b + sw
    const int rhi = er * S4 + E * n0r - sw;   // b >= E/2: b ^ sw = b - sw
    wave_exchange<T, E>(v, xf, [&](int i) { return wb + S4 * i; },
                        [&](int i) { return (i < HE ? rlo : rhi) + i; });
  }
  // inverse stage C: rows lane + 64 f, f < E/2
  dft_half_out<E, +1>(v);
}

// GP: load this lane's G_hat values at the start (they then share the
// latency of the tile loads) instead of after the forward transform.
// TB: twiddles of stage 2 and of the inverse stages A and B from LDS tables.
// FILL: the z direction is even or odd (a.fill_z = +1 or -1, nz = M/2):
// rows n >= M/2 of the line are a.fill_z times row M - 1 - n instead of the
// zero padding, read from the column's LDS slot, and the first stage is full.
template <typename T, int E, int CW, bool GP, bool TB, bool FILL = false>
__device__ __forceinline__ void zwave_body(cx<T>* __restrict__ W, const PassArgs& a, unsigned bx) {
  using Z = ZWave<E>;
  constexpr int M = Z::M, A = Z::A, E2 = Z::E2;
  constexpr int CS = zwave_slot<E, CW>();
  constexpr unsigned CB = sizeof(cx<T>);
  // every twiddle run reads rows 2^j of the 64 x 64 product table (run
  // lengths E and A): the workgroup copies those rows into LDS once
  constexpr int NR = 31 - __builtin_clz(E > A ? E : A);
  constexpr bool LT = zwave_lds_twiddles<E>();
  __shared__ cx<T> tile[CW * CS];
  __shared__ cx<T> twl[LT ? NR * 64 : 1];
  __shared__ cx<T> ztab[TB ? ZTab<E>::total : 1];
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_z);
  // row 2^j, column x of the product table, from LDS or from the table
  auto trow = [&](int j, int x) { return LT ? twl[64 * j + x] : tw_row(tw, M, 1u << j)[x]; };

  const int ntiles = (a.kx + CW - 1) / CW;
  const ColMap mp = zmap(bx, ntiles, a.my, a.ncomp, col_slots<T, CW>(ntiles));
  if (!mp.active) return;  // uniform over the workgroup, before any barrier
  const int t = threadIdx.x;
  const int lane = t & 63, c = t >> 6;
  const int kx0 = mp.tile * CW;
  const int ky = mp.line;
  cx<T>* ubase = W + mp.comp * a.comp_w + (long long)ky * a.px + kx0;
  const int nz = a.nz;
  const bool full = nz == M / 2;
  // G_hat line of this wave's column: kz = lane + 64 r + E^2 m2 reads
  // octant row iz = min(kz, M - kz)
  const T* gline;
  {
    const int cg = (kx0 + c < a.kx) ? c : a.kx - 1 - kx0;
    const int iy = ky <= a.my - ky ? ky : a.my - ky;
    gline = static_cast<const T*>(a.ghat) + iy * a.g_plane + (long long)(kx0 + cg) * a.gz;
  }
  // register i holds kz = lane + base(i), base(i) = 64 (i / A) + E^2 (i % A); a
  // base below M/2 keeps the whole wave below M/2 (iz = kz, ascending), a base
  // at or above M/2 keeps it above (iz = M - kz, descending): a constant
  // offset from one of two per-lane pointers, no per-element index math
  const T* gup = gline + lane;
  const T* gdn = gline - lane;
  auto gload = [&](int i) {
    const int base = 64 * (i / A) + E2 * (i % A);
    return ld_r<nt_load<kNtGhatBit>()>(base < M / 2 ? gup + base : gdn + (M - base));
  };
  T gpre[GP ? E : 1];
  if constexpr (GP) {
    static_for<0, E>([&](auto ii) { gpre[decltype(ii)::value] = gload(decltype(ii)::value); });
  }

  if constexpr (LT) {
    for (int i = t; i < NR * 64; i += 64 * CW) twl[i] = tw_row(tw, M, 1u << (i / 64))[i % 64];
  }
  if constexpr (TB) zw_fill_tables<T, E>(ztab, tw, t, 64 * CW);

  // ---- coalesced tile load: thread (tc, tr) moves rows tr + 64 i of column tc
  const int tc = t % CW, tr = t / CW;
  // (with a.nyq column 0 belongs to the pair launch: loaded, not stored)
  const bool tvalid = kx0 + tc < a.kx && !(a.nyq && kx0 + tc == 0);
  const bool tload = kx0 + tc < a.kx;
  const int tcl = tload ? tc : a.kx - 1 - kx0;  // in-bounds column for the loads
  const unsigned toff = (unsigned(tr) * unsigned(a.plane) + unsigned(tcl)) * CB;
  cx<T>* tslot = tile + tc * CS;
  if (full) {
    cx<T> ld[E / 2];
    static_for<0, E / 2>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      ld[i] = ld_at<nt_load<2>()>(ubase + (long long)(64 * i) * a.plane, toff);
    });
    static_for<0, E / 2>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      tslot[tr + 64 * i] = ld[i];
    });
  } else {
    // rows >= nz are the zero padding: not loaded.  The 64-row block goes
    // into the 64-bit base as in the full case, so the per-lane offset stays
    // below 64 planes (a row index times the plane in 32 bits would wrap
    // for FP64 lines of 1024 with 1024 x 528 planes).
    static_for<0, E / 2>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      const int row = tr + 64 * i;
      cx<T> val = zero_c<T>();
      if (row < nz) val = ld_at<nt_load<2>()>(ubase + (long long)(64 * i) * a.plane, toff);
      tslot[row] = val;
    });
  }
  __syncthreads();

  // ---- wave c: the line of column kx0 + c
  cx<T>* slot = tile + c * CS;
  T* xf = reinterpret_cast<T*>(slot);
  cx<T> v[E];
  static_for<0, E / 2>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    v[j] = slot[lane + 64 * j];
  });
  if constexpr (FILL) {
    // row lane + 64 j, j >= E/2, mirrors row (63 - lane) + 64 (E - 1 - j)
    const T fs = T(a.fill_z);
    static_for<E / 2, E>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      v[j] = scale(slot[(63 - lane) + 64 * (E - 1 - j)], fs);
    });
  }
  zw_forward<T, E, TB, FILL>(v, xf, lane, trow, ztab);
  // G_hat: lane L, register r A + m2 holds kz = L + 64 r + E^2 m2
  static_for<0, E>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    if constexpr (GP) v[i] = scale(v[i], gpre[i]);
    else v[i] = scale(v[i], gload(i));
  });
  zw_inverse<T, E, TB>(v, xf, lane, trow, ztab);
  wave_fence();
  static_for<0, E / 2>([&](auto ff) {
    constexpr int f = decltype(ff)::value;
    slot[lane + 64 * f] = v[f];
  });
  __syncthreads();

  // ---- coalesced tile store, rows z < nz
  if (tvalid) {
    if (full) {
      static_for<0, E / 2>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        st_at<nt_store<2>()>(ubase + (long long)(64 * i) * a.plane, toff, tslot[tr + 64 * i]);
      });
    } else {
      static_for<0, E / 2>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        if (tr + 64 * i < nz) st_at<nt_store<2>()>(ubase + (long long)(64 * i) * a.plane, toff, tslot[tr + 64 * i]);
      });
    }
  }
}

// Column 0 of a W that carries C = X0 + i XN (X0 = X[0], XN = X[mx/2],
// each real in y and z; PassArgs::nyq).  After the y and z forward
// transforms F_C = F_0 + i F_N with F_0 and F_N Hermitian in (ky, kz), so
// F_0(ky, kz) = (F_C(ky, kz) + conj F_C(-ky, -kz)) / 2 and
// F_N = (F_C - conj F_C(-ky, -kz)) / 2i.  The product the solve needs,
// G0 F_0 + i GN F_N (G0, GN: the real G_hat lines of kx = 0 and mx/2), is
//   R(ky, kz) = F_C(ky, kz) (G0 + GN)/2 + conj F_C(-ky, -kz) (G0 - GN)/2,
// and its inverse is the solve's kx = 0 part plus i times its kx = mx/2
// part.  Block b takes the lines ky = b and my - ky (once for ky = 0 and
// my/2), one wave each: it loads rows z < nz of column 0, transforms them,
// swaps the spectra through LDS, inverts the products and writes rows
// z < nz of column 0 back.  It runs beside the z pass's main launch, which
// loads column 0 with its tile but does not store it.
template <typename T, int E>
__global__ void __launch_bounds__(128) k_zpair(cx<T>* __restrict__ W, PassArgs a) {
  using Z = ZWave<E>;
  constexpr int M = Z::M, A = Z::A, E2 = Z::E2;
  __shared__ cx<T> spec[2][M];
  __shared__ T xfa[2][Z::xfloats];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int ky = blockIdx.x, comp = blockIdx.y;
  const int kb = ky == 0 ? 0 : a.my - ky;
  const bool self = kb == ky;
  const bool active = !(self && w == 1);   // uniform over the wave
  const int line = w ? kb : ky;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_z);
  auto trow = [&](int j, int x) { return tw_row(tw, M, 1u << j)[x]; };
  T* xf = xfa[w];
  cx<T>* col = W + comp * a.comp_w + (long long)line * a.px;
  cx<T> v[E];
  if (active) {
    static_for<0, E / 2>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      const int z = lane + 64 * j;
      v[j] = z < a.nz ? col[(long long)z * a.plane] : zero_c<T>();
    });
    zw_forward<T, E, false>(v, xf, lane, trow, static_cast<const cx<T>*>(nullptr));
    static_for<0, E>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      spec[w][lane + 64 * (i / A) + E2 * (i % A)] = v[i];
    });
  }
  __syncthreads();
  if (!active) return;  // after the only barrier
  // G_hat lines of kx = 0 and kx = mx/2 (column a.kx), iy = ky
  const T* g0 = static_cast<const T*>(a.ghat) + (long long)ky * a.g_plane;
  const T* gn = g0 + (long long)a.kx * a.gz;
  const cx<T>* other = spec[self ? 0 : 1 - w];
  static_for<0, E>([&](auto ii) {
    constexpr int i = decltype(ii)::value;
    const int k = lane + 64 * (i / A) + E2 * (i % A);
    const int iz = k <= M - k ? k : M - k;
    const T gp = T(0.5) * (g0[iz] + gn[iz]), gm = T(0.5) * (g0[iz] - gn[iz]);
    v[i] = scale(v[i], gp) + scale(conj(other[(M - k) & (M - 1)]), gm);
  });
  zw_inverse<T, E, false>(v, xf, lane, trow, static_cast<const cx<T>*>(nullptr));
  static_for<0, E / 2>([&](auto ff) {
    constexpr int f = decltype(ff)::value;
    const int z = lane + 64 * f;
    if (z < a.nz) col[(long long)z * a.plane] = v[f];
  });
}

template <typename T, int E>
void launch_zpair_t(const PassArgs& a, void* W, hipStream_t s) {
  hipLaunchKernelGGL((k_zpair<T, E>), dim3(a.my / 2 + 1, a.ncomp), dim3(128), 0, s, static_cast<cx<T>*>(W), a);
}

// OCC: minimum waves per SIMD asked of the register allocator (1: no
// constraint; 8 caps registers at 64, spilling a few values to scratch).
template <typename T, int E, int CW, bool GP, int OCC, bool TB, bool FILL = false>
__global__ void __launch_bounds__(64 * CW) __attribute__((amdgpu_waves_per_eu(OCC)))
k_zwave(cx<T>* __restrict__ W, PassArgs a) {
  zwave_body<T, E, CW, GP, TB, FILL>(W, a, blockIdx.x);
}
template <typename T, int E, int CW, bool GP, bool TB, bool FILL = false>
__global__ void __launch_bounds__(64 * CW) k_zwave_g(GroupArgs g) {
  unsigned lin;
  bool live;
  const GroupEntry& e = group_entry(g, &lin, &live);
  if (!live) return;  // uniform over the workgroup, before any barrier
  zwave_body<T, E, CW, GP, TB, FILL>(static_cast<cx<T>*>(group_out(g, e)), e.a, lin);
}

template <typename T, int CW>
inline unsigned zwave_blocks(const PassArgs& a) {
  return zmap_blocks(cdiv(a.kx, CW), a.my, a.ncomp, col_slots<T, CW>(cdiv(a.kx, CW)));
}
template <typename T, int E, int CW, bool GP, int OCC, bool TB, bool FILL = false>
void launch_zwave(const PassArgs& a, const void*, void* out, hipStream_t s) {
  hipLaunchKernelGGL((k_zwave<T, E, CW, GP, OCC, TB, FILL>), dim3(zwave_blocks<T, CW>(a)), dim3(64 * CW), 0, s,
                     static_cast<cx<T>*>(out), a);
}
template <typename T, int E, int CW, bool GP, bool TB, bool FILL = false>
void launchg_zwave(const GroupArgs& g, unsigned nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_zwave_g<T, E, CW, GP, TB, FILL>), dim3(nblocks), dim3(64 * CW), 0, s, g);
}

// P = E, Q = 64 (line length 64 E), tile = CW columns, nch = 0 marks the
// wave-per-line family; the "_g" variants load G_hat at the start, "_o8"
// asks for 8 waves per SIMD, "_t" takes the later twiddles from LDS tables.
#define ZWV(T, E, CW, SUF, GP, OCC, TB)                                                           \
  PassVariant{PASS_ZCONV, is64<T>(), 64 * E, E, 64, CW, 0, 64 * CW,                               \
              zwave_lds_bytes<T, E, CW, TB>(), "zconv_" #T "_w" #E "_c" #CW SUF,                  \
              &launch_zwave<T, E, CW, GP, OCC, TB>, &launchg_zwave<T, E, CW, GP, TB>}
#define ZW(T, E, CW) ZWV(T, E, CW, "", false, 1, false)
#define ZWO(T, E, CW) ZWV(T, E, CW, "_o8", false, 8, false)
#define ZWG(T, E, CW) ZWV(T, E, CW, "_g", true, 1, false)
#define ZWT(T, E, CW) ZWV(T, E, CW, "_t", false, 1, true)
// the z pass along an even or odd direction (mirrored fill, suffix "_e")
#define ZWE(T, E, CW, TB)                                                                         \
  PassVariant{PASS_ZCONV, is64<T>(), 64 * E, E, 64, CW, 0, 64 * CW,                               \
              zwave_lds_bytes<T, E, CW, TB>(), "zconv_" #T "_w" #E "_c" #CW "_e",                 \
              &launch_zwave<T, E, CW, false, 1, TB, true>, &launchg_zwave<T, E, CW, false, TB, true>, 1}

}  // namespace ups
