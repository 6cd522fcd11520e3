// Pass 4 with one wavefront per y line: inverse DFT along y of all M = my
// rows, keep rows y < ny (in place).
//
// The transform is the second half of the wave-per-line z pass (stages A,
// B, C of zwave.hpp), which takes its input in the layout the forward
// stages leave: lane L, register r A + m2 holds row L + 64 r + E^2 m2.  A
// workgroup of CW waves holds CW adjacent columns of one z plane.  The M
// input rows of the tile come into LDS in two halves of M/2 rows (coalesced
// loads, rows of CW columns); after each half every wave reads the rows of
// its column that fall in that half straight into those registers.  The
// kept rows go back through the column slot to coalesced stores.
//
// Pass 2 the same way: the tile's ny <= M/2 input rows come into LDS, each
// wave takes rows lane + 64 j of its column (the forward stages' input
// layout), runs the forward stages of the z pass, and the M output rows
// leave through the column slots in two halves of M/2 rows.
#pragma once
#include "zwave.hpp"

namespace ups {

// FILL: the y direction is even or odd (a.fill_y = +1 or -1, ny = M/2):
// rows n >= M/2 are a.fill_y times row M - 1 - n, read from the column's LDS
// slot, and the first stage is full.
template <typename T, int E, int CW, bool FILL = false>
__device__ __forceinline__ void ywfwd_body(cx<T>* __restrict__ W, const PassArgs& a, unsigned bx) {
  using Z = ZWave<E>;
  constexpr int M = Z::M, A = Z::A, E2 = Z::E2;
  constexpr int H2 = M / 2;
  constexpr int CS = zwave_slot<E, CW>();
  constexpr unsigned CB = sizeof(cx<T>);
  constexpr int NR = 31 - __builtin_clz(E > A ? E : A);
  constexpr bool LT = zwave_lds_twiddles<E>();
  __shared__ cx<T> tile[CW * CS];
  __shared__ cx<T> twl[LT ? NR * 64 : 1];
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_y);
  auto trow = [&](int j, int x) { return LT ? twl[64 * j + x] : tw_row(tw, M, 1u << j)[x]; };

  const int ntiles = (a.kx + CW - 1) / CW;
  const ColMap mp = ymap(bx, ntiles, a.nz, a.ncomp, col_slots<T, CW>(ntiles));
  if (!mp.active) return;  // uniform over the workgroup, before any barrier
  const int t = threadIdx.x;
  const int lane = t & 63, c = t >> 6;
  const int kx0 = mp.tile * CW;
  cx<T>* ubase = W + mp.comp * a.comp_w + mp.line * a.plane + kx0;
  const int ny = a.ny;

  if constexpr (LT) {
    for (int i = t; i < NR * 64; i += 64 * CW) twl[i] = tw_row(tw, M, 1u << (i / 64))[i % 64];
  }

  // tile rows: thread (tc, tr) moves rows tr + 64 i of column tc
  const int tc = t % CW, tr = t / CW;
  const bool tvalid = kx0 + tc < a.kx;
  const int tcl = tvalid ? tc : a.kx - 1 - kx0;  // in-bounds column for the loads
  const unsigned toff = (unsigned(tr) * unsigned(a.px) + unsigned(tcl)) * CB;
  cx<T>* tslot = tile + tc * CS;
  if (ny == H2) {
    cx<T> ld[E / 2];
    static_for<0, E / 2>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      ld[i] = ld_at<nt_load<1>()>(ubase + (long long)(64 * i) * a.px, toff);
    });
    static_for<0, E / 2>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      tslot[tr + 64 * i] = ld[i];
    });
  } else {
    static_for<0, E / 2>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      const int row = tr + 64 * i;
      const int rowc = row < ny ? row : ny - 1;  // clamped: loads stay in bounds
      const cx<T> val = ld_at<nt_load<1>()>(ubase, (unsigned(rowc) * unsigned(a.px) + unsigned(tcl)) * CB);
      tslot[row] = row < ny ? val : zero_c<T>();
    });
  }
  __syncthreads();

  cx<T>* slot = tile + c * CS;
  T* xf = reinterpret_cast<T*>(slot);
  cx<T> v[E];
  static_for<0, E / 2>([&](auto jj) {
    constexpr int j = decltype(jj)::value;
    v[j] = slot[lane + 64 * j];
  });
  if constexpr (FILL) {
    // row lane + 64 j, j >= E/2, mirrors row (63 - lane) + 64 (E - 1 - j)
    const T fs = T(a.fill_y);
    static_for<E / 2, E>([&](auto jj) {
      constexpr int j = decltype(jj)::value;
      v[j] = scale(slot[(63 - lane) + 64 * (E - 1 - j)], fs);
    });
  }
  zw_forward<T, E, false, FILL>(v, xf, lane, trow, static_cast<const cx<T>*>(nullptr));
  // output rows k = lane + base(i) (base a multiple of 64: a wave's rows lie
  // in one half), half h through the slots
  static_for<0, 2>([&](auto hh) {
    constexpr int h = decltype(hh)::value;
    __syncthreads();  // h = 0: every wave is past its input reads; h = 1: the first half is stored
    static_for<0, E>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      constexpr int base = 64 * (i / A) + E2 * (i % A);
      if constexpr (base / H2 == h) slot[lane + base - H2 * h] = v[i];
    });
    __syncthreads();
    if (tvalid) {
      static_for<0, E / 2>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        st_at<nt_store<1>()>(ubase + (long long)(H2 * h + 64 * i) * a.px, toff, tslot[tr + 64 * i]);
      });
    }
  });
}

template <typename T, int E, int CW, bool FILL = false>
__global__ void __launch_bounds__(64 * CW) k_ywfwd(cx<T>* __restrict__ W, PassArgs a) {
  ywfwd_body<T, E, CW, FILL>(W, a, blockIdx.x);
}
template <typename T, int E, int CW, bool FILL = false>
__global__ void __launch_bounds__(64 * CW) k_ywfwd_g(GroupArgs g) {
  unsigned lin;
  bool live;
  const GroupEntry& e = group_entry(g, &lin, &live);
  if (!live) return;  // uniform over the workgroup, before any barrier
  ywfwd_body<T, E, CW, FILL>(static_cast<cx<T>*>(group_out(g, e)), e.a, lin);
}
template <typename T, int E, int CW, bool FILL = false>
void launch_ywfwd(const PassArgs& a, const void*, void* out, hipStream_t s) {
  hipLaunchKernelGGL((k_ywfwd<T, E, CW, FILL>), dim3(ypass_blocks<T, CW>(a)), dim3(64 * CW), 0, s,
                     static_cast<cx<T>*>(out), a);
}
template <typename T, int E, int CW, bool FILL = false>
void launchg_ywfwd(const GroupArgs& g, unsigned nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_ywfwd_g<T, E, CW, FILL>), dim3(nblocks), dim3(64 * CW), 0, s, g);
}
#define YFW(T, E, CW)                                                                             \
  PassVariant{PASS_YFWD, is64<T>(), 64 * E, E, 64, CW, 0, 64 * CW, zwave_lds_bytes<T, E, CW>(),   \
              "yfwd_" #T "_w" #E "_c" #CW, &launch_ywfwd<T, E, CW>, &launchg_ywfwd<T, E, CW>}
// the y forward pass along an even or odd direction (mirrored fill, suffix "_e")
#define YFWE(T, E, CW)                                                                            \
  PassVariant{PASS_YFWD, is64<T>(), 64 * E, E, 64, CW, 0, 64 * CW, zwave_lds_bytes<T, E, CW>(),   \
              "yfwd_" #T "_w" #E "_c" #CW "_e", &launch_ywfwd<T, E, CW, true>,                    \
              &launchg_ywfwd<T, E, CW, true>, 1}

// PRE: issue the loads of both halves at the start (the second half waits
// in registers while the first is read out of LDS).  TB: twiddles of the
// inverse stages A and B from LDS tables.
template <typename T, int E, int CW, bool PRE, bool TB>
__device__ __forceinline__ void ywinv_body(cx<T>* __restrict__ W, const PassArgs& a, unsigned bx) {
  using Z = ZWave<E>;
  constexpr int M = Z::M, A = Z::A, E2 = Z::E2;
  constexpr int H2 = M / 2;
  constexpr int CS = zwave_slot<E, CW>();
  constexpr unsigned CB = sizeof(cx<T>);
  constexpr int NR = 31 - __builtin_clz(E > A ? E : A);
  constexpr bool LT = zwave_lds_twiddles<E>();
  __shared__ cx<T> tile[CW * CS];
  __shared__ cx<T> twl[LT ? NR * 64 : 1];
  __shared__ cx<T> ztab[TB ? ZTab<E>::total : 1];
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_y);
  // row 2^j, column x of the product table, from LDS or from the table
  auto trow = [&](int j, int x) { return LT ? twl[64 * j + x] : tw_row(tw, M, 1u << j)[x]; };

  const int ntiles = (a.kx + CW - 1) / CW;
  const ColMap mp = ymap(bx, ntiles, a.nz, a.ncomp, col_slots<T, CW>(ntiles));
  if (!mp.active) return;  // uniform over the workgroup, before any barrier
  const int t = threadIdx.x;
  const int lane = t & 63, c = t >> 6;
  const int kx0 = mp.tile * CW;
  cx<T>* ubase = W + mp.comp * a.comp_w + mp.line * a.plane + kx0;
  const int ny = a.ny;
  const bool full = ny == H2;

  if constexpr (LT) {
    for (int i = t; i < NR * 64; i += 64 * CW) twl[i] = tw_row(tw, M, 1u << (i / 64))[i % 64];
  }
  if constexpr (TB) zw_fill_tables<T, E>(ztab, tw, t, 64 * CW);

  // tile rows: thread (tc, tr) moves rows tr + 64 i of column tc
  const int tc = t % CW, tr = t / CW;
  const bool tvalid = kx0 + tc < a.kx;
  const int tcl = tvalid ? tc : a.kx - 1 - kx0;  // in-bounds column for the loads
  const unsigned toff = (unsigned(tr) * unsigned(a.px) + unsigned(tcl)) * CB;
  cx<T>* tslot = tile + tc * CS;
  cx<T>* slot = tile + c * CS;
  T* xf = reinterpret_cast<T*>(slot);
  cx<T> v[E];
  cx<T> ld[PRE ? E : E / 2];
  auto load_half = [&](int h, cx<T>* dst) {
    static_for<0, E / 2>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      dst[i] = ld_at<nt_load<kNtYinvWaveBit>()>(ubase + (long long)(H2 * h + 64 * i) * a.px, toff);
    });
  };
  if constexpr (PRE) {
    load_half(0, ld);
    load_half(1, ld + E / 2);
  }
  static_for<0, 2>([&](auto hh) {
    constexpr int h = decltype(hh)::value;
    if constexpr (h > 0) __syncthreads();  // every wave has read the first half
    if constexpr (!PRE) load_half(h, ld);
    static_for<0, E / 2>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      tslot[tr + 64 * i] = ld[(PRE ? h * (E / 2) : 0) + i];
    });
    __syncthreads();
    // register i takes row lane + base(i); base(i) is a multiple of 64, so
    // the whole wave's rows lie in one half
    static_for<0, E>([&](auto ii) {
      constexpr int i = decltype(ii)::value;
      constexpr int base = 64 * (i / A) + E2 * (i % A);
      if constexpr (base / H2 == h) v[i] = slot[lane + base - H2 * h];
    });
  });
  zw_inverse<T, E, TB>(v, xf, lane, trow, ztab);
  wave_fence();
  static_for<0, E / 2>([&](auto ff) {
    constexpr int f = decltype(ff)::value;
    slot[lane + 64 * f] = v[f];
  });
  __syncthreads();

  // coalesced store, rows y < ny
  if (tvalid) {
    if (full) {
      static_for<0, E / 2>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        st_at<nt_store<kNtYinvWaveBit>()>(ubase + (long long)(64 * i) * a.px, toff, tslot[tr + 64 * i]);
      });
    } else {
      // rows >= ny write row ny - 1 again (the same value): no per-row branch
      static_for<0, E / 2>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        const int row = tr + 64 * i;
        const int rowc = row < ny ? row : ny - 1;
        st_at<nt_store<kNtYinvWaveBit>()>(ubase, (unsigned(rowc) * unsigned(a.px) + unsigned(tcl)) * CB, tslot[rowc]);
      });
    }
  }
}

template <typename T, int E, int CW, bool PRE, bool TB>
__global__ void __launch_bounds__(64 * CW) k_ywinv(cx<T>* __restrict__ W, PassArgs a) {
  ywinv_body<T, E, CW, PRE, TB>(W, a, blockIdx.x);
}
template <typename T, int E, int CW, bool PRE, bool TB>
__global__ void __launch_bounds__(64 * CW) k_ywinv_g(GroupArgs g) {
  unsigned lin;
  bool live;
  const GroupEntry& e = group_entry(g, &lin, &live);
  if (!live) return;  // uniform over the workgroup, before any barrier
  ywinv_body<T, E, CW, PRE, TB>(static_cast<cx<T>*>(group_out(g, e)), e.a, lin);
}
template <typename T, int E, int CW, bool PRE, bool TB>
void launch_ywinv(const PassArgs& a, const void*, void* out, hipStream_t s) {
  hipLaunchKernelGGL((k_ywinv<T, E, CW, PRE, TB>), dim3(ypass_blocks<T, CW>(a)), dim3(64 * CW), 0, s,
                     static_cast<cx<T>*>(out), a);
}
template <typename T, int E, int CW, bool PRE, bool TB>
void launchg_ywinv(const GroupArgs& g, unsigned nblocks, hipStream_t s) {
  hipLaunchKernelGGL((k_ywinv_g<T, E, CW, PRE, TB>), dim3(nblocks), dim3(64 * CW), 0, s, g);
}

// P = E, Q = 64 (line length 64 E), tile = CW columns, nch = 0 marks the
// wave-per-line family; "_p" variants issue all their loads at the start,
// "_t" variants take the inverse twiddles from LDS tables.
#define YIWV(T, E, CW, SUF, PRE, TB)                                                              \
  PassVariant{PASS_YINV, is64<T>(), 64 * E, E, 64, CW, 0, 64 * CW, zwave_lds_bytes<T, E, CW, TB>(), \
              "yinv_" #T "_w" #E "_c" #CW SUF, &launch_ywinv<T, E, CW, PRE, TB>,                  \
              &launchg_ywinv<T, E, CW, PRE, TB>}
#define YIW(T, E, CW) YIWV(T, E, CW, "", false, false)
#define YIWP(T, E, CW) YIWV(T, E, CW, "_p", true, false)
#define YIWT(T, E, CW) YIWV(T, E, CW, "_pt", true, true)

}  // namespace ups
