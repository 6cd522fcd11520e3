// FFT pass kernels of the zero-padded free-space convolution (gfx950).
//
// Every length-L line transform is split L = P * Q (four-step): element
// n = q + Q p, frequency k = k1 + P k2.  A thread first runs length-P DFTs
// over p in registers, applies exp(DIR 2 pi i q k1 / L), hands the values to
// other threads through LDS, and those run length-Q DFTs over q.  Inverse
// transforms run the same steps mirrored.  With the zero padding, inputs
// n >= L/2 are zero (p >= P/2) so the first P-DFT skips its upper half; with
// the crop, outputs n >= L/2 are discarded so the last P-DFT computes only
// its lower half.
//
// Workgroup shapes: X passes (contiguous rows) put TL threads on each of RW
// rows, thread index = tl + TL r, so consecutive lanes touch consecutive
// elements of a row.  Y and Z passes (strided lines) put C adjacent columns
// on consecutive lanes, thread index = c + C tl, so every wave reads and
// writes C-element contiguous segments of several lines.
//
// LDS exchanges run in NCH phases, each over one group of rows (columns): a
// thread keeps its line data in registers until its group's phase, so the
// workgroup needs LDS for only RW/NCH rows (C/NCH columns) at a time and the
// register peak stays at one line share per thread.
#pragma once
#include "passes.hpp"
#include "dft.hpp"

namespace ups {

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }

// Line of length L = P Q over TL = gcd(P, Q) threads: each thread runs
// D1 = Q/TL DFTs of length P, then D3 = P/TL DFTs of length Q, and holds
// E = D1 P = D3 Q values.
template <int P, int Q>
struct Split {
  static constexpr int L = P * Q;
  static constexpr int TL = cgcd(P, Q);  // threads per line
  static constexpr int D1 = Q / TL;      // P-DFTs per thread
  static constexpr int D3 = P / TL;      // Q-DFTs per thread
  static constexpr int E = D1 * P;       // values per thread
  // twiddle runs are rows of the 64 x 64 product table
  static_assert(P <= 64 && Q <= 64, "line split factors must be <= 64");
};

// per-thread spectrum of a line: w[d3][k2] = X[k1 + P k2], k1 = tl + TL d3
template <typename T, int P, int Q>
using ColSpec = cx<T>[Split<P, Q>::D3][Q];

// Loads and stores at a wave-uniform base plus a 32-bit per-thread byte
// offset, so addresses need one vector register instead of a 64-bit pair.
// NT: a nontemporal access (see the cache hints below).
template <bool NT = false, typename T>
__device__ __forceinline__ cx<T> ld_cx(const cx<T>* p) {
  if constexpr (NT) {
    typedef T V2 __attribute__((ext_vector_type(2)));
    const V2 v = __builtin_nontemporal_load(reinterpret_cast<const V2*>(p));
    return cx<T>{v.x, v.y};
  } else {
    return *p;
  }
}
template <bool NT = false, typename T>
__device__ __forceinline__ void st_cx(cx<T>* p, cx<T> v) {
  if constexpr (NT) {
    typedef T V2 __attribute__((ext_vector_type(2)));
    const V2 w = {v.re, v.im};
    __builtin_nontemporal_store(w, reinterpret_cast<V2*>(p));
  } else {
    *p = v;
  }
}
template <bool NT = false, typename T>
__device__ __forceinline__ T ld_r(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT = false, typename T>
__device__ __forceinline__ void st_r(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}
template <bool NT = false, typename T>
__device__ __forceinline__ cx<T> ld_at(const cx<T>* ubase, unsigned byte_off) {
  return ld_cx<NT>(reinterpret_cast<const cx<T>*>(reinterpret_cast<const char*>(ubase) + byte_off));
}
template <bool NT = false, typename T>
__device__ __forceinline__ void st_at(cx<T>* ubase, unsigned byte_off, cx<T> v) {
  st_cx<NT>(reinterpret_cast<cx<T>*>(reinterpret_cast<char*>(ubase) + byte_off), v);
}

// Cache hints of the data sweeps.  Every pass reads its input and writes its
// output once, so those lines need not stay in L2; a nontemporal load or
// store says so, and leaves L2 to the twiddle rows and G_hat lines that
// several workgroups share.  Whether that pays differs per pass (it changes
// how reads and writes interleave at the memory controllers, and whether
// the next pass finds recent lines still cached), so it is set per pass from
// measurement: bit k of the load (store) mask marks pass k's data loads
// (stores), k = 0 xfwd, 1 yfwd, 2 zconv, 3 yinv, 4 xinv; bit 5 of the load
// mask marks the G_hat loads of the z pass, bit 6 the wave-per-line kernels
// of pass 4 and bit 7 those of pass 5 (bits 3 and 4 then cover the column
// and four-step kernels; for pass 5 the loads of bit 7 are those of the
// variant that takes mirrored values from LDS).  Measured on MI355X at
// 512^3 (FP32 and FP64): nontemporal loads and stores in both forward passes
// shorten them and the z pass after them, nontemporal loads and stores
// shorten the wave-per-line pass 4 and the x pass after it, and nontemporal
// stores shorten the wave-per-row pass 5 a little, as do nontemporal loads
// in its variant that reads each value once; every other hint slows the
// pass it is in or the one after (nontemporal stores in the four-step
// pass 5 slow the small solves of a batch by about 6%).
#ifndef UPS_NT_LOAD_MASK
#define UPS_NT_LOAD_MASK 0xC3
#endif
#ifndef UPS_NT_STORE_MASK
#define UPS_NT_STORE_MASK 0xC3
#endif
constexpr int kNtGhatBit = 5;
constexpr int kNtYinvWaveBit = 6;
constexpr int kNtXinvWaveBit = 7;  // wave-per-row pass 5: stores, and loads of the variant reading each value once
template <int K>
constexpr bool nt_load() { return ((UPS_NT_LOAD_MASK) >> K) & 1; }
template <int K>
constexpr bool nt_store() { return ((UPS_NT_STORE_MASK) >> K) & 1; }
// twiddle table entry exp(-2 pi i idx / M)
template <typename T>
__device__ __forceinline__ cx<T> tw_at(const cx<T>* tw, unsigned idx) {
  return ld_at(tw, idx * unsigned(sizeof(cx<T>)));
}
// Row a of the product block that follows the M entries of a twiddle table:
// row[b] = exp(-2 pi i (a b mod M) / M) for a, b < kTw2Row.
constexpr int kTw2Row = 64;
template <typename T>
__device__ __forceinline__ const cx<T>* tw_row(const cx<T>* tw, int M, unsigned a) {
  return tw + M + a * unsigned(kTw2Row);
}

// v[k] *= w^(k x) (conjugated if CONJ) for k = 1 .. K-1, given pw(j) =
// w^(2^j x): the other powers are products of earlier ones (k = 2^j + r,
// w^(k x) = w^(2^j x) w^(r x)), so a run of K - 1 twiddles costs
// ceil(log2 K) table loads and a few products (error a few ulp).
template <int K, bool CONJ, typename T, typename PW>
__device__ __forceinline__ void twiddle_run(cx<T>* v, PW pw) {
  cx<T> p[K];
  static_for<1, K>([&](auto kk) {
    constexpr int k = decltype(kk)::value;
    constexpr int hb = 1 << (31 - __builtin_clz(k));   // largest power of two <= k
    if constexpr (hb == k) {
      p[k] = pw(31 - __builtin_clz(k));
    } else {
      p[k] = cmul(p[hb], p[k - hb]);
    }
    v[k] = CONJ ? cmulc(v[k], p[k]) : cmul(v[k], p[k]);
  });
}

template <typename T>
__device__ __forceinline__ cx<T> zero_c() { return cx<T>{T(0), T(0)}; }

// forward P-DFT of a line whose upper half is zero (P even), or a full DFT
template <int P, int DIR, typename T>
__device__ __forceinline__ void first_dft(cx<T>* v) {
  if constexpr (P % 2 == 0) dft_half_in<P, DIR>(v);
  else dft<P, DIR>(v);
}
template <int P, int DIR, typename T>
__device__ __forceinline__ void last_dft(cx<T>* v) {
  if constexpr (P % 2 == 0) dft_half_out<P, DIR>(v);
  else dft<P, DIR>(v);
}
template <int P>
constexpr int live_in() { return P % 2 == 0 ? P / 2 : P; }


// ============================================================================
// Pass 1: zero-pad + real-to-complex DFT along x (contiguous rows).
// Row of nx reals, padded to mx = 2L, packed as z[m] = x[2m] + i x[2m+1]
// (length L), transformed, then untangled:
//   X[k] = (Z[k] + conj Z[L-k])/2 - (i/2) w^k (Z[k] - conj Z[L-k]),  k <= L.
// ============================================================================
template <int P, int Q>
constexpr int xfwd_row_stride() {
  constexpr int ys = P * (Q + 1), zs = P * Q + 1;
  return (ys > zs ? ys : zs) | 1;
}

// FILL: an even or odd direction (a.fill_x = +1 or -1, nx = L, nx even):
// the extended row x[2 nx - 1 - n] = +-x[n] packs to z[m] = +-swap(z[L-1-m])
// for m >= L/2, which the threads load instead of the zero padding; the
// first stage is then a full DFT.
template <typename T, int P, int Q, int RW, int NCH, bool FILL = false>
__device__ __forceinline__ void xfwd_body(const T* __restrict__ f, cx<T>* __restrict__ W, const PassArgs& a,
                                          unsigned bx, unsigned by) {
  using S = Split<P, Q>;
  constexpr int L = S::L, TL = S::TL, RG = RW / NCH;
  constexpr int RS = xfwd_row_stride<P, Q>();
  static_assert(RW % NCH == 0, "row groups");
  static_assert(2 * (P - 1) < kTw2Row, "twiddle run w_M^(2 q k1) must fit a table row");
  __shared__ cx<T> lds[RG * RS];

  const int tid = threadIdx.x;
  const int tl = tid % TL, r = tid / TL;
  const long long row = (long long)bx * RW + r;
  const int comp = int(by);
  const long long nrows = (long long)a.ny * a.nz;
  const bool valid = row < nrows;
  const long long rowc = valid ? row : nrows - 1;  // in-bounds row for the loads
  const int y = int(rowc % a.ny);
  const int z = int(rowc / a.ny);
  const T* src = f + comp * a.comp_f + rowc * a.nx;
  cx<T>* dst = W + comp * a.comp_w + z * a.plane + (long long)y * a.px;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_x);  // length mx = 2L
  cx<T>* my = lds + (r % RG) * RS;
  const int nx = a.nx;
  const bool even_nx = (nx & 1) == 0;
  // every loaded pair 2m, 2m+1 (m < Q live_in<P>) lies inside the row
  const bool full = even_nx && nx >= 2 * Q * live_in<P>();

  cx<T> v[S::D1][P];
  static_for<0, S::D1>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int q = tl + TL * d;
    if (full) {
      static_for<0, live_in<P>()>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        v[d][p] = ld_cx<nt_load<0>()>(reinterpret_cast<const cx<T>*>(src + 2 * (q + Q * p)));
      });
    } else {
      static_for<0, live_in<P>()>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        const int m = q + Q * p;  // packed index: reals 2m, 2m+1
        cx<T> val = zero_c<T>();
        if (even_nx) {
          if (2 * m < nx) val = ld_cx<nt_load<0>()>(reinterpret_cast<const cx<T>*>(src + 2 * m));
        } else {
          if (2 * m < nx) val.re = ld_r<nt_load<0>()>(src + 2 * m);
          if (2 * m + 1 < nx) val.im = ld_r<nt_load<0>()>(src + 2 * m + 1);
        }
        v[d][p] = val;
      });
    }
    if constexpr (FILL) {
      static_assert(P % 2 == 0, "mirrored rows need an even split");
      const T sg = T(a.fill_x);
      static_for<P / 2, P>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        const int mq = L - 1 - (q + Q * p);
        const cx<T> zv = ld_cx<nt_load<0>()>(reinterpret_cast<const cx<T>*>(src + 2 * mq));
        v[d][p] = cx<T>{sg * zv.im, sg * zv.re};
      });
      dft<P, -1>(v[d]);
    } else {
      first_dft<P, -1>(v[d]);
    }
    const cx<T>* trow = tw_row(tw, 2 * L, unsigned(q));
    // w_L^{q k1} = w_M^{2 q k1}
    twiddle_run<P, false>(v[d], [&](int j) { return trow[2 << j]; });
  });
  static_for<0, NCH>([&](auto hh) {
    constexpr int h = decltype(hh)::value;
    const bool mine = r / RG == h;
    if constexpr (h > 0) __syncthreads();
    if (mine) {
      static_for<0, S::D1>([&](auto dd) {
        constexpr int d = decltype(dd)::value;
        const int q = tl + TL * d;
        static_for<0, P>([&](auto kk) {
          constexpr int k1 = decltype(kk)::value;
          my[k1 * (Q + 1) + q] = v[d][k1];
        });
      });
    }
    __syncthreads();
    ColSpec<T, P, Q> w;
    if (mine) {
      static_for<0, S::D3>([&](auto dd) {
        constexpr int d = decltype(dd)::value;
        const int k1 = tl + TL * d;
        static_for<0, Q>([&](auto qq) {
          constexpr int q = decltype(qq)::value;
          w[d][q] = my[k1 * (Q + 1) + q];
        });
        dft<Q, -1>(w[d]);
      });
    }
    __syncthreads();
    if (mine) {
      static_for<0, S::D3>([&](auto dd) {
        constexpr int d = decltype(dd)::value;
        const int k1 = tl + TL * d;
        static_for<0, Q>([&](auto kk) {
          constexpr int k2 = decltype(kk)::value;
          my[k1 + P * k2] = w[d][k2];
        });
      });
    }
    __syncthreads();
    if (mine && valid) {
      const cx<T> wtl = tw_at(tw, unsigned(tl));
      // k = tl + TL i for i < L/TL, then k = L on lane tl = 0
      static_for<0, L / TL + 1>([&](auto ii) {
        constexpr int i = decltype(ii)::value;
        const int k = tl + TL * i;
        if (i < L / TL || tl == 0) {
          const int kk = i < L / TL ? k : L;
          const cx<T> zk = my[kk == L ? 0 : kk];
          const cx<T> zm = conj(my[kk == 0 ? 0 : L - kk]);
          const cx<T> e = scale(zk + zm, T(0.5));
          const cx<T> o = scale(mul_i<-1>(zk - zm), T(0.5));  // (Z - conj Z')/(2i)
          // w_M^kk = w_M^tl w_M^(TL i) (kk = L: w_M^L = -i... as a constant)
          const cx<T> wk = i < L / TL ? twiddle_c<(long long)TL * i, 2 * L, -1>(wtl)
                                      : twiddle_c<(long long)L, 2 * L, -1>(cx<T>{T(1), T(0)});
          st_cx<nt_store<0>()>(dst + kk, e + cmul(o, wk));
        }
      });
    }
  });
}

// ============================================================================
// Pass 5: complex-to-real inverse DFT along x + crop to x < nx.
//   Z[k] = (X[k] + conj X[L-k]) + i w^{-k} (X[k] - conj X[L-k]),  k < L,
// inverse length-L DFT of Z gives u[2m] + i u[2m+1] (unnormalised).
// ============================================================================
template <int P, int Q>
constexpr int xinv_row_stride() { return (Q * (P + 1)) | 1; }

template <typename T, int P, int Q, int RW, int NCH>
__device__ __forceinline__ void xinv_body(const cx<T>* __restrict__ W, T* __restrict__ u, const PassArgs& a,
                                          unsigned bx, unsigned by) {
  using S = Split<P, Q>;
  constexpr int L = S::L, TL = S::TL, RG = RW / NCH;
  constexpr int VS = xinv_row_stride<P, Q>();
  static_assert(RW % NCH == 0, "row groups");
  static_assert(2 * (Q - 1) < kTw2Row, "twiddle run w_M^(2 k1 n2) must fit a table row");
  __shared__ cx<T> lds[RG * VS];

  const int tid = threadIdx.x;
  const int tl = tid % TL, r = tid / TL;
  const long long row = (long long)bx * RW + r;
  const int comp = int(by);
  const long long nrows = (long long)a.ny * a.nz;
  const bool valid = row < nrows;
  const long long rowc = valid ? row : nrows - 1;  // in-bounds row for the loads
  const int y = int(rowc % a.ny);
  const int z = int(rowc / a.ny);
  const cx<T>* src = W + comp * a.comp_w + z * a.plane + (long long)y * a.px;
  T* dst = u + comp * a.comp_f + row * a.nx;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_x);
  cx<T>* my = lds + (r % RG) * VS;

  ColSpec<T, P, Q> w;
  static_for<0, S::D3>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int k1 = tl + TL * d;
    const cx<T> wk1 = tw_at(tw, unsigned(k1));
    static_for<0, Q>([&](auto kk) {
      constexpr int k2 = decltype(kk)::value;
      const int k = k1 + P * k2;
      const cx<T> xk = ld_cx<nt_load<4>()>(src + k);
      const cx<T> xm = conj(ld_cx<nt_load<4>()>(src + (L - k)));
      // conj w_M^k = conj w_M^k1 conj w_M^(P k2)
      w[d][k2] = (xk + xm) + mul_i<+1>(twiddle_c<(long long)P * k2, 2 * L, +1>(cmulc(xk - xm, wk1)));
    });
    dft<Q, +1>(w[d]);
    const cx<T>* trow = tw_row(tw, 2 * L, unsigned(k1));
    twiddle_run<Q, true>(w[d], [&](int j) { return trow[2 << j]; });
  });
  const int nx = a.nx;
  const bool even_nx = (nx & 1) == 0;
  // every stored pair 2m, 2m+1 (m < Q live_in<P>) lies inside the row
  const bool full = even_nx && nx >= 2 * Q * live_in<P>();
  static_for<0, NCH>([&](auto hh) {
    constexpr int h = decltype(hh)::value;
    const bool mine = r / RG == h;
    if constexpr (h > 0) __syncthreads();
    if (mine) {
      static_for<0, S::D3>([&](auto dd) {
        constexpr int d = decltype(dd)::value;
        const int k1 = tl + TL * d;
        static_for<0, Q>([&](auto nn) {
          constexpr int n2 = decltype(nn)::value;
          my[n2 * (P + 1) + k1] = w[d][n2];
        });
      });
    }
    __syncthreads();
    if (mine) {
      static_for<0, S::D1>([&](auto dd) {
        constexpr int d = decltype(dd)::value;
        const int n2 = tl + TL * d;
        cx<T> v[P];
        static_for<0, P>([&](auto kk) {
          constexpr int k1 = decltype(kk)::value;
          v[k1] = my[n2 * (P + 1) + k1];
        });
        last_dft<P, +1>(v);
        if (valid) {
          if (full) {
            static_for<0, live_in<P>()>([&](auto nn) {
              constexpr int n1 = decltype(nn)::value;
              st_cx<nt_store<4>()>(reinterpret_cast<cx<T>*>(dst + 2 * (n2 + Q * n1)), v[n1]);
            });
          } else {
            static_for<0, live_in<P>()>([&](auto nn) {
              constexpr int n1 = decltype(nn)::value;
              const int m = n2 + Q * n1;
              if (even_nx) {
                if (2 * m < nx) st_cx<nt_store<4>()>(reinterpret_cast<cx<T>*>(dst + 2 * m), v[n1]);
              } else {
                if (2 * m < nx) st_r<nt_store<4>()>(dst + 2 * m, v[n1].re);
                if (2 * m + 1 < nx) st_r<nt_store<4>()>(dst + 2 * m + 1, v[n1].im);
              }
            });
          }
        }
      });
    }
  });
}

// ============================================================================
// Column passes.  Thread (c, tl): c = column in the tile, tl = position on
// the line.  A workgroup's lines start at a wave-uniform base (the tile's
// first column); each element address is that base plus a multiple of the
// line stride that is uniform across the wave plus one 32-bit per-thread
// byte offset.  Exchanges go through LDS laid out [k1][q (+1 pad)][c'] for
// the CG = C/NCH columns c' of the current phase.
// ============================================================================

// Forward step on lines of length M = P Q with inputs n < nlive (n = q + Q p,
// p < P/2 when P is even).  ubase = element 0 of the tile's first column,
// elements of a line `stride` apart.  Leaves w[d3][k2] = X[k1 + P k2],
// k1 = tl + TL d3.
// TWP: a thread's twiddle run from log2 table loads and products (fewer
// loads, more VALU) instead of one table load per twiddle.
// FILL: an even or odd direction (nlive = M/2, fill_sign = +1 or -1): rows
// n >= M/2 are fill_sign times row M - 1 - n, loaded instead of the zero
// padding, and the first stage is a full DFT.
template <typename T, int P, int Q, int C, int NCH, bool TWP, bool NTL, bool FILL = false>
__device__ __forceinline__ void col_forward(const cx<T>* ubase, long long stride, int cload, int nlive,
                                            const cx<T>* tw, cx<T>* lds, int c, int tl,
                                            ColSpec<T, P, Q>& w, T fill_sign = T(0)) {
  using S = Split<P, Q>;
  constexpr int TL = S::TL, CG = C / NCH;
  constexpr unsigned CB = sizeof(cx<T>);
  // One register buffer holds the step-1 lines (D1 x P) and, after the
  // exchange, the step-3 lines (D3 x Q): a thread's values are overwritten
  // in place in its own phase, so both layouts share registers.
  cx<T>* buf = &w[0][0];
  static_for<0, S::D1>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int q = tl + TL * d;
    cx<T>* v = buf + d * P;
    const unsigned toff = (unsigned(q) * unsigned(stride) + unsigned(cload)) * CB;
    if (nlive >= Q * live_in<P>()) {  // every loaded row is live (the zero-padded case)
      static_for<0, live_in<P>()>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        v[p] = ld_at<NTL>(ubase + (long long)(Q * p) * stride, toff);
      });
    } else {
      static_for<0, live_in<P>()>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        v[p] = q + Q * p < nlive ? ld_at<NTL>(ubase + (long long)(Q * p) * stride, toff) : zero_c<T>();
      });
    }
    if constexpr (FILL) {
      static_assert(P % 2 == 0, "mirrored rows need an even split");
      static_for<P / 2, P>([&](auto pp) {
        constexpr int p = decltype(pp)::value;
        const int mr = P * Q - 1 - (q + Q * p);  // < M/2
        v[p] = scale(ld_at<NTL>(ubase + (long long)mr * stride, unsigned(cload) * CB), fill_sign);
      });
      dft<P, -1>(v);
    } else {
      first_dft<P, -1>(v);
    }
    const cx<T>* trow = tw_row(tw, S::L, unsigned(q));
    if constexpr (TWP) {
      twiddle_run<P, false>(v, [&](int j) { return trow[1 << j]; });
    } else {
      static_for<1, P>([&](auto kk) {
        constexpr int k1 = decltype(kk)::value;
        v[k1] = cmul(v[k1], trow[k1]);
      });
    }
  });
  const int cl = c % CG;
  static_for<0, NCH>([&](auto hh) {
    constexpr int h = decltype(hh)::value;
    const bool mine = c / CG == h;
    if constexpr (h > 0) __syncthreads();
    if (mine) {
      static_for<0, S::D1>([&](auto dd) {
        constexpr int d = decltype(dd)::value;
        const int q = tl + TL * d;
        static_for<0, P>([&](auto kk) {
          constexpr int k1 = decltype(kk)::value;
          lds[(k1 * (Q + 1) + q) * CG + cl] = buf[d * P + k1];
        });
      });
    }
    __syncthreads();
    if (mine) {
      static_for<0, S::D3>([&](auto dd) {
        constexpr int d = decltype(dd)::value;
        const int k1 = tl + TL * d;
        static_for<0, Q>([&](auto qq) {
          constexpr int q = decltype(qq)::value;
          buf[d * Q + q] = lds[(k1 * (Q + 1) + q) * CG + cl];
        });
      });
    }
  });
  static_for<0, S::D3>([&](auto dd) { dft<Q, -1>(w[decltype(dd)::value]); });
}

// Inverse step: per thread w[d3][k2] = X[k1 + P k2] (k1 = tl + TL d3) in,
// stores x[n2 + Q n1] for n1 < P/2 (n2 = tl + TL d1) where n < nkeep.
// Starts with a barrier (the LDS may still be read by a previous phase).
template <typename T, int P, int Q, int C, int NCH, bool TWP, bool NTS>
__device__ __forceinline__ void col_inverse(ColSpec<T, P, Q>& w, cx<T>* ubase, long long stride, bool valid,
                                            int nkeep, const cx<T>* tw, cx<T>* lds, int c, int tl) {
  using S = Split<P, Q>;
  constexpr int TL = S::TL, CG = C / NCH;
  constexpr unsigned CB = sizeof(cx<T>);
  cx<T>* buf = &w[0][0];
  static_for<0, S::D3>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int k1 = tl + TL * d;
    dft<Q, +1>(w[d]);
    const cx<T>* trow = tw_row(tw, S::L, unsigned(k1));
    if constexpr (TWP) {
      twiddle_run<Q, true>(w[d], [&](int j) { return trow[1 << j]; });
    } else {
      static_for<1, Q>([&](auto nn) {
        constexpr int n2 = decltype(nn)::value;
        w[d][n2] = cmulc(w[d][n2], trow[n2]);
      });
    }
  });
  const int cl = c % CG;
  static_for<0, NCH>([&](auto hh) {
    constexpr int h = decltype(hh)::value;
    const bool mine = c / CG == h;
    __syncthreads();
    if (mine) {
      static_for<0, S::D3>([&](auto dd) {
        constexpr int d = decltype(dd)::value;
        const int k1 = tl + TL * d;
        static_for<0, Q>([&](auto nn) {
          constexpr int n2 = decltype(nn)::value;
          lds[(n2 * (P + 1) + k1) * CG + cl] = buf[d * Q + n2];
        });
      });
    }
    __syncthreads();
    if (mine) {
      static_for<0, S::D1>([&](auto dd) {
        constexpr int d = decltype(dd)::value;
        const int n2 = tl + TL * d;
        static_for<0, P>([&](auto kk) {
          constexpr int k1 = decltype(kk)::value;
          buf[d * P + k1] = lds[(n2 * (P + 1) + k1) * CG + cl];
        });
      });
    }
  });
  static_for<0, S::D1>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int n2 = tl + TL * d;
    cx<T>* v = buf + d * P;
    last_dft<P, +1>(v);
    if (valid) {
      const unsigned toff = (unsigned(n2) * unsigned(stride) + unsigned(c)) * CB;
      static_for<0, live_in<P>()>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        cx<T>* bp = ubase + (long long)(Q * n1) * stride;
        if (n2 + Q * n1 < nkeep) st_at<NTS>(bp, toff, v[n1]);
      });
    }
  });
}

template <int P, int Q, int C, int NCH>
constexpr int col_lds_elems() {
  constexpr int a = P * (Q + 1) * (C / NCH);
  constexpr int b = Q * (P + 1) * (C / NCH);
  return a > b ? a : b;
}

// Block orders of the column passes.  Consecutive linear block ids go
// round-robin to the eight XCDs, each with its own L2.  A tile of C columns
// may cover only part of a 128-byte line (C = 8 float columns = 64 bytes), so
// the H = (128 B / element) / C tiles of one line are made "slots" of one
// group, with linear ids 8 apart: same XCD, close in time, so the line is
// fetched from HBM once.  The z pass adds to the group every workgroup that
// reads the same G_hat octant line (ky = iy and my - iy, every component).
template <typename T, int C>
constexpr int tile_slots() {
  constexpr int per_line = 128 / int(sizeof(cx<T>));
  return per_line > C ? per_line / C : 1;
}

// Slots per group, capped by the number of tiles: a launch over a few
// columns (the remainder of an aligned split) gets no empty slots.
template <typename T, int C>
__host__ __device__ inline int col_slots(int ntiles) {
  constexpr int h = tile_slots<T, C>();
  return h > ntiles ? ntiles : h;
}

struct ColMap {
  int tile, line, comp;   // line = z (y passes) or ky (z pass)
  bool active;
};

// y passes: groups (tile group, z, comp), slots = tile within the group
__device__ __forceinline__ ColMap ymap(unsigned b, int ntiles, int nz, int ncomp, int H) {
  const unsigned x = b % 8u, rest = b / 8u;
  const int slot = int(rest % unsigned(H));
  const unsigned g = (rest / unsigned(H)) * 8u + x;
  const unsigned ntg = unsigned((ntiles + H - 1) / H);
  ColMap m;
  m.active = g < ntg * unsigned(nz) * unsigned(ncomp);
  const unsigned tg = g % ntg, r = g / ntg;
  m.line = int(r % unsigned(nz));
  m.comp = int(r / unsigned(nz));
  m.tile = int(tg) * H + slot;
  if (m.tile >= ntiles) m.active = false;
  return m;
}
__host__ __device__ inline unsigned ymap_blocks(int ntiles, int nz, int ncomp, int H) {
  const long long groups = (long long)((ntiles + H - 1) / H) * nz * ncomp;
  return unsigned((groups + 7) / 8 * 8 * H);
}

// z pass: groups (tile group, iy), slots = (tile in group, side, comp)
__device__ __forceinline__ ColMap zmap(unsigned b, int ntiles, int my, int ncomp, int H) {
  const int slots = H * 2 * ncomp;
  const unsigned x = b % 8u, rest = b / 8u;
  const int slot = int(rest % unsigned(slots));
  const unsigned g = (rest / unsigned(slots)) * 8u + x;
  const int oy = my / 2 + 1;
  const unsigned ntg = unsigned((ntiles + H - 1) / H);
  ColMap m;
  m.active = g < ntg * unsigned(oy);
  const int iy = int(g / ntg);
  const int half = slot % H, side = (slot / H) & 1;
  m.comp = slot / (2 * H);
  m.tile = int(g % ntg) * H + half;
  m.line = side ? my - iy : iy;
  if (m.tile >= ntiles) m.active = false;
  if (side && (iy == 0 || 2 * iy == my)) m.active = false;  // self-mirrored line
  return m;
}
__host__ __device__ inline unsigned zmap_blocks(int ntiles, int my, int ncomp, int H) {
  const long long groups = (long long)((ntiles + H - 1) / H) * (my / 2 + 1);
  return unsigned((groups + 7) / 8 * 8 * H * 2 * ncomp);
}

// Pass 2: DFT along y, rows y < ny live, all my outputs kept (in place).
template <typename T, int P, int Q, int C, int NCH, bool FILL = false>
__device__ __forceinline__ void yfwd_body(cx<T>* __restrict__ W, const PassArgs& a, unsigned blin) {
  using S = Split<P, Q>;
  static_assert(C % NCH == 0, "column groups");
  __shared__ cx<T> lds[col_lds_elems<P, Q, C, NCH>()];
  const int tid = threadIdx.x;
  const int c = tid % C, tl = tid / C;
  const ColMap mp = ymap(blin, (a.kx + C - 1) / C, a.nz, a.ncomp, col_slots<T, C>((a.kx + C - 1) / C));
  if (!mp.active) return;  // uniform over the workgroup, before any barrier
  const int kx0 = mp.tile * C;
  const int z = mp.line, comp = mp.comp;
  const bool valid = kx0 + c < a.kx;
  const int cload = valid ? c : a.kx - 1 - kx0;  // in-bounds column for the loads
  cx<T>* ubase = W + comp * a.comp_w + z * a.plane + kx0;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_y);
  ColSpec<T, P, Q> w;
  col_forward<T, P, Q, C, NCH, false, nt_load<1>(), FILL>(ubase, a.px, cload, a.ny, tw, lds, c, tl, w,
                                                           T(a.fill_y));
  if (valid) {
    static_for<0, S::D3>([&](auto dd) {
      constexpr int d = decltype(dd)::value;
      const int k1 = tl + S::TL * d;
      const unsigned toff = (unsigned(k1) * unsigned(a.px) + unsigned(c)) * unsigned(sizeof(cx<T>));
      static_for<0, Q>([&](auto kk) {
        constexpr int k2 = decltype(kk)::value;
        st_at<nt_store<1>()>(ubase + (long long)(P * k2) * a.px, toff, w[d][k2]);
      });
    });
  }
}

// Pass 4: inverse DFT along y, all my rows in, rows y < ny kept (in place).
template <typename T, int P, int Q, int C, int NCH>
__device__ __forceinline__ void yinv_body(cx<T>* __restrict__ W, const PassArgs& a, unsigned blin) {
  using S = Split<P, Q>;
  static_assert(C % NCH == 0, "column groups");
  __shared__ cx<T> lds[col_lds_elems<P, Q, C, NCH>()];
  const int tid = threadIdx.x;
  const int c = tid % C, tl = tid / C;
  const ColMap mp = ymap(blin, (a.kx + C - 1) / C, a.nz, a.ncomp, col_slots<T, C>((a.kx + C - 1) / C));
  if (!mp.active) return;  // uniform over the workgroup, before any barrier
  const int kx0 = mp.tile * C;
  const int z = mp.line, comp = mp.comp;
  const bool valid = kx0 + c < a.kx;
  const int cload = valid ? c : a.kx - 1 - kx0;
  cx<T>* ubase = W + comp * a.comp_w + z * a.plane + kx0;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_y);
  ColSpec<T, P, Q> w;
  static_for<0, S::D3>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int k1 = tl + S::TL * d;
    const unsigned toff = (unsigned(k1) * unsigned(a.px) + unsigned(cload)) * unsigned(sizeof(cx<T>));
    static_for<0, Q>([&](auto kk) {
      constexpr int k2 = decltype(kk)::value;
      w[d][k2] = ld_at<nt_load<3>()>(ubase + (long long)(P * k2) * a.px, toff);
    });
  });
  col_inverse<T, P, Q, C, NCH, false, nt_store<3>()>(w, ubase, a.px, valid, a.ny, tw, lds, c, tl);
}

// Pass 3: along z, forward DFT (z < nz live), times G_hat, inverse DFT, keep
// z < nz; in place.  One workgroup per (column tile, ky, component).
template <typename T, int P, int Q, int C, int NCH, bool FILL = false>
__device__ __forceinline__ void zconv_body(cx<T>* __restrict__ W, const PassArgs& a, unsigned bx) {
  using S = Split<P, Q>;
  constexpr int M = S::L;
  static_assert(C % NCH == 0, "column groups");
  __shared__ cx<T> lds[col_lds_elems<P, Q, C, NCH>()];
  const int ntiles = (a.kx + C - 1) / C;
  const ColMap mp = zmap(bx, ntiles, a.my, a.ncomp, col_slots<T, C>(ntiles));
  if (!mp.active) return;  // uniform over the workgroup, before any barrier
  const int tid = threadIdx.x;
  const int c = tid % C, tl = tid / C;
  const int kx0 = mp.tile * C;
  const int ky = mp.line;
  const bool valid = kx0 + c < a.kx;
  const int iy = ky <= a.my - ky ? ky : a.my - ky;
  const T* gbase = static_cast<const T*>(a.ghat) + iy * a.g_plane + (long long)kx0 * a.gz;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_z);
  const int cload = valid ? c : a.kx - 1 - kx0;
  cx<T>* ubase = W + mp.comp * a.comp_w + (long long)ky * a.px + kx0;
  ColSpec<T, P, Q> w;
  col_forward<T, P, Q, C, NCH, true, nt_load<2>(), FILL>(ubase, a.plane, cload, a.nz, tw, lds, c, tl, w,
                                                          T(a.fill_z));
  static_for<0, S::D3>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int k1 = tl + S::TL * d;
    static_for<0, Q>([&](auto kk) {
      constexpr int k2 = decltype(kk)::value;
      const int kz = k1 + P * k2;
      const int iz = kz <= M - kz ? kz : M - kz;
      const unsigned goff = (unsigned(c) * unsigned(a.gz) + unsigned(iz)) * unsigned(sizeof(T));
      // (the branch also keeps the scheduler from hoisting these loads,
      // which would hold 32 more registers through the forward transform)
      const T g = valid ? ld_r<nt_load<kNtGhatBit>()>(reinterpret_cast<const T*>(reinterpret_cast<const char*>(gbase) + goff))
                        : T(0);
      w[d][k2] = scale(w[d][k2], g);
    });
  });
  col_inverse<T, P, Q, C, NCH, true, nt_store<2>()>(w, ubase, a.plane, valid, a.nz, tw, lds, c, tl);
}

// ============================================================================
// Entry points.  Single-problem kernels take PassArgs by value; grouped
// kernels run one pass for many problems in one launch: block b belongs to
// entry bmap[b] of the GroupEntry table, which holds that problem's
// PassArgs, buffers and first block (a multiple of 8, which keeps the z
// pass XCD mapping intact).
// ============================================================================
__host__ __device__ inline int cdiv(long long a, long long b) { return int((a + b - 1) / b); }

template <typename T, int C>
inline unsigned zconv_blocks(const PassArgs& a) {
  return zmap_blocks(cdiv(a.kx, C), a.my, a.ncomp, col_slots<T, C>(cdiv(a.kx, C)));
}
template <typename T, int C>
inline unsigned ypass_blocks(const PassArgs& a) {
  return ymap_blocks(cdiv(a.kx, C), a.nz, a.ncomp, col_slots<T, C>(cdiv(a.kx, C)));
}

// The problem of this block; *lin = block index inside the problem.  Blocks
// past the problem's own count (padding to a multiple of 8) return false.
__device__ __forceinline__ const GroupEntry& group_entry(const GroupArgs& g, unsigned* lin, bool* live) {
  const GroupEntry& e = g.ents[g.bmap[blockIdx.x]];
  *lin = blockIdx.x - e.block0;
  *live = *lin < e.nblocks;
  return e;
}
__device__ __forceinline__ const void* group_in(const GroupArgs& g, const GroupEntry& e) {
  return e.io_in >= 0 ? g.io[e.io_in] : e.in;
}
__device__ __forceinline__ void* group_out(const GroupArgs& g, const GroupEntry& e) {
  return e.io_out >= 0 ? const_cast<void*>(g.io[e.io_out]) : e.out;
}

template <typename T, int P, int Q, int RW, int NCH, bool FILL = false>
__global__ void __launch_bounds__((RW * Split<P, Q>::TL))
k_xfwd(const T* __restrict__ f, cx<T>* __restrict__ W, PassArgs a) {
  xfwd_body<T, P, Q, RW, NCH, FILL>(f, W, a, blockIdx.x, blockIdx.y);
}
template <typename T, int P, int Q, int RW, int NCH, bool FILL = false>
__global__ void __launch_bounds__((RW * Split<P, Q>::TL)) k_xfwd_g(GroupArgs g) {
  unsigned lin;
  bool live;
  const GroupEntry& e = group_entry(g, &lin, &live);
  if (!live) return;  // uniform over the workgroup, before any barrier
  const unsigned gx = unsigned(cdiv((long long)e.a.ny * e.a.nz, RW));
  xfwd_body<T, P, Q, RW, NCH, FILL>(static_cast<const T*>(group_in(g, e)), static_cast<cx<T>*>(group_out(g, e)),
                                    e.a, lin % gx, lin / gx);
}
template <typename T, int P, int Q, int RW, int NCH>
__global__ void __launch_bounds__((RW * Split<P, Q>::TL))
k_xinv(const cx<T>* __restrict__ W, T* __restrict__ u, PassArgs a) {
  xinv_body<T, P, Q, RW, NCH>(W, u, a, blockIdx.x, blockIdx.y);
}
template <typename T, int P, int Q, int RW, int NCH>
__global__ void __launch_bounds__((RW * Split<P, Q>::TL)) k_xinv_g(GroupArgs g) {
  unsigned lin;
  bool live;
  const GroupEntry& e = group_entry(g, &lin, &live);
  if (!live) return;  // uniform over the workgroup, before any barrier
  const unsigned gx = unsigned(cdiv((long long)e.a.ny * e.a.nz, RW));
  xinv_body<T, P, Q, RW, NCH>(static_cast<const cx<T>*>(group_in(g, e)), static_cast<T*>(group_out(g, e)), e.a,
                              lin % gx, lin / gx);
}
template <typename T, int P, int Q, int C, int NCH, bool FILL = false>
__global__ void __launch_bounds__((C * Split<P, Q>::TL)) k_yfwd(cx<T>* __restrict__ W, PassArgs a) {
  yfwd_body<T, P, Q, C, NCH, FILL>(W, a, blockIdx.x);
}
template <typename T, int P, int Q, int C, int NCH, bool FILL = false>
__global__ void __launch_bounds__((C * Split<P, Q>::TL)) k_yfwd_g(GroupArgs g) {
  unsigned lin;
  bool live;
  const GroupEntry& e = group_entry(g, &lin, &live);
  if (!live) return;  // uniform over the workgroup, before any barrier
  yfwd_body<T, P, Q, C, NCH, FILL>(static_cast<cx<T>*>(group_out(g, e)), e.a, lin);
}
template <typename T, int P, int Q, int C, int NCH>
__global__ void __launch_bounds__((C * Split<P, Q>::TL)) k_yinv(cx<T>* __restrict__ W, PassArgs a) {
  yinv_body<T, P, Q, C, NCH>(W, a, blockIdx.x);
}
template <typename T, int P, int Q, int C, int NCH>
__global__ void __launch_bounds__((C * Split<P, Q>::TL)) k_yinv_g(GroupArgs g) {
  unsigned lin;
  bool live;
  const GroupEntry& e = group_entry(g, &lin, &live);
  if (!live) return;  // uniform over the workgroup, before any barrier
  yinv_body<T, P, Q, C, NCH>(static_cast<cx<T>*>(group_out(g, e)), e.a, lin);
}
template <typename T, int P, int Q, int C, int NCH, bool FILL = false>
__global__ void __launch_bounds__((C * Split<P, Q>::TL)) k_zconv(cx<T>* __restrict__ W, PassArgs a) {
  zconv_body<T, P, Q, C, NCH, FILL>(W, a, blockIdx.x);
}
template <typename T, int P, int Q, int C, int NCH, bool FILL = false>
__global__ void __launch_bounds__((C * Split<P, Q>::TL)) k_zconv_g(GroupArgs g) {
  unsigned lin;
  bool live;
  const GroupEntry& e = group_entry(g, &lin, &live);
  if (!live) return;  // uniform over the workgroup, before any barrier
  zconv_body<T, P, Q, C, NCH, FILL>(static_cast<cx<T>*>(group_out(g, e)), e.a, lin);
}

template <typename T, int P, int Q, int RW, int NCH, bool FILL = false>
void launch_xfwd(const PassArgs& a, const void* in, void* out, hipStream_t s) {
  dim3 grid(cdiv((long long)a.ny * a.nz, RW), a.ncomp);
  hipLaunchKernelGGL((k_xfwd<T, P, Q, RW, NCH, FILL>), grid, dim3(RW * Split<P, Q>::TL), 0, s,
                     static_cast<const T*>(in), static_cast<cx<T>*>(out), a);
}
template <typename T, int P, int Q, int RW, int NCH>
void launch_xinv(const PassArgs& a, const void* in, void* out, hipStream_t s) {
  dim3 grid(cdiv((long long)a.ny * a.nz, RW), a.ncomp);
  hipLaunchKernelGGL((k_xinv<T, P, Q, RW, NCH>), grid, dim3(RW * Split<P, Q>::TL), 0, s,
                     static_cast<const cx<T>*>(in), static_cast<T*>(out), a);
}
template <typename T, int P, int Q, int C, int NCH, bool FILL = false>
void launch_yfwd(const PassArgs& a, const void*, void* out, hipStream_t s) {
  hipLaunchKernelGGL((k_yfwd<T, P, Q, C, NCH, FILL>), dim3(ypass_blocks<T, C>(a)), dim3(C * Split<P, Q>::TL), 0,
                     s, static_cast<cx<T>*>(out), a);
}
template <typename T, int P, int Q, int C, int NCH>
void launch_yinv(const PassArgs& a, const void*, void* out, hipStream_t s) {
  hipLaunchKernelGGL((k_yinv<T, P, Q, C, NCH>), dim3(ypass_blocks<T, C>(a)), dim3(C * Split<P, Q>::TL), 0, s,
                     static_cast<cx<T>*>(out), a);
}
template <typename T, int P, int Q, int C, int NCH, bool FILL = false>
void launch_zconv(const PassArgs& a, const void*, void* out, hipStream_t s) {
  hipLaunchKernelGGL((k_zconv<T, P, Q, C, NCH, FILL>), dim3(zconv_blocks<T, C>(a)), dim3(C * Split<P, Q>::TL), 0,
                     s, static_cast<cx<T>*>(out), a);
}
#define UPS_GROUPED_LAUNCHER(kname)                                                                   \
  template <typename T, int P, int Q, int B, int NCH>                                                  \
  void launchg_##kname(const GroupArgs& g, unsigned nblocks, hipStream_t s) {                         \
    hipLaunchKernelGGL((k_##kname##_g<T, P, Q, B, NCH>), dim3(nblocks), dim3(B * Split<P, Q>::TL), 0, s, g); \
  }
#define UPS_GROUPED_LAUNCHER_FILL(kname)                                                              \
  template <typename T, int P, int Q, int B, int NCH, bool FILL = false>                               \
  void launchg_##kname(const GroupArgs& g, unsigned nblocks, hipStream_t s) {                         \
    hipLaunchKernelGGL((k_##kname##_g<T, P, Q, B, NCH, FILL>), dim3(nblocks), dim3(B * Split<P, Q>::TL), 0, s, \
                       g);                                                                             \
  }
UPS_GROUPED_LAUNCHER_FILL(xfwd)
UPS_GROUPED_LAUNCHER(xinv)
UPS_GROUPED_LAUNCHER_FILL(yfwd)
UPS_GROUPED_LAUNCHER(yinv)
UPS_GROUPED_LAUNCHER_FILL(zconv)

template <typename T>
constexpr int is64() { return sizeof(T) == 8 ? 1 : 0; }

#define XF_VARIANT(T, P, Q, RW, NCH)                                                           \
  PassVariant{PASS_XFWD, is64<T>(), 2 * P * Q, P, Q, RW, NCH, RW * Split<P, Q>::TL,            \
              int(sizeof(cx<T>)) * (RW / NCH) * xfwd_row_stride<P, Q>(),                        \
              "xfwd_" #T "_" #P "x" #Q "_r" #RW "_h" #NCH, &launch_xfwd<T, P, Q, RW, NCH>,  \
              &launchg_xfwd<T, P, Q, RW, NCH>}
#define XI_VARIANT(T, P, Q, RW, NCH)                                                           \
  PassVariant{PASS_XINV, is64<T>(), 2 * P * Q, P, Q, RW, NCH, RW * Split<P, Q>::TL,            \
              int(sizeof(cx<T>)) * (RW / NCH) * xinv_row_stride<P, Q>(),                        \
              "xinv_" #T "_" #P "x" #Q "_r" #RW "_h" #NCH, &launch_xinv<T, P, Q, RW, NCH>,  \
              &launchg_xinv<T, P, Q, RW, NCH>}
#define X_VARIANTS(T, P, Q, RW, NCH) XF_VARIANT(T, P, Q, RW, NCH), XI_VARIANT(T, P, Q, RW, NCH)

#define COL_VARIANT(KIND, kname, T, P, Q, C, NCH)                                              \
  PassVariant{KIND, is64<T>(), P * Q, P, Q, C, NCH, C * Split<P, Q>::TL,                       \
              int(sizeof(cx<T>)) * col_lds_elems<P, Q, C, NCH>(),                               \
              #kname "_" #T "_" #P "x" #Q "_c" #C "_h" #NCH, &launch_##kname<T, P, Q, C, NCH>, \
              &launchg_##kname<T, P, Q, C, NCH>}
#define COL_VARIANTS(T, P, Q, C, NCH)                                                          \
  COL_VARIANT(PASS_YFWD, yfwd, T, P, Q, C, NCH), COL_VARIANT(PASS_ZCONV, zconv, T, P, Q, C, NCH), \
      COL_VARIANT(PASS_YINV, yinv, T, P, Q, C, NCH)

// Forward passes for even and odd directions (mirrored second half, full
// first stage): one per padded length, named with the suffix "_e".
#define XF_FILL(T, P, Q, RW, NCH)                                                              \
  PassVariant{PASS_XFWD, is64<T>(), 2 * P * Q, P, Q, RW, NCH, RW * Split<P, Q>::TL,            \
              int(sizeof(cx<T>)) * (RW / NCH) * xfwd_row_stride<P, Q>(),                        \
              "xfwd_" #T "_" #P "x" #Q "_r" #RW "_h" #NCH "_e", &launch_xfwd<T, P, Q, RW, NCH, true>, \
              &launchg_xfwd<T, P, Q, RW, NCH, true>, 1}
#define COL_FILL(KIND, kname, T, P, Q, C, NCH)                                                 \
  PassVariant{KIND, is64<T>(), P * Q, P, Q, C, NCH, C * Split<P, Q>::TL,                       \
              int(sizeof(cx<T>)) * col_lds_elems<P, Q, C, NCH>(),                               \
              #kname "_" #T "_" #P "x" #Q "_c" #C "_h" #NCH "_e", &launch_##kname<T, P, Q, C, NCH, true>, \
              &launchg_##kname<T, P, Q, C, NCH, true>, 1}
#define YF_FILL(T, P, Q, C, NCH) COL_FILL(PASS_YFWD, yfwd, T, P, Q, C, NCH)
#define ZC_FILL(T, P, Q, C, NCH) COL_FILL(PASS_ZCONV, zconv, T, P, Q, C, NCH)
#define FILL_VARIANTS(T, XP, XQ, XRW, XNCH, YP, YQ, YC, YNCH, ZP, ZQ, ZC, ZNCH) \
  XF_FILL(T, XP, XQ, XRW, XNCH), YF_FILL(T, YP, YQ, YC, YNCH), ZC_FILL(T, ZP, ZQ, ZC, ZNCH)

#define XF(T, P, Q, RW, NCH) XF_VARIANT(T, P, Q, RW, NCH)
#define XI(T, P, Q, RW, NCH) XI_VARIANT(T, P, Q, RW, NCH)
#define YF(T, P, Q, C, NCH) COL_VARIANT(PASS_YFWD, yfwd, T, P, Q, C, NCH)
#define ZC(T, P, Q, C, NCH) COL_VARIANT(PASS_ZCONV, zconv, T, P, Q, C, NCH)
#define YI(T, P, Q, C, NCH) COL_VARIANT(PASS_YINV, yinv, T, P, Q, C, NCH)

std::vector<PassVariant> variants_f32_pow2();
std::vector<PassVariant> variants_f32_mixed();
std::vector<PassVariant> variants_f64();

}  // namespace ups
