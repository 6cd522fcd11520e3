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
#include "passes.hpp"
#include "dft.hpp"

namespace ups {

template <int P, int Q>
struct Split {
  static constexpr int E = P > Q ? P : Q;
  static constexpr int L = P * Q;
  static constexpr int TL = L / E;   // threads per line
  static constexpr int D1 = Q / TL;  // P-DFTs per thread
  static constexpr int D3 = P / TL;  // Q-DFTs per thread
  static_assert(D1 * TL == Q && D3 * TL == P, "P must divide Q or Q divide P");
};

// per-thread spectrum of a column line: w[d3][k2] = X[k1 + P k2], k1 = tl + TL d3
template <typename T, int P, int Q>
using ColSpec = cx<T>[Split<P, Q>::D3][Q];

template <typename T>
__device__ __forceinline__ cx<T> ldg(const cx<T>* p) { return *p; }

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
template <typename T, int P, int Q, int RW>
__global__ void __launch_bounds__((RW * Split<P, Q>::TL))
k_xfwd(const T* __restrict__ f, cx<T>* __restrict__ W, PassArgs a) {
  using S = Split<P, Q>;
  constexpr int L = S::L, TL = S::TL;
  constexpr int YS = P * (Q + 1);
  constexpr int ZS = L + 1;
  constexpr int RS = (YS > ZS ? YS : ZS) | 1;
  __shared__ cx<T> lds[RW * RS];

  const int tid = threadIdx.x;
  const int tl = tid % TL, r = tid / TL;
  const long long row = (long long)blockIdx.x * RW + r;
  const int comp = blockIdx.y;
  const long long nrows = (long long)a.ny * a.nz;
  const bool valid = row < nrows;
  const int y = valid ? int(row % a.ny) : 0;
  const int z = valid ? int(row / a.ny) : 0;
  const T* src = f + comp * a.comp_f + row * a.nx;
  cx<T>* dst = W + comp * a.comp_w + z * a.plane + (long long)y * a.px;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_x);  // length mx = 2L
  cx<T>* my = lds + r * RS;
  const int nx = a.nx;
  const bool even_nx = (nx & 1) == 0;

  static_for<0, S::D1>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int q = tl + TL * d;
    cx<T> v[P];
    static_for<0, live_in<P>()>([&](auto pp) {
      constexpr int p = decltype(pp)::value;
      const int m = q + Q * p;  // packed index: reals 2m, 2m+1
      cx<T> val = zero_c<T>();
      if (valid) {
        if (even_nx) {
          if (2 * m < nx) val = *reinterpret_cast<const cx<T>*>(src + 2 * m);
        } else {
          if (2 * m < nx) val.re = src[2 * m];
          if (2 * m + 1 < nx) val.im = src[2 * m + 1];
        }
      }
      v[p] = val;
    });
    first_dft<P, -1>(v);
    static_for<1, P>([&](auto kk) {
      constexpr int k1 = decltype(kk)::value;
      v[k1] = cmul(v[k1], tw[2 * q * k1]);  // w_L^{q k1} = w_M^{2 q k1}
    });
    static_for<0, P>([&](auto kk) {
      constexpr int k1 = decltype(kk)::value;
      my[k1 * (Q + 1) + q] = v[k1];
    });
  });
  __syncthreads();
  ColSpec<T, P, Q> w;
  static_for<0, S::D3>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int k1 = tl + TL * d;
    static_for<0, Q>([&](auto qq) {
      constexpr int q = decltype(qq)::value;
      w[d][q] = my[k1 * (Q + 1) + q];
    });
    dft<Q, -1>(w[d]);
  });
  __syncthreads();
  static_for<0, S::D3>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int k1 = tl + TL * d;
    static_for<0, Q>([&](auto kk) {
      constexpr int k2 = decltype(kk)::value;
      my[k1 + P * k2] = w[d][k2];
    });
  });
  __syncthreads();
  if (valid) {
    for (int k = tl; k <= L; k += TL) {
      const cx<T> zk = my[k == L ? 0 : k];
      const cx<T> zm = conj(my[k == 0 ? 0 : L - k]);
      const cx<T> e = scale(zk + zm, T(0.5));
      const cx<T> o = scale(mul_i<-1>(zk - zm), T(0.5));  // (Z - conj Z')/(2i)
      dst[k] = e + cmul(o, tw[k]);
    }
  }
}

// ============================================================================
// Pass 5: complex-to-real inverse DFT along x + crop to x < nx.
//   Z[k] = (X[k] + conj X[L-k]) + i w^{-k} (X[k] - conj X[L-k]),  k < L,
// inverse length-L DFT of Z gives u[2m] + i u[2m+1] (unnormalised).
// ============================================================================
template <typename T, int P, int Q, int RW>
__global__ void __launch_bounds__((RW * Split<P, Q>::TL))
k_xinv(const cx<T>* __restrict__ W, T* __restrict__ u, PassArgs a) {
  using S = Split<P, Q>;
  constexpr int L = S::L, TL = S::TL;
  constexpr int VS = (Q * (P + 1)) | 1;
  __shared__ cx<T> lds[RW * VS];

  const int tid = threadIdx.x;
  const int tl = tid % TL, r = tid / TL;
  const long long row = (long long)blockIdx.x * RW + r;
  const int comp = blockIdx.y;
  const long long nrows = (long long)a.ny * a.nz;
  const bool valid = row < nrows;
  const int y = valid ? int(row % a.ny) : 0;
  const int z = valid ? int(row / a.ny) : 0;
  const cx<T>* src = W + comp * a.comp_w + z * a.plane + (long long)y * a.px;
  T* dst = u + comp * a.comp_f + row * a.nx;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_x);
  cx<T>* my = lds + r * VS;

  static_for<0, S::D3>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int k1 = tl + TL * d;
    cx<T> w[Q];
    static_for<0, Q>([&](auto kk) {
      constexpr int k2 = decltype(kk)::value;
      const int k = k1 + P * k2;
      cx<T> zk = zero_c<T>();
      if (valid) {
        const cx<T> xk = src[k];
        const cx<T> xm = conj(src[L - k]);
        zk = (xk + xm) + mul_i<+1>(cmulc(xk - xm, tw[k]));
      }
      w[k2] = zk;
    });
    dft<Q, +1>(w);
    static_for<0, Q>([&](auto nn) {
      constexpr int n2 = decltype(nn)::value;
      const cx<T> t = (n2 == 0) ? w[n2] : cmulc(w[n2], tw[2 * n2 * k1]);
      my[n2 * (P + 1) + k1] = t;
    });
  });
  __syncthreads();
  const int nx = a.nx;
  const bool even_nx = (nx & 1) == 0;
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
      static_for<0, live_in<P>()>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        const int m = n2 + Q * n1;
        if (even_nx) {
          if (2 * m < nx) *reinterpret_cast<cx<T>*>(dst + 2 * m) = v[n1];
        } else {
          if (2 * m < nx) dst[2 * m] = v[n1].re;
          if (2 * m + 1 < nx) dst[2 * m + 1] = v[n1].im;
        }
      });
    }
  });
}

// ============================================================================
// Column passes.  Thread (c, tl): c = column in the tile, tl = position on
// the line.  The exchange between the two halves of the four-step goes
// through LDS laid out [k1 - chunk][q (+1 pad)][c] in NCH chunks of k1.
// ============================================================================

// Forward step on lines of length M = P Q with inputs n < nlive (n = q + Q p,
// p < P/2 when P is even).  base points at element 0 of column c; elements
// are stride apart.  Returns, per thread, w[d3][k2] = X[k1 + P k2] with
// k1 = tl + TL d3.
template <typename T, int P, int Q, int C, int NCH>
__device__ __forceinline__ void col_forward(const cx<T>* base, long long stride, bool valid, int nlive,
                                            const cx<T>* tw, cx<T>* lds, int c, int tl,
                                            ColSpec<T, P, Q>& w) {
  using S = Split<P, Q>;
  constexpr int TL = S::TL, KC = P / NCH;
  cx<T> v[S::D1][P];
  static_for<0, S::D1>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int q = tl + TL * d;
    static_for<0, live_in<P>()>([&](auto pp) {
      constexpr int p = decltype(pp)::value;
      const int n = q + Q * p;
      v[d][p] = (valid && n < nlive) ? ldg(base + n * stride) : zero_c<T>();
    });
    first_dft<P, -1>(v[d]);
    static_for<1, P>([&](auto kk) {
      constexpr int k1 = decltype(kk)::value;
      v[d][k1] = cmul(v[d][k1], tw[q * k1]);
    });
  });
  static_for<0, NCH>([&](auto hh) {
    constexpr int h = decltype(hh)::value;
    if constexpr (h > 0) __syncthreads();
    static_for<0, S::D1>([&](auto dd) {
      constexpr int d = decltype(dd)::value;
      const int q = tl + TL * d;
      static_for<0, KC>([&](auto kk) {
        constexpr int kr = decltype(kk)::value;
        lds[(kr * (Q + 1) + q) * C + c] = v[d][h * KC + kr];
      });
    });
    __syncthreads();
    static_for<0, S::D3>([&](auto dd) {
      constexpr int d = decltype(dd)::value;
      const int k1 = tl + TL * d;
      if (k1 / KC == h) {
        const int kr = k1 - h * KC;
        static_for<0, Q>([&](auto qq) {
          constexpr int q = decltype(qq)::value;
          w[d][q] = lds[(kr * (Q + 1) + q) * C + c];
        });
      }
    });
  });
  static_for<0, S::D3>([&](auto dd) { dft<Q, -1>(w[decltype(dd)::value]); });
}

// Inverse step: per thread w[d3][k2] = X[k1 + P k2] (k1 = tl + TL d3) in,
// stores x[n2 + Q n1] for n1 < P/2 (n2 = tl + TL d1) where n < nkeep.
template <typename T, int P, int Q, int C, int NCH>
__device__ __forceinline__ void col_inverse(ColSpec<T, P, Q>& w, cx<T>* base, long long stride,
                                            bool valid, int nkeep, const cx<T>* tw, cx<T>* lds, int c,
                                            int tl) {
  using S = Split<P, Q>;
  constexpr int TL = S::TL, QC = Q / NCH;
  static_for<0, S::D3>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int k1 = tl + TL * d;
    dft<Q, +1>(w[d]);
    static_for<1, Q>([&](auto nn) {
      constexpr int n2 = decltype(nn)::value;
      w[d][n2] = cmulc(w[d][n2], tw[n2 * k1]);
    });
  });
  cx<T> v[S::D1][P];
  static_for<0, NCH>([&](auto hh) {
    constexpr int h = decltype(hh)::value;
    __syncthreads();
    static_for<0, S::D3>([&](auto dd) {
      constexpr int d = decltype(dd)::value;
      const int k1 = tl + TL * d;
      static_for<0, QC>([&](auto nn) {
        constexpr int nr = decltype(nn)::value;
        lds[(nr * (P + 1) + k1) * C + c] = w[d][h * QC + nr];
      });
    });
    __syncthreads();
    static_for<0, S::D1>([&](auto dd) {
      constexpr int d = decltype(dd)::value;
      const int n2 = tl + TL * d;
      if (n2 / QC == h) {
        const int nr = n2 - h * QC;
        static_for<0, P>([&](auto kk) {
          constexpr int k1 = decltype(kk)::value;
          v[d][k1] = lds[(nr * (P + 1) + k1) * C + c];
        });
      }
    });
  });
  static_for<0, S::D1>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int n2 = tl + TL * d;
    last_dft<P, +1>(v[d]);
    if (valid) {
      static_for<0, live_in<P>()>([&](auto nn) {
        constexpr int n1 = decltype(nn)::value;
        const int n = n2 + Q * n1;
        if (n < nkeep) base[n * stride] = v[d][n1];
      });
    }
  });
}

template <int P, int Q, int C, int NCH>
constexpr int col_lds_elems() {
  constexpr int a = (P / NCH) * (Q + 1) * C;
  constexpr int b = (Q / NCH) * (P + 1) * C;
  return a > b ? a : b;
}

// Pass 2: DFT along y, rows y < ny live, all my outputs kept (in place).
template <typename T, int P, int Q, int C, int NCH>
__global__ void __launch_bounds__((C * Split<P, Q>::TL))
k_yfwd(cx<T>* __restrict__ W, PassArgs a) {
  using S = Split<P, Q>;
  __shared__ cx<T> lds[col_lds_elems<P, Q, C, NCH>()];
  const int tid = threadIdx.x;
  const int c = tid % C, tl = tid / C;
  const int kx = blockIdx.x * C + c;
  const int z = blockIdx.y, comp = blockIdx.z;
  const bool valid = kx < a.kx;
  cx<T>* base = W + comp * a.comp_w + z * a.plane + kx;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_y);
  ColSpec<T, P, Q> w;
  col_forward<T, P, Q, C, NCH>(base, a.px, valid, a.ny, tw, lds, c, tl, w);
  if (valid) {
    static_for<0, S::D3>([&](auto dd) {
      constexpr int d = decltype(dd)::value;
      const int k1 = tl + S::TL * d;
      static_for<0, Q>([&](auto kk) {
        constexpr int k2 = decltype(kk)::value;
        base[(long long)(k1 + P * k2) * a.px] = w[d][k2];
      });
    });
  }
}

// Pass 4: inverse DFT along y, all my rows in, rows y < ny kept (in place).
template <typename T, int P, int Q, int C, int NCH>
__global__ void __launch_bounds__((C * Split<P, Q>::TL))
k_yinv(cx<T>* __restrict__ W, PassArgs a) {
  using S = Split<P, Q>;
  __shared__ cx<T> lds[col_lds_elems<P, Q, C, NCH>()];
  const int tid = threadIdx.x;
  const int c = tid % C, tl = tid / C;
  const int kx = blockIdx.x * C + c;
  const int z = blockIdx.y, comp = blockIdx.z;
  const bool valid = kx < a.kx;
  cx<T>* base = W + comp * a.comp_w + z * a.plane + kx;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_y);
  ColSpec<T, P, Q> w;
  static_for<0, S::D3>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int k1 = tl + S::TL * d;
    static_for<0, Q>([&](auto kk) {
      constexpr int k2 = decltype(kk)::value;
      w[d][k2] = valid ? ldg(base + (long long)(k1 + P * k2) * a.px) : zero_c<T>();
    });
  });
  col_inverse<T, P, Q, C, NCH>(w, base, a.px, valid, a.ny, tw, lds, c, tl);
}

// Pass 3: along z, forward DFT (z < nz live), times Ghat, inverse DFT, keep
// z < nz; in place.  One workgroup per (column tile, ky); the Ghat octant
// line iy = min(ky, my - ky) is loaded once and applied to every component.
template <typename T, int P, int Q, int C, int NCH>
__global__ void __launch_bounds__((C * Split<P, Q>::TL))
k_zconv(cx<T>* __restrict__ W, PassArgs a) {
  using S = Split<P, Q>;
  constexpr int M = S::L;
  __shared__ cx<T> lds[col_lds_elems<P, Q, C, NCH>()];
  const int tid = threadIdx.x;
  const int c = tid % C, tl = tid / C;
  const int kx = blockIdx.x * C + c;
  const int ky = blockIdx.y;
  const bool valid = kx < a.kx;
  const int iy = ky <= a.my - ky ? ky : a.my - ky;
  const T* g = static_cast<const T*>(a.ghat) + iy * a.g_plane + kx;
  const cx<T>* tw = static_cast<const cx<T>*>(a.tw_z);
  T gv[S::D3][Q];
  static_for<0, S::D3>([&](auto dd) {
    constexpr int d = decltype(dd)::value;
    const int k1 = tl + S::TL * d;
    static_for<0, Q>([&](auto kk) {
      constexpr int k2 = decltype(kk)::value;
      const int kz = k1 + P * k2;
      const int iz = kz <= M - kz ? kz : M - kz;
      gv[d][k2] = valid ? g[(long long)iz * a.px] : T(0);
    });
  });
  for (int comp = 0; comp < a.ncomp; ++comp) {
    cx<T>* base = W + comp * a.comp_w + (long long)ky * a.px + kx;
    ColSpec<T, P, Q> w;
    if (comp > 0) __syncthreads();
    col_forward<T, P, Q, C, NCH>(base, a.plane, valid, a.nz, tw, lds, c, tl, w);
    static_for<0, S::D3>([&](auto dd) {
      constexpr int d = decltype(dd)::value;
      static_for<0, Q>([&](auto kk) {
        constexpr int k2 = decltype(kk)::value;
        w[d][k2] = scale(w[d][k2], gv[d][k2]);
      });
    });
    col_inverse<T, P, Q, C, NCH>(w, base, a.plane, valid, a.nz, tw, lds, c, tl);
  }
}

// ============================================================================
// launchers and the variant table
// ============================================================================
static inline int cdiv(long long a, long long b) { return int((a + b - 1) / b); }

template <typename T, int P, int Q, int RW>
void launch_xfwd(const PassArgs& a, const void* in, void* out, hipStream_t s) {
  dim3 grid(cdiv((long long)a.ny * a.nz, RW), a.ncomp);
  hipLaunchKernelGGL((k_xfwd<T, P, Q, RW>), grid, dim3(RW * Split<P, Q>::TL), 0, s,
                     static_cast<const T*>(in), static_cast<cx<T>*>(out), a);
}
template <typename T, int P, int Q, int RW>
void launch_xinv(const PassArgs& a, const void* in, void* out, hipStream_t s) {
  dim3 grid(cdiv((long long)a.ny * a.nz, RW), a.ncomp);
  hipLaunchKernelGGL((k_xinv<T, P, Q, RW>), grid, dim3(RW * Split<P, Q>::TL), 0, s,
                     static_cast<const cx<T>*>(in), static_cast<T*>(out), a);
}
template <typename T, int P, int Q, int C, int NCH>
void launch_yfwd(const PassArgs& a, const void*, void* out, hipStream_t s) {
  dim3 grid(cdiv(a.kx, C), a.nz, a.ncomp);
  hipLaunchKernelGGL((k_yfwd<T, P, Q, C, NCH>), grid, dim3(C * Split<P, Q>::TL), 0, s,
                     static_cast<cx<T>*>(out), a);
}
template <typename T, int P, int Q, int C, int NCH>
void launch_yinv(const PassArgs& a, const void*, void* out, hipStream_t s) {
  dim3 grid(cdiv(a.kx, C), a.nz, a.ncomp);
  hipLaunchKernelGGL((k_yinv<T, P, Q, C, NCH>), grid, dim3(C * Split<P, Q>::TL), 0, s,
                     static_cast<cx<T>*>(out), a);
}
template <typename T, int P, int Q, int C, int NCH>
void launch_zconv(const PassArgs& a, const void*, void* out, hipStream_t s) {
  dim3 grid(cdiv(a.kx, C), a.my, 1);
  hipLaunchKernelGGL((k_zconv<T, P, Q, C, NCH>), grid, dim3(C * Split<P, Q>::TL), 0, s,
                     static_cast<cx<T>*>(out), a);
}

template <typename T>
constexpr int is64() { return sizeof(T) == 8 ? 1 : 0; }

#define UPS_STR2(x) #x
#define UPS_STR(x) UPS_STR2(x)

#define X_VARIANTS(T, P, Q, RW)                                                                  \
  PassVariant{PASS_XFWD, is64<T>(), 2 * P * Q, P, Q, RW, 1, RW * Split<P, Q>::TL,               \
              int(sizeof(cx<T>)) * RW * ((P * (Q + 1) > P * Q + 1 ? P * (Q + 1) : P * Q + 1) | 1), \
              "xfwd_" #T "_" #P "x" #Q "_r" #RW, &launch_xfwd<T, P, Q, RW>},                     \
  PassVariant{PASS_XINV, is64<T>(), 2 * P * Q, P, Q, RW, 1, RW * Split<P, Q>::TL,               \
              int(sizeof(cx<T>)) * RW * ((Q * (P + 1)) | 1),                                     \
              "xinv_" #T "_" #P "x" #Q "_r" #RW, &launch_xinv<T, P, Q, RW>}

#define COL_VARIANTS(T, P, Q, C, NCH)                                                         \
  PassVariant{PASS_YFWD, is64<T>(), P * Q, P, Q, C, NCH, C * Split<P, Q>::TL,                \
              int(sizeof(cx<T>)) * col_lds_elems<P, Q, C, NCH>(),                             \
              "yfwd_" #T "_" #P "x" #Q "_c" #C "_h" #NCH, &launch_yfwd<T, P, Q, C, NCH>},     \
  PassVariant{PASS_ZCONV, is64<T>(), P * Q, P, Q, C, NCH, C * Split<P, Q>::TL,               \
              int(sizeof(cx<T>)) * col_lds_elems<P, Q, C, NCH>(),                             \
              "zconv_" #T "_" #P "x" #Q "_c" #C "_h" #NCH, &launch_zconv<T, P, Q, C, NCH>},   \
  PassVariant{PASS_YINV, is64<T>(), P * Q, P, Q, C, NCH, C * Split<P, Q>::TL,                \
              int(sizeof(cx<T>)) * col_lds_elems<P, Q, C, NCH>(),                             \
              "yinv_" #T "_" #P "x" #Q "_c" #C "_h" #NCH, &launch_yinv<T, P, Q, C, NCH>}

const std::vector<PassVariant>& pass_variants() {
  static const std::vector<PassVariant> table = {
      // ---- float ----
      X_VARIANTS(float, 4, 4, 16),      // mx = 32
      X_VARIANTS(float, 4, 8, 16),      // mx = 64
      X_VARIANTS(float, 8, 8, 16),      // mx = 128
      X_VARIANTS(float, 8, 16, 16),     // mx = 256
      X_VARIANTS(float, 16, 16, 16),    // mx = 512
      X_VARIANTS(float, 16, 32, 16),    // mx = 1024
      COL_VARIANTS(float, 4, 8, 16, 1),     // 32
      COL_VARIANTS(float, 8, 8, 16, 1),     // 64
      COL_VARIANTS(float, 8, 16, 16, 1),    // 128
      COL_VARIANTS(float, 16, 16, 16, 1),   // 256
      COL_VARIANTS(float, 16, 32, 16, 1),   // 512
      COL_VARIANTS(float, 32, 32, 16, 2),   // 1024
      COL_VARIANTS(float, 32, 32, 8, 1),    // 1024
      // ---- double ----
      X_VARIANTS(double, 4, 4, 8),
      X_VARIANTS(double, 4, 8, 8),
      X_VARIANTS(double, 8, 8, 8),
      X_VARIANTS(double, 8, 16, 8),
      X_VARIANTS(double, 16, 16, 8),
      X_VARIANTS(double, 16, 32, 8),
      COL_VARIANTS(double, 4, 8, 8, 1),
      COL_VARIANTS(double, 8, 8, 8, 1),
      COL_VARIANTS(double, 8, 16, 8, 1),
      COL_VARIANTS(double, 16, 16, 8, 1),
      COL_VARIANTS(double, 16, 32, 8, 1),
      COL_VARIANTS(double, 32, 32, 8, 2),
  };
  return table;
}

int blocks_for(const PassVariant& v, const PassArgs& a, int* gx, int* gy, int* gz) {
  switch (v.kind) {
    case PASS_XFWD:
    case PASS_XINV:
      *gx = cdiv((long long)a.ny * a.nz, v.tile); *gy = a.ncomp; *gz = 1; break;
    case PASS_YFWD:
    case PASS_YINV:
      *gx = cdiv(a.kx, v.tile); *gy = a.nz; *gz = a.ncomp; break;
    default:
      *gx = cdiv(a.kx, v.tile); *gy = a.my; *gz = 1; break;
  }
  return (*gx) * (*gy) * (*gz);
}

}  // namespace ups
