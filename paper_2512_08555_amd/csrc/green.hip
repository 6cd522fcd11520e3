// Green's spectrum builder (setup, double precision on the device).
//
// G1, the lattice Green's function of the 7-point Laplacian (L G1 = delta,
// paper Sec. 2.2, stencil of eq. cross_discr2), has the Fourier integral
//   G1[n] = -(2pi)^-3 \int e^{i k.n} / sigma(k) dk,  sigma = sum_i (2 - 2 cos k_i),
// and with 1/sigma = \int_0^inf e^{-sigma t} dt and the Bessel generating
// integral it becomes separable:
//   G1[n] = - \int_0^inf prod_i e^{-2t} I_{n_i}(2t) dt.
// The integral on [0, T] uses composite 16-point Gauss-Legendre panels of
// width 1 in s = ln t on [-40, ln T]; on [T, inf) each factor is replaced by
// its large-argument expansion e^{-x} I_n(x) ~ (2 pi x)^-1/2 sum_k c_k(n) x^-k,
// c_k(n) = (-1)^k prod_{m<=k} (4n^2 - (2m-1)^2) / (k! 8^k), whose product is
// integrated term by term.  Both parts are sums of products of per-axis
// factors, so the whole octant is one contraction
//   S[nz][ny][nx] = sum_col Az[nz][col] Ay[ny][col] Ax[nx][col],  G1 = -S,
// evaluated as a batched GEMM.  e^{-x} I_n(x) at the quadrature nodes comes
// from Miller's backward recurrence normalised by e^{-x}(I_0 + 2 sum I_k) = 1.
//
// G_hat on the octant is the DCT-I of G1 along each axis (the DFT of the
// evenly periodised kernel), applied as three GEMMs with the cosine matrix,
// each rotating the axes (z,y,x) -> (x,z,y) so the next axis comes last.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>
#include <vector>

#include "green.hpp"
#include "cplx.hpp"
#include "../../include/ups.h"

namespace ups {

// ---------------------------------------------------------------------------
// host: Gauss-Legendre rule (Newton on P_n, Abramowitz & Stegun 25.4.29)
// ---------------------------------------------------------------------------
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int j = 1; j <= n; ++j) {
        double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
      }
      dp = n * (z * p0 - p1) / (z * z - 1.0);
      double dz = p0 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    x[i] = -z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void lgf_quadrature(int n_max, std::vector<double>& t, std::vector<double>& w, double* T_out) {
  const double T = std::max(400.0, 40.0 * double(n_max) * double(n_max));
  const double s_lo = -40.0, s_hi = std::log(T);
  const int npan = int(std::ceil((s_hi - s_lo) / 1.0));
  std::vector<double> gx, gw;
  gauss_legendre(16, gx, gw);
  t.clear();
  w.clear();
  for (int p = 0; p < npan; ++p) {
    const double a = s_lo + (s_hi - s_lo) * p / npan;
    const double b = s_lo + (s_hi - s_lo) * (p + 1) / npan;
    const double half = 0.5 * (b - a), mid = 0.5 * (b + a);
    for (int i = 0; i < 16; ++i) {
      const double s = mid + half * gx[i];
      const double ts = std::exp(s);
      t.push_back(ts);
      w.push_back(half * gw[i] * ts);  // dt = t ds
    }
  }
  *T_out = T;
}

// ---------------------------------------------------------------------------
// device: e^{-x} I_k(x) for k < kmax at x = 2 t_j, one thread per node
// ---------------------------------------------------------------------------
__global__ void k_bessel_ive(const double* __restrict__ t, int J, int kmax, double* __restrict__ B) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  const double x = 2.0 * t[j];
  const int top = kmax + 32 + int(10.0 * sqrt(x));
  const double big = 1e200, small = 1e-200;
  double ip = 0.0;      // I_{k+1}
  double ic = 1e-280;   // I_k, k = top
  double sum = 0.0, comp = 0.0;  // compensated sum over k >= 1 of I_k
  for (int k = top; k >= 1; --k) {
    // I_{k-1} = I_{k+1} + (2k/x) I_k
    const double in = ip + (2.0 * k / x) * ic;
    {
      const double yk = ic - comp;
      const double tk = sum + yk;
      comp = (tk - sum) - yk;
      sum = tk;
    }
    if (k < kmax) B[(size_t)k * J + j] = ic;
    ip = ic;
    ic = in;
    if (fabs(ic) > big) {
      ip *= small;
      ic *= small;
      sum *= small;
      comp *= small;
      const int hi = top < kmax - 1 ? top : kmax - 1;
      for (int m = k; m <= hi; ++m) B[(size_t)m * J + j] *= small;
    }
  }
  // ic = I_0
  const double norm = ic + 2.0 * sum;
  B[j] = ic / norm;
  const double inv = 1.0 / norm;
  for (int m = 1; m < kmax; ++m) B[(size_t)m * J + j] *= inv;
}

// Per-axis factor table A[n][col], col < J: quadrature (weight w folded in
// when `weighted`), col = J + p: tail pair p = (a, b) with a + b <= K.
//   role 0 (z): c_a(n)           role 1 (y): c_b(n)
//   role 2 (x): sum_{c <= K-a-b} c_c(n) g[a+b+c],
//   g[m] = (4 pi)^-3/2 2^-m T^{-1/2-m} / (m + 1/2).
constexpr int kTailK = 6;
constexpr int kTailPairs = (kTailK + 1) * (kTailK + 2) / 2;

__device__ double hankel_c(int k, double n) {
  double mu = 4.0 * n * n, prod = 1.0, fact = 1.0, p8 = 1.0;
  for (int m = 1; m <= k; ++m) {
    prod *= (mu - double((2 * m - 1) * (2 * m - 1)));
    fact *= m;
    p8 *= 8.0;
  }
  return ((k & 1) ? -1.0 : 1.0) * prod / (fact * p8);
}

__global__ void k_axis_table(const double* __restrict__ B, const double* __restrict__ w, int J, int kext,
                             int role, double T, double* __restrict__ A) {
  const int cols = J + kTailPairs;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)kext * cols) return;
  const int n = int(idx / cols), col = int(idx % cols);
  double v;
  if (col < J) {
    v = B[(size_t)n * J + col];
    if (role == 0) v *= w[col];
  } else {
    int p = col - J, a = 0;
    while (p > kTailK - a) { p -= kTailK - a + 1; ++a; }
    const int b = p;
    if (role == 0) {
      v = hankel_c(a, n);
    } else if (role == 1) {
      v = hankel_c(b, n);
    } else {
      v = 0.0;
      const double c0 = pow(4.0 * kPi, -1.5);
      for (int c = 0; c <= kTailK - a - b; ++c) {
        const int m = a + b + c;
        const double g = c0 * pow(2.0, -m) * pow(T, -0.5 - m) / (m + 0.5);
        v += hankel_c(c, n) * g;
      }
    }
  }
  A[idx] = v;
}

// ---------------------------------------------------------------------------
// device: batched double GEMM-NT with an optional per-batch column scale
//   out[b][i][j] = alpha * sum_l (S ? S[b*ldS + l] : 1) * X[i][l] * Y[j][l]
// 64x64 output tile per workgroup, 256 threads with 4x4 outputs each.
// ---------------------------------------------------------------------------
constexpr int GT = 64, GK = 16;
__global__ void __launch_bounds__(256)
k_gemm_nt(const double* __restrict__ X, int ni, const double* __restrict__ Y, int nj, int nl,
          const double* __restrict__ S, long long ldS, double alpha, double* __restrict__ out,
          long long out_bstride) {
  __shared__ double xs[GK][GT + 1];
  __shared__ double ys[GK][GT + 1];
  const int b = blockIdx.z;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  const int tid = threadIdx.x;
  const int ti = tid / 16, tj = tid % 16;
  double acc[4][4] = {};
  const double* Sb = S ? S + (long long)b * ldS : nullptr;
  for (int l0 = 0; l0 < nl; l0 += GK) {
    for (int e = tid; e < GT * GK; e += 256) {
      const int r = e / GK, l = e % GK;
      const int gi = i0 + r, gj = j0 + r, gl = l0 + l;
      double s = 1.0;
      if (Sb && gl < nl) s = Sb[gl];
      xs[l][r] = (gi < ni && gl < nl) ? s * X[(long long)gi * nl + gl] : 0.0;
      ys[l][r] = (gj < nj && gl < nl) ? Y[(long long)gj * nl + gl] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int l = 0; l < GK; ++l) {
      double xv[4], yv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) xv[a] = xs[l][ti + 16 * a];
#pragma unroll
      for (int a = 0; a < 4; ++a) yv[a] = ys[l][tj + 16 * a];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = fma(xv[a], yv[c], acc[a][c]);
    }
    __syncthreads();
  }
  double* ob = out + (long long)b * out_bstride;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int gi = i0 + ti + 16 * a;
    if (gi >= ni) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gj = j0 + tj + 16 * c;
      if (gj < nj) ob[(long long)gi * nj + gj] = alpha * acc[a][c];
    }
  }
}

// G_hat[iy][kx][iz] (iz pitch gz, type T) = scale * D[iz][iy][kx]
template <typename T>
__global__ void k_store_ghat(const double* __restrict__ D, int kz, int ky, int kx, int gz, double scale,
                             T* __restrict__ g) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)kz * ky * kx;
  if (idx >= tot) return;
  const int x = int(idx % kx);
  const int y = int((idx / kx) % ky);
  const int z = int(idx / ((long long)kx * ky));
  g[((long long)y * kx + x) * gz + z] = T(scale * D[idx]);  // [iy][kx][iz]
}

// ---------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------
static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

static void cosine_matrix(int K, std::vector<double>& C) {
  // C[k][n] = w_n cos(pi n k / (K-1)), w_0 = w_{K-1} = 1, else 2 (DCT-I)
  const long long M = 2LL * (K - 1);
  C.assign((size_t)K * K, 0.0);
  for (int k = 0; k < K; ++k)
    for (int n = 0; n < K; ++n) {
      const double wn = (n == 0 || n == K - 1) ? 1.0 : 2.0;
      C[(size_t)k * K + n] = wn * unit_root((long long)n * k, M).c;
    }
}

GreenScratch green_scratch_layout(int kz, int ky, int kx) {
  GreenScratch s{};
  const int kmax = std::max(kz, std::max(ky, kx));
  std::vector<double> t, w;
  double Tsplit;
  lgf_quadrature(kmax - 1, t, w, &Tsplit);
  const int J = int(t.size());
  const int cols = J + kTailPairs;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  s.J = J;
  s.cols = cols;
  s.off_t = take(sizeof(double) * J);
  s.off_w = take(sizeof(double) * J);
  s.off_B = take(sizeof(double) * (size_t)kmax * J);
  s.off_Az = take(sizeof(double) * (size_t)kz * cols);
  s.off_Ay = take(sizeof(double) * (size_t)ky * cols);
  s.off_Ax = take(sizeof(double) * (size_t)kx * cols);
  s.off_Cx = take(sizeof(double) * (size_t)kx * kx);
  s.off_Cy = take(sizeof(double) * (size_t)ky * ky);
  s.off_Cz = take(sizeof(double) * (size_t)kz * kz);
  const size_t vol = sizeof(double) * (size_t)kz * ky * kx;
  s.off_G0 = take(vol);
  s.off_G1 = take(vol);
  s.bytes = off;
  return s;
}

#define GCHECK(x)                                  \
  do {                                             \
    hipError_t e_ = (x);                           \
    if (e_ != hipSuccess) return e_;               \
  } while (0)

// S = -G1 on the octant kz x ky x kx into L.off_G0 (layout L of these
// extents).  The host vectors must stay alive until the stream is synchronised.
static hipError_t lgf7_octant(int kz, int ky, int kx, const GreenScratch& L, char* base, std::vector<double>& t,
                              std::vector<double>& w, hipStream_t st) {
  auto P = [&](size_t off) { return reinterpret_cast<double*>(base + off); };
  const int kmax = std::max(kz, std::max(ky, kx));
  double Tsplit;
  lgf_quadrature(kmax - 1, t, w, &Tsplit);
  const int J = L.J, cols = L.cols;
  GCHECK(hipMemcpyAsync(P(L.off_t), t.data(), sizeof(double) * J, hipMemcpyHostToDevice, st));
  GCHECK(hipMemcpyAsync(P(L.off_w), w.data(), sizeof(double) * J, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_bessel_ive, dim3((J + 63) / 64), dim3(64), 0, st, P(L.off_t), J, kmax, P(L.off_B));
  GCHECK(hipGetLastError());
  const int ext[3] = {kz, ky, kx};
  const size_t offA[3] = {L.off_Az, L.off_Ay, L.off_Ax};
  for (int role = 0; role < 3; ++role) {
    const long long n = (long long)ext[role] * cols;
    hipLaunchKernelGGL(k_axis_table, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, P(L.off_B),
                       P(L.off_w), J, ext[role], role, Tsplit, P(offA[role]));
    GCHECK(hipGetLastError());
  }
  // S[nz][ny][nx] = sum_col Az[nz][col] Ay[ny][col] Ax[nx][col] -> G0 (= -G1)
  dim3 grid((kx + GT - 1) / GT, (ky + GT - 1) / GT, kz);
  hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, P(L.off_Ay), ky, P(L.off_Ax), kx, cols, P(L.off_Az),
                     (long long)cols, 1.0, P(L.off_G0), (long long)ky * kx);
  GCHECK(hipGetLastError());
  return hipSuccess;
}

// G_hat[iy][kx][iz] = scale * DCT-I (three axes) of the octant table
// [kz][ky][kx] held at L.off_G0 (L.off_G1 is the second buffer).
template <typename T>
static hipError_t dct3_store(int kz, int ky, int kx, int gz, double scale, const GreenScratch& L, char* base,
                             std::vector<double>& Cx, std::vector<double>& Cy, std::vector<double>& Cz, void* ghat,
                             hipStream_t st) {
  auto P = [&](size_t off) { return reinterpret_cast<double*>(base + off); };
  cosine_matrix(kx, Cx);
  cosine_matrix(ky, Cy);
  cosine_matrix(kz, Cz);
  GCHECK(hipMemcpyAsync(P(L.off_Cx), Cx.data(), sizeof(double) * Cx.size(), hipMemcpyHostToDevice, st));
  GCHECK(hipMemcpyAsync(P(L.off_Cy), Cy.data(), sizeof(double) * Cy.size(), hipMemcpyHostToDevice, st));
  GCHECK(hipMemcpyAsync(P(L.off_Cz), Cz.data(), sizeof(double) * Cz.size(), hipMemcpyHostToDevice, st));
  // DCT-I along x: out[kx'][nz][ny] = sum_n Cx[kx'][n] G0[(nz,ny)][n]
  {
    const int a = kz * ky;
    dim3 grid((a + GT - 1) / GT, (kx + GT - 1) / GT, 1);
    hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, P(L.off_Cx), kx, P(L.off_G0), a, kx,
                       (const double*)nullptr, 0LL, 1.0, P(L.off_G1), 0LL);
    GCHECK(hipGetLastError());
  }
  // along y: array (kx', nz, ny) -> out[ky'][kx'][nz]
  {
    const int a = kx * kz;
    dim3 grid((a + GT - 1) / GT, (ky + GT - 1) / GT, 1);
    hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, P(L.off_Cy), ky, P(L.off_G1), a, ky,
                       (const double*)nullptr, 0LL, 1.0, P(L.off_G0), 0LL);
    GCHECK(hipGetLastError());
  }
  // along z: array (ky', kx', nz) -> out[kz'][ky'][kx']
  {
    const int a = ky * kx;
    dim3 grid((a + GT - 1) / GT, (kz + GT - 1) / GT, 1);
    hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, P(L.off_Cz), kz, P(L.off_G0), a, kz,
                       (const double*)nullptr, 0LL, 1.0, P(L.off_G1), 0LL);
    GCHECK(hipGetLastError());
  }
  const long long tot = (long long)kz * ky * kx;
  hipLaunchKernelGGL((k_store_ghat<T>), dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, P(L.off_G1), kz,
                     ky, kx, gz, scale, static_cast<T*>(ghat));
  GCHECK(hipGetLastError());
  return hipSuccess;
}

template <typename T>
hipError_t build_green_t(int kz, int ky, int kx, int gz, double h, int mx, int my, int mz, void* ghat,
                         void* scratch, hipStream_t st) {
  const GreenScratch L = green_scratch_layout(kz, ky, kx);
  char* base = static_cast<char*>(scratch);
  std::vector<double> t, w, Cx, Cy, Cz;  // host data of the asynchronous copies
  GCHECK(lgf7_octant(kz, ky, kx, L, base, t, w, st));
  // G_hat = -(h^2 / (mx my mz)) * DCT(S)
  GCHECK(dct3_store<T>(kz, ky, kx, gz, -(h * h) / (double(mx) * double(my) * double(mz)), L, base, Cx, Cy, Cz,
                       ghat, st));
  // the host vectors above must outlive the copies
  return hipStreamSynchronize(st);
}

// ---------------------------------------------------------------------------
// Directions that are not all unbounded (Sec. 2.2).  Axis indices 0, 1, 2 =
// x, y, z; octant index m_i in [0, M_i/2] of the padded grid; the symbol of
// the 3-point second difference at m_i is s_i = 4 sin^2(pi m_i / M_i).
//   * No unbounded direction: G~ = -1/sigma, sigma = sum s_i (0 at sigma = 0).
//   * One unbounded direction a: for each transverse mode (m_b, m_c) the
//     decaying solution of G[n+1] - 2 G[n] + G[n-1] - s G[n] = delta[n],
//     s = s_b + s_c, is G[n] = -rho^|n| / sqrt(s (s+4)) with
//     rho = 1 / (1 + s/2 + sqrt(s + s^2/4)) (the one-dimensional LGF |n|/2
//     at s = 0); its DCT-I along a.
//   * Two unbounded directions a, b (eq. 2unbkernel): at m_c = 0 the DCT-I of
//     the two-dimensional LGF, normalised by G[0, 0] = 0,
//       G[n] = -\int_0^inf (e^{-4t} I_{n_a}(2t) I_{n_b}(2t) - e^{-4t} I_0(2t)^2) dt,
//     by the quadrature and Hankel tail of the three-dimensional one (the
//     leading tail terms cancel); -1/sigma at every other m_c.
// A periodic direction of N points is zero-padded to M = 2N like an
// unbounded one: the kernel then is the N-periodic Green's function on
// |d| < N, whose DFT on the 2N grid is twice its N-point spectrum at even
// m and zero at odd m.  The stored value is h^2 / (Mx My Mz) times
// G~ times that weight.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double symbol_1d(int m, int M) {
  const double sv = sin(kPi * double(m) / double(M));
  return 4.0 * sv * sv;
}

__global__ void k_lgf2d(const double* __restrict__ B, const double* __restrict__ w, int J, int k0, int k1,
                        double T, double* __restrict__ out) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)k0 * k1) return;
  const int n0 = int(idx / k1), n1 = int(idx % k1);
  double acc = 0.0;
  for (int j = 0; j < J; ++j) {
    const double b0 = B[(size_t)j];
    acc = fma(w[j], B[(size_t)n0 * J + j] * B[(size_t)n1 * J + j] - b0 * b0, acc);
  }
  // tail: sum over a + b = m >= 1 of (c_a(n0) c_b(n1) - c_a(0) c_b(0))
  // \int_T^inf (4 pi t)^-1 (2t)^-m dt
  double tail = 0.0;
  for (int a = 0; a <= kTailK; ++a)
    for (int b = 0; a + b <= kTailK; ++b) {
      const int m = a + b;
      if (m == 0) continue;
      const double g = pow(2.0, -m) * pow(T, -double(m)) / (4.0 * kPi * m);
      tail += g * (hankel_c(a, n0) * hankel_c(b, n1) - hankel_c(a, 0) * hankel_c(b, 0));
    }
  out[idx] = -(acc + tail);
}

// Tt[t][n] = screened 1-D LGF at offset n < ka for transverse mode
// t = mb kc + mc (mb < kb, mc < kc)
__global__ void k_lgf1d_table(int ka, int kb, int kc, int Mb, int Mc, double* __restrict__ out) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)ka * kb * kc) return;
  const int n = int(idx % ka);
  const long long t = idx / ka;
  const int mb = int(t / kc), mc = int(t % kc);
  const double s = symbol_1d(mb, Mb) + symbol_1d(mc, Mc);
  double v;
  if (s == 0.0) {
    v = 0.5 * n;
  } else {
    const double root = sqrt(s * (s + 4.0));
    const double log_rho = -log1p(0.5 * s + 0.5 * root);
    v = -exp(double(n) * log_rho) / root;
  }
  out[idx] = v;
}

struct MixedBc {
  int bc[3];       // ups_bc per axis (x, y, z)
  int M[3];        // padded lengths
  int K[3];        // octant extents M/2 + 1
  int du;          // unbounded directions
  int a, b, c;     // du = 1: a unbounded, b < c the others; du = 2: a < b unbounded, c the other
};

template <typename T>
__global__ void k_store_ghat_mixed(MixedBc q, const double* __restrict__ D, int gz, double scale,
                                   T* __restrict__ g) {
  const long long tot = (long long)q.K[0] * q.K[1] * q.K[2];
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  int m[3];
  m[0] = int(idx % q.K[0]);
  m[1] = int((idx / q.K[0]) % q.K[1]);
  m[2] = int(idx / ((long long)q.K[0] * q.K[1]));
  double wgt = 1.0;
  for (int i = 0; i < 3; ++i)
    if (q.bc[i] == UPS_BC_PER) wgt *= (m[i] & 1) ? 0.0 : 2.0;
  double v = 0.0;
  if (wgt != 0.0) {
    const double sigma = symbol_1d(m[0], q.M[0]) + symbol_1d(m[1], q.M[1]) + symbol_1d(m[2], q.M[2]);
    if (q.du == 0) {
      v = sigma > 0.0 ? -1.0 / sigma : 0.0;
    } else if (q.du == 1) {
      const long long t = (long long)m[q.b] * q.K[q.c] + m[q.c];
      v = D[(long long)m[q.a] * ((long long)q.K[q.b] * q.K[q.c]) + t];
    } else {
      v = m[q.c] == 0 ? D[(long long)m[q.a] * q.K[q.b] + m[q.b]] : -1.0 / sigma;
    }
  }
  g[((long long)m[1] * q.K[0] + m[0]) * gz + m[2]] = T(scale * wgt * v);  // [iy][kx][iz]
}

template <typename T>
hipError_t build_green_mixed_t(const int bc[3], int kz, int ky, int kx, int gz, double h, int mx, int my,
                               int mz, void* ghat, void* scratch, hipStream_t st) {
  const GreenScratch L = green_scratch_layout(kz, ky, kx);
  char* base = static_cast<char*>(scratch);
  auto P = [&](size_t off) { return reinterpret_cast<double*>(base + off); };
  MixedBc q{};
  const int Ms[3] = {mx, my, mz}, Ks[3] = {kx, ky, kz};
  int unb[3], spec[3], nu = 0, ns = 0;
  for (int i = 0; i < 3; ++i) {
    q.bc[i] = bc[i];
    q.M[i] = Ms[i];
    q.K[i] = Ks[i];
    if (bc[i] == UPS_BC_UNB) unb[nu++] = i;
    else spec[ns++] = i;
  }
  q.du = nu;
  const size_t cofs[3] = {L.off_Cx, L.off_Cy, L.off_Cz};
  std::vector<double> Ca, Cb, t, w;  // host data of the asynchronous copies
  const double* D = nullptr;
  if (nu == 1) {
    q.a = unb[0];
    q.b = spec[0];
    q.c = spec[1];
    const int ka = Ks[q.a], kb = Ks[q.b], kc = Ks[q.c];
    const long long ntr = (long long)kb * kc;
    const long long n = ntr * ka;
    hipLaunchKernelGGL(k_lgf1d_table, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, ka, kb, kc, Ms[q.b],
                       Ms[q.c], P(L.off_G0));
    GCHECK(hipGetLastError());
    cosine_matrix(ka, Ca);
    GCHECK(hipMemcpyAsync(P(cofs[q.a]), Ca.data(), sizeof(double) * Ca.size(), hipMemcpyHostToDevice, st));
    // DCT-I along a: out[ma][t] = sum_n C[ma][n] Tt[t][n]
    dim3 grid(unsigned((ntr + GT - 1) / GT), (ka + GT - 1) / GT, 1);
    hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, P(cofs[q.a]), ka, P(L.off_G0), int(ntr), ka,
                       (const double*)nullptr, 0LL, 1.0, P(L.off_G1), 0LL);
    GCHECK(hipGetLastError());
    D = P(L.off_G1);
  } else if (nu == 2) {
    q.a = unb[0];
    q.b = unb[1];
    q.c = spec[0];
    const int ka = Ks[q.a], kb = Ks[q.b];
    const int kmax = std::max(ka, kb);
    double Tsplit;
    lgf_quadrature(kmax - 1, t, w, &Tsplit);
    const int J = int(t.size());
    GCHECK(hipMemcpyAsync(P(L.off_t), t.data(), sizeof(double) * J, hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync(P(L.off_w), w.data(), sizeof(double) * J, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_bessel_ive, dim3((J + 63) / 64), dim3(64), 0, st, P(L.off_t), J, kmax, P(L.off_B));
    GCHECK(hipGetLastError());
    const long long n = (long long)ka * kb;
    hipLaunchKernelGGL(k_lgf2d, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, P(L.off_B), P(L.off_w), J,
                       ka, kb, Tsplit, P(L.off_G0));
    GCHECK(hipGetLastError());
    cosine_matrix(ka, Ca);
    cosine_matrix(kb, Cb);
    GCHECK(hipMemcpyAsync(P(cofs[q.a]), Ca.data(), sizeof(double) * Ca.size(), hipMemcpyHostToDevice, st));
    GCHECK(hipMemcpyAsync(P(cofs[q.b]), Cb.data(), sizeof(double) * Cb.size(), hipMemcpyHostToDevice, st));
    // along b: out[mb][na] = sum_nb Cb[mb][nb] G2[na][nb]
    {
      dim3 grid((ka + GT - 1) / GT, (kb + GT - 1) / GT, 1);
      hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, P(cofs[q.b]), kb, P(L.off_G0), ka, kb,
                         (const double*)nullptr, 0LL, 1.0, P(L.off_G1), 0LL);
      GCHECK(hipGetLastError());
    }
    // along a: out[ma][mb] = sum_na Ca[ma][na] out1[mb][na]
    {
      dim3 grid((kb + GT - 1) / GT, (ka + GT - 1) / GT, 1);
      hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, P(cofs[q.a]), ka, P(L.off_G1), kb, ka,
                         (const double*)nullptr, 0LL, 1.0, P(L.off_G0), 0LL);
      GCHECK(hipGetLastError());
    }
    D = P(L.off_G0);
  }
  const double scale = (h * h) / (double(mx) * double(my) * double(mz));
  const long long tot = (long long)kz * ky * kx;
  hipLaunchKernelGGL((k_store_ghat_mixed<T>), dim3(unsigned((tot + 255) / 256)), dim3(256), 0, st, q, D, gz,
                     scale, static_cast<T*>(ghat));
  GCHECK(hipGetLastError());
  // the host vectors above must outlive the copies
  return hipStreamSynchronize(st);
}

// ---------------------------------------------------------------------------
// Mehrstellen kernels (eqs. mehrstellen_discr4 / _discr6, Sec. 3.2).  With
// s_i = 4 sin^2(k_i / 2) the operator L has the symbol -sigma_L,
//   sigma_4 = sum s - (1/6) sum_{i<j} s_i s_j,  sigma_6 = sigma_4 + (1/30) s_x s_y s_z,
// and the right-hand-side stencil R is
//   R_4 = 1 + (1/12) sum d2,  R_6 = R_4 + (1/90) sum_{i<j} d2_i d2_j - (1/240) sum d2_i^2
// (the printed "delta_y delta_z^2" of R_6 taken as d2_y d2_z).  For a source
// that vanishes outside the box, u = h^2 G_L * (R f) = h^2 (R G_L) * f, so the
// kernel K = R G_L goes through the unchanged solve.  G_L = G1 + D with
//   D[n] = -(1/pi^3) \int_{[0,pi]^3} prod cos(n_i k_i) (sigma_2 - sigma_L) / (sigma_L sigma_2) dk,
// a bounded integrand (sigma_2 - sigma_L = (1/6) sum s_i s_j [- (1/30) s_x s_y s_z]
// is formed directly, so nothing cancels near k = 0), integrated by the tensor
// cube of a composite Gauss-Legendre rule whose panels halve towards k = 0
// and are split into parts of at most 16 periods of cos(n_max k) (16, 32 or
// 64 nodes a part by its number of periods).  The triple sum is three
// contractions: over x nodes, y nodes, then z nodes, in chunks of z nodes.
// ---------------------------------------------------------------------------
constexpr int kMehrGrade = 22;  // the panel next to k = 0 is [0, pi 2^-22]

static void mehr_rule(int n_max, std::vector<double>& k, std::vector<double>& w) {
  std::vector<double> x16, w16, x32, w32, x64, w64;
  gauss_legendre(16, x16, w16);
  gauss_legendre(32, x32, w32);
  gauss_legendre(64, x64, w64);
  k.clear();
  w.clear();
  std::vector<double> edges{0.0};
  for (int j = kMehrGrade; j >= 0; --j) edges.push_back(kPi * std::ldexp(1.0, -j));
  for (size_t e = 0; e + 1 < edges.size(); ++e) {
    const double a = edges[e], b = edges[e + 1];
    const double periods = (b - a) * std::max(n_max, 1) / (2.0 * kPi);
    const int parts = std::max(1, int(std::ceil(periods / 16.0)));
    const double pp = periods / parts;
    const std::vector<double>& gx = pp <= 1.5 ? x16 : pp <= 5.0 ? x32 : x64;
    const std::vector<double>& gw = pp <= 1.5 ? w16 : pp <= 5.0 ? w32 : w64;
    for (int p = 0; p < parts; ++p) {
      const double c = a + (b - a) * p / parts, d = a + (b - a) * (p + 1) / parts;
      const double half = 0.5 * (d - c), mid = 0.5 * (d + c);
      for (size_t i = 0; i < gx.size(); ++i) {
        k.push_back(mid + half * gx[i]);
        w.push_back(half * gw[i]);
      }
    }
  }
}

// T[n][a] = cos(n k_a) w_a, n < ext
__global__ void k_mehr_cos(const double* __restrict__ k, const double* __restrict__ w, int K, int ext,
                           double* __restrict__ T) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)ext * K) return;
  const int n = int(idx / K), a = int(idx % K);
  T[idx] = cos(double(n) * k[a]) * w[a];
}

// X[al][b][c] = (sigma_2 - sigma_L) / (sigma_L sigma_2) at (s_x, s_y, s_z) =
// (s[c], s[b], s[a0 + al])
__global__ void k_mehr_delta(const double* __restrict__ s, int K, int a0, int na, int order,
                             double* __restrict__ X) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)na * K * K) return;
  const int c = int(idx % K);
  const int b = int((idx / K) % K);
  const int al = int(idx / ((long long)K * K));
  const double sx = s[c], sy = s[b], sz = s[a0 + al];
  const double S = sx + sy + sz;
  double dif = (sx * sy + sy * sz + sz * sx) / 6.0;  // sigma_2 - sigma_L
  if (order == 6) dif -= sx * sy * sz / 30.0;
  const double sl = S - dif;
  X[idx] = dif / (sl * S);
}

// General strided double GEMM, 64 x 64 tiles:
//   C[i * sCi + j] (=, or += when acc) alpha * sum_l A[i * sAi + l * sAl] * B[j * sBj + l * sBl]
// over batch b (blockIdx.z) with offsets b * sAb, b * sBb, b * sCb.
__global__ void __launch_bounds__(256)
k_gemm_s(const double* __restrict__ A, long long sAb, long long sAi, long long sAl, const double* __restrict__ B,
         long long sBb, long long sBj, long long sBl, double* __restrict__ C, long long sCb, long long sCi, int ni,
         int nj, int nl, double alpha, int acc) {
  __shared__ double as[GK][GT + 1];
  __shared__ double bs[GK][GT + 1];
  const int bt = blockIdx.z;
  const int i0 = blockIdx.y * GT, j0 = blockIdx.x * GT;
  const int tid = threadIdx.x;
  const int ti = tid / 16, tj = tid % 16;
  const double* Ab = A + bt * sAb;
  const double* Bb = B + bt * sBb;
  double accv[4][4] = {};
  for (int l0 = 0; l0 < nl; l0 += GK) {
    for (int e = tid; e < GT * GK; e += 256) {
      // the fast index of the load follows whichever of the operand's
      // strides is 1 (coalesced rows of the tile)
      int r, l;
      if (sAl == 1) { r = e / GK; l = e % GK; } else { l = e / GT; r = e % GT; }
      const int gi = i0 + r, gl = l0 + l;
      as[l][r] = (gi < ni && gl < nl) ? Ab[gi * sAi + gl * sAl] : 0.0;
      if (sBl == 1) { r = e / GK; l = e % GK; } else { l = e / GT; r = e % GT; }
      const int gj = j0 + r, gl2 = l0 + l;
      bs[l][r] = (gj < nj && gl2 < nl) ? Bb[gj * sBj + gl2 * sBl] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int l = 0; l < GK; ++l) {
      double xv[4], yv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) xv[q] = as[l][ti + 16 * q];
#pragma unroll
      for (int q = 0; q < 4; ++q) yv[q] = bs[l][tj + 16 * q];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int c = 0; c < 4; ++c) accv[q][c] = fma(xv[q], yv[c], accv[q][c]);
    }
    __syncthreads();
  }
  double* Cb = C + bt * sCb;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gi = i0 + ti + 16 * q;
    if (gi >= ni) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gj = j0 + tj + 16 * c;
      if (gj >= nj) continue;
      double* o = Cb + gi * sCi + gj;
      *o = acc ? *o + alpha * accv[q][c] : alpha * accv[q][c];
    }
  }
}

static hipError_t gemm_s(const double* A, long long sAb, long long sAi, long long sAl, const double* B, long long sBb,
                         long long sBj, long long sBl, double* C, long long sCb, long long sCi, int ni, int nj, int nl,
                         int batch, double alpha, bool acc, hipStream_t st) {
  dim3 grid((nj + GT - 1) / GT, (ni + GT - 1) / GT, batch);
  hipLaunchKernelGGL(k_gemm_s, grid, dim3(256), 0, st, A, sAb, sAi, sAl, B, sBb, sBj, sBl, C, sCb, sCi, ni, nj, nl,
                     alpha, acc ? 1 : 0);
  return hipGetLastError();
}

// R applied to the even table G (octant of extents ez x ey x ex): K[n] =
// sum_o coef_o G[|n + o|] on the octant kz x ky x kx.
struct MehrStencil {
  int n;
  int o[33][3];  // offsets (x, y, z)
  double c[33];
};

static MehrStencil mehr_rhs_stencil(int order) {
  // R on a 5^3 grid: apply the difference operators to a unit impulse
  double d[5][5][5] = {}, t1[5][5][5] = {}, t2[5][5][5] = {};
  auto d2 = [](const double (&in)[5][5][5], double (&out)[5][5][5], int axis) {
    for (int z = 0; z < 5; ++z)
      for (int y = 0; y < 5; ++y)
        for (int x = 0; x < 5; ++x) {
          auto at = [&](int dz, int dy, int dx) {
            const int zz = z + dz, yy = y + dy, xx = x + dx;
            return (zz < 0 || zz > 4 || yy < 0 || yy > 4 || xx < 0 || xx > 4) ? 0.0 : in[zz][yy][xx];
          };
          const int e[3][3] = {{0, 0, 1}, {0, 1, 0}, {1, 0, 0}};  // x, y, z as (dz, dy, dx)
          out[z][y][x] = at(e[axis][0], e[axis][1], e[axis][2]) - 2.0 * in[z][y][x] +
                         at(-e[axis][0], -e[axis][1], -e[axis][2]);
        }
  };
  double R[5][5][5] = {};
  d[2][2][2] = 1.0;
  R[2][2][2] = 1.0;
  for (int i = 0; i < 3; ++i) {
    d2(d, t1, i);
    for (int z = 0; z < 5; ++z)
      for (int y = 0; y < 5; ++y)
        for (int x = 0; x < 5; ++x) R[z][y][x] += t1[z][y][x] / 12.0;
    if (order == 6) {
      d2(t1, t2, i);  // d4 along i
      for (int z = 0; z < 5; ++z)
        for (int y = 0; y < 5; ++y)
          for (int x = 0; x < 5; ++x) R[z][y][x] -= t2[z][y][x] / 240.0;
      for (int j = i + 1; j < 3; ++j) {
        d2(t1, t2, j);
        for (int z = 0; z < 5; ++z)
          for (int y = 0; y < 5; ++y)
            for (int x = 0; x < 5; ++x) R[z][y][x] += t2[z][y][x] / 90.0;
      }
    }
  }
  MehrStencil m{};
  for (int z = 0; z < 5; ++z)
    for (int y = 0; y < 5; ++y)
      for (int x = 0; x < 5; ++x)
        if (R[z][y][x] != 0.0 && m.n < 33) {
          m.o[m.n][0] = x - 2;
          m.o[m.n][1] = y - 2;
          m.o[m.n][2] = z - 2;
          m.c[m.n] = R[z][y][x];
          ++m.n;
        }
  return m;
}

__global__ void k_mehr_rhs(MehrStencil m, const double* __restrict__ G, int ez, int ey, int ex, int kz, int ky,
                           int kx, double* __restrict__ K) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)kz * ky * kx) return;
  const int x = int(idx % kx);
  const int y = int((idx / kx) % ky);
  const int z = int(idx / ((long long)kx * ky));
  double v = 0.0;
  for (int q = 0; q < m.n; ++q) {
    const int xx = abs(x + m.o[q][0]), yy = abs(y + m.o[q][1]), zz = abs(z + m.o[q][2]);
    v = fma(m.c[q], G[((long long)zz * ey + yy) * ex + xx], v);
  }
  K[idx] = v;
}

// G_L = -S + D on the extended octant (S = -G1 at off_G0, D at off_D)
__global__ void k_mehr_sum(const double* __restrict__ S, long long n, double* __restrict__ D) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < n) D[idx] -= S[idx];
}

MehrScratch mehr_scratch_layout(int kz, int ky, int kx, int order) {
  MehrScratch m{};
  m.r = order == 6 ? 2 : 1;
  m.ez = kz + m.r;
  m.ey = ky + m.r;
  m.ex = kx + m.r;
  m.base = green_scratch_layout(m.ez, m.ey, m.ex);
  std::vector<double> k, w;
  mehr_rule(std::max(m.ez, std::max(m.ey, m.ex)) - 1, k, w);
  m.K = int(k.size());
  const long long KK = (long long)m.K * m.K;
  m.chunk = int(std::max(1LL, std::min((long long)m.K, (32LL << 20) / KK)));
  size_t off = m.base.bytes;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes, 256); return o; };
  m.off_k = take(sizeof(double) * m.K);
  m.off_w = take(sizeof(double) * m.K);
  m.off_s = take(sizeof(double) * m.K);
  m.off_Tz = take(sizeof(double) * (size_t)m.ez * m.K);
  m.off_Ty = take(sizeof(double) * (size_t)m.ey * m.K);
  m.off_Tx = take(sizeof(double) * (size_t)m.ex * m.K);
  m.off_X = take(sizeof(double) * (size_t)m.chunk * KK);
  m.off_T1 = take(sizeof(double) * (size_t)m.chunk * m.K * m.ex);
  m.off_T2 = take(sizeof(double) * (size_t)m.chunk * m.ey * m.ex);
  m.off_D = take(sizeof(double) * (size_t)m.ez * m.ey * m.ex);
  m.bytes = off;
  return m;
}

template <typename T>
hipError_t build_green_mehr_t(int order, int kz, int ky, int kx, int gz, double h, int mx, int my, int mz,
                              void* ghat, void* scratch, hipStream_t st) {
  const MehrScratch m = mehr_scratch_layout(kz, ky, kx, order);
  char* base = static_cast<char*>(scratch);
  auto P = [&](size_t off) { return reinterpret_cast<double*>(base + off); };
  std::vector<double> t, w, k, kw, sv, Cx, Cy, Cz;  // host data of the asynchronous copies
  // G1 on the extended octant: S = -G1 at base.off_G0
  GCHECK(lgf7_octant(m.ez, m.ey, m.ex, m.base, base, t, w, st));
  // D by the graded tensor rule
  mehr_rule(std::max(m.ez, std::max(m.ey, m.ex)) - 1, k, kw);
  const int K = m.K;
  sv.resize(K);
  for (int a = 0; a < K; ++a) {
    const double sn = std::sin(0.5 * k[a]);
    sv[a] = 4.0 * sn * sn;
  }
  GCHECK(hipMemcpyAsync(P(m.off_k), k.data(), sizeof(double) * K, hipMemcpyHostToDevice, st));
  GCHECK(hipMemcpyAsync(P(m.off_w), kw.data(), sizeof(double) * K, hipMemcpyHostToDevice, st));
  GCHECK(hipMemcpyAsync(P(m.off_s), sv.data(), sizeof(double) * K, hipMemcpyHostToDevice, st));
  const int ext[3] = {m.ez, m.ey, m.ex};
  const size_t offT[3] = {m.off_Tz, m.off_Ty, m.off_Tx};
  for (int i = 0; i < 3; ++i) {
    const long long n = (long long)ext[i] * K;
    hipLaunchKernelGGL(k_mehr_cos, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, P(m.off_k), P(m.off_w), K,
                       ext[i], P(offT[i]));
    GCHECK(hipGetLastError());
  }
  const long long plane = (long long)m.ey * m.ex;
  for (int a0 = 0; a0 < K; a0 += m.chunk) {
    const int na = std::min(m.chunk, K - a0);
    const long long n = (long long)na * K * K;
    hipLaunchKernelGGL(k_mehr_delta, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, P(m.off_s), K, a0, na,
                       order, P(m.off_X));
    GCHECK(hipGetLastError());
    // T1[(a, b)][nx] = sum_c X[(a, b)][c] Tx[nx][c]
    GCHECK(gemm_s(P(m.off_X), 0, K, 1, P(m.off_Tx), 0, K, 1, P(m.off_T1), 0, m.ex, na * K, m.ex, K, 1, 1.0,
                  false, st));
    // T2[a][ny][nx] = sum_b Ty[ny][b] T1[a][b][nx]
    GCHECK(gemm_s(P(m.off_Ty), 0, K, 1, P(m.off_T1), (long long)K * m.ex, 1, m.ex, P(m.off_T2), plane, m.ex, m.ey,
                  m.ex, K, na, 1.0, false, st));
    // D[nz][(ny, nx)] += -(1/pi^3) sum_a Tz[nz][a0 + a] T2[a][(ny, nx)]
    GCHECK(gemm_s(P(m.off_Tz) + a0, 0, K, 1, P(m.off_T2), 0, 1, plane, P(m.off_D), 0, plane, m.ez, int(plane), na,
                  1, -1.0 / (kPi * kPi * kPi), a0 > 0, st));
  }
  // G_L = G1 + D (in place at off_D), then K = R G_L on the octant -> off_G0
  {
    const long long n = (long long)m.ez * plane;
    hipLaunchKernelGGL(k_mehr_sum, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, P(m.base.off_G0), n,
                       P(m.off_D));
    GCHECK(hipGetLastError());
    const long long nk = (long long)kz * ky * kx;
    hipLaunchKernelGGL(k_mehr_rhs, dim3(unsigned((nk + 255) / 256)), dim3(256), 0, st, mehr_rhs_stencil(order),
                       P(m.off_D), m.ez, m.ey, m.ex, kz, ky, kx, P(m.base.off_G0));
    GCHECK(hipGetLastError());
  }
  // G_hat = (h^2 / (mx my mz)) * DCT(K)
  GCHECK(dct3_store<T>(kz, ky, kx, gz, (h * h) / (double(mx) * double(my) * double(mz)), m.base, base, Cx, Cy, Cz,
                       ghat, st));
  // the host vectors above must outlive the copies
  return hipStreamSynchronize(st);
}

template <typename T>
__global__ void k_twiddles(const double* __restrict__ src, int n, cx<T>* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = cx<T>{T(src[2 * i]), T(src[2 * i + 1])};
}

// Twiddle table of one axis: entries m < M hold exp(-2 pi i m / M); the
// kTw2 x kTw2 block after them holds T[a][b] = exp(-2 pi i (a b mod M) / M),
// so a thread's run of twiddles w^(q k), k = 0, 1, ..., is one row (one base
// address plus constant offsets) and a wave's w^(k l) over lanes l is one
// contiguous row as well.  The later-stage tables of the wave-per-line
// kernels (ztab.hpp) follow for M = 512 .. 4096.
template <typename T>
hipError_t build_twiddles_t(int M, void* dst, void* scratch, hipStream_t st) {
  const size_t n = twiddle_entries(M);
  std::vector<double> tw(2 * n);
  for (int m = 0; m < M; ++m) {
    const cs_pair r = unit_root(-(long long)m, M);  // exp(-2 pi i m / M)
    tw[2 * m] = r.c;
    tw[2 * m + 1] = r.s;
  }
  for (int a = 0; a < kTw2; ++a)
    for (int b = 0; b < kTw2; ++b) {
      const size_t i = (size_t)M + (size_t)a * kTw2 + b;
      const long long m = ((long long)a * b) % M;
      tw[2 * i] = tw[2 * m];
      tw[2 * i + 1] = tw[2 * m + 1];
    }
  const size_t z0 = (size_t)M + (size_t)kTw2 * kTw2;
  const int nz = ztab_entries(M);
  for (int i = 0; i < nz; ++i) {
    long long m = 0;
    switch (M) {
      case 512: m = ztab_exponent<8>(i); break;
      case 1024: m = ztab_exponent<16>(i); break;
      case 2048: m = ztab_exponent<32>(i); break;
      default: m = ztab_exponent<64>(i); break;
    }
    tw[2 * (z0 + i)] = tw[2 * m];
    tw[2 * (z0 + i) + 1] = tw[2 * m + 1];
  }
  GCHECK(hipMemcpyAsync(scratch, tw.data(), sizeof(double) * tw.size(), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL((k_twiddles<T>), dim3(unsigned((n + 255) / 256)), dim3(256), 0, st,
                     static_cast<const double*>(scratch), int(n), static_cast<cx<T>*>(dst));
  GCHECK(hipGetLastError());
  // the host vector must outlive the copy
  GCHECK(hipStreamSynchronize(st));
  return hipSuccess;
}

hipError_t build_green(bool f64, const int bc[3], int green, int kz, int ky, int kx, int gz, double h, int mx,
                       int my, int mz, void* ghat, void* scratch, hipStream_t st) {
  const bool all_unb = !bc || (bc[0] == UPS_BC_UNB && bc[1] == UPS_BC_UNB && bc[2] == UPS_BC_UNB);
  hipError_t e;
  if (green == UPS_GREEN_LGF4_MEHR || green == UPS_GREEN_LGF6_MEHR) {
    const int order = green == UPS_GREEN_LGF4_MEHR ? 4 : 6;
    e = f64 ? build_green_mehr_t<double>(order, kz, ky, kx, gz, h, mx, my, mz, ghat, scratch, st)
            : build_green_mehr_t<float>(order, kz, ky, kx, gz, h, mx, my, mz, ghat, scratch, st);
  } else if (all_unb)
    e = f64 ? build_green_t<double>(kz, ky, kx, gz, h, mx, my, mz, ghat, scratch, st)
            : build_green_t<float>(kz, ky, kx, gz, h, mx, my, mz, ghat, scratch, st);
  else
    e = f64 ? build_green_mixed_t<double>(bc, kz, ky, kx, gz, h, mx, my, mz, ghat, scratch, st)
            : build_green_mixed_t<float>(bc, kz, ky, kx, gz, h, mx, my, mz, ghat, scratch, st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}

hipError_t build_twiddles(bool f64, int M, void* dst, void* scratch, hipStream_t st) {
  return f64 ? build_twiddles_t<double>(M, dst, scratch, st) : build_twiddles_t<float>(M, dst, scratch, st);
}

}  // namespace ups
