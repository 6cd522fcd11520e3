// Kernels of the multigrid cycle (Sec. 3.1, Alg. amg_vcycle): red-black
// Gauss-Seidel, residual, full-weighting restriction with injection and the
// full-approximation right-hand side, trilinear prolongation of the
// correction, cubic reconstruction of the ghost layers and residual norms.
// All are bound by HBM traffic: one thread per node, 64 threads along x,
// neighbours of a node come from the caches.  The
// arithmetic follows the order of the definitions (interpolation and full
// weighting one axis at a time, z, then y, then x).
#include <hip/hip_runtime.h>

#include "mg.hpp"

namespace ups {
namespace {

constexpr int kBX = 64, kBY = 4;

__device__ __forceinline__ size_t lin(int x, int y, int z, const MgGrid& g) {
  return ((size_t)z * g.ny + y) * g.nx + x;
}

__device__ __forceinline__ bool is_ghost(int x, int y, int z, const MgGrid& g) {
  return x == 0 || y == 0 || z == 0 || x == g.nx - 1 || y == g.ny - 1 || z == g.nz - 1;
}

// Trilinear prolongation at fine node (x, y, z) of the correction on the
// footprint, E(i, j, k) = up[node (ox + i, oy + j, oz + k)] - uhat[i, j, k]:
// along z, then y, then x, an odd fine index takes the mean of its two
// coarse neighbours.
template <typename T>
__device__ __forceinline__ T interp_lin(const T* __restrict__ up, const T* __restrict__ uhat, const MgGrid& gp,
                                        const MgBox& b, int x, int y, int z) {
  const int i0 = x >> 1, j0 = y >> 1, k0 = z >> 1;
  const int oi = x & 1, oj = y & 1, ok = z & 1;
  T yv[2];
  for (int a = 0; a <= oi; ++a) {
    T zv[2];
    for (int bb = 0; bb <= oj; ++bb) {
      T e[2];
      for (int c = 0; c <= ok; ++c) {
        const int i = i0 + a, j = j0 + bb, k = k0 + c;
        e[c] = up[lin(b.ox + i, b.oy + j, b.oz + k, gp)] - uhat[((size_t)k * (b.my + 1) + j) * (b.mx + 1) + i];
      }
      zv[bb] = ok ? T(0.5) * (e[0] + e[1]) : e[0];
    }
    yv[a] = oj ? T(0.5) * (zv[0] + zv[1]) : zv[0];
  }
  return oi ? T(0.5) * (yv[0] + yv[1]) : yv[0];
}

template <typename T>
__device__ __forceinline__ T cubic4(T a, T b, T c, T d) {
  return (-a + T(9) * b + T(9) * c - d) / T(16);
}

// Ghost reconstruction at fine node (x, y, z) from the parent: along z,
// then y, then x, an odd fine index takes (-1, 9, 9, -1)/16 of the four
// nearest parent nodes (footprint indices i0 - 1 .. i0 + 2, which lie in the
// parent because the box keeps one parent node free on every side).
template <typename T>
__device__ __forceinline__ T interp_cubic(const T* __restrict__ up, const MgGrid& gp, const MgBox& b, int x, int y,
                                          int z) {
  const int i0 = x >> 1, j0 = y >> 1, k0 = z >> 1;
  const bool oi = x & 1, oj = y & 1, ok = z & 1;
  auto zval = [&](int i, int j) -> T {
    if (!ok) return up[lin(b.ox + i, b.oy + j, b.oz + k0, gp)];
    T v[4];
    for (int c = 0; c < 4; ++c) v[c] = up[lin(b.ox + i, b.oy + j, b.oz + k0 - 1 + c, gp)];
    return cubic4(v[0], v[1], v[2], v[3]);
  };
  auto yval = [&](int i) -> T {
    if (!oj) return zval(i, j0);
    T v[4];
    for (int c = 0; c < 4; ++c) v[c] = zval(i, j0 - 1 + c);
    return cubic4(v[0], v[1], v[2], v[3]);
  };
  if (!oi) return yval(i0);
  T v[4];
  for (int c = 0; c < 4; ++c) v[c] = yval(i0 - 1 + c);
  return cubic4(v[0], v[1], v[2], v[3]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_mg_ghosts(T* __restrict__ u, MgGrid g, const T* __restrict__ up, MgGrid gp,
                                                   MgBox b) {
  // ghost nodes numbered: the planes z = 0 and z = nz - 1, then the ring of
  // each plane z = 1 .. nz - 2 (rows y = 0 and ny - 1, then x = 0 and nx - 1)
  const long long plane = (long long)g.nx * g.ny;
  const long long ring = 2LL * g.nx + 2LL * (g.ny - 2);
  const long long total = 2 * plane + (long long)(g.nz - 2) * ring;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  int x, y, z;
  if (t < 2 * plane) {
    z = t < plane ? 0 : g.nz - 1;
    const long long j = t < plane ? t : t - plane;
    y = int(j / g.nx);
    x = int(j - (long long)y * g.nx);
  } else {
    const long long s = t - 2 * plane;
    z = 1 + int(s / ring);
    const int j = int(s - (long long)(z - 1) * ring);
    if (j < g.nx) {
      y = 0;
      x = j;
    } else if (j < 2 * g.nx) {
      y = g.ny - 1;
      x = j - g.nx;
    } else {
      const int q = j - 2 * g.nx;
      y = 1 + (q >> 1);
      x = (q & 1) ? g.nx - 1 : 0;
    }
  }
  u[lin(x, y, z, g)] = interp_cubic(up, gp, b, x, y, z);
}

template <typename T>
__global__ void __launch_bounds__(kBX * kBY) k_mg_rbgs(T* __restrict__ u, const T* __restrict__ f, MgGrid g, T h2,
                                                       int color) {
  const int z = blockIdx.z + 1;
  const int y = blockIdx.y * kBY + threadIdx.y + 1;
  if (y > g.ny - 2) return;
  const int p = (color + y + z) & 1;           // parity of x for this colour
  const int x = (2 - p) + 2 * int(blockIdx.x * kBX + threadIdx.x);
  if (x > g.nx - 2) return;
  const size_t sy = g.nx, sz = (size_t)g.nx * g.ny;
  const size_t i = lin(x, y, z, g);
  const T nb = u[i + sz] + u[i - sz] + u[i + sy] + u[i - sy] + u[i + 1] + u[i - 1];
  u[i] = (nb - h2 * f[i]) / T(6);
}

template <typename T>
__device__ __forceinline__ T residual_at(const T* __restrict__ u, const T* __restrict__ f, size_t i, size_t sy,
                                         size_t sz, T h2) {
  const T s = u[i + sz] + u[i - sz] + u[i + sy] + u[i - sy] + u[i + 1] + u[i - 1] - T(6) * u[i];
  return f[i] - s / h2;
}

template <typename T>
__global__ void __launch_bounds__(kBX * kBY) k_mg_residual(const T* __restrict__ u, const T* __restrict__ f,
                                                           T* __restrict__ r, MgGrid g, T h2) {
  const int z = blockIdx.z + 1;
  const int y = blockIdx.y * kBY + threadIdx.y + 1;
  const int x = blockIdx.x * kBX + threadIdx.x + 1;
  if (y > g.ny - 2 || x > g.nx - 2) return;
  const size_t i = lin(x, y, z, g);
  r[i] = residual_at(u, f, i, (size_t)g.nx, (size_t)g.nx * g.ny, h2);
}

template <typename T>
__global__ void __launch_bounds__(kBX * kBY) k_mg_restrict(const T* __restrict__ u, const T* __restrict__ r, MgGrid g,
                                                           T* __restrict__ up, T* __restrict__ fp,
                                                           T* __restrict__ uhat, MgGrid gp, MgBox b, T hp2) {
  const int k = blockIdx.z;
  const int j = blockIdx.y * kBY + threadIdx.y;
  const int i = blockIdx.x * kBX + threadIdx.x;
  if (j > b.my || i > b.mx) return;
  const size_t ih = ((size_t)k * (b.my + 1) + j) * (b.mx + 1) + i;
  const size_t ip = lin(b.ox + i, b.oy + j, b.oz + k, gp);
  const bool inner = i > 0 && j > 0 && k > 0 && i < b.mx && j < b.my && k < b.mz;
  if (!inner) {
    uhat[ih] = up[ip];
    return;
  }
  const size_t sy = g.nx, sz = (size_t)g.nx * g.ny;
  const size_t c = lin(2 * i, 2 * j, 2 * k, g);
  const T ui = u[c];
  // full weighting, one axis at a time: z, then y, then x
  T A[3][3];
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      const size_t q = c + (long long)dy * (long long)sy + dx;
      A[dy + 1][dx + 1] = T(0.25) * r[q - sz] + T(0.5) * r[q] + T(0.25) * r[q + sz];
    }
  T B[3];
  for (int dx = 0; dx < 3; ++dx) B[dx] = T(0.25) * A[0][dx] + T(0.5) * A[1][dx] + T(0.25) * A[2][dx];
  const T rc = T(0.25) * B[0] + T(0.5) * B[1] + T(0.25) * B[2];
  // the parent's values after the injection: fine values at the footprint
  // interior, the parent's own on the footprint boundary
  auto nbv = [&](int di, int dj, int dk) -> T {
    const int a = i + di, bb = j + dj, cc = k + dk;
    const bool in = a > 0 && bb > 0 && cc > 0 && a < b.mx && bb < b.my && cc < b.mz;
    return in ? u[lin(2 * a, 2 * bb, 2 * cc, g)] : up[lin(b.ox + a, b.oy + bb, b.oz + cc, gp)];
  };
  const T s = nbv(0, 0, 1) + nbv(0, 0, -1) + nbv(0, 1, 0) + nbv(0, -1, 0) + nbv(1, 0, 0) + nbv(-1, 0, 0) - T(6) * ui;
  up[ip] = ui;
  fp[ip] = rc + s / hp2;
  uhat[ih] = ui;
}

template <typename T>
__global__ void __launch_bounds__(kBX * kBY) k_mg_prolong(T* __restrict__ u, MgGrid g, const T* __restrict__ up,
                                                          const T* __restrict__ uhat, MgGrid gp, MgBox b) {
  const int z = blockIdx.z;
  const int y = blockIdx.y * kBY + threadIdx.y;
  const int x = blockIdx.x * kBX + threadIdx.x;
  if (y >= g.ny || x >= g.nx) return;
  const size_t i = lin(x, y, z, g);
  if (is_ghost(x, y, z, g))
    u[i] = interp_cubic(up, gp, b, x, y, z);
  else
    u[i] += interp_lin(up, uhat, gp, b, x, y, z);
}

template <typename T>
__global__ void __launch_bounds__(kBX * kBY) k_mg_resnorm(const T* __restrict__ u, const T* __restrict__ f, MgGrid g,
                                                          T h2, MgBox ch, int has_child,
                                                          unsigned long long* __restrict__ out) {
  const int z = blockIdx.z + 1;
  const int y = blockIdx.y * kBY + threadIdx.y + 1;
  const int x = blockIdx.x * kBX + threadIdx.x + 1;
  double v = 0.0;
  if (y <= g.ny - 2 && x <= g.nx - 2) {
    const bool skip = has_child && x > ch.ox && x < ch.ox + ch.mx && y > ch.oy && y < ch.oy + ch.my && z > ch.oz &&
                      z < ch.oz + ch.mz;
    if (!skip) v = fabs((double)residual_at(u, f, lin(x, y, z, g), (size_t)g.nx, (size_t)g.nx * g.ny, h2));
  }
  // non-negative doubles order like their bit patterns (NaN above all)
  unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(bits, o, 64);
    bits = w > bits ? w : bits;
  }
  if (((threadIdx.y * kBX + threadIdx.x) & 63) == 0 && bits) atomicMax(out, bits);
}

__global__ void k_mg_zero(double* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

dim3 grid_xyz(int nx, int ny, int nz) {
  return dim3(unsigned((nx + kBX - 1) / kBX), unsigned((ny + kBY - 1) / kBY), unsigned(nz));
}

}  // namespace

hipError_t mg_fill_ghosts(bool f64, void* u, MgGrid g, const void* up, MgGrid gp, MgBox b, hipStream_t st) {
  const long long total = 2LL * g.nx * g.ny + (long long)(g.nz - 2) * (2LL * g.nx + 2LL * (g.ny - 2));
  const dim3 grid(unsigned((total + 255) / 256));
  if (f64)
    hipLaunchKernelGGL(k_mg_ghosts<double>, grid, dim3(256), 0, st, static_cast<double*>(u), g,
                       static_cast<const double*>(up), gp, b);
  else
    hipLaunchKernelGGL(k_mg_ghosts<float>, grid, dim3(256), 0, st, static_cast<float*>(u), g,
                       static_cast<const float*>(up), gp, b);
  return hipGetLastError();
}

hipError_t mg_smooth(bool f64, void* u, const void* f, MgGrid g, double h, int color, hipStream_t st) {
  const int nxc = (g.nx - 1) / 2;             // unknowns of one colour per row, at most
  const dim3 grid = grid_xyz(nxc, g.ny - 2, g.nz - 2), block(kBX, kBY);
  if (f64)
    hipLaunchKernelGGL(k_mg_rbgs<double>, grid, block, 0, st, static_cast<double*>(u), static_cast<const double*>(f),
                       g, h * h, color);
  else
    hipLaunchKernelGGL(k_mg_rbgs<float>, grid, block, 0, st, static_cast<float*>(u), static_cast<const float*>(f), g,
                       float(h * h), color);
  return hipGetLastError();
}

hipError_t mg_residual(bool f64, const void* u, const void* f, void* r, MgGrid g, double h, hipStream_t st) {
  const dim3 grid = grid_xyz(g.nx - 2, g.ny - 2, g.nz - 2), block(kBX, kBY);
  if (f64)
    hipLaunchKernelGGL(k_mg_residual<double>, grid, block, 0, st, static_cast<const double*>(u),
                       static_cast<const double*>(f), static_cast<double*>(r), g, h * h);
  else
    hipLaunchKernelGGL(k_mg_residual<float>, grid, block, 0, st, static_cast<const float*>(u),
                       static_cast<const float*>(f), static_cast<float*>(r), g, float(h * h));
  return hipGetLastError();
}

hipError_t mg_restrict(bool f64, const void* u, const void* r, MgGrid g, void* up, void* fp, void* uhat, MgGrid gp,
                       MgBox b, double hp, hipStream_t st) {
  const dim3 grid = grid_xyz(b.mx + 1, b.my + 1, b.mz + 1), block(kBX, kBY);
  if (f64)
    hipLaunchKernelGGL(k_mg_restrict<double>, grid, block, 0, st, static_cast<const double*>(u),
                       static_cast<const double*>(r), g, static_cast<double*>(up), static_cast<double*>(fp),
                       static_cast<double*>(uhat), gp, b, hp * hp);
  else
    hipLaunchKernelGGL(k_mg_restrict<float>, grid, block, 0, st, static_cast<const float*>(u),
                       static_cast<const float*>(r), g, static_cast<float*>(up), static_cast<float*>(fp),
                       static_cast<float*>(uhat), gp, b, float(hp * hp));
  return hipGetLastError();
}

hipError_t mg_prolong(bool f64, void* u, MgGrid g, const void* up, const void* uhat, MgGrid gp, MgBox b,
                      hipStream_t st) {
  const dim3 grid = grid_xyz(g.nx, g.ny, g.nz), block(kBX, kBY);
  if (f64)
    hipLaunchKernelGGL(k_mg_prolong<double>, grid, block, 0, st, static_cast<double*>(u), g,
                       static_cast<const double*>(up), static_cast<const double*>(uhat), gp, b);
  else
    hipLaunchKernelGGL(k_mg_prolong<float>, grid, block, 0, st, static_cast<float*>(u), g,
                       static_cast<const float*>(up), static_cast<const float*>(uhat), gp, b);
  return hipGetLastError();
}

hipError_t mg_residual_norm(bool f64, const void* u, const void* f, MgGrid g, double h, const MgBox* child,
                            double* out, hipStream_t st) {
  const dim3 grid = grid_xyz(g.nx - 2, g.ny - 2, g.nz - 2), block(kBX, kBY);
  const MgBox ch = child ? *child : MgBox{0, 0, 0, 0, 0, 0};
  unsigned long long* o = reinterpret_cast<unsigned long long*>(out);
  if (f64)
    hipLaunchKernelGGL(k_mg_resnorm<double>, grid, block, 0, st, static_cast<const double*>(u),
                       static_cast<const double*>(f), g, h * h, ch, child ? 1 : 0, o);
  else
    hipLaunchKernelGGL(k_mg_resnorm<float>, grid, block, 0, st, static_cast<const float*>(u),
                       static_cast<const float*>(f), g, float(h * h), ch, child ? 1 : 0, o);
  return hipGetLastError();
}

hipError_t mg_zero(double* p, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_mg_zero, dim3(unsigned((n + 63) / 64)), dim3(64), 0, st, p, n);
  return hipGetLastError();
}

}  // namespace ups
