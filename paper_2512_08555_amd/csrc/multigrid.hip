// Kernels of the multigrid cycle (Sec. 3.1, Alg. amg_vcycle): red-black
// Gauss-Seidel, residual, full-weighting restriction with injection and the
// full-approximation right-hand side, trilinear prolongation of the
// correction, cubic reconstruction of the ghost layers and residual norms.
// All are bound by HBM traffic: one thread per node, 64 threads along x,
// neighbours of a node come from the caches.  The
// arithmetic follows the order of the definitions (interpolation and full
// weighting one axis at a time, z, then y, then x).
#include <hip/hip_runtime.h>

#include <algorithm>

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

// One whole red-black iteration from uin into uout (two different arrays),
// the same arithmetic as a red half-step followed by a black one.  A block
// owns a tile of 64 (x) by TY (y) nodes and a chunk of kZC planes, and
// marches up z with rings of planes in LDS: u_in with a halo of 2, the
// half-updated values H (red unknowns new, every other node as in u_in)
// with a halo of 1, and f.  H of plane p is computed on the tile and its
// halo from u_in (the halo's red values again, so no block reads what
// another writes); the black unknowns of plane p - 1 then follow from H of
// planes p - 2 .. p.  Every node of the tile, ghost layer included, is
// written to uout.  The chunk starts two planes early to fill the rings,
// and the next plane's loads are in flight while the current one is
// updated.
constexpr int kZC = 32;

template <typename T, int TY>
__global__ void __launch_bounds__(256) k_mg_gs2(const T* __restrict__ uin, T* __restrict__ uout,
                                                const T* __restrict__ f, MgGrid g, T h2) {
  constexpr int TX = 64;
  constexpr int UX = TX + 4, UY = TY + 4;
  constexpr int HX = TX + 2, HY = TY + 2;
  constexpr int NU = (UX * UY + 255) / 256;   // u_in values each thread stages per plane
  constexpr int NH = (HX * HY + 255) / 256;   // f and H values per thread
  constexpr int NB = TX * TY / 256;           // outputs per thread
  __shared__ T U[3][UY][UX];
  __shared__ T H[3][HY][HX];
  __shared__ T F[3][HY][HX];   // three slots: f of p + 1 is staged while black reads f of p - 1
  // XCD-aware tile order: blocks are dealt to the 8 XCDs in turn, so block
  // b runs on XCD b % 8; each XCD takes one contiguous run of tiles ordered
  // y fastest, then x, then z chunk, and tiles that share halo rows run on
  // the same XCD (its L2) at about the same time.
  const int nty = (g.ny + TY - 1) / TY, ntx = (g.nx + TX - 1) / TX;
  const int ntiles = nty * ntx * ((g.nz + kZC - 1) / kZC);
  const int per_xcd = (ntiles + 7) / 8;
  const int unit = int(blockIdx.x % 8) * per_xcd + int(blockIdx.x / 8);
  if (unit >= ntiles) return;
  const int tyi = unit % nty, txi = (unit / nty) % ntx, tzi = unit / (nty * ntx);
  const int tid = threadIdx.y * kBX + threadIdx.x;
  const int x0 = txi * TX, y0 = tyi * TY;
  const int zs = tzi * kZC, ze = min(zs + kZC, g.nz);
  const size_t sy = g.nx, sz = (size_t)g.nx * g.ny;
  auto in_grid = [&](int x, int y, int z) {
    return z >= 0 && z < g.nz && y >= 0 && y < g.ny && x >= 0 && x < g.nx;
  };
  auto unknown = [&](int x, int y, int z) {
    return z >= 1 && z <= g.nz - 2 && y >= 1 && y <= g.ny - 2 && x >= 1 && x <= g.nx - 2;
  };
  // plane p of u_in (halo 2) and of f (halo 1) into registers; the loads
  // are issued here and waited for only when the registers go to LDS
  T ru[NU], rf[NH];
  auto fetch = [&](int pu, int pf) {
#pragma unroll
    for (int t = 0; t < NU; ++t) {
      const int e = tid + 256 * t;
      const int ly = e / UX, lx = e - ly * UX;
      const int x = x0 - 2 + lx, y = y0 - 2 + ly;
      ru[t] = (e < UX * UY && in_grid(x, y, pu)) ? uin[(size_t)pu * sz + (size_t)y * sy + x] : T(0);
    }
#pragma unroll
    for (int t = 0; t < NH; ++t) {
      const int e = tid + 256 * t;
      const int ly = e / HX, lx = e - ly * HX;
      const int x = x0 - 1 + lx, y = y0 - 1 + ly;
      rf[t] = (e < HX * HY && in_grid(x, y, pf)) ? f[(size_t)pf * sz + (size_t)y * sy + x] : T(0);
    }
  };
  auto stage = [&](int pu, int pf) {
    T(*du)[UX] = U[(pu + 6) % 3];
#pragma unroll
    for (int t = 0; t < NU; ++t) {
      const int e = tid + 256 * t;
      if (e < UX * UY) du[e / UX][e % UX] = ru[t];
    }
    T(*df)[HX] = F[(pf + 6) % 3];
#pragma unroll
    for (int t = 0; t < NH; ++t) {
      const int e = tid + 256 * t;
      if (e < HX * HY) df[e / HX][e % HX] = rf[t];
    }
  };
  auto red = [&](int p) {
    const T(*Um)[UX] = U[(p + 5) % 3];
    const T(*U0)[UX] = U[(p + 6) % 3];
    const T(*Up)[UX] = U[(p + 7) % 3];
    const T(*Fp)[HX] = F[(p + 6) % 3];
    T(*Hd)[HX] = H[(p + 6) % 3];
#pragma unroll
    for (int t = 0; t < NH; ++t) {
      const int e = tid + 256 * t;
      if (e >= HX * HY) break;
      const int ly = e / HX, lx = e - ly * HX;
      const int x = x0 - 1 + lx, y = y0 - 1 + ly;
      const int ux = lx + 1, uy = ly + 1;
      T v = U0[uy][ux];
      if (unknown(x, y, p) && ((x + y + p) & 1) == 0) {
        const T nb = Up[uy][ux] + Um[uy][ux] + U0[uy + 1][ux] + U0[uy - 1][ux] + U0[uy][ux + 1] + U0[uy][ux - 1];
        v = (nb - h2 * Fp[ly][lx]) / T(6);
      }
      Hd[ly][lx] = v;
    }
  };
  auto black = [&](int q) {
    const T(*Hm)[HX] = H[(q + 5) % 3];
    const T(*H0)[HX] = H[(q + 6) % 3];
    const T(*Hp)[HX] = H[(q + 7) % 3];
    const T(*Fq)[HX] = F[(q + 6) % 3];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int e = tid + 256 * t;
      const int ly = e / TX, lx = e - ly * TX;
      const int x = x0 + lx, y = y0 + ly;
      if (x >= g.nx || y >= g.ny) continue;
      const int hx = lx + 1, hy = ly + 1;
      T v = H0[hy][hx];
      if (unknown(x, y, q) && ((x + y + q) & 1) == 1) {
        const T nb = Hp[hy][hx] + Hm[hy][hx] + H0[hy + 1][hx] + H0[hy - 1][hx] + H0[hy][hx + 1] + H0[hy][hx - 1];
        v = (nb - h2 * Fq[hy][hx]) / T(6);
      }
      uout[(size_t)q * sz + (size_t)y * sy + x] = v;
    }
  };
  // prologue: u_in planes zs - 2 and zs - 1 staged, zs and f of zs - 1 in flight
  fetch(zs - 2, zs - 1);
  stage(zs - 2, zs - 1);
  fetch(zs - 1, zs - 1);
  stage(zs - 1, zs - 1);
  fetch(zs, zs - 1);
  for (int p = zs - 1; p <= ze; ++p) {
    stage(p + 1, p);          // u_in of p + 1, f of p
    fetch(p + 2, p + 1);      // in flight during the updates below
    __syncthreads();
    red(p);
    __syncthreads();
    if (p - 1 >= zs) black(p - 1);
  }
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

// One thread per coarse footprint node (i, j, k): it updates the fine
// unknowns 2 (i, j, k) + (a, b, c), a, b, c in {0, 1} (only 0 where the
// index is m), from the correction at the corners of its coarse cell, so
// neighbouring threads write neighbouring fine pairs and share their
// corner loads.  Fine nodes on the ghost layer are left to the ghost kernel.
template <typename T>
__global__ void __launch_bounds__(kBX * kBY) k_mg_prolong(T* __restrict__ u, MgGrid g, const T* __restrict__ up,
                                                          const T* __restrict__ uhat, MgGrid gp, MgBox b) {
  const int k = blockIdx.z;
  const int j = blockIdx.y * kBY + threadIdx.y;
  const int i = blockIdx.x * kBX + threadIdx.x;
  if (j > b.my || i > b.mx) return;
  // corners (i + di, j + dj, k + dk); where the index is m the far corner
  // is not needed and is clamped to the near one
  const int i1 = i < b.mx ? i + 1 : i, j1 = j < b.my ? j + 1 : j, k1 = k < b.mz ? k + 1 : k;
  const int ci[2] = {i, i1}, cj[2] = {j, j1}, ck[2] = {k, k1};
  T E[2][2][2];   // [dk][dj][di]
#pragma unroll
  for (int dk = 0; dk < 2; ++dk)
#pragma unroll
    for (int dj = 0; dj < 2; ++dj)
#pragma unroll
      for (int di = 0; di < 2; ++di)
        E[dk][dj][di] = up[lin(b.ox + ci[di], b.oy + cj[dj], b.oz + ck[dk], gp)] -
                        uhat[((size_t)ck[dk] * (b.my + 1) + cj[dj]) * (b.mx + 1) + ci[di]];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int z = 2 * k + c;
    if (z == 0 || z >= g.nz - 1) continue;
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const int y = 2 * j + bb;
      if (y == 0 || y >= g.ny - 1) continue;
      T yv[2];   // at the x corners: along z, then y
#pragma unroll
      for (int di = 0; di < 2; ++di) {
        const T z0 = c ? T(0.5) * (E[0][0][di] + E[1][0][di]) : E[0][0][di];
        const T z1 = c ? T(0.5) * (E[0][1][di] + E[1][1][di]) : E[0][1][di];
        yv[di] = bb ? T(0.5) * (z0 + z1) : z0;
      }
      const size_t row = ((size_t)z * g.ny + y) * g.nx;
      if (i > 0 && i < b.mx) u[row + 2 * i] += yv[0];
      if (i < b.mx) u[row + 2 * i + 1] += T(0.5) * (yv[0] + yv[1]);
    }
  }
}

// Max |f - Lap u| over the unknowns outside the child's footprint interior:
// a grid-stride loop over rows (4 per block pass, 64 threads along x), a
// reduction in the block, one atomic per block.
template <typename T>
__global__ void __launch_bounds__(kBX * kBY) k_mg_resnorm(const T* __restrict__ u, const T* __restrict__ f, MgGrid g,
                                                          T h2, MgBox ch, int has_child,
                                                          unsigned long long* __restrict__ out) {
  const long long rows = (long long)(g.ny - 2) * (g.nz - 2);
  const size_t sy = g.nx, sz = (size_t)g.nx * g.ny;
  double v = 0.0;
  for (long long r = (long long)blockIdx.x * kBY + threadIdx.y; r < rows; r += (long long)gridDim.x * kBY) {
    const int z = 1 + int(r / (g.ny - 2));
    const int y = 1 + int(r - (long long)(z - 1) * (g.ny - 2));
    const bool yz_in = has_child && y > ch.oy && y < ch.oy + ch.my && z > ch.oz && z < ch.oz + ch.mz;
    for (int x = 1 + threadIdx.x; x <= g.nx - 2; x += kBX) {
      if (yz_in && x > ch.ox && x < ch.ox + ch.mx) continue;
      const double e = fabs((double)residual_at(u, f, lin(x, y, z, g), sy, sz, h2));
      v = e > v || e != e ? e : v;
    }
  }
  // non-negative doubles order like their bit patterns (NaN above all)
  unsigned long long bits = (unsigned long long)__double_as_longlong(v);
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long w = __shfl_xor(bits, o, 64);
    bits = w > bits ? w : bits;
  }
  __shared__ unsigned long long wmax[kBY];
  if (threadIdx.x == 0) wmax[threadIdx.y] = bits;
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    for (int w = 1; w < kBY; ++w) bits = wmax[w] > bits ? wmax[w] : bits;
    if (bits) atomicMax(out, bits);
  }
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

hipError_t mg_smooth_iterations(bool f64, void* u, void* s, const void* f, MgGrid g, double h, int nu,
                                hipStream_t st) {
  hipError_t e = hipSuccess;
  if (nu & 1) {
    e = mg_smooth(f64, u, f, g, h, 0, st);
    if (e == hipSuccess) e = mg_smooth(f64, u, f, g, h, 1, st);
  }
  constexpr int TY64 = 8, TY32 = 8;
  const int ty = f64 ? TY64 : TY32;
  const long long ntiles = (long long)((g.nx + 63) / 64) * ((g.ny + ty - 1) / ty) * ((g.nz + kZC - 1) / kZC);
  const dim3 grid(unsigned(8 * ((ntiles + 7) / 8)));
  const dim3 block(kBX, kBY);
  for (int it = 0; it < nu / 2 && e == hipSuccess; ++it) {
    for (int half = 0; half < 2 && e == hipSuccess; ++half) {
      const void* a = half ? s : u;
      void* b = half ? u : s;
      if (f64)
        hipLaunchKernelGGL((k_mg_gs2<double, TY64>), grid, block, 0, st, static_cast<const double*>(a),
                           static_cast<double*>(b), static_cast<const double*>(f), g, h * h);
      else
        hipLaunchKernelGGL((k_mg_gs2<float, TY32>), grid, block, 0, st, static_cast<const float*>(a),
                           static_cast<float*>(b), static_cast<const float*>(f), g, float(h * h));
      e = hipGetLastError();
    }
  }
  return e;
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
  const dim3 grid = grid_xyz(b.mx + 1, b.my + 1, b.mz + 1), block(kBX, kBY);
  if (f64)
    hipLaunchKernelGGL(k_mg_prolong<double>, grid, block, 0, st, static_cast<double*>(u), g,
                       static_cast<const double*>(up), static_cast<const double*>(uhat), gp, b);
  else
    hipLaunchKernelGGL(k_mg_prolong<float>, grid, block, 0, st, static_cast<float*>(u), g,
                       static_cast<const float*>(up), static_cast<const float*>(uhat), gp, b);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? mg_fill_ghosts(f64, u, g, up, gp, b, st) : e;
}

hipError_t mg_residual_norm(bool f64, const void* u, const void* f, MgGrid g, double h, const MgBox* child,
                            double* out, hipStream_t st) {
  const long long rows = (long long)(g.ny - 2) * (g.nz - 2);
  const dim3 grid(unsigned(std::min<long long>((rows + kBY - 1) / kBY, 2048))), block(kBX, kBY);
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
