// Kernels of the multigrid cycle (Sec. 3.1, Alg. amg_vcycle): red-black
// Gauss-Seidel, residual, full-weighting restriction with injection and the
// full-approximation right-hand side, trilinear prolongation of the
// correction, cubic reconstruction of the ghost layers and residual norms.
// All are bound by HBM traffic.  The smoother (k_mg_gs2, and k_mg_gsr, its
// last pre-smoothing iteration fused with the residual) marches tiles up
// chunks of planes with LDS and register rings; the others take one thread
// per node, 64 threads along x, and the neighbours of a node from the
// caches.  The arithmetic follows the order of the definitions
// (interpolation and full weighting one axis at a time, z, then y, then x).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

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

// One whole red-black iteration from uin into uout (two different arrays),
// the same arithmetic as a red half-step followed by a black one.
//
// Tiles start at node 1: a block owns TX x TY columns (x0 .. x0 + TX - 1,
// y0 .. y0 + TY - 1, x0 and y0 = 1 mod TX and TY) and a chunk of zc
// planes from zs = 1 mod zc, and marches up z.  Levels of 2^k + 1 nodes
// then split into whole tiles; the ghost nodes at index 0 belong to no tile
// and are written through by the blocks next to them.
//
// Each thread owns TX TY / NT interior columns and up to NR columns of the
// frame of width 2 around the tile, and keeps their values of u_in (planes
// p - 1 .. p + 2) and f in a ring of four register slots: the loop is
// unrolled by four so that slot indices are compile-time constants and no
// register copy waits on a load in flight.  Step p:
//   - u_in of plane p goes to LDS (halo 2), then one barrier;
//   - red of plane p on the tile and its halo of 1 (the halo's values again,
//     so that no block reads what another writes) from the LDS plane and the
//     column's own z neighbours; H (red new, black as in u_in) to LDS;
//   - black of plane p - 1 on the tile from the H plane written one step
//     earlier and the column's own H of planes p - 2 and p, then the store;
//   - loads of plane p + 3 into the slot of plane p - 1.
// The LDS planes of u_in and H are double-buffered, which is what makes one
// barrier per step enough.  Loads use clamped addresses: a value outside the
// level only ever feeds a stencil whose result is discarded.  Addresses are a
// wave-uniform plane base plus a 32-bit byte offset in the plane: the cycle
// smooths refined levels only, which hold at most 2^31 - 1 nodes in at least
// 5 planes, so a plane stays below 2^32 bytes in FP64.

template <int K>
struct Slot {
  static constexpr int value = K;
};

template <typename T, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) k_mg_gs2(const T* __restrict__ uin, T* __restrict__ uout,
                                               const T* __restrict__ f, MgGrid g, T h2, int zc) {
  constexpr int UX = TX + 4, UY = TY + 4, HX = TX + 2, HY = TY + 2;
  static_assert((TX * TY) % NT == 0, "interior columns split evenly over the threads");
  constexpr int NI = TX * TY / NT;          // interior columns per thread
  constexpr int NRING = 4 * UX + 4 * TY;    // frame of width 2
  constexpr int NR = (NRING + NT - 1) / NT;
  __shared__ T Us[2][UY][UX];
  __shared__ T Hs[2][HY][HX];
  // XCD-aware tile order: block b runs on XCD b % 8, and each XCD takes one
  // contiguous run of tiles ordered y fastest, then x, then z chunk, so that
  // tiles sharing halo rows run on the same XCD (its L2) at about the same time
  const int nty = (g.ny - 1 + TY - 1) / TY, ntx = (g.nx - 1 + TX - 1) / TX;
  const int ntiles = nty * ntx * ((g.nz - 1 + zc - 1) / zc);
  const int per_xcd = (ntiles + 7) / 8;
  const int unit = int(blockIdx.x % 8) * per_xcd + int(blockIdx.x / 8);
  if (unit >= ntiles) return;
  const int tyi = unit % nty, txi = (unit / nty) % ntx, tzi = unit / (nty * ntx);
  const int x0 = 1 + txi * TX, y0 = 1 + tyi * TY;
  const int zs = 1 + tzi * zc, ze = min(zs + zc, g.nz);
  const int t = threadIdx.x;
  const size_t sz = (size_t)g.nx * g.ny;
  auto clampi = [](int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); };
  // byte offset of column (x, y) in a plane, clamped into the level
  auto col_off = [&](int x, int y) {
    return unsigned(clampi(y, 0, g.ny - 1) * g.nx + clampi(x, 0, g.nx - 1)) * unsigned(sizeof(T));
  };
  int ilx[NI], ily[NI];   // interior columns, in LDS coordinates (halo 2)
  unsigned ioff[NI];
  bool iok[NI];
#pragma unroll
  for (int s = 0; s < NI; ++s) {
    const int e = t + NT * s;
    ilx[s] = 2 + e % TX;
    ily[s] = 2 + e / TX;
    const int x = x0 - 2 + ilx[s], y = y0 - 2 + ily[s];
    iok[s] = x < g.nx && y < g.ny;
    ioff[s] = col_off(x, y);
  }
  // frame columns r: rows 0, 1 and UY - 2, UY - 1 whole, then columns 0, 1,
  // UX - 2, UX - 1 of rows 2 .. TY + 1
  int rlx[NR], rly[NR];
  unsigned roff[NR], rfoff[NR];
  bool rval[NR], rin[NR], rgh[NR];
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    const int r = t + NT * s;
    int lx, ly;
    if (r < 2 * UX) {
      ly = r / UX;
      lx = r - ly * UX;
    } else if (r < 4 * UX) {
      const int r2 = r - 2 * UX;
      ly = UY - 2 + r2 / UX;
      lx = r2 % UX;
    } else {
      const int r3 = r - 4 * UX, c = r3 & 3;
      ly = 2 + (r3 >> 2);
      lx = c < 2 ? c : UX - 4 + c;
    }
    rval[s] = r < NRING;
    if (!rval[s]) lx = ly = 2;
    rlx[s] = lx;
    rly[s] = ly;
    const int x = x0 - 2 + lx, y = y0 - 2 + ly;
    rin[s] = rval[s] && lx >= 1 && ly >= 1 && lx <= UX - 2 && ly <= UY - 2;   // in the halo of 1
    rgh[s] = rval[s] && x >= 0 && y >= 0 && x < g.nx && y < g.ny &&
             ((x == 0 && (y >= y0 || y == 0) && y < y0 + TY) || (y == 0 && x >= x0 && x < x0 + TX));
    roff[s] = col_off(x, y);
    // f is needed on the halo of 1 only: outer columns load their nearest
    // such column's value (the same cache line)
    rfoff[s] = col_off(x0 - 2 + clampi(lx, 1, UX - 2), y0 - 2 + clampi(ly, 1, UY - 2));
  }
  auto ld = [&](const T* a, unsigned off, int p) -> T {
    const char* base = reinterpret_cast<const char*>(a + (size_t)clampi(p, 0, g.nz - 1) * sz);
    return *reinterpret_cast<const T*>(base + off);
  };
  auto st = [&](int p, unsigned off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(uout + (size_t)p * sz) + off) = v;
  };
  auto unknown = [&](int x, int y, int z) {
    return z >= 1 && z <= g.nz - 2 && y >= 1 && y <= g.ny - 2 && x >= 1 && x <= g.nx - 2;
  };
  // ring slots: plane p lives in slot (p - p0) & 3
  T iu[4][NI], iF[4][NI], ih[4][NI], ru[4][NR], rF[4][NR];
  const int p0 = zs - 1;
#pragma unroll
  for (int s = 0; s < NI; ++s) {
    iu[3][s] = ld(uin, ioff[s], p0 - 1);
    iu[0][s] = ld(uin, ioff[s], p0);
    iu[1][s] = ld(uin, ioff[s], p0 + 1);
    iu[2][s] = ld(uin, ioff[s], p0 + 2);
    iF[0][s] = ld(f, ioff[s], p0);
    iF[1][s] = ld(f, ioff[s], p0 + 1);
    iF[2][s] = ld(f, ioff[s], p0 + 2);
    iF[3][s] = T(0);
    ih[0][s] = ih[1][s] = ih[2][s] = ih[3][s] = T(0);
  }
#pragma unroll
  for (int s = 0; s < NR; ++s) {
    ru[3][s] = ld(uin, roff[s], p0 - 1);
    ru[0][s] = ld(uin, roff[s], p0);
    ru[1][s] = ld(uin, roff[s], p0 + 1);
    ru[2][s] = ld(uin, roff[s], p0 + 2);
    rF[0][s] = ld(f, rfoff[s], p0);
    rF[1][s] = ld(f, rfoff[s], p0 + 1);
    rF[2][s] = ld(f, rfoff[s], p0 + 2);
    rF[3][s] = T(0);
  }
  auto step = [&](auto slot, int p) {
    constexpr int k = decltype(slot)::value;   // plane p
    constexpr int km = (k + 3) & 3, kp = (k + 1) & 3, kmm = (k + 2) & 3;   // p - 1, p + 1, p - 2
    T(*U)[UX] = Us[p & 1];
    T(*Hw)[HX] = Hs[p & 1];
#pragma unroll
    for (int s = 0; s < NI; ++s) U[ily[s]][ilx[s]] = iu[k][s];
#pragma unroll
    for (int s = 0; s < NR; ++s)
      if (rval[s]) U[rly[s]][rlx[s]] = ru[k][s];
    __syncthreads();
    // red of plane p on the tile and its halo
#pragma unroll
    for (int s = 0; s < NI; ++s) {
      const int lx = ilx[s], ly = ily[s], x = x0 - 2 + lx, y = y0 - 2 + ly;
      T v = iu[k][s];
      if (unknown(x, y, p) && ((x + y + p) & 1) == 0) {
        const T nb = iu[kp][s] + iu[km][s] + U[ly + 1][lx] + U[ly - 1][lx] + U[ly][lx + 1] + U[ly][lx - 1];
        v = (nb - h2 * iF[k][s]) / T(6);
      }
      ih[k][s] = v;
      Hw[ly - 1][lx - 1] = v;
    }
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      if (!rin[s]) continue;
      const int lx = rlx[s], ly = rly[s], x = x0 - 2 + lx, y = y0 - 2 + ly;
      T v = ru[k][s];
      if (unknown(x, y, p) && ((x + y + p) & 1) == 0) {
        const T nb = ru[kp][s] + ru[km][s] + U[ly + 1][lx] + U[ly - 1][lx] + U[ly][lx + 1] + U[ly][lx - 1];
        v = (nb - h2 * rF[k][s]) / T(6);
      }
      Hw[ly - 1][lx - 1] = v;
    }
    if (p == 0) {   // the ghost plane z = 0, ahead of the first chunk
#pragma unroll
      for (int s = 0; s < NI; ++s)
        if (iok[s]) st(0, ioff[s], iu[k][s]);
#pragma unroll
      for (int s = 0; s < NR; ++s)
        if (rgh[s]) st(0, roff[s], ru[k][s]);
    }
    // black of plane q = p - 1 on the tile
    const int q = p - 1;
    if (q >= zs) {
#pragma unroll
      for (int s = 0; s < NR; ++s)
        if (rgh[s]) st(q, roff[s], ru[km][s]);
      const T(*Hq)[HX] = Hs[q & 1];
#pragma unroll
      for (int s = 0; s < NI; ++s) {
        if (!iok[s]) continue;
        const int hx = ilx[s] - 1, hy = ily[s] - 1, x = x0 - 2 + ilx[s], y = y0 - 2 + ily[s];
        T v = ih[km][s];
        if (unknown(x, y, q) && ((x + y + q) & 1) == 1) {
          const T nb = ih[k][s] + ih[kmm][s] + Hq[hy + 1][hx] + Hq[hy - 1][hx] + Hq[hy][hx + 1] + Hq[hy][hx - 1];
          v = (nb - h2 * iF[km][s]) / T(6);
        }
        st(q, ioff[s], v);
      }
    }
    // plane p + 3 into the slot of plane p - 1
#pragma unroll
    for (int s = 0; s < NI; ++s) {
      iu[km][s] = ld(uin, ioff[s], p + 3);
      iF[km][s] = ld(f, ioff[s], p + 3);
    }
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      ru[km][s] = ld(uin, roff[s], p + 3);
      rF[km][s] = ld(f, rfoff[s], p + 3);
    }
  };
  for (int p = p0; p <= ze; p += 4) {
    step(Slot<0>(), p);
    if (p + 1 > ze) break;
    step(Slot<1>(), p + 1);
    if (p + 2 > ze) break;
    step(Slot<2>(), p + 2);
    if (p + 3 > ze) break;
    step(Slot<3>(), p + 3);
  }
}

// The last pre-smoothing iteration fused with the residual of its result:
// uout as k_mg_gs2 writes it, and r = f - (sum of the six neighbours -
// 6 u) / h^2 at the unknowns, the same values as k_mg_residual on uout.  It
// reads u and f and writes u and r once, where an iteration followed by the
// residual kernel reads u and f twice.
//
// The frame around the tile is 3 wide: red runs on the tile and its halo of
// 2, black on the halo of 1, the residual on the tile.  A thread owns TX TY /
// NT interior columns, then frame columns numbered ring by ring from the
// outside in; a column's depth is its ring (0 outermost), 3 in the tile.
// Step p:
//   - u_in of plane p to LDS (halo 3), one barrier;
//   - red of plane p at depth >= 1 into the H ring and the H plane (halo 2);
//   - black of plane p - 1 at depth >= 2 into the V ring and the V plane
//     (halo 1), stored in the tile (and passed through on the ghost faces);
//   - the residual of plane p - 2 in the tile, from the V plane written one
//     step earlier and the column's own V of planes p - 3 and p - 1;
//   - loads: u_in of plane p + 3 into the slot of p - 1, f of plane p + 1
//     into the slot of p - 3 (f is read at planes p, p - 1 and p - 2).
// Block order, clamped loads, 32-bit offsets and the ghost plane z = 0 are
// those of k_mg_gs2; the three LDS planes are double-buffered by parity.
template <typename T, int TX, int TY, int NT>
__global__ void __launch_bounds__(NT) k_mg_gsr(const T* __restrict__ uin, T* __restrict__ uout,
                                               const T* __restrict__ f, T* __restrict__ r, MgGrid g, T h2, int zc) {
  constexpr int W = 3, UX = TX + 2 * W, UY = TY + 2 * W;
  static_assert((TX * TY) % NT == 0, "interior columns split evenly over the threads");
  constexpr int NI = TX * TY / NT;
  constexpr int NRING = UX * UY - TX * TY;
  constexpr int NC = NI + (NRING + NT - 1) / NT;
  __shared__ T Us[2][UY][UX];
  __shared__ T Hs[2][TY + 4][TX + 4];
  __shared__ T Vs[2][TY + 2][TX + 2];
  const int nty = (g.ny - 1 + TY - 1) / TY, ntx = (g.nx - 1 + TX - 1) / TX;
  const int ntiles = nty * ntx * ((g.nz - 1 + zc - 1) / zc);
  const int per_xcd = (ntiles + 7) / 8;
  const int unit = int(blockIdx.x % 8) * per_xcd + int(blockIdx.x / 8);
  if (unit >= ntiles) return;
  const int tyi = unit % nty, txi = (unit / nty) % ntx, tzi = unit / (nty * ntx);
  const int x0 = 1 + txi * TX, y0 = 1 + tyi * TY;
  const int zs = 1 + tzi * zc, ze = min(zs + zc, g.nz);
  const int t = threadIdx.x;
  const size_t sz = (size_t)g.nx * g.ny;
  auto clampi = [](int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); };
  auto col_off = [&](int x, int y) {
    return unsigned(clampi(y, 0, g.ny - 1) * g.nx + clampi(x, 0, g.nx - 1)) * unsigned(sizeof(T));
  };
  int clx[NC], cly[NC], cdep[NC];   // LDS coordinates (halo 3) and depth
  unsigned coff[NC], cfoff[NC];
  bool cval[NC], cst[NC], cgh[NC];
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    int lx, ly, dep = W;
    bool val = true;
    if (s < NI) {
      const int e = t + NT * s;
      lx = W + e % TX;
      ly = W + e / TX;
    } else {
      // ring d is the border of the (UX - 2d) x (UY - 2d) box at (d, d):
      // its top row, its bottom row, then its two side columns row by row
      int q = t + NT * (s - NI);
      val = q < NRING;
      if (!val) q = 0;
      int w = UX, hh = UY;
      dep = 0;
      while (dep < W - 1 && q >= 2 * w + 2 * (hh - 2)) {
        q -= 2 * w + 2 * (hh - 2);
        ++dep;
        w -= 2;
        hh -= 2;
      }
      if (q < w) {
        lx = dep + q;
        ly = dep;
      } else if (q < 2 * w) {
        lx = dep + q - w;
        ly = dep + hh - 1;
      } else {
        const int q2 = q - 2 * w;
        lx = dep + ((q2 & 1) ? w - 1 : 0);
        ly = dep + 1 + (q2 >> 1);
      }
    }
    clx[s] = lx;
    cly[s] = ly;
    cdep[s] = dep;
    cval[s] = val;
    const int x = x0 - W + lx, y = y0 - W + ly;
    coff[s] = col_off(x, y);
    // f is read from depth 1 in: the outer ring loads its inner neighbour's
    cfoff[s] = col_off(x0 - W + clampi(lx, 1, UX - 2), y0 - W + clampi(ly, 1, UY - 2));
    cst[s] = dep == W && x < g.nx && y < g.ny;
    cgh[s] = val && x >= 0 && y >= 0 && x < g.nx && y < g.ny &&
             ((x == 0 && (y >= y0 || y == 0) && y < y0 + TY) || (y == 0 && x >= x0 && x < x0 + TX));
  }
  auto ld = [&](const T* a, unsigned off, int p) -> T {
    const char* base = reinterpret_cast<const char*>(a + (size_t)clampi(p, 0, g.nz - 1) * sz);
    return *reinterpret_cast<const T*>(base + off);
  };
  auto st = [&](T* a, int p, unsigned off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(a + (size_t)p * sz) + off) = v;
  };
  auto unknown = [&](int x, int y, int z) {
    return z >= 1 && z <= g.nz - 2 && y >= 1 && y <= g.ny - 2 && x >= 1 && x <= g.nx - 2;
  };
  // ring slots: plane p lives in slot (p - p0) & 3
  T U[4][NC], H[4][NC], V[4][NC], F[4][NC];
  const int p0 = zs - 2;
#pragma unroll
  for (int s = 0; s < NC; ++s) {
    U[3][s] = ld(uin, coff[s], p0 - 1);
    U[0][s] = ld(uin, coff[s], p0);
    U[1][s] = ld(uin, coff[s], p0 + 1);
    U[2][s] = ld(uin, coff[s], p0 + 2);
    F[0][s] = ld(f, cfoff[s], p0);
    F[1][s] = F[2][s] = F[3][s] = T(0);   // planes p0 - 2 and p0 - 1 feed only discarded results
#pragma unroll
    for (int j = 0; j < 4; ++j) H[j][s] = V[j][s] = T(0);
  }
  auto step = [&](auto slot, int p) {
    constexpr int k = decltype(slot)::value;   // plane p
    constexpr int km = (k + 3) & 3, kp = (k + 1) & 3, kmm = (k + 2) & 3;   // p - 1, p + 1 (and p - 3), p - 2
#pragma unroll
    for (int s = 0; s < NC; ++s)
      if (cval[s]) Us[p & 1][cly[s]][clx[s]] = U[k][s];
    __syncthreads();
    {   // red of plane p at depth >= 1
      const T(*Ur)[UX] = Us[p & 1];
      T(*Hw)[TX + 4] = Hs[p & 1];
#pragma unroll
      for (int s = 0; s < NC; ++s) {
        if (!cval[s] || cdep[s] < 1) continue;
        const int lx = clx[s], ly = cly[s], x = x0 - W + lx, y = y0 - W + ly;
        T v = U[k][s];
        if (unknown(x, y, p) && ((x + y + p) & 1) == 0) {
          const T nb = U[kp][s] + U[km][s] + Ur[ly + 1][lx] + Ur[ly - 1][lx] + Ur[ly][lx + 1] + Ur[ly][lx - 1];
          v = (nb - h2 * F[k][s]) / T(6);
        }
        H[k][s] = v;
        Hw[ly - 1][lx - 1] = v;
      }
    }
    if (p == 0) {   // the ghost plane z = 0, ahead of the first chunk
#pragma unroll
      for (int s = 0; s < NC; ++s)
        if (cst[s] || cgh[s]) st(uout, 0, coff[s], U[k][s]);
    }
    {   // black of plane q = p - 1 at depth >= 2
      const int q = p - 1;
      const bool keep = q >= zs && q < ze;
      const T(*Hr)[TX + 4] = Hs[q & 1];
      T(*Vw)[TX + 2] = Vs[q & 1];
#pragma unroll
      for (int s = 0; s < NC; ++s) {
        if (!cval[s] || cdep[s] < 2) continue;
        const int lx = clx[s], ly = cly[s], x = x0 - W + lx, y = y0 - W + ly;
        T v = H[km][s];
        if (unknown(x, y, q) && ((x + y + q) & 1) == 1) {
          const T nb = H[k][s] + H[kmm][s] + Hr[ly][lx - 1] + Hr[ly - 2][lx - 1] + Hr[ly - 1][lx] + Hr[ly - 1][lx - 2];
          v = (nb - h2 * F[km][s]) / T(6);
        }
        V[km][s] = v;
        Vw[ly - 2][lx - 2] = v;
        if (keep && (cst[s] || cgh[s])) st(uout, q, coff[s], v);
      }
    }
    {   // residual of plane q = p - 2 in the tile
      const int q = p - 2;
      if (q >= zs && q < ze) {
        const T(*Vr)[TX + 2] = Vs[q & 1];
#pragma unroll
        for (int s = 0; s < NC; ++s) {
          if (!cst[s]) continue;
          const int lx = clx[s], ly = cly[s], x = x0 - W + lx, y = y0 - W + ly;
          if (!unknown(x, y, q)) continue;
          const T sum = V[km][s] + V[kp][s] + Vr[ly - 1][lx - 2] + Vr[ly - 3][lx - 2] + Vr[ly - 2][lx - 1] +
                        Vr[ly - 2][lx - 3] - T(6) * V[kmm][s];
          st(r, q, coff[s], F[kmm][s] - sum / h2);
        }
      }
    }
#pragma unroll
    for (int s = 0; s < NC; ++s) {
      U[km][s] = ld(uin, coff[s], p + 3);
      F[kp][s] = ld(f, cfoff[s], p + 1);
    }
  };
  const int pe = ze + 1;   // the residual of plane ze - 1
  for (int p = p0; p <= pe; p += 4) {
    step(Slot<0>(), p);
    if (p + 1 > pe) break;
    step(Slot<1>(), p + 1);
    if (p + 2 > pe) break;
    step(Slot<2>(), p + 2);
    if (p + 3 > pe) break;
    step(Slot<3>(), p + 3);
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
// It reads u_in and writes u_out = u_in + correction at every fine unknown:
// the two may be one array (each node is read and written by one thread).
template <typename T>
__global__ void __launch_bounds__(kBX * kBY) k_mg_prolong(const T* uin, T* uout, MgGrid g, const T* __restrict__ up,
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
      if (i > 0 && i < b.mx) uout[row + 2 * i] = uin[row + 2 * i] + yv[0];
      if (i < b.mx) uout[row + 2 * i + 1] = uin[row + 2 * i + 1] + T(0.5) * (yv[0] + yv[1]);
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

namespace {

// Tile shapes of the fused iteration (x width, y height, threads), widest
// first; a level takes the first one whose tiles pad its nx - 1 columns
// least.  Measured at 513^3: 256 x 8 (FP32) and 128 x 16 (FP64) are the
// fastest shapes that split the level into whole tiles.
struct GsShape {
  int tx, ty, nt;
};
constexpr GsShape kGs32[] = {{256, 8, 1024}, {128, 16, 1024}, {64, 16, 512}};
constexpr GsShape kGs64[] = {{128, 16, 1024}, {64, 16, 512}};

int gs_shape(const GsShape* c, int n, int nx) {
  auto padded = [&](int i) { return (nx - 1 + c[i].tx - 1) / c[i].tx * c[i].tx; };
  int best = 0;
  for (int i = 1; i < n; ++i)
    if (padded(i) < padded(best)) best = i;
  return best;
}

// Planes per z chunk of the tiled smoothers.  A block pays the start of its
// plane pipeline (four planes of loads before the first store) once per
// chunk, so long chunks are cheaper, as long as the tiles still fill the
// GPU.  The chunk count n minimises rounds(n) (ceil(planes / n) + 8), where
// rounds(n) is how many times the n * layer blocks (layer = tiles per plane)
// refill `slots` resident blocks.  Measured at 513^3 (FP32 256 x 8 tiles, one
// block per CU, 128 tiles per plane): 2 chunks of 256 planes 375 us, 4 of 128
// 387 us, 16 of 32 431-468 us; at 257^3 (32 tiles per plane), 8 chunks of 32
// planes 47 us, 2 of 128 148 us.
int chunk_planes(long long layer, int planes, long long slots) {
  int best_n = 1;
  long long best = -1;
  const int nmax = std::max(1, planes / 8);
  for (int n = 1; n <= nmax; ++n) {
    const long long zc = (planes + n - 1) / n;
    const long long rounds = (layer * n + slots - 1) / slots;
    const long long cost = rounds * (zc + 8);
    if (best < 0 || cost < best) {
      best = cost;
      best_n = n;
    }
  }
  return (planes + best_n - 1) / best_n;
}

// Blocks of `kernel` (nt threads) one compute unit holds, at least 1.
int blocks_per_cu(const void* kernel, int nt) {
  int n = 0;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, nt, 0) == hipSuccess ? std::max(n, 1) : 1;
}

// Chunk length and grid of a tiled smoother over level g: the blocks the
// current device holds at once are its compute units times per_cu.
void tile_grid(int tx, int ty, MgGrid g, int per_cu, int* zc, unsigned* blocks) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 1;
  const long long layer = (long long)((g.nx - 1 + tx - 1) / tx) * ((g.ny - 1 + ty - 1) / ty);
  *zc = chunk_planes(layer, g.nz - 1, (long long)std::max(cus, 1) * per_cu);
  const long long ntiles = layer * ((g.nz - 1 + *zc - 1) / *zc);
  *blocks = unsigned(8 * ((ntiles + 7) / 8));
}

template <typename T, int TX, int TY, int NT>
hipError_t launch_gs2(const void* a, void* b, const void* f, MgGrid g, double h, hipStream_t st) {
  static const int per_cu = blocks_per_cu(reinterpret_cast<const void*>(k_mg_gs2<T, TX, TY, NT>), NT);
  int zc = 0;
  unsigned blocks = 0;
  tile_grid(TX, TY, g, per_cu, &zc, &blocks);
  hipLaunchKernelGGL((k_mg_gs2<T, TX, TY, NT>), dim3(blocks), dim3(NT), 0, st, static_cast<const T*>(a),
                     static_cast<T*>(b), static_cast<const T*>(f), g, T(h * h), zc);
  return hipGetLastError();
}

// Tile shapes of the iteration fused with the residual, chosen the same way.
// Measured at 513^3: 128 x 16 (FP32) and 128 x 8 (FP64) with 1024 threads.
constexpr GsShape kGr32[] = {{128, 16, 1024}, {64, 16, 1024}};
constexpr GsShape kGr64[] = {{128, 8, 1024}, {64, 16, 1024}};

template <typename T, int TX, int TY, int NT>
hipError_t launch_gsr(const void* a, void* b, const void* f, void* r, MgGrid g, double h, hipStream_t st) {
  static const int per_cu = blocks_per_cu(reinterpret_cast<const void*>(k_mg_gsr<T, TX, TY, NT>), NT);
  int zc = 0;
  unsigned blocks = 0;
  tile_grid(TX, TY, g, per_cu, &zc, &blocks);
  hipLaunchKernelGGL((k_mg_gsr<T, TX, TY, NT>), dim3(blocks), dim3(NT), 0, st, static_cast<const T*>(a),
                     static_cast<T*>(b), static_cast<const T*>(f), static_cast<T*>(r), g, T(h * h), zc);
  return hipGetLastError();
}

hipError_t smooth_residual_fused(bool f64, const void* a, void* b, const void* f, void* r, MgGrid g, double h,
                                 hipStream_t st) {
  static_assert(kGr64[0].tx == 128 && kGr64[1].tx == 64 && kGr32[0].tx == 128 && kGr32[1].tx == 64,
                "launch table below");
  if (f64)
    return gs_shape(kGr64, 2, g.nx) == 0 ? launch_gsr<double, 128, 8, 1024>(a, b, f, r, g, h, st)
                                          : launch_gsr<double, 64, 16, 1024>(a, b, f, r, g, h, st);
  return gs_shape(kGr32, 2, g.nx) == 0 ? launch_gsr<float, 128, 16, 1024>(a, b, f, r, g, h, st)
                                        : launch_gsr<float, 64, 16, 1024>(a, b, f, r, g, h, st);
}

hipError_t smooth_fused(bool f64, const void* a, void* b, const void* f, MgGrid g, double h, hipStream_t st) {
  static_assert(kGs64[0].tx == 128 && kGs64[1].tx == 64, "launch table below");
  static_assert(kGs32[0].tx == 256 && kGs32[1].tx == 128 && kGs32[2].tx == 64, "launch table below");
  if (f64)
    return gs_shape(kGs64, 2, g.nx) == 0 ? launch_gs2<double, 128, 16, 1024>(a, b, f, g, h, st)
                                          : launch_gs2<double, 64, 16, 512>(a, b, f, g, h, st);
  switch (gs_shape(kGs32, 3, g.nx)) {
    case 0: return launch_gs2<float, 256, 8, 1024>(a, b, f, g, h, st);
    case 1: return launch_gs2<float, 128, 16, 1024>(a, b, f, g, h, st);
    default: return launch_gs2<float, 64, 16, 512>(a, b, f, g, h, st);
  }
}

}  // namespace

hipError_t mg_smooth_iterations(bool f64, void* u, void* s, const void* f, MgGrid g, double h, int nu,
                                hipStream_t st, bool from_s) {
  // nu fused iterations, alternately between u and s from wherever the
  // values are; if they end in s they are copied back (2 arrays of traffic,
  // against the 3 of an iteration split into two in-place half-steps)
  hipError_t e = hipSuccess;
  void* a = from_s ? s : u;
  void* b = from_s ? u : s;
  for (int it = 0; it < nu && e == hipSuccess; ++it) {
    e = smooth_fused(f64, a, b, f, g, h, st);
    std::swap(a, b);
  }
  if (e == hipSuccess && a == s)
    e = hipMemcpyAsync(u, s, (size_t)g.nx * g.ny * g.nz * (f64 ? sizeof(double) : sizeof(float)),
                       hipMemcpyDeviceToDevice, st);
  return e;
}

hipError_t mg_smooth_residual(bool f64, void* u, void* s, const void* f, void* r, MgGrid g, double h, int nu,
                              hipStream_t st, void** out) {
  *out = u;
  if (nu == 0) return mg_residual(f64, u, f, r, g, h, st);
  // nu - 1 plain iterations, u -> s -> u ..., then the fused one from
  // wherever they left the values; they end in s after an odd count
  hipError_t e = hipSuccess;
  void* a = u;
  void* b = s;
  for (int it = 0; it + 1 < nu && e == hipSuccess; ++it) {
    e = smooth_fused(f64, a, b, f, g, h, st);
    std::swap(a, b);
  }
  if (e == hipSuccess) e = smooth_residual_fused(f64, a, b, f, r, g, h, st);
  *out = b;
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

hipError_t mg_prolong(bool f64, const void* uin, void* u, MgGrid g, const void* up, const void* uhat, MgGrid gp,
                      MgBox b, hipStream_t st) {
  const dim3 grid = grid_xyz(b.mx + 1, b.my + 1, b.mz + 1), block(kBX, kBY);
  if (f64)
    hipLaunchKernelGGL(k_mg_prolong<double>, grid, block, 0, st, static_cast<const double*>(uin), static_cast<double*>(u), g,
                       static_cast<const double*>(up), static_cast<const double*>(uhat), gp, b);
  else
    hipLaunchKernelGGL(k_mg_prolong<float>, grid, block, 0, st, static_cast<const float*>(uin), static_cast<float*>(u), g,
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
