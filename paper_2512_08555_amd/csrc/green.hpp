// Setup-time builders: the Green's spectrum octant and the twiddle tables.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <vector>

#include "ztab.hpp"

namespace ups {

// Byte offsets of the double-precision scratch arrays the builder uses
// inside the caller's work buffer.
struct GreenScratch {
  int J, cols;
  size_t off_t, off_w, off_B, off_Az, off_Ay, off_Ax, off_Cx, off_Cy, off_Cz, off_G0, off_G1;
  size_t bytes;
};

GreenScratch green_scratch_layout(int kz, int ky, int kx);

// Quadrature nodes t_j and weights w_j (dt folded in) on [0, T], and T.
void lgf_quadrature(int n_max, std::vector<double>& t, std::vector<double>& w, double* T_out);

// Scratch of the Mehrstellen builder: the 7-point layout on the octant
// extended by the stencil radius r of R, the quadrature tables, the chunk
// buffers of the three contractions and the difference table D.
struct MehrScratch {
  int r, ez, ey, ex, K, chunk;
  GreenScratch base;
  size_t off_k, off_w, off_s, off_Tz, off_Ty, off_Tx, off_X, off_T1, off_T2, off_D;
  size_t bytes;
};
// order 4 or 6
MehrScratch mehr_scratch_layout(int kz, int ky, int kx, int order);

// Ghat[iy][kx][iz] (iz pitch gz) = h^2/(mx my mz) * DCT-I(G1) on the octant
// kz x ky x kx = (mz/2+1) x (my/2+1) x (mx/2+1) when every direction is
// unbounded (bc NULL or all UPS_BC_UNB) and green = UPS_GREEN_LGF2; the
// DCT-I of R G_L for the Mehrstellen kernels (green.hip,
// build_green_mehr_t); otherwise the mixed kernel of build_green_mixed_t
// for the ups_bc per axis bc[0..2] = x, y, z.  Waits for completion.
hipError_t build_green(bool f64, const int bc[3], int green, int kz, int ky, int kx, int gz, double h, int mx,
                       int my, int mz, void* ghat, void* scratch, hipStream_t st);

// dst[m] = exp(-2 pi i m / M), m < M, complex float or double; waits.
// Complex entries of one axis's twiddle table: M (exp(-2 pi i m / M)), a
// kTw2 x kTw2 block of products, then the later-stage tables of ztab.hpp
// (see build_twiddles_t).
constexpr int kTw2 = 64;
inline size_t twiddle_entries(int M) { return (size_t)M + (size_t)kTw2 * kTw2 + (size_t)ztab_entries(M); }
hipError_t build_twiddles(bool f64, int M, void* dst, void* scratch, hipStream_t st);

}  // namespace ups
