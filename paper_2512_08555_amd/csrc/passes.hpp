// The five FFT passes of the free-space convolution and their variant table.
//
// Data layout (all complex<T>, x-frequency fastest):
//   W[c][z][y][kx]   z < Nz, y < My, kx < Kx = Mx/2+1, row pitch px >= Kx,
//                    plane = My * px; the x pass fills rows y < Ny, the
//                    y-forward pass expands each plane in place to My rows.
//                    With PassArgs::nyq, column 0 carries X[0] + i X[Mx/2]
//                    and the passes see Kx = Mx/2 columns.
//   Ghat[iy][kx][iz] octant iy <= My/2, iz <= Mz/2, iz fastest with pitch gz
//                    (real T), so a z line's spectrum is contiguous.
//   f, u             real T [c][Nz][Ny][Nx], contiguous.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <string>
#include <vector>

namespace ups {

struct PassArgs {
  int nx, ny, nz;        // source points per axis
  int mx, my, mz;        // padded FFT lengths (even)
  int kx;                // mx/2 + 1 stored x frequencies
  int px;                // row pitch of W and Ghat (elements)
  long long plane;       // my * px
  long long comp_w;      // nz * plane: component stride of W
  long long comp_f;      // nx * ny * nz: component stride of f and u
  long long g_plane;     // kx * gz: iy stride of Ghat
  int gz;                // iz pitch of Ghat (>= mz/2 + 1): kx stride
  int ncomp;
  const void* tw_x;      // exp(-2 pi i m / mx), m < mx
  const void* tw_y;
  const void* tw_z;
  const void* ghat;
  // even (+1) or odd (-1) direction, else 0: the forward pass along that
  // axis fills rows n >= n_axis with +-(row 2 n_axis - 1 - n) instead of zeros
  int fill_x, fill_y, fill_z;
  // 1: column 0 of W carries X[0] + i X[mx/2] (both real for a real source)
  // and kx counts the mx/2 columns 0 .. mx/2 - 1.  The x-forward pass packs
  // them, the x-inverse pass unpacks them, and the z pass's main launch
  // leaves column 0 to the pair launch (launch_zpair) beside it.
  int nyq;
};

// One problem of a grouped launch (many problems, one pass, one kernel).
// in/out are the pass's fixed buffers; io_in/io_out >= 0 take the pointer
// from GroupArgs::io instead (the caller's f and u, set per solve).
struct GroupEntry {
  PassArgs a;
  const void* in;
  void* out;
  int io_in, io_out;
  unsigned block0;   // first block of this problem (a multiple of 8)
  unsigned nblocks;
};

struct GroupArgs {
  const GroupEntry* ents;        // device table
  const unsigned short* bmap;    // block -> entry index
  const void* const* io;         // device table of caller pointers
};

enum PassKind { PASS_XFWD = 0, PASS_YFWD = 1, PASS_ZCONV = 2, PASS_YINV = 3, PASS_XINV = 4, NUM_PASSES = 5 };

// One compiled kernel variant of one pass for one (precision, length).
struct PassVariant {
  PassKind kind;
  int is_f64;       // 1: double, 0: float
  int length;       // mx for X passes, my for Y passes, mz for Z pass
  int P, Q;         // line split: length (or length/2 for X passes) = P * Q
  int tile;         // rows (X passes) or columns (Y, Z passes) per workgroup
  int nch;          // LDS exchange chunks
  int threads;      // workgroup size
  int lds_bytes;
  const char* name;
  // enqueue on stream: in -> out (for in-place passes in == out == W)
  void (*launch)(const PassArgs&, const void* in, void* out, hipStream_t);
  // enqueue one grouped launch of nblocks blocks
  void (*launch_grouped)(const GroupArgs&, unsigned nblocks, hipStream_t);
  // 1: a forward pass for an even or odd direction (mirrored second half of
  // the line, full first stage); the other passes and directions take 0
  int fill;
};

const std::vector<PassVariant>& pass_variants();
// The pair launch of the z pass when a.nyq (mz = 512 or 1024): it pairs
// the lines (ky, my - ky) of column 0, forms the products with the G_hat
// columns kx = 0 and kx = mx/2 (2-D Hermitian symmetry of each real part),
// inverts both and writes rows z < nz of column 0 back.  It may run beside
// the main launch, which does not store column 0.
hipError_t launch_zpair(bool f64, const PassArgs& a, void* W, hipStream_t st);
// The narrowest variant of column pass v (same pass, length, precision and
// kernel family) if it is narrower than v, else nullptr.
const PassVariant* narrow_variant(const PassVariant& v);

// helpers shared with the plan
int blocks_for(const PassVariant& v, const PassArgs& a, int* gx, int* gy, int* gz);

}  // namespace ups
