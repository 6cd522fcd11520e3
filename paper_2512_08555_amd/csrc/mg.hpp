// Kernels of the multigrid cycle (Sec. 3.1, Alg. amg_vcycle) on node grids
// laid out [z][y][x], x fastest, in float or double.
#pragma once
#include <hip/hip_runtime.h>

namespace ups {

// node counts of one level
struct MgGrid {
  int nx, ny, nz;
};

// a refined box inside its parent: node 0 of the box lies on parent node
// (ox, oy, oz); the box spans (mx, my, mz) parent cells, 2 m + 1 nodes
struct MgBox {
  int ox, oy, oz, mx, my, mz;
};

// ghost layer of u (grid g) = cubic reconstruction from the parent up (grid
// gp): at each odd fine index, one axis at a time (z, y, x), (-1, 9, 9,
// -1)/16 of the four nearest parent nodes, which reach one node beyond the
// footprint of box b on every side
hipError_t mg_fill_ghosts(bool f64, void* u, MgGrid g, const void* up, MgGrid gp, MgBox b, hipStream_t st);

// nu red-black iterations on u, the same values as 2 nu half-steps (red:
// every unknown with (x + y + z) even set to (sum of its six neighbours -
// h^2 f) / 6, then black): whole iterations by the fused kernel, u -> s ->
// u ..., and a copy back into u if they end in s (s: a scratch array of the
// level's size).  With from_s the values start in s instead of u.
hipError_t mg_smooth_iterations(bool f64, void* u, void* s, const void* f, MgGrid g, double h, int nu,
                                hipStream_t st, bool from_s = false);

// nu red-black iterations from u, alternately into s and back, then r =
// f - Lap u on the unknowns, the last iteration and the residual in one
// kernel.  The smoothed values end in u after an even nu and in s after an
// odd one; *out says which (s: a scratch array of the level's size,
// different from r)
hipError_t mg_smooth_residual(bool f64, void* u, void* s, const void* f, void* r, MgGrid g, double h, int nu,
                              hipStream_t st, void** out);

// r = f - Lap u on the unknowns (the ghost layer of r is not written)
hipError_t mg_residual(bool f64, const void* u, const void* f, void* r, MgGrid g, double h, hipStream_t st);

// on the parent's unknowns inside the footprint of b: up = injection of u,
// fp = full weighting of r + Lap up (parent spacing hp); uhat = up on the
// whole footprint ((mx+1) (my+1) (mz+1) values, x fastest)
hipError_t mg_restrict(bool f64, const void* u, const void* r, MgGrid g, void* up, void* fp, void* uhat, MgGrid gp,
                       MgBox b, double hp, hipStream_t st);

// unknowns of u = those of uin + trilinear prolongation of (up - uhat)
// (uin may be u); ghost layer of u = cubic reconstruction from up
hipError_t mg_prolong(bool f64, const void* uin, void* u, MgGrid g, const void* up, const void* uhat, MgGrid gp,
                      MgBox b, hipStream_t st);

// *out = max(*out, max |f - Lap u|) over the unknowns of g outside the
// interior of the footprint of `child` (none if null); *out must start at 0
hipError_t mg_residual_norm(bool f64, const void* u, const void* f, MgGrid g, double h, const MgBox* child,
                            double* out, hipStream_t st);

// n doubles of p set to 0
hipError_t mg_zero(double* p, int n, hipStream_t st);

}  // namespace ups
