// C ABI of the multigrid V(nu1, nu2) cycle around the solve (Sec. 3.1, Alg.
// amg_vcycle): validation, work-buffer layout and the sequence of kernel
// launches of one cycle.  The kernels are in multigrid.hip; the coarsest
// level is solved by the plan's own five-pass schedule.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <vector>

#include "../../include/ups.h"
#include "mg.hpp"
#include "plan.hpp"
#include "trace.hpp"

using namespace ups;

struct ups_mg_s {
  ups_plan_t plan = nullptr;
  int levels = 0;
  std::vector<MgGrid> grid;       // levels 0 .. l
  std::vector<MgBox> box;         // box k+1 (a child of level k) at index k
  std::vector<double> h;          // spacing of each level
  std::vector<size_t> off_F;      // modified sources of levels 0 .. l-1
  std::vector<size_t> off_uhat;   // stored footprint of box k+1 at index k
  std::vector<size_t> off_s;      // the smoother's scratch array of level k at index k - 1
  size_t off_norm = 0, off_r = 0, bytes = 0;
  void* work = nullptr;
};

namespace {

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

size_t nodes(const MgGrid& g) { return (size_t)g.nx * g.ny * g.nz; }

ups_status check_arrays(ups_mg_t mg, const void* const* f, void* const* u) {
  if (!f || !u) return set_error(UPS_ERR_INVALID_ARG, "f and u must be host arrays of device pointers");
  const uintptr_t al = 2 * mg->plan->g.elem - 1;
  for (int k = 0; k <= mg->levels; ++k) {
    if (!f[k] || !u[k]) return set_error(UPS_ERR_INVALID_ARG, "null level array");
    if ((reinterpret_cast<uintptr_t>(f[k]) | reinterpret_cast<uintptr_t>(u[k])) & al)
      return set_error(UPS_ERR_INVALID_ARG, "level arrays must be aligned to 2 * sizeof(element) bytes");
  }
  return UPS_OK;
}

ups_status check_ready(ups_mg_t mg) {
  if (!mg) return set_error(UPS_ERR_INVALID_ARG, "cycle object is NULL");
  if (!mg->work) return set_error(UPS_ERR_STATE, "ups_mg_setup has not bound a work buffer");
  if (!mg->plan->ready) return set_error(UPS_ERR_STATE, "the coarse plan is not set up");
  return UPS_OK;
}

}  // namespace

extern "C" {

ups_status ups_mg_create(ups_plan_t coarse, const ups_mg_hierarchy* hier, ups_mg_t* out) {
  if (!out) return set_error(UPS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!coarse || !hier) return set_error(UPS_ERR_INVALID_ARG, "plan and hierarchy must not be NULL");
  const PlanGeom& pg = coarse->g;
  if (pg.ncomp != 1) return set_error(UPS_ERR_UNSUPPORTED, "the coarse plan must have one component");
  if (pg.green != UPS_GREEN_LGF2)
    return set_error(UPS_ERR_UNSUPPORTED,
                     "the coarse kernel must be the LGF of the 7-point operator the cycle smooths with");
  if (hier->levels < 0 || hier->levels > UPS_MG_MAX_LEVELS)
    return set_error(UPS_ERR_UNSUPPORTED, "levels must be 0 .. UPS_MG_MAX_LEVELS");
  ups_mg_s* mg = new ups_mg_s();
  mg->plan = coarse;
  mg->levels = hier->levels;
  mg->grid.push_back(MgGrid{pg.nx, pg.ny, pg.nz});
  mg->h.push_back(pg.h);
  for (int k = 0; k < hier->levels; ++k) {
    const MgGrid& p = mg->grid.back();
    const int np[3] = {p.nx, p.ny, p.nz};
    int n[3];
    for (int a = 0; a < 3; ++a) {
      const int c = hier->origin[k][a], m = hier->cells[k][a];
      if (m < 2 || c < 1 || (long long)c + m > (long long)np[a] - 2) {
        delete mg;
        return set_error(UPS_ERR_INVALID_ARG,
                         "every box needs cells >= 2, origin >= 1 and origin + cells <= parent nodes - 2 on every axis");
      }
      n[a] = 2 * m + 1;
    }
    if ((long long)n[0] * n[1] * n[2] > INT_MAX) {
      delete mg;
      return set_error(UPS_ERR_INVALID_ARG, "a level holds more than 2^31 - 1 nodes");
    }
    mg->box.push_back(MgBox{hier->origin[k][0], hier->origin[k][1], hier->origin[k][2], hier->cells[k][0],
                            hier->cells[k][1], hier->cells[k][2]});
    mg->grid.push_back(MgGrid{n[0], n[1], n[2]});
    mg->h.push_back(mg->h.back() * 0.5);
  }
  for (const MgGrid& g : mg->grid)
    if (g.nz > 65535 || g.ny > 4 * 65535) {
      delete mg;
      return set_error(UPS_ERR_UNSUPPORTED, "a level has more than 65535 nodes along z or 262140 along y");
    }
  const size_t el = pg.elem;
  size_t off = 0;
  mg->off_norm = off;
  off = align256(off + sizeof(double) * (UPS_MG_MAX_LEVELS + 1));
  for (int k = 0; k < mg->levels; ++k) {
    mg->off_F.push_back(off);
    off = align256(off + nodes(mg->grid[k]) * el);
  }
  size_t rmax = 0;
  for (int k = 1; k <= mg->levels; ++k) rmax = std::max(rmax, nodes(mg->grid[k]) * el);
  mg->off_r = off;
  off = align256(off + rmax);
  for (int k = 1; k <= mg->levels; ++k) {
    mg->off_s.push_back(off);
    off = align256(off + nodes(mg->grid[k]) * el);
  }
  for (int k = 0; k < mg->levels; ++k) {
    const MgBox& b = mg->box[k];
    mg->off_uhat.push_back(off);
    off = align256(off + (size_t)(b.mx + 1) * (b.my + 1) * (b.mz + 1) * el);
  }
  mg->bytes = off;
  if (log_level() >= 2) {
    logf(2, "cycle %p: %d refined level(s) over plan %p, work %zu B", static_cast<void*>(mg), mg->levels,
         static_cast<void*>(coarse), mg->bytes);
    for (int k = 0; k <= mg->levels; ++k)
      logf(2, "cycle %p level %d: %d x %d x %d nodes, h %.6g", static_cast<void*>(mg), k, mg->grid[k].nx,
           mg->grid[k].ny, mg->grid[k].nz, mg->h[k]);
  }
  *out = mg;
  return set_error(UPS_OK, "");
}

ups_status ups_mg_level_shape(ups_mg_t mg, int level, int n[3]) {
  if (!mg || !n) return set_error(UPS_ERR_INVALID_ARG, "NULL argument");
  if (level < 0 || level > mg->levels) return set_error(UPS_ERR_INVALID_ARG, "level out of range");
  n[0] = mg->grid[level].nx;
  n[1] = mg->grid[level].ny;
  n[2] = mg->grid[level].nz;
  return set_error(UPS_OK, "");
}

ups_status ups_mg_sizes(ups_mg_t mg, size_t* work_bytes) {
  if (!mg || !work_bytes) return set_error(UPS_ERR_INVALID_ARG, "NULL argument");
  *work_bytes = mg->bytes;
  return set_error(UPS_OK, "");
}

ups_status ups_mg_setup(ups_mg_t mg, void* work, size_t work_bytes) {
  if (!mg || !work) return set_error(UPS_ERR_INVALID_ARG, "NULL argument");
  if (reinterpret_cast<uintptr_t>(work) & 255) return set_error(UPS_ERR_INVALID_ARG, "work must be 256-byte aligned");
  if (work_bytes < mg->bytes) return set_error(UPS_ERR_WORKSPACE, "work buffer smaller than ups_mg_sizes");
  mg->work = work;
  return set_error(UPS_OK, "");
}

ups_status ups_mg_cycle(ups_mg_t mg, const void* const* f, void* const* u, int nu1, int nu2, void* stream) {
  ups_status s = check_ready(mg);
  if (s != UPS_OK) return s;
  s = check_arrays(mg, f, u);
  if (s != UPS_OK) return s;
  if (nu1 < 0 || nu1 > 64 || nu2 < 0 || nu2 > 64)
    return set_error(UPS_ERR_INVALID_ARG, "nu1 and nu2 must be 0 .. 64");
  TraceRange range("ups_mg_cycle");
  logf(3, "cycle %p: V(%d, %d), stream %p", static_cast<void*>(mg), nu1, nu2, stream);
  const bool f64 = mg->plan->g.f64;
  const size_t el = mg->plan->g.elem;
  const int L = mg->levels;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* wb = static_cast<char*>(mg->work);
  // the source each level smooths with: the caller's on the finest level,
  // the modified copies below it
  std::vector<void*> F(L + 1);
  for (int k = 0; k < L; ++k) F[k] = wb + mg->off_F[k];
  F[L] = const_cast<void*>(f[L]);
  void* r = wb + mg->off_r;
  // where each refined level's pre-smoothed values are: u[k] or its scratch
  // array, which no other level touches, so they stay there until the
  // prolongation reads them
  std::vector<void*> cur(L + 1);
  hipError_t e = hipSuccess;
  for (int k = 0; k < L && e == hipSuccess; ++k)
    e = hipMemcpyAsync(F[k], f[k], nodes(mg->grid[k]) * el, hipMemcpyDeviceToDevice, st);
  for (int k = L; k >= 1 && e == hipSuccess; --k) {
    const MgGrid& g = mg->grid[k];
    const MgGrid& gp = mg->grid[k - 1];
    const MgBox& b = mg->box[k - 1];
    e = mg_fill_ghosts(f64, u[k], g, u[k - 1], gp, b, st);
    if (e == hipSuccess)
      e = mg_smooth_residual(f64, u[k], wb + mg->off_s[k - 1], F[k], r, g, mg->h[k], nu1, st, &cur[k]);
    if (e == hipSuccess)
      e = mg_restrict(f64, cur[k], r, g, u[k - 1], F[k - 1], wb + mg->off_uhat[k - 1], gp, b, mg->h[k - 1], st);
  }
  if (e != hipSuccess) return set_error(UPS_ERR_DEVICE, hipGetErrorString(e));
  ups_plan_t p = mg->plan;
  s = enqueue_solve(p->g, p->var, p->args, p->slab, F[0], u[0], p->wbuf(), st, p->use_side ? &p->side : nullptr);
  if (s != UPS_OK) return s;
  for (int k = 1; k <= L && e == hipSuccess; ++k) {
    const MgGrid& g = mg->grid[k];
    void* sm = wb + mg->off_s[k - 1];
    // after an odd nu2 the iterations end where they did not start: the
    // prolongation then writes into the scratch array, and no copy is needed
    const bool odd = nu2 & 1;
    e = mg_prolong(f64, cur[k], odd ? sm : u[k], g, u[k - 1], wb + mg->off_uhat[k - 1], mg->grid[k - 1],
                   mg->box[k - 1], st);
    if (e == hipSuccess) e = mg_smooth_iterations(f64, u[k], sm, F[k], g, mg->h[k], nu2, st, odd);
  }
  if (e != hipSuccess) return set_error(UPS_ERR_DEVICE, hipGetErrorString(e));
  return set_error(UPS_OK, "");
}

ups_status ups_mg_residual(ups_mg_t mg, const void* const* f, void* const* u, double* norms, void* stream) {
  ups_status s = check_ready(mg);
  if (s != UPS_OK) return s;
  s = check_arrays(mg, f, u);
  if (s != UPS_OK) return s;
  if (!norms) return set_error(UPS_ERR_INVALID_ARG, "norms is NULL");
  const bool f64 = mg->plan->g.f64;
  const int L = mg->levels;
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* dn = reinterpret_cast<double*>(static_cast<char*>(mg->work) + mg->off_norm);
  hipError_t e = mg_zero(dn, L + 1, st);
  for (int k = 1; k <= L && e == hipSuccess; ++k)
    e = mg_fill_ghosts(f64, u[k], mg->grid[k], u[k - 1], mg->grid[k - 1], mg->box[k - 1], st);
  for (int k = 0; k <= L && e == hipSuccess; ++k) {
    const MgGrid& g = mg->grid[k];
    if (g.nx < 3 || g.ny < 3 || g.nz < 3) continue;
    e = mg_residual_norm(f64, u[k], f[k], g, mg->h[k], k < L ? &mg->box[k] : nullptr, dn + k, st);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(norms, dn, sizeof(double) * (L + 1), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return set_error(UPS_ERR_DEVICE, hipGetErrorString(e));
  return set_error(UPS_OK, "");
}

ups_status ups_mg_destroy(ups_mg_t mg) {
  delete mg;
  return set_error(UPS_OK, "");
}

}  // extern "C"
