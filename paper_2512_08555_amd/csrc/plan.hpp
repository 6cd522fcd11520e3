// Plan geometry and the opaque plan object behind ups_plan_t.
#pragma once
#include <cstddef>

#include "../../include/ups.h"
#include "passes.hpp"

namespace ups {

struct PlanGeom {
  bool f64;
  size_t elem;               // bytes of one real element
  int nx, ny, nz;            // points
  int mx, my, mz;            // padded lengths
  int kx, oy, oz;            // stored x frequencies, octant extents in y and z
  int px;                    // row pitch of W (elements)
  int gz;                    // iz pitch of G_hat [iy][kx][iz] (elements)
  int ncomp;
  int bc[3];                 // ups_bc per axis (x, y, z); both sides equal
  int green;                 // ups_green
  double h;
  long long plane, comp_w;   // W strides (complex elements)
  size_t solve_work;         // bytes of W
  size_t guard;              // bytes of each canary band around W (guard mode), else 0
  size_t work_bytes;         // max(guard + W + guard, setup scratch)
  size_t green_bytes;
  size_t off_ghat, off_twx, off_twy, off_twz;
  size_t off_status;         // one status word of the debug checks (green buffer)
  // W's column 0 carries X[0] + i X[mx/2] (single plans at mx = 1024 whose
  // x and z passes run the wave-per-line kernels; see PassArgs::nyq)
  bool nyq;
};

ups_status validate_problem(const ups_problem* p, PlanGeom* g);
// guards: lay out canary bands around W in the work buffer (guard mode)
void plan_layout(PlanGeom& g, bool guards = false);
double model_bytes(const PlanGeom& g, int pass);
// fill: 1 for the mirrored-fill forward variants of even and odd directions
const PassVariant* find_variant(PassKind kind, bool f64, int length, const char* name, int fill = 0);
// 1 if pass `kind` runs along an even or odd direction of g and needs a
// mirrored-fill variant, else 0
int pass_fill(PassKind kind, const PlanGeom& g);
const PassVariant* tuned_variant(PassKind kind, bool f64, int length, const PlanGeom& g);
// Whether variant v may run its pass on g: with g.nyq the x passes and the
// z pass must be wave-per-line kernels (the ones that pack, unpack and pair
// column 0)
bool variant_allowed(const PassVariant& v, const PlanGeom& g);
// Decide g.nyq for a single plan (before plan_layout): FP32, mx = 1024,
// mz = 512 or 1024, x and z neither even nor odd, one column slab
void choose_nyq(PlanGeom& g);
PassArgs make_args(const PlanGeom& g, const void* green);
ups_status check_device(int* dev_out);
ups_status set_error(ups_status s, const char* msg);
// A second stream (default priority) and its events.  With one column slab
// the remainder launch of a split column pass runs beside the main launch
// (fork on `fork`, join on `join`).  With several slabs the z pass runs on
// the second stream, slab by slab, while the main stream runs the y passes
// of the other slabs (ev[2 s]: y-forward of slab s done, ev[2 s + 1]: z of
// slab s done).
struct SideStream {
  static constexpr int kMaxSlabs = 16;
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipEvent_t ev[2 * kMaxSlabs] = {};
};
ups_status enqueue_solve(const PlanGeom& g, const PassVariant* const var[5], const PassArgs& a, int slab,
                         const void* f, void* u, void* work, hipStream_t st, const SideStream* side);
int default_slab(const PlanGeom& g);
bool default_side(const PlanGeom& g);
hipError_t enqueue_colpass(const PlanGeom& g, const PassVariant* v, const PassArgs& a, void* ws, hipStream_t st,
                           const SideStream* side = nullptr);
int slab_count(const PlanGeom& g, int slab);
PassArgs slab_args(const PlanGeom& g, const PassArgs& a, int slab, int s, void* work, void** wslab);

}  // namespace ups

struct ups_plan_s {
  ups_problem prob;
  ups::PlanGeom g;
  const ups::PassVariant* var[5];
  void* green = nullptr;
  void* work = nullptr;
  int device = 0;
  bool ready = false;
  int slab = 0;              // kx columns per y/z/y slab (0: one slab)
  ups::PassArgs args{};
  ups::SideStream side;
  bool use_side = false;     // remainder launches on the side stream
  bool check_finite = false; // ups_solve first checks its input for NaN / Inf
  bool guards = false;       // guard mode (UPS_DEBUG_GUARDS): canary bands, NaN poison
  // the solve's W: the work buffer, past the low canary band in guard mode
  void* wbuf() const { return static_cast<char*>(work) + g.guard; }
  ~ups_plan_s();
};
