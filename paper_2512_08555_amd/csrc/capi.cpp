// C ABI of libups: problem validation, plans, buffer layout, and the solve
// entry points.  See include/ups.h for the contract of every call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>

#include "../../include/ups.h"
#include "debug.hpp"
#include "green.hpp"
#include "passes.hpp"
#include "plan.hpp"
#include "trace.hpp"

using namespace ups;

namespace {
thread_local std::string g_err;

ups_status fail(ups_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  if (s != UPS_OK) logf(1, "error %d: %s", int(s), buf);
  return s;
}
ups_status ok() {
  g_err.clear();
  return UPS_OK;
}
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
}  // namespace

namespace ups {

ups_status set_error(ups_status s, const char* msg) { return fail(s, "%s", msg); }

const PassVariant* find_variant(PassKind kind, bool f64, int length, const char* name, int fill) {
  const PassVariant* best = nullptr;
  for (const PassVariant& v : pass_variants()) {
    if (v.kind != kind || v.is_f64 != (f64 ? 1 : 0) || v.length != length || v.fill != fill) continue;
    if (name && std::strcmp(name, v.name) != 0) continue;
    if (!best) best = &v;
  }
  return best;
}

int pass_fill(PassKind kind, const PlanGeom& g) {
  const int axis = kind == PASS_XFWD ? 0 : kind == PASS_YFWD ? 1 : kind == PASS_ZCONV ? 2 : -1;
  return axis >= 0 && (g.bc[axis] == UPS_BC_EVEN || g.bc[axis] == UPS_BC_ODD) ? 1 : 0;
}

bool length_supported(int len, bool f64) {
  return find_variant(PASS_XFWD, f64, len, nullptr) && find_variant(PASS_YFWD, f64, len, nullptr) &&
         find_variant(PASS_ZCONV, f64, len, nullptr);
}

ups_status validate_problem(const ups_problem* p, PlanGeom* g) {
  if (!p) return fail(UPS_ERR_INVALID_ARG, "problem is NULL");
  for (int i = 0; i < 3; ++i) {
    if (p->n[i] < 2) return fail(UPS_ERR_INVALID_ARG, "n[%d] = %d: need at least 2 points", i, p->n[i]);
    if (p->n[i] > 4096) return fail(UPS_ERR_UNSUPPORTED, "n[%d] = %d exceeds 4096", i, p->n[i]);
    if (!(p->h[i] > 0.0) || !std::isfinite(p->h[i]))
      return fail(UPS_ERR_INVALID_ARG, "h[%d] must be positive and finite", i);
    for (int s = 0; s < 2; ++s) {
      if (p->bc[i][s] < UPS_BC_UNB || p->bc[i][s] > UPS_BC_ODD)
        return fail(UPS_ERR_INVALID_ARG, "bc[%d][%d] = %d is not a ups_bc", i, s, p->bc[i][s]);
    }
    if (p->bc[i][0] != p->bc[i][1])
      return fail(UPS_ERR_UNSUPPORTED, "bc[%d]: both sides of an axis must carry the same condition", i);
    if ((p->bc[i][0] == UPS_BC_EVEN || p->bc[i][0] == UPS_BC_ODD) && p->center != UPS_CELL)
      return fail(UPS_ERR_UNSUPPORTED, "bc[%d]: even and odd directions mirror about cell faces (UPS_CELL)", i);
  }
  const bool any_spectral = p->bc[0][0] != UPS_BC_UNB || p->bc[1][0] != UPS_BC_UNB || p->bc[2][0] != UPS_BC_UNB;
  if (std::fabs(p->h[0] - p->h[1]) > 1e-12 * p->h[0] || std::fabs(p->h[0] - p->h[2]) > 1e-12 * p->h[0])
    return fail(UPS_ERR_UNSUPPORTED, "anisotropic spacing is not supported (h must be equal)");
  if (p->green < UPS_GREEN_LGF2 || p->green > UPS_GREEN_LGF6_MEHR)
    return fail(UPS_ERR_INVALID_ARG, "green = %d is not a ups_green", p->green);

  if (p->prec != UPS_F64 && p->prec != UPS_F32) return fail(UPS_ERR_INVALID_ARG, "prec = %d", p->prec);
  if (p->center != UPS_CELL && p->center != UPS_NODE)
    return fail(UPS_ERR_INVALID_ARG, "center = %d", p->center);
  if (p->ncomp < 1 || p->ncomp > 8) return fail(UPS_ERR_INVALID_ARG, "ncomp = %d not in 1..8", p->ncomp);
  const bool f64 = p->prec == UPS_F64;
  int M[3];
  for (int i = 0; i < 3; ++i) {
    // Any even M >= 2n - 2 makes the circular convolution exact, but the
    // kernels prune on inputs n >= M/2 being zero and outputs n >= M/2
    // being dropped, which needs M >= 2n.
    M[i] = p->pad[i] ? p->pad[i] : 2 * p->n[i];
    if (M[i] % 2 || M[i] < 2 * p->n[i])
      return fail(UPS_ERR_INVALID_ARG, "pad[%d] = %d: must be even and >= 2 n = %d", i, M[i], 2 * p->n[i]);
    // a periodic direction is padded to exactly 2 n: its kernel is the
    // n-periodic Green's function, whose spectrum lives on the even
    // frequencies of that grid
    if (p->bc[i][0] == UPS_BC_PER && M[i] != 2 * p->n[i])
      return fail(UPS_ERR_INVALID_ARG, "pad[%d] = %d: a periodic direction takes pad = 2 n = %d (or 0)", i, M[i],
                  2 * p->n[i]);
    // an even or odd direction is extended to 2 n by its mirror image
    const bool mirror = p->bc[i][0] == UPS_BC_EVEN || p->bc[i][0] == UPS_BC_ODD;
    if (mirror && M[i] != 2 * p->n[i])
      return fail(UPS_ERR_INVALID_ARG, "pad[%d] = %d: an even or odd direction takes pad = 2 n = %d (or 0)", i,
                  M[i], 2 * p->n[i]);
    if (mirror && i == 0 && p->n[0] % 2)
      return fail(UPS_ERR_UNSUPPORTED, "an even or odd x direction needs an even n[0] (got %d)", p->n[0]);
    const PassKind fwd = i == 0 ? PASS_XFWD : i == 1 ? PASS_YFWD : PASS_ZCONV;
    if (mirror && !find_variant(fwd, p->prec == UPS_F64, M[i], nullptr, 1))
      return fail(UPS_ERR_UNSUPPORTED, "even/odd direction %d: no mirrored-fill kernel for length %d", i, M[i]);
  }
  if (any_spectral && p->green != UPS_GREEN_LGF2)
    return fail(UPS_ERR_UNSUPPORTED, "non-unbounded directions are solved with the 7-point kernel only");
  if (p->green != UPS_GREEN_LGF2 && (M[0] > 1024 || M[1] > 1024 || M[2] > 1024))
    return fail(UPS_ERR_UNSUPPORTED, "Mehrstellen kernels are built for padded lengths up to 1024");
  for (int i = 0; i < 3; ++i) {
    if (!length_supported(M[i], f64))
      return fail(UPS_ERR_UNSUPPORTED, "padded length %d (axis %d) has no compiled %s kernel", M[i], i,
                  f64 ? "double" : "float");
  }
  g->f64 = f64;
  g->elem = f64 ? 8 : 4;
  g->nx = p->n[0];
  g->ny = p->n[1];
  g->nz = p->n[2];
  g->mx = M[0];
  g->my = M[1];
  g->mz = M[2];
  g->kx = g->mx / 2 + 1;
  g->oy = g->my / 2 + 1;
  g->oz = g->mz / 2 + 1;
  g->px = int(align_up(size_t(g->kx), 16));
  g->gz = int(align_up(size_t(g->oz), 16));
  g->ncomp = p->ncomp;
  g->h = p->h[0];
  for (int i = 0; i < 3; ++i) g->bc[i] = p->bc[i][0];
  g->green = p->green;
  // Every kernel addresses W as a wave-uniform 64-bit base plus a 32-bit
  // per-lane byte offset of at most 64 line strides (a row of a 64-row
  // block or of a split factor <= 64) plus a tile column; the longest line
  // stride is the plane.  Refuse geometries where that could wrap.
  const unsigned long long lane_max =
      (64ull * (unsigned long long)g->my * (unsigned long long)g->px + 16ull) * (2ull * g->elem);
  if (lane_max >= (1ull << 32))
    return fail(UPS_ERR_UNSUPPORTED, "padded lengths (%d, %d, %d): per-lane offsets exceed 32 bits", g->mx, g->my,
                g->mz);
  return UPS_OK;
}

bool variant_allowed(const PassVariant& v, const PlanGeom& g) {
  if (!g.nyq) return true;
  return !(v.kind == PASS_XFWD || v.kind == PASS_XINV || v.kind == PASS_ZCONV) || v.nch == 0;
}

void choose_nyq(PlanGeom& g) {
  const bool mirrored_xz = g.bc[0] == UPS_BC_EVEN || g.bc[0] == UPS_BC_ODD || g.bc[2] == UPS_BC_EVEN ||
                           g.bc[2] == UPS_BC_ODD;
  g.nyq = !g.f64 && g.mx == 1024 && (g.mz == 512 || g.mz == 1024) && !mirrored_xz && default_slab(g) == 0;
}

void plan_layout(PlanGeom& g, bool guards) {
  const size_t ce = 2 * g.elem;  // complex element
  g.plane = (long long)g.my * g.px;
  g.comp_w = (long long)g.nz * g.plane;
  g.solve_work = align_up(ce * (size_t)g.comp_w * g.ncomp, 256);
  g.guard = guards ? kGuardBytes : 0;
  const size_t gbytes = g.green == UPS_GREEN_LGF2
                            ? green_scratch_layout(g.oz, g.oy, g.kx).bytes
                            : mehr_scratch_layout(g.oz, g.oy, g.kx, g.green == UPS_GREEN_LGF4_MEHR ? 4 : 6).bytes;
  const int mmax = std::max(g.mx, std::max(g.my, g.mz));
  const size_t setup = std::max(gbytes, align_up(sizeof(double) * 2 * twiddle_entries(mmax), 256));
  g.work_bytes = std::max(g.solve_work + 2 * g.guard, setup);
  size_t off = 0;
  g.off_ghat = off;
  off = align_up(off + g.elem * (size_t)g.oy * g.kx * g.gz, 256);
  g.off_twx = off;
  off = align_up(off + ce * twiddle_entries(g.mx), 256);
  g.off_twy = off;
  off = align_up(off + ce * twiddle_entries(g.my), 256);
  g.off_twz = off;
  off = align_up(off + ce * twiddle_entries(g.mz), 256);
  g.off_status = off;
  off += 256;
  g.green_bytes = off;
}

double model_bytes(const PlanGeom& g, int pass) {
  const double s = double(g.elem), c = 2.0 * s, nc = g.ncomp;
  const double nxyz = double(g.nx) * g.ny * g.nz;
  const double xw = double(g.kx) * g.ny * g.nz;        // x-transformed, rows y < ny
  const double yw = double(g.kx) * g.my * g.nz;        // y-expanded
  const double gh = double(g.kx) * g.oy * g.oz * s;    // G_hat octant
  switch (pass) {
    case 0: return nc * (nxyz * s + xw * c);
    case 1: return nc * (xw * c + yw * c);
    case 2: return nc * (2.0 * yw * c) + gh;
    case 3: return nc * (yw * c + xw * c);
    case 4: return nc * (xw * c + nxyz * s);
    case -1: {
      double t = 0;
      for (int i = 0; i < 5; ++i) t += model_bytes(g, i);
      return t;
    }
    default: return 0.0;
  }
}

ups_status check_device(int* dev_out) {
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return fail(UPS_ERR_DEVICE, "no HIP device available");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(UPS_ERR_DEVICE, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return fail(UPS_ERR_DEVICE, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(UPS_ERR_DEVICE, "device %d is %s; this library is built for gfx950 only", dev,
                prop.gcnArchName);
  *dev_out = dev;
  return UPS_OK;
}

PassArgs make_args(const PlanGeom& g, const void* green) {
  PassArgs a{};
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.mx = g.mx;
  a.my = g.my;
  a.mz = g.mz;
  a.kx = g.nyq ? g.kx - 1 : g.kx;
  a.nyq = g.nyq ? 1 : 0;
  a.px = g.px;
  a.plane = g.plane;
  a.comp_w = g.comp_w;
  a.comp_f = (long long)g.nx * g.ny * g.nz;
  a.gz = g.gz;
  a.g_plane = (long long)g.kx * g.gz;
  a.ncomp = g.ncomp;
  auto sign = [](int bc) { return bc == UPS_BC_EVEN ? 1 : bc == UPS_BC_ODD ? -1 : 0; };
  a.fill_x = sign(g.bc[0]);
  a.fill_y = sign(g.bc[1]);
  a.fill_z = sign(g.bc[2]);
  if (green) {  // (a geometry-only PassArgs, e.g. for block counts, has no buffers)
    const char* gb = static_cast<const char*>(green);
    a.ghat = gb + g.off_ghat;
    a.tw_x = gb + g.off_twx;
    a.tw_y = gb + g.off_twy;
    a.tw_z = gb + g.off_twz;
  }
  return a;
}

// Column slabs.  The y-forward, z and y-inverse passes act on each kx
// column independently, so they can run slab by slab: y-forward, z, y-inverse
// on columns [k0, k0 + w), then the next slab.  A slab's padded spectrum
// (w * my * nz complex values per component) then stays in the device's
// last-level cache from the pass that writes it to the pass that reads it.
// Slab starts are multiples of 16 columns (128-byte lines of float complex
// values); the last slab also takes the remainder.
// Run one after the other, slabs do not pay (measured on MI355X at 512^3:
// the column passes are not limited by HBM traffic).  Pipelined over two
// streams (enqueue_solve), the z pass of one slab runs beside the y passes
// of the others; measured at 512^3 that takes FP64 from 6.29 to 6.12 ms
// with 128-column slabs and slows FP32 (3.09 -> 3.13 ms), so FP64 plans with
// at least 384 columns start with 128-column slabs on two streams.
// With one slab, running the narrow remainder launches of the three column
// passes on the second stream (enqueue_solve) takes FP64 at 256^3 from 0.741
// to 0.733 ms (forked after the x pass) and FP32 at 512^3 from 3.000 to
// 2.984 ms (forked after the main y-forward launch), so every plan starts
// with the second stream on.
int default_slab(const PlanGeom& g) { return g.f64 && g.kx >= 384 ? 128 : 0; }
bool default_side(const PlanGeom&) { return true; }

int slab_count(const PlanGeom& g, int slab) {
  if (slab <= 0 || slab >= g.kx) return 1;
  return std::max(1, g.kx / slab);
}

PassArgs slab_args(const PlanGeom& g, const PassArgs& a, int slab, int s, void* work, void** wslab) {
  const int ns = slab_count(g, slab);
  if (ns == 1) {
    *wslab = work;
    return a;
  }
  const int k0 = s * slab;
  const int k1 = s == ns - 1 ? g.kx : k0 + slab;
  PassArgs b = a;
  b.kx = k1 - k0;
  b.ghat = static_cast<const char*>(a.ghat) + size_t(k0) * g.gz * g.elem;
  *wslab = static_cast<char*>(work) + size_t(k0) * 2 * g.elem;
  return b;
}

// A column pass over columns [k0, k0 + w) of W (and of G_hat).
static PassArgs column_range(const PlanGeom& g, const PassArgs& a, int k0, int w, void* ws, void** out) {
  PassArgs b = a;
  b.kx = w;
  b.ghat = static_cast<const char*>(a.ghat) + size_t(k0) * g.gz * g.elem;
  *out = static_cast<char*>(ws) + size_t(k0) * 2 * g.elem;
  return b;
}

// The column passes (y-forward, z, y-inverse) run best when every XCD keeps
// the same columns for all lines and all XCDs get equal shares (measured on
// MI355X: 20% for the y-forward pass at 512^3): the launch covers a multiple
// of 8 x (columns per 128-byte line) columns, and the columns left over get
// a second launch (tail_variant).
static int colpass_align(const PlanGeom& g) { return 8 * (128 / int(2 * g.elem)); }

// The variant for the `rest` columns past the aligned launch: the narrowest
// variant of the pass for a single column, the pass's own variant (its last
// tile partly filled) for more.  The narrow variants read one value per
// 128-byte line, so running many columns through them is slow (measured on
// MI355X at 512^3 FP64: 13.1 ms with 96-column slabs, whose 32-column
// remainders went to them, against 6.05 ms with 64-column slabs).
static const PassVariant* tail_variant(const PassVariant& v, int rest) {
  const PassVariant* nv = narrow_variant(v);
  if (!nv) return nullptr;
  return rest == 1 ? nv : &v;
}

hipError_t enqueue_colpass(const PlanGeom& g, const PassVariant* v, const PassArgs& a, void* ws, hipStream_t st,
                           const SideStream* side) {
  const int align = colpass_align(g);
  const int kmain = a.kx / align * align;
  const PassVariant* nv = tail_variant(*v, a.kx - kmain);
  if (!nv || kmain == 0 || kmain == a.kx) {
    if (a.nyq && v->kind == PASS_ZCONV) {
      // the pair launch owns column 0: beside the main launch on the side
      // stream (forked and joined here), else after it
      hipError_t e = hipSuccess;
      const bool fork = side && side->s;
      if (fork) {
        e = hipEventRecord(side->fork, st);
        if (e == hipSuccess) e = hipStreamWaitEvent(side->s, side->fork, 0);
        if (e == hipSuccess) e = launch_zpair(g.f64, a, ws, side->s);
        if (e == hipSuccess) e = hipEventRecord(side->join, side->s);
      }
      if (e != hipSuccess) return e;
      v->launch(a, ws, ws, st);
      e = hipGetLastError();
      if (e == hipSuccess) e = fork ? hipStreamWaitEvent(st, side->join, 0) : launch_zpair(g.f64, a, ws, st);
      return e;
    }
    v->launch(a, ws, ws, st);
    return hipGetLastError();
  }
  void* wm = nullptr;
  void* wr = nullptr;
  const PassArgs am = column_range(g, a, 0, kmain, ws, &wm);
  const PassArgs ar = column_range(g, a, kmain, a.kx - kmain, ws, &wr);
  if (side && side->s) {
    // nothing is enqueued on the side stream unless the fork is in place,
    // and the caller's stream waits for the join before it continues
    hipError_t e = hipEventRecord(side->fork, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(side->s, side->fork, 0);
    if (e != hipSuccess) return e;
    nv->launch(ar, wr, wr, side->s);
    e = hipEventRecord(side->join, side->s);
    v->launch(am, wm, wm, st);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, side->join, 0);
    if (e != hipSuccess) return e;
  } else {
    v->launch(am, wm, wm, st);
    nv->launch(ar, wr, wr, st);
  }
  return hipGetLastError();
}

ups_status enqueue_solve(const PlanGeom& g, const PassVariant* const var[5], const PassArgs& a, int slab,
                         const void* f, void* u, void* work, hipStream_t st, const SideStream* side) {
  static const char* const kRange[5] = {"ups:xfwd", "ups:yfwd", "ups:zconv", "ups:yinv", "ups:xinv"};
  {
    TraceRange r(kRange[0]);
    var[0]->launch(a, f, work, st);
  }
  const int ns = slab_count(g, slab);
  if (side && side->s && ns > 1 && ns <= SideStream::kMaxSlabs) {
    // pipeline: the y passes on st, the z pass on the side stream, so that a
    // slab's z pass (bound by arithmetic) overlaps other slabs' y passes
    // (bound by memory)
    void* ws[SideStream::kMaxSlabs];
    PassArgs b[SideStream::kMaxSlabs];
    hipError_t ee = hipSuccess;  // first failing event call
    auto chk = [&](hipError_t r) {
      if (ee == hipSuccess) ee = r;
    };
    for (int s = 0; s < ns; ++s) b[s] = slab_args(g, a, slab, s, work, &ws[s]);
    {
      TraceRange r("ups:yfwd+zconv (slab pipeline)");
      for (int s = 0; s < ns; ++s) {
        chk(enqueue_colpass(g, var[1], b[s], ws[s], st));
        chk(hipEventRecord(side->ev[2 * s], st));
        chk(hipStreamWaitEvent(side->s, side->ev[2 * s], 0));
        chk(enqueue_colpass(g, var[2], b[s], ws[s], side->s));
        chk(hipEventRecord(side->ev[2 * s + 1], side->s));
      }
    }
    {
      TraceRange r(kRange[3]);
      for (int s = 0; s < ns; ++s) {
        chk(hipStreamWaitEvent(st, side->ev[2 * s + 1], 0));
        chk(enqueue_colpass(g, var[3], b[s], ws[s], st));
      }
    }
    {
      TraceRange r(kRange[4]);
      var[4]->launch(a, work, u, st);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = ee;
    if (e != hipSuccess) return fail(UPS_ERR_DEVICE, "solve enqueue failed: %s", hipGetErrorString(e));
    return UPS_OK;
  }
  if (side && side->s && ns == 1) {
    // one slab with a second stream: the few columns past the aligned launch
    // width go through all three column passes on the side stream, beside the
    // main launches, with one fork after the x pass and one join before the
    // last one
    const int align = colpass_align(g);
    const int kmain = a.kx / align * align;
    const int rest = a.kx - kmain;
    const PassVariant* nv[3] = {tail_variant(*var[1], rest), tail_variant(*var[2], rest),
                                tail_variant(*var[3], rest)};
    if (kmain > 0 && rest > 0 && nv[0] && nv[1] && nv[2]) {
      void* wm = nullptr;
      void* wr = nullptr;
      const PassArgs am = column_range(g, a, 0, kmain, work, &wm);
      const PassArgs ar = column_range(g, a, kmain, a.kx - kmain, work, &wr);
      // FP32 forks after the main y-forward launch, so that the narrow
      // launches run beside the z pass (bound by arithmetic) rather than the
      // y pass (bound by memory); FP64 forks after the x pass
      const int late = g.f64 ? 0 : 1;
      if (late) {
        TraceRange r(kRange[1]);
        var[1]->launch(am, wm, wm, st);
      }
      hipError_t ee = hipEventRecord(side->fork, st);
      if (ee == hipSuccess) ee = hipStreamWaitEvent(side->s, side->fork, 0);
      {
        TraceRange r("ups:last columns (second stream)");
        for (int p = 0; p < 3 && ee == hipSuccess; ++p) nv[p]->launch(ar, wr, wr, side->s);
      }
      if (ee == hipSuccess) ee = hipEventRecord(side->join, side->s);
      for (int p = 1 + late; p <= 3 && ee == hipSuccess; ++p) {
        TraceRange r(kRange[p]);
        var[p]->launch(am, wm, wm, st);
      }
      if (ee == hipSuccess) ee = hipStreamWaitEvent(st, side->join, 0);
      if (ee == hipSuccess) {
        TraceRange r(kRange[4]);
        var[4]->launch(a, work, u, st);
      }
      hipError_t e = hipGetLastError();
      if (e == hipSuccess) e = ee;
      if (e != hipSuccess) return fail(UPS_ERR_DEVICE, "solve enqueue failed: %s", hipGetErrorString(e));
      return UPS_OK;
    }
  }
  hipError_t e = hipGetLastError();
  for (int s = 0; s < ns && e == hipSuccess; ++s) {
    void* ws = nullptr;
    const PassArgs b = slab_args(g, a, slab, s, work, &ws);
    for (int p = 1; p <= 3 && e == hipSuccess; ++p) {
      TraceRange r(kRange[p]);
      e = enqueue_colpass(g, var[p], b, ws, st, side);
    }
  }
  if (e == hipSuccess) {
    TraceRange r(kRange[4]);
    var[4]->launch(a, work, u, st);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail(UPS_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return UPS_OK;
}

}  // namespace ups

ups_plan_s::~ups_plan_s() {
  if (!side.s) return;
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  if (have && cur != device) hipSetDevice(device);
  hipEventDestroy(side.fork);
  hipEventDestroy(side.join);
  for (hipEvent_t ev : side.ev)
    if (ev) hipEventDestroy(ev);
  hipStreamDestroy(side.s);
  if (have && cur != device) hipSetDevice(cur);
}

// ============================================================================
extern "C" {

int ups_abi_version(void) { return UPS_ABI_VERSION; }

const char* ups_last_error(void) { return g_err.c_str(); }

int ups_supported_length(int len, int prec) {
  if (len < 2 || len % 2) return 0;
  return length_supported(len, prec == UPS_F64) ? 1 : 0;
}

void ups_problem_init(ups_problem* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->green = UPS_GREEN_LGF2;
  p->prec = UPS_F64;
  p->center = UPS_CELL;
  p->ncomp = 1;
}

ups_status ups_plan_create(const ups_problem* prob, ups_plan_t* out) {
  if (!out) return fail(UPS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  PlanGeom g{};
  ups_status s = validate_problem(prob, &g);
  if (s != UPS_OK) return s;
  const char* gv = std::getenv("UPS_DEBUG_GUARDS");
  const bool guards = gv && *gv && std::strcmp(gv, "0") != 0;
  choose_nyq(g);
  plan_layout(g, guards);
  const int len[5] = {g.mx, g.my, g.mz, g.my, g.mx};
  const PassKind kinds[5] = {PASS_XFWD, PASS_YFWD, PASS_ZCONV, PASS_YINV, PASS_XINV};
  ups_plan_s* p = new ups_plan_s();
  p->prob = *prob;
  p->g = g;
  p->slab = default_slab(g);
  p->use_side = default_side(g);
  p->guards = guards;
  for (int i = 0; i < 5; ++i) {
    p->var[i] = tuned_variant(kinds[i], g.f64, len[i], g);
    if (!p->var[i]) {
      delete p;
      return fail(UPS_ERR_UNSUPPORTED, "no kernel for pass %d at length %d", i, len[i]);
    }
  }
  logf(2,
       "plan %p: %d x %d x %d (x, y, z) %s, %d component(s), padded %d x %d x %d; kernels %s %s %s %s %s; "
       "slab %d, second stream %d, Nyquist column packed %d, guards %d; G_hat buffer %zu B, work %zu B",
       static_cast<void*>(p), g.nx, g.ny, g.nz, g.f64 ? "FP64" : "FP32", g.ncomp, g.mx, g.my, g.mz,
       p->var[0]->name, p->var[1]->name, p->var[2]->name, p->var[3]->name, p->var[4]->name, p->slab,
       int(p->use_side), int(g.nyq), int(guards), g.green_bytes, g.work_bytes);
  *out = p;
  return ok();
}

ups_status ups_plan_sizes(ups_plan_t plan, size_t* green_bytes, size_t* work_bytes) {
  if (!plan) return fail(UPS_ERR_INVALID_ARG, "plan is NULL");
  if (green_bytes) *green_bytes = plan->g.green_bytes;
  if (work_bytes) *work_bytes = plan->g.work_bytes;
  return ok();
}

ups_status ups_plan_setup(ups_plan_t plan, void* green, size_t green_bytes, void* work, size_t work_bytes,
                          void* stream) {
  if (!plan) return fail(UPS_ERR_INVALID_ARG, "plan is NULL");
  if (!green || !work) return fail(UPS_ERR_INVALID_ARG, "green and work must be device pointers");
  if ((reinterpret_cast<uintptr_t>(green) | reinterpret_cast<uintptr_t>(work)) & 255)
    return fail(UPS_ERR_INVALID_ARG, "green and work must be 256-byte aligned");
  const PlanGeom& g = plan->g;
  if (green_bytes < g.green_bytes)
    return fail(UPS_ERR_WORKSPACE, "green buffer has %zu bytes, plan needs %zu", green_bytes, g.green_bytes);
  if (work_bytes < g.work_bytes)
    return fail(UPS_ERR_WORKSPACE, "work buffer has %zu bytes, plan needs %zu", work_bytes, g.work_bytes);
  int dev = 0;
  ups_status s = check_device(&dev);
  if (s != UPS_OK) return s;
  TraceRange range("ups_plan_setup");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* gb = static_cast<char*>(green);
  hipError_t e = build_twiddles(g.f64, g.mx, gb + g.off_twx, work, st);
  if (e == hipSuccess) e = build_twiddles(g.f64, g.my, gb + g.off_twy, work, st);
  if (e == hipSuccess) e = build_twiddles(g.f64, g.mz, gb + g.off_twz, work, st);
  if (e == hipSuccess)
    e = build_green(g.f64, g.bc, g.green, g.oz, g.oy, g.kx, g.gz, g.h, g.mx, g.my, g.mz, gb + g.off_ghat, work,
                    st);
  if (e == hipSuccess) e = enqueue_set_word(reinterpret_cast<unsigned*>(gb + g.off_status), 0u, st);
  if (e == hipSuccess && g.guard) {
    // canary bands below and above W (the Green's build used them as scratch)
    char* wb = static_cast<char*>(work);
    e = enqueue_fill_words(wb, g.guard, kCanaryWord, st);
    if (e == hipSuccess) e = enqueue_fill_words(wb + g.guard + g.solve_work, g.guard, kCanaryWord, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(UPS_ERR_DEVICE, "setup failed: %s", hipGetErrorString(e));
  if (!plan->side.s) {
    e = hipStreamCreateWithFlags(&plan->side.s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->side.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->side.join, hipEventDisableTiming);
    for (hipEvent_t& ev : plan->side.ev)
      if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return fail(UPS_ERR_DEVICE, "side stream: %s", hipGetErrorString(e));
  }
  plan->green = green;
  plan->work = work;
  plan->device = dev;
  plan->args = make_args(g, green);
  plan->ready = true;
  return ok();
}

static ups_status check_io(ups_plan_t plan, const void* in, const void* out) {
  if (!plan) return fail(UPS_ERR_INVALID_ARG, "plan is NULL");
  if (!plan->ready) return fail(UPS_ERR_STATE, "ups_plan_setup has not completed on this plan");
  if (!in || !out) return fail(UPS_ERR_INVALID_ARG, "input and output must be device pointers");
  const uintptr_t al = 2 * plan->g.elem - 1;
  if ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & al)
    return fail(UPS_ERR_INVALID_ARG, "arrays must be aligned to %zu bytes", size_t(al + 1));
  return UPS_OK;
}

// Read the plan's status word into *out, waiting for the stream.
static hipError_t read_status(ups_plan_t plan, hipStream_t st, unsigned* out) {
  const char* gb = static_cast<const char*>(plan->green);
  hipError_t e = hipMemcpyAsync(out, gb + plan->g.off_status, sizeof(unsigned), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

static unsigned* status_word(ups_plan_t plan) {
  return reinterpret_cast<unsigned*>(static_cast<char*>(plan->green) + plan->g.off_status);
}

// Any NaN or infinity among the ncomp nx ny nz values of x?  Waits.
static ups_status check_nonfinite(ups_plan_t plan, const void* x, hipStream_t st, bool* bad) {
  const PlanGeom& g = plan->g;
  const size_t n = (size_t)g.ncomp * g.nx * g.ny * g.nz;
  unsigned* w = status_word(plan);
  hipError_t e = enqueue_set_word(w, 0u, st);
  if (e == hipSuccess) e = enqueue_nonfinite(g.f64, x, n, w, st);
  unsigned v = 0;
  if (e == hipSuccess) e = read_status(plan, st, &v);
  if (e != hipSuccess) return fail(UPS_ERR_DEVICE, "non-finite check failed: %s", hipGetErrorString(e));
  *bad = (v & kStatNonfinite) != 0;
  return UPS_OK;
}

// Guard mode: the five passes one at a time on the caller's stream, with W
// filled with NaN words before the first pass, the rows y >= ny of every
// plane poisoned again before the last (pass 4 must read rows y < ny only),
// and both canary bands checked after every pass.  Waits after every pass.
static ups_status guarded_solve(ups_plan_t plan, const void* f, void* u, hipStream_t st) {
  const PlanGeom& g = plan->g;
  char* wb = static_cast<char*>(plan->work);
  void* W = plan->wbuf();
  unsigned* w = status_word(plan);
  static const char* kPass[5] = {"x-forward", "y-forward", "z-convolution", "y-inverse", "x-inverse"};
  hipError_t e = enqueue_set_word(w, 0u, st);
  if (e == hipSuccess) e = enqueue_fill_words(W, g.solve_work, kNanWord, st);
  for (int p = 0; p < 5 && e == hipSuccess; ++p) {
    if (p == 4) {
      const size_t cb = 2 * g.elem;
      e = enqueue_poison_rows(W, (long long)g.nz * g.ncomp, size_t(g.plane) * cb, size_t(g.ny) * g.px * cb,
                              size_t(g.my - g.ny) * g.px * cb, kNanWord, st);
      if (e != hipSuccess) break;
    }
    if (p == 0) plan->var[0]->launch(plan->args, f, W, st);
    else if (p == 4) plan->var[4]->launch(plan->args, W, u, st);
    else e = enqueue_colpass(g, plan->var[p], plan->args, W, st, nullptr);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = enqueue_check_words(wb, g.guard, kCanaryWord, w, kStatGuardLow, st);
    if (e == hipSuccess)
      e = enqueue_check_words(wb + g.guard + g.solve_work, g.guard, kCanaryWord, w, kStatGuardHigh, st);
    unsigned v = 0;
    if (e == hipSuccess) e = read_status(plan, st, &v);
    if (e != hipSuccess) break;
    if (v & (kStatGuardLow | kStatGuardHigh))
      return fail(UPS_ERR_INTERNAL, "guard mode: the canary band %s the work buffer was overwritten by the %s pass",
                  (v & kStatGuardLow) ? "below" : "above", kPass[p]);
  }
  if (e != hipSuccess) return fail(UPS_ERR_DEVICE, "guarded solve: %s", hipGetErrorString(e));
  return UPS_OK;
}

ups_status ups_solve(ups_plan_t plan, const void* f, void* u, void* stream) {
  ups_status s = check_io(plan, f, u);
  if (s != UPS_OK) return s;
  TraceRange range("ups_solve");
  logf(3, "solve plan %p f %p u %p stream %p", static_cast<void*>(plan), f, static_cast<void*>(u), stream);
  hipStream_t st = static_cast<hipStream_t>(stream);
  bool bad = false;
  if (plan->check_finite || plan->guards) {
    s = check_nonfinite(plan, f, st, &bad);
    if (s != UPS_OK) return s;
    if (bad && plan->check_finite)
      return fail(UPS_ERR_NONFINITE, "the input holds NaN or infinite values; nothing was solved");
  }
  if (plan->guards) {
    s = guarded_solve(plan, f, u, st);
    if (s != UPS_OK) return s;
    // NaN poison in the output of a finite input: a pass read work-buffer
    // data that no earlier pass wrote
    bool ubad = false;
    if (!bad) s = check_nonfinite(plan, u, st, &ubad);
    if (s != UPS_OK) return s;
    if (ubad) return fail(UPS_ERR_INTERNAL, "guard mode: NaN poison reached the output of a finite input");
    return ok();
  }
  s = enqueue_solve(plan->g, plan->var, plan->args, plan->slab, f, u, plan->wbuf(), st,
                    plan->use_side ? &plan->side : nullptr);
  return s == UPS_OK ? ok() : s;
}

// ---- allocation-free solve ---------------------------------------------------
// W of ups_solve_noalloc: one array per device in the library's own device
// memory, held from when the code object loads on a device until the process
// ends.  Its name is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
static __device__ __align__(256) unsigned char scratch[UPS_NOALLOC_MAX_WORK];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `dev`, which must be the current device.
hipError_t scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

ups_status ups_solve_noalloc(ups_plan_t plan, const void* f, void* u, void* stream) {
  ups_status s = check_io(plan, f, u);
  if (s != UPS_OK) return s;
  const PlanGeom& g = plan->g;
  if (plan->guards)
    return fail(UPS_ERR_UNSUPPORTED, "guard mode needs the canary bands of the plan's work buffer; use ups_solve");
  if (g.solve_work > size_t(UPS_NOALLOC_MAX_WORK))
    return fail(UPS_ERR_UNSUPPORTED, "the plan's W takes %zu bytes; ups_solve_noalloc holds at most %zu",
                g.solve_work, size_t(UPS_NOALLOC_MAX_WORK));
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(UPS_ERR_DEVICE, "hipGetDevice failed");
  if (cur != plan->device)
    return fail(UPS_ERR_INVALID_ARG, "the plan was set up on device %d; device %d is current", plan->device, cur);
  if (cur < 0 || cur >= kMaxDevices) return fail(UPS_ERR_DEVICE, "device %d out of range", cur);
  void* W = nullptr;
  hipError_t e = scratch_address(cur, &W);
  if (e != hipSuccess) return fail(UPS_ERR_DEVICE, "hipGetSymbolAddress: %s", hipGetErrorString(e));
  TraceRange range("ups_solve_noalloc");
  logf(3, "solve (no allocation) plan %p f %p u %p stream %p", static_cast<void*>(plan), f, static_cast<void*>(u),
       stream);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (plan->check_finite) {
    bool bad = false;
    s = check_nonfinite(plan, f, st, &bad);
    if (s != UPS_OK) return s;
    if (bad) return fail(UPS_ERR_NONFINITE, "the input holds NaN or infinite values; nothing was solved");
  }
  s = enqueue_solve(g, plan->var, plan->args, plan->slab, f, u, W, st, plan->use_side ? &plan->side : nullptr);
  return s == UPS_OK ? ok() : s;
}

ups_status ups_plan_set_check_finite(ups_plan_t plan, int enable) {
  if (!plan) return fail(UPS_ERR_INVALID_ARG, "plan is NULL");
  plan->check_finite = enable != 0;
  return ok();
}

int ups_plan_guard_mode(ups_plan_t plan) { return plan ? (plan->guards ? 1 : 0) : -1; }

ups_status ups_solve_adjoint(ups_plan_t plan, const void* grad_u, void* grad_f, void* stream) {
  // K^T = K: G1[i - j] = G1[j - i] for the symmetric 7-point stencil.
  return ups_solve(plan, grad_u, grad_f, stream);
}

ups_status ups_run_pass(ups_plan_t plan, int pass, const void* in, void* out, void* stream) {
  if (pass < 0 || pass > 4) return fail(UPS_ERR_INVALID_ARG, "pass %d not in 0..4", pass);
  if (plan && !plan->ready) return fail(UPS_ERR_STATE, "ups_plan_setup has not completed on this plan");
  const void* i = pass == 0 ? in : plan ? plan->wbuf() : nullptr;
  void* o = pass == 4 ? out : plan ? plan->wbuf() : nullptr;
  ups_status s = check_io(plan, i, o);
  if (s != UPS_OK) return s;
  hipError_t e = hipSuccess;
  if (pass >= 1 && pass <= 3) {
    e = enqueue_colpass(plan->g, plan->var[pass], plan->args, o, static_cast<hipStream_t>(stream),
                        plan->use_side ? &plan->side : nullptr);
  } else {
    plan->var[pass]->launch(plan->args, i, o, static_cast<hipStream_t>(stream));
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail(UPS_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return ok();
}

ups_status ups_plan_layout(ups_plan_t plan, int* pitch, long long* plane, long long* comp_stride,
                           size_t* ghat_offset, long long* ghat_plane) {
  if (!plan) return fail(UPS_ERR_INVALID_ARG, "plan is NULL");
  if (pitch) *pitch = plan->g.px;
  if (plane) *plane = plan->g.plane;
  if (comp_stride) *comp_stride = plan->g.comp_w;
  if (ghat_offset) *ghat_offset = plan->g.off_ghat;
  if (ghat_plane) *ghat_plane = (long long)plan->g.kx * plan->g.gz;
  return ok();
}

const char* ups_plan_kernel(ups_plan_t plan, int pass) {
  if (!plan || pass < 0 || pass > 4) return nullptr;
  return plan->var[pass]->name;
}

ups_status ups_plan_set_kernel(ups_plan_t plan, int pass, const char* name) {
  if (!plan || pass < 0 || pass > 4 || !name) return fail(UPS_ERR_INVALID_ARG, "bad plan, pass or name");
  const PassKind kinds[5] = {PASS_XFWD, PASS_YFWD, PASS_ZCONV, PASS_YINV, PASS_XINV};
  const int len[5] = {plan->g.mx, plan->g.my, plan->g.mz, plan->g.my, plan->g.mx};
  const PassVariant* v = find_variant(kinds[pass], plan->g.f64, len[pass], name, pass_fill(kinds[pass], plan->g));
  if (!v) return fail(UPS_ERR_INVALID_ARG, "no variant '%s' for pass %d at length %d", name, pass, len[pass]);
  if (!variant_allowed(*v, plan->g))
    return fail(UPS_ERR_UNSUPPORTED, "'%s' cannot run pass %d of a plan whose column 0 carries the Nyquist column",
                name, pass);
  plan->var[pass] = v;
  return ok();
}

static int list_variants(int pass, int prec, int len, int fill, const char** names, int cap) {
  if (pass < 0 || pass > 4 || (prec != UPS_F64 && prec != UPS_F32) || cap < 0 || (cap > 0 && !names)) return 0;
  const PassKind kinds[5] = {PASS_XFWD, PASS_YFWD, PASS_ZCONV, PASS_YINV, PASS_XINV};
  int n = 0;
  for (const PassVariant& v : pass_variants()) {
    if (v.kind != kinds[pass] || v.is_f64 != (prec == UPS_F64 ? 1 : 0) || v.length != len || v.fill != fill) continue;
    if (n < cap) names[n] = v.name;
    ++n;
  }
  return n;
}

int ups_kernel_variants(int pass, int prec, int len, const char** names, int cap) {
  return list_variants(pass, prec, len, 0, names, cap);
}

int ups_kernel_fill_variants(int pass, int prec, int len, const char** names, int cap) {
  return list_variants(pass, prec, len, 1, names, cap);
}

ups_status ups_plan_set_slab(ups_plan_t plan, int columns) {
  if (!plan) return fail(UPS_ERR_INVALID_ARG, "plan is NULL");
  if (columns < 0 || (columns > 0 && columns % 16 != 0))
    return fail(UPS_ERR_INVALID_ARG, "slab width %d is not 0 or a positive multiple of 16", columns);
  if (plan->g.nyq && columns > 0 && columns < plan->g.kx)
    return fail(UPS_ERR_UNSUPPORTED, "a plan whose column 0 carries the Nyquist column runs one slab");
  plan->slab = columns >= plan->g.kx ? 0 : columns;
  return ok();
}

int ups_plan_slab(ups_plan_t plan) { return plan ? plan->slab : -1; }

int ups_plan_nyquist_packed(ups_plan_t plan) { return plan ? (plan->g.nyq ? 1 : 0) : -1; }

ups_status ups_plan_set_side_stream(ups_plan_t plan, int enable) {
  if (!plan) return fail(UPS_ERR_INVALID_ARG, "plan is NULL");
  plan->use_side = enable != 0;
  return ok();
}

int ups_plan_side_stream(ups_plan_t plan) { return plan ? (plan->use_side ? 1 : 0) : -1; }

size_t ups_plan_work_offset(ups_plan_t plan) { return plan ? plan->g.guard : 0; }

double ups_plan_model_bytes(ups_plan_t plan, int pass) {
  if (!plan || pass < -1 || pass > 4) return 0.0;
  return model_bytes(plan->g, pass);
}

ups_status ups_plan_destroy(ups_plan_t plan) {
  delete plan;
  return ok();
}

}  // extern "C"
