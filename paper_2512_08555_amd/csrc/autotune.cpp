// Autotuner: per (pass, precision, padded length, size class), time every
// compiled kernel variant on the plan's own buffers with HIP events and keep
// the fastest.  The size class is floor(log2) of the number of lines the
// pass transforms, so a tune on a thin grid does not decide for a large one
// of the same padded length.  Choices live in a process-wide cache that new
// plans and batches consult; with UPS_TUNE_CACHE=<path> the cache is read
// from and written to that JSON file
// ({"zconv/f32/1024/l19": "zconv_float_w16_c16_t", ...}).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ups.h"
#include "passes.hpp"
#include "plan.hpp"
#include "trace.hpp"

using namespace ups;

namespace {

const char* kKindName[5] = {"xfwd", "yfwd", "zconv", "yinv", "xinv"};
const PassKind kKinds[5] = {PASS_XFWD, PASS_YFWD, PASS_ZCONV, PASS_YINV, PASS_XINV};

std::mutex g_mu;
std::map<std::string, std::string> g_cache;
bool g_loaded = false;

}  // namespace

namespace ups {

// Lines one launch of pass `kind` transforms on geometry g: rows for the x
// passes, (kx, z) columns for the y passes, (kx, ky) columns for the z pass.
long long pass_lines(PassKind kind, const PlanGeom& g) {
  switch (kind) {
    case PASS_XFWD:
    case PASS_XINV: return (long long)g.ny * g.nz * g.ncomp;
    case PASS_YFWD:
    case PASS_YINV: return (long long)g.kx * g.nz * g.ncomp;
    default: return (long long)g.kx * g.my * g.ncomp;
  }
}

std::string tune_key(PassKind kind, const PlanGeom& g) {
  const int length = kind == PASS_XFWD || kind == PASS_XINV ? g.mx : kind == PASS_ZCONV ? g.mz : g.my;
  long long lines = pass_lines(kind, g);
  int lg = 0;
  while (lines > 1) {
    lines >>= 1;
    ++lg;
  }
  char buf[64];
  snprintf(buf, sizeof buf, "%s/%s/%d/l%d%s", kKindName[int(kind)], g.f64 ? "f64" : "f32", length, lg,
           pass_fill(kind, g) ? "/e" : "");
  return buf;
}

}  // namespace ups

namespace {

// minimal reader for a flat {"key": "value", ...} object
void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("UPS_TUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream in(path);
  if (!in) return;
  std::stringstream ss;
  ss << in.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  auto next_str = [&](std::string& out) -> bool {
    size_t a = s.find('"', i);
    if (a == std::string::npos) return false;
    size_t b = s.find('"', a + 1);
    if (b == std::string::npos) return false;
    out = s.substr(a + 1, b - a - 1);
    i = b + 1;
    return true;
  };
  std::string k, v;
  while (next_str(k) && next_str(v)) g_cache[k] = v;
}

void save_locked() {
  const char* path = std::getenv("UPS_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream out(path);
  if (!out) return;
  out << "{\n";
  size_t n = 0;
  for (const auto& kv : g_cache) {
    out << "  \"" << kv.first << "\": \"" << kv.second << "\"" << (++n < g_cache.size() ? ",\n" : "\n");
  }
  out << "}\n";
}

}  // namespace

namespace ups {

// The variant a new plan uses: the cached tuning result if any, else the
// table default.
const PassVariant* tuned_variant(PassKind kind, bool f64, int length, const PlanGeom& g) {
  std::string name;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    auto it = g_cache.find(tune_key(kind, g));
    if (it != g_cache.end()) name = it->second;
  }
  const int fill = pass_fill(kind, g);
  if (!name.empty()) {
    const PassVariant* v = find_variant(kind, f64, length, name.c_str(), fill);
    if (v && variant_allowed(*v, g)) return v;
  }
  const PassVariant* v = find_variant(kind, f64, length, nullptr, fill);
  if (v && variant_allowed(*v, g)) return v;
  for (const PassVariant& w : pass_variants())   // the first allowed one
    if (w.kind == kind && w.is_f64 == (f64 ? 1 : 0) && w.length == length && w.fill == fill && variant_allowed(w, g))
      return &w;
  return nullptr;
}

}  // namespace ups

extern "C" {

ups_status ups_autotune(ups_plan_t plan, const void* f, void* u, void* stream, double budget_ms) {
  if (!plan) return set_error(UPS_ERR_INVALID_ARG, "plan is NULL");
  if (!plan->ready) return set_error(UPS_ERR_STATE, "ups_plan_setup has not completed on this plan");
  if (!f || !u) return set_error(UPS_ERR_INVALID_ARG, "f and u must be device arrays laid out as for ups_solve");
  const uintptr_t al = 2 * plan->g.elem - 1;
  if ((reinterpret_cast<uintptr_t>(f) | reinterpret_cast<uintptr_t>(u)) & al)
    return set_error(UPS_ERR_INVALID_ARG, "f and u are misaligned");
  TraceRange range("ups_autotune");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const PlanGeom& g = plan->g;
  const int len[5] = {g.mx, g.my, g.mz, g.my, g.mx};
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return set_error(UPS_ERR_DEVICE, "hipEventCreate failed");
  // Candidates are timed inside whole solves with the current choices for
  // the other passes and the plan's schedule, from the caller's f into the
  // caller's u: a pass's speed depends on how the pass before it left the
  // caches (measured: timing one pass in a loop picks different, slower
  // variants), so the x passes must see the traffic of a real solve.
  void* work = plan->wbuf();
  const SideStream* side = plan->use_side ? &plan->side : nullptr;
  double spent = 0.0;
  hipError_t err = hipSuccess;
  auto time_once = [&](float* ms_out) {
    const int reps = 5;
    ups_status s = enqueue_solve(g, plan->var, plan->args, plan->slab, f, u, work, st, side);  // warm-up
    if (s != UPS_OK) return hipErrorLaunchFailure;
    hipError_t e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r)
      if (enqueue_solve(g, plan->var, plan->args, plan->slab, f, u, work, st, side) != UPS_OK)
        e = hipErrorLaunchFailure;
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    *ms_out = ms / reps;
    spent += double(ms) * (reps + 1) / reps;
    return e;
  };
  // best of two measurements: run-to-run noise is about 1% of a solve
  auto time_solves = [&](float* ms_out) {
    float a = 0.f, b = 0.f;
    hipError_t e = time_once(&a);
    if (e == hipSuccess) e = time_once(&b);
    *ms_out = a < b ? a : b;
    return e;
  };
  for (int k = 0; k < 5 && err == hipSuccess; ++k) {
    std::vector<const PassVariant*> cands;
    for (const PassVariant& v : pass_variants())
      if (v.kind == kKinds[k] && v.is_f64 == (g.f64 ? 1 : 0) && v.length == len[k] &&
          v.fill == pass_fill(kKinds[k], g) && variant_allowed(v, g))
        cands.push_back(&v);
    // the current choice first; a candidate replaces it only if it is faster
    // by more than the noise (1%)
    const PassVariant* best = plan->var[k];
    float best_ms = 0.f;
    err = time_solves(&best_ms);
    for (const PassVariant* v : cands) {
      if (err != hipSuccess) break;
      if (v == best || spent > budget_ms) continue;
      plan->var[k] = v;
      float ms = 0.f;
      err = time_solves(&ms);
      logf(2, "autotune plan %p pass %d: %s %.4f ms per solve (current %s %.4f ms)", static_cast<void*>(plan), k,
           v->name, double(ms), best->name, double(best_ms));
      if (err == hipSuccess && ms < 0.99f * best_ms) {
        best_ms = ms;
        best = v;
      }
    }
    plan->var[k] = best;
    logf(2, "autotune plan %p pass %d: keeps %s", static_cast<void*>(plan), k, best->name);
    std::lock_guard<std::mutex> lk(g_mu);
    load_locked();
    g_cache[tune_key(kKinds[k], g)] = best->name;
  }
  // then the column schedule: one slab on one or two streams, or 128- or
  // 256-column slabs pipelined over two streams (plans with at least 256
  // columns)
  if (err == hipSuccess && g.kx >= 256 && !g.nyq) {
    const int cur_slab = plan->slab;
    const bool cur_side = plan->use_side;
    float best_ms = 0.f;
    err = time_solves(&best_ms);
    int best_slab = cur_slab;
    bool best_side = cur_side;
    const int slabs[4] = {0, 0, 128, 256};
    const bool sides[4] = {false, true, true, true};
    for (int i = 0; i < 4 && err == hipSuccess; ++i) {
      const int sl = slabs[i];
      const bool sd = sides[i];
      if ((sl == cur_slab && sd == cur_side) || spent > budget_ms || (sl > 0 && sl >= g.kx)) continue;
      plan->slab = sl;
      plan->use_side = sd;
      side = plan->use_side ? &plan->side : nullptr;
      float ms = 0.f;
      err = time_solves(&ms);
      if (err == hipSuccess && ms < 0.99f * best_ms) {
        best_ms = ms;
        best_slab = sl;
        best_side = sd;
      }
    }
    plan->slab = best_slab;
    plan->use_side = best_side;
    logf(2, "autotune plan %p: schedule slab %d, second stream %d (%.4f ms per solve)", static_cast<void*>(plan),
         best_slab, int(best_side), double(best_ms));
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (err != hipSuccess) return set_error(UPS_ERR_DEVICE, hipGetErrorString(err));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    save_locked();
  }
  return set_error(UPS_OK, "");
}

}  // extern "C"
