// Registry of the compiled pass kernels (instantiated in passes_f32.hip,
// passes_f32m.hip and passes_f64.hip).
#include "passes_impl.hpp"

namespace ups {

std::vector<PassVariant> variants_f32_pow2();
std::vector<PassVariant> variants_f32_mixed();
std::vector<PassVariant> variants_f64();

const std::vector<PassVariant>& pass_variants() {
  static const std::vector<PassVariant> table = [] {
    std::vector<PassVariant> t = variants_f32_pow2();
    for (auto* f : {&variants_f32_mixed, &variants_f64}) {
      std::vector<PassVariant> more = (*f)();
      t.insert(t.end(), more.begin(), more.end());
    }
    return t;
  }();
  return table;
}

static inline int cdiv_ll(long long a, long long b) { return int((a + b - 1) / b); }

const PassVariant* narrow_variant(const PassVariant& v) {
  if (v.kind == PASS_XFWD || v.kind == PASS_XINV) return nullptr;
  const PassVariant* best = nullptr;
  for (const PassVariant& w : pass_variants()) {
    if (w.kind != v.kind || w.is_f64 != v.is_f64 || w.length != v.length || w.fill != v.fill) continue;
    if ((w.nch == 0) != (v.nch == 0)) continue;  // same kernel family
    if (!best || w.tile < best->tile) best = &w;
  }
  return best && best->tile < v.tile ? best : nullptr;
}

// Blocks one launch of variant v needs for problem a (as the launchers in
// passes_impl.hpp compute them).
int blocks_for(const PassVariant& v, const PassArgs& a, int* gx, int* gy, int* gz) {
  const int per_line = 128 / (v.is_f64 ? 16 : 8);
  int H = per_line > v.tile ? per_line / v.tile : 1;
  const int ntiles = cdiv_ll(a.kx, v.tile);
  if (v.kind != PASS_XFWD && v.kind != PASS_XINV && H > ntiles) H = ntiles;  // as col_slots()
  *gy = 1;
  *gz = 1;
  switch (v.kind) {
    case PASS_XFWD:
    case PASS_XINV:
      *gx = cdiv_ll((long long)a.ny * a.nz, v.tile); *gy = a.ncomp; break;
    case PASS_YFWD:
    case PASS_YINV:
      *gx = int(ymap_blocks(ntiles, a.nz, a.ncomp, H)); break;
    default:
      *gx = int(zmap_blocks(ntiles, a.my, a.ncomp, H)); break;
  }
  return (*gx) * (*gy) * (*gz);
}

}  // namespace ups
