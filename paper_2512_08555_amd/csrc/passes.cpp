// Registry of the compiled pass kernels (instantiated in passes_f32.hip,
// passes_f32m.hip and passes_f64.hip).
#include "passes.hpp"

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

int blocks_for(const PassVariant& v, const PassArgs& a, int* gx, int* gy, int* gz) {
  switch (v.kind) {
    case PASS_XFWD:
    case PASS_XINV:
      *gx = cdiv_ll((long long)a.ny * a.nz, v.tile); *gy = a.ncomp; *gz = 1; break;
    case PASS_YFWD:
    case PASS_YINV:
      *gx = cdiv_ll(a.kx, v.tile); *gy = a.nz; *gz = a.ncomp; break;
    default: {
      const long long groups = (long long)cdiv_ll(a.kx, v.tile) * (a.my / 2 + 1);
      *gx = int(cdiv_ll(groups, 8) * 8LL * 2 * a.ncomp); *gy = 1; *gz = 1; break;
    }
  }
  return (*gx) * (*gy) * (*gz);
}

}  // namespace ups
