// Kernel instantiations: float, 2^a 3^b 5^c padded lengths for uneven grids
// (80, 96, 144, 160, 192, 288, 320, 384).
#include "passes_impl.hpp"

namespace ups {

std::vector<PassVariant> variants_f32_mixed() {
  return {
      X_VARIANTS(float, 4, 10, 16, 1),      // mx = 80
      X_VARIANTS(float, 4, 12, 16, 1),      // mx = 96
      X_VARIANTS(float, 6, 12, 16, 2),      // mx = 144
      X_VARIANTS(float, 4, 20, 16, 2),      // mx = 160
      X_VARIANTS(float, 8, 12, 16, 2),      // mx = 192
      X_VARIANTS(float, 12, 12, 16, 2),     // mx = 288
      X_VARIANTS(float, 8, 20, 16, 2),      // mx = 320
      X_VARIANTS(float, 8, 24, 16, 2),      // mx = 384
      COL_VARIANTS(float, 4, 20, 16, 1),    // 80
      COL_VARIANTS(float, 8, 12, 16, 1),    // 96
      COL_VARIANTS(float, 12, 12, 16, 1),   // 144
      COL_VARIANTS(float, 8, 20, 16, 2),    // 160
      COL_VARIANTS(float, 8, 24, 16, 2),    // 192
      COL_VARIANTS(float, 12, 24, 16, 2),   // 288
      COL_VARIANTS(float, 8, 40, 16, 2),    // 320
      COL_VARIANTS(float, 16, 24, 16, 2),   // 384
  };
}

}  // namespace ups
