// Kernel instantiations: double, power-of-two padded lengths 32 .. 1024.
// The first variant listed for a (pass, length) is the default (ordered by
// measured time on MI355X for the 256^3 and 512^3 grids).
#include "xwave.hpp"
#include "ywave.hpp"

namespace ups {

std::vector<PassVariant> variants_f64() {
  return {
      X_VARIANTS(double, 4, 4, 8, 1),
      X_VARIANTS(double, 4, 8, 8, 1),
      X_VARIANTS(double, 8, 8, 8, 2),
      X_VARIANTS(double, 8, 16, 8, 2),
      X_VARIANTS(double, 16, 16, 8, 2),
      XFW(double, 8, 8), XFW(double, 8, 4), XIWM(double, 8, 8), XIW(double, 8, 8),   // mx = 1024
      XF(double, 16, 32, 8, 2), XF(double, 16, 32, 8, 4),
      XI(double, 16, 32, 8, 2), XI(double, 16, 32, 8, 4),
      COL_VARIANTS(double, 4, 8, 8, 1),
      COL_VARIANTS(double, 8, 8, 8, 1),
      COL_VARIANTS(double, 8, 16, 8, 2),
      COL_VARIANTS(double, 16, 16, 8, 2),
      YF(double, 16, 32, 8, 2), YF(double, 16, 32, 8, 4),   // 512
      ZWG(double, 8, 4), ZW(double, 8, 8), ZWG(double, 8, 8), ZW(double, 8, 4), ZW(double, 8, 1),
      ZC(double, 16, 32, 8, 2), ZC(double, 16, 32, 8, 4),
      YIW(double, 8, 8), YIW(double, 8, 4), YIW(double, 8, 1), YIWP(double, 8, 8),
      YFW(double, 8, 8), YFW(double, 8, 4), YFW(double, 8, 1),
      YI(double, 16, 32, 8, 4), YI(double, 16, 32, 8, 2),
      YF(double, 16, 32, 2, 1), YI(double, 16, 32, 2, 1),
      YFW(double, 16, 8), YF(double, 32, 32, 8, 4), YF(double, 32, 32, 8, 2),   // 1024
      ZW(double, 16, 8), ZWG(double, 16, 8), ZW(double, 16, 4), ZWG(double, 16, 4), ZW(double, 16, 1),
      ZW(double, 16, 16), ZWT(double, 16, 4),
      ZC(double, 32, 32, 8, 2), ZC(double, 32, 32, 8, 4),
      YIWP(double, 16, 8), YIW(double, 16, 8), YIW(double, 16, 4), YIW(double, 16, 1),
      YFW(double, 16, 4), YFW(double, 16, 1),
      YI(double, 32, 32, 8, 2), YI(double, 32, 32, 8, 4),
      YF(double, 32, 32, 2, 1), YI(double, 32, 32, 2, 1),
      // even and odd directions: the wave-per-line forward passes (y and z at
      // 512 and 1024, x at 1024), ahead of the four-step ones below, so the defaults
      ZWE(double, 8, 4, false), ZWE(double, 8, 1, false), YFWE(double, 8, 8), YFWE(double, 8, 1),
      ZWE(double, 16, 8, false), ZWE(double, 16, 1, false), YFWE(double, 16, 8), YFWE(double, 16, 1),
      XFWE(double, 8, 8),   // mx = 1024
      // even and odd directions, mx/my/mz = 32 .. 1024
      FILL_VARIANTS(double, 4, 4, 8, 1, 4, 8, 8, 1, 4, 8, 8, 1),
      FILL_VARIANTS(double, 4, 8, 8, 1, 8, 8, 8, 1, 8, 8, 8, 1),
      FILL_VARIANTS(double, 8, 8, 8, 2, 8, 16, 8, 2, 8, 16, 8, 2),
      FILL_VARIANTS(double, 8, 16, 8, 2, 16, 16, 8, 2, 16, 16, 8, 2),
      FILL_VARIANTS(double, 16, 16, 8, 2, 16, 32, 8, 2, 16, 32, 8, 2),
      FILL_VARIANTS(double, 16, 32, 8, 2, 32, 32, 8, 2, 32, 32, 8, 2),
  };
}

}  // namespace ups
