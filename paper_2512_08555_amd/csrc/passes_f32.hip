// Kernel instantiations: float, power-of-two padded lengths 32 .. 1024.
// The first variant listed for a (pass, length) is the default (ordered by
// measured time on MI355X for the 512^3 grid).
#include "xwave.hpp"
#include "ywave.hpp"

namespace ups {

std::vector<PassVariant> variants_f32_pow2() {
  return {
      X_VARIANTS(float, 4, 4, 16, 1),       // mx = 32
      X_VARIANTS(float, 4, 8, 16, 1),       // mx = 64
      X_VARIANTS(float, 8, 8, 16, 2),       // mx = 128
      X_VARIANTS(float, 8, 16, 16, 2),      // mx = 256
      X_VARIANTS(float, 16, 16, 16, 2),     // mx = 512
      XFW(float, 8, 4), XFW(float, 8, 8), XIWM(float, 8, 8), XIWM(float, 8, 4), XIW(float, 8, 8), XIW(float, 8, 4),   // mx = 1024
      XF(float, 16, 32, 4, 1), XF(float, 16, 32, 8, 2), XF(float, 16, 32, 8, 1),
      XF(float, 32, 16, 8, 2), XF(float, 16, 32, 16, 2), XF(float, 16, 32, 16, 4),
      XI(float, 16, 32, 16, 4), XI(float, 16, 32, 4, 1), XI(float, 16, 32, 8, 1),
      XI(float, 32, 16, 8, 2), XI(float, 16, 32, 8, 2), XI(float, 16, 32, 16, 2),
      COL_VARIANTS(float, 4, 8, 16, 1),     // 32
      COL_VARIANTS(float, 8, 8, 16, 1),     // 64
      COL_VARIANTS(float, 8, 16, 16, 2),    // 128
      COL_VARIANTS(float, 16, 16, 16, 2),   // 256
      ZWT(float, 8, 16), ZW(float, 8, 16), ZWG(float, 8, 8), ZW(float, 8, 8), ZW(float, 8, 4),   // 512
      ZW(float, 8, 1),
      COL_VARIANTS(float, 16, 32, 16, 2),
      YF(float, 16, 32, 2, 1), YI(float, 16, 32, 2, 1),
      YIW(float, 8, 16), YIW(float, 8, 8), YIW(float, 8, 1), YIWP(float, 8, 8),
      YFW(float, 8, 16), YFW(float, 8, 8), YFW(float, 8, 1),
      YFW(float, 16, 16), YF(float, 32, 32, 16, 2), YF(float, 32, 32, 16, 4), YF(float, 32, 32, 8, 2),   // 1024
      YF(float, 32, 32, 8, 1), YF(float, 32, 32, 4, 1), YF(float, 32, 32, 4, 2),
      ZWT(float, 16, 16), ZW(float, 16, 16), ZW(float, 16, 8), ZWO(float, 16, 8), ZWG(float, 16, 8), ZW(float, 16, 4), ZWG(float, 16, 4),
      ZW(float, 16, 1), ZWT(float, 16, 8),
      ZC(float, 32, 32, 8, 2), ZC(float, 32, 32, 16, 2), ZC(float, 32, 32, 16, 4),
      ZC(float, 32, 32, 8, 1), ZC(float, 32, 32, 4, 1), ZC(float, 32, 32, 4, 2),
      YIWP(float, 16, 16), YIW(float, 16, 16), YIW(float, 16, 8), YIW(float, 16, 1), YIWP(float, 16, 8),
      YIWT(float, 16, 16), YFW(float, 16, 8), YFW(float, 16, 1),
      YI(float, 32, 32, 8, 1), YI(float, 32, 32, 8, 2), YI(float, 32, 32, 16, 2),
      YI(float, 32, 32, 16, 4), YI(float, 32, 32, 4, 1), YI(float, 32, 32, 4, 2),
      YF(float, 32, 32, 2, 1), YI(float, 32, 32, 2, 1),
      // even and odd directions: the wave-per-line forward passes (y and z at
      // 512 and 1024, x at 1024), ahead of the four-step ones below, so the defaults
      ZWE(float, 8, 16, true), ZWE(float, 8, 1, false), YFWE(float, 8, 16), YFWE(float, 8, 1),
      ZWE(float, 16, 16, true), ZWE(float, 16, 1, false), YFWE(float, 16, 16), YFWE(float, 16, 1),
      XFWE(float, 8, 4),   // mx = 1024
      // even and odd directions, mx/my/mz = 32 .. 1024
      FILL_VARIANTS(float, 4, 4, 16, 1, 4, 8, 16, 1, 4, 8, 16, 1),
      FILL_VARIANTS(float, 4, 8, 16, 1, 8, 8, 16, 1, 8, 8, 16, 1),
      FILL_VARIANTS(float, 8, 8, 16, 2, 8, 16, 16, 2, 8, 16, 16, 2),
      FILL_VARIANTS(float, 8, 16, 16, 2, 16, 16, 16, 2, 16, 16, 16, 2),
      FILL_VARIANTS(float, 16, 16, 16, 2, 16, 32, 16, 2, 16, 32, 16, 2),
      FILL_VARIANTS(float, 16, 32, 4, 1, 32, 32, 16, 2, 32, 32, 8, 2),
  };
}

hipError_t launch_zpair(bool f64, const PassArgs& a, void* W, hipStream_t st) {
  if (f64) return hipErrorInvalidValue;   // single plans pair column 0 in FP32 only
  if (a.mz == 1024) launch_zpair_t<float, 16>(a, W, st);
  else if (a.mz == 512) launch_zpair_t<float, 8>(a, W, st);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace ups
