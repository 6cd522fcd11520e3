// Checking kernels of the optional debug modes (include/ups.h):
//   - the non-finite input check of ups_solve (ups_plan_set_check_finite);
//   - the guard mode (UPS_DEBUG_GUARDS=1): canary bands on both sides of the
//     work buffer, checked after every pass, and NaN poison in the parts of
//     the work buffer that the next pass must not read.
// Status words live in the plan's green buffer; they are cleared by a kernel
// (not a memset node) so that the sequence stays valid inside a captured
// graph.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "debug.hpp"

namespace ups {

__global__ void k_set_word(unsigned* w, unsigned v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *w = v;
}

// flag |= 1 if any of the n values of x is NaN or infinite
template <typename T>
__global__ void k_nonfinite(const T* __restrict__ x, size_t n, unsigned* flag) {
  bool bad = false;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1u);
}

// n 32-bit words of w = v
__global__ void k_fill_words(unsigned* __restrict__ w, size_t n, unsigned v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    w[i] = v;
}

// flag |= bit if any of the n words of g differs from v
__global__ void k_check_words(const unsigned* __restrict__ g, size_t n, unsigned v, unsigned* flag, unsigned bit) {
  bool bad = false;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    bad |= g[i] != v;
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, bit);
}

// Rows y in [y0, my) of every (component, z) plane of W set to the NaN word
// pattern: `rows` complex rows of `pitch` elements of `cb` bytes per plane.
__global__ void k_poison_rows(unsigned* __restrict__ W, long long planes, long long plane_words, long long off_words,
                              long long span_words, unsigned v) {
  const long long tot = planes * span_words;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
       i += (long long)gridDim.x * blockDim.x) {
    const long long p = i / span_words, r = i % span_words;
    W[p * plane_words + off_words + r] = v;
  }
}

static unsigned grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  return unsigned(b < 1 ? 1 : b);
}

hipError_t enqueue_set_word(unsigned* w, unsigned v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_word, dim3(1), dim3(64), 0, st, w, v);
  return hipGetLastError();
}

hipError_t enqueue_nonfinite(bool f64, const void* x, size_t n, unsigned* flag, hipStream_t st) {
  if (f64)
    hipLaunchKernelGGL(k_nonfinite<double>, dim3(grid_for(n)), dim3(256), 0, st, static_cast<const double*>(x), n,
                       flag);
  else
    hipLaunchKernelGGL(k_nonfinite<float>, dim3(grid_for(n)), dim3(256), 0, st, static_cast<const float*>(x), n,
                       flag);
  return hipGetLastError();
}

hipError_t enqueue_fill_words(void* w, size_t nbytes, unsigned v, hipStream_t st) {
  const size_t n = nbytes / 4;
  hipLaunchKernelGGL(k_fill_words, dim3(grid_for(n)), dim3(256), 0, st, static_cast<unsigned*>(w), n, v);
  return hipGetLastError();
}

hipError_t enqueue_check_words(const void* g, size_t nbytes, unsigned v, unsigned* flag, unsigned bit,
                               hipStream_t st) {
  const size_t n = nbytes / 4;
  hipLaunchKernelGGL(k_check_words, dim3(grid_for(n)), dim3(256), 0, st, static_cast<const unsigned*>(g), n, v, flag,
                     bit);
  return hipGetLastError();
}

hipError_t enqueue_poison_rows(void* W, long long planes, size_t plane_bytes, size_t off_bytes, size_t span_bytes,
                               unsigned v, hipStream_t st) {
  const long long span = (long long)(span_bytes / 4);
  hipLaunchKernelGGL(k_poison_rows, dim3(grid_for(size_t(planes * span))), dim3(256), 0, st,
                     static_cast<unsigned*>(W), planes, (long long)(plane_bytes / 4), (long long)(off_bytes / 4), span,
                     v);
  return hipGetLastError();
}

}  // namespace ups
