// Enqueue helpers of the debug modes (debug.hip): non-finite input check,
// canary bands and NaN poison of the work buffer.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace ups {

// Bytes of each canary band on either side of W in the guard mode.
constexpr size_t kGuardBytes = 64 * 1024;
// Word patterns: canary bands, and a quiet-NaN word (as FP32 it is a NaN;
// two of them make an FP64 NaN as well).
constexpr unsigned kCanaryWord = 0xC0DEC0DEu;
constexpr unsigned kNanWord = 0x7FC00001u;
// Status bits in the green buffer's status word.
constexpr unsigned kStatNonfinite = 1u;
constexpr unsigned kStatGuardLow = 2u;
constexpr unsigned kStatGuardHigh = 4u;

hipError_t enqueue_set_word(unsigned* w, unsigned v, hipStream_t st);
hipError_t enqueue_nonfinite(bool f64, const void* x, size_t n, unsigned* flag, hipStream_t st);
hipError_t enqueue_fill_words(void* w, size_t nbytes, unsigned v, hipStream_t st);
hipError_t enqueue_check_words(const void* g, size_t nbytes, unsigned v, unsigned* flag, unsigned bit,
                               hipStream_t st);
// In each of `planes` planes of plane_bytes, span_bytes starting at off_bytes.
hipError_t enqueue_poison_rows(void* W, long long planes, size_t plane_bytes, size_t off_bytes, size_t span_bytes,
                               unsigned v, hipStream_t st);

}  // namespace ups
