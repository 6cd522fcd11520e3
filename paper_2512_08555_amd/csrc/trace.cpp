// UPS_LOG_LEVEL logging (see trace.hpp).
#include "trace.hpp"

#include <cstdarg>
#include <cstdio>
#include <cstdlib>

namespace ups {

int log_level() {
  static const int level = [] {
    const char* v = std::getenv("UPS_LOG_LEVEL");
    if (!v || !*v) return 0;
    const int n = std::atoi(v);
    return n < 0 ? 0 : (n > 3 ? 3 : n);
  }();
  return level;
}

void logf(int level, const char* fmt, ...) {
  if (level > log_level()) return;
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[ups] %s\n", buf);
}

}  // namespace ups
