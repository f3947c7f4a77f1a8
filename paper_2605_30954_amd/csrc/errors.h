// Thread-local error message of the C ABI (gpgomea_last_error).
#pragma once
#include <cstdarg>
#include <cstdio>
#include <string>

namespace gg {

std::string& last_error();

// Record a formatted message and return `code` (for `return fail(...)`).
inline int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  last_error() = buf;
  return code;
}

}  // namespace gg
