// Shared helpers of the tnfem library: status codes, per-thread error text.
#pragma once

#include <cstdarg>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "../../include/tnfem.h"

namespace tnfem {

// Exception carrying a TNFEM_E* status; converted to a return code at the C ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw Error(code, buf);
}

#define TNFEM_REQUIRE(cond, ...)                        \
  do {                                                  \
    if (!(cond)) ::tnfem::fail(TNFEM_EINVAL, __VA_ARGS__); \
  } while (0)

void set_last_error(const char* msg);

}  // namespace tnfem
