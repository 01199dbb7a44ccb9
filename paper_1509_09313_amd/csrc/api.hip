// Error reporting and version of libnmf.
#include <stdio.h>

#include "nmf_common.h"

namespace {
thread_local char g_err[512] = "";
}

namespace nmf {

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

}  // namespace nmf

extern "C" const char* nmf_last_error(void) { return g_err; }

extern "C" const char* nmf_version(void) { return "libnmf 0.1 (gfx950)"; }
