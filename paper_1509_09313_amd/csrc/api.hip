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

KernelMark& kernel_mark() {
  static thread_local KernelMark m;
  return m;
}

}  // namespace nmf

extern "C" int nmf_events_create(int n, void** events) {
  if (n < 0 || (n > 0 && !events)) return nmf::fail(NMF_EINVAL, "nmf_events_create: bad arguments");
  for (int i = 0; i < n; ++i) {
    hipEvent_t e;
    const hipError_t rc = hipEventCreate(&e);
    if (rc != hipSuccess) return nmf::fail(NMF_EHIP, "nmf_events_create: %s", hipGetErrorString(rc));
    events[i] = e;
  }
  return NMF_OK;
}

extern "C" int nmf_events_destroy(int n, void** events) {
  for (int i = 0; i < n; ++i)
    if (events[i]) hipEventDestroy(static_cast<hipEvent_t>(events[i]));
  return NMF_OK;
}

extern "C" int nmf_events_elapsed_ms(void* start, void* stop, float* ms) {
  if (!start || !stop || !ms) return nmf::fail(NMF_EINVAL, "nmf_events_elapsed_ms: null");
  const hipError_t rc = hipEventElapsedTime(ms, static_cast<hipEvent_t>(start), static_cast<hipEvent_t>(stop));
  if (rc != hipSuccess) return nmf::fail(NMF_EHIP, "nmf_events_elapsed_ms: %s", hipGetErrorString(rc));
  return NMF_OK;
}

extern "C" const char* nmf_last_error(void) { return g_err; }

extern "C" const char* nmf_version(void) { return "libnmf 0.1 (gfx950)"; }
