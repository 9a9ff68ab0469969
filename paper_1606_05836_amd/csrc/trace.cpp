// Optional rocTX ranges around the library's entry points, for timelines
// (rocprofv3 --marker-trace): with PERMHIP_ROCTX=1 in the environment the
// first traced call loads the rocTX library and every traced entry point pushes a
// range named after itself until it returns.  Without the variable, or when
// the library cannot be loaded, the ranges cost one flag test.
#include <dlfcn.h>

#include <cstdlib>
#include <cstring>
#include <mutex>

#include "ph_host.hpp"

namespace ph {

namespace {
int (*g_push)(const char*) = nullptr;
int (*g_pop)() = nullptr;
bool g_on = false;
std::once_flag g_once;

void trace_init() {
  const char* e = getenv("PERMHIP_ROCTX");
  if (!e || strcmp(e, "1") != 0) return;
  // the rocprofiler-sdk rocTX library (what rocprofv3 records), else the older one
  void* h = nullptr;
  for (const char* lib : {"librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so", "libroctx64.so"})
    if ((h = dlopen(lib, RTLD_NOW | RTLD_LOCAL))) break;
  if (!h) return;
  g_push = reinterpret_cast<int (*)(const char*)>(dlsym(h, "roctxRangePushA"));
  g_pop = reinterpret_cast<int (*)()>(dlsym(h, "roctxRangePop"));
  g_on = g_push && g_pop;
}
}  // namespace

TraceRange::TraceRange(const char* name) {
  std::call_once(g_once, trace_init);
  on = g_on;
  if (on) g_push(name);
}

TraceRange::~TraceRange() {
  if (on) g_pop();
}

}  // namespace ph
