// Optional roctx ranges around the host-side phases of a solve. With PPRPA_ROCTX=1 in the
// environment the roctx library of the ROCm profiler SDK is opened on first use and every
// TraceRange pushes a named range on the calling thread; rocprofv3 --marker-trace then records
// them next to the kernel trace. Without the variable, or when the library cannot be opened,
// a TraceRange does nothing. The ranges mark host time (kernel launches are asynchronous, so
// a phase that only enqueues work is short and the wait that follows carries the GPU time).
#include <dlfcn.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "internal.h"

namespace pprpa {
namespace {

using push_fn = int (*)(const char*);
using pop_fn = int (*)();

struct Roctx {
  push_fn push = nullptr;
  pop_fn pop = nullptr;
};

Roctx open_roctx() {
  Roctx r;
  const char* on = std::getenv("PPRPA_ROCTX");
  if (!on || std::strcmp(on, "1") != 0) return r;
  void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
  if (!h) h = dlopen("librocprofiler-sdk-roctx.so", RTLD_NOW | RTLD_LOCAL);
  if (!h) {
    std::fprintf(stderr, "pprpa: PPRPA_ROCTX=1 but the roctx library could not be opened (%s)\n",
                 dlerror());
    return r;
  }
  r.push = reinterpret_cast<push_fn>(dlsym(h, "roctxRangePushA"));
  r.pop = reinterpret_cast<pop_fn>(dlsym(h, "roctxRangePop"));
  if (!r.push || !r.pop) {
    std::fprintf(stderr, "pprpa: the roctx library lacks roctxRangePushA/roctxRangePop\n");
    r = Roctx{};
  }
  return r;
}

const Roctx& roctx() {
  static const Roctx r = open_roctx();  // thread-safe one-time initialisation
  return r;
}

}  // namespace

bool trace_enabled() { return roctx().push != nullptr; }

TraceRange::TraceRange(const char* name) : on_(false) {
  const Roctx& r = roctx();
  if (r.push) {
    r.push(name);
    on_ = true;
  }
}

TraceRange::~TraceRange() {
  if (on_) roctx().pop();
}

}  // namespace pprpa
