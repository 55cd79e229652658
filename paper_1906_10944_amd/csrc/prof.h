// Optional per-kernel timing with HIP events, recorded on the stream each
// kernel is launched on.  Off by default; never active inside graph capture.
#pragma once
#include <hip/hip_runtime.h>

namespace geneo {

bool prof_on();
// Returns a slot to pass to prof_stop, or -1 when timing is off / capturing.
int prof_start(const char* name, hipStream_t st, double bytes, double flops);
void prof_stop(int slot, hipStream_t st);

struct ProfScope {
  int slot;
  hipStream_t st;
  ProfScope(const char* name, hipStream_t s, double bytes = 0.0, double flops = 0.0)
      : slot(prof_start(name, s, bytes, flops)), st(s) {}
  ~ProfScope() { prof_stop(slot, st); }
};

}  // namespace geneo
