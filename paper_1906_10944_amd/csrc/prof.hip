// Event-pair registry behind geneo_prof_enable / geneo_prof_query.
#include <mutex>
#include <string>
#include <vector>

#include "geneo.h"
#include "prof.h"

namespace geneo {
namespace {
struct Rec {
  std::string name;
  hipEvent_t a = nullptr, b = nullptr;
  double bytes = 0.0, flops = 0.0;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;

void clear_locked() {
  for (auto& r : g_recs) {
    if (r.a) (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
  }
  g_recs.clear();
}
}  // namespace

bool prof_on() { return g_on; }

int prof_start(const char* name, hipStream_t st, double bytes, double flops) {
  if (!g_on || !name) return -1;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
  std::lock_guard<std::mutex> lk(g_mu);
  Rec r;
  r.name = name;
  r.bytes = bytes;
  r.flops = flops;
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return -1;
  if (hipEventRecord(r.a, st) != hipSuccess) return -1;
  g_recs.push_back(r);
  return (int)g_recs.size() - 1;
}

void prof_stop(int slot, hipStream_t st) {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (slot < (int)g_recs.size()) (void)hipEventRecord(g_recs[slot].b, st);
}

}  // namespace geneo

extern "C" {

void geneo_prof_enable(int on) {
  std::lock_guard<std::mutex> lk(geneo::g_mu);
  geneo::clear_locked();
  geneo::g_on = on != 0;
}

int geneo_prof_query(const char* kernel, double* total_ms, int* launches, double* bytes,
                     double* flops) {
  if (!kernel || !total_ms || !launches) return GENEO_ERR_ARG;
  std::lock_guard<std::mutex> lk(geneo::g_mu);
  double t = 0.0, by = 0.0, fl = 0.0;
  int n = 0;
  for (auto& r : geneo::g_recs) {
    if (r.name != kernel) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return GENEO_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return GENEO_ERR_HIP;
    t += ms;
    by += r.bytes;
    fl += r.flops;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  if (bytes) *bytes = by;
  if (flops) *flops = fl;
  return GENEO_OK;
}

}  // extern "C"
