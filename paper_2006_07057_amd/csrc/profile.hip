// Optional per-launch timing with HIP events recorded on the launch's own
// stream (off by default; used by the benchmark to time the persistent
// solver and the other kernels of the path without host synchronisation).
#include "sk_internal.h"

#include <mutex>
#include <vector>

namespace sk {
namespace {

struct Rec {
  hipEvent_t a, b;
  int kind;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;

}  // namespace

void* prof_begin(int kind, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return nullptr;
  Rec r;
  r.kind = kind;
  if (hipEventCreate(&r.a) != hipSuccess) return nullptr;
  if (hipEventCreate(&r.b) != hipSuccess) {
    (void)hipEventDestroy(r.a);
    return nullptr;
  }
  (void)hipEventRecord(r.a, s);
  g_recs.push_back(r);
  return reinterpret_cast<void*>(g_recs.size());
}

void prof_end(void* token, hipStream_t s) {
  if (!token) return;
  std::lock_guard<std::mutex> lk(g_mu);
  const size_t idx = reinterpret_cast<size_t>(token) - 1;
  if (idx < g_recs.size()) (void)hipEventRecord(g_recs[idx].b, s);
}

}  // namespace sk

extern "C" {

int sinkhorn_profile(int32_t enable) {
  std::lock_guard<std::mutex> lk(sk::g_mu);
  for (auto& r : sk::g_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  sk::g_recs.clear();
  sk::g_on = enable != 0;
  return SK_OK;
}

int sinkhorn_profile_read(int32_t kind, double* total_ms, int64_t* launches,
                          double* max_ms) {
  if (!total_ms || !launches) return SK_EINVAL;
  std::lock_guard<std::mutex> lk(sk::g_mu);
  double tot = 0.0, mx = 0.0;
  int64_t cnt = 0;
  for (auto& r : sk::g_recs) {
    if (r.kind != kind) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return SK_EHIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return SK_EHIP;
    tot += ms;
    mx = ms > mx ? ms : mx;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  if (max_ms) *max_ms = mx;
  return SK_OK;
}

}  // extern "C"
