// Optional per-kernel-family timing with HIP events recorded on the launch
// stream around every launch of a family, plus the algorithmic flops and
// HBM bytes of each launch (counted from the true subdomain sizes, not the
// padded ones).  Off by default; enabled through mw_timer_enable.
#include <map>
#include <mutex>
#include <utility>

#include "kernels.hpp"

namespace mw {

namespace {
const char* kNames[KF_COUNT] = {"trsm_gemm", "trsm_leaf", "lu_gemm", "lu_panel", "lu_other", "spmm",
                                "cgs_dots", "cgs_update", "restrict", "prolong", "vector", "bgs_dots",
                                "bgs_update", "coarse"};
struct Fam {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double flops = 0, bytes = 0;
  int64_t launches = 0;
};
struct Timer {
  bool on = false;
  Fam fam[KF_COUNT];
  std::vector<hipEvent_t> pool;
  std::map<std::pair<int, hipStream_t>, hipEvent_t> pending;   // open launch per (family, stream)
  std::mutex mu;
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e;
    MW_HIP(hipEventCreate(&e));
    return e;
  }
} g_t;
}  // namespace

bool kt_enabled() { return g_t.on; }

void kt_begin(int f, hipStream_t st) {
  if (!g_t.on) return;
  std::lock_guard<std::mutex> g(g_t.mu);
  hipEvent_t e = g_t.get();
  MW_HIP(hipEventRecord(e, st));
  g_t.pending[{f, st}] = e;
}

void kt_end(int f, hipStream_t st, double flops, double bytes) {
  if (!g_t.on) return;
  std::lock_guard<std::mutex> g(g_t.mu);
  hipEvent_t e = g_t.get();
  MW_HIP(hipEventRecord(e, st));
  auto it = g_t.pending.find({f, st});
  if (it == g_t.pending.end()) {   // kt_begin was not called while the timer was on
    g_t.pool.push_back(e);
    return;
  }
  g_t.fam[f].ev.push_back({it->second, e});
  g_t.pending.erase(it);
  g_t.fam[f].flops += flops;
  g_t.fam[f].bytes += bytes;
  g_t.fam[f].launches++;
}

}  // namespace mw

using namespace mw;

extern "C" {

int32_t mw_timer_families(void) { return KF_COUNT; }
const char* mw_timer_name(int32_t f) { return (f >= 0 && f < KF_COUNT) ? kNames[f] : ""; }

void mw_timer_enable(int32_t on) { g_t.on = on != 0; }

void mw_timer_reset(void) {
  std::lock_guard<std::mutex> g(g_t.mu);
  for (auto& f : g_t.fam) {
    for (auto& p : f.ev) { g_t.pool.push_back(p.first); g_t.pool.push_back(p.second); }
    f.ev.clear();
    f.flops = f.bytes = 0;
    f.launches = 0;
  }
}

// launches, summed milliseconds between the events, algorithmic flops and bytes
// of family f since the last reset (waits for the recorded events).
mw_status mw_timer_read(int32_t f, int64_t* launches, double* ms, double* flops, double* bytes) {
  if (f < 0 || f >= KF_COUNT || !launches || !ms || !flops || !bytes) return MW_EINVAL;
  std::lock_guard<std::mutex> g(g_t.mu);
  double tot = 0;
  for (auto& p : g_t.fam[f].ev) {
    if (hipEventSynchronize(p.second) != hipSuccess) return MW_EDEVICE;
    float t = 0;
    if (hipEventElapsedTime(&t, p.first, p.second) != hipSuccess) return MW_EDEVICE;
    tot += t;
  }
  *launches = g_t.fam[f].launches;
  *ms = tot;
  *flops = g_t.fam[f].flops;
  *bytes = g_t.fam[f].bytes;
  return MW_OK;
}

}  // extern "C"
