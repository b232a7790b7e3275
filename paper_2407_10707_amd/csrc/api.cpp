// Error reporting and launch timing shared by every entry point.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"

namespace rga {

static thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RGA_EHIP, "%s: %s", what, hipGetErrorString(e));
  return RGA_OK;
}

namespace {
struct Rec {
  std::string name;
  hipEvent_t a = nullptr, b = nullptr;
};
std::mutex g_mu;
bool g_on = false;
std::string g_filter;           // empty: time every kernel
std::vector<Rec> g_recs;        // completed or pending start/stop pairs
std::vector<hipEvent_t> g_pool; // reusable events
std::vector<std::pair<std::string, std::pair<double, int64_t>>> g_sums;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  hipEventCreate(&e);
  return e;
}

void drain_locked() {
  for (auto& r : g_recs) {
    if (!r.a || !r.b) continue;
    hipEventSynchronize(r.b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, r.a, r.b);
    bool found = false;
    for (auto& s : g_sums)
      if (s.first == r.name) {
        s.second.first += ms;
        s.second.second += 1;
        found = true;
        break;
      }
    if (!found) g_sums.push_back({r.name, {ms, 1}});
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
}
}  // namespace

bool timing_on() { return g_on; }

void timing_mark(const char* name, hipStream_t s, bool start) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_filter.empty() && g_filter != name) return;
  if (start) {
    Rec r;
    r.name = name;
    r.a = take_event();
    hipEventRecord(r.a, s);
    g_recs.push_back(r);
  } else {
    for (auto it = g_recs.rbegin(); it != g_recs.rend(); ++it)
      if (!it->b && it->name == name) {
        it->b = take_event();
        hipEventRecord(it->b, s);
        break;
      }
    if (g_recs.size() > 4096) drain_locked();
  }
}

}  // namespace rga

extern "C" {

const char* rga_last_error(void) { return rga::g_err; }

int rga_abi_version(void) { return 3; }

int rga_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(rga::g_mu);
  rga::g_on = on != 0;
  return RGA_OK;
}

int rga_timing_filter(const char* kernel) {
  std::lock_guard<std::mutex> lk(rga::g_mu);
  rga::g_filter = kernel ? kernel : "";
  return RGA_OK;
}

int rga_timing_reset(void) {
  std::lock_guard<std::mutex> lk(rga::g_mu);
  rga::drain_locked();
  rga::g_sums.clear();
  return RGA_OK;
}

int rga_timing_read(const char* kernel, double* total_ms, int64_t* launches) {
  if (!kernel || !total_ms || !launches) return rga::fail(RGA_EINVAL, "rga_timing_read: null");
  std::lock_guard<std::mutex> lk(rga::g_mu);
  rga::drain_locked();
  *total_ms = 0.0;
  *launches = 0;
  for (auto& s : rga::g_sums)
    if (s.first == kernel) {
      *total_ms = s.second.first;
      *launches = s.second.second;
    }
  return RGA_OK;
}

}  // extern "C"
