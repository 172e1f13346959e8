// Kernel timer of the library: HIP events around each launch, aggregated per
// kernel name.  Off by default; never active while a stream is capturing.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/acat.h"
#include "acat_internal.hpp"

namespace acat {
namespace {

struct Record {
  std::string name;
  hipEvent_t start, stop;
};

struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<Record> open;          // recorded, not yet read
  std::vector<hipEvent_t> pool;      // free events
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

Profiler& prof() {
  static Profiler P;
  return P;
}

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return true;
  return st != hipStreamCaptureStatusNone;
}

}  // namespace

ProfScope::ProfScope(const char* name, hipStream_t s) : slot(-1), stream(s) {
  Profiler& P = prof();
  if (!P.on) return;
  std::lock_guard<std::mutex> g(P.mu);
  if (!P.on || capturing(s)) return;
  Record r{name, P.get(), P.get()};
  if (!r.start || !r.stop) return;
  if (hipEventRecord(r.start, s) != hipSuccess) return;
  P.open.push_back(r);
  slot = (int)P.open.size() - 1;
}

ProfScope::~ProfScope() {
  if (slot < 0) return;
  Profiler& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  if (slot < (int)P.open.size()) (void)hipEventRecord(P.open[slot].stop, stream);
}

}  // namespace acat

using namespace acat;

extern "C" {

acat_status acat_profile_enable(int32_t on) {
  Profiler& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  for (auto& r : P.open) {
    (void)hipEventSynchronize(r.stop);
    P.pool.push_back(r.start);
    P.pool.push_back(r.stop);
  }
  P.open.clear();
  P.on = on != 0;
  return ACAT_OK;
}

acat_status acat_profile_read(int32_t max_kernels, char* names, double* total_ms, int64_t* launches,
                              int32_t* n_kernels) {
  if (!n_kernels) return ACAT_ERR_NULL;
  Profiler& P = prof();
  std::lock_guard<std::mutex> g(P.mu);
  std::vector<std::string> nm;
  std::vector<double> ms;
  std::vector<int64_t> cnt;
  for (auto& r : P.open) {
    if (hipEventSynchronize(r.stop) != hipSuccess) return ACAT_ERR_DEVICE;
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.start, r.stop) != hipSuccess) return ACAT_ERR_DEVICE;
    size_t k = 0;
    while (k < nm.size() && nm[k] != r.name) ++k;
    if (k == nm.size()) {
      nm.push_back(r.name);
      ms.push_back(0.0);
      cnt.push_back(0);
    }
    ms[k] += t;
    cnt[k] += 1;
  }
  *n_kernels = (int32_t)nm.size();
  for (size_t k = 0; k < nm.size() && (int32_t)k < max_kernels; ++k) {
    if (names) {
      std::strncpy(names + 64 * k, nm[k].c_str(), 63);
      names[64 * k + 63] = '\0';
    }
    if (total_ms) total_ms[k] = ms[k];
    if (launches) launches[k] = cnt[k];
  }
  return ACAT_OK;
}

}  // extern "C"
