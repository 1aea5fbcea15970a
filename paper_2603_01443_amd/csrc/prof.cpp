// Kernel timing.  When enabled, every kernel the library launches (of the
// families selected by the mask) is bracketed by a pair of HIP events recorded
// on the stream it is launched on; reading the profile waits for those events
// and accumulates launches and milliseconds per kernel family.  Events come
// from a pool and are reused.  Timing events add a little time between
// launches, so timing only the kernel of interest keeps the rest unperturbed.
#include <cstring>
#include <mutex>
#include <vector>

#include "ccut_internal.h"

namespace ccut {

namespace {

struct Record {
  int kernel;
  hipEvent_t a, b;
};

std::mutex g_mu;
bool g_on = false;
uint32_t g_mask = ~0u;  // kernel families that are timed while profiling is on
std::vector<Record> g_open;
std::vector<hipEvent_t> g_pool;
int64_t g_count[PROF_N] = {};
double g_ms[PROF_N] = {};

const char* const kNames[PROF_N] = {"sim",    "merge_f32", "split",  "tables",
                                    "merge_gemm", "reduce", "mlp",     "expect"};

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

int prof_begin(int kernel, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on || !((g_mask >> kernel) & 1u)) return -1;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
  Record r{kernel, take(), take()};
  if (!r.a || !r.b) return -1;
  if (hipEventRecord(r.a, s) != hipSuccess) return -1;
  g_open.push_back(r);
  return (int)g_open.size() - 1;
}

void prof_end(int token, hipStream_t s) {
  if (token < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (token < (int)g_open.size()) (void)hipEventRecord(g_open[token].b, s);
}

const char* prof_name(int k) { return (k >= 0 && k < PROF_N) ? kNames[k] : "?"; }

}  // namespace ccut

using namespace ccut;

extern "C" int ccut_profile_enable(int32_t on) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  return CCUT_OK;
}

extern "C" int ccut_profile_mask(uint32_t mask) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  g_mask = mask;
  return CCUT_OK;
}

extern "C" int ccut_profile_read(int32_t kernel, int64_t* launches, double* total_ms, const char** name) {
  clear_error();
  if (kernel < 0 || kernel >= PROF_N) return fail(CCUT_EINVAL, "kernel id %d out of range", kernel);
  std::lock_guard<std::mutex> lk(g_mu);
  for (Record& r : g_open) {
    float ms = 0.f;
    CCUT_HIP(hipEventSynchronize(r.b));
    CCUT_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    g_count[r.kernel] += 1;
    g_ms[r.kernel] += ms;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_open.clear();
  if (launches) *launches = g_count[kernel];
  if (total_ms) *total_ms = g_ms[kernel];
  if (name) *name = kNames[kernel];
  return CCUT_OK;
}

extern "C" int ccut_profile_reset(void) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  for (Record& r : g_open) {
    (void)hipEventSynchronize(r.b);
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_open.clear();
  std::memset(g_count, 0, sizeof(g_count));
  std::memset(g_ms, 0, sizeof(g_ms));
  return CCUT_OK;
}
