// Opt-in kernel timer (see ktimer.h) and its C-ABI controls.
#include <string.h>
#include <atomic>
#include <vector>
#include "ktimer.h"

namespace mmf {

namespace {
struct Timer {
  char name[64] = {0};
  bool armed = false;
  std::vector<hipEvent_t> ev;     // 2 per launch
  std::vector<double> work;
  size_t used = 0;
};
Timer g_timer;
constexpr size_t KT_MAX = 1 << 17;
}  // namespace

// profiling throttle: wait for the device after every g_sync_every launches
std::atomic<int64_t> g_sync_every{0};
std::atomic<int64_t> g_launches{0};

int launch_check() {
  if (hipGetLastError() != hipSuccess) return 1;
  const int64_t every = g_sync_every.load(std::memory_order_relaxed);
  if (every > 0 && (g_launches.fetch_add(1, std::memory_order_relaxed) + 1) % every == 0)
    if (hipDeviceSynchronize() != hipSuccess) return 1;
  return 0;
}

bool ktimer_armed(const char *name) { return g_timer.armed && strcmp(g_timer.name, name) == 0; }

int ktimer_begin(const char *name, hipStream_t st) {
  if (!ktimer_armed(name)) return -1;
  if (g_timer.used >= KT_MAX) return -1;
  const size_t s = g_timer.used++;
  if (g_timer.ev.size() < 2 * (s + 1)) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { --g_timer.used; return -1; }
    g_timer.ev.push_back(a);
    g_timer.ev.push_back(b);
    g_timer.work.push_back(0.0);
  }
  if (hipEventRecord(g_timer.ev[2 * s], st) != hipSuccess) return -1;
  return (int)s;
}

void ktimer_end(int slot, hipStream_t st, double work) {
  if (slot < 0) return;
  (void)hipEventRecord(g_timer.ev[2 * slot + 1], st);
  g_timer.work[slot] = work;
}

}  // namespace mmf

using namespace mmf;

// Arm the timer for one kernel class ("hemv", ...); clears previous records.
extern "C" int mmf_ktimer_arm(const char *kernel) {
  if (!kernel || strlen(kernel) >= sizeof(g_timer.name)) return -1;
  strcpy(g_timer.name, kernel);
  g_timer.armed = true;
  g_timer.used = 0;
  return MMF_OK;
}

// Disarm, wait for the recorded events and report the launch count, the sum
// of kernel durations (ms) and the summed attributed work.
extern "C" int mmf_ktimer_read(int64_t *launches, double *total_ms, double *work) {
  if (!launches) return -1;
  if (!total_ms) return -2;
  if (!work) return -3;
  g_timer.armed = false;
  double t = 0.0, wsum = 0.0;
  for (size_t s = 0; s < g_timer.used; ++s) {
    float ms = 0.f;
    if (hipEventSynchronize(g_timer.ev[2 * s + 1]) != hipSuccess) return MMF_ERR_HIP;
    if (hipEventElapsedTime(&ms, g_timer.ev[2 * s], g_timer.ev[2 * s + 1]) != hipSuccess) return MMF_ERR_HIP;
    t += ms;
    wsum += g_timer.work[s];
  }
  *launches = (int64_t)g_timer.used;
  *total_ms = t;
  *work = wsum;
  return MMF_OK;
}

// Profiling aid: wait for the device after every n library launches (n <= 0
// turns it off).
extern "C" int mmf_profile_sync_every(int64_t n) {
  g_sync_every.store(n > 0 ? n : 0);
  g_launches.store(0);
  return MMF_OK;
}
