// Opt-in timing of one kernel class for benchmarks (internal header).
// While a timer is armed for kernel class `name`, every launch of that class
// is bracketed by HIP events recorded on the launch stream, and the
// algorithmic bytes (or flops) that the caller attributes to the launch are
// summed.  Process-wide state, single-threaded use only; off by default.
#pragma once
#include "common.h"

namespace mmf {

bool ktimer_armed(const char *name);
// Record the start event; returns a slot handle (or -1 when not armed / full).
int ktimer_begin(const char *name, hipStream_t st);
void ktimer_end(int slot, hipStream_t st, double work);

}  // namespace mmf
