// Internal hooks of the launch profiler (gumap_profile.h).  prof_begin
// returns a mark (or -1 when recording is off); prof_end records the stop
// event; prof_set_bytes fills in bytes known only after device counters were
// read; prof_resolve runs after the stream drained.
#pragma once

#include <hip/hip_runtime.h>

namespace gm {

bool prof_on();
int prof_begin(const char *name, hipStream_t s);
void prof_end(int mark, hipStream_t s, double bytes);
void prof_set_bytes(int mark, double bytes);
// Bytes a launch moves beyond its algorithmic bytes (reported separately).
void prof_set_extra(int mark, double bytes);
void prof_resolve();

}  // namespace gm
