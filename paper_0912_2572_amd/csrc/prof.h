// prof.h -- optional HIP-event timing of the library's kernel launches.
#pragma once

#include <hip/hip_runtime.h>

namespace tsqr {

// Records a start event for `tag` on `st` when profiling is on; returns a
// slot id for prof_end (or -1 when profiling is off).
int prof_begin(const char *tag, hipStream_t st);
void prof_end(int slot, hipStream_t st);
// No events are recorded between prof_suspend(true) and prof_suspend(false)
// (used while a stream is captured into a graph).
void prof_suspend(bool on);

// RAII bracket around one launch.
struct ProfScope {
    int slot;
    hipStream_t st;
    ProfScope(const char *tag, hipStream_t s) : slot(prof_begin(tag, s)), st(s) {}
    ~ProfScope() { prof_end(slot, st); }
};

}  // namespace tsqr
