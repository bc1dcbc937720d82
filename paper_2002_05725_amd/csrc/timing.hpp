// Optional HIP-event timing of apply_H launches (off by default).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace syk {

void timing_enable(bool on);
bool timing_enabled();
void timing_begin(hipStream_t s);   // records a start event on s (no-op when disabled)
void timing_end(hipStream_t s);     // records the matching stop event
// Waits for the recorded events; number of timed launches and their summed duration.
void timing_read(int64_t* launches, double* total_ms);
void timing_reset();

}  // namespace syk
