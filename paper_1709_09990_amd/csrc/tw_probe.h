// Random-access reference kernel: the rate the machine sustains for the access
// pattern of the table insert (random 16-byte reads, random 64-bit CAS).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace twk {

// mode 0: one 16-byte load per operation, one in flight per lane;
// mode 1: one 64-bit compare-and-swap per operation;
// mode 2: 16-byte loads, eight in flight per lane.
hipError_t launch_probe_rate(void *buf, uint64_t bytes, uint64_t per_thread, int mode, unsigned blocks,
                             uint32_t *sink, hipStream_t s);

constexpr int kProbeBlock = 256;

}  // namespace twk
