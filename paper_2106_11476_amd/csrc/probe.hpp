// Streaming probes of libfw2 (measurement): plain one-thread-per-element
// kernels whose HBM rate is the reference for the step kernels' traffic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fw2 {

// kind 0 copies the first half of buf to the second (16 bytes per thread);
// kind 1 reads 12 and writes 9 FP32 arrays of stream_probe_elements points
// each, laid out one after another in buf.
uint64_t stream_probe_elements(int kind, uint64_t bytes);
hipError_t launch_stream_probe(int kind, void *buf, uint64_t bytes, hipStream_t stream);

}  // namespace fw2
