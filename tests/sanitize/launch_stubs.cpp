// Test double for the sanitizer build of the library's host code: the device
// launchers of the kernel translation units replaced by functions that
// enqueue nothing and report that there is no device.  Linked only into
// tests/sanitize/abi_driver; the library itself never uses it.
#include "kernels.hpp"
#include "probe.hpp"

namespace fw2 {

hipError_t launch_pressure(const StepArgs &, int, int, const KernelConfig &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_velocity(const StepArgs &, int, int, const KernelConfig &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_sources(const SparseArgs &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_receivers(const SparseArgs &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_fill(float *, int64_t, float, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_check(const float *, const Geometry &, float, int *, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_set_counter(long long *, long long, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_pack(const PlaneSet &, const Geometry &, float *, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_unpack(const PlaneSet &, const Geometry &, const float *, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_medium(const MediumArgs &, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_stream_probe(int, void *, uint64_t, hipStream_t) { return hipErrorNoDevice; }
hipError_t launch_batch_step(const BatchTable *, int, int, unsigned, hipStream_t) { return hipErrorNoDevice; }
void prepare_batch_launches() {}
hipError_t claim_static_batch_table(int, BatchTable **table, bool *busy)
{
    *table = nullptr;
    *busy = false;
    return hipErrorNoDevice;
}
void release_static_batch_table(int) {}
hipError_t launch_adjoint_step(const StepArgs &, const SparseArgs &, const SparseArgs &, int, const float *,
                               const float *, const AdjointBuffers &, long long, bool, const float *, hipStream_t,
                               bool *)
{
    return hipErrorNoDevice;
}
hipError_t launch_adjoint_gradient(const StepArgs &, const AdjointBuffers &, hipStream_t) { return hipErrorNoDevice; }

}  // namespace fw2
