// gfx950 kernels of libfw2: launchers of the time step (the kernels are
// instantiated per dimension and phase in step_p2/v2/p3/v3.hip), the sparse
// source and receiver kernels and small utilities.
#include "step_kernels.hpp"

namespace fw2 {

namespace {

__global__ void source_kernel(const SparseArgs s)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= s.n) return;
    const long long step = *s.step;
    if (step >= s.n_t) return;
    const int64_t pi = padded_index(s.geo, s.idx[q]);
    s.p[pi] = s.p[pi] + s.w[q] * s.signals[(int64_t)s.sig[q] * s.n_t + step];
}

// One block: record the receivers of the current step, then advance the
// device step counter (single block, so no other block reads it meanwhile).
__global__ void __launch_bounds__(256) receiver_kernel(const SparseArgs s)
{
    record_receivers(s);
}

__global__ void fill_kernel(float *dst, int64_t n, float value)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = value;
}

__global__ void set_counter_kernel(long long *counter, long long value)
{
    if (threadIdx.x == 0) counter[0] = value;
}

__global__ void check_kernel(const float *p, const Geometry g, float limit, int *flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.n[0]) return;
    // grid y and z are at most 65535 blocks: stride over larger extents
    bool bad = false;
    for (int k = blockIdx.z; k < g.n[2]; k += gridDim.z)
        for (int j = blockIdx.y; j < g.n[1]; j += gridDim.y) {
            const float v = p[g.origin + (int64_t)k * g.plane + (int64_t)j * g.pitch + i];
            bad |= !(fabsf(v) <= limit);                 // also catches NaN
        }
    if (bad) atomicOr(flag, 1);
}

}  // namespace

hipError_t launch_pressure(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t st)
{
    return a.geo.ndim == 2 ? launch_pressure_2d(a, L, scheme, kc, st) : launch_pressure_3d(a, L, scheme, kc, st);
}

hipError_t launch_velocity(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t st)
{
    return a.geo.ndim == 2 ? launch_velocity_2d(a, L, scheme, kc, st) : launch_velocity_3d(a, L, scheme, kc, st);
}

hipError_t launch_sources(const SparseArgs &s, hipStream_t st)
{
    if (s.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(source_kernel, dim3((s.n + 255) / 256), dim3(256), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_receivers(const SparseArgs &s, hipStream_t st)
{
    hipLaunchKernelGGL(receiver_kernel, dim3(1), dim3(256), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_fill(float *dst, int64_t n, float value, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, n, value);
    return hipGetLastError();
}

hipError_t launch_set_counter(long long *counter, long long value, hipStream_t st)
{
    hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(64), 0, st, counter, value);
    return hipGetLastError();
}

hipError_t launch_check(const float *p, const Geometry &g, float limit, int *flag, hipStream_t st)
{
    hipLaunchKernelGGL(check_kernel, dim3((g.n[0] + 255) / 256, std::min(g.n[1], 65535), std::min(g.n[2], 65535)),
                       dim3(256), 0, st, p, g, limit, flag);
    return hipGetLastError();
}

}  // namespace fw2
