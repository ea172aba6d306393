// gfx950 kernels of libfw2: one time step of the staggered Fullwave 2 system.
//
// Pressure phase (Eq. general6 with nabla_2, Sec. 3.1 / 3.2), per p point:
//   D_a = (D^- v_a), memory terms of each mechanism, S = sum_a (w D_a + M),
//   p <- p - dt S / (kappa0 (1 + kappa0 (1 - 2 beta) p)).
// Velocity phase (Eq. general5 with nabla_1), per v_a point inside the grid:
//   D = (D^+ p)_a, memory terms, S = w D + M,
//   v_a <- v_a - dt S / (rho_a (1 + kappa0_a pbar)),
//   rho_a, kappa0_a, pbar the means of the two neighbouring cells.
// Memory terms: printed   m <- b m + c D, M = m (after the update);
//               centred   M = m (before the update), m <- b m + c D,
// with w, b, c from the per-axis (boundary slot, tissue label) tables.
//
// The work is bandwidth bound (about 1 flop per byte), so there is no MFMA:
// threads map to consecutive x (coalesced 256-byte rows per wavefront) and
// each thread walks several rows, the stencil taps reusing L1/L2-resident
// neighbours.
#include "kernels.hpp"

namespace fw2 {

namespace {

constexpr int kBX = 64;     // threads along x (one wavefront per row segment)
constexpr int kBY = 4;      // rows of threads per block
constexpr int kRY = 2;      // rows per thread

__device__ __forceinline__ int slot_int(int x, int n, int nb)
{
    // distance (cells) from the inner edge of the layer, pressure positions
    const int s = max(nb - x, x - (n - 1 - nb));
    return max(s, 0);
}

__device__ __forceinline__ int slot_half(int x, int n, int nb)
{
    // velocity position x + 1/2: slot k <-> distance k - 1/2 (k >= 1)
    const int s = max(nb - x, x - (n - 2 - nb));
    return max(s, 0);
}

template <int NDIM>
__device__ __forceinline__ int64_t axis_offset(const Geometry &g, int a)
{
    return a == 0 ? (int64_t)1 : (a == 1 ? g.pitch : g.plane);
}

template <int NDIM, int L, bool CENTRED>
__global__ void __launch_bounds__(kBX * kBY) pressure_kernel(const StepArgs a)
{
    const Geometry &g = a.geo;
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int k = blockIdx.z;
    if (i >= g.n[0]) return;
    const int j0 = (blockIdx.y * kBY + threadIdx.y) * kRY;
#pragma unroll
    for (int r = 0; r < kRY; ++r) {
        const int j = j0 + r;
        if (j >= g.n[1]) break;
        const int c[3] = {i, j, k};
        const int64_t idx = g.origin + (int64_t)k * g.plane + (int64_t)j * g.pitch + i;
        const int lab = a.label ? (int)a.label[idx] : 0;
        float S = 0.0f;
#pragma unroll
        for (int ax = 0; ax < NDIM; ++ax) {
            const float *va = a.v + ax * g.stride;
            const int64_t o = axis_offset<NDIM>(g, ax);
            float D = a.g[0] * (va[idx] - va[idx - o]);
            D = fmaf(a.g[1], va[idx + o] - va[idx - 2 * o], D);
            D = fmaf(a.g[2], va[idx + 2 * o] - va[idx - 3 * o], D);
            D = fmaf(a.g[3], va[idx + 3 * o] - va[idx - 4 * o], D);
            float cr = 0.0f;
#pragma unroll
            for (int bx = 0; bx < NDIM; ++bx) {
                if (bx == ax) continue;
                const int64_t o2 = axis_offset<NDIM>(g, bx);
                cr += (va[idx + o2] - va[idx - o + o2]) + (va[idx - o2] - va[idx - o - o2]);
            }
            D = fmaf(a.g11, cr, D);
            const int s = slot_int(c[ax], g.n[ax], a.nb[ax]);
            const int t = s * a.n_labels + lab;
            const float2 *bc = a.bc2[ax] + (int64_t)t * L;
            float Sa = a.w2[ax][t] * D;
            float *ps = a.psi2 + (int64_t)ax * L * g.stride + idx;
#pragma unroll
            for (int nu = 0; nu < L; ++nu) {
                const float2 q = bc[nu];
                const float m = ps[nu * g.stride];
                const float mn = fmaf(q.x, m, q.y * D);
                Sa += CENTRED ? m : mn;
                ps[nu * g.stride] = mn;
            }
            S += Sa;
        }
        const float pold = a.p[idx];
        const float kappa = a.kap[idx] * (1.0f + a.nlq[idx] * pold);
        a.p[idx] = pold - a.dt * S / kappa;
    }
}

template <int NDIM, int L, bool CENTRED>
__global__ void __launch_bounds__(kBX * kBY) velocity_kernel(const StepArgs a)
{
    const Geometry &g = a.geo;
    const int i = blockIdx.x * kBX + threadIdx.x;
    const int k = blockIdx.z;
    if (i >= g.n[0]) return;
    const int j0 = (blockIdx.y * kBY + threadIdx.y) * kRY;
#pragma unroll
    for (int r = 0; r < kRY; ++r) {
        const int j = j0 + r;
        if (j >= g.n[1]) break;
        const int c[3] = {i, j, k};
        const int64_t idx = g.origin + (int64_t)k * g.plane + (int64_t)j * g.pitch + i;
        const int lab = a.label ? (int)a.label[idx] : 0;
        const float *p = a.p;
        const float p0 = p[idx];
        const float r0 = a.rho[idx];
        const float k0 = a.kap[idx];
#pragma unroll
        for (int ax = 0; ax < NDIM; ++ax) {
            if (c[ax] == g.n[ax] - 1) continue;          // outside the grid, held at zero
            const int64_t o = axis_offset<NDIM>(g, ax);
            const float p1 = p[idx + o];
            float D = a.g[0] * (p1 - p0);
            D = fmaf(a.g[1], p[idx + 2 * o] - p[idx - o], D);
            D = fmaf(a.g[2], p[idx + 3 * o] - p[idx - 2 * o], D);
            D = fmaf(a.g[3], p[idx + 4 * o] - p[idx - 3 * o], D);
            float cr = 0.0f;
#pragma unroll
            for (int bx = 0; bx < NDIM; ++bx) {
                if (bx == ax) continue;
                const int64_t o2 = axis_offset<NDIM>(g, bx);
                cr += (p[idx + o + o2] - p[idx + o2]) + (p[idx + o - o2] - p[idx - o2]);
            }
            D = fmaf(a.g11, cr, D);
            const int s = slot_half(c[ax], g.n[ax], a.nb[ax]);
            const int t = s * a.n_labels + lab;
            const float2 *bc = a.bc1[ax] + (int64_t)t * L;
            float S = a.w1[ax][t] * D;
            float *ps = a.psi1 + (int64_t)ax * L * g.stride + idx;
#pragma unroll
            for (int nu = 0; nu < L; ++nu) {
                const float2 q = bc[nu];
                const float m = ps[nu * g.stride];
                const float mn = fmaf(q.x, m, q.y * D);
                S += CENTRED ? m : mn;
                ps[nu * g.stride] = mn;
            }
            const float pbar = 0.5f * (p0 + p1);
            const float rho_a = 0.5f * (r0 + a.rho[idx + o]);
            const float kap_a = 0.5f * (k0 + a.kap[idx + o]);
            float *va = a.v + ax * g.stride;
            va[idx] = va[idx] - a.dt * S / (rho_a * (1.0f + kap_a * pbar));
        }
    }
}

__device__ __forceinline__ int64_t padded_index(const Geometry &g, int64_t f)
{
    const int64_t x = f % g.n[0];
    const int64_t t = f / g.n[0];
    const int64_t y = t % g.n[1];
    const int64_t z = t / g.n[1];
    return g.origin + z * g.plane + y * g.pitch + x;
}

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
    const long long step = *s.step;
    if (step < s.cap)
        for (int r = threadIdx.x; r < s.n; r += blockDim.x)
            s.trace[step * s.n + r] = s.p[padded_index(s.geo, s.idx[r])];
    __syncthreads();
    if (threadIdx.x == 0) s.step[0] = step + 1;
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
    const int j = blockIdx.y;
    const int k = blockIdx.z;
    if (i >= g.n[0]) return;
    const float v = p[g.origin + (int64_t)k * g.plane + (int64_t)j * g.pitch + i];
    if (!(fabsf(v) <= limit)) atomicOr(flag, 1);     // also catches NaN
}

template <int NDIM, int L, bool C>
hipError_t launch_p(const StepArgs &a, hipStream_t st)
{
    dim3 block(kBX, kBY);
    dim3 grid((a.geo.n[0] + kBX - 1) / kBX, (a.geo.n[1] + kBY * kRY - 1) / (kBY * kRY), a.geo.n[2]);
    hipLaunchKernelGGL((pressure_kernel<NDIM, L, C>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <int NDIM, int L, bool C>
hipError_t launch_v(const StepArgs &a, hipStream_t st)
{
    dim3 block(kBX, kBY);
    dim3 grid((a.geo.n[0] + kBX - 1) / kBX, (a.geo.n[1] + kBY * kRY - 1) / (kBY * kRY), a.geo.n[2]);
    hipLaunchKernelGGL((velocity_kernel<NDIM, L, C>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <bool P, int NDIM, int L>
hipError_t dispatch_scheme(const StepArgs &a, int scheme, hipStream_t st)
{
    if (scheme == 0) return P ? launch_p<NDIM, L, false>(a, st) : launch_v<NDIM, L, false>(a, st);
    return P ? launch_p<NDIM, L, true>(a, st) : launch_v<NDIM, L, true>(a, st);
}

template <bool P, int NDIM>
hipError_t dispatch_L(const StepArgs &a, int L, int scheme, hipStream_t st)
{
    switch (L) {
    case 1: return dispatch_scheme<P, NDIM, 1>(a, scheme, st);
    case 2: return dispatch_scheme<P, NDIM, 2>(a, scheme, st);
    case 3: return dispatch_scheme<P, NDIM, 3>(a, scheme, st);
    case 4: return dispatch_scheme<P, NDIM, 4>(a, scheme, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_pressure(const StepArgs &a, int L, int scheme, hipStream_t st)
{
    return a.geo.ndim == 2 ? dispatch_L<true, 2>(a, L, scheme, st) : dispatch_L<true, 3>(a, L, scheme, st);
}

hipError_t launch_velocity(const StepArgs &a, int L, int scheme, hipStream_t st)
{
    return a.geo.ndim == 2 ? dispatch_L<false, 2>(a, L, scheme, st) : dispatch_L<false, 3>(a, L, scheme, st);
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
    hipLaunchKernelGGL(check_kernel, dim3((g.n[0] + 255) / 256, g.n[1], g.n[2]), dim3(256), 0, st,
                       p, g, limit, flag);
    return hipGetLastError();
}

}  // namespace fw2
