// gfx950 kernels of libfw2 around the time step: the halo planes of a slab
// of a grid split along z (pack / unpack), the medium of a domain built
// from device maps, and the streaming probes of the measurement.
//
// All are plain streaming kernels (bandwidth bound, no reuse): one thread
// per element, consecutive threads on consecutive x, so every wavefront
// reads and writes 256 contiguous bytes.
#include "kernels.hpp"
#include "probe.hpp"

#include <algorithm>

namespace fw2 {

namespace {

constexpr int kPackBX = 256;

// Range q of a plane set holding packed plane `pl`, and the plane's z.
__device__ __forceinline__ void plane_of(const PlaneSet &s, int pl, int &q, int &z)
{
    q = 0;
    int base = 0;
    while (q < s.n - 1 && pl >= base + s.nz[q]) {
        base += s.nz[q];
        ++q;
    }
    z = s.z0[q] + (pl - base);
}

// Grid dimensions y and z are limited to 65535 blocks: larger extents are
// covered by striding.
constexpr int kMaxGridYZ = 65535;

// grid: (x blocks, rows, planes of the set); packed layout [plane][ny][nx].
template <bool PACK>
__global__ void __launch_bounds__(kPackBX) halo_copy(const PlaneSet s, const Geometry g, float *packed)
{
    const int x = blockIdx.x * kPackBX + threadIdx.x;
    const int pl = blockIdx.z;
    if (x >= g.n[0]) return;
    int q, z;
    plane_of(s, pl, q, z);
    for (int y = blockIdx.y; y < g.n[1]; y += gridDim.y) {
        float *f = const_cast<float *>(s.arr[q]) + g.origin + (int64_t)z * g.plane + (int64_t)y * g.pitch + x;
        float *b = packed + ((int64_t)pl * g.n[1] + y) * g.n[0] + x;
        if (PACK)
            *b = *f;
        else
            *f = *b;
    }
}

// Medium values of one point from device maps, in FP64 with the host
// conversion's operation order and no contraction, so both give the same
// FP32 values.
__device__ __forceinline__ void medium_point(const MediumArgs &m, int x, int y, int z)
{
#pragma clang fp contract(off)
    const Geometry &g = m.geo;
    const int64_t q = ((int64_t)z * g.n[1] + y) * g.n[0] + x;
    const int64_t o = g.origin + (int64_t)z * g.plane + (int64_t)y * g.pitch + x;
    const float cf = m.c[q], rf = m.rho[q], bf = m.beta[q];
    const bool ok_c = cf > 0.0f && cf <= __FLT_MAX__;       // positive and finite (NaN fails)
    const bool ok_r = rf > 0.0f && rf <= __FLT_MAX__;
    const bool ok_b = bf >= -__FLT_MAX__ && bf <= __FLT_MAX__;
    const int lab = m.label ? (int)m.label[q] : 0;
    if (!(ok_c && ok_r && ok_b) || lab >= m.n_labels) {
        atomicOr(&m.stats[2], 1u);
        return;
    }
    // largest c: max of the bit patterns of positive floats; smallest c: max
    // of (bits of +inf - bits)
    const unsigned int bits = __float_as_uint(cf);
    atomicMax(&m.stats[0], bits);
    atomicMax(&m.stats[1], 0x7f800000u - bits);
    const double c = cf, rr = rf, b = bf;
    const double k0 = 1.0 / (rr * c * c);
    m.kap[o] = (float)k0;
    m.nlq[o] = (float)(k0 * (m.B0 + m.B1 * b));
    m.rhop[o] = (float)rr;
    if (m.labp) m.labp[o] = (uint8_t)lab;
}

__global__ void __launch_bounds__(256) medium_kernel(const MediumArgs m)
{
    const int x = blockIdx.x * 256 + threadIdx.x;
    if (x >= m.geo.n[0]) return;
    for (int z = blockIdx.z; z < m.geo.n[2]; z += gridDim.z)
        for (int y = blockIdx.y; y < m.geo.n[1]; y += gridDim.y) medium_point(m, x, y, z);
}

}  // namespace

hipError_t launch_pack(const PlaneSet &s, const Geometry &g, float *dst, hipStream_t st)
{
    if (s.total <= 0) return hipSuccess;
    const dim3 grid((g.n[0] + kPackBX - 1) / kPackBX, std::min(g.n[1], kMaxGridYZ), s.total);
    hipLaunchKernelGGL(halo_copy<true>, grid, dim3(kPackBX), 0, st, s, g, dst);
    return hipGetLastError();
}

hipError_t launch_unpack(const PlaneSet &s, const Geometry &g, const float *src, hipStream_t st)
{
    if (s.total <= 0) return hipSuccess;
    const dim3 grid((g.n[0] + kPackBX - 1) / kPackBX, std::min(g.n[1], kMaxGridYZ), s.total);
    hipLaunchKernelGGL(halo_copy<false>, grid, dim3(kPackBX), 0, st, s, g, const_cast<float *>(src));
    return hipGetLastError();
}

hipError_t launch_medium(const MediumArgs &m, hipStream_t st)
{
    const dim3 grid((m.geo.n[0] + 255) / 256, std::min(m.geo.n[1], kMaxGridYZ), std::min(m.geo.n[2], kMaxGridYZ));
    hipLaunchKernelGGL(medium_kernel, grid, dim3(256), 0, st, m);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Streaming probes (measurement).  They give the HBM rate that a plain
// kernel of a given access pattern reaches on the device, the reference
// against which the step kernels' measured traffic is read.  One thread per
// element, no loop, so the resident waves always cover one compact address
// window.
// ---------------------------------------------------------------------------

namespace {

constexpr int kProbeBX = 256;

__global__ void __launch_bounds__(kProbeBX) probe_copy16(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                         uint64_t n)
{
    const uint64_t i = blockIdx.x * (uint64_t)kProbeBX + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// The velocity phase's per-point byte mix at L = 2 in 3D without its
// stencil: 12 FP32 arrays read (p, three v, rho, kappa0, six memory
// variables), 9 written (three v, six memory variables).
struct MixArgs {
    const float *r[12];
    float *w[9];
};

__global__ void __launch_bounds__(kProbeBX) probe_mix(const MixArgs m, uint64_t n)
{
    const uint64_t i = blockIdx.x * (uint64_t)kProbeBX + threadIdx.x;
    if (i >= n) return;
    float x[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) x[q] = m.r[q][i];
    const float t = (x[0] + x[4]) + x[5];
#pragma unroll
    for (int q = 0; q < 3; ++q) m.w[q][i] = x[1 + q] + t;
#pragma unroll
    for (int q = 0; q < 6; ++q) m.w[3 + q][i] = fmaf(0.5f, x[6 + q], t);
}

}  // namespace

uint64_t stream_probe_elements(int kind, uint64_t bytes)
{
    if (kind == 0) return bytes / 32;                         // float4 pairs: half read, half written
    return bytes / (21 * 4) / 64 * 64;                         // points per array, arrays 256-byte aligned
}

hipError_t launch_stream_probe(int kind, void *buf, uint64_t bytes, hipStream_t stream)
{
    const uint64_t n = stream_probe_elements(kind, bytes);
    const unsigned blocks = (unsigned)((n + kProbeBX - 1) / kProbeBX);
    if (kind == 0) {
        const float4 *src = (const float4 *)buf;
        hipLaunchKernelGGL(probe_copy16, dim3(blocks), dim3(kProbeBX), 0, stream, src, (float4 *)buf + n, n);
    } else {
        MixArgs m;
        float *f = (float *)buf;
        for (int q = 0; q < 12; ++q) m.r[q] = f + (uint64_t)q * n;
        for (int q = 0; q < 9; ++q) m.w[q] = f + (uint64_t)(12 + q) * n;
        hipLaunchKernelGGL(probe_mix, dim3(blocks), dim3(kProbeBX), 0, stream, m, n);
    }
    return hipGetLastError();
}

}  // namespace fw2
