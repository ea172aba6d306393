// gfx950 kernels of libfw2: one time step of the staggered Fullwave 2 system
// (templates, included by the translation units that instantiate them).
//
// Pressure phase (Eq. general6 with nabla_2, Sec. 3.1 / 3.2), per p point:
//   D_a = (D^- v_a), memory terms of each mechanism, S = sum_a (w D_a + M),
//   p <- p - dt S / (kappa0 (1 + kappa0 B p)), kappa0 B = nlq (B = 1 - 2 beta
//   as printed in Eq. state2).
// Velocity phase (Eq. general5 with nabla_1), per v_a point inside the grid:
//   D = (D^+ p)_a, memory terms, S = w D + M,
//   v_a <- v_a - dt S / (rho_a (1 + A kappa0_a pbar)) (A = 1 as printed),
//   rho_a, kappa0_a, pbar the means of the two neighbouring cells.
// Memory terms: printed   m <- b m + c D, M = m (after the update);
//               centred   M = m (before the update), m <- b m + c D,
// with w, b, c from the per-axis (boundary slot, tissue label) tables.
//
// The work is bandwidth bound (about 1 flop per byte), so there is no MFMA:
// threads map to consecutive x (coalesced 256-byte rows per wavefront) and
// each thread walks several rows, the stencil taps reusing L1/L2-resident
// neighbours.
#pragma once

#include "kernels.hpp"

#include <algorithm>

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

// Points along axis ax of the whole grid (a slab's z axis is the global one).
__device__ __forceinline__ int axis_n(const StepArgs &a, int ax) { return ax == 2 ? a.nz_glob : a.geo.n[ax]; }

// Stencil weights over h at one point: the global set, or (PP) the set of
// the point's own r^2 = s, from the fixed polynomials in s.
struct Wts {
    float g0, g1, g2, g3, g11;
};

template <bool PP>
__device__ __forceinline__ Wts weights(const StepArgs &a, float s)
{
    if constexpr (PP) {
        Wts w;
        w.g0 = fmaf(fmaf(fmaf(a.pw[0][3], s, a.pw[0][2]), s, a.pw[0][1]), s, a.pw[0][0]);
        w.g1 = fmaf(fmaf(fmaf(a.pw[1][3], s, a.pw[1][2]), s, a.pw[1][1]), s, a.pw[1][0]);
        w.g2 = fmaf(fmaf(fmaf(a.pw[2][3], s, a.pw[2][2]), s, a.pw[2][1]), s, a.pw[2][0]);
        w.g3 = fmaf(fmaf(fmaf(a.pw[3][3], s, a.pw[3][2]), s, a.pw[3][1]), s, a.pw[3][0]);
        w.g11 = a.g11s * s;
        return w;
    } else {
        (void)s;
        return Wts{a.g[0], a.g[1], a.g[2], a.g[3], a.g11};
    }
}

// r^2 of a cell from its rho and kappa0 (c^2 = 1 / (rho kappa0)).
__device__ __forceinline__ float cell_r2(const StepArgs &a, float rho, float kap) { return a.q2 / (rho * kap); }

template <int NDIM, int L, bool CENTRED, bool PP>
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
        const int c[3] = {i, j, k + a.z_off};         // global coordinates
        const int64_t idx = g.origin + (int64_t)k * g.plane + (int64_t)j * g.pitch + i;
        const int lab = a.label ? (int)a.label[idx] : 0;
        const Wts W = weights<PP>(a, PP ? cell_r2(a, a.rho[idx], a.kap[idx]) : 0.0f);
        float S = 0.0f;
#pragma unroll
        for (int ax = 0; ax < NDIM; ++ax) {
            const float *va = a.v + ax * g.stride;
            const int64_t o = axis_offset<NDIM>(g, ax);
            float D = W.g0 * (va[idx] - va[idx - o]);
            D = fmaf(W.g1, va[idx + o] - va[idx - 2 * o], D);
            D = fmaf(W.g2, va[idx + 2 * o] - va[idx - 3 * o], D);
            D = fmaf(W.g3, va[idx + 3 * o] - va[idx - 4 * o], D);
            float cr = 0.0f;
#pragma unroll
            for (int bx = 0; bx < NDIM; ++bx) {
                if (bx == ax) continue;
                const int64_t o2 = axis_offset<NDIM>(g, bx);
                cr += (va[idx + o2] - va[idx - o + o2]) + (va[idx - o2] - va[idx - o - o2]);
            }
            D = fmaf(W.g11, cr, D);
            const int s = slot_int(c[ax], axis_n(a, ax), a.nb[ax]);
            const int t = s * a.n_labels + lab;
            const float2 *bc = a.bc2[ax] + (int64_t)t * L;
            float Sa = a.w2[ax][t] * D;
            float *ps = a.psi2 + (int64_t)ax * L * g.stride + idx;
#pragma unroll
            for (int nu = 0; nu < L; ++nu) {
                const float2 q = bc[nu];
                const float m = ntld(&ps[nu * g.stride]);
                const float mn = fmaf(q.x, m, q.y * D);
                Sa += CENTRED ? m : mn;
                ntst(&ps[nu * g.stride + a.out], mn);
            }
            S += Sa;
        }
        const float pold = a.p[idx];
        const float kappa = a.kap[idx] * (1.0f + a.nlq[idx] * pold);
        a.p[idx + a.out] = pold - a.dt * S / kappa;
    }
}

template <int NDIM, int L, bool CENTRED, bool PP>
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
        const int c[3] = {i, j, k + a.z_off};         // global coordinates
        const int64_t idx = g.origin + (int64_t)k * g.plane + (int64_t)j * g.pitch + i;
        const int lab = a.label ? (int)a.label[idx] : 0;
        const float *p = a.p;
        const float p0 = p[idx];
        const float r0 = a.rho[idx];
        const float k0 = a.kap[idx];
        const float s0 = PP ? cell_r2(a, r0, k0) : 0.0f;
#pragma unroll
        for (int ax = 0; ax < NDIM; ++ax) {
            if (c[ax] == axis_n(a, ax) - 1) continue;    // outside the grid, held at zero
            const int64_t o = axis_offset<NDIM>(g, ax);
            const float p1 = p[idx + o];
            // v point between this cell and the next: mean of the two cells' r^2
            const Wts W = weights<PP>(a, PP ? 0.5f * (s0 + cell_r2(a, a.rho[idx + o], a.kap[idx + o])) : 0.0f);
            float D = W.g0 * (p1 - p0);
            D = fmaf(W.g1, p[idx + 2 * o] - p[idx - o], D);
            D = fmaf(W.g2, p[idx + 3 * o] - p[idx - 2 * o], D);
            D = fmaf(W.g3, p[idx + 4 * o] - p[idx - 3 * o], D);
            float cr = 0.0f;
#pragma unroll
            for (int bx = 0; bx < NDIM; ++bx) {
                if (bx == ax) continue;
                const int64_t o2 = axis_offset<NDIM>(g, bx);
                cr += (p[idx + o + o2] - p[idx + o2]) + (p[idx + o - o2] - p[idx - o2]);
            }
            D = fmaf(W.g11, cr, D);
            const int s = slot_half(c[ax], axis_n(a, ax), a.nb[ax]);
            const int t = s * a.n_labels + lab;
            const float2 *bc = a.bc1[ax] + (int64_t)t * L;
            float S = a.w1[ax][t] * D;
            float *ps = a.psi1 + (int64_t)ax * L * g.stride + idx;
#pragma unroll
            for (int nu = 0; nu < L; ++nu) {
                const float2 q = bc[nu];
                const float m = ntld(&ps[nu * g.stride]);
                const float mn = fmaf(q.x, m, q.y * D);
                S += CENTRED ? m : mn;
                ntst(&ps[nu * g.stride + a.out], mn);
            }
            const float pbar = 0.5f * (p0 + p1);
            const float rho_a = 0.5f * (r0 + a.rho[idx + o]);
            const float kap_a = 0.5f * (k0 + a.kap[idx + o]);
            float *va = a.v + ax * g.stride;
            va[idx + a.out] = va[idx] - a.dt * S / (rho_a * (1.0f + (a.nlA * kap_a) * pbar));
        }
    }
}

// ---------------------------------------------------------------------------
// 2D sweep kernels.  A block of BX threads owns BX consecutive columns and
// walks `rows` rows in +y.  Each thread keeps the 8-row window of the
// y-stencil field for its own column in registers (one new row per step);
// rows of the x-stencil field live in small LDS rings (one barrier per row),
// so every array is read from HBM once per launch apart from the short
// column halo.  Tiles are numbered so that each XCD (blocks b = k mod 8)
// takes a contiguous band of tiles, keeping halo lines in one L2.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int tile_of_block(int bid, int nblocks)
{
    if (nblocks % 8 != 0) return bid;
    return (bid % 8) * (nblocks / 8) + bid / 8;
}

// Pointers into device global memory (address space 1), so that the
// loads and stores through a rebuilt base keep the global forms.
typedef const __attribute__((address_space(1))) char *gbase;
typedef const __attribute__((address_space(1))) float *gcfloat;
typedef __attribute__((address_space(1))) float *gfloat;

template <typename T>
__device__ __forceinline__ gbase plane_base(const T *f, const Geometry &g, int z)
{
    // planes -4 .. n[2] + 3 exist (zero halo planes, or a slab's neighbour
    // planes); anything further out reads the zero corner of plane -1
    const int zz = (z >= -kHalo && z < g.n[2] + kHalo) ? z : -1;
    const uint64_t u = reinterpret_cast<uint64_t>(f + (g.origin + (int64_t)zz * g.plane - g.pitch - 1));
    // the same for every lane (z is uniform over the block): scalar registers
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return (gbase)(((uint64_t)hi << 32) | lo);
}

// Element offset of (x, y) from a plane base; outside the grid, the zero
// halo point (-1, -1) of the same plane.
__device__ __forceinline__ uint32_t plane_point(const Geometry &g, int x, int y)
{
    const bool in = (unsigned)x < (unsigned)g.n[0] && (unsigned)y < (unsigned)g.n[1];
    return in ? (uint32_t)((y + 1) * (int)g.pitch + (x + 1)) : 0u;
}

__device__ __forceinline__ gcfloat at_plane(gbase base, uint32_t pt) { return (gcfloat)(base + pt * 4u); }
__device__ __forceinline__ gfloat at_plane_w(gbase base, uint32_t pt) { return (gfloat)(base + pt * 4u); }
__device__ __forceinline__ int label_at(gbase base, uint32_t pt)
{
    return (int)((const __attribute__((address_space(1))) uint8_t *)base)[pt];
}
__device__ __forceinline__ float ntld(gcfloat p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void ntst(gfloat p, float v) { __builtin_nontemporal_store(v, p); }

// Value of a padded 2D array at (x, y): inside the grid the sample itself,
// else the halo cell (-1, -1), which is zero in every array (never written),
// so the load is branch-free.  A 2D array is one plane (z = 0).
__device__ __forceinline__ float ldz(const float *__restrict__ f, const Geometry &g, int x, int y)
{
    return *at_plane(plane_base(f, g, 0), plane_point(g, x, y));
}

// LDS hand-off between the threads of a block.  A one-wavefront block needs
// no hardware barrier (a wavefront's LDS operations complete in order); the
// fences keep the compiler from moving LDS accesses across it, and global
// loads of the next row stay in flight.
template <int BX>
__device__ __forceinline__ void lds_sync()
{
    if constexpr (BX == 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Column of halo lane t (t < 8) of a tile starting at x0: x0-4..x0-1 and
// x0+BX..x0+BX+3; its slot in an LDS row whose column c holds x0 - 4 + c.
template <int BX>
__device__ __forceinline__ int halo_x(int t, int x0) { return t < 4 ? x0 - 4 + t : x0 + BX + (t - 4); }
template <int BX>
__device__ __forceinline__ int halo_c(int t) { return t < 4 ? t : BX + t; }

template <int L>
struct PRow {                 // everything the pressure sweep loads for one row
    float vyn, vxn, hx, hy;   // window row j+3, ring row j+1, halos
    float p0, k0, q0, r0;     // r0: rho, loaded for per-point weights only
    int l;
    float m[2][L];
};

template <int L, int BX, bool PP>
__device__ __forceinline__ void p_load_row(PRow<L> &r, const StepArgs &a, int i, int t, int x0, int j, bool live)
{
    const Geometry &g = a.geo;
    const float *__restrict__ vx = a.v;
    const float *__restrict__ vy = a.v + g.stride;
    r.vyn = ldz(vy, g, i, j + 3);
    r.vxn = ldz(vx, g, i, j + 1);
    r.hx = t < 8 ? ldz(vx, g, halo_x<BX>(t, x0), j + 1) : 0.0f;
    r.hy = t < 2 ? ldz(vy, g, t == 0 ? x0 - 1 : x0 + BX, j) : 0.0f;
    const uint32_t pt = plane_point(g, i, j);
    if (live) {
        r.p0 = *at_plane(plane_base(a.p, g, 0), pt);
        r.k0 = *at_plane(plane_base(a.kap, g, 0), pt);
        r.q0 = *at_plane(plane_base(a.nlq, g, 0), pt);
        r.r0 = PP ? *at_plane(plane_base(a.rho, g, 0), pt) : 1.0f;
        r.l = a.label ? label_at(plane_base(a.label, g, 0), pt) : 0;
#pragma unroll
        for (int ax = 0; ax < 2; ++ax)
#pragma unroll
            for (int nu = 0; nu < L; ++nu)
                r.m[ax][nu] = ntld(at_plane(plane_base(a.psi2 + (int64_t)(ax * L + nu) * g.stride, g, 0), pt));
    }
}

// One tile (columns x0..x0+BX-1, rows y0..y0+rows-1) of the 2D pressure
// sweep; sx / sy are the block's LDS rings.
template <int L, bool CENTRED, int BX, bool PF, bool PP>
__device__ __forceinline__ void pressure_tile2d(const StepArgs &a, int rows, int x0, int y0,
                                                float (*sx)[BX + 8], float (*sy)[BX + 2])
{
    const Geometry &g = a.geo;
    const int t = threadIdx.x;
    const int i = x0 + t;
    const int nx = g.n[0], ny = g.n[1];
    const bool live = i < nx;
    const float *__restrict__ vx = a.v;
    const float *__restrict__ vy = a.v + g.stride;
    float *__restrict__ pp = a.p + a.out;        // written only
    float *__restrict__ psi = a.psi2 + a.out;

    // prologue: window rows y0-4 .. y0+2, rings rows y0-1 and y0
    float w[8];
    w[0] = 0.0f;
#pragma unroll
    for (int k = 1; k < 8; ++k) w[k] = ldz(vy, g, i, y0 - 5 + k);
#pragma unroll
    for (int r = -1; r <= 0; ++r) {
        sx[(y0 + r) & 3][t + 4] = ldz(vx, g, i, y0 + r);
        if (t < 8) sx[(y0 + r) & 3][halo_c<BX>(t)] = ldz(vx, g, halo_x<BX>(t, x0), y0 + r);
    }
    sy[(y0 + 2) % 3][t + 1] = ldz(vy, g, i, y0 - 1);
    if (t < 2) sy[(y0 + 2) % 3][t == 0 ? 0 : BX + 1] = ldz(vy, g, t == 0 ? x0 - 1 : x0 + BX, y0 - 1);

    const int sxs = max(max(a.nb[0] - i, i - (nx - 1 - a.nb[0])), 0);
    const int yend = min(y0 + rows, ny);
    PRow<L> cur, nxt;
    if (PF) p_load_row<L, BX, PP>(cur, a, i, t, x0, y0, live);
    for (int j = y0; j < yend; ++j) {
        if (!PF) p_load_row<L, BX, PP>(cur, a, i, t, x0, j, live);        // rows loaded in turn
        else if (j + 1 < yend) p_load_row<L, BX, PP>(nxt, a, i, t, x0, j + 1, live);   // next row in flight
#pragma unroll
        for (int k = 0; k < 7; ++k) w[k] = w[k + 1];
        w[7] = cur.vyn;
        sx[(j + 1) & 3][t + 4] = cur.vxn;
        if (t < 8) sx[(j + 1) & 3][halo_c<BX>(t)] = cur.hx;
        sy[j % 3][t + 1] = w[4];
        if (t < 2) sy[j % 3][t == 0 ? 0 : BX + 1] = cur.hy;
        lds_sync<BX>();
        if (live) {
            const Wts W = weights<PP>(a, PP ? cell_r2(a, cur.r0, cur.k0) : 0.0f);
            const float *r0 = sx[j & 3], *rp = sx[(j + 1) & 3], *rm = sx[(j + 3) & 3];
            float Dx = W.g0 * (r0[t + 4] - r0[t + 3]);
            Dx = fmaf(W.g1, r0[t + 5] - r0[t + 2], Dx);
            Dx = fmaf(W.g2, r0[t + 6] - r0[t + 1], Dx);
            Dx = fmaf(W.g3, r0[t + 7] - r0[t], Dx);
            Dx = fmaf(W.g11, (rp[t + 4] - rp[t + 3]) + (rm[t + 4] - rm[t + 3]), Dx);
            const float *c0 = sy[j % 3], *cm = sy[(j + 2) % 3];
            float Dy = W.g0 * (w[4] - w[3]);
            Dy = fmaf(W.g1, w[5] - w[2], Dy);
            Dy = fmaf(W.g2, w[6] - w[1], Dy);
            Dy = fmaf(W.g3, w[7] - w[0], Dy);
            Dy = fmaf(W.g11, (c0[t + 2] - cm[t + 2]) + (c0[t] - cm[t]), Dy);
            const int sys = max(max(a.nb[1] - j, j - (ny - 1 - a.nb[1])), 0);
            float S = 0.0f;
#pragma unroll
            for (int ax = 0; ax < 2; ++ax) {
                const float D = ax == 0 ? Dx : Dy;
                const int tt = (ax == 0 ? sxs : sys) * a.n_labels + cur.l;
                const float2 *__restrict__ bc = a.bc2[ax] + (int64_t)tt * L;
                float Sa = a.w2[ax][tt] * D;
#pragma unroll
                for (int nu = 0; nu < L; ++nu) {
                    const float2 q = bc[nu];
                    const float mn = fmaf(q.x, cur.m[ax][nu], q.y * D);
                    Sa += CENTRED ? cur.m[ax][nu] : mn;
                    cur.m[ax][nu] = mn;
                }
                S += Sa;
            }
            const uint32_t pt = plane_point(g, i, j);
            const float kappa = cur.k0 * (1.0f + cur.q0 * cur.p0);
            *at_plane_w(plane_base(pp, g, 0), pt) = cur.p0 - a.dt * S / kappa;
#pragma unroll
            for (int ax = 0; ax < 2; ++ax)
#pragma unroll
                for (int nu = 0; nu < L; ++nu)
                    ntst(at_plane_w(plane_base(psi + (int64_t)(ax * L + nu) * g.stride, g, 0), pt), cur.m[ax][nu]);
        }
        if (PF) cur = nxt;
    }
}

template <int L>
struct VRow {                 // everything the velocity sweep loads for one row
    float pn, rn, kn, hp, hr, hk;   // window row j+4, rho/kappa0 row j+1, halos
    float ux, uy;
    int l;
    float m[2][L];
};

template <int L, int BX>
__device__ __forceinline__ void v_load_row(VRow<L> &r, const StepArgs &a, int i, int t, int x0, int j, bool live)
{
    const Geometry &g = a.geo;
    r.pn = ldz(a.p, g, i, j + 4);
    r.rn = ldz(a.rho, g, i, j + 1);
    r.kn = ldz(a.kap, g, i, j + 1);
    r.hp = t < 8 ? ldz(a.p, g, halo_x<BX>(t, x0), j + 1) : 0.0f;
    r.hr = t == 0 ? ldz(a.rho, g, x0 + BX, j + 1) : 0.0f;
    r.hk = t == 0 ? ldz(a.kap, g, x0 + BX, j + 1) : 0.0f;
    const uint32_t pt = plane_point(g, i, j);
    if (live) {
        r.ux = *at_plane(plane_base(a.v, g, 0), pt);
        r.uy = *at_plane(plane_base(a.v + g.stride, g, 0), pt);
        r.l = a.label ? label_at(plane_base(a.label, g, 0), pt) : 0;
#pragma unroll
        for (int ax = 0; ax < 2; ++ax)
#pragma unroll
            for (int nu = 0; nu < L; ++nu)
                r.m[ax][nu] = ntld(at_plane(plane_base(a.psi1 + (int64_t)(ax * L + nu) * g.stride, g, 0), pt));
    }
}

// One tile of the 2D velocity sweep; sp / sr / sk are the block's LDS rings.
template <int L, bool CENTRED, int BX, bool PF, bool PP>
__device__ __forceinline__ void velocity_tile2d(const StepArgs &a, int rows, int x0, int y0,
                                                float (*sp)[BX + 8], float (*sr)[BX + 1], float (*sk)[BX + 1])
{
    const Geometry &g = a.geo;
    const int t = threadIdx.x;
    const int i = x0 + t;
    const int nx = g.n[0], ny = g.n[1];
    const bool live = i < nx;
    const float *__restrict__ pp = a.p;
    float *__restrict__ vx = a.v + a.out;        // written only
    float *__restrict__ vy = a.v + g.stride + a.out;
    float *__restrict__ psi = a.psi1 + a.out;

    // prologue: window rows y0-3 .. y0+3; p ring rows y0-1, y0; rho/kappa row y0
    float w[8];
    w[0] = 0.0f;
#pragma unroll
    for (int k = 1; k < 8; ++k) w[k] = ldz(pp, g, i, y0 - 4 + k);
#pragma unroll
    for (int r = -1; r <= 0; ++r) {
        sp[(y0 + r) & 3][t + 4] = ldz(pp, g, i, y0 + r);
        if (t < 8) sp[(y0 + r) & 3][halo_c<BX>(t)] = ldz(pp, g, halo_x<BX>(t, x0), y0 + r);
    }
    sr[y0 % 3][t] = ldz(a.rho, g, i, y0);
    sk[y0 % 3][t] = ldz(a.kap, g, i, y0);
    if (t == 0) {
        sr[y0 % 3][BX] = ldz(a.rho, g, x0 + BX, y0);
        sk[y0 % 3][BX] = ldz(a.kap, g, x0 + BX, y0);
    }

    const int sxs = max(max(a.nb[0] - i, i - (nx - 2 - a.nb[0])), 0);
    const int yend = min(y0 + rows, ny);
    VRow<L> cur, nxt;
    if (PF) v_load_row<L, BX>(cur, a, i, t, x0, y0, live);
    for (int j = y0; j < yend; ++j) {
        if (!PF) v_load_row<L, BX>(cur, a, i, t, x0, j, live);
        else if (j + 1 < yend) v_load_row<L, BX>(nxt, a, i, t, x0, j + 1, live);
#pragma unroll
        for (int k = 0; k < 7; ++k) w[k] = w[k + 1];
        w[7] = cur.pn;
        sp[(j + 1) & 3][t + 4] = w[4];
        if (t < 8) sp[(j + 1) & 3][halo_c<BX>(t)] = cur.hp;
        sr[(j + 1) % 3][t] = cur.rn;
        sk[(j + 1) % 3][t] = cur.kn;
        if (t == 0) {
            sr[(j + 1) % 3][BX] = cur.hr;
            sk[(j + 1) % 3][BX] = cur.hk;
        }
        lds_sync<BX>();
        if (live) {
            const uint32_t pt = plane_point(g, i, j);
            const float *r0 = sp[j & 3], *rp = sp[(j + 1) & 3], *rm = sp[(j + 3) & 3];
            const float *rr0 = sr[j % 3], *kk0 = sk[j % 3];
            const float s0 = PP ? cell_r2(a, rr0[t], kk0[t]) : 0.0f;
            // v_x at (i + 1/2, j)
            if (i < nx - 1) {
                const Wts W = weights<PP>(a, PP ? 0.5f * (s0 + cell_r2(a, rr0[t + 1], kk0[t + 1])) : 0.0f);
                float D = W.g0 * (r0[t + 5] - r0[t + 4]);
                D = fmaf(W.g1, r0[t + 6] - r0[t + 3], D);
                D = fmaf(W.g2, r0[t + 7] - r0[t + 2], D);
                D = fmaf(W.g3, r0[t + 8] - r0[t + 1], D);
                D = fmaf(W.g11, (rp[t + 5] - rp[t + 4]) + (rm[t + 5] - rm[t + 4]), D);
                const int tt = sxs * a.n_labels + cur.l;
                const float2 *__restrict__ bc = a.bc1[0] + (int64_t)tt * L;
                float S = a.w1[0][tt] * D;
#pragma unroll
                for (int nu = 0; nu < L; ++nu) {
                    const float2 q = bc[nu];
                    const float mn = fmaf(q.x, cur.m[0][nu], q.y * D);
                    S += CENTRED ? cur.m[0][nu] : mn;
                    cur.m[0][nu] = mn;
                }
                const float pbar = 0.5f * (r0[t + 4] + r0[t + 5]);
                const float rho_a = 0.5f * (rr0[t] + rr0[t + 1]);
                const float kap_a = 0.5f * (kk0[t] + kk0[t + 1]);
                *at_plane_w(plane_base(vx, g, 0), pt) =
                    cur.ux - a.dt * S / (rho_a * (1.0f + (a.nlA * kap_a) * pbar));
#pragma unroll
                for (int nu = 0; nu < L; ++nu)
                    ntst(at_plane_w(plane_base(psi + (int64_t)nu * g.stride, g, 0), pt), cur.m[0][nu]);
            }
            // v_y at (i, j + 1/2)
            if (j < ny - 1) {
                const int sys = max(max(a.nb[1] - j, j - (ny - 2 - a.nb[1])), 0);
                const Wts W = weights<PP>(
                    a, PP ? 0.5f * (s0 + cell_r2(a, sr[(j + 1) % 3][t], sk[(j + 1) % 3][t])) : 0.0f);
                float D = W.g0 * (w[4] - w[3]);
                D = fmaf(W.g1, w[5] - w[2], D);
                D = fmaf(W.g2, w[6] - w[1], D);
                D = fmaf(W.g3, w[7] - w[0], D);
                D = fmaf(W.g11, (rp[t + 5] - r0[t + 5]) + (rp[t + 3] - r0[t + 3]), D);
                const int tt = sys * a.n_labels + cur.l;
                const float2 *__restrict__ bc = a.bc1[1] + (int64_t)tt * L;
                float S = a.w1[1][tt] * D;
#pragma unroll
                for (int nu = 0; nu < L; ++nu) {
                    const float2 q = bc[nu];
                    const float mn = fmaf(q.x, cur.m[1][nu], q.y * D);
                    S += CENTRED ? cur.m[1][nu] : mn;
                    cur.m[1][nu] = mn;
                }
                const float pbar = 0.5f * (w[3] + w[4]);
                const float rho_a = 0.5f * (rr0[t] + sr[(j + 1) % 3][t]);
                const float kap_a = 0.5f * (kk0[t] + sk[(j + 1) % 3][t]);
                *at_plane_w(plane_base(vy, g, 0), pt) =
                    cur.uy - a.dt * S / (rho_a * (1.0f + (a.nlA * kap_a) * pbar));
#pragma unroll
                for (int nu = 0; nu < L; ++nu)
                    ntst(at_plane_w(plane_base(psi + (int64_t)(L + nu) * g.stride, g, 0), pt), cur.m[1][nu]);
            }
        }
        if (PF) cur = nxt;
    }
}

template <int L, bool CENTRED, int BX, bool PF, bool PP>
__global__ void __launch_bounds__(BX) pressure_sweep2d(const StepArgs a, int rows, int nbx, int nblocks)
{
    __shared__ float sx[4][BX + 8];     // v_x rows, column c <-> x0 - 4 + c
    __shared__ float sy[3][BX + 2];     // v_y rows, column c <-> x0 - 1 + c
    const int tile = tile_of_block(blockIdx.x, nblocks);
    pressure_tile2d<L, CENTRED, BX, PF, PP>(a, rows, (tile % nbx) * BX, (tile / nbx) * rows, sx, sy);
}

// Padded element offset of a flat unpadded index x + nx (y + ny z).
__device__ __forceinline__ int64_t padded_index(const Geometry &g, int64_t f)
{
    const int64_t x = f % g.n[0];
    const int64_t t = f / g.n[0];
    const int64_t y = t % g.n[1];
    const int64_t z = t / g.n[1];
    return g.origin + z * g.plane + y * g.pitch + x;
}

// The receivers of the current step, recorded by one whole block, then the
// device step counter advanced (one block, so no other block reads the
// counter meanwhile).
__device__ __forceinline__ void record_receivers(const SparseArgs &s)
{
    const long long step = *s.step;
    if (step < s.cap)
        for (int r = threadIdx.x; r < s.n; r += blockDim.x)
            s.trace[step * s.n + r] = s.p[padded_index(s.geo, s.idx[r])];
    __syncthreads();
    if (threadIdx.x == 0) s.step[0] = step + 1;
}

template <int L, bool CENTRED, int BX, bool PF, bool PP>
__global__ void __launch_bounds__(BX) velocity_sweep2d(const StepArgs a, int rows, int nbx, int nblocks)
{
    // with receivers, block 0 records them (dispatched first, it overlaps the
    // tiles instead of trailing them) and blocks 1.. take the tiles
    const int shift = a.rcv.step ? 1 : 0;
    if ((int)blockIdx.x < shift) {
        record_receivers(a.rcv);
        return;
    }
    __shared__ float sp[4][BX + 8];     // p rows, column c <-> x0 - 4 + c
    __shared__ float sr[3][BX + 1];     // rho rows, column c <-> x0 + c
    __shared__ float sk[3][BX + 1];     // kappa0 rows
    const int tile = tile_of_block((int)blockIdx.x - shift, nblocks);
    velocity_tile2d<L, CENTRED, BX, PF, PP>(a, rows, (tile % nbx) * BX, (tile / nbx) * rows, sp, sr, sk);
}

// ---------------------------------------------------------------------------
// 3D sweep kernels.  A block of BX x BY threads owns a BX x BY column tile
// and walks `rows` planes in +z.  The z-stencil field of each column sits in
// an 8-plane register window; planes of the x/y-stencil fields (with their
// halos) are staged cooperatively into LDS rings, one barrier per plane.
// ---------------------------------------------------------------------------

// 3D arrays are several GB, so a per-lane element index needs 64 bits, and
// a 64-bit address per lane and array costs two VGPRs each.  The 3D sweeps
// instead address one plane at a time: a base that is uniform over the block
// (scalar registers; the array, the plane and the (-1, -1) corner folded in)
// plus a 32-bit per-lane byte offset within the plane, the scalar-base form
// of the global loads and stores.  A plane holds fewer than 2^29 points
// (checked when the domain is created), so the offsets fit.
__device__ __forceinline__ float ldz3(const float *__restrict__ f, const Geometry &g, int x, int y, int z)
{
    return *at_plane(plane_base(f, g, z), plane_point(g, x, y));
}

// Stage the (H x W) window of plane z whose (0, 0) is (xs, ys) into LDS.
template <int W, int H, int NT>
__device__ __forceinline__ void stage(float *dst, const float *__restrict__ f, const Geometry &g, int xs, int ys,
                                      int z, int tid)
{
#pragma unroll
    for (int e = tid; e < W * H; e += NT) {
        const int r = e / W, c = e - r * W;
        dst[e] = ldz3(f, g, xs + c, ys + r, z);
    }
}

// The same staging in two halves, for prefetching: the elements a thread
// stages (e = tid + q NT) are loaded into registers one plane ahead and
// stored into LDS in the next iteration.
template <int W, int H, int NT>
struct Staged {
    static constexpr int N = (W * H + NT - 1) / NT;
    float r[N];
};

template <int W, int H, int NT>
__device__ __forceinline__ void stage_load(Staged<W, H, NT> &s, const float *__restrict__ f, const Geometry &g,
                                           int xs, int ys, int z, int tid)
{
#pragma unroll
    for (int q = 0; q < Staged<W, H, NT>::N; ++q) {
        const int e = tid + q * NT;
        if (e < W * H) {
            const int r = e / W, c = e - r * W;
            s.r[q] = ldz3(f, g, xs + c, ys + r, z);
        }
    }
}

template <int W, int H, int NT>
__device__ __forceinline__ void stage_store(float *dst, const Staged<W, H, NT> &s, int tid)
{
#pragma unroll
    for (int q = 0; q < Staged<W, H, NT>::N; ++q) {
        const int e = tid + q * NT;
        if (e < W * H) dst[e] = s.r[q];
    }
}

// PF: 0 -- every plane's loads issued in its own iteration; 1 -- all loads
// of plane k + 1 issued during plane k; 2 -- only the staged planes and the
// z window one plane ahead, the point's own values (medium, memory
// variables) issued at the top of their own plane (fewer registers).
template <int L, bool CENTRED, int BX, int BY, bool PP, int PF>
__global__ void __launch_bounds__(BX *BY) pressure_sweep3d(const StepArgs a, int rows, int nbx, int nby, int nblocks)
{
    constexpr int NT = BX * BY;
    constexpr int XW = BX + 8, XH = BY + 2;     // v_x tile: x halo 4, y halo 1
    constexpr int YW = BX + 2, YH = BY + 8;     // v_y tile: x halo 1, y halo 4
    constexpr int ZW = BX + 2, ZH = BY + 2;     // v_z tile: halo 1
    const Geometry &g = a.geo;
    const int tile = tile_of_block(blockIdx.x, nblocks);
    const int tx_ = tile % nbx, rest = tile / nbx;
    const int x0 = tx_ * BX, y0 = (rest % nby) * BY, z0 = (rest / nby) * rows;
    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int i = x0 + tx, j = y0 + ty;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const bool live = i < nx && j < ny;
    const uint32_t pt = plane_point(g, i, j);      // own point in its plane
    const float *__restrict__ vx = a.v;
    const float *__restrict__ vy = a.v + g.stride;
    const float *__restrict__ vz = a.v + 2 * g.stride;

    __shared__ float sx[4][XH * XW];
    __shared__ float sy[4][YH * YW];
    __shared__ float sz[3][ZH * ZW];

    float w[8];
    w[0] = 0.0f;
#pragma unroll
    for (int q = 1; q < 8; ++q) w[q] = ldz3(vz, g, i, j, z0 - 5 + q);
#pragma unroll
    for (int r = -1; r <= 0; ++r) {
        stage<XW, XH, NT>(sx[(z0 + r) & 3], vx, g, x0 - 4, y0 - 1, z0 + r, tid);
        stage<YW, YH, NT>(sy[(z0 + r) & 3], vy, g, x0 - 1, y0 - 4, z0 + r, tid);
    }
    stage<ZW, ZH, NT>(sz[(z0 + 2) % 3], vz, g, x0 - 1, y0 - 1, z0 - 1, tid);

    const int s0 = max(max(a.nb[0] - i, i - (nx - 1 - a.nb[0])), 0);
    const int s1 = max(max(a.nb[1] - j, j - (ny - 1 - a.nb[1])), 0);
    const int zend = min(z0 + rows, nz);
    // what one plane k needs from global memory besides the staged planes
    struct Own {
        float vzn, p0, k0, q0, r0;
        int l;
        float m[3][L];
    };
    auto load_zwin = [&](Own &o, int k) { o.vzn = ldz3(vz, g, i, j, k + 3); };
    auto load_point = [&](Own &o, int k) {
        o.p0 = 0.0f;
        o.k0 = 1.0f;
        o.q0 = 0.0f;
        o.r0 = 1.0f;
        o.l = 0;
        if (live && k < nz) {
            o.p0 = *at_plane(plane_base(a.p, g, k), pt);
            o.k0 = *at_plane(plane_base(a.kap, g, k), pt);
            o.q0 = *at_plane(plane_base(a.nlq, g, k), pt);
            if (PP) o.r0 = *at_plane(plane_base(a.rho, g, k), pt);
            o.l = a.label ? label_at(plane_base(a.label, g, k), pt) : 0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
#pragma unroll
                for (int nu = 0; nu < L; ++nu)
                    o.m[ax][nu] = ntld(at_plane(plane_base(a.psi2 + (int64_t)(ax * L + nu) * g.stride, g, k), pt));
        }
    };
    auto load_own = [&](Own &o, int k) {
        load_zwin(o, k);
        load_point(o, k);
    };
    Staged<XW, XH, NT> px;
    Staged<YW, YH, NT> py;
    Staged<ZW, ZH, NT> pz;
    Own cur;
    if (PF) {                                   // plane z0: staged x/y planes z0 + 1, z plane z0
        stage_load<XW, XH, NT>(px, vx, g, x0 - 4, y0 - 1, z0 + 1, tid);
        stage_load<YW, YH, NT>(py, vy, g, x0 - 1, y0 - 4, z0 + 1, tid);
        stage_load<ZW, ZH, NT>(pz, vz, g, x0 - 1, y0 - 1, z0, tid);
        if (PF == 1)
            load_own(cur, z0);
        else
            load_zwin(cur, z0);
    }
    for (int k = z0; k < zend; ++k) {
        if (PF) {
            stage_store<XW, XH, NT>(sx[(k + 1) & 3], px, tid);
            stage_store<YW, YH, NT>(sy[(k + 1) & 3], py, tid);
            stage_store<ZW, ZH, NT>(sz[k % 3], pz, tid);
        } else {
            stage<XW, XH, NT>(sx[(k + 1) & 3], vx, g, x0 - 4, y0 - 1, k + 1, tid);
            stage<YW, YH, NT>(sy[(k + 1) & 3], vy, g, x0 - 1, y0 - 4, k + 1, tid);
            stage<ZW, ZH, NT>(sz[k % 3], vz, g, x0 - 1, y0 - 1, k, tid);
            load_own(cur, k);
        }
        Own o = cur;
        if (PF == 2) load_point(o, k);
        if (PF && k + 1 < zend) {               // next plane's loads in flight during this one
            stage_load<XW, XH, NT>(px, vx, g, x0 - 4, y0 - 1, k + 2, tid);
            stage_load<YW, YH, NT>(py, vy, g, x0 - 1, y0 - 4, k + 2, tid);
            stage_load<ZW, ZH, NT>(pz, vz, g, x0 - 1, y0 - 1, k + 1, tid);
            if (PF == 1)
                load_own(cur, k + 1);
            else
                load_zwin(cur, k + 1);
        }
        const float p0 = o.p0, k0 = o.k0, q0 = o.q0, r0 = o.r0;
        const int l = o.l;
        float m[3][L];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
#pragma unroll
            for (int nu = 0; nu < L; ++nu) m[ax][nu] = o.m[ax][nu];
#pragma unroll
        for (int q = 0; q < 7; ++q) w[q] = w[q + 1];
        w[7] = o.vzn;
        __syncthreads();
        if (live) {
            const Wts W = weights<PP>(a, PP ? cell_r2(a, r0, k0) : 0.0f);
            const float *X0 = sx[k & 3], *Xp = sx[(k + 1) & 3], *Xm = sx[(k + 3) & 3];
            const int cx = (ty + 1) * XW + tx + 4;          // own sample in the v_x tile
            float Dx = W.g0 * (X0[cx] - X0[cx - 1]);
            Dx = fmaf(W.g1, X0[cx + 1] - X0[cx - 2], Dx);
            Dx = fmaf(W.g2, X0[cx + 2] - X0[cx - 3], Dx);
            Dx = fmaf(W.g3, X0[cx + 3] - X0[cx - 4], Dx);
            Dx = fmaf(W.g11, ((X0[cx + XW] - X0[cx + XW - 1]) + (X0[cx - XW] - X0[cx - XW - 1])) +
                                 ((Xp[cx] - Xp[cx - 1]) + (Xm[cx] - Xm[cx - 1])), Dx);
            const float *Y0 = sy[k & 3], *Yp = sy[(k + 1) & 3], *Ym = sy[(k + 3) & 3];
            const int cy = (ty + 4) * YW + tx + 1;
            float Dy = W.g0 * (Y0[cy] - Y0[cy - YW]);
            Dy = fmaf(W.g1, Y0[cy + YW] - Y0[cy - 2 * YW], Dy);
            Dy = fmaf(W.g2, Y0[cy + 2 * YW] - Y0[cy - 3 * YW], Dy);
            Dy = fmaf(W.g3, Y0[cy + 3 * YW] - Y0[cy - 4 * YW], Dy);
            Dy = fmaf(W.g11, ((Y0[cy + 1] - Y0[cy + 1 - YW]) + (Y0[cy - 1] - Y0[cy - 1 - YW])) +
                                 ((Yp[cy] - Yp[cy - YW]) + (Ym[cy] - Ym[cy - YW])), Dy);
            const float *Z0 = sz[k % 3], *Zm = sz[(k + 2) % 3];
            const int cz = (ty + 1) * ZW + tx + 1;
            float Dz = W.g0 * (w[4] - w[3]);
            Dz = fmaf(W.g1, w[5] - w[2], Dz);
            Dz = fmaf(W.g2, w[6] - w[1], Dz);
            Dz = fmaf(W.g3, w[7] - w[0], Dz);
            Dz = fmaf(W.g11, ((Z0[cz + 1] - Zm[cz + 1]) + (Z0[cz - 1] - Zm[cz - 1])) +
                                 ((Z0[cz + ZW] - Zm[cz + ZW]) + (Z0[cz - ZW] - Zm[cz - ZW])), Dz);
            const int kg = k + a.z_off, s2 = max(max(a.nb[2] - kg, kg - (a.nz_glob - 1 - a.nb[2])), 0);
            float S = 0.0f;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const float D = ax == 0 ? Dx : (ax == 1 ? Dy : Dz);
                const int tt = (ax == 0 ? s0 : (ax == 1 ? s1 : s2)) * a.n_labels + l;
                const float2 *__restrict__ bc = a.bc2[ax] + (int64_t)tt * L;
                float Sa = a.w2[ax][tt] * D;
#pragma unroll
                for (int nu = 0; nu < L; ++nu) {
                    const float2 q = bc[nu];
                    const float mn = fmaf(q.x, m[ax][nu], q.y * D);
                    Sa += CENTRED ? m[ax][nu] : mn;
                    m[ax][nu] = mn;
                }
                S += Sa;
            }
            const float kappa = k0 * (1.0f + q0 * p0);
            *at_plane_w(plane_base(a.p + a.out, g, k), pt) = p0 - a.dt * S / kappa;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
#pragma unroll
                for (int nu = 0; nu < L; ++nu)
                    ntst(at_plane_w(plane_base(a.psi2 + a.out + (int64_t)(ax * L + nu) * g.stride, g, k), pt), m[ax][nu]);
        }
    }
}

template <int L, bool CENTRED, int BX, int BY, bool PP, int PF>
__global__ void __launch_bounds__(BX *BY) velocity_sweep3d(const StepArgs a, int rows, int nbx, int nby, int nblocks)
{
    // with receivers, block 0 records them and blocks 1.. take the tiles
    const int shift = a.rcv.step ? 1 : 0;
    if ((int)blockIdx.x < shift) {
        record_receivers(a.rcv);
        return;
    }
    constexpr int NT = BX * BY;
    constexpr int PW = BX + 8, PH = BY + 8;     // p tile: halo 4 (x0-4.., y0-4..)
    constexpr int RW = BX + 1, RH = BY + 1;     // rho / kappa0 tiles: +1 halo
    const Geometry &g = a.geo;
    const int tile = tile_of_block((int)blockIdx.x - shift, nblocks);
    const int tx_ = tile % nbx, rest = tile / nbx;
    const int x0 = tx_ * BX, y0 = (rest % nby) * BY, z0 = (rest / nby) * rows;
    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int i = x0 + tx, j = y0 + ty;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const bool live = i < nx && j < ny;
    const uint32_t pt = plane_point(g, i, j);      // own point in its plane
    const float *__restrict__ pp = a.p;

    __shared__ float sp[4][PH * PW];
    __shared__ float sr[3][RH * RW];
    __shared__ float sk[3][RH * RW];

    float w[8];
    w[0] = 0.0f;
#pragma unroll
    for (int q = 1; q < 8; ++q) w[q] = ldz3(pp, g, i, j, z0 - 4 + q);
#pragma unroll
    for (int r = -1; r <= 0; ++r) stage<PW, PH, NT>(sp[(z0 + r) & 3], pp, g, x0 - 4, y0 - 4, z0 + r, tid);
    stage<RW, RH, NT>(sr[z0 % 3], a.rho, g, x0, y0, z0, tid);
    stage<RW, RH, NT>(sk[z0 % 3], a.kap, g, x0, y0, z0, tid);

    const int s0 = max(max(a.nb[0] - i, i - (nx - 2 - a.nb[0])), 0);
    const int s1 = max(max(a.nb[1] - j, j - (ny - 2 - a.nb[1])), 0);
    const int zend = min(z0 + rows, nz);
    struct Own {
        float pn, u[3];
        int l;
        float m[3][L];
    };
    auto load_zwin = [&](Own &o, int k) { o.pn = ldz3(pp, g, i, j, k + 4); };
    auto load_point = [&](Own &o, int k) {
        o.u[0] = o.u[1] = o.u[2] = 0.0f;
        o.l = 0;
        if (live && k < nz) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) o.u[ax] = *at_plane(plane_base(a.v + (int64_t)ax * g.stride, g, k), pt);
            o.l = a.label ? label_at(plane_base(a.label, g, k), pt) : 0;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax)
#pragma unroll
                for (int nu = 0; nu < L; ++nu)
                    o.m[ax][nu] = ntld(at_plane(plane_base(a.psi1 + (int64_t)(ax * L + nu) * g.stride, g, k), pt));
        }
    };
    auto load_own = [&](Own &o, int k) {
        load_zwin(o, k);
        load_point(o, k);
    };
    Staged<PW, PH, NT> ps;
    Staged<RW, RH, NT> rs, ks;
    Own cur;
    if (PF) {
        stage_load<PW, PH, NT>(ps, pp, g, x0 - 4, y0 - 4, z0 + 1, tid);
        stage_load<RW, RH, NT>(rs, a.rho, g, x0, y0, z0 + 1, tid);
        stage_load<RW, RH, NT>(ks, a.kap, g, x0, y0, z0 + 1, tid);
        if (PF == 1)
            load_own(cur, z0);
        else
            load_zwin(cur, z0);
    }
    for (int k = z0; k < zend; ++k) {
        if (PF) {
            stage_store<PW, PH, NT>(sp[(k + 1) & 3], ps, tid);
            stage_store<RW, RH, NT>(sr[(k + 1) % 3], rs, tid);
            stage_store<RW, RH, NT>(sk[(k + 1) % 3], ks, tid);
        } else {
            stage<PW, PH, NT>(sp[(k + 1) & 3], pp, g, x0 - 4, y0 - 4, k + 1, tid);
            stage<RW, RH, NT>(sr[(k + 1) % 3], a.rho, g, x0, y0, k + 1, tid);
            stage<RW, RH, NT>(sk[(k + 1) % 3], a.kap, g, x0, y0, k + 1, tid);
            load_own(cur, k);
        }
        Own o = cur;
        if (PF == 2) load_point(o, k);
        if (PF && k + 1 < zend) {
            stage_load<PW, PH, NT>(ps, pp, g, x0 - 4, y0 - 4, k + 2, tid);
            stage_load<RW, RH, NT>(rs, a.rho, g, x0, y0, k + 2, tid);
            stage_load<RW, RH, NT>(ks, a.kap, g, x0, y0, k + 2, tid);
            if (PF == 1)
                load_own(cur, k + 1);
            else
                load_zwin(cur, k + 1);
        }
        const float u[3] = {o.u[0], o.u[1], o.u[2]};
        const int l = o.l;
        float m[3][L];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
#pragma unroll
            for (int nu = 0; nu < L; ++nu) m[ax][nu] = o.m[ax][nu];
#pragma unroll
        for (int q = 0; q < 7; ++q) w[q] = w[q + 1];
        w[7] = o.pn;
        __syncthreads();
        if (live) {
            const float *P0 = sp[k & 3], *Pp = sp[(k + 1) & 3], *Pm = sp[(k + 3) & 3];
            const float *R0 = sr[k % 3], *Rp = sr[(k + 1) % 3], *K0 = sk[k % 3], *Kp = sk[(k + 1) % 3];
            const int c = (ty + 4) * PW + tx + 4;           // own sample in the p tile
            const int cr = ty * RW + tx;                    // own sample in the rho tile
            const int kg = k + a.z_off, s2 = max(max(a.nb[2] - kg, kg - (a.nz_glob - 2 - a.nb[2])), 0);
            const float sc = PP ? cell_r2(a, R0[cr], K0[cr]) : 0.0f;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                if ((ax == 0 && i == nx - 1) || (ax == 1 && j == ny - 1) || (ax == 2 && kg == a.nz_glob - 1)) continue;
                float D, pbar, rho_a, kap_a;
                if (ax == 0) {
                    const Wts W = weights<PP>(a, PP ? 0.5f * (sc + cell_r2(a, R0[cr + 1], K0[cr + 1])) : 0.0f);
                    D = W.g0 * (P0[c + 1] - P0[c]);
                    D = fmaf(W.g1, P0[c + 2] - P0[c - 1], D);
                    D = fmaf(W.g2, P0[c + 3] - P0[c - 2], D);
                    D = fmaf(W.g3, P0[c + 4] - P0[c - 3], D);
                    D = fmaf(W.g11, ((P0[c + 1 + PW] - P0[c + PW]) + (P0[c + 1 - PW] - P0[c - PW])) +
                                        ((Pp[c + 1] - Pp[c]) + (Pm[c + 1] - Pm[c])), D);
                    pbar = 0.5f * (P0[c] + P0[c + 1]);
                    rho_a = 0.5f * (R0[cr] + R0[cr + 1]);
                    kap_a = 0.5f * (K0[cr] + K0[cr + 1]);
                } else if (ax == 1) {
                    const Wts W = weights<PP>(a, PP ? 0.5f * (sc + cell_r2(a, R0[cr + RW], K0[cr + RW])) : 0.0f);
                    D = W.g0 * (P0[c + PW] - P0[c]);
                    D = fmaf(W.g1, P0[c + 2 * PW] - P0[c - PW], D);
                    D = fmaf(W.g2, P0[c + 3 * PW] - P0[c - 2 * PW], D);
                    D = fmaf(W.g3, P0[c + 4 * PW] - P0[c - 3 * PW], D);
                    D = fmaf(W.g11, ((P0[c + PW + 1] - P0[c + 1]) + (P0[c + PW - 1] - P0[c - 1])) +
                                        ((Pp[c + PW] - Pp[c]) + (Pm[c + PW] - Pm[c])), D);
                    pbar = 0.5f * (P0[c] + P0[c + PW]);
                    rho_a = 0.5f * (R0[cr] + R0[cr + RW]);
                    kap_a = 0.5f * (K0[cr] + K0[cr + RW]);
                } else {
                    const Wts W = weights<PP>(a, PP ? 0.5f * (sc + cell_r2(a, Rp[cr], Kp[cr])) : 0.0f);
                    D = W.g0 * (w[4] - w[3]);
                    D = fmaf(W.g1, w[5] - w[2], D);
                    D = fmaf(W.g2, w[6] - w[1], D);
                    D = fmaf(W.g3, w[7] - w[0], D);
                    D = fmaf(W.g11, ((Pp[c + 1] - P0[c + 1]) + (Pp[c - 1] - P0[c - 1])) +
                                        ((Pp[c + PW] - P0[c + PW]) + (Pp[c - PW] - P0[c - PW])), D);
                    pbar = 0.5f * (w[3] + w[4]);
                    rho_a = 0.5f * (R0[cr] + Rp[cr]);
                    kap_a = 0.5f * (K0[cr] + Kp[cr]);
                }
                const int tt = (ax == 0 ? s0 : (ax == 1 ? s1 : s2)) * a.n_labels + l;
                const float2 *__restrict__ bc = a.bc1[ax] + (int64_t)tt * L;
                float S = a.w1[ax][tt] * D;
#pragma unroll
                for (int nu = 0; nu < L; ++nu) {
                    const float2 q = bc[nu];
                    const float mn = fmaf(q.x, m[ax][nu], q.y * D);
                    S += CENTRED ? m[ax][nu] : mn;
                    m[ax][nu] = mn;
                }
                *at_plane_w(plane_base(a.v + a.out + (int64_t)ax * g.stride, g, k), pt) =
                    u[ax] - a.dt * S / (rho_a * (1.0f + (a.nlA * kap_a) * pbar));
#pragma unroll
                for (int nu = 0; nu < L; ++nu)
                    ntst(at_plane_w(plane_base(a.psi1 + a.out + (int64_t)(ax * L + nu) * g.stride, g, k), pt), m[ax][nu]);
            }
        }
    }
}

template <int L, bool C, bool PF, bool PP>
hipError_t launch_sweep(const StepArgs &a, bool pressure, const KernelConfig &kc, hipStream_t st)
{
    const int nbx = (a.geo.n[0] + kc.bx - 1) / kc.bx;
    const int nby = (a.geo.n[1] + kc.rows - 1) / kc.rows;
    const int nblocks = nbx * nby;
#define FW2_SWEEP(BXV)                                                                                  \
    if constexpr (L <= 4 || BXV == 256)                                                                 \
    if (kc.bx == BXV) {                                                                                 \
        if (pressure)                                                                                   \
            hipLaunchKernelGGL((pressure_sweep2d<L, C, BXV, PF, PP>), dim3(nblocks), dim3(BXV), 0, st, a, kc.rows, nbx, nblocks); \
        else                                                                                            \
            hipLaunchKernelGGL((velocity_sweep2d<L, C, BXV, PF, PP>), dim3(nblocks + (a.rcv.step ? 1 : 0)), dim3(BXV), 0, st, \
                               a, kc.rows, nbx, nblocks);                                                  \
        return hipGetLastError();                                                                       \
    }
    FW2_SWEEP(64)
    FW2_SWEEP(128)
    FW2_SWEEP(256)
#undef FW2_SWEEP
    return hipErrorInvalidValue;
}

template <int L, bool C, bool PP, int PF>
hipError_t launch_sweep3(const StepArgs &a, bool pressure, const KernelConfig &kc, hipStream_t st)
{
    // tile BX x BY: kc.bx selects 16 x 16, 32 x 16 or 64 x 8 (kc.by = 0), or
    // with kc.by the 256-thread tiles 64 x 4 and 32 x 8 (variant 3 only)
#define FW2_SWEEP3(BXV, BYV, COND)                                                                      \
    if constexpr (COND)                                                                                 \
    if (kc.bx == BXV && (kc.by == 0 ? (BYV == (BXV == 64 ? 8 : 16)) : kc.by == BYV)) {                  \
        const int nbx = (a.geo.n[0] + BXV - 1) / BXV, nby = (a.geo.n[1] + BYV - 1) / BYV;                \
        const int nbz = (a.geo.n[2] + kc.rows - 1) / kc.rows;                                           \
        const int nblocks = nbx * nby * nbz;                                                            \
        if (pressure)                                                                                   \
            hipLaunchKernelGGL((pressure_sweep3d<L, C, BXV, BYV, PP, PF>), dim3(nblocks), dim3(BXV * BYV), 0, st, \
                               a, kc.rows, nbx, nby, nblocks);                                          \
        else                                                                                            \
            hipLaunchKernelGGL((velocity_sweep3d<L, C, BXV, BYV, PP, PF>), dim3(nblocks + (a.rcv.step ? 1 : 0)),   \
                               dim3(BXV * BYV), 0, st,                                                  \
                               a, kc.rows, nbx, nby, nblocks);                                          \
        return hipGetLastError();                                                                       \
    }
    FW2_SWEEP3(32, 16, L <= 4)
    FW2_SWEEP3(64, 8, true)
    FW2_SWEEP3(16, 16, L <= 4)
    FW2_SWEEP3(64, 4, L <= 4 && PF == 2)
    FW2_SWEEP3(32, 8, L <= 4 && PF == 2)
#undef FW2_SWEEP3
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Batched 2D step: the same per-tile code as the single-domain sweeps, over
// the tiles of every entry of a device table.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int batch_entry_of_tile(const BatchTable *__restrict__ T, int t)
{
    int d = 0;
    for (int k = 1; k < T->n; ++k)
        if (T->e[k].tile_base <= t) d = k;
    return d;
}

// One tile of one batch entry with the single-domain sweep's per-tile code.
template <bool PRESSURE, int BX, int L, bool C, bool PP>
__device__ __forceinline__ void batch_tile(const StepArgs &sa, int rows, int x0, int y0, float (*r0)[BX + 8],
                                           float (*r1)[BX + 2], float (*r2)[BX + 1])
{
    if (PRESSURE)
        pressure_tile2d<L, C, BX, false, PP>(sa, rows, x0, y0, r0, r1);
    else
        velocity_tile2d<L, C, BX, false, PP>(sa, rows, x0, y0, r0, r2, reinterpret_cast<float(*)[BX + 1]>(&r1[0][0]));
}

// Mechanism counts L0 .. L0 + 3 and both memory-variable schemes:
// key = (L - L0) * 2 + scheme.
template <bool PRESSURE, int BX, int L0, bool PP>
__device__ __forceinline__ void batch_dispatch(int key, const StepArgs &sa, int rows, int x0, int y0,
                                               float (*r0)[BX + 8], float (*r1)[BX + 2], float (*r2)[BX + 1])
{
    switch (key) {
#define FW2_BCASE(K, DL, C) \
    case K: batch_tile<PRESSURE, BX, L0 + DL, C, PP>(sa, rows, x0, y0, r0, r1, r2); break;
    FW2_BCASE(0, 0, false) FW2_BCASE(1, 0, true) FW2_BCASE(2, 1, false) FW2_BCASE(3, 1, true)
    FW2_BCASE(4, 2, false) FW2_BCASE(5, 2, true) FW2_BCASE(6, 3, false) FW2_BCASE(7, 3, true)
#undef FW2_BCASE
    default: break;
    }
}

// One phase of the entries of one class of the table: CLASS bit 0 set for
// 5..8 mechanisms (else 1..4), bit 1 set for per-point stencil weights.
// Each class present gets a launch of its own, so that the larger register
// demand of many mechanisms or per-point weights does not lower the
// occupancy of the common class; entries are grouped by class, and each
// launch walks only its class's range of the tile list.
template <bool PRESSURE, int BX, int CLASS>
__global__ void __launch_bounds__(BX) batch_phase(const BatchTable *__restrict__ T)
{
    constexpr bool MANY = (CLASS & 1) != 0, PP = (CLASS & 2) != 0;
    __shared__ float r0[4][BX + 8];
    __shared__ float r1[3][BX + 2];
    __shared__ float r2[3][BX + 1];
    // the class's own tiles: entries are grouped by class, so they are one
    // contiguous range of the tile list
    const int begin = T->class_begin[CLASS], total = T->class_end[CLASS] - begin, rows = T->rows;
    // Blocks are dealt to the 8 XCDs round-robin; with a grid that is a
    // multiple of 8, the blocks of XCD x walk one contiguous eighth of the
    // range, so neighbouring tiles (which share halo rows) meet in the same L2.
    int t = blockIdx.x, t_end = total, t_step = gridDim.x;
    if (gridDim.x % 8 == 0) {
        const int x = blockIdx.x % 8, q = total / 8, rem = total % 8;
        const int start = x * q + min(x, rem);
        t = start + blockIdx.x / 8;
        t_end = start + q + (x < rem ? 1 : 0);
        t_step = gridDim.x / 8;
    }
    for (; t < t_end; t += t_step) {
        const int tile = begin + t;
        const int d = batch_entry_of_tile(T, tile);
        const BatchEntry &e = T->e[d];
        if (batch_class(e.L, e.a.local_stencil) != CLASS) continue;     // (never: the range is the class's)
        const long long step = *e.rcv.step;
        // pressure phase of step s runs while the counter reads s; velocity after it moved to s + 1
        const bool active = PRESSURE ? step < e.n_steps : (step >= 1 && step <= e.n_steps);
        if (!active) continue;                      // uniform over the block
        // the entry's arguments are read in place: the address is uniform
        // over the block, so they load into scalar registers as a kernel's
        // own arguments do
        const StepArgs &sa = e.a;
        const int nbx = (sa.geo.n[0] + BX - 1) / BX;
        const int lt = tile - e.tile_base;
        const int x0 = (lt % nbx) * BX, y0 = (lt / nbx) * rows;
        const int key = (e.L - (MANY ? 5 : 1)) * 2 + e.scheme;
        batch_dispatch<PRESSURE, BX, MANY ? 5 : 1, PP>(key, sa, rows, x0, y0, r0, r1, r2);
        __syncthreads();                            // the LDS rings are reused by the next tile
    }
}

template <int NDIM, int L, bool C, bool PP>
hipError_t launch_p(const StepArgs &a, hipStream_t st)
{
    dim3 block(kBX, kBY);
    dim3 grid((a.geo.n[0] + kBX - 1) / kBX, (a.geo.n[1] + kBY * kRY - 1) / (kBY * kRY), a.geo.n[2]);
    hipLaunchKernelGGL((pressure_kernel<NDIM, L, C, PP>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <int NDIM, int L, bool C, bool PP>
hipError_t launch_v(const StepArgs &a, hipStream_t st)
{
    dim3 block(kBX, kBY);
    dim3 grid((a.geo.n[0] + kBX - 1) / kBX, (a.geo.n[1] + kBY * kRY - 1) / (kBY * kRY), a.geo.n[2]);
    hipLaunchKernelGGL((velocity_kernel<NDIM, L, C, PP>), grid, block, 0, st, a);
    return hipGetLastError();
}

template <bool P, int NDIM, int L, bool C, bool PP>
hipError_t dispatch_variant(const StepArgs &a, const KernelConfig &kc, hipStream_t st)
{
    if constexpr (L > 4) {
        // more than four mechanisms: the generic kernel, or one sweep shape per
        // dimension (256-column 2D rows; 64 x 8 3D columns without the plane
        // prefetch, whose second copy of the memory variables would not fit
        // the registers)
        if (kc.variant == 0) return P ? launch_p<NDIM, L, C, PP>(a, st) : launch_v<NDIM, L, C, PP>(a, st);
        if (NDIM == 2) return launch_sweep<L, C, false, PP>(a, P, KernelConfig{1, 256, kc.rows}, st);
        return launch_sweep3<L, C, PP, 0>(a, P, KernelConfig{1, 64, kc.rows}, st);
    } else {
        if (NDIM == 3 && kc.variant == 1) return launch_sweep3<L, C, PP, 0>(a, P, kc, st);
        if (NDIM == 3 && kc.variant == 2) return launch_sweep3<L, C, PP, 1>(a, P, kc, st);
        if (NDIM == 3 && kc.variant == 3) return launch_sweep3<L, C, PP, 2>(a, P, kc, st);
        if (NDIM == 2 && kc.variant == 1) return launch_sweep<L, C, false, PP>(a, P, kc, st);
        if (NDIM == 2 && kc.variant == 2) return launch_sweep<L, C, true, PP>(a, P, kc, st);
        return P ? launch_p<NDIM, L, C, PP>(a, st) : launch_v<NDIM, L, C, PP>(a, st);
    }
}

template <bool P, int NDIM, int L>
hipError_t dispatch_scheme(const StepArgs &a, int scheme, const KernelConfig &kc, hipStream_t st)
{
    const bool pp = a.local_stencil != 0;
    if (scheme == 0)
        return pp ? dispatch_variant<P, NDIM, L, false, true>(a, kc, st) : dispatch_variant<P, NDIM, L, false, false>(a, kc, st);
    return pp ? dispatch_variant<P, NDIM, L, true, true>(a, kc, st) : dispatch_variant<P, NDIM, L, true, false>(a, kc, st);
}

template <bool P, int NDIM>
hipError_t dispatch_L(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t st)
{
    switch (L) {
    case 1: return dispatch_scheme<P, NDIM, 1>(a, scheme, kc, st);
    case 2: return dispatch_scheme<P, NDIM, 2>(a, scheme, kc, st);
    case 3: return dispatch_scheme<P, NDIM, 3>(a, scheme, kc, st);
    case 4: return dispatch_scheme<P, NDIM, 4>(a, scheme, kc, st);
    case 5: return dispatch_scheme<P, NDIM, 5>(a, scheme, kc, st);
    case 6: return dispatch_scheme<P, NDIM, 6>(a, scheme, kc, st);
    case 7: return dispatch_scheme<P, NDIM, 7>(a, scheme, kc, st);
    case 8: return dispatch_scheme<P, NDIM, 8>(a, scheme, kc, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

}  // namespace fw2
