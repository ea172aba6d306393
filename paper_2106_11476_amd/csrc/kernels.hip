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

// Value of a padded array at (x, y) inside the grid, else 0 (no access).
__device__ __forceinline__ float ld2(const float *__restrict__ f, const Geometry &g, int x, int y)
{
    if (x < 0 || x >= g.n[0] || y < 0 || y >= g.n[1]) return 0.0f;
    return f[g.origin + (int64_t)y * g.pitch + x];
}

template <int L, bool CENTRED, int BX>
__global__ void __launch_bounds__(BX) pressure_sweep2d(const StepArgs a, int rows, int nbx, int nblocks)
{
    const Geometry &g = a.geo;
    const int tile = tile_of_block(blockIdx.x, nblocks);
    const int x0 = (tile % nbx) * BX, y0 = (tile / nbx) * rows;
    const int t = threadIdx.x;
    const int i = x0 + t;
    const int nx = g.n[0], ny = g.n[1];
    const int64_t P = g.pitch;
    const float *__restrict__ vx = a.v;
    const float *__restrict__ vy = a.v + g.stride;
    float *__restrict__ pp = a.p;
    float *__restrict__ psi = a.psi2;
    const float *__restrict__ kap = a.kap;
    const float *__restrict__ nlq = a.nlq;
    const uint8_t *__restrict__ lab = a.label;

    __shared__ float sx[4][BX + 8];     // v_x rows, column c <-> x0 - 4 + c
    __shared__ float sy[3][BX + 2];     // v_y rows, column c <-> x0 - 1 + c

    // prologue: window rows y0-4 .. y0+2, rings rows y0-1 and y0
    float w[8];
    w[0] = 0.0f;
#pragma unroll
    for (int k = 1; k < 8; ++k) w[k] = ld2(vy, g, i, y0 - 5 + k);
#pragma unroll
    for (int r = -1; r <= 0; ++r) {
        sx[(y0 + r) & 3][t + 4] = ld2(vx, g, i, y0 + r);
        if (t < 8) {
            const int xc = t < 4 ? x0 - 4 + t : x0 + BX + (t - 4);
            sx[(y0 + r) & 3][t < 4 ? t : BX + t] = ld2(vx, g, xc, y0 + r);
        }
    }
    sy[(y0 + 2) % 3][t + 1] = ld2(vy, g, i, y0 - 1);
    if (t < 2) sy[(y0 + 2) % 3][t == 0 ? 0 : BX + 1] = ld2(vy, g, t == 0 ? x0 - 1 : x0 + BX, y0 - 1);

    const int sxs = a.nb[0] > 0 ? max(max(a.nb[0] - i, i - (nx - 1 - a.nb[0])), 0) : 0;
    const int yend = min(y0 + rows, ny);
    for (int j = y0; j < yend; ++j) {
        const bool live = i < nx;
        const int64_t idx = g.origin + (int64_t)j * P + i;
        // loads of this row
        const float vyn = ld2(vy, g, i, j + 3);
        const float vxn = ld2(vx, g, i, j + 1);
        float hx = 0.0f, hy = 0.0f;
        if (t < 8) hx = ld2(vx, g, t < 4 ? x0 - 4 + t : x0 + BX + (t - 4), j + 1);
        if (t < 2) hy = ld2(vy, g, t == 0 ? x0 - 1 : x0 + BX, j);
        float p0 = 0.0f, k0 = 1.0f, q0 = 0.0f;
        float m[2][L];
        int l = 0;
        if (live) {
            p0 = pp[idx];
            k0 = kap[idx];
            q0 = nlq[idx];
            l = lab ? (int)lab[idx] : 0;
#pragma unroll
            for (int ax = 0; ax < 2; ++ax)
#pragma unroll
                for (int nu = 0; nu < L; ++nu) m[ax][nu] = psi[(int64_t)(ax * L + nu) * g.stride + idx];
        }
#pragma unroll
        for (int k = 0; k < 7; ++k) w[k] = w[k + 1];
        w[7] = vyn;
        sx[(j + 1) & 3][t + 4] = vxn;
        if (t < 8) sx[(j + 1) & 3][t < 4 ? t : BX + t] = hx;
        sy[j % 3][t + 1] = w[4];
        if (t < 2) sy[j % 3][t == 0 ? 0 : BX + 1] = hy;
        __syncthreads();
        if (!live) continue;
        const float *r0 = sx[j & 3], *rp = sx[(j + 1) & 3], *rm = sx[(j + 3) & 3];
        float Dx = a.g[0] * (r0[t + 4] - r0[t + 3]);
        Dx = fmaf(a.g[1], r0[t + 5] - r0[t + 2], Dx);
        Dx = fmaf(a.g[2], r0[t + 6] - r0[t + 1], Dx);
        Dx = fmaf(a.g[3], r0[t + 7] - r0[t], Dx);
        Dx = fmaf(a.g11, (rp[t + 4] - rp[t + 3]) + (rm[t + 4] - rm[t + 3]), Dx);
        const float *c0 = sy[j % 3], *cm = sy[(j + 2) % 3];
        float Dy = a.g[0] * (w[4] - w[3]);
        Dy = fmaf(a.g[1], w[5] - w[2], Dy);
        Dy = fmaf(a.g[2], w[6] - w[1], Dy);
        Dy = fmaf(a.g[3], w[7] - w[0], Dy);
        Dy = fmaf(a.g11, (c0[t + 2] - cm[t + 2]) + (c0[t] - cm[t]), Dy);
        const int sys = a.nb[1] > 0 ? max(max(a.nb[1] - j, j - (ny - 1 - a.nb[1])), 0) : 0;
        float S = 0.0f;
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) {
            const float D = ax == 0 ? Dx : Dy;
            const int tt = (ax == 0 ? sxs : sys) * a.n_labels + l;
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
        pp[idx] = p0 - a.dt * S / kappa;
#pragma unroll
        for (int ax = 0; ax < 2; ++ax)
#pragma unroll
            for (int nu = 0; nu < L; ++nu) psi[(int64_t)(ax * L + nu) * g.stride + idx] = m[ax][nu];
    }
}

template <int L, bool CENTRED, int BX>
__global__ void __launch_bounds__(BX) velocity_sweep2d(const StepArgs a, int rows, int nbx, int nblocks)
{
    const Geometry &g = a.geo;
    const int tile = tile_of_block(blockIdx.x, nblocks);
    const int x0 = (tile % nbx) * BX, y0 = (tile / nbx) * rows;
    const int t = threadIdx.x;
    const int i = x0 + t;
    const int nx = g.n[0], ny = g.n[1];
    const int64_t P = g.pitch;
    const float *__restrict__ pp = a.p;
    float *__restrict__ vx = a.v;
    float *__restrict__ vy = a.v + g.stride;
    float *__restrict__ psi = a.psi1;
    const float *__restrict__ rho = a.rho;
    const float *__restrict__ kap = a.kap;
    const uint8_t *__restrict__ lab = a.label;

    __shared__ float sp[4][BX + 8];     // p rows, column c <-> x0 - 4 + c
    __shared__ float sr[3][BX + 1];     // rho rows, column c <-> x0 + c
    __shared__ float sk[3][BX + 1];     // kappa0 rows

    // prologue: window rows y0-3 .. y0+3; p ring rows y0-1, y0; rho/kappa row y0
    float w[8];
    w[0] = 0.0f;
#pragma unroll
    for (int k = 1; k < 8; ++k) w[k] = ld2(pp, g, i, y0 - 4 + k);
#pragma unroll
    for (int r = -1; r <= 0; ++r) {
        sp[(y0 + r) & 3][t + 4] = ld2(pp, g, i, y0 + r);
        if (t < 8) {
            const int xc = t < 4 ? x0 - 4 + t : x0 + BX + (t - 4);
            sp[(y0 + r) & 3][t < 4 ? t : BX + t] = ld2(pp, g, xc, y0 + r);
        }
    }
    sr[y0 % 3][t] = ld2(rho, g, i, y0);
    sk[y0 % 3][t] = ld2(kap, g, i, y0);
    if (t == 0) {
        sr[y0 % 3][BX] = ld2(rho, g, x0 + BX, y0);
        sk[y0 % 3][BX] = ld2(kap, g, x0 + BX, y0);
    }

    const int sxs = a.nb[0] > 0 ? max(max(a.nb[0] - i, i - (nx - 2 - a.nb[0])), 0) : 0;
    const int yend = min(y0 + rows, ny);
    for (int j = y0; j < yend; ++j) {
        const bool live = i < nx;
        const int64_t idx = g.origin + (int64_t)j * P + i;
        const float pn = ld2(pp, g, i, j + 4);
        const float rn = ld2(rho, g, i, j + 1);
        const float kn = ld2(kap, g, i, j + 1);
        float hp = 0.0f, hr = 0.0f, hk = 0.0f;
        if (t < 8) hp = ld2(pp, g, t < 4 ? x0 - 4 + t : x0 + BX + (t - 4), j + 1);
        if (t == 0) {
            hr = ld2(rho, g, x0 + BX, j + 1);
            hk = ld2(kap, g, x0 + BX, j + 1);
        }
        float ux = 0.0f, uy = 0.0f;
        float m[2][L];
        int l = 0;
        if (live) {
            ux = vx[idx];
            uy = vy[idx];
            l = lab ? (int)lab[idx] : 0;
#pragma unroll
            for (int ax = 0; ax < 2; ++ax)
#pragma unroll
                for (int nu = 0; nu < L; ++nu) m[ax][nu] = psi[(int64_t)(ax * L + nu) * g.stride + idx];
        }
#pragma unroll
        for (int k = 0; k < 7; ++k) w[k] = w[k + 1];
        w[7] = pn;
        sp[(j + 1) & 3][t + 4] = w[4];
        if (t < 8) sp[(j + 1) & 3][t < 4 ? t : BX + t] = hp;
        sr[(j + 1) % 3][t] = rn;
        sk[(j + 1) % 3][t] = kn;
        if (t == 0) {
            sr[(j + 1) % 3][BX] = hr;
            sk[(j + 1) % 3][BX] = hk;
        }
        __syncthreads();
        if (!live) continue;
        const float *r0 = sp[j & 3], *rp = sp[(j + 1) & 3], *rm = sp[(j + 3) & 3];
        const float *rr0 = sr[j % 3], *kk0 = sk[j % 3];
        const int sys = a.nb[1] > 0 ? max(max(a.nb[1] - j, j - (ny - 2 - a.nb[1])), 0) : 0;
        // v_x at (i + 1/2, j)
        if (i < nx - 1) {
            float D = a.g[0] * (r0[t + 5] - r0[t + 4]);
            D = fmaf(a.g[1], r0[t + 6] - r0[t + 3], D);
            D = fmaf(a.g[2], r0[t + 7] - r0[t + 2], D);
            D = fmaf(a.g[3], r0[t + 8] - r0[t + 1], D);
            D = fmaf(a.g11, (rp[t + 5] - rp[t + 4]) + (rm[t + 5] - rm[t + 4]), D);
            const int tt = sxs * a.n_labels + l;
            const float2 *__restrict__ bc = a.bc1[0] + (int64_t)tt * L;
            float S = a.w1[0][tt] * D;
#pragma unroll
            for (int nu = 0; nu < L; ++nu) {
                const float2 q = bc[nu];
                const float mn = fmaf(q.x, m[0][nu], q.y * D);
                S += CENTRED ? m[0][nu] : mn;
                m[0][nu] = mn;
            }
            const float pbar = 0.5f * (r0[t + 4] + r0[t + 5]);
            const float rho_a = 0.5f * (rr0[t] + rr0[t + 1]);
            const float kap_a = 0.5f * (kk0[t] + kk0[t + 1]);
            vx[idx] = ux - a.dt * S / (rho_a * (1.0f + kap_a * pbar));
#pragma unroll
            for (int nu = 0; nu < L; ++nu) psi[(int64_t)nu * g.stride + idx] = m[0][nu];
        }
        // v_y at (i, j + 1/2)
        if (j < ny - 1) {
            float D = a.g[0] * (w[4] - w[3]);
            D = fmaf(a.g[1], w[5] - w[2], D);
            D = fmaf(a.g[2], w[6] - w[1], D);
            D = fmaf(a.g[3], w[7] - w[0], D);
            D = fmaf(a.g11, (rp[t + 5] - r0[t + 5]) + (rp[t + 3] - r0[t + 3]), D);
            const int tt = sys * a.n_labels + l;
            const float2 *__restrict__ bc = a.bc1[1] + (int64_t)tt * L;
            float S = a.w1[1][tt] * D;
#pragma unroll
            for (int nu = 0; nu < L; ++nu) {
                const float2 q = bc[nu];
                const float mn = fmaf(q.x, m[1][nu], q.y * D);
                S += CENTRED ? m[1][nu] : mn;
                m[1][nu] = mn;
            }
            const float pbar = 0.5f * (w[3] + w[4]);
            const float rho_a = 0.5f * (rr0[t] + sr[(j + 1) % 3][t]);
            const float kap_a = 0.5f * (kk0[t] + sk[(j + 1) % 3][t]);
            vy[idx] = uy - a.dt * S / (rho_a * (1.0f + kap_a * pbar));
#pragma unroll
            for (int nu = 0; nu < L; ++nu) psi[(int64_t)(L + nu) * g.stride + idx] = m[1][nu];
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

template <int L, bool C>
hipError_t launch_sweep(const StepArgs &a, bool pressure, const KernelConfig &kc, hipStream_t st)
{
    const int nbx = (a.geo.n[0] + kc.bx - 1) / kc.bx;
    const int nby = (a.geo.n[1] + kc.rows - 1) / kc.rows;
    const int nblocks = nbx * nby;
#define FW2_SWEEP(BXV)                                                                                  \
    if (kc.bx == BXV) {                                                                                 \
        if (pressure)                                                                                   \
            hipLaunchKernelGGL((pressure_sweep2d<L, C, BXV>), dim3(nblocks), dim3(BXV), 0, st, a, kc.rows, nbx, nblocks); \
        else                                                                                            \
            hipLaunchKernelGGL((velocity_sweep2d<L, C, BXV>), dim3(nblocks), dim3(BXV), 0, st, a, kc.rows, nbx, nblocks); \
        return hipGetLastError();                                                                       \
    }
    FW2_SWEEP(64)
    FW2_SWEEP(128)
    FW2_SWEEP(256)
#undef FW2_SWEEP
    return hipErrorInvalidValue;
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
hipError_t dispatch_scheme(const StepArgs &a, int scheme, const KernelConfig &kc, hipStream_t st)
{
    if (NDIM == 2 && kc.variant == 1) {
        if (scheme == 0) return launch_sweep<L, false>(a, P, kc, st);
        return launch_sweep<L, true>(a, P, kc, st);
    }
    if (scheme == 0) return P ? launch_p<NDIM, L, false>(a, st) : launch_v<NDIM, L, false>(a, st);
    return P ? launch_p<NDIM, L, true>(a, st) : launch_v<NDIM, L, true>(a, st);
}

template <bool P, int NDIM>
hipError_t dispatch_L(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t st)
{
    switch (L) {
    case 1: return dispatch_scheme<P, NDIM, 1>(a, scheme, kc, st);
    case 2: return dispatch_scheme<P, NDIM, 2>(a, scheme, kc, st);
    case 3: return dispatch_scheme<P, NDIM, 3>(a, scheme, kc, st);
    case 4: return dispatch_scheme<P, NDIM, 4>(a, scheme, kc, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_pressure(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t st)
{
    return a.geo.ndim == 2 ? dispatch_L<true, 2>(a, L, scheme, kc, st) : dispatch_L<true, 3>(a, L, scheme, kc, st);
}

hipError_t launch_velocity(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t st)
{
    return a.geo.ndim == 2 ? dispatch_L<false, 2>(a, L, scheme, kc, st) : dispatch_L<false, 3>(a, L, scheme, kc, st);
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
