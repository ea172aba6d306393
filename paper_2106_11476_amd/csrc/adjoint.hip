// gfx950 kernels of the discrete adjoint of one time step (time-centred
// memory scheme), for the gradient of J = 1/2 sum (trace - obs)^2 with
// respect to kappa0 (and through it the sound speed).
//
// The relaxation is not time-reversible (Sec. 5: the adjoint of the
// relaxation operators must be derived explicitly), so the reverse step is
// the transpose of the forward step's linearisation, taken phase by phase in
// reverse order, about the forward state at the step's input:
//   A0  pressure points: recompute S = sum_a (w2 D^-v_a + sum psi2) and
//       p'' = p - dt S / K (+ sources, A_src), K = kappa0 (1 + kappa0 (1-2beta) p)
//   A1  v points inside the grid: velocity phase reversed, pointwise:
//       lam_S' = -dt lam_v / Q, lam_Q = dt S' lam_v / Q^2, lam_psi1 <- lam_S' + b1 lam_psi1,
//       and the adjoints of D^+ p'', of pbar and of kappa0_a kept per axis
//   A_rcv  lam_p[R] += trace_n - obs_n
//   A2  pressure points: lam_p'' = lam_p - sum_a D^-(lam_D'_a) + means of lam_pbar,
//       gradient from the velocity multipliers, then the pressure phase
//       reversed: lam_S = -dt lam_p''/K, lam_K = dt S lam_p''/K^2,
//       lam_p = lam_p'' + lam_K kappa0 kappa0 (1-2beta),
//       grad += lam_K (1 + 2 kappa0 (1-2beta) p), lam_psi2 <- lam_S + b2 lam_psi2,
//       lam_D_a = w2 lam_S + sum c2 lam_psi2 (new)
//   A3  v points inside the grid: lam_v_a -= D^+(lam_D_a)
// using (D^-)^T = -(D^+) and (D^+)^T = -(D^-).
// The phases run as one-thread-per-point kernels, two per step: A3 of a step
// is deferred into the velocity kernel (A1) of the next call, A_rcv runs in
// extra blocks of that kernel, and A0 of the step before is fused into the
// pressure kernel (A2) when its state is at hand.  A 2D variant as two row sweeps per step is kept below behind a
// compile-time switch.
#include "kernels.hpp"

#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace fw2 {

namespace {

constexpr int kABX = 256, kABY = 1;       // default block of the per-point kernels (measured best)

// Block shape of the per-point kernels: FW2_ADJ_BLOCK="bx,by" with bx * by =
// 256 (a tuning knob), else kABX x kABY.
dim3 adj_block()
{
    static dim3 b = [] {
        int bx = kABX, by = kABY;
        if (const char *e = std::getenv("FW2_ADJ_BLOCK")) {
            int x = 0, y = 0;
            if (std::sscanf(e, "%d,%d", &x, &y) == 2 && x > 0 && y > 0 && x * y == kABX * kABY) {
                bx = x;
                by = y;
            }
        }
        return dim3(bx, by);
    }();
    return b;
}

struct AdjArgs {
    StepArgs f;              // medium, tables, stencil of the domain (f.p etc. unused)
    const float *sp;         // forward state at the step input: p, v, psi1, psi2 blocks
    const float *sq;         // forward state of the step before (A0 fused into A2), or unused
    float *lp;               // adjoint state: same layout
    float *pp;               // p'' (forward recompute)
    float *sS;               // S of the pressure phase (forward recompute)
    float *lDv;              // [ndim] adjoint of D^+ p'' at v points
    float *lpb;              // [ndim] adjoint of pbar
    float *lkv;              // [ndim] adjoint of kappa0_a
    float *lDp;              // [ndim] adjoint of D^- v_a at p points
    float *gk;               // dJ/dkappa0
    int nbx, nby, nblocks;   // blocks along x and y; point blocks in the 1D launch
    const int64_t *rcv_idx;  // receivers (flat indices), added into lam_p by the
    const float *residual;   // velocity kernel's extra blocks: trace - obs of this step
    int n_rcv;               // 0: no receiver blocks
};

// Point block of a 1D launch.  Blocks are dealt to the 8 XCDs round-robin
// (block b runs on XCD b mod 8); renumbering them so that XCD x takes one
// contiguous run of point blocks keeps the stencil rows that neighbouring
// blocks share in that XCD's L2 instead of fetching them once per XCD.
// A bijection of [0, nblocks) for any nblocks.
__device__ __forceinline__ int xcd_block(int bid, int nblocks)
{
    const int x = bid % 8, q = nblocks / 8, rem = nblocks % 8;
    return x * q + min(x, rem) + bid / 8;
}

__device__ __forceinline__ int64_t aoff(const Geometry &g, int a)
{
    return a == 0 ? (int64_t)1 : (a == 1 ? g.pitch : g.plane);
}

__device__ __forceinline__ float dminus(const float *__restrict__ f, const Geometry &g, const float *gw, float g11,
                                        int a, int nd, int64_t idx)
{
    const int64_t o = aoff(g, a);
    float D = gw[0] * (f[idx] - f[idx - o]);
    D = fmaf(gw[1], f[idx + o] - f[idx - 2 * o], D);
    D = fmaf(gw[2], f[idx + 2 * o] - f[idx - 3 * o], D);
    D = fmaf(gw[3], f[idx + 3 * o] - f[idx - 4 * o], D);
    float cr = 0.0f;
    for (int b = 0; b < nd; ++b) {
        if (b == a) continue;
        const int64_t o2 = aoff(g, b);
        cr += (f[idx + o2] - f[idx - o + o2]) + (f[idx - o2] - f[idx - o - o2]);
    }
    return fmaf(g11, cr, D);
}

__device__ __forceinline__ float dplus(const float *__restrict__ f, const Geometry &g, const float *gw, float g11,
                                       int a, int nd, int64_t idx)
{
    const int64_t o = aoff(g, a);
    float D = gw[0] * (f[idx + o] - f[idx]);
    D = fmaf(gw[1], f[idx + 2 * o] - f[idx - o], D);
    D = fmaf(gw[2], f[idx + 3 * o] - f[idx - 2 * o], D);
    D = fmaf(gw[3], f[idx + 4 * o] - f[idx - 3 * o], D);
    float cr = 0.0f;
    for (int b = 0; b < nd; ++b) {
        if (b == a) continue;
        const int64_t o2 = aoff(g, b);
        cr += (f[idx + o + o2] - f[idx + o2]) + (f[idx + o - o2] - f[idx - o2]);
    }
    return fmaf(g11, cr, D);
}

__device__ __forceinline__ int slot_p(int x, int n, int nb) { return max(max(nb - x, x - (n - 1 - nb)), 0); }
__device__ __forceinline__ int slot_v(int x, int n, int nb) { return max(max(nb - x, x - (n - 2 - nb)), 0); }

#define ADJ_POINT                                                                  \
    const Geometry &g = A.f.geo;                                                   \
    const int blk = xcd_block(blockIdx.x, A.nblocks);                              \
    const int bxy = blk % (A.nbx * A.nby);                                         \
    const int i = (bxy % A.nbx) * blockDim.x + threadIdx.x;                        \
    const int j = (bxy / A.nbx) * blockDim.y + threadIdx.y;                        \
    const int k = blk / (A.nbx * A.nby);                                           \
    if (i >= g.n[0] || j >= g.n[1]) return;                                        \
    const int c3[3] = {i, j, k};                                                   \
    const int64_t idx = g.origin + (int64_t)k * g.plane + (int64_t)j * g.pitch + i; \
    const int lab = A.f.label ? (int)A.f.label[idx] : 0;                           \
    (void)c3;                                                                      \
    (void)lab;

// A0: forward recompute of the pressure phase (without sources).
template <int ND, int L>
__global__ void __launch_bounds__(kABX *kABY) adj_forward_p(const AdjArgs A)
{
    constexpr int nd = ND;
    ADJ_POINT
    const int64_t st = g.stride;
    const float *v = A.sp + st;
    const float *m2 = A.sp + (int64_t)(1 + nd + nd * L) * st;
    float S = 0.0f;
#pragma unroll
    for (int a = 0; a < nd; ++a) {
        const float D = dminus(v + a * st, g, A.f.g, A.f.g11, a, nd, idx);
        const int t = slot_p(c3[a], g.n[a], A.f.nb[a]) * A.f.n_labels + lab;
        float Sa = A.f.w2[a][t] * D;
#pragma unroll
        for (int nu = 0; nu < L; ++nu) Sa += ntld(&m2[(int64_t)(a * L + nu) * st + idx]);
        S += Sa;
    }
    const float p0 = A.sp[idx];
    const float K = A.f.kap[idx] * (1.0f + A.f.nlq[idx] * p0);
    A.pp[idx] = p0 - A.f.dt * S / K;
    A.sS[idx] = S;
}

__device__ __forceinline__ int64_t pidx(const Geometry &g, int64_t f)
{
    const int64_t x = f % g.n[0];
    const int64_t t = f / g.n[0];
    return g.origin + (t / g.n[1]) * g.plane + (t % g.n[1]) * g.pitch + x;
}

__global__ void adj_sources(float *pp, const SparseArgs s, long long step)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= s.n || step >= s.n_t) return;
    const int64_t pi = pidx(s.geo, s.idx[q]);
    pp[pi] = pp[pi] + s.w[q] * s.signals[(int64_t)s.sig[q] * s.n_t + step];
}

// A1: velocity phase reversed at v points.  DEFER_A3: first apply the A3 of
// the step after (lam_v -= D^+ lam_Dp, lam_Dp left by the previous call).
// Blocks past the point blocks add the receiver residual into lam_p (A_rcv),
// which this kernel neither reads nor writes otherwise.
template <int ND, int L, bool DEFER_A3>
__global__ void __launch_bounds__(kABX *kABY) adj_velocity(const AdjArgs A)
{
    constexpr int nd = ND;
    if ((int)blockIdx.x >= A.nblocks) {
        const int q = ((int)blockIdx.x - A.nblocks) * (int)(blockDim.x * blockDim.y) +
                      (int)(threadIdx.y * blockDim.x + threadIdx.x);
        if (q < A.n_rcv) atomicAdd(&A.lp[pidx(A.f.geo, A.rcv_idx[q])], A.residual[q]);
        return;
    }
    ADJ_POINT
    const int64_t st = g.stride;
    const float *m1 = A.sp + (int64_t)(1 + nd) * st;
    float *lv = A.lp + st;
    float *lm1 = A.lp + (int64_t)(1 + nd) * st;
#pragma unroll
    for (int a = 0; a < nd; ++a) {
        float *oDv = A.lDv + a * st, *opb = A.lpb + a * st, *okv = A.lkv + a * st;
        if (c3[a] == g.n[a] - 1) {                       // outside the grid: no adjoint flow
            oDv[idx] = 0.0f;
            opb[idx] = 0.0f;
            okv[idx] = 0.0f;
            continue;
        }
        const int64_t o = aoff(g, a);
        const float D = dplus(A.pp, g, A.f.g, A.f.g11, a, nd, idx);
        const int t = slot_v(c3[a], g.n[a], A.f.nb[a]) * A.f.n_labels + lab;
        const float2 *bc = A.f.bc1[a] + (int64_t)t * L;
        const float w = A.f.w1[a][t];
        float Sv = w * D;
#pragma unroll
        for (int nu = 0; nu < L; ++nu) Sv += ntld(&m1[(int64_t)(a * L + nu) * st + idx]);
        const float pbar = 0.5f * (A.pp[idx] + A.pp[idx + o]);
        const float rho_a = 0.5f * (A.f.rho[idx] + A.f.rho[idx + o]);
        const float kap_a = 0.5f * (A.f.kap[idx] + A.f.kap[idx + o]);
        const float Q = rho_a * (1.0f + kap_a * pbar);
        float lva = lv[a * st + idx];
        if (DEFER_A3) {
            lva -= dplus(A.lDp + a * st, g, A.f.g, A.f.g11, a, nd, idx);
            lv[a * st + idx] = lva;
        }
        const float lS = -A.f.dt * lva / Q;
        const float lQ = A.f.dt * Sv * lva / (Q * Q);
        float lD = w * lS;
#pragma unroll
        for (int nu = 0; nu < L; ++nu) {
            const int64_t c = (int64_t)(a * L + nu) * st + idx;
            const float2 q = bc[nu];
            const float lmn = ntld(&lm1[c]);
            lD = fmaf(q.y, lmn, lD);
            ntst(&lm1[c], fmaf(q.x, lmn, lS));
        }
        oDv[idx] = lD;
        opb[idx] = lQ * rho_a * kap_a;
        okv[idx] = lQ * rho_a * pbar;
    }
}

// A2: gather of the velocity-phase adjoints, then the pressure phase reversed.
// WITH_A0: then A0 of the step before at the same point, from the state sq
// (S of this step is read before that of the step before overwrites it).
template <int ND, int L, bool WITH_A0>
__global__ void __launch_bounds__(kABX *kABY) adj_pressure(const AdjArgs A)
{
    constexpr int nd = ND;
    ADJ_POINT
    const int64_t st = g.stride;
    float lpp = A.lp[idx];
    float gk = A.gk[idx];
#pragma unroll
    for (int a = 0; a < nd; ++a) {
        const int64_t o = aoff(g, a);
        lpp -= dminus(A.lDv + a * st, g, A.f.g, A.f.g11, a, nd, idx);
        lpp += 0.5f * (A.lpb[a * st + idx] + A.lpb[a * st + idx - o]);
        gk += 0.5f * (A.lkv[a * st + idx] + A.lkv[a * st + idx - o]);
    }
    const float p0 = A.sp[idx];
    const float x = A.f.kap[idx], q = A.f.nlq[idx];
    const float K = x * (1.0f + q * p0);
    const float S = A.sS[idx];
    const float lS = -A.f.dt * lpp / K;
    const float lK = A.f.dt * S * lpp / (K * K);
    A.lp[idx] = lpp + lK * x * q;
    A.gk[idx] = gk + lK * (1.0f + 2.0f * q * p0);
    float *lm2 = A.lp + (int64_t)(1 + nd + nd * L) * st;
#pragma unroll
    for (int a = 0; a < nd; ++a) {
        const int t = slot_p(c3[a], g.n[a], A.f.nb[a]) * A.f.n_labels + lab;
        const float2 *bc = A.f.bc2[a] + (int64_t)t * L;
        float lD = A.f.w2[a][t] * lS;
#pragma unroll
        for (int nu = 0; nu < L; ++nu) {
            const int64_t c = (int64_t)(a * L + nu) * st + idx;
            const float2 qq = bc[nu];
            const float lmn = ntld(&lm2[c]);
            lD = fmaf(qq.y, lmn, lD);
            ntst(&lm2[c], fmaf(qq.x, lmn, lS));
        }
        A.lDp[a * st + idx] = lD;
    }
    if (WITH_A0) {
        const float *vq = A.sq + st;
        const float *m2q = A.sq + (int64_t)(1 + nd + nd * L) * st;
        float S0 = 0.0f;
#pragma unroll
        for (int a = 0; a < nd; ++a) {
            const float D = dminus(vq + a * st, g, A.f.g, A.f.g11, a, nd, idx);
            const int t = slot_p(c3[a], g.n[a], A.f.nb[a]) * A.f.n_labels + lab;
            float Sa = A.f.w2[a][t] * D;
#pragma unroll
            for (int nu = 0; nu < L; ++nu) Sa += ntld(&m2q[(int64_t)(a * L + nu) * st + idx]);
            S0 += Sa;
        }
        const float q0 = A.sq[idx];
        const float K0 = x * (1.0f + q * q0);
        A.pp[idx] = q0 - A.f.dt * S0 / K0;
        A.sS[idx] = S0;
    }
}

// dJ/dc = dJ/dkappa0 * (-2 kappa0 / c), with c = 1/sqrt(rho kappa0).
__global__ void __launch_bounds__(kABX *kABY) adj_grad_c(const AdjArgs A, float *out)
{
    ADJ_POINT
    const float x = A.f.kap[idx];
    out[idx] = A.gk[idx] * (-2.0f * x * sqrtf(A.f.rho[idx] * x));
}

// The 2D row sweeps below are compiled only with FW2_ADJOINT_SWEEPS defined:
// a GPU run that included their first execution ended with a GPU fault whose
// cause is not established (they pass a CPU bounds check and agree with the
// one-thread-per-point kernels there), so every dimension uses the
// one-thread-per-point kernels until it is.
#ifdef FW2_ADJOINT_SWEEPS
// ---------------------------------------------------------------------------
// 2D reverse step as two row sweeps (the layout and ring conventions of the
// forward sweeps: a block of BX threads owns BX columns and walks `rows`
// rows; y-stencil fields sit in 8-row register windows, x-stencil fields in
// 4-row LDS rings with a 4-column halo, cross-term rows in 3-row rings).
//
//   V sweep (v points):  A3 of the step after (lam_v -= D^+ lam_Dp, deferred
//                        from the previous call) and A1 of this step
//   P sweep (p points):  A2 of this step, and A0 of the step before when its
//                        forward state is at hand (p'' and S of that step,
//                        sources added by adj_sources afterwards)
// The receiver residual goes into lam_p in extra blocks of the V launch (the
// V sweep does not touch lam_p).  A0 alone (the first reverse step of a
// segment) is the P sweep with A2 switched off, so p'' and S are computed by
// the same code whichever way they are reached.
// ---------------------------------------------------------------------------

struct AdjSweep {
    StepArgs f;              // medium, tables and stencil of the domain
    const float *sp;         // forward state at the input of this step
    const float *sq;         // forward state whose p'' / S the P sweep recomputes (A0)
    float *lp;               // adjoint state (same layout as the state block)
    float *pp, *sS, *lDv, *lpb, *lkv, *lDp, *gk;
    int rows, nbx, nblocks;
    // receivers (V sweep extra blocks)
    const int64_t *rcv_idx;
    const float *residual;
    int n_rcv;
};

__device__ __forceinline__ int adj_tile(int bid, int nblocks)
{
    if (nblocks % 8 != 0) return bid;
    return (bid % 8) * (nblocks / 8) + bid / 8;          // contiguous band of tiles per XCD
}

// Value at (x, y) of a padded 2D array; outside the grid the zero halo cell.
__device__ __forceinline__ float adj_ldz(const float *__restrict__ f, const Geometry &g, int x, int y)
{
    const bool in = (unsigned)x < (unsigned)g.n[0] && (unsigned)y < (unsigned)g.n[1];
    return f[in ? g.origin + (int64_t)y * g.pitch + x : g.origin - g.pitch - 1];
}

template <int BX>
__device__ __forceinline__ int adj_halo_x(int t, int x0) { return t < 4 ? x0 - 4 + t : x0 + BX + (t - 4); }
template <int BX>
__device__ __forceinline__ int adj_halo_c(int t) { return t < 4 ? t : BX + t; }

template <int L, int BX>
__global__ void __launch_bounds__(BX) adj_v_sweep2d(const AdjSweep A)
{
    if ((int)blockIdx.x >= A.nblocks) {                  // receiver residual into lam_p
        const int q = ((int)blockIdx.x - A.nblocks) * BX + (int)threadIdx.x;
        if (q < A.n_rcv) atomicAdd(&A.lp[pidx(A.f.geo, A.rcv_idx[q])], A.residual[q]);
        return;
    }
    __shared__ float sp_[4][BX + 8];     // p'' rows, column c <-> x0 - 4 + c
    __shared__ float sd[4][BX + 8];      // lam_Dp_x rows
    __shared__ float sq[3][BX + 2];      // lam_Dp_y rows, column c <-> x0 - 1 + c
    __shared__ float sr[3][BX + 1];      // rho rows, column c <-> x0 + c
    __shared__ float sk[3][BX + 1];      // kappa0 rows
    const StepArgs &a = A.f;
    const Geometry &g = a.geo;
    const int64_t st = g.stride;
    const int tile = adj_tile(blockIdx.x, A.nblocks);
    const int x0 = (tile % A.nbx) * BX, y0 = (tile / A.nbx) * A.rows;
    const int t = threadIdx.x, i = x0 + t;
    const int nx = g.n[0], ny = g.n[1];
    const bool live = i < nx;
    const float *__restrict__ pp = A.pp;
    const float *__restrict__ dpx = A.lDp;
    const float *__restrict__ dpy = A.lDp + st;
    const float *__restrict__ m1 = A.sp + 3 * st;
    float *__restrict__ lv = A.lp + st;
    float *__restrict__ lm1 = A.lp + 3 * st;

    float wp[8], wq[8];                  // p'' and lam_Dp_y, rows j-3 .. j+4
    wp[0] = wq[0] = 0.0f;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        wp[k] = adj_ldz(pp, g, i, y0 - 4 + k);
        wq[k] = adj_ldz(dpy, g, i, y0 - 4 + k);
    }
#pragma unroll
    for (int r = -1; r <= 0; ++r) {
        sp_[(y0 + r) & 3][t + 4] = adj_ldz(pp, g, i, y0 + r);
        sd[(y0 + r) & 3][t + 4] = adj_ldz(dpx, g, i, y0 + r);
        if (t < 8) {
            sp_[(y0 + r) & 3][adj_halo_c<BX>(t)] = adj_ldz(pp, g, adj_halo_x<BX>(t, x0), y0 + r);
            sd[(y0 + r) & 3][adj_halo_c<BX>(t)] = adj_ldz(dpx, g, adj_halo_x<BX>(t, x0), y0 + r);
        }
    }
    sq[y0 % 3][t + 1] = adj_ldz(dpy, g, i, y0);
    if (t < 2) sq[y0 % 3][t == 0 ? 0 : BX + 1] = adj_ldz(dpy, g, t == 0 ? x0 - 1 : x0 + BX, y0);
    sr[y0 % 3][t] = adj_ldz(a.rho, g, i, y0);
    sk[y0 % 3][t] = adj_ldz(a.kap, g, i, y0);
    if (t == 0) {
        sr[y0 % 3][BX] = adj_ldz(a.rho, g, x0 + BX, y0);
        sk[y0 % 3][BX] = adj_ldz(a.kap, g, x0 + BX, y0);
    }

    const int sxs = max(max(a.nb[0] - i, i - (nx - 2 - a.nb[0])), 0);
    const int yend = min(y0 + A.rows, ny);
    for (int j = y0; j < yend; ++j) {
        // loads of this row
        const float pn = adj_ldz(pp, g, i, j + 4), qn = adj_ldz(dpy, g, i, j + 4);
        const float dxn = adj_ldz(dpx, g, i, j + 1);
        float hp = 0.0f, hd = 0.0f, hq = 0.0f, hr = 0.0f, hk = 0.0f;
        if (t < 8) {
            hp = adj_ldz(pp, g, adj_halo_x<BX>(t, x0), j + 1);
            hd = adj_ldz(dpx, g, adj_halo_x<BX>(t, x0), j + 1);
        }
        if (t < 2) hq = adj_ldz(dpy, g, t == 0 ? x0 - 1 : x0 + BX, j + 1);
        if (t == 0) {
            hr = adj_ldz(a.rho, g, x0 + BX, j + 1);
            hk = adj_ldz(a.kap, g, x0 + BX, j + 1);
        }
        const float rn = adj_ldz(a.rho, g, i, j + 1), kn = adj_ldz(a.kap, g, i, j + 1);
        const int64_t idx = g.origin + (int64_t)j * g.pitch + i;
        float lvx = 0.0f, lvy = 0.0f, m[2][L], lm[2][L];
        int lab = 0;
        if (live) {
            lvx = lv[idx];
            lvy = lv[st + idx];
            lab = a.label ? (int)a.label[idx] : 0;
#pragma unroll
            for (int ax = 0; ax < 2; ++ax)
#pragma unroll
        #pragma unroll
        for (int nu = 0; nu < L; ++nu) {
                    m[ax][nu] = m1[(int64_t)(ax * L + nu) * st + idx];
                    lm[ax][nu] = lm1[(int64_t)(ax * L + nu) * st + idx];
                }
        }
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            wp[k] = wp[k + 1];
            wq[k] = wq[k + 1];
        }
        wp[7] = pn;
        wq[7] = qn;
        sp_[(j + 1) & 3][t + 4] = wp[4];
        sd[(j + 1) & 3][t + 4] = dxn;
        if (t < 8) {
            sp_[(j + 1) & 3][adj_halo_c<BX>(t)] = hp;
            sd[(j + 1) & 3][adj_halo_c<BX>(t)] = hd;
        }
        sq[(j + 1) % 3][t + 1] = wq[4];
        if (t < 2) sq[(j + 1) % 3][t == 0 ? 0 : BX + 1] = hq;
        sr[(j + 1) % 3][t] = rn;
        sk[(j + 1) % 3][t] = kn;
        if (t == 0) {
            sr[(j + 1) % 3][BX] = hr;
            sk[(j + 1) % 3][BX] = hk;
        }
        __syncthreads();
        if (live) {
            const float *P0 = sp_[j & 3], *Pp = sp_[(j + 1) & 3], *Pm = sp_[(j + 3) & 3];
            const float *X0 = sd[j & 3], *Xp = sd[(j + 1) & 3], *Xm = sd[(j + 3) & 3];
            const float *Q0 = sq[j % 3], *Qp = sq[(j + 1) % 3];
            const float *rr0 = sr[j % 3], *kk0 = sk[j % 3];
            // v_x at (i + 1/2, j)
            if (i < nx - 1) {
                float Dq = a.g[0] * (X0[t + 5] - X0[t + 4]);
                Dq = fmaf(a.g[1], X0[t + 6] - X0[t + 3], Dq);
                Dq = fmaf(a.g[2], X0[t + 7] - X0[t + 2], Dq);
                Dq = fmaf(a.g[3], X0[t + 8] - X0[t + 1], Dq);
                Dq = fmaf(a.g11, (Xp[t + 5] - Xp[t + 4]) + (Xm[t + 5] - Xm[t + 4]), Dq);
                lvx -= Dq;                                              // A3 of the step after
                float D = a.g[0] * (P0[t + 5] - P0[t + 4]);
                D = fmaf(a.g[1], P0[t + 6] - P0[t + 3], D);
                D = fmaf(a.g[2], P0[t + 7] - P0[t + 2], D);
                D = fmaf(a.g[3], P0[t + 8] - P0[t + 1], D);
                D = fmaf(a.g11, (Pp[t + 5] - Pp[t + 4]) + (Pm[t + 5] - Pm[t + 4]), D);
                const int tt = sxs * a.n_labels + lab;
                const float2 *__restrict__ bc = a.bc1[0] + (int64_t)tt * L;
                const float w = a.w1[0][tt];
                float Sv = w * D;
#pragma unroll
                for (int nu = 0; nu < L; ++nu) Sv += m[0][nu];
                const float pbar = 0.5f * (P0[t + 4] + P0[t + 5]);
                const float rho_a = 0.5f * (rr0[t] + rr0[t + 1]);
                const float kap_a = 0.5f * (kk0[t] + kk0[t + 1]);
                const float Q = rho_a * (1.0f + kap_a * pbar);
                const float lS = -a.dt * lvx / Q;
                const float lQ = a.dt * Sv * lvx / (Q * Q);
                float lD = w * lS;
#pragma unroll
        #pragma unroll
        for (int nu = 0; nu < L; ++nu) {
                    const float2 q = bc[nu];
                    lD = fmaf(q.y, lm[0][nu], lD);
                    lm[0][nu] = fmaf(q.x, lm[0][nu], lS);
                }
                lv[idx] = lvx;
                A.lDv[idx] = lD;
                A.lpb[idx] = lQ * rho_a * kap_a;
                A.lkv[idx] = lQ * rho_a * pbar;
#pragma unroll
                for (int nu = 0; nu < L; ++nu) lm1[(int64_t)nu * st + idx] = lm[0][nu];
            }
            // v_y at (i, j + 1/2)
            if (j < ny - 1) {
                float Dq = a.g[0] * (wq[4] - wq[3]);
                Dq = fmaf(a.g[1], wq[5] - wq[2], Dq);
                Dq = fmaf(a.g[2], wq[6] - wq[1], Dq);
                Dq = fmaf(a.g[3], wq[7] - wq[0], Dq);
                Dq = fmaf(a.g11, (Qp[t + 2] - Q0[t + 2]) + (Qp[t] - Q0[t]), Dq);
                lvy -= Dq;
                const int sys = max(max(a.nb[1] - j, j - (ny - 2 - a.nb[1])), 0);
                float D = a.g[0] * (wp[4] - wp[3]);
                D = fmaf(a.g[1], wp[5] - wp[2], D);
                D = fmaf(a.g[2], wp[6] - wp[1], D);
                D = fmaf(a.g[3], wp[7] - wp[0], D);
                D = fmaf(a.g11, (Pp[t + 5] - P0[t + 5]) + (Pp[t + 3] - P0[t + 3]), D);
                const int tt = sys * a.n_labels + lab;
                const float2 *__restrict__ bc = a.bc1[1] + (int64_t)tt * L;
                const float w = a.w1[1][tt];
                float Sv = w * D;
#pragma unroll
                for (int nu = 0; nu < L; ++nu) Sv += m[1][nu];
                const float pbar = 0.5f * (wp[3] + wp[4]);
                const float rho_a = 0.5f * (rr0[t] + sr[(j + 1) % 3][t]);
                const float kap_a = 0.5f * (kk0[t] + sk[(j + 1) % 3][t]);
                const float Q = rho_a * (1.0f + kap_a * pbar);
                const float lS = -a.dt * lvy / Q;
                const float lQ = a.dt * Sv * lvy / (Q * Q);
                float lD = w * lS;
#pragma unroll
        #pragma unroll
        for (int nu = 0; nu < L; ++nu) {
                    const float2 q = bc[nu];
                    lD = fmaf(q.y, lm[1][nu], lD);
                    lm[1][nu] = fmaf(q.x, lm[1][nu], lS);
                }
                lv[st + idx] = lvy;
                A.lDv[st + idx] = lD;
                A.lpb[st + idx] = lQ * rho_a * kap_a;
                A.lkv[st + idx] = lQ * rho_a * pbar;
#pragma unroll
                for (int nu = 0; nu < L; ++nu) lm1[(int64_t)(L + nu) * st + idx] = lm[1][nu];
            }
        }
    }
}

template <int L, int BX, bool DO_A2, bool DO_A0>
__global__ void __launch_bounds__(BX) adj_p_sweep2d(const AdjSweep A)
{
    __shared__ float sxa[4][BX + 8];     // lam_Dv_x rows, column c <-> x0 - 4 + c
    __shared__ float sya[3][BX + 2];     // lam_Dv_y rows, column c <-> x0 - 1 + c
    __shared__ float sxb[4][BX + 8];     // v_x rows of the recomputed state
    __shared__ float syb[3][BX + 2];     // v_y rows of the recomputed state
    __shared__ float spb[2][BX + 1];     // lam_pbar_x of the row, column c <-> x0 - 1 + c
    __shared__ float skv[2][BX + 1];     // lam_kappa0_x of the row
    const StepArgs &a = A.f;
    const Geometry &g = a.geo;
    const int64_t st = g.stride;
    const int tile = adj_tile(blockIdx.x, A.nblocks);
    const int x0 = (tile % A.nbx) * BX, y0 = (tile / A.nbx) * A.rows;
    const int t = threadIdx.x, i = x0 + t;
    const int nx = g.n[0], ny = g.n[1];
    const bool live = i < nx;
    const float *__restrict__ dvx = A.lDv;
    const float *__restrict__ dvy = A.lDv + st;
    const float *__restrict__ vx = A.sq + st;
    const float *__restrict__ vy = A.sq + 2 * st;
    const float *__restrict__ m2q = A.sq + (int64_t)(3 + 2 * L) * st;
    float *__restrict__ lm2 = A.lp + (int64_t)(3 + 2 * L) * st;

    float wa[8], wb[8];                  // lam_Dv_y and v_y, rows j-4 .. j+3
    wa[0] = wb[0] = 0.0f;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        wa[k] = DO_A2 ? adj_ldz(dvy, g, i, y0 - 5 + k) : 0.0f;
        wb[k] = DO_A0 ? adj_ldz(vy, g, i, y0 - 5 + k) : 0.0f;
    }
#pragma unroll
    for (int r = -1; r <= 0; ++r) {
        if (DO_A2) {
            sxa[(y0 + r) & 3][t + 4] = adj_ldz(dvx, g, i, y0 + r);
            if (t < 8) sxa[(y0 + r) & 3][adj_halo_c<BX>(t)] = adj_ldz(dvx, g, adj_halo_x<BX>(t, x0), y0 + r);
        }
        if (DO_A0) {
            sxb[(y0 + r) & 3][t + 4] = adj_ldz(vx, g, i, y0 + r);
            if (t < 8) sxb[(y0 + r) & 3][adj_halo_c<BX>(t)] = adj_ldz(vx, g, adj_halo_x<BX>(t, x0), y0 + r);
        }
    }
    if (DO_A2) {
        sya[(y0 + 2) % 3][t + 1] = adj_ldz(dvy, g, i, y0 - 1);
        if (t < 2) sya[(y0 + 2) % 3][t == 0 ? 0 : BX + 1] = adj_ldz(dvy, g, t == 0 ? x0 - 1 : x0 + BX, y0 - 1);
    }
    if (DO_A0) {
        syb[(y0 + 2) % 3][t + 1] = adj_ldz(vy, g, i, y0 - 1);
        if (t < 2) syb[(y0 + 2) % 3][t == 0 ? 0 : BX + 1] = adj_ldz(vy, g, t == 0 ? x0 - 1 : x0 + BX, y0 - 1);
    }
    // lam_pbar_y and lam_kappa0_y of the row above, carried down the sweep
    float pby_up = DO_A2 ? adj_ldz(A.lpb + st, g, i, y0 - 1) : 0.0f;
    float kvy_up = DO_A2 ? adj_ldz(A.lkv + st, g, i, y0 - 1) : 0.0f;

    const int sxs = max(max(a.nb[0] - i, i - (nx - 1 - a.nb[0])), 0);
    const int yend = min(y0 + A.rows, ny);
    for (int j = y0; j < yend; ++j) {
        const int64_t idx = g.origin + (int64_t)j * g.pitch + i;
        float an = 0.0f, axn = 0.0f, ha = 0.0f, hya = 0.0f, pbx = 0.0f, kvx = 0.0f, hpb = 0.0f, hkv = 0.0f;
        float bn = 0.0f, bxn = 0.0f, hb = 0.0f, hyb = 0.0f;
        if (DO_A2) {
            an = adj_ldz(dvy, g, i, j + 3);
            axn = adj_ldz(dvx, g, i, j + 1);
            if (t < 8) ha = adj_ldz(dvx, g, adj_halo_x<BX>(t, x0), j + 1);
            if (t < 2) hya = adj_ldz(dvy, g, t == 0 ? x0 - 1 : x0 + BX, j);
            pbx = adj_ldz(A.lpb, g, i, j);
            kvx = adj_ldz(A.lkv, g, i, j);
            if (t == 0) {
                hpb = adj_ldz(A.lpb, g, x0 - 1, j);
                hkv = adj_ldz(A.lkv, g, x0 - 1, j);
            }
        }
        if (DO_A0) {
            bn = adj_ldz(vy, g, i, j + 3);
            bxn = adj_ldz(vx, g, i, j + 1);
            if (t < 8) hb = adj_ldz(vx, g, adj_halo_x<BX>(t, x0), j + 1);
            if (t < 2) hyb = adj_ldz(vy, g, t == 0 ? x0 - 1 : x0 + BX, j);
        }
        float kap = 1.0f, nlq = 0.0f;
        int lab = 0;
        if (live) {
            kap = a.kap[idx];
            nlq = a.nlq[idx];
            lab = a.label ? (int)a.label[idx] : 0;
        }
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            wa[k] = wa[k + 1];
            wb[k] = wb[k + 1];
        }
        wa[7] = an;
        wb[7] = bn;
        if (DO_A2) {
            sxa[(j + 1) & 3][t + 4] = axn;
            if (t < 8) sxa[(j + 1) & 3][adj_halo_c<BX>(t)] = ha;
            sya[j % 3][t + 1] = wa[4];
            if (t < 2) sya[j % 3][t == 0 ? 0 : BX + 1] = hya;
            spb[j & 1][t + 1] = pbx;
            skv[j & 1][t + 1] = kvx;
            if (t == 0) {
                spb[j & 1][0] = hpb;
                skv[j & 1][0] = hkv;
            }
        }
        if (DO_A0) {
            sxb[(j + 1) & 3][t + 4] = bxn;
            if (t < 8) sxb[(j + 1) & 3][adj_halo_c<BX>(t)] = hb;
            syb[j % 3][t + 1] = wb[4];
            if (t < 2) syb[j % 3][t == 0 ? 0 : BX + 1] = hyb;
        }
        __syncthreads();
        const float pby = DO_A2 ? adj_ldz(A.lpb + st, g, i, j) : 0.0f;
        const float kvy = DO_A2 ? adj_ldz(A.lkv + st, g, i, j) : 0.0f;
        if (live) {
            const int sys = max(max(a.nb[1] - j, j - (ny - 1 - a.nb[1])), 0);
            if (DO_A2) {
                const float *r0 = sxa[j & 3], *rp = sxa[(j + 1) & 3], *rm = sxa[(j + 3) & 3];
                float Dx = a.g[0] * (r0[t + 4] - r0[t + 3]);
                Dx = fmaf(a.g[1], r0[t + 5] - r0[t + 2], Dx);
                Dx = fmaf(a.g[2], r0[t + 6] - r0[t + 1], Dx);
                Dx = fmaf(a.g[3], r0[t + 7] - r0[t], Dx);
                Dx = fmaf(a.g11, (rp[t + 4] - rp[t + 3]) + (rm[t + 4] - rm[t + 3]), Dx);
                const float *c0 = sya[j % 3], *cm = sya[(j + 2) % 3];
                float Dy = a.g[0] * (wa[4] - wa[3]);
                Dy = fmaf(a.g[1], wa[5] - wa[2], Dy);
                Dy = fmaf(a.g[2], wa[6] - wa[1], Dy);
                Dy = fmaf(a.g[3], wa[7] - wa[0], Dy);
                Dy = fmaf(a.g11, (c0[t + 2] - cm[t + 2]) + (c0[t] - cm[t]), Dy);
                float lpp = A.lp[idx];
                float gk = A.gk[idx];
                lpp -= Dx;
                lpp += 0.5f * (spb[j & 1][t + 1] + spb[j & 1][t]);
                gk += 0.5f * (skv[j & 1][t + 1] + skv[j & 1][t]);
                lpp -= Dy;
                lpp += 0.5f * (pby + pby_up);
                gk += 0.5f * (kvy + kvy_up);
                const float p0 = A.sp[idx];
                const float K = kap * (1.0f + nlq * p0);
                const float S = A.sS[idx];
                const float lS = -a.dt * lpp / K;
                const float lK = a.dt * S * lpp / (K * K);
                A.lp[idx] = lpp + lK * kap * nlq;
                A.gk[idx] = gk + lK * (1.0f + 2.0f * nlq * p0);
#pragma unroll
                for (int ax = 0; ax < 2; ++ax) {
                    const int tt = (ax == 0 ? sxs : sys) * a.n_labels + lab;
                    const float2 *__restrict__ bc = a.bc2[ax] + (int64_t)tt * L;
                    float lD = a.w2[ax][tt] * lS;
#pragma unroll
            #pragma unroll
        for (int nu = 0; nu < L; ++nu) {
                        const int64_t c = (int64_t)(ax * L + nu) * st + idx;
                        const float2 q = bc[nu];
                        const float lmn = lm2[c];
                        lD = fmaf(q.y, lmn, lD);
                        lm2[c] = fmaf(q.x, lmn, lS);
                    }
                    A.lDp[ax * st + idx] = lD;
                }
            }
            if (DO_A0) {                                         // p'' and S of the state sq
                const float *r0 = sxb[j & 3], *rp = sxb[(j + 1) & 3], *rm = sxb[(j + 3) & 3];
                float Dx = a.g[0] * (r0[t + 4] - r0[t + 3]);
                Dx = fmaf(a.g[1], r0[t + 5] - r0[t + 2], Dx);
                Dx = fmaf(a.g[2], r0[t + 6] - r0[t + 1], Dx);
                Dx = fmaf(a.g[3], r0[t + 7] - r0[t], Dx);
                Dx = fmaf(a.g11, (rp[t + 4] - rp[t + 3]) + (rm[t + 4] - rm[t + 3]), Dx);
                const float *c0 = syb[j % 3], *cm = syb[(j + 2) % 3];
                float Dy = a.g[0] * (wb[4] - wb[3]);
                Dy = fmaf(a.g[1], wb[5] - wb[2], Dy);
                Dy = fmaf(a.g[2], wb[6] - wb[1], Dy);
                Dy = fmaf(a.g[3], wb[7] - wb[0], Dy);
                Dy = fmaf(a.g11, (c0[t + 2] - cm[t + 2]) + (c0[t] - cm[t]), Dy);
                float S = 0.0f;
#pragma unroll
                for (int ax = 0; ax < 2; ++ax) {
                    const int tt = (ax == 0 ? sxs : sys) * a.n_labels + lab;
                    float Sa = a.w2[ax][tt] * (ax == 0 ? Dx : Dy);
#pragma unroll
                    for (int nu = 0; nu < L; ++nu) Sa += m2q[(int64_t)(ax * L + nu) * st + idx];
                    S += Sa;
                }
                const float q0 = A.sq[idx];
                const float K = kap * (1.0f + nlq * q0);
                A.pp[idx] = q0 - a.dt * S / K;
                A.sS[idx] = S;
            }
        }
        pby_up = pby;
        kvy_up = kvy;
    }
}

#endif  // FW2_ADJOINT_SWEEPS

}  // namespace

#ifdef FW2_ADJOINT_SWEEPS
namespace {

constexpr int kAdjBX = 256, kAdjRows = 8;

template <int L>
hipError_t adjoint_step_2d(AdjSweep A, const SparseArgs &src, const float *state, const float *state_prev,
                           long long step, bool have_pp, const SparseArgs &rcv, const float *residual,
                           hipStream_t st, bool *pp_next)
{
    const Geometry &g = A.f.geo;
    A.rows = kAdjRows;
    A.nbx = (g.n[0] + kAdjBX - 1) / kAdjBX;
    A.nblocks = A.nbx * ((g.n[1] + kAdjRows - 1) / kAdjRows);
    A.sp = state;
    const dim3 block(kAdjBX);
    if (!have_pp) {                                      // A0 of this step on its own
        A.sq = state;
        hipLaunchKernelGGL((adj_p_sweep2d<L, kAdjBX, false, true>), dim3(A.nblocks), block, 0, st, A);
        if (src.n > 0 && step < src.n_t)
            hipLaunchKernelGGL(adj_sources, dim3((src.n + 255) / 256), dim3(256), 0, st, A.pp, src, step);
    }
    A.rcv_idx = rcv.idx;
    A.residual = residual;
    A.n_rcv = residual ? rcv.n : 0;
    const int nrb = (A.n_rcv + kAdjBX - 1) / kAdjBX;
    hipLaunchKernelGGL((adj_v_sweep2d<L, kAdjBX>), dim3(A.nblocks + nrb), block, 0, st, A);
    if (state_prev && step >= 1) {                      // A2 of this step with A0 of the step before
        A.sq = state_prev;
        hipLaunchKernelGGL((adj_p_sweep2d<L, kAdjBX, true, true>), dim3(A.nblocks), block, 0, st, A);
        if (src.n > 0 && step - 1 < src.n_t)
            hipLaunchKernelGGL(adj_sources, dim3((src.n + 255) / 256), dim3(256), 0, st, A.pp, src, step - 1);
        *pp_next = true;
    } else {
        hipLaunchKernelGGL((adj_p_sweep2d<L, kAdjBX, true, false>), dim3(A.nblocks), block, 0, st, A);
        *pp_next = false;
    }
    return hipGetLastError();
}

}  // namespace
#endif  // FW2_ADJOINT_SWEEPS

namespace {

// Sets the block counts of a 1D launch of point blocks of the given shape
// over the grid (z planes of one block each) and returns the block count.
unsigned point_grid(AdjArgs &A, dim3 block)
{
    const Geometry &g = A.f.geo;
    A.nbx = (g.n[0] + (int)block.x - 1) / (int)block.x;
    A.nby = (g.n[1] + (int)block.y - 1) / (int)block.y;
    A.nblocks = A.nbx * A.nby * g.n[2];
    return (unsigned)A.nblocks;
}

// One thread per point.  A3 of each step is deferred into the velocity
// kernel of the next call; A0 of the step before is fused into the pressure
// kernel when its state is given, else run at the start of the next call.
template <int ND, int L>
hipError_t adjoint_step_points(const StepArgs &f, const SparseArgs &src, const SparseArgs &rcv, const float *state,
                               const float *state_prev, const AdjointBuffers &b, long long step, bool have_pp,
                               const float *residual, hipStream_t st, bool *pp_next)
{
    AdjArgs A;
    A.f = f;
    A.sp = state;
    A.sq = state_prev;
    A.lp = b.lp;
    A.pp = b.pp;
    A.sS = b.sS;
    A.lDv = b.lDv;
    A.lpb = b.lpb;
    A.lkv = b.lkv;
    A.lDp = b.lDp;
    A.gk = b.gk;
    const dim3 block = adj_block();
    const dim3 grid(point_grid(A, block));
    A.rcv_idx = rcv.idx;
    A.residual = residual;
    A.n_rcv = residual ? rcv.n : 0;
    const unsigned nt = block.x * block.y;
    const dim3 vgrid(grid.x + (unsigned)((A.n_rcv + (int)nt - 1) / (int)nt));
    if (!have_pp) {
        hipLaunchKernelGGL((adj_forward_p<ND, L>), grid, block, 0, st, A);
        if (src.n > 0 && step < src.n_t)
            hipLaunchKernelGGL(adj_sources, dim3((src.n + 255) / 256), dim3(256), 0, st, b.pp, src, step);
    }
    hipLaunchKernelGGL((adj_velocity<ND, L, true>), vgrid, block, 0, st, A);
    if (state_prev && step >= 1) {
        hipLaunchKernelGGL((adj_pressure<ND, L, true>), grid, block, 0, st, A);
        if (src.n > 0 && step - 1 < src.n_t)
            hipLaunchKernelGGL(adj_sources, dim3((src.n + 255) / 256), dim3(256), 0, st, b.pp, src, step - 1);
        *pp_next = true;
    } else {
        hipLaunchKernelGGL((adj_pressure<ND, L, false>), grid, block, 0, st, A);
        *pp_next = false;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint_step(const StepArgs &f, const SparseArgs &src, const SparseArgs &rcv, int L,
                               const float *state, const float *state_prev, const AdjointBuffers &b,
                               long long step, bool have_pp, const float *residual, hipStream_t st,
                               bool *pp_next)
{
#ifdef FW2_ADJOINT_SWEEPS
    if (f.geo.ndim == 2) {
        AdjSweep A;
        std::memset(&A, 0, sizeof(A));
        A.f = f;
        A.lp = b.lp;
        A.pp = b.pp;
        A.sS = b.sS;
        A.lDv = b.lDv;
        A.lpb = b.lpb;
        A.lkv = b.lkv;
        A.lDp = b.lDp;
        A.gk = b.gk;
        switch (L) {
        case 1: return adjoint_step_2d<1>(A, src, state, state_prev, step, have_pp, rcv, residual, st, pp_next);
        case 2: return adjoint_step_2d<2>(A, src, state, state_prev, step, have_pp, rcv, residual, st, pp_next);
        case 3: return adjoint_step_2d<3>(A, src, state, state_prev, step, have_pp, rcv, residual, st, pp_next);
        case 4: return adjoint_step_2d<4>(A, src, state, state_prev, step, have_pp, rcv, residual, st, pp_next);
        default: return hipErrorInvalidValue;
        }
    }
#endif
    switch (f.geo.ndim * 8 + L) {            // L = 1..8
    case 2 * 8 + 1: return adjoint_step_points<2, 1>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 2 * 8 + 2: return adjoint_step_points<2, 2>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 2 * 8 + 3: return adjoint_step_points<2, 3>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 2 * 8 + 4: return adjoint_step_points<2, 4>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 3 * 8 + 1: return adjoint_step_points<3, 1>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 3 * 8 + 2: return adjoint_step_points<3, 2>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 3 * 8 + 3: return adjoint_step_points<3, 3>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 3 * 8 + 4: return adjoint_step_points<3, 4>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 2 * 8 + 5: return adjoint_step_points<2, 5>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 2 * 8 + 6: return adjoint_step_points<2, 6>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 2 * 8 + 7: return adjoint_step_points<2, 7>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 2 * 8 + 8: return adjoint_step_points<2, 8>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 3 * 8 + 5: return adjoint_step_points<3, 5>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 3 * 8 + 6: return adjoint_step_points<3, 6>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 3 * 8 + 7: return adjoint_step_points<3, 7>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    case 3 * 8 + 8: return adjoint_step_points<3, 8>(f, src, rcv, state, state_prev, b, step, have_pp, residual, st, pp_next);
    default: return hipErrorInvalidValue;
    }
}


hipError_t launch_adjoint_gradient(const StepArgs &f, const AdjointBuffers &b, hipStream_t st)
{
    AdjArgs A;
    std::memset(&A, 0, sizeof(A));
    A.f = f;
    A.gk = b.gk;
    const dim3 block = adj_block();
    const dim3 grid(point_grid(A, block));
    hipLaunchKernelGGL(adj_grad_c, grid, block, 0, st, A, b.out);
    return hipGetLastError();
}

}  // namespace fw2
