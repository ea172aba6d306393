// gfx950 kernels of the discrete adjoint of one time step (time-centred
// memory scheme), for the gradient of J = 1/2 sum (trace - obs)^2 with
// respect to kappa0 (and through it the sound speed).
//
// The memory-variable recursion is dissipative, so running the forward
// scheme backwards in time does not give its adjoint (Sec. 5, full waveform
// inversion): the reverse step here is the transpose of the forward step's
// linearisation, taken phase by phase in
// reverse order, about the forward state at the step's input:
//   A0  pressure points: recompute S = sum_a (w2 D^-v_a + sum psi2) and
//       p'' = p - dt S / K (+ sources, A_src), K = kappa0 (1 + kappa0 B p),
//       kappa0 B = nlq (B = 1 - 2 beta as printed; B does not depend on kappa0)
//   A1  v points inside the grid: velocity phase reversed, pointwise:
//       Q = rho_a (1 + A kappa0_a pbar) (A = 1 as printed),
//       lam_S' = -dt lam_v / Q, lam_Q = dt S' lam_v / Q^2, lam_psi1 <- lam_S' + b1 lam_psi1,
//       and per axis the adjoint of D^+ p'' and lam_Q rho_a A, from which the
//       adjoints of pbar (lam_Q rho_a A kappa0_a) and kappa0_a
//       (lam_Q rho_a A pbar) follow where they are gathered
//   A_rcv  lam_p[R] += trace_n - obs_n
//   A2  pressure points: lam_p'' = lam_p - sum_a D^-(lam_D'_a) + means of lam_pbar,
//       gradient from the velocity multipliers, then the pressure phase
//       reversed: lam_S = -dt lam_p''/K, lam_K = dt S lam_p''/K^2,
//       lam_p = lam_p'' + lam_K kappa0 nlq,
//       grad += lam_K (1 + 2 nlq p), lam_psi2 <- lam_S + b2 lam_psi2,
//       lam_D_a = w2 lam_S + sum c2 lam_psi2 (new)
//   A3  v points inside the grid: lam_v_a -= D^+(lam_D_a)
// using (D^-)^T = -(D^+) and (D^+)^T = -(D^-).
// The phases run as one-thread-per-point kernels, two per step: A3 of a step
// is deferred into the velocity kernel (A1) of the next call, A_rcv runs in
// extra blocks of that kernel, and A0 of the step before is fused into the
// pressure kernel (A2) when its state is at hand, writing that step's p''
// into the second p'' buffer (this step's is still read by neighbours).
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
    float *pp;               // p'' of this step (forward recompute)
    float *pq;               // p'' of the step before (written by the fused A0)
    float *sS;               // S of the pressure phase (forward recompute)
    float *lDv;              // [ndim] adjoint of D^+ p'' at v points
    float *lqr;              // [ndim] lam_Q rho_a at v points
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
        float *oDv = A.lDv + a * st, *oqr = A.lqr + a * st;
        if (c3[a] == g.n[a] - 1) {                       // outside the grid: no adjoint flow
            oDv[idx] = 0.0f;
            oqr[idx] = 0.0f;
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
        const float Q = rho_a * (1.0f + (A.f.nlA * kap_a) * pbar);
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
        oqr[idx] = (lQ * rho_a) * A.f.nlA;      // the multiplier's coefficient A folded in
    }
}

// A2: gather of the velocity-phase adjoints, then the pressure phase reversed.
// The adjoints of pbar and kappa0_a at the two v points of each axis are
// lam_Q rho_a times kappa0_a and pbar, recomputed here from kappa0 and this
// step's p'' as the velocity phase formed them.  WITH_A0: then A0 of the step
// before at the same point, from the state sq, into the second p'' buffer
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
        // v points idx (between idx and idx + o) and idx - o
        const float q1 = A.lqr[a * st + idx], q0 = A.lqr[a * st + idx - o];
        const float k1 = 0.5f * (A.f.kap[idx] + A.f.kap[idx + o]);
        const float k0 = 0.5f * (A.f.kap[idx - o] + A.f.kap[idx]);
        const float b1 = 0.5f * (A.pp[idx] + A.pp[idx + o]);
        const float b0 = 0.5f * (A.pp[idx - o] + A.pp[idx]);
        lpp += 0.5f * (q1 * k1 + q0 * k0);
        gk += 0.5f * (q1 * b1 + q0 * b0);
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
        A.pq[idx] = q0 - A.f.dt * S0 / K0;
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
    A.pq = b.pq;
    A.sS = b.sS;
    A.lDv = b.lDv;
    A.lqr = b.lqr;
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
            hipLaunchKernelGGL(adj_sources, dim3((src.n + 255) / 256), dim3(256), 0, st, b.pq, src, step - 1);
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
