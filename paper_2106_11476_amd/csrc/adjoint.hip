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
#include "kernels.hpp"

#include <cstring>

namespace fw2 {

namespace {

constexpr int kABX = 64, kABY = 4;

struct AdjArgs {
    StepArgs f;              // medium, tables, stencil of the domain (f.p etc. unused)
    const float *sp;         // forward state at the step input: p, v, psi1, psi2 blocks
    float *lp;               // adjoint state: same layout
    float *pp;               // p'' (forward recompute)
    float *sS;               // S of the pressure phase (forward recompute)
    float *lDv;              // [ndim] adjoint of D^+ p'' at v points
    float *lpb;              // [ndim] adjoint of pbar
    float *lkv;              // [ndim] adjoint of kappa0_a
    float *lDp;              // [ndim] adjoint of D^- v_a at p points
    float *gk;               // dJ/dkappa0
    int L;
};

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
    const int i = blockIdx.x * kABX + threadIdx.x;                                 \
    const int j = blockIdx.y * kABY + threadIdx.y;                                 \
    const int k = blockIdx.z;                                                      \
    if (i >= g.n[0] || j >= g.n[1]) return;                                        \
    const int c3[3] = {i, j, k};                                                   \
    const int nd = g.ndim;                                                         \
    const int64_t idx = g.origin + (int64_t)k * g.plane + (int64_t)j * g.pitch + i; \
    const int lab = A.f.label ? (int)A.f.label[idx] : 0;                           \
    const int L = A.L;                                                             \
    (void)c3;                                                                      \
    (void)lab;

// A0: forward recompute of the pressure phase (without sources).
__global__ void __launch_bounds__(kABX *kABY) adj_forward_p(const AdjArgs A)
{
    ADJ_POINT
    const int64_t st = g.stride;
    const float *v = A.sp + st;
    const float *m2 = A.sp + (int64_t)(1 + nd + nd * L) * st;
    float S = 0.0f;
    for (int a = 0; a < nd; ++a) {
        const float D = dminus(v + a * st, g, A.f.g, A.f.g11, a, nd, idx);
        const int t = slot_p(c3[a], g.n[a], A.f.nb[a]) * A.f.n_labels + lab;
        float Sa = A.f.w2[a][t] * D;
        for (int nu = 0; nu < L; ++nu) Sa += m2[(int64_t)(a * L + nu) * st + idx];
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

// A1: velocity phase reversed at v points.
__global__ void __launch_bounds__(kABX *kABY) adj_velocity(const AdjArgs A)
{
    ADJ_POINT
    const int64_t st = g.stride;
    const float *m1 = A.sp + (int64_t)(1 + nd) * st;
    float *lv = A.lp + st;
    float *lm1 = A.lp + (int64_t)(1 + nd) * st;
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
        for (int nu = 0; nu < L; ++nu) Sv += m1[(int64_t)(a * L + nu) * st + idx];
        const float pbar = 0.5f * (A.pp[idx] + A.pp[idx + o]);
        const float rho_a = 0.5f * (A.f.rho[idx] + A.f.rho[idx + o]);
        const float kap_a = 0.5f * (A.f.kap[idx] + A.f.kap[idx + o]);
        const float Q = rho_a * (1.0f + kap_a * pbar);
        const float lva = lv[a * st + idx];
        const float lS = -A.f.dt * lva / Q;
        const float lQ = A.f.dt * Sv * lva / (Q * Q);
        float lD = w * lS;
        for (int nu = 0; nu < L; ++nu) {
            const int64_t c = (int64_t)(a * L + nu) * st + idx;
            const float2 q = bc[nu];
            const float lmn = lm1[c];
            lD = fmaf(q.y, lmn, lD);
            lm1[c] = fmaf(q.x, lmn, lS);
        }
        oDv[idx] = lD;
        opb[idx] = lQ * rho_a * kap_a;
        okv[idx] = lQ * rho_a * pbar;
    }
}

__global__ void adj_receivers(float *lp, const SparseArgs r, const float *__restrict__ residual)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= r.n) return;
    atomicAdd(&lp[pidx(r.geo, r.idx[q])], residual[q]);
}

// A2: gather of the velocity-phase adjoints, then the pressure phase reversed.
__global__ void __launch_bounds__(kABX *kABY) adj_pressure(const AdjArgs A)
{
    ADJ_POINT
    const int64_t st = g.stride;
    float lpp = A.lp[idx];
    float gk = A.gk[idx];
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
    for (int a = 0; a < nd; ++a) {
        const int t = slot_p(c3[a], g.n[a], A.f.nb[a]) * A.f.n_labels + lab;
        const float2 *bc = A.f.bc2[a] + (int64_t)t * L;
        float lD = A.f.w2[a][t] * lS;
        for (int nu = 0; nu < L; ++nu) {
            const int64_t c = (int64_t)(a * L + nu) * st + idx;
            const float2 qq = bc[nu];
            const float lmn = lm2[c];
            lD = fmaf(qq.y, lmn, lD);
            lm2[c] = fmaf(qq.x, lmn, lS);
        }
        A.lDp[a * st + idx] = lD;
    }
}

// A3: lam_v_a -= D^+(lam_D_a) at v points inside the grid.
__global__ void __launch_bounds__(kABX *kABY) adj_vel_from_p(const AdjArgs A)
{
    ADJ_POINT
    const int64_t st = g.stride;
    float *lv = A.lp + st;
    for (int a = 0; a < nd; ++a) {
        if (c3[a] == g.n[a] - 1) continue;
        lv[a * st + idx] -= dplus(A.lDp + a * st, g, A.f.g, A.f.g11, a, nd, idx);
    }
}

// dJ/dc = dJ/dkappa0 * (-2 kappa0 / c), with c = 1/sqrt(rho kappa0).
__global__ void __launch_bounds__(kABX *kABY) adj_grad_c(const AdjArgs A, float *out)
{
    ADJ_POINT
    const float x = A.f.kap[idx];
    out[idx] = A.gk[idx] * (-2.0f * x * sqrtf(A.f.rho[idx] * x));
}

}  // namespace

hipError_t launch_adjoint_step(const StepArgs &f, const SparseArgs &src, const SparseArgs &rcv, int L,
                               const float *state, const AdjointBuffers &b, long long step,
                               const float *residual, hipStream_t st)
{
    AdjArgs A;
    A.f = f;
    A.sp = state;
    A.lp = b.lp;
    A.pp = b.pp;
    A.sS = b.sS;
    A.lDv = b.lDv;
    A.lpb = b.lpb;
    A.lkv = b.lkv;
    A.lDp = b.lDp;
    A.gk = b.gk;
    A.L = L;
    const Geometry &g = f.geo;
    dim3 block(kABX, kABY), grid((g.n[0] + kABX - 1) / kABX, (g.n[1] + kABY - 1) / kABY, g.n[2]);
    hipLaunchKernelGGL(adj_forward_p, grid, block, 0, st, A);
    if (src.n > 0)
        hipLaunchKernelGGL(adj_sources, dim3((src.n + 255) / 256), dim3(256), 0, st, b.pp, src, step);
    hipLaunchKernelGGL(adj_velocity, grid, block, 0, st, A);
    if (rcv.n > 0 && residual)
        hipLaunchKernelGGL(adj_receivers, dim3((rcv.n + 255) / 256), dim3(256), 0, st, b.lp, rcv, residual);
    hipLaunchKernelGGL(adj_pressure, grid, block, 0, st, A);
    hipLaunchKernelGGL(adj_vel_from_p, grid, block, 0, st, A);
    return hipGetLastError();
}

hipError_t launch_adjoint_gradient(const StepArgs &f, const AdjointBuffers &b, hipStream_t st)
{
    AdjArgs A;
    std::memset(&A, 0, sizeof(A));
    A.f = f;
    A.gk = b.gk;
    const Geometry &g = f.geo;
    dim3 block(kABX, kABY), grid((g.n[0] + kABX - 1) / kABX, (g.n[1] + kABY - 1) / kABY, g.n[2]);
    hipLaunchKernelGGL(adj_grad_c, grid, block, 0, st, A, b.out);
    return hipGetLastError();
}

}  // namespace fw2
