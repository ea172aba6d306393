// Device data layout and kernel launchers of libfw2.
//
// Every per-point array (fields, memory variables, medium, labels) uses one
// padded layout: a 4-cell zero halo on each side of every axis, rows of
// `pitch` elements (a multiple of 64, so rows start on 256-byte boundaries),
// planes of `plane` = pitch * (ny + 8) elements (3D).  Element (x, y, z) is at
// origin + z * plane + y * pitch + x, and the arrays are placed so that x = 0
// of every row is 256-byte aligned.  The halo of p and v is never written, so
// stencil taps read zero outside the grid without bounds checks.  A slab of a
// grid split along z is the exception: its z halo planes hold the
// neighbouring slabs' planes, written by the halo exchange.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fw2 {

constexpr int kHalo = 4;

// Memory variables are read and written once per step, by one kernel:
// non-temporal accesses keep them from displacing the stencil fields that
// the other kernel of the step reads back from cache.
__device__ __forceinline__ float ntld(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void ntst(float *p, float v) { __builtin_nontemporal_store(v, p); }

struct Geometry {
    int32_t ndim;
    int32_t n[3];            // nx, ny, nz (nz = 1 in 2D)
    int64_t pitch, plane;    // element strides of y and z
    int64_t origin;          // element offset of (0, 0, 0)
    int64_t stride;          // elements between consecutive arrays
};

struct SparseArgs {
    Geometry geo;
    float *p;
    long long *step;         // device step counter
    const int64_t *idx;      // flat unpadded indices
    const int32_t *sig;      // sources: signal of each point
    const float *w;          // sources: weight of each point
    const float *signals;    // sources: [n_sig][n_t]
    float *trace;            // receivers: [cap][n]
    int32_t n;               // points
    int32_t n_t;             // sources: samples per signal
    long long cap;           // receivers: trace rows
};

struct StepArgs {
    Geometry geo;
    float *p;
    float *v;                // v_a = v + a * stride
    float *psi1;             // psi1[a][nu] = psi1 + (a * L + nu) * stride
    float *psi2;
    // Element offset from the fields a phase reads to those it writes: 0 steps
    // in place; an out-of-place step reads one state block and writes the next.
    int64_t out;
    const float *kap;        // kappa0 = 1 / (rho c^2)
    const float *nlq;        // kappa0 B, B = 1 - 2 beta as printed
    const float *rho;        // rho0
    const uint8_t *label;    // nullptr: a single relaxation tuple
    int32_t n_labels;
    int32_t nb[3];           // boundary cells per axis
    const float *w2[3];      // pressure-point tables per axis: [slot][label]
    const float2 *bc2[3];    //   [slot][label][nu] (b, c)
    const float *w1[3];      // velocity-point tables per axis
    const float2 *bc1[3];
    float g[4];              // g_m0 / h
    float g11;               // g_11 / h
    float dt;
    // Momentum multiplier rho_a (1 + nlA kappa0_a pbar); nlA = 1 as printed.
    // (The mass multiplier's coefficient is folded into nlq.)
    float nlA;
    // Slab of a grid split along z: local plane k is global plane k + z_off
    // of nz_glob planes (the boundary layer and the last v_z sample follow
    // the global index).  A whole grid has z_off = 0, nz_glob = n[2].
    int32_t z_off, nz_glob;
    // Per-point stencil weights (local_stencil != 0): with s = r^2 of the
    // point, g_m0(s) / h = sum_k pw[m-1][k] s^k and g_11(s) / h = g11s * s;
    // a cell's s = q2 / (rho kappa0), q2 = (dt / h)^2.
    int32_t local_stencil;
    float pw[4][4];
    float g11s;
    float q2;
    // Receivers recorded (and the step counter advanced) by one extra block
    // of the velocity sweep launch, which reads p without writing it and runs
    // after the sources; rcv.step == nullptr: a separate launch does it.
    SparseArgs rcv;
};


// Kernel variant and tile shape.  variant 0: one thread per point over a
// (64 x 8) tile, every stencil tap a cached global load (any ndim).
// variant 1 (2D): row sweeps of `bx` columns x `rows` rows with a register
// window along y and LDS rings along x; variant 2: the same with the next
// row's loads issued before the current row is computed.  variant 1 (3D):
// plane sweeps of a column tile (32x16, 64x8 or 16x16 for bx = 32, 64, 16)
// over `rows` planes with a register window along z and LDS plane rings;
// variant 2 (3D): the same with every load of the next plane issued during
// the current one; variant 3 (3D): only the staged planes and the z window
// one plane ahead, the point's own values at the top of their plane.
struct KernelConfig {
    int variant;
    int bx;
    int rows;
    int by = 0;              // 3D: tile rows in y (0: the default of bx)
};

// Many 2D domains advanced by one launch per phase (batched serving).  The
// table lives in device memory; blocks of a fixed, persistent grid walk all
// tiles of all entries, so a captured step loop does not depend on which
// domains are active.  A domain whose step counter has reached n_steps is
// skipped (its counter keeps counting while it stays in the table).
constexpr int kMaxBatch = 64;

struct BatchEntry {
    StepArgs a;
    SparseArgs src, rcv;
    long long n_steps;
    int32_t L, scheme;
    int32_t tile_base, tiles;        // tiles of bx columns x rows
};

struct BatchTable {
    int32_t n;
    int32_t total_tiles;
    int32_t rows;                    // tile rows; tile columns bx = 64 or 256
    // Entries are ordered by launch class; the tiles of class c are
    // [class_begin[c], class_end[c]) of the tile list.
    int32_t class_begin[4], class_end[4];
    BatchEntry e[kMaxBatch];
};

// Launch class of a batch entry: bit 0 for 5..8 mechanisms, bit 1 for
// per-point stencil weights.
__host__ __device__ inline int batch_class(int L, int local_stencil)
{
    return (L > 4 ? 1 : 0) | (local_stencil ? 2 : 0);
}

// One step of every entry.  classes: bit c set when the table holds entries
// of class c (classes 1 and 3 need bx = 256).
hipError_t launch_batch_step(const BatchTable *dev_table, int n_entries_max, int bx, unsigned classes,
                             hipStream_t stream);
// Sizes the persistent grids of the batch kernels (occupancy queries); call
// outside stream capture before the first batched step.
void prepare_batch_launches();
// The library's own batch table on `device` (the current device), for a
// batch that allocates nothing: *busy is set (and *table left NULL) while
// another such batch holds it.  Released by release_static_batch_table.
hipError_t claim_static_batch_table(int device, BatchTable **table, bool *busy);
void release_static_batch_table(int device);

// Discrete adjoint of one step (adjoint.hip): device arrays of the adjoint
// state (same layout as the forward state block) and the per-step temporaries.
struct AdjointBuffers {
    float *lp, *pp, *pq, *sS, *lDv, *lqr, *lDp, *gk, *out;
};
// One reverse step.  state: forward state block at the step's input;
// state_prev: that of the step before, or nullptr.  have_pp: b.pp / b.sS
// already hold this step's p'' and S (from the previous call); *pp_next is
// set when b.pq / b.sS now hold those of step - 1 (the caller then swaps
// b.pp and b.pq).
hipError_t launch_adjoint_step(const StepArgs &f, const SparseArgs &src, const SparseArgs &rcv, int L,
                               const float *state, const float *state_prev, const AdjointBuffers &b,
                               long long step, bool have_pp, const float *residual, hipStream_t stream,
                               bool *pp_next);
hipError_t launch_adjoint_gradient(const StepArgs &f, const AdjointBuffers &b, hipStream_t stream);

// Per-dimension, per-phase launchers (step_p2/v2/p3/v3.hip), called by
// launch_pressure / launch_velocity.
hipError_t launch_pressure_2d(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t stream);
hipError_t launch_velocity_2d(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t stream);
hipError_t launch_pressure_3d(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t stream);
hipError_t launch_velocity_3d(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t stream);

// Launchers (kernels.hip).  All enqueue on `stream` and return the launch error.
hipError_t launch_pressure(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t stream);
hipError_t launch_velocity(const StepArgs &a, int L, int scheme, const KernelConfig &kc, hipStream_t stream);
hipError_t launch_sources(const SparseArgs &s, hipStream_t stream);
hipError_t launch_receivers(const SparseArgs &s, hipStream_t stream);   // also advances the counter
hipError_t launch_fill(float *dst, int64_t n, float value, hipStream_t stream);
hipError_t launch_check(const float *p, const Geometry &g, float limit, int *flag, hipStream_t stream);
hipError_t launch_set_counter(long long *counter, long long value, hipStream_t stream);

// Halo planes of a slab (halo.hip).  A plane set lists `n` (array, first
// plane, plane count) ranges; pack gathers their unpadded [ny][nx] planes in
// order into dst, unpack scatters src back into the same planes.
struct PlaneSet {
    const float *arr[4];
    int32_t z0[4];
    int32_t nz[4];
    int32_t n;
    int32_t total;           // sum of nz
};
hipError_t launch_pack(const PlaneSet &s, const Geometry &g, float *dst, hipStream_t stream);
hipError_t launch_unpack(const PlaneSet &s, const Geometry &g, const float *src, hipStream_t stream);

// Medium from device maps (halo.hip): kappa0 = 1/(rho c^2), kappa0 (B0 + B1
// beta) and rho into the padded arrays (FP64 arithmetic, FP32 results, the
// host conversion's operation order), labels copied; stats[0] / [1] receive
// the bits of the largest / smallest c (atomics on the bit patterns of
// positive floats) and stats[2] a nonzero flag for an invalid sample.
struct MediumArgs {
    Geometry geo;
    const float *c, *rho, *beta;
    const uint8_t *label;    // nullptr: none
    float *kap, *nlq, *rhop;
    uint8_t *labp;           // nullptr: not stored
    double B0, B1;
    int32_t n_labels;
    unsigned int *stats;     // [3], zeroed by the caller
};
hipError_t launch_medium(const MediumArgs &m, hipStream_t stream);

}  // namespace fw2
