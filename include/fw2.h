/*
 * fw2.h -- C ABI of libfw2, the gfx950 time stepper of the Fullwave 2 system
 * (Sode & Pinton, arXiv 2106.11476): the first-order nonlinear acoustic
 * equations with coordinate-stretched derivatives (Sec. 2.2, Eqs. general5 and
 * general6) on a staggered grid with the (8,4) stencil (Sec. 3.1), memory
 * variables for L relaxation mechanisms (Sec. 3.2) and the two-stage C-PML
 * with its transition layer (Sec. 3.3, Table 1).
 *
 * Conventions
 *   - Grids are x fastest: flat index = x + nx * (y + ny * z); nz = 1 in 2D.
 *   - Pressure p sits at integer positions; v_a (a = x, y, z) sits half a cell
 *     along a.  The v_a sample past the last pressure sample along a lies
 *     outside the grid and is held at zero.  Fields outside the grid are zero.
 *   - All device arithmetic is FP32; derived coefficients are computed in FP64
 *     during fw2_create_domain (on the host, or on the GPU for device maps).
 *   - A slab domain (slab_nz > 0) is the exception to "zero outside the grid"
 *     along z: its z halos hold the neighbouring slabs' planes.
 *   - Every call returns fw2_status; nothing throws across the ABI.  On error
 *     fw2_last_error() returns a message for the calling thread.
 *   - A domain is not thread-safe; distinct domains may be used from
 *     different threads and streams at the same time.
 */
#ifndef FW2_H
#define FW2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fw2_domain fw2_domain;

typedef enum {
    FW2_OK = 0,
    FW2_E_INVALID = 1,      /* bad argument; nothing was changed */
    FW2_E_NOMEM = 2,        /* workspace too small or host allocation failed */
    FW2_E_HIP = 3,          /* a HIP runtime call failed */
    FW2_E_STATE = 4,        /* call not valid in the domain's current state */
    FW2_E_UNSTABLE = 5,     /* watchdog found a non-finite or runaway field */
    FW2_E_UNSUPPORTED = 6   /* valid request the library does not implement */
} fw2_status;

#define FW2_MAX_RELAX 8     /* largest number of relaxation mechanisms L */
#define FW2_MAX_LABELS 256  /* relaxation tuples addressable by a uint8 label */

/* Field selection for fw2_read_fields / fw2_write_fields.  Selected fields
 * are packed in this order, each as FP32 [nz][ny][nx] arrays:
 *   P: p;  V: v_x, v_y[, v_z];  PSI1: psi1[axis][mechanism] (nabla_1 memory
 *   variables, at the v points);  PSI2: psi2[axis][mechanism] (nabla_2, at the
 *   p points). */
enum {
    FW2_FIELD_P = 1u,
    FW2_FIELD_V = 2u,
    FW2_FIELD_PSI1 = 4u,
    FW2_FIELD_PSI2 = 8u,
    FW2_FIELD_ALL = 15u
};

/* Memory pointer kinds. */
enum { FW2_HOST = 0, FW2_DEVICE = 1 };

/* Evaluation of the memory variables (Sec. 3.2).
 *   FW2_RELAX_PRINTED: Eq. relaxation_psi as printed, psi^n = b psi^{n-1} +
 *     a D^{n-1/2}, the updated psi used in the same step.
 *   FW2_RELAX_CENTRED: the same exponential convolution evaluated at the time
 *     of the newest derivative sample, with the derivative linear between
 *     samples; same state and cost, and it reproduces the dispersion relation
 *     (Eq. dispersion_relations), which the printed form misses by about a
 *     fifth of the attenuation at 12 points per wavelength, CFL 0.4. */
enum { FW2_RELAX_PRINTED = 0, FW2_RELAX_CENTRED = 1 };

/* Nonlinear terms (Sec. 2.2, Eqs. state1 and state2): the momentum update
 * divides by rho0 (1 + A kappa0 p), the mass update by kappa0 (1 + kappa0 B p).
 *   FW2_NL_PRINTED: A = 1, B = 1 - 2 beta, the equations of state as printed
 *     (the default of a zero-initialised descriptor).  Their plane-wave
 *     coefficient of nonlinearity is beta - 1 (a simple wave of the printed
 *     system travels at 1/sqrt(rho(p) kappa(p))).
 *   FW2_NL_CUSTOM: A = nl_A, B = nl_B0 + nl_B1 beta.  A = 0, B = -2 beta gives
 *     the plane-wave coefficient beta, that of the Westervelt equation to
 *     which Sec. 2.2 reduces the system once the locally nonlinear terms are
 *     dropped. */
enum { FW2_NL_PRINTED = 0, FW2_NL_CUSTOM = 1 };

/* Stencil weights (Sec. 3.1: the (8,4) operator of a time-space design whose
 * weights depend on the Courant number r = c dt / h).
 *   FW2_STENCIL_GLOBAL: one set for the grid, at r = fd_r (or max(c) dt / h).
 *   FW2_STENCIL_LOCAL: every point uses the set of its own r: a pressure
 *     point r^2 = (c dt / h)^2 of its cell, a velocity point the mean of the
 *     r^2 of the two cells it lies between.  The weights are fixed cubic
 *     polynomials in r^2 (the Taylor conditions are linear in the weights
 *     with right-hand side 1, r^2, r^4, r^6), evaluated in the kernels from
 *     rho and kappa0; fd_r is then unused.  Not available to the adjoint
 *     (FW2_E_UNSUPPORTED there). */
enum { FW2_STENCIL_GLOBAL = 0, FW2_STENCIL_LOCAL = 1 };

typedef struct {
    int32_t ndim;             /* 2 or 3 */
    int32_t n_relax;          /* L, 1..FW2_MAX_RELAX */
    int64_t n[3];             /* nx, ny, nz including the boundary layers; nz = 1 in 2D;
                                 each 1..2^20; a padded plane must stay addressable with
                                 32-bit byte offsets: (nx + 72)(ny + 8) < 2^30 in 2D and
                                 < 2^29 in 3D (FW2_E_INVALID otherwise) */
    double h;                 /* grid step (m) */
    double dt;                /* time step (s) */
    int32_t bound_cells[3];   /* L_C-PML per side per axis, in cells (Sec. 3.3) */
    int32_t trans_cells[3];   /* L_Transition per side per axis, 0..bound_cells */
    double pml_Rc;            /* R_c of Table 1's d target, 0 < R_c < 1 */
    int32_t pml_npoly;        /* polynomial order N of Eq. polynomial_transition, >= 1 */
    double pml_cp;            /* c_p of Table 1's d target; <= 0: largest c of the map */
    double fd_r;              /* Courant number of the (8,4) weights; <= 0: max(c) dt / h */
    int32_t relax_scheme;     /* FW2_RELAX_PRINTED or FW2_RELAX_CENTRED */
    int32_t stencil_mode;     /* FW2_STENCIL_GLOBAL or FW2_STENCIL_LOCAL */
    const float *c;           /* [nz][ny][nx] sound speed (m/s), > 0 (host or device: map_kind) */
    const float *rho;         /* [nz][ny][nx] equilibrium density rho_0 (kg/m^3), > 0 */
    const float *beta;        /* [nz][ny][nx] coefficient of nonlinearity 1 + B/2A */
    const uint8_t *label;     /* [nz][ny][nx] relaxation-tuple index, or NULL (all 0) */
    int32_t n_labels;         /* rows of relax_table, 1..FW2_MAX_LABELS */
    const double *relax_table;/* host [n_labels][2 + 4L]: k1, k2, d1[L], d2[L], alpha1[L],
                                 alpha2[L] -- the 2 + 4L isotropic parameters of Sec. 3.2 */
    void *stream;             /* hipStream_t for all work of the domain; NULL = null stream */
    int32_t nonlinear_form;   /* FW2_NL_PRINTED (0) or FW2_NL_CUSTOM */
    double nl_A, nl_B0, nl_B1;/* FW2_NL_CUSTOM coefficients (finite); ignored otherwise */
    int32_t map_kind;         /* FW2_HOST (0): c, rho, beta, label are host arrays;
                                 FW2_DEVICE: device arrays, converted on the GPU (same
                                 FP64 arithmetic, bitwise the same domain) */
    int64_t slab_z0;          /* slab_nz > 0: this domain is planes [slab_z0, slab_z0 + nz)   */
    int64_t slab_nz;          /*   of a 3D grid of slab_nz planes (see the slab calls below); */
                              /*   0: the domain is the whole grid                           */
} fw2_domain_desc;

/* Bytes of device workspace a domain described by desc needs (host-only
 * computation; validates desc).  Returns FW2_E_INVALID for a bad desc. */
fw2_status fw2_workspace_bytes(const fw2_domain_desc *desc, uint64_t *bytes);

/* Create a domain (Sec. 3 setup: stencil weights from r, per-tissue and
 * per-boundary-position memory coefficients from Eqs. relaxation_a / _b and
 * Table 1's profiles, medium values from c, rho, beta).
 *   dev_workspace: caller-owned device buffer of at least fw2_workspace_bytes,
 *     256-byte aligned; it must outlive the domain.  The library performs no
 *     device allocation of its own beyond HIP events and graphs.
 *   The host maps are read during the call and may be freed afterwards.
 *   All fields start at zero; the step counter starts at 0.
 *   Rejects a time step above the scheme's stability limit (FW2_E_INVALID). */
fw2_status fw2_create_domain(const fw2_domain_desc *desc, void *dev_workspace,
                             uint64_t workspace_bytes, fw2_domain **out);

/* Additive pressure sources (reading of the source model: the paper names the
 * pulse, not the injection).  After the pressure update of step k (0-based),
 * p[flat_idx[q]] += weight[q] * signals[sig_id[q]][k] for k < n_t.
 *   flat_idx, sig_id, weight, signals: caller-owned DEVICE arrays that must
 *     stay valid while the domain steps; flat indices must be distinct and in
 *     range, sig_id in [0, n_sig) (checked here with a device-to-host copy).
 *   A call replaces the previous source set; n_pts = 0 removes all sources. */
fw2_status fw2_add_source(fw2_domain *dom, int32_t n_pts, const int64_t *flat_idx,
                          const int32_t *sig_id, const float *weight, int32_t n_sig,
                          int32_t n_t, const float *signals);

/* Pressure receivers (library infrastructure: the paper's experiments record
 * the pressure at receiving positions, e.g. the echoes of Sec. 5's transmit
 * events): after the sources of step k, trace[k][r] = p[flat_idx[r]]
 * for k < cap_steps (rows are global step indices).
 *   flat_idx and trace: caller-owned DEVICE arrays, trace is [cap_steps][n_rcv]
 *   FP32.  A call replaces the previous receiver set; n_rcv = 0 removes it. */
fw2_status fw2_add_receivers(fw2_domain *dom, int32_t n_rcv, const int64_t *flat_idx,
                             float *trace, int64_t cap_steps);

/* Advance n >= 0 steps, asynchronously on the domain's stream.  One step is
 * the pressure phase, sources, receivers, then the velocity phase (Sec. 3.1
 * leapfrog).  After fw2_step(n) from a zero state p is at t = n dt and v at
 * (n + 1/2) dt. */
fw2_status fw2_step(fw2_domain *dom, int32_t n);

/* Copy the selected fields (order of the FW2_FIELD_ enum) into dst, packed,
 * unpadded FP32 (the state of Sec. 3.1's scheme: p, v and the memory variables
 * of Sec. 3.2).  dst_kind FW2_HOST or FW2_DEVICE.  Synchronises the stream.
 * FW2_E_STATE for a NULL domain, FW2_E_INVALID for a bad mask, kind or NULL
 * dst. */
fw2_status fw2_read_fields(fw2_domain *dom, uint32_t field_mask, void *dst, int32_t dst_kind);

/* Overwrite the selected fields from src (same packing; library
 * infrastructure for checkpoint and resume of Sec. 3.1's state).  Values at v
 * samples outside the grid are ignored (kept zero).  Synchronises the stream.
 * Errors as fw2_read_fields. */
fw2_status fw2_write_fields(fw2_domain *dom, uint32_t field_mask, const void *src, int32_t src_kind);

/* Library infrastructure.  Global index of the next step (sources and
 * receivers use it); -1 for a NULL domain. */
int64_t fw2_current_step(const fw2_domain *dom);

/* Library infrastructure.  Set the global step index (resume from a
 * checkpoint).  Synchronises.  FW2_E_INVALID for step < 0. */
fw2_status fw2_set_current_step(fw2_domain *dom, int64_t step);

/* Library infrastructure.  Move the domain to another stream: finishes the work queued on its current
 * stream, then queues every later call of this domain (steps, transfers,
 * checkpoints, the adjoint) on stream (NULL: the default stream).  The caller
 * keeps the stream alive while the domain uses it.  A domain can be built on
 * a setup stream while other work runs, then stepped on a serving stream. */
fw2_status fw2_set_stream(fw2_domain *dom, void *stream);

/* Library infrastructure.  Steps captured per HIP graph replay (0 disables graphs; default 32).
 * Graph and direct launches give bitwise identical results. */
fw2_status fw2_set_graph_chunk(fw2_domain *dom, int32_t steps);

/* Library infrastructure (measurement).  Per-kernel HIP-event timing on the domain's stream.  While enabled, steps
 * are launched directly (no graphs) with events around the pressure and
 * velocity kernels.  fw2_get_kernel_timing synchronises and returns the total
 * milliseconds and launch counts since timing was enabled:
 * index 0 = pressure kernel, 1 = velocity kernel. */
fw2_status fw2_enable_kernel_timing(fw2_domain *dom, int32_t enable);
fw2_status fw2_get_kernel_timing(fw2_domain *dom, double ms[2], int64_t count[2]);

/* Library infrastructure (watchdog): synchronises and checks that every
 * pressure sample is finite and below limit in magnitude; FW2_E_UNSTABLE
 * otherwise. */
fw2_status fw2_check_finite(fw2_domain *dom, float limit);

/* ---- State blocks and the discrete adjoint ------------------------------
 * The state of a domain (p, v, psi1, psi2 in the library's padded layout) is
 * one contiguous block of fw2_state_bytes bytes.  fw2_save_state copies it to
 * a caller-owned device buffer and fw2_load_state copies one back and sets
 * the step counter (both asynchronous on the domain's stream): checkpoints.
 *
 * fw2_step_into advances n steps out of place through caller-owned state
 * blocks, for recomputing the forward states between two checkpoints (the
 * checkpointed recomputation of the adjoint below; library infrastructure):
 * step i (i = 0..n-1) reads block i-1 (dev_first for i = 0) and writes block
 * i of dev_states (n consecutive blocks of fw2_state_bytes), i.e. block i
 * holds the state after step s + i + 1 when dev_first holds the state at the
 * domain's current step s.  Sources are added and receivers recorded as in
 * fw2_step, and the step counter advances by n; the domain's own fields are
 * neither read nor written (they stay at step s: fw2_load_state before
 * stepping the domain itself again).  Only cells inside the grid are written,
 * so the cells outside it (the halo, and the last sample of each velocity
 * component and its psi1 along that component's axis) must hold zero in
 * every destination block, as in a zero-filled buffer or a block written by
 * fw2_save_state; they then stay zero.  Blocks need 4-byte alignment; at
 * 240 bytes past a 256-byte boundary (where the domain's own block starts)
 * every row starts on a cache line.  dev_first must not overlap the
 * destination blocks.
 * n = 0 does nothing (the pointers may then be NULL).
 * Asynchronous on the domain's stream; the n steps are captured in a HIP
 * graph (reused while dev_first, dev_states and n stay the same, dropped
 * when sources or receivers change) unless graphs are off
 * (fw2_set_graph_chunk 0) or kernel timing is on.  Errors: n < 0, a NULL or
 * misaligned block pointer, or an overlap: FW2_E_INVALID; a half-done step
 * (fw2_step_phase): FW2_E_STATE; slabs: FW2_E_UNSUPPORTED.
 *
 * The discrete adjoint (the paper's extension to full waveform inversion,
 * Sec. 5: the memory-variable recursion is dissipative, so the reverse step
 * is the transpose of the linearised forward step, not the scheme run
 * backwards) gives the gradient of J = 1/2 sum_k sum_r (trace[k][r] -
 * obs[k][r])^2 with respect to the sound-speed map.  It is the exact
 * transpose of the time-centred scheme's step (FW2_RELAX_CENTRED only;
 * FW2_E_UNSUPPORTED otherwise), linearised about the forward state; c enters
 * through kappa0 = 1/(rho c^2) (fd_r and pml_cp are fixed inputs).
 *   fw2_adjoint_begin: attaches a caller-owned device workspace of
 *     fw2_adjoint_workspace_bytes (256-byte aligned) and zeroes the adjoint
 *     state and the gradient.
 *   fw2_adjoint_step: reverse of forward step `step`, given the saved state
 *     block at that step's input and the device residual trace[step] - obs[step]
 *     ([n_rcv] FP32, or NULL for no residual).  Call for step = n-1 down to 0.
 *     dev_state_prev, if not NULL, is the state block at the input of step - 1:
 *     the library then recomputes that step's pressure phase in the same pass
 *     (the next call must be for step - 1; otherwise that work is redone).
 *     The buffers dev_state and dev_state_prev must stay unchanged until the
 *     work queued on the domain's stream has run.
 *   fw2_adjoint_gradient: dJ/dc, packed FP32 [nz][ny][nx] into dst (host or
 *     device); synchronises. */
fw2_status fw2_state_bytes(const fw2_domain *dom, uint64_t *bytes);
fw2_status fw2_save_state(fw2_domain *dom, void *dev_dst);
fw2_status fw2_load_state(fw2_domain *dom, const void *dev_src, int64_t step);
fw2_status fw2_step_into(fw2_domain *dom, int32_t n, const void *dev_first, void *dev_states);
fw2_status fw2_adjoint_workspace_bytes(const fw2_domain *dom, uint64_t *bytes);
fw2_status fw2_adjoint_begin(fw2_domain *dom, void *dev_workspace, uint64_t workspace_bytes);
fw2_status fw2_adjoint_step(fw2_domain *dom, const void *dev_state, const void *dev_state_prev, int64_t step,
                            const float *dev_residual);
fw2_status fw2_adjoint_gradient(fw2_domain *dom, float *dst, int32_t dst_kind);

/* ---- Batched stepping of many 2D domains (continuous batching) ----------
 * A batch advances several resident 2D domains of any sizes, L, memory
 * scheme and stencil mode with one launch per phase (two when domains with
 * more than four mechanisms are present: those run in a launch of their own,
 * in 256-column tiles): blocks of a fixed grid walk the tiles of every active
 * domain (the per-tile arithmetic is the single-domain sweep's,
 * so results are bitwise those of stepping each domain alone).  Each domain
 * stops by itself when its step counter reaches its own n_steps, so domains
 * with different step counts share step loops; the loop is captured as a HIP
 * graph that does not depend on which domains are active.
 *   fw2_batch_workspace_bytes: device bytes of the batch table for up to
 *     max_domains (1..64) domains; the caller allocates them (256-byte
 *     aligned) and keeps them alive while the batch exists.
 *   fw2_batch_set_domains: replaces the active set (synchronises the batch
 *     stream).  Every domain must be 2D, created on the same device, and at
 *     step < n_steps[k]; a domain that leaves the set gets its step counter
 *     back (fw2_current_step stays exact).  n = 0 empties the batch.
 *   fw2_batch_step: n steps of every active domain, asynchronously on the
 *     batch stream (the domains' own streams are not used meanwhile).
 *   fw2_batch_set_tile: tile of the batched sweep, cols = 64 or 256 columns by
 *     rows >= 1 rows; only while the batch is empty.
 * Errors: FW2_E_INVALID for bad arguments, FW2_E_UNSUPPORTED for 3D domains
 * and for domains with more than four mechanisms when the tile has 64
 * columns, FW2_E_HIP for runtime failures. */
typedef struct fw2_batch fw2_batch;
fw2_status fw2_batch_workspace_bytes(int32_t max_domains, uint64_t *bytes);
fw2_status fw2_batch_create(int32_t max_domains, void *dev_workspace, uint64_t workspace_bytes,
                            void *stream, fw2_batch **out);
fw2_status fw2_batch_set_domains(fw2_batch *b, int32_t n, fw2_domain *const *domains, const int64_t *n_steps);
fw2_status fw2_batch_step(fw2_batch *b, int32_t n);
fw2_status fw2_batch_set_tile(fw2_batch *b, int32_t cols, int32_t rows);
void fw2_batch_destroy(fw2_batch *b);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * it): fw2_batch_create without a workspace.  The batch uses the library's
 * own table, a file-scope device array of sizeof the 64-domain table (46 KiB,
 * one per GPU, held until the process ends), instead of caller memory; the
 * call allocates no device memory.  max_domains is 1..64 (FW2_E_INVALID
 * beyond: the table holds 64 domains).  The table is cleared by this call
 * and rewritten by fw2_batch_set_domains; it keeps the last batch's contents
 * otherwise.  One such batch per GPU at a time: while one exists on the
 * current device another call returns FW2_E_STATE (calls that shared the
 * table would race); fw2_batch_destroy frees it for the next.  Everything
 * else is as for fw2_batch_create. */
fw2_status fw2_batch_create_noalloc(int32_t max_domains, void *stream, fw2_batch **out);

/* ---- Relaxation maps to labels -------------------------------------------
 * Sec. 3.2 gives every point its own 2 + 4L relaxation parameters; the library
 * stores a label per point and a table of the distinct tuples.  This call
 * turns dense per-point maps into that form.
 *   maps: host FP64 [2 + 4L][n_pts] -- one map per parameter, in the
 *     relax_table row order (k1, k2, d1[L], d2[L], alpha1[L], alpha2[L]), each
 *     [nz][ny][nx].
 *   label: host [n_pts] output; table: host [FW2_MAX_LABELS][2 + 4L] output
 *     (distinct tuples in order of first appearance, compared bitwise);
 *     *n_labels: their count.
 * FW2_E_INVALID for NULL pointers, n_pts < 1, a bad n_relax, or more than
 * FW2_MAX_LABELS distinct tuples (then label and table are unspecified). */
fw2_status fw2_label_relaxation_map(int64_t n_pts, int32_t n_relax, const double *maps, uint8_t *label,
                                    double *table, int32_t *n_labels);

/* ---- Slabs of a 3D grid ----------------------------------------------------
 * The finite-difference update is local (Sec. 5.3 remarks that this suits
 * several GPUs): a 3D grid split along z into slabs advances each slab with
 * the same kernels once its z halos hold the neighbours' planes.  A slab
 * domain (slab_nz > 0, ndim 3, nz >= 4, fd_r > 0 and pml_cp > 0 so that every
 * slab uses the same stencil and layer constants) follows the global plane
 * index for the boundary layer and the last v_z sample; its maps, sources and
 * receivers are its own planes only.  Halo kinds:
 *   FW2_HALO_P       4 planes of p (exchange after the pressure phase);
 *   FW2_HALO_V       4 planes of v_z and 1 plane each of v_x and v_y (the g_11
 *                    cross terms), after the velocity phase;
 *   FW2_HALO_MEDIUM  1 plane of rho and of kappa0 (the staggered means at the
 *                    last plane), once after creation.
 * The memory variables are point-local and never exchanged.  With neighbours
 * A (below) and B (above), one exchange is pack(A, HIGH) -> unpack(B, LOW) and
 * pack(B, LOW) -> unpack(A, HIGH); a side without a neighbour keeps its zero
 * halo.  On several GPUs the packed faces travel between the pack and the
 * unpack (e.g. over RCCL); on one GPU they are plain device buffers.
 *   fw2_halo_bytes: bytes of one packed face of the kind.
 *   fw2_halo_pack: the planes the neighbour on `side` needs, unpadded FP32
 *     [planes][ny][nx], into the caller's device buffer (async on the
 *     domain's stream).
 *   fw2_halo_unpack: a neighbour's packed face into this domain's halo on
 *     `side` (async on the domain's stream).
 *   fw2_step_phase: half a step, FW2_PHASE_PRESSURE (pressure phase and
 *     sources) or FW2_PHASE_VELOCITY (receivers and velocity phase; the step
 *     counter then advances); the phases must alternate (FW2_E_STATE), and
 *     fw2_step is refused between them.
 * Errors: FW2_E_INVALID for a bad kind, side or phase or a NULL buffer,
 * FW2_E_UNSUPPORTED for halo calls on a domain that is not a slab. */
enum { FW2_HALO_P = 0, FW2_HALO_V = 1, FW2_HALO_MEDIUM = 2 };
enum { FW2_LOW = 0, FW2_HIGH = 1 };
enum { FW2_PHASE_PRESSURE = 0, FW2_PHASE_VELOCITY = 1 };
fw2_status fw2_halo_bytes(const fw2_domain *dom, int32_t kind, uint64_t *bytes);
fw2_status fw2_halo_pack(fw2_domain *dom, int32_t kind, int32_t side, void *dev_dst);
fw2_status fw2_halo_unpack(fw2_domain *dom, int32_t kind, int32_t side, const void *dev_src);
fw2_status fw2_step_phase(fw2_domain *dom, int32_t phase);

/* Library infrastructure (measurement): streaming probes.  Plain one-thread-
 * per-element kernels whose HBM rate is the reference for the step kernels'
 * measured traffic; they compute nothing of the method.
 *   FW2_PROBE_COPY          copies the first half of buf to the second, 16
 *                           bytes per thread (bytes / 32 float4 elements);
 *   FW2_PROBE_VELOCITY_MIX  the velocity phase's per-point byte mix at L = 2
 *                           in 3D without its stencil: buf holds 21 FP32
 *                           arrays of n = floor(bytes / 84 / 64) * 64 points,
 *                           one after another; every point reads x_0..x_11
 *                           (arrays 0..11) and writes t = (x_0 + x_4) + x_5,
 *                           x_{1+q} + t (q < 3, arrays 12..14) and
 *                           fma(0.5, x_{6+q}, t) (q < 6, arrays 15..20).
 * buf: caller-owned device memory, 256-byte aligned, overwritten where
 * written; bytes in [64 KiB, 1 TiB].  Asynchronous on stream (hipStream_t;
 * NULL: the default stream).  Errors: FW2_E_INVALID for an unknown kind, a
 * NULL or misaligned buf or bytes out of range. */
enum { FW2_PROBE_COPY = 0, FW2_PROBE_VELOCITY_MIX = 1 };
fw2_status fw2_stream_probe(int32_t kind, void *dev_buf, uint64_t bytes, void *stream);

/* Library infrastructure.  Message of the last failed call on this thread ("" if none). */
const char *fw2_last_error(void);

/* Library infrastructure.  Free host-side state (events, graphs).  Does not touch the workspace,
 * sources or traces, which the caller owns.  NULL is a no-op. */
void fw2_destroy_domain(fw2_domain *dom);

#ifdef __cplusplus
}
#endif

#endif /* FW2_H */
