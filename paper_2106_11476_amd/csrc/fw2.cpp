// libfw2: C ABI (include/fw2.h) around the gfx950 step kernels.
#include "fw2.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "probe.hpp"
#include "setup.hpp"

namespace {

thread_local std::string g_err;

fw2_status fail(fw2_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

#define FW2_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(FW2_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));   \
    } while (0)

constexpr uint64_t kAlign = 256;
constexpr int kTimingRing = 256;

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

struct Layout {
    fw2::Geometry geo;
    int n_float;               // float arrays
    uint64_t float_base;       // byte offset of array 0 (x = 0 lands 256-byte aligned)
    uint64_t label_off;        // 0 if no label array
    uint64_t tab_off[2][3];    // [nabla-1][axis] (b, c) tables
    uint64_t w_off[2][3];      // [nabla-1][axis] w tables
    int n_slots[2][3];
    uint64_t total;
};

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// Everything that can be checked without reading the maps.
fw2_status validate_scalars(const fw2_domain_desc *d)
{
    if (!d) return fail(FW2_E_INVALID, "desc is NULL");
    if (d->ndim != 2 && d->ndim != 3) return fail(FW2_E_INVALID, "ndim must be 2 or 3");
    if (d->n_relax < 1 || d->n_relax > FW2_MAX_RELAX)
        return fail(FW2_E_INVALID, "n_relax must be in 1..8");
    const bool slab = d->slab_nz != 0;
    if (slab) {
        if (d->ndim != 3) return fail(FW2_E_INVALID, "slab domains are 3D");
        if (d->slab_nz < 0 || d->slab_nz > (1 << 20) || d->slab_z0 < 0 || d->slab_z0 + d->n[2] > d->slab_nz)
            return fail(FW2_E_INVALID, "need 0 <= slab_z0 and slab_z0 + nz <= slab_nz <= 2^20");
        if (d->n[2] < fw2::kHalo) return fail(FW2_E_INVALID, "a slab needs at least 4 planes");
        if (!(d->fd_r > 0.0) || !(d->pml_cp > 0.0))
            return fail(FW2_E_INVALID, "slabs need fd_r > 0 and pml_cp > 0 (the same constants in every slab)");
    }
    for (int a = 0; a < 3; ++a) {
        const int64_t na = d->n[a];
        if (a < d->ndim) {
            if (na < 1 || na > (1 << 20)) return fail(FW2_E_INVALID, "grid size out of range");
            if (d->bound_cells[a] < 0 || d->trans_cells[a] < 0 || d->trans_cells[a] > d->bound_cells[a])
                return fail(FW2_E_INVALID, "need 0 <= trans_cells <= bound_cells");
            if (2 * (int64_t)d->bound_cells[a] > (a == 2 && slab ? d->slab_nz : na))
                return fail(FW2_E_INVALID, "boundary layers wider than the grid");
        } else if (na != 1) {
            return fail(FW2_E_INVALID, "n[2] must be 1 in 2D");
        }
    }
    // the sweeps address a padded plane (pitch <= nx + 71 elements, ny + 8
    // rows) with 32-bit byte offsets: below 2^30 points in 2D, 2^29 in 3D
    if ((d->n[0] + 72) * (d->n[1] + 8) >= ((int64_t)1 << (d->ndim == 3 ? 29 : 30)))
        return fail(FW2_E_INVALID, d->ndim == 3 ? "a 3D plane (nx x ny) must hold fewer than 2^29 points"
                                                : "a 2D grid (nx x ny) must hold fewer than 2^30 points");
    if (d->nonlinear_form != FW2_NL_PRINTED && d->nonlinear_form != FW2_NL_CUSTOM)
        return fail(FW2_E_INVALID, "nonlinear_form must be 0 or 1");
    if (d->nonlinear_form == FW2_NL_CUSTOM &&
        !(std::isfinite(d->nl_A) && std::isfinite(d->nl_B0) && std::isfinite(d->nl_B1)))
        return fail(FW2_E_INVALID, "nl_A, nl_B0, nl_B1 must be finite");
    if (d->map_kind != FW2_HOST && d->map_kind != FW2_DEVICE) return fail(FW2_E_INVALID, "map_kind must be 0 or 1");
    if (!finite_pos(d->h) || !finite_pos(d->dt)) return fail(FW2_E_INVALID, "h and dt must be positive");
    if (!(d->pml_Rc > 0.0 && d->pml_Rc < 1.0)) return fail(FW2_E_INVALID, "pml_Rc must be in (0, 1)");
    if (d->pml_npoly < 1 || d->pml_npoly > 8) return fail(FW2_E_INVALID, "pml_npoly must be in 1..8");
    if (!std::isfinite(d->pml_cp) || !std::isfinite(d->fd_r)) return fail(FW2_E_INVALID, "non-finite pml_cp/fd_r");
    if (d->relax_scheme != FW2_RELAX_PRINTED && d->relax_scheme != FW2_RELAX_CENTRED)
        return fail(FW2_E_INVALID, "relax_scheme must be 0 or 1");
    if (d->stencil_mode != FW2_STENCIL_GLOBAL && d->stencil_mode != FW2_STENCIL_LOCAL)
        return fail(FW2_E_INVALID, "stencil_mode must be 0 or 1");
    if (d->n_labels < 1 || d->n_labels > FW2_MAX_LABELS) return fail(FW2_E_INVALID, "n_labels must be in 1..256");
    if (!d->c || !d->rho || !d->beta || !d->relax_table) return fail(FW2_E_INVALID, "NULL map or table");
    const int L = d->n_relax, row = 2 + 4 * L;
    for (int lab = 0; lab < d->n_labels; ++lab) {
        const double *r = d->relax_table + (size_t)lab * row;
        if (!finite_pos(r[0]) || !finite_pos(r[1])) return fail(FW2_E_INVALID, "kappa must be positive");
        for (int q = 2; q < row; ++q)
            if (!std::isfinite(r[q]) || r[q] < 0.0) return fail(FW2_E_INVALID, "d and alpha must be >= 0");
    }
    return FW2_OK;
}

void make_layout(const fw2_domain_desc *d, Layout *ly)
{
    fw2::Geometry &g = ly->geo;
    g.ndim = d->ndim;
    for (int a = 0; a < 3; ++a) g.n[a] = (int32_t)d->n[a];
    const int64_t H = fw2::kHalo;
    g.pitch = (int64_t)align_up((uint64_t)(g.n[0] + 2 * H), 64);
    g.plane = g.pitch * (g.n[1] + 2 * H);
    const int64_t planes = d->ndim == 3 ? g.n[2] + 2 * H : 1;
    g.stride = g.plane * planes;                           // multiple of 64 elements
    g.origin = (d->ndim == 3 ? H * g.plane : 0) + H * g.pitch + H;
    const int L = d->n_relax;
    ly->n_float = 1 + d->ndim + 2 * d->ndim * L + 3;
    ly->float_base = kAlign + kAlign - (uint64_t)(H * 4) % kAlign;   // x = 0 on a 256-byte boundary
    uint64_t end = ly->float_base + (uint64_t)ly->n_float * g.stride * 4;
    end = align_up(end, kAlign);
    ly->label_off = 0;
    if (d->n_labels > 1) {
        ly->label_off = end;
        end = align_up(end + (uint64_t)g.stride, kAlign);
    }
    for (int nab = 0; nab < 2; ++nab)
        for (int a = 0; a < 3; ++a) {
            if (a >= d->ndim) {
                ly->n_slots[nab][a] = 0;
                ly->tab_off[nab][a] = ly->w_off[nab][a] = 0;
                continue;
            }
            const int nb = d->bound_cells[a];
            const int ns = nab == 0 ? nb + 2 : nb + 1;     // nabla_1: half positions
            ly->n_slots[nab][a] = ns;
            ly->tab_off[nab][a] = end;
            end = align_up(end + (uint64_t)ns * d->n_labels * L * 8, kAlign);
            ly->w_off[nab][a] = end;
            end = align_up(end + (uint64_t)ns * d->n_labels * 4, kAlign);
        }
    ly->total = end;
}

// (A, B0, B1) of the multipliers rho0 (1 + A kappa0 p), kappa0 (1 + kappa0 B p).
void nl_coefficients(const fw2_domain_desc *d, double *A, double *B0, double *B1)
{
    if (d->nonlinear_form == FW2_NL_CUSTOM) {
        *A = d->nl_A;
        *B0 = d->nl_B0;
        *B1 = d->nl_B1;
    } else {                       // Eqs. state1 / state2 as printed
        *A = 1.0;
        *B0 = 1.0;
        *B1 = -2.0;
    }
}

// Per-point weights: every point's r lies in [min c, max c] dt / h (a
// velocity point's r^2 is a mean of two cells'), so the scheme is checked
// at a sweep of r over that range with the weights of each r.
bool local_stencil_stable(const fw2_domain_desc *d, double cmin, double cmax)
{
    const double r0 = cmin * d->dt / d->h, r1 = cmax * d->dt / d->h;
    const int K = 16;
    for (int k = 0; k <= K; ++k) {
        const double r = std::sqrt(r0 * r0 + (r1 * r1 - r0 * r0) * k / K);
        double gw[4], g11;
        fw2::stencil_weights(r, d->ndim, gw, &g11);
        if (fw2::stability_factor(r, d->ndim, gw, g11) >= 1.0) return false;
    }
    return true;
}

struct TimingSlot {
    hipEvent_t ev[4];
    bool pending;
};

}  // namespace

struct fw2_domain {
    fw2_domain_desc desc;      // scalars only (host pointers cleared)
    Layout ly;
    uint8_t *ws = nullptr;
    long long *counter = nullptr;
    int *flag = nullptr;
    fw2::StepArgs args;
    fw2::KernelConfig kc;
    fw2::SparseArgs src, rcv;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    int64_t step = 0;
    int graph_chunk = 32;
    hipGraphExec_t graph = nullptr;
    bool timing = false;
    std::vector<TimingSlot> ring;
    int64_t timed_steps = 0;
    double ms[2] = {0.0, 0.0};
    int64_t count[2] = {0, 0};
    bool adjoint = false;
    fw2::AdjointBuffers adj;
    int64_t adj_pp_step = -1;        // step whose p'' and S the adjoint buffers hold
    bool mid_step = false;           // fw2_step_phase ran the pressure phase of a step
    hipGraphExec_t into_graph = nullptr;   // fw2_step_into's last capture and its arguments
    const void *into_first = nullptr;
    void *into_states = nullptr;
    int32_t into_n = 0;
    int64_t npts() const { return (int64_t)ly.geo.n[0] * ly.geo.n[1] * ly.geo.n[2]; }
};

namespace {

// The velocity sweeps record the receivers in an extra block of their
// launch; the one-thread-per-point kernel leaves them to a launch of their own.
void sync_receiver_args(fw2_domain *d)
{
    d->args.rcv = d->rcv;
    if (d->kc.variant == 0) d->args.rcv.step = nullptr;
}

void drop_graph(fw2_domain *d)
{
    if (d->graph) {
        (void)hipGraphExecDestroy(d->graph);
        d->graph = nullptr;
    }
    if (d->into_graph) {
        (void)hipGraphExecDestroy(d->into_graph);
        d->into_graph = nullptr;
    }
}

fw2_status enqueue_step(fw2_domain *d, TimingSlot *ts)
{
    const int L = d->desc.n_relax, sch = d->desc.relax_scheme;
    if (ts) FW2_HIP(hipEventRecord(ts->ev[0], d->stream));
    FW2_HIP(fw2::launch_pressure(d->args, L, sch, d->kc, d->stream));
    if (ts) FW2_HIP(hipEventRecord(ts->ev[1], d->stream));
    FW2_HIP(fw2::launch_sources(d->src, d->stream));
    if (!d->args.rcv.step) FW2_HIP(fw2::launch_receivers(d->rcv, d->stream));
    if (ts) FW2_HIP(hipEventRecord(ts->ev[2], d->stream));
    FW2_HIP(fw2::launch_velocity(d->args, L, sch, d->kc, d->stream));
    if (ts) FW2_HIP(hipEventRecord(ts->ev[3], d->stream));
    return FW2_OK;
}

fw2_status enqueue_step_on(fw2_domain *d, hipStream_t s)
{
    const int L = d->desc.n_relax, sch = d->desc.relax_scheme;
    FW2_HIP(fw2::launch_pressure(d->args, L, sch, d->kc, s));
    FW2_HIP(fw2::launch_sources(d->src, s));
    if (!d->args.rcv.step) FW2_HIP(fw2::launch_receivers(d->rcv, s));
    FW2_HIP(fw2::launch_velocity(d->args, L, sch, d->kc, s));
    return FW2_OK;
}

fw2_status build_graph(fw2_domain *d)
{
    if (!d->capture) FW2_HIP(hipStreamCreateWithFlags(&d->capture, hipStreamNonBlocking));
    FW2_HIP(hipStreamBeginCapture(d->capture, hipStreamCaptureModeThreadLocal));
    fw2_status st = FW2_OK;
    for (int k = 0; k < d->graph_chunk && st == FW2_OK; ++k) st = enqueue_step_on(d, d->capture);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(d->capture, &graph);
    if (st != FW2_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(FW2_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&d->graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        d->graph = nullptr;
        return fail(FW2_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    return FW2_OK;
}

fw2_status collect_slot(fw2_domain *d, TimingSlot &s)
{
    if (!s.pending) return FW2_OK;
    FW2_HIP(hipEventSynchronize(s.ev[3]));
    float a = 0.f, b = 0.f;
    FW2_HIP(hipEventElapsedTime(&a, s.ev[0], s.ev[1]));
    FW2_HIP(hipEventElapsedTime(&b, s.ev[2], s.ev[3]));
    d->ms[0] += a;
    d->ms[1] += b;
    d->count[0] += 1;
    d->count[1] += 1;
    s.pending = false;
    return FW2_OK;
}

// Copy between the packed [nz][ny][nx] layout and the padded device layout
// for the sub-box [0, ext[0]) x [0, ext[1]) x [0, ext[2]).
fw2_status copy_box(fw2_domain *d, float *dev_base, void *packed, bool to_device, hipMemcpyKind kind,
                    const int ext[3])
{
    const fw2::Geometry &g = d->ly.geo;
    const size_t row_b = (size_t)g.n[0] * 4;
    for (int z = 0; z < ext[2]; ++z) {
        float *dev = dev_base + g.origin + (int64_t)z * g.plane;
        char *host = (char *)packed + (size_t)z * g.n[1] * row_b;
        if (to_device)
            FW2_HIP(hipMemcpy2DAsync(dev, (size_t)g.pitch * 4, host, row_b, (size_t)ext[0] * 4, ext[1], kind, d->stream));
        else
            FW2_HIP(hipMemcpy2DAsync(host, row_b, dev, (size_t)g.pitch * 4, (size_t)ext[0] * 4, ext[1], kind, d->stream));
    }
    return FW2_OK;
}

fw2_status transfer_fields(fw2_domain *d, uint32_t mask, void *buf, int32_t kind, bool to_device)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (!buf) return fail(FW2_E_INVALID, "buffer is NULL");
    if (mask == 0 || (mask & ~FW2_FIELD_ALL)) return fail(FW2_E_INVALID, "bad field mask");
    if (kind != FW2_HOST && kind != FW2_DEVICE) return fail(FW2_E_INVALID, "bad pointer kind");
    const hipMemcpyKind k = kind == FW2_DEVICE ? hipMemcpyDeviceToDevice
                                               : (to_device ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost);
    const fw2::Geometry &g = d->ly.geo;
    const int nd = g.ndim, L = d->desc.n_relax;
    const size_t field_b = (size_t)d->npts() * 4;
    char *cur = (char *)buf;
    FW2_HIP(hipStreamSynchronize(d->stream));
    auto one = [&](float *base, int axis) -> fw2_status {
        int ext[3] = {g.n[0], g.n[1], g.n[2]};
        if (axis >= 0 && to_device) ext[axis] -= 1;      // v sample past the grid stays zero
        if (axis >= 0 && to_device && ext[axis] == 0) {
            cur += field_b;
            return FW2_OK;
        }
        fw2_status st = copy_box(d, base, cur, to_device, k, ext);
        cur += field_b;
        return st;
    };
    fw2_status st = FW2_OK;
    if (mask & FW2_FIELD_P) st = one(d->args.p, -1);
    if (st == FW2_OK && (mask & FW2_FIELD_V))
        for (int a = 0; a < nd && st == FW2_OK; ++a) st = one(d->args.v + a * g.stride, a);
    if (st == FW2_OK && (mask & FW2_FIELD_PSI1))
        for (int a = 0; a < nd; ++a)
            for (int nu = 0; nu < L && st == FW2_OK; ++nu)
                st = one(d->args.psi1 + (int64_t)(a * L + nu) * g.stride, a);
    if (st == FW2_OK && (mask & FW2_FIELD_PSI2))
        for (int a = 0; a < nd; ++a)
            for (int nu = 0; nu < L && st == FW2_OK; ++nu)
                st = one(d->args.psi2 + (int64_t)(a * L + nu) * g.stride, -1);
    if (st != FW2_OK) return st;
    FW2_HIP(hipStreamSynchronize(d->stream));
    return FW2_OK;
}

// Planes of a slab's halo exchange (see fw2.h): for a pack, the planes the
// neighbour on `side` needs from this slab; for an unpack, this slab's halo
// planes on `side`.
fw2::PlaneSet halo_planes(const fw2_domain *d, int kind, int side, bool unpack)
{
    const fw2::StepArgs &a = d->args;
    const int64_t S = d->ly.geo.stride;
    const int nz = d->ly.geo.n[2];
    fw2::PlaneSet s;
    std::memset(&s, 0, sizeof(s));
    auto add = [&](const float *arr, int count) {
        // low side: planes [0, count) packed, [-count, 0) unpacked;
        // high side: [nz - count, nz) packed, [nz, nz + count) unpacked
        const int z0 = side == FW2_LOW ? (unpack ? -count : 0) : (unpack ? nz : nz - count);
        s.arr[s.n] = arr;
        s.z0[s.n] = z0;
        s.nz[s.n] = count;
        s.total += count;
        s.n++;
    };
    if (kind == FW2_HALO_P) {
        add(a.p, fw2::kHalo);
    } else if (kind == FW2_HALO_V) {
        add(a.v + 2 * S, fw2::kHalo);     // v_z: the z stencil
        add(a.v, 1);                      // v_x, v_y: the g_11 cross terms
        add(a.v + S, 1);
    } else {
        add(a.rho, 1);
        add(a.kap, 1);
    }
    return s;
}

fw2_status halo_check(const fw2_domain *d, int kind, int side)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (d->desc.slab_nz <= 0) return fail(FW2_E_UNSUPPORTED, "halo exchange is for slab domains");
    if (kind != FW2_HALO_P && kind != FW2_HALO_V && kind != FW2_HALO_MEDIUM)
        return fail(FW2_E_INVALID, "bad halo kind");
    if (side != FW2_LOW && side != FW2_HIGH) return fail(FW2_E_INVALID, "side must be FW2_LOW or FW2_HIGH");
    return FW2_OK;
}

}  // namespace

extern "C" {

const char *fw2_last_error(void) { return g_err.c_str(); }

fw2_status fw2_workspace_bytes(const fw2_domain_desc *desc, uint64_t *bytes)
{
    fw2_status st = validate_scalars(desc);
    if (st != FW2_OK) return st;
    if (!bytes) return fail(FW2_E_INVALID, "bytes is NULL");
    Layout ly;
    make_layout(desc, &ly);
    *bytes = ly.total;
    return FW2_OK;
}

fw2_status fw2_create_domain(const fw2_domain_desc *desc, void *dev_workspace, uint64_t workspace_bytes,
                             fw2_domain **out)
{
    fw2_status st = validate_scalars(desc);
    if (st != FW2_OK) return st;
    if (!out) return fail(FW2_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!dev_workspace) return fail(FW2_E_INVALID, "workspace is NULL");
    if ((uintptr_t)dev_workspace % kAlign) return fail(FW2_E_INVALID, "workspace must be 256-byte aligned");
    Layout ly;
    make_layout(desc, &ly);
    if (workspace_bytes < ly.total) return fail(FW2_E_NOMEM, "workspace too small");

    const fw2::Geometry &g = ly.geo;
    const int nd = desc->ndim, L = desc->n_relax;
    const int64_t npts = (int64_t)g.n[0] * g.n[1] * g.n[2];

    // Host maps: checked here, with the largest and smallest sound speed
    // (stencil r, Table 1 c_p, the per-point stability sweep).  Device maps
    // are checked by the conversion kernel below.
    const bool dev_maps = desc->map_kind == FW2_DEVICE;
    double cmax = 0.0, cmin = HUGE_VAL;
    if (!dev_maps) {
        for (int64_t q = 0; q < npts; ++q) {
            if (!finite_pos(desc->c[q]) || !finite_pos(desc->rho[q]) || !std::isfinite(desc->beta[q]))
                return fail(FW2_E_INVALID, "c and rho must be positive and finite, beta finite");
            if (desc->label && desc->label[q] >= desc->n_labels) return fail(FW2_E_INVALID, "label >= n_labels");
            cmax = std::max(cmax, (double)desc->c[q]);
            cmin = std::min(cmin, (double)desc->c[q]);
        }
    }

    fw2_domain *d = new (std::nothrow) fw2_domain();
    if (!d) return fail(FW2_E_NOMEM, "host allocation failed");
    d->desc = *desc;
    d->desc.c = d->desc.rho = d->desc.beta = nullptr;
    d->desc.label = nullptr;
    d->desc.relax_table = nullptr;
    d->ly = ly;
    d->ws = (uint8_t *)dev_workspace;
    d->stream = (hipStream_t)desc->stream;
    d->counter = (long long *)d->ws;
    d->flag = (int *)(d->ws + 8);

    auto cleanup = [&](fw2_status s) {
        delete d;
        return s;
    };
#define FW2_HIP_C(call)                                                                              \
    do {                                                                                             \
        hipError_t e_ = (call);                                                                      \
        if (e_ != hipSuccess) return cleanup(fail(FW2_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_))); \
    } while (0)

    FW2_HIP_C(hipMemsetAsync(d->ws, 0, ly.total, d->stream));
    FW2_HIP_C(hipStreamSynchronize(d->stream));     // the uploads below use blocking copies

    float *fb = (float *)(d->ws + ly.float_base);
    fw2::StepArgs &a = d->args;
    a.geo = g;
    a.p = fb;
    a.v = fb + g.stride;
    a.psi1 = fb + (1 + nd) * g.stride;
    a.psi2 = a.psi1 + (int64_t)nd * L * g.stride;
    a.out = 0;                                       // in place
    float *kap = a.psi2 + (int64_t)nd * L * g.stride;
    float *nlq = kap + g.stride;
    float *rho = nlq + g.stride;
    a.kap = kap;
    a.nlq = nlq;
    a.rho = rho;
    a.label = ly.label_off ? d->ws + ly.label_off : nullptr;
    a.n_labels = desc->n_labels;
    double nlA, nlB0, nlB1;
    nl_coefficients(desc, &nlA, &nlB0, &nlB1);
    a.nlA = (float)nlA;
    a.z_off = desc->slab_nz > 0 ? (int32_t)desc->slab_z0 : 0;
    a.nz_glob = desc->slab_nz > 0 ? (int32_t)desc->slab_nz : g.n[2];

    // Medium planes: kappa0 = 1/(rho c^2), kappa0 B with B = B0 + B1 beta
    // (1 - 2 beta as printed), rho (FP64, stored FP32).
    if (dev_maps) {
        // on the GPU, with the maps checked and c's extremes reduced there;
        // three words past the step counter and flag hold the results
        fw2::MediumArgs m;
        m.geo = g;
        m.c = desc->c;
        m.rho = desc->rho;
        m.beta = desc->beta;
        m.label = desc->label;
        m.kap = kap;
        m.nlq = nlq;
        m.rhop = rho;
        m.labp = (uint8_t *)a.label;
        m.B0 = nlB0;
        m.B1 = nlB1;
        m.n_labels = desc->n_labels;
        m.stats = (unsigned int *)(d->ws + 16);
        FW2_HIP_C(fw2::launch_medium(m, d->stream));
        unsigned int st3[3] = {0, 0, 0};
        FW2_HIP_C(hipMemcpyAsync(st3, m.stats, sizeof(st3), hipMemcpyDeviceToHost, d->stream));
        FW2_HIP_C(hipStreamSynchronize(d->stream));
        FW2_HIP_C(hipMemsetAsync(m.stats, 0, sizeof(st3), d->stream));
        if (st3[2]) return cleanup(fail(FW2_E_INVALID, "c and rho must be positive and finite, beta finite, label < n_labels"));
        float fmax, fmin;
        const unsigned int bmin = 0x7f800000u - st3[1];
        std::memcpy(&fmax, &st3[0], 4);
        std::memcpy(&fmin, &bmin, 4);
        cmax = fmax;
        cmin = fmin;
    } else {
        // Planes are converted in chunks of about 16 M points by up to 16
        // host threads (a share of the chunk's rows each) and each chunk is
        // uploaded with one copy per array: the planes of a chunk are
        // contiguous on the device.  Halo cells of the staging buffers are
        // never written and stay zero.
        const size_t plane_n = (size_t)g.plane;
        const int nz = g.n[2];
        const int cz = (int)std::max<size_t>(1, std::min<size_t>((size_t)nz, ((size_t)1 << 24) / plane_n));
        const size_t chunk_n = plane_n * (size_t)cz;
        std::vector<float> hk(chunk_n, 0.f), hn(chunk_n, 0.f), hr(chunk_n, 0.f);
        std::vector<uint8_t> hl(a.label ? chunk_n : 0, 0);
        const int64_t z0 = nd == 3 ? fw2::kHalo : 0;
        const unsigned hw = std::thread::hardware_concurrency();
        const int n_thr = (int)std::max(1u, std::min(16u, hw ? hw : 1u));
        for (int zc = 0; zc < nz; zc += cz) {
            const int nzc = std::min(cz, nz - zc);
            const int64_t rows = (int64_t)nzc * g.n[1];
            auto convert = [&](int64_t r0, int64_t r1) {
                for (int64_t r = r0; r < r1; ++r) {
                    const int zl = (int)(r / g.n[1]), y = (int)(r % g.n[1]);
                    const int64_t q0 = ((int64_t)(zc + zl) * g.n[1] + y) * g.n[0];
                    const size_t o0 = (size_t)zl * plane_n + (size_t)(y + fw2::kHalo) * g.pitch + fw2::kHalo;
                    for (int x = 0; x < g.n[0]; ++x) {
                        const int64_t q = q0 + x;
                        const size_t o = o0 + x;
                        const double c = desc->c[q], rr = desc->rho[q], b = desc->beta[q];
                        const double k0 = 1.0 / (rr * c * c);
                        hk[o] = (float)k0;
                        hn[o] = (float)(k0 * (nlB0 + nlB1 * b));
                        hr[o] = (float)rr;
                        if (a.label) hl[o] = desc->label[q];
                    }
                }
            };
            const int nt = (int)std::min<int64_t>(n_thr, std::max<int64_t>(1, rows / 64));
            // ranges whose thread could not be started run on this thread
            std::vector<std::thread> pool;
            int started = 0;
            try {
                pool.reserve(nt);
                for (int t = 1; t < nt; ++t, ++started)
                    pool.emplace_back(convert, rows * t / nt, rows * (t + 1) / nt);
            } catch (...) {
            }
            convert(0, rows / nt);
            for (int t = 1 + started; t < nt; ++t) convert(rows * t / nt, rows * (t + 1) / nt);
            for (auto &th : pool) th.join();
            const int64_t off = (zc + z0) * g.plane;
            const size_t n = plane_n * (size_t)nzc;
            FW2_HIP_C(hipMemcpy(kap + off, hk.data(), n * 4, hipMemcpyHostToDevice));
            FW2_HIP_C(hipMemcpy(nlq + off, hn.data(), n * 4, hipMemcpyHostToDevice));
            FW2_HIP_C(hipMemcpy(rho + off, hr.data(), n * 4, hipMemcpyHostToDevice));
            if (a.label)
                FW2_HIP_C(hipMemcpy((uint8_t *)a.label + off, hl.data(), n, hipMemcpyHostToDevice));
        }
    }

    const double r = desc->fd_r > 0.0 ? desc->fd_r : cmax * desc->dt / desc->h;
    double gw[4], g11;
    fw2::stencil_weights(r, nd, gw, &g11);
    const double r_run = cmax * desc->dt / desc->h;
    if (desc->stencil_mode == FW2_STENCIL_GLOBAL ? fw2::stability_factor(r_run, nd, gw, g11) >= 1.0
                                                 : !local_stencil_stable(desc, cmin, cmax))
        return cleanup(fail(FW2_E_INVALID, "time step above the stability limit of the (8,4) scheme"));
    for (int k = 0; k < 4; ++k) a.g[k] = (float)(gw[k] / desc->h);
    a.g11 = (float)(g11 / desc->h);
    a.dt = (float)desc->dt;
    a.local_stencil = desc->stencil_mode == FW2_STENCIL_LOCAL ? 1 : 0;
    {
        double pw[4][4], g11s;
        fw2::stencil_polynomials(nd, pw, &g11s);
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 4; ++k) a.pw[j][k] = (float)(pw[j][k] / desc->h);
        a.g11s = (float)(g11s / desc->h);
        a.q2 = (float)((desc->dt / desc->h) * (desc->dt / desc->h));
    }

    // Relaxation tables per axis (Sec. 3.2, Sec. 3.3 / Table 1).
    const double cp = desc->pml_cp > 0.0 ? desc->pml_cp : cmax;
    for (int ax = 0; ax < nd; ++ax) {
        const int nb = desc->bound_cells[ax], ntr = desc->trans_cells[ax];
        fw2::TableInput in;
        in.n_labels = desc->n_labels;
        in.L = L;
        in.scheme = desc->relax_scheme;
        in.table = desc->relax_table;
        in.h = desc->h;
        in.dt = desc->dt;
        in.npoly = desc->pml_npoly;
        in.d_target = nb > 0 ? -(desc->pml_npoly + 1) * cp * std::log(desc->pml_Rc) / (2.0 * nb * desc->h) : 0.0;
        a.nb[ax] = nb;
        for (int nab = 0; nab < 2; ++nab) {
            const fw2::AxisTables t = fw2::build_axis_tables(in, nab + 1, nb, ntr);
            float2 *bc = (float2 *)(d->ws + ly.tab_off[nab][ax]);
            float *w = (float *)(d->ws + ly.w_off[nab][ax]);
            FW2_HIP_C(hipMemcpy(bc, t.bc.data(), t.bc.size() * 4, hipMemcpyHostToDevice));
            FW2_HIP_C(hipMemcpy(w, t.w.data(), t.w.size() * 4, hipMemcpyHostToDevice));
            if (nab == 0) {
                a.bc1[ax] = bc;
                a.w1[ax] = w;
            } else {
                a.bc2[ax] = bc;
                a.w2[ax] = w;
            }
        }
    }
    for (int ax = nd; ax < 3; ++ax) {
        a.nb[ax] = 0;
        a.bc1[ax] = a.bc2[ax] = nullptr;
        a.w1[ax] = a.w2[ax] = nullptr;
    }

    d->kc = nd == 2 ? fw2::KernelConfig{1, 256, 4} : fw2::KernelConfig{3, 64, 64};
    if (const char *ev = std::getenv("FW2_KERNEL_CONFIG")) {      // "variant,bx,rows[,by]" (tuning runs)
        int v = 0, bx = 0, ry = 0, by = 0;
        const int nparsed = std::sscanf(ev, "%d,%d,%d,%d", &v, &bx, &ry, &by);
        const bool parsed = nparsed == 3 || nparsed == 4;
        const bool ok2 = nd == 2 && by == 0 && (v == 0 || v == 1 || v == 2) && (bx == 64 || bx == 128 || bx == 256);
        const bool tile3 = by == 0 ? (bx == 16 || bx == 32 || bx == 64)
                                   : (v == 3 && ((bx == 64 && by == 4) || (bx == 32 && by == 8)));
        const bool ok3 = nd == 3 && (v == 0 || ((v >= 1 && v <= 3) && tile3));
        if (parsed && (ok2 || ok3) && ry >= 1 && ry <= 1024)
            d->kc = fw2::KernelConfig{v, bx, ry, by};
    }

    std::memset(&d->src, 0, sizeof(d->src));
    std::memset(&d->rcv, 0, sizeof(d->rcv));
    d->src.geo = d->rcv.geo = g;
    d->src.p = d->rcv.p = a.p;
    d->src.step = d->rcv.step = d->counter;
    sync_receiver_args(d);
    FW2_HIP_C(hipStreamSynchronize(d->stream));
#undef FW2_HIP_C
    *out = d;
    return FW2_OK;
}

fw2_status fw2_add_source(fw2_domain *d, int32_t n_pts, const int64_t *flat_idx, const int32_t *sig_id,
                          const float *weight, int32_t n_sig, int32_t n_t, const float *signals)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (n_pts < 0) return fail(FW2_E_INVALID, "n_pts < 0");
    if (n_pts > 0) {
        if (!flat_idx || !sig_id || !weight || !signals) return fail(FW2_E_INVALID, "NULL source array");
        if (n_sig < 1 || n_t < 1) return fail(FW2_E_INVALID, "need n_sig >= 1 and n_t >= 1");
        std::vector<int64_t> hi(n_pts);
        std::vector<int32_t> hs(n_pts);
        FW2_HIP(hipMemcpy(hi.data(), flat_idx, (size_t)n_pts * 8, hipMemcpyDeviceToHost));
        FW2_HIP(hipMemcpy(hs.data(), sig_id, (size_t)n_pts * 4, hipMemcpyDeviceToHost));
        const int64_t np = d->npts();
        for (int32_t q = 0; q < n_pts; ++q) {
            if (hi[q] < 0 || hi[q] >= np) return fail(FW2_E_INVALID, "source index out of range");
            if (hs[q] < 0 || hs[q] >= n_sig) return fail(FW2_E_INVALID, "sig_id out of range");
        }
        std::sort(hi.begin(), hi.end());
        if (std::adjacent_find(hi.begin(), hi.end()) != hi.end())
            return fail(FW2_E_INVALID, "source indices must be distinct");
    }
    drop_graph(d);
    d->src.n = n_pts;
    d->src.idx = flat_idx;
    d->src.sig = sig_id;
    d->src.w = weight;
    d->src.signals = signals;
    d->src.n_t = n_t;
    return FW2_OK;
}

fw2_status fw2_add_receivers(fw2_domain *d, int32_t n_rcv, const int64_t *flat_idx, float *trace,
                             int64_t cap_steps)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (n_rcv < 0 || cap_steps < 0) return fail(FW2_E_INVALID, "negative size");
    if (n_rcv > 0) {
        if (!flat_idx || !trace) return fail(FW2_E_INVALID, "NULL receiver array");
        std::vector<int64_t> hi(n_rcv);
        FW2_HIP(hipMemcpy(hi.data(), flat_idx, (size_t)n_rcv * 8, hipMemcpyDeviceToHost));
        for (int64_t v : hi)
            if (v < 0 || v >= d->npts()) return fail(FW2_E_INVALID, "receiver index out of range");
    }
    drop_graph(d);
    d->rcv.n = n_rcv;
    d->rcv.idx = flat_idx;
    d->rcv.trace = trace;
    d->rcv.cap = n_rcv > 0 ? cap_steps : 0;
    sync_receiver_args(d);
    return FW2_OK;
}

fw2_status fw2_step(fw2_domain *d, int32_t n)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (n < 0) return fail(FW2_E_INVALID, "n < 0");
    if (d->mid_step) return fail(FW2_E_STATE, "a step is half done (fw2_step_phase): run its velocity phase first");
    if (n == 0) return FW2_OK;
    if (d->timing) {
        for (int32_t s = 0; s < n; ++s) {
            TimingSlot &ts = d->ring[(size_t)(d->timed_steps % kTimingRing)];
            fw2_status st = collect_slot(d, ts);
            if (st != FW2_OK) return st;
            st = enqueue_step(d, &ts);
            if (st != FW2_OK) return st;
            ts.pending = true;
            d->timed_steps++;
            d->step++;
        }
        return FW2_OK;
    }
    int32_t left = n;
    if (d->graph_chunk > 0 && n >= d->graph_chunk) {
        if (!d->graph) {
            fw2_status st = build_graph(d);
            if (st != FW2_OK) return st;
        }
        while (left >= d->graph_chunk) {
            FW2_HIP(hipGraphLaunch(d->graph, d->stream));
            left -= d->graph_chunk;
            d->step += d->graph_chunk;
        }
    }
    for (; left > 0; --left) {
        fw2_status st = enqueue_step(d, nullptr);
        if (st != FW2_OK) return st;
        d->step++;
    }
    return FW2_OK;
}

fw2_status fw2_read_fields(fw2_domain *d, uint32_t mask, void *dst, int32_t kind)
{
    return transfer_fields(d, mask, dst, kind, false);
}

fw2_status fw2_write_fields(fw2_domain *d, uint32_t mask, const void *src, int32_t kind)
{
    return transfer_fields(d, mask, const_cast<void *>(src), kind, true);
}

int64_t fw2_current_step(const fw2_domain *d) { return d ? d->step : -1; }

fw2_status fw2_set_current_step(fw2_domain *d, int64_t step)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (step < 0) return fail(FW2_E_INVALID, "step < 0");
    FW2_HIP(fw2::launch_set_counter(d->counter, step, d->stream));
    FW2_HIP(hipStreamSynchronize(d->stream));
    d->step = step;
    return FW2_OK;
}

fw2_status fw2_set_stream(fw2_domain *d, void *stream)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    FW2_HIP(hipStreamSynchronize(d->stream));
    d->stream = (hipStream_t)stream;
    d->desc.stream = stream;
    return FW2_OK;
}

fw2_status fw2_set_graph_chunk(fw2_domain *d, int32_t steps)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (steps < 0 || steps > 4096) return fail(FW2_E_INVALID, "graph chunk must be in 0..4096");
    if (steps != d->graph_chunk) drop_graph(d);
    d->graph_chunk = steps;
    return FW2_OK;
}

fw2_status fw2_enable_kernel_timing(fw2_domain *d, int32_t enable)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (enable && !d->timing) {
        if (d->ring.empty()) {
            d->ring.resize(kTimingRing);
            for (auto &s : d->ring) {
                for (auto &e : s.ev) FW2_HIP(hipEventCreate(&e));
                s.pending = false;
            }
        }
        d->ms[0] = d->ms[1] = 0.0;
        d->count[0] = d->count[1] = 0;
    }
    if (!enable && d->timing)
        for (auto &s : d->ring) {
            fw2_status st = collect_slot(d, s);
            if (st != FW2_OK) return st;
        }
    d->timing = enable != 0;
    return FW2_OK;
}

fw2_status fw2_get_kernel_timing(fw2_domain *d, double ms[2], int64_t count[2])
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (!ms || !count) return fail(FW2_E_INVALID, "NULL output");
    FW2_HIP(hipStreamSynchronize(d->stream));
    for (auto &s : d->ring) {
        fw2_status st = collect_slot(d, s);
        if (st != FW2_OK) return st;
    }
    ms[0] = d->ms[0];
    ms[1] = d->ms[1];
    count[0] = d->count[0];
    count[1] = d->count[1];
    return FW2_OK;
}

static int64_t state_floats(const fw2_domain *d)
{
    const int nd = d->desc.ndim, L = d->desc.n_relax;
    return (int64_t)(1 + nd + 2 * nd * L) * d->ly.geo.stride;
}

fw2_status fw2_state_bytes(const fw2_domain *d, uint64_t *bytes)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (!bytes) return fail(FW2_E_INVALID, "bytes is NULL");
    *bytes = (uint64_t)state_floats(d) * 4;
    return FW2_OK;
}

fw2_status fw2_save_state(fw2_domain *d, void *dev_dst)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (!dev_dst) return fail(FW2_E_INVALID, "dst is NULL");
    FW2_HIP(hipMemcpyAsync(dev_dst, d->args.p, (size_t)state_floats(d) * 4, hipMemcpyDeviceToDevice, d->stream));
    return FW2_OK;
}

fw2_status fw2_load_state(fw2_domain *d, const void *dev_src, int64_t step)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (!dev_src || step < 0) return fail(FW2_E_INVALID, "src is NULL or step < 0");
    FW2_HIP(hipMemcpyAsync(d->args.p, dev_src, (size_t)state_floats(d) * 4, hipMemcpyDeviceToDevice, d->stream));
    FW2_HIP(fw2::launch_set_counter(d->counter, step, d->stream));
    d->step = step;
    return FW2_OK;
}

namespace {

// One step out of place: the state block at src (the domain's field layout)
// to the block at dst.  The pressure phase reads p, v, psi2 of src and writes
// p, psi2 of dst; the sources add into dst's p; the velocity phase reads that
// p and v, psi1 of src and writes v, psi1 of dst.
fw2_status enqueue_step_into(fw2_domain *d, const float *src, float *dst, hipStream_t s)
{
    const int L = d->desc.n_relax, sch = d->desc.relax_scheme, nd = d->desc.ndim;
    const int64_t S = d->ly.geo.stride;
    fw2::StepArgs a = d->args;
    a.p = const_cast<float *>(src);
    a.v = a.p + S;
    a.psi1 = a.p + (int64_t)(1 + nd) * S;
    a.psi2 = a.psi1 + (int64_t)nd * L * S;
    a.out = ((int64_t)(uintptr_t)dst - (int64_t)(uintptr_t)src) / 4;   // both 4-byte aligned
    FW2_HIP(fw2::launch_pressure(a, L, sch, d->kc, s));
    fw2::SparseArgs src_pts = d->src, rcv = d->rcv;
    src_pts.p = dst;
    rcv.p = dst;
    a.p = dst;
    a.rcv.p = dst;
    FW2_HIP(fw2::launch_sources(src_pts, s));
    if (!a.rcv.step) FW2_HIP(fw2::launch_receivers(rcv, s));
    FW2_HIP(fw2::launch_velocity(a, L, sch, d->kc, s));
    return FW2_OK;
}

fw2_status enqueue_steps_into(fw2_domain *d, int32_t n, const float *first, float *states, hipStream_t s)
{
    const int64_t B = state_floats(d);
    for (int32_t i = 0; i < n; ++i) {
        fw2_status st = enqueue_step_into(d, i == 0 ? first : states + (int64_t)(i - 1) * B, states + (int64_t)i * B, s);
        if (st != FW2_OK) return st;
    }
    return FW2_OK;
}

}  // namespace

fw2_status fw2_step_into(fw2_domain *d, int32_t n, const void *dev_first, void *dev_states)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (n < 0) return fail(FW2_E_INVALID, "n < 0");
    if (d->mid_step) return fail(FW2_E_STATE, "a step is half done (fw2_step_phase): run its velocity phase first");
    if (d->desc.slab_nz > 0) return fail(FW2_E_UNSUPPORTED, "slabs exchange halos between phases: use fw2_step_phase");
    if (n == 0) return FW2_OK;
    if (!dev_first || !dev_states) return fail(FW2_E_INVALID, "first or states is NULL");
    if ((uintptr_t)dev_first % 4 || (uintptr_t)dev_states % 4) return fail(FW2_E_INVALID, "blocks must be 4-byte aligned");
    const uint64_t bytes = (uint64_t)state_floats(d) * 4;
    const uintptr_t f0 = (uintptr_t)dev_first, s0 = (uintptr_t)dev_states, s1 = s0 + (uint64_t)n * bytes;
    if (f0 + bytes > s0 && f0 < s1) return fail(FW2_E_INVALID, "first overlaps the destination blocks");
    const float *first = (const float *)dev_first;
    float *states = (float *)dev_states;
    if (d->timing || d->graph_chunk <= 0 || n < 2) {
        fw2_status st = enqueue_steps_into(d, n, first, states, d->stream);
        if (st != FW2_OK) return st;
        d->step += n;
        return FW2_OK;
    }
    if (!d->into_graph || d->into_first != dev_first || d->into_states != dev_states || d->into_n != n) {
        if (d->into_graph) {
            (void)hipGraphExecDestroy(d->into_graph);
            d->into_graph = nullptr;
        }
        if (!d->capture) FW2_HIP(hipStreamCreateWithFlags(&d->capture, hipStreamNonBlocking));
        FW2_HIP(hipStreamBeginCapture(d->capture, hipStreamCaptureModeThreadLocal));
        fw2_status st = enqueue_steps_into(d, n, first, states, d->capture);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(d->capture, &graph);
        if (st != FW2_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(FW2_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&d->into_graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            d->into_graph = nullptr;
            return fail(FW2_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        d->into_first = dev_first;
        d->into_states = dev_states;
        d->into_n = n;
    }
    FW2_HIP(hipGraphLaunch(d->into_graph, d->stream));
    d->step += n;
    return FW2_OK;
}

fw2_status fw2_adjoint_workspace_bytes(const fw2_domain *d, uint64_t *bytes)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (!bytes) return fail(FW2_E_INVALID, "bytes is NULL");
    const int nd = d->desc.ndim;
    *bytes = (uint64_t)(state_floats(d) + (int64_t)(5 + 3 * nd) * d->ly.geo.stride) * 4;
    return FW2_OK;
}

fw2_status fw2_adjoint_begin(fw2_domain *d, void *dev_workspace, uint64_t bytes)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (d->desc.relax_scheme != FW2_RELAX_CENTRED)
        return fail(FW2_E_UNSUPPORTED, "the adjoint is derived for the time-centred memory scheme");
    if (d->desc.stencil_mode != FW2_STENCIL_GLOBAL)
        return fail(FW2_E_UNSUPPORTED, "the adjoint is derived for global stencil weights");
    if (d->desc.slab_nz > 0) return fail(FW2_E_UNSUPPORTED, "the adjoint runs on whole grids, not slabs");
    uint64_t need = 0;
    fw2_status st = fw2_adjoint_workspace_bytes(d, &need);
    if (st != FW2_OK) return st;
    if (!dev_workspace || (uintptr_t)dev_workspace % kAlign) return fail(FW2_E_INVALID, "workspace NULL or unaligned");
    if (bytes < need) return fail(FW2_E_NOMEM, "adjoint workspace too small");
    const int64_t S = d->ly.geo.stride;
    const int nd = d->desc.ndim;
    float *base = (float *)dev_workspace;
    fw2::AdjointBuffers &b = d->adj;
    b.lp = base;
    b.pp = base + state_floats(d);
    b.pq = b.pp + S;
    b.sS = b.pq + S;
    b.lDv = b.sS + S;
    b.lqr = b.lDv + nd * S;
    b.lDp = b.lqr + nd * S;
    b.gk = b.lDp + nd * S;
    b.out = b.gk + S;
    FW2_HIP(hipMemsetAsync(dev_workspace, 0, need, d->stream));
    d->adjoint = true;
    d->adj_pp_step = -1;
    return FW2_OK;
}

fw2_status fw2_adjoint_step(fw2_domain *d, const void *dev_state, const void *dev_state_prev, int64_t step,
                            const float *dev_residual)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (!d->adjoint) return fail(FW2_E_STATE, "fw2_adjoint_begin first");
    if (!dev_state || step < 0) return fail(FW2_E_INVALID, "state is NULL or step < 0");
    bool next = false;
    const hipError_t e = fw2::launch_adjoint_step(d->args, d->src, d->rcv, d->desc.n_relax, (const float *)dev_state,
                                                  (const float *)dev_state_prev, d->adj, step,
                                                  d->adj_pp_step == step, dev_residual, d->stream, &next);
    d->adj_pp_step = -1;
    FW2_HIP(e);
    if (next) {                          // p'' of step - 1 is in the second buffer
        std::swap(d->adj.pp, d->adj.pq);
        d->adj_pp_step = step - 1;
    }
    return FW2_OK;
}

fw2_status fw2_adjoint_gradient(fw2_domain *d, float *dst, int32_t kind)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (!d->adjoint) return fail(FW2_E_STATE, "fw2_adjoint_begin first");
    if (!dst || (kind != FW2_HOST && kind != FW2_DEVICE)) return fail(FW2_E_INVALID, "bad destination");
    FW2_HIP(fw2::launch_adjoint_gradient(d->args, d->adj, d->stream));
    const hipMemcpyKind k = kind == FW2_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const int ext[3] = {d->ly.geo.n[0], d->ly.geo.n[1], d->ly.geo.n[2]};
    fw2_status st = copy_box(d, d->adj.out, dst, false, k, ext);
    if (st != FW2_OK) return st;
    FW2_HIP(hipStreamSynchronize(d->stream));
    return FW2_OK;
}

fw2_status fw2_label_relaxation_map(int64_t n_pts, int32_t n_relax, const double *maps, uint8_t *label,
                                    double *table, int32_t *n_labels)
{
    if (!maps || !label || !table || !n_labels) return fail(FW2_E_INVALID, "NULL argument");
    if (n_pts < 1) return fail(FW2_E_INVALID, "n_pts < 1");
    if (n_relax < 1 || n_relax > FW2_MAX_RELAX) return fail(FW2_E_INVALID, "n_relax must be in 1..8");
    const int nrow = 2 + 4 * n_relax;
    // distinct rows are kept in `table`; a hash of each row's bit patterns
    // (FNV-1a over its 8-byte words) finds candidates, compared bitwise
    std::unordered_multimap<uint64_t, int> seen;
    int count = 0, last = -1;
    double row[2 + 4 * FW2_MAX_RELAX];
    for (int64_t i = 0; i < n_pts; ++i) {
        for (int q = 0; q < nrow; ++q) row[q] = maps[(int64_t)q * n_pts + i];
        int lab = -1;
        if (last >= 0 && std::memcmp(table + (size_t)last * nrow, row, (size_t)nrow * 8) == 0) {
            lab = last;                      // neighbouring points mostly share a tissue
        } else {
            uint64_t hsh = 1469598103934665603ull;
            for (int q = 0; q < nrow; ++q) {
                uint64_t bits;
                std::memcpy(&bits, &row[q], 8);
                hsh = (hsh ^ bits) * 1099511628211ull;
            }
            auto range = seen.equal_range(hsh);
            for (auto it = range.first; it != range.second && lab < 0; ++it)
                if (std::memcmp(table + (size_t)it->second * nrow, row, (size_t)nrow * 8) == 0) lab = it->second;
            if (lab < 0) {
                if (count == FW2_MAX_LABELS) return fail(FW2_E_INVALID, "more than 256 distinct relaxation tuples");
                lab = count++;
                std::memcpy(table + (size_t)lab * nrow, row, (size_t)nrow * 8);
                seen.emplace(hsh, lab);
            }
        }
        label[i] = (uint8_t)lab;
        last = lab;
    }
    *n_labels = count;
    return FW2_OK;
}

fw2_status fw2_halo_bytes(const fw2_domain *d, int32_t kind, uint64_t *bytes)
{
    fw2_status st = halo_check(d, kind, FW2_LOW);
    if (st != FW2_OK) return st;
    if (!bytes) return fail(FW2_E_INVALID, "bytes is NULL");
    const fw2::PlaneSet s = halo_planes(d, kind, FW2_LOW, false);
    *bytes = (uint64_t)s.total * (uint64_t)d->ly.geo.n[0] * (uint64_t)d->ly.geo.n[1] * 4u;
    return FW2_OK;
}

fw2_status fw2_halo_pack(fw2_domain *d, int32_t kind, int32_t side, void *dev_dst)
{
    fw2_status st = halo_check(d, kind, side);
    if (st != FW2_OK) return st;
    if (!dev_dst) return fail(FW2_E_INVALID, "dst is NULL");
    FW2_HIP(fw2::launch_pack(halo_planes(d, kind, side, false), d->ly.geo, (float *)dev_dst, d->stream));
    return FW2_OK;
}

fw2_status fw2_halo_unpack(fw2_domain *d, int32_t kind, int32_t side, const void *dev_src)
{
    fw2_status st = halo_check(d, kind, side);
    if (st != FW2_OK) return st;
    if (!dev_src) return fail(FW2_E_INVALID, "src is NULL");
    FW2_HIP(fw2::launch_unpack(halo_planes(d, kind, side, true), d->ly.geo, (const float *)dev_src, d->stream));
    return FW2_OK;
}

fw2_status fw2_stream_probe(int32_t kind, void *dev_buf, uint64_t bytes, void *stream)
{
    if (kind != FW2_PROBE_COPY && kind != FW2_PROBE_VELOCITY_MIX) return fail(FW2_E_INVALID, "unknown probe kind");
    if (!dev_buf) return fail(FW2_E_INVALID, "buf is NULL");
    if ((uintptr_t)dev_buf % kAlign != 0) return fail(FW2_E_INVALID, "buf must be 256-byte aligned");
    if (bytes < 64 * 1024 || bytes > ((uint64_t)1 << 40)) return fail(FW2_E_INVALID, "bytes must lie in [64 KiB, 1 TiB]");
    FW2_HIP(fw2::launch_stream_probe(kind, dev_buf, bytes, (hipStream_t)stream));
    return FW2_OK;
}

fw2_status fw2_step_phase(fw2_domain *d, int32_t phase)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    const int L = d->desc.n_relax, sch = d->desc.relax_scheme;
    if (phase == FW2_PHASE_PRESSURE) {
        if (d->mid_step) return fail(FW2_E_STATE, "the pressure phase of this step already ran");
        FW2_HIP(fw2::launch_pressure(d->args, L, sch, d->kc, d->stream));
        FW2_HIP(fw2::launch_sources(d->src, d->stream));
        d->mid_step = true;
        return FW2_OK;
    }
    if (phase == FW2_PHASE_VELOCITY) {
        if (!d->mid_step) return fail(FW2_E_STATE, "run the pressure phase of the step first");
        if (!d->args.rcv.step) FW2_HIP(fw2::launch_receivers(d->rcv, d->stream));
        FW2_HIP(fw2::launch_velocity(d->args, L, sch, d->kc, d->stream));
        d->mid_step = false;
        d->step++;
        return FW2_OK;
    }
    return fail(FW2_E_INVALID, "phase must be FW2_PHASE_PRESSURE or FW2_PHASE_VELOCITY");
}

fw2_status fw2_check_finite(fw2_domain *d, float limit)
{
    if (!d) return fail(FW2_E_STATE, "domain is NULL");
    if (!(limit > 0.0f)) return fail(FW2_E_INVALID, "limit must be positive");
    FW2_HIP(hipMemsetAsync(d->flag, 0, sizeof(int), d->stream));
    FW2_HIP(fw2::launch_check(d->args.p, d->ly.geo, limit, d->flag, d->stream));
    int h = 0;
    FW2_HIP(hipMemcpyAsync(&h, d->flag, sizeof(int), hipMemcpyDeviceToHost, d->stream));
    FW2_HIP(hipStreamSynchronize(d->stream));
    if (h) return fail(FW2_E_UNSTABLE, "pressure field is not finite or exceeds the limit");
    return FW2_OK;
}

}  // extern "C"

struct fw2_batch {
    int max_domains = 0;
    fw2::BatchTable *dev = nullptr;
    fw2::BatchTable host;
    std::vector<fw2_domain *> doms;
    std::vector<int64_t> target;
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;
    hipGraphExec_t graph = nullptr;
    int graph_chunk = 32;
    int rows = 4;
    int bx = 256;
    unsigned classes = 0;               // launch classes present in the table (fw2::batch_class)
    int static_device = -1;             // >= 0: the table is the library's own on this device
};

namespace {

void batch_drop_graph(fw2_batch *b)
{
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
}

fw2_status batch_build_graph(fw2_batch *b)
{
    if (!b->capture) FW2_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
    FW2_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < b->graph_chunk && e == hipSuccess; ++k)
        e = fw2::launch_batch_step(b->dev, b->max_domains, b->bx, b->classes, b->capture);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->capture, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(FW2_E_HIP, std::string("batch capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&b->graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        b->graph = nullptr;
        return fail(FW2_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    return FW2_OK;
}

// Give domains that leave the batch their exact step counter back.
fw2_status batch_release(fw2_batch *b)
{
    for (fw2_domain *d : b->doms) {
        FW2_HIP(fw2::launch_set_counter(d->counter, d->step, b->stream));
    }
    FW2_HIP(hipStreamSynchronize(b->stream));
    b->doms.clear();
    b->target.clear();
    return FW2_OK;
}

}  // namespace

extern "C" {

fw2_status fw2_batch_workspace_bytes(int32_t max_domains, uint64_t *bytes)
{
    if (max_domains < 1 || max_domains > fw2::kMaxBatch) return fail(FW2_E_INVALID, "max_domains must be in 1..64");
    if (!bytes) return fail(FW2_E_INVALID, "bytes is NULL");
    *bytes = align_up(sizeof(fw2::BatchTable), kAlign);
    return FW2_OK;
}

fw2_status fw2_batch_create(int32_t max_domains, void *dev_workspace, uint64_t workspace_bytes, void *stream,
                            fw2_batch **out)
{
    uint64_t need = 0;
    fw2_status st = fw2_batch_workspace_bytes(max_domains, &need);
    if (st != FW2_OK) return st;
    if (!out) return fail(FW2_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!dev_workspace || (uintptr_t)dev_workspace % kAlign) return fail(FW2_E_INVALID, "workspace NULL or unaligned");
    if (workspace_bytes < need) return fail(FW2_E_NOMEM, "batch workspace too small");
    fw2_batch *b = new (std::nothrow) fw2_batch();
    if (!b) return fail(FW2_E_NOMEM, "host allocation failed");
    fw2::prepare_batch_launches();
    b->max_domains = max_domains;
    b->dev = (fw2::BatchTable *)dev_workspace;
    b->stream = (hipStream_t)stream;
    std::memset(&b->host, 0, sizeof(b->host));
    b->host.rows = b->rows;
    hipError_t e = hipMemcpy(b->dev, &b->host, sizeof(b->host), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete b;
        return fail(FW2_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    *out = b;
    return FW2_OK;
}

fw2_status fw2_batch_set_domains(fw2_batch *b, int32_t n, fw2_domain *const *domains, const int64_t *n_steps)
{
    if (!b) return fail(FW2_E_STATE, "batch is NULL");
    if (n < 0 || n > b->max_domains) return fail(FW2_E_INVALID, "n out of range");
    if (n > 0 && (!domains || !n_steps)) return fail(FW2_E_INVALID, "NULL domains or n_steps");
    for (int32_t k = 0; k < n; ++k) {
        const fw2_domain *d = domains[k];
        if (!d) return fail(FW2_E_INVALID, "NULL domain");
        if (d->desc.ndim != 2) return fail(FW2_E_UNSUPPORTED, "batched stepping is 2D only");
        if (d->desc.n_relax > 4 && b->bx != 256)
            return fail(FW2_E_UNSUPPORTED, "batched domains with more than 4 mechanisms need 256-column tiles");
        if (d->step >= n_steps[k]) return fail(FW2_E_INVALID, "domain already at or past its n_steps");
        for (int32_t q = 0; q < k; ++q)
            if (domains[q] == d) return fail(FW2_E_INVALID, "domain listed twice");
    }
    FW2_HIP(hipStreamSynchronize(b->stream));
    fw2_status st = batch_release(b);
    if (st != FW2_OK) return st;
    fw2::BatchTable &T = b->host;
    std::memset(&T, 0, sizeof(T));
    T.rows = b->rows;
    int tiles = 0, m = 0;
    unsigned classes = 0;
    for (int32_t k = 0; k < n; ++k) {
        fw2_domain *d = domains[k];
        classes |= 1u << fw2::batch_class(d->desc.n_relax, d->args.local_stencil);
        // the domain's own queued work must be finished before the batch stream touches it
        FW2_HIP(hipStreamSynchronize(d->stream));
        b->doms.push_back(d);
        b->target.push_back(n_steps[k]);
    }
    // entries grouped by launch class, so that each class launch walks only
    // its own tiles, spread over every XCD
    for (int c = 0; c < 4; ++c) {
        T.class_begin[c] = tiles;
        for (int32_t k = 0; k < n; ++k) {
            fw2_domain *d = domains[k];
            if (fw2::batch_class(d->desc.n_relax, d->args.local_stencil) != c) continue;
            fw2::BatchEntry &e = T.e[m++];
            e.a = d->args;
            e.src = d->src;
            e.rcv = d->rcv;
            e.n_steps = n_steps[k];
            e.L = d->desc.n_relax;
            e.scheme = d->desc.relax_scheme;
            const int nbx = (d->ly.geo.n[0] + b->bx - 1) / b->bx;
            const int nby = (d->ly.geo.n[1] + b->rows - 1) / b->rows;
            e.tiles = nbx * nby;
            e.tile_base = tiles;
            tiles += e.tiles;
        }
        T.class_end[c] = tiles;
    }
    if (m != n) return fail(FW2_E_INVALID, "a domain of no launch class");
    T.n = n;
    T.total_tiles = tiles;
    if (classes != b->classes) batch_drop_graph(b);    // the captured launches differ
    b->classes = classes;
    FW2_HIP(hipMemcpyAsync(b->dev, &T, sizeof(T), hipMemcpyHostToDevice, b->stream));
    FW2_HIP(hipStreamSynchronize(b->stream));
    return FW2_OK;
}

fw2_status fw2_batch_step(fw2_batch *b, int32_t n)
{
    if (!b) return fail(FW2_E_STATE, "batch is NULL");
    if (n < 0) return fail(FW2_E_INVALID, "n < 0");
    if (n == 0 || b->doms.empty()) return FW2_OK;
    int32_t left = n;
    if (b->graph_chunk > 0 && n >= b->graph_chunk) {
        if (!b->graph) {
            fw2_status st = batch_build_graph(b);
            if (st != FW2_OK) return st;
        }
        for (; left >= b->graph_chunk; left -= b->graph_chunk) FW2_HIP(hipGraphLaunch(b->graph, b->stream));
    }
    for (; left > 0; --left) FW2_HIP(fw2::launch_batch_step(b->dev, b->max_domains, b->bx, b->classes, b->stream));
    for (size_t k = 0; k < b->doms.size(); ++k)
        b->doms[k]->step = std::min<int64_t>(b->doms[k]->step + n, b->target[k]);
    return FW2_OK;
}

fw2_status fw2_batch_set_tile(fw2_batch *b, int32_t cols, int32_t rows)
{
    if (!b) return fail(FW2_E_STATE, "batch is NULL");
    if (rows < 1 || rows > 1024) return fail(FW2_E_INVALID, "rows must be in 1..1024");
    if (cols != 64 && cols != 256) return fail(FW2_E_INVALID, "cols must be 64 or 256");
    if (!b->doms.empty()) return fail(FW2_E_STATE, "set the tile while the batch is empty");
    if (cols != b->bx) batch_drop_graph(b);
    b->bx = cols;
    b->rows = rows;
    b->host.rows = rows;
    FW2_HIP(hipMemcpy(b->dev, &b->host, sizeof(b->host), hipMemcpyHostToDevice));
    return FW2_OK;
}

fw2_status fw2_batch_create_noalloc(int32_t max_domains, void *stream, fw2_batch **out)
{
    if (!out) return fail(FW2_E_INVALID, "out is NULL");
    *out = nullptr;
    if (max_domains < 1 || max_domains > fw2::kMaxBatch)
        return fail(FW2_E_INVALID, "max_domains must be in 1..64 (the library's own table holds 64 domains)");
    int device = -1;
    FW2_HIP(hipGetDevice(&device));
    fw2::BatchTable *table = nullptr;
    bool busy = false;
    FW2_HIP(fw2::claim_static_batch_table(device, &table, &busy));
    if (busy) return fail(FW2_E_STATE, "another no-allocation batch holds this device's table");
    fw2_batch *b = new (std::nothrow) fw2_batch();
    if (!b) {
        fw2::release_static_batch_table(device);
        return fail(FW2_E_NOMEM, "host allocation failed");
    }
    fw2::prepare_batch_launches();
    b->max_domains = max_domains;
    b->dev = table;
    b->static_device = device;
    b->stream = (hipStream_t)stream;
    std::memset(&b->host, 0, sizeof(b->host));
    b->host.rows = b->rows;
    // the table keeps the last batch's contents: start from the empty table
    hipError_t e = hipMemcpy(b->dev, &b->host, sizeof(b->host), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        fw2::release_static_batch_table(device);
        delete b;
        return fail(FW2_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    }
    *out = b;
    return FW2_OK;
}

void fw2_batch_destroy(fw2_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    (void)batch_release(b);
    batch_drop_graph(b);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->static_device >= 0) fw2::release_static_batch_table(b->static_device);
    delete b;
}

void fw2_destroy_domain(fw2_domain *d)
{
    if (!d) return;
    if (d->stream) (void)hipStreamSynchronize(d->stream);
    drop_graph(d);
    if (d->capture) (void)hipStreamDestroy(d->capture);
    for (auto &s : d->ring)
        for (auto &e : s.ev) (void)hipEventDestroy(e);
    delete d;
}

}  // extern "C"
