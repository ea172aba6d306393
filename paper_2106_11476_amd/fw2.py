"""Thin ctypes binding of libfw2 (include/fw2.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch provides device memory (the workspace, source tables, traces) and the
stream.  The binding fails loudly if the library has not been built.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfw2.so")

FW2_OK = 0
STATUS = {0: "FW2_OK", 1: "FW2_E_INVALID", 2: "FW2_E_NOMEM", 3: "FW2_E_HIP", 4: "FW2_E_STATE",
          5: "FW2_E_UNSTABLE", 6: "FW2_E_UNSUPPORTED"}
FIELD_P, FIELD_V, FIELD_PSI1, FIELD_PSI2, FIELD_ALL = 1, 2, 4, 8, 15
HOST, DEVICE = 0, 1
RELAX_PRINTED, RELAX_CENTRED = 0, 1
STENCIL_GLOBAL, STENCIL_LOCAL = 0, 1
NL_PRINTED, NL_CUSTOM = 0, 1
HALO_P, HALO_V, HALO_MEDIUM = 0, 1, 2
PROBE_COPY, PROBE_VELOCITY_MIX = 0, 1
LOW, HIGH = 0, 1
PHASE_PRESSURE, PHASE_VELOCITY = 0, 1
MAX_LABELS = 256

EXPORTS = ["fw2_workspace_bytes", "fw2_create_domain", "fw2_add_source", "fw2_add_receivers",
           "fw2_step", "fw2_read_fields", "fw2_write_fields", "fw2_current_step",
           "fw2_set_current_step", "fw2_set_stream", "fw2_set_graph_chunk", "fw2_enable_kernel_timing",
           "fw2_get_kernel_timing", "fw2_check_finite", "fw2_last_error", "fw2_destroy_domain",
           "fw2_batch_workspace_bytes", "fw2_batch_create", "fw2_batch_set_domains",
           "fw2_batch_step", "fw2_batch_set_tile", "fw2_batch_destroy",
           "fw2_state_bytes", "fw2_save_state", "fw2_load_state", "fw2_adjoint_workspace_bytes",
           "fw2_adjoint_begin", "fw2_adjoint_step", "fw2_adjoint_gradient",
           "fw2_label_relaxation_map", "fw2_halo_bytes", "fw2_halo_pack", "fw2_halo_unpack",
           "fw2_step_phase", "fw2_batch_create_noalloc", "fw2_step_into", "fw2_stream_probe"]


class Fw2Error(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class DomainDesc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("n_relax", ctypes.c_int32), ("n", ctypes.c_int64 * 3),
        ("h", ctypes.c_double), ("dt", ctypes.c_double),
        ("bound_cells", ctypes.c_int32 * 3), ("trans_cells", ctypes.c_int32 * 3),
        ("pml_Rc", ctypes.c_double), ("pml_npoly", ctypes.c_int32), ("pml_cp", ctypes.c_double),
        ("fd_r", ctypes.c_double), ("relax_scheme", ctypes.c_int32), ("stencil_mode", ctypes.c_int32),
        ("c", ctypes.c_void_p), ("rho", ctypes.c_void_p), ("beta", ctypes.c_void_p),
        ("label", ctypes.c_void_p), ("n_labels", ctypes.c_int32), ("relax_table", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("nonlinear_form", ctypes.c_int32), ("nl_A", ctypes.c_double), ("nl_B0", ctypes.c_double),
        ("nl_B1", ctypes.c_double), ("map_kind", ctypes.c_int32),
        ("slab_z0", ctypes.c_int64), ("slab_nz", ctypes.c_int64),
    ]


_lib = None


def lib():
    """Load libfw2.so; raise if it is missing (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libfw2.so is not built (run __graft_entry__.build()); there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
        sig = {
            "fw2_workspace_bytes": [ctypes.POINTER(DomainDesc), ctypes.POINTER(u64)],
            "fw2_create_domain": [ctypes.POINTER(DomainDesc), vp, u64, ctypes.POINTER(vp)],
            "fw2_add_source": [vp, i32, vp, vp, vp, i32, i32, vp],
            "fw2_add_receivers": [vp, i32, vp, vp, i64],
            "fw2_step": [vp, i32],
            "fw2_read_fields": [vp, u32, vp, i32],
            "fw2_write_fields": [vp, u32, vp, i32],
            "fw2_set_current_step": [vp, i64],
            "fw2_set_graph_chunk": [vp, i32],
            "fw2_set_stream": [vp, vp],
            "fw2_enable_kernel_timing": [vp, i32],
            "fw2_get_kernel_timing": [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)],
            "fw2_check_finite": [vp, ctypes.c_float],
            "fw2_batch_workspace_bytes": [i32, ctypes.POINTER(u64)],
            "fw2_batch_create": [i32, vp, u64, vp, ctypes.POINTER(vp)],
            "fw2_batch_set_domains": [vp, i32, ctypes.POINTER(vp), ctypes.POINTER(i64)],
            "fw2_batch_step": [vp, i32],
            "fw2_batch_set_tile": [vp, i32, i32],
            "fw2_state_bytes": [vp, ctypes.POINTER(u64)],
            "fw2_save_state": [vp, vp],
            "fw2_load_state": [vp, vp, i64],
            "fw2_step_into": [vp, i32, vp, vp],
            "fw2_adjoint_workspace_bytes": [vp, ctypes.POINTER(u64)],
            "fw2_adjoint_begin": [vp, vp, u64],
            "fw2_adjoint_step": [vp, vp, vp, i64, vp],
            "fw2_adjoint_gradient": [vp, vp, i32],
            "fw2_label_relaxation_map": [i64, i32, vp, vp, vp, ctypes.POINTER(i32)],
            "fw2_halo_bytes": [vp, i32, ctypes.POINTER(u64)],
            "fw2_halo_pack": [vp, i32, i32, vp],
            "fw2_halo_unpack": [vp, i32, i32, vp],
            "fw2_step_phase": [vp, i32],
            "fw2_batch_create_noalloc": [i32, vp, ctypes.POINTER(vp)],
            "fw2_stream_probe": [i32, vp, u64, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.fw2_current_step.argtypes = [vp]
        L.fw2_current_step.restype = i64
        L.fw2_last_error.argtypes = []
        L.fw2_last_error.restype = ctypes.c_char_p
        L.fw2_destroy_domain.argtypes = [vp]
        L.fw2_destroy_domain.restype = None
        L.fw2_batch_destroy.argtypes = [vp]
        L.fw2_batch_destroy.restype = None
        _lib = L
    return _lib


def _check(status):
    if status != FW2_OK:
        raise Fw2Error(status, lib().fw2_last_error().decode())


def make_desc(prob, stream=None):
    """Fill a DomainDesc from a problem description (workloads.Problem-like).

    Returns (desc, keepalive) -- the numpy buffers must outlive the call that
    consumes desc."""
    nd = len(prob.shape)
    keep = []

    def host(arr, dtype):
        a = np.ascontiguousarray(np.asarray(arr), dtype=dtype)
        keep.append(a)
        return a.ctypes.data

    d = DomainDesc()
    d.ndim = nd
    d.n_relax = int(prob.n_relax)
    n3 = list(prob.shape) + [1] * (3 - nd)
    for a in range(3):
        d.n[a] = int(n3[a])
        d.bound_cells[a] = int(prob.bound_cells[a]) if a < nd else 0
        d.trans_cells[a] = int(prob.trans_cells[a]) if a < nd else 0
    d.h, d.dt = float(prob.h), float(prob.dt)
    d.pml_Rc, d.pml_npoly, d.pml_cp = float(prob.pml_Rc), int(prob.pml_npoly), float(prob.pml_cp or 0.0)
    d.fd_r = float(prob.fd_r or 0.0)
    d.relax_scheme = int(getattr(prob, "relax_scheme", RELAX_CENTRED))
    d.stencil_mode = int(getattr(prob, "stencil_mode", STENCIL_GLOBAL))
    d.c = host(prob.c, np.float32)
    d.rho = host(prob.rho, np.float32)
    d.beta = host(prob.beta, np.float32)
    table = np.asarray(prob.relax_table, dtype=np.float64)
    d.n_labels = int(table.shape[0])
    d.relax_table = host(table, np.float64)
    d.label = host(prob.label, np.uint8) if (prob.label is not None and d.n_labels > 1) else None
    d.stream = stream.value if isinstance(stream, ctypes.c_void_p) else stream
    d.nonlinear_form = int(getattr(prob, "nonlinear_form", NL_PRINTED))
    d.nl_A = float(getattr(prob, "nl_A", 1.0))
    d.nl_B0 = float(getattr(prob, "nl_B0", 1.0))
    d.nl_B1 = float(getattr(prob, "nl_B1", -2.0))
    d.map_kind = HOST
    d.slab_z0 = int(getattr(prob, "slab_z0", 0))
    d.slab_nz = int(getattr(prob, "slab_nz", 0))
    return d, keep


def stream_probe_elements(kind, nbytes):
    """Elements the probe of `kind` covers in a buffer of nbytes: float4
    copies for PROBE_COPY, points per array for PROBE_VELOCITY_MIX."""
    return nbytes // 32 if kind == PROBE_COPY else nbytes // 84 // 64 * 64


def stream_probe(kind, buf, stream=None):
    """Run fw2_stream_probe over the device buffer `buf` (a torch tensor),
    asynchronously on `stream` (default: torch's current stream)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(buf.device)
    _check(lib().fw2_stream_probe(int(kind), ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                                  ctypes.c_void_p(st.cuda_stream)))


def label_relaxation_map(maps, n_relax):
    """fw2_label_relaxation_map: dense per-point relaxation maps
    ([2 + 4L] + grid, FP64) to (uint8 labels of the grid's shape, table
    [n_labels][2 + 4L])."""
    m = np.ascontiguousarray(np.asarray(maps, dtype=np.float64))
    nrow = 2 + 4 * int(n_relax)
    if m.shape[0] != nrow:
        raise ValueError("maps must have 2 + 4L = %d parameter maps" % nrow)
    npts = int(np.prod(m.shape[1:]))
    label = np.empty(npts, np.uint8)
    table = np.empty((MAX_LABELS, nrow), np.float64)
    n = ctypes.c_int32(0)
    _check(lib().fw2_label_relaxation_map(npts, int(n_relax), ctypes.c_void_p(m.ctypes.data),
                                          ctypes.c_void_p(label.ctypes.data), ctypes.c_void_p(table.ctypes.data),
                                          ctypes.byref(n)))
    return label.reshape(m.shape[1:]), table[:int(n.value)].copy()


def workspace_bytes(prob):
    d, keep = make_desc(prob)
    out = ctypes.c_uint64(0)
    _check(lib().fw2_workspace_bytes(ctypes.byref(d), ctypes.byref(out)))
    return int(out.value)


class Domain:
    """One simulation domain resident on the GPU (fw2_create_domain).

    The workspace is a torch uint8 tensor; sources, receivers and traces are
    torch device tensors held by this object for as long as the library may
    read them."""

    def __init__(self, prob, device="cuda", stream=None, device_maps=False):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.shape = tuple(int(s) for s in prob.shape)
        self.ndim = len(self.shape)
        self.L = int(prob.n_relax)
        self.slab_z0 = int(getattr(prob, "slab_z0", 0))
        self.slab_nz = int(getattr(prob, "slab_nz", 0))
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        d, keep = make_desc(prob, ctypes.c_void_p(stream.cuda_stream))
        if device_maps:
            # c, rho, beta (and labels) handed over as device tensors; the
            # library converts them on the GPU
            grid = self.shape[::-1]
            dev = {}
            for name in ("c", "rho", "beta"):
                dev[name] = torch.as_tensor(np.ascontiguousarray(np.asarray(getattr(prob, name), np.float32)
                                                                 .reshape(grid)), device=self.device)
            d.c, d.rho, d.beta = (ctypes.c_void_p(dev[n].data_ptr()).value for n in ("c", "rho", "beta"))
            if d.label:
                dev["label"] = torch.as_tensor(np.ascontiguousarray(np.asarray(prob.label, np.uint8).reshape(grid)),
                                               device=self.device)
                d.label = dev["label"].data_ptr()
            d.map_kind = DEVICE
            keep.append(dev)
        nbytes = ctypes.c_uint64(0)
        _check(lib().fw2_workspace_bytes(ctypes.byref(d), ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        # inputs prepared on the current stream are complete before the library
        # uses them on its own stream (other streams keep running)
        torch.cuda.current_stream(self.device).synchronize()
        h = ctypes.c_void_p()
        _check(lib().fw2_create_domain(ctypes.byref(d), ctypes.c_void_p(self.workspace.data_ptr()),
                                       self.workspace_bytes, ctypes.byref(h)))
        self._h = h
        del keep
        self._src = None
        self._rcv = None
        self.trace = None

    # -- C entry points -------------------------------------------------
    def add_source(self, flat_idx, sig_id, weight, signals):
        t = self.torch
        idx = t.as_tensor(np.asarray(flat_idx, np.int64), device=self.device).contiguous()
        sig = t.as_tensor(np.asarray(sig_id, np.int32), device=self.device).contiguous()
        w = t.as_tensor(np.asarray(weight, np.float32), device=self.device).contiguous()
        s = np.asarray(signals, np.float32)
        if s.ndim == 1:
            s = s[None, :]
        sg = t.as_tensor(np.ascontiguousarray(s), device=self.device).contiguous()
        t.cuda.current_stream(self.device).synchronize()
        _check(lib().fw2_add_source(self._h, int(idx.numel()), ctypes.c_void_p(idx.data_ptr()),
                                    ctypes.c_void_p(sig.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                    int(sg.shape[0]), int(sg.shape[1]), ctypes.c_void_p(sg.data_ptr())))
        self._src = (idx, sig, w, sg)

    def add_receivers(self, flat_idx, cap_steps):
        t = self.torch
        idx = t.as_tensor(np.asarray(flat_idx, np.int64), device=self.device).contiguous()
        n = int(idx.numel())
        trace = t.zeros((int(cap_steps), max(n, 1)), dtype=t.float32, device=self.device)
        t.cuda.current_stream(self.device).synchronize()
        _check(lib().fw2_add_receivers(self._h, n, ctypes.c_void_p(idx.data_ptr()),
                                       ctypes.c_void_p(trace.data_ptr()), int(cap_steps)))
        self._rcv = idx
        self.trace = trace[:, :n]

    def step(self, n):
        _check(lib().fw2_step(self._h, int(n)))

    def current_step(self):
        return int(lib().fw2_current_step(self._h))

    def set_current_step(self, step):
        _check(lib().fw2_set_current_step(self._h, int(step)))

    def set_graph_chunk(self, steps):
        _check(lib().fw2_set_graph_chunk(self._h, int(steps)))

    def set_stream(self, stream):
        """Queue this domain's later calls on another torch stream (after the
        work on its current stream has finished)."""
        _check(lib().fw2_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def enable_kernel_timing(self, enable=True):
        _check(lib().fw2_enable_kernel_timing(self._h, 1 if enable else 0))

    def get_kernel_timing(self):
        ms = (ctypes.c_double * 2)()
        cnt = (ctypes.c_int64 * 2)()
        _check(lib().fw2_get_kernel_timing(self._h, ms, cnt))
        return [ms[0], ms[1]], [cnt[0], cnt[1]]

    def check_finite(self, limit=1e12):
        _check(lib().fw2_check_finite(self._h, float(limit)))

    # -- slabs of a grid split along z -------------------------------------
    def step_phase(self, phase):
        _check(lib().fw2_step_phase(self._h, int(phase)))

    def halo_numel(self, kind):
        n = ctypes.c_uint64(0)
        _check(lib().fw2_halo_bytes(self._h, int(kind), ctypes.byref(n)))
        return int(n.value) // 4

    def halo_pack(self, kind, side, dst):
        _check(lib().fw2_halo_pack(self._h, int(kind), int(side), ctypes.c_void_p(dst.data_ptr())))

    def halo_unpack(self, kind, side, src):
        _check(lib().fw2_halo_unpack(self._h, int(kind), int(side), ctypes.c_void_p(src.data_ptr())))

    # -- state blocks and the discrete adjoint -----------------------------
    def state_bytes(self):
        n = ctypes.c_uint64(0)
        _check(lib().fw2_state_bytes(self._h, ctypes.byref(n)))
        return int(n.value)

    def new_state_buffer(self, count=None):
        """Zero-filled device buffer for one state block, or [count] blocks.
        Each block starts 240 bytes past a 256-byte boundary, as the domain's
        own fields do, so that its rows sit on the same cache lines."""
        B = self.state_bytes() // 4
        n = 1 if count is None else int(count)
        raw = self.torch.zeros(n * B + 64, dtype=self.torch.float32, device=self.device)
        off = ((240 - raw.data_ptr() % 256) % 256) // 4
        buf = raw[off:off + n * B]
        return buf if count is None else buf.view(n, B)

    def save_state(self, dst):
        _check(lib().fw2_save_state(self._h, ctypes.c_void_p(dst.data_ptr())))

    def load_state(self, src, step):
        _check(lib().fw2_load_state(self._h, ctypes.c_void_p(src.data_ptr()), int(step)))

    def step_into(self, n, first, states):
        """n steps out of place from the state block `first` (at the current
        step) into states[0..n-1] (zero-filled once, see new_state_buffer);
        the domain's own fields are left as they are."""
        if n > 0 and (states.dim() != 2 or states.shape[0] < n or states.shape[1] * 4 != self.state_bytes()):
            raise ValueError("states must be [>= n, state_bytes / 4]")
        _check(lib().fw2_step_into(self._h, int(n), ctypes.c_void_p(first.data_ptr()),
                                   ctypes.c_void_p(states.data_ptr())))

    def adjoint_begin(self):
        n = ctypes.c_uint64(0)
        _check(lib().fw2_adjoint_workspace_bytes(self._h, ctypes.byref(n)))
        self._adj_ws = self.torch.empty(int(n.value), dtype=self.torch.uint8, device=self.device)
        self.torch.cuda.synchronize(self.device)
        _check(lib().fw2_adjoint_begin(self._h, ctypes.c_void_p(self._adj_ws.data_ptr()), int(n.value)))

    def adjoint_step(self, state, step, residual=None, prev=None):
        """Reverse of step `step` from its input state; prev: the input state
        of step - 1 if at hand (lets the library fuse its recompute)."""
        r = ctypes.c_void_p(residual.data_ptr()) if residual is not None else None
        q = ctypes.c_void_p(prev.data_ptr()) if prev is not None else None
        _check(lib().fw2_adjoint_step(self._h, ctypes.c_void_p(state.data_ptr()), q, int(step), r))

    def adjoint_gradient(self):
        """dJ/dc as a device tensor of the grid's shape ([nz][ny][nx])."""
        out = self.torch.empty(self.shape[::-1],
                               dtype=self.torch.float32, device=self.device)
        _check(lib().fw2_adjoint_gradient(self._h, ctypes.c_void_p(out.data_ptr()), DEVICE))
        return out

    def _sizes(self, mask):
        grid = self.shape[::-1]
        out = []
        if mask & FIELD_P:
            out.append(("p", grid))
        if mask & FIELD_V:
            out.append(("v", (self.ndim,) + grid))
        if mask & FIELD_PSI1:
            out.append(("psi1", (self.ndim, self.L) + grid))
        if mask & FIELD_PSI2:
            out.append(("psi2", (self.ndim, self.L) + grid))
        return out

    def read_fields(self, mask=FIELD_ALL):
        """Return {name: float32 numpy array} of the selected fields."""
        parts = self._sizes(mask)
        total = sum(int(np.prod(s)) for _, s in parts)
        buf = np.empty(total, np.float32)
        _check(lib().fw2_read_fields(self._h, mask, ctypes.c_void_p(buf.ctypes.data), HOST))
        out, o = {}, 0
        for name, s in parts:
            k = int(np.prod(s))
            out[name] = buf[o:o + k].reshape(s)
            o += k
        return out

    def field_numel(self, mask=FIELD_ALL):
        """Elements of the packed layout of the selected fields."""
        return sum(int(np.prod(s)) for _, s in self._sizes(mask))

    def read_fields_device(self, mask=FIELD_ALL):
        """Selected fields packed into one torch device tensor."""
        total = self.field_numel(mask)
        buf = self.torch.empty(total, dtype=self.torch.float32, device=self.device)
        _check(lib().fw2_read_fields(self._h, mask, ctypes.c_void_p(buf.data_ptr()), DEVICE))
        return buf

    def write_fields_device(self, buf, mask=FIELD_ALL):
        """Write the selected fields from one packed torch device tensor (the
        layout read_fields_device returns)."""
        total = self.field_numel(mask)
        if buf.numel() != total or buf.dtype != self.torch.float32 or not buf.is_contiguous():
            raise ValueError("expected a contiguous float32 tensor of %d elements" % total)
        self.torch.cuda.current_stream(self.device).synchronize()
        _check(lib().fw2_write_fields(self._h, mask, ctypes.c_void_p(buf.data_ptr()), DEVICE))

    def field_views(self, buf, mask=FIELD_ALL):
        """{name: view} of a packed field tensor (host or device)."""
        out, o = {}, 0
        for name, s in self._sizes(mask):
            k = int(np.prod(s))
            out[name] = buf[o:o + k].reshape(s)
            o += k
        return out

    def write_fields(self, fields, mask=None):
        """fields: dict name -> array (names as read_fields returns)."""
        if mask is None:
            mask = sum(b for n, b in (("p", FIELD_P), ("v", FIELD_V), ("psi1", FIELD_PSI1),
                                      ("psi2", FIELD_PSI2)) if n in fields)
        parts = self._sizes(mask)
        buf = np.concatenate([np.asarray(fields[n], np.float32).reshape(-1) for n, _ in parts])
        _check(lib().fw2_write_fields(self._h, mask, ctypes.c_void_p(buf.ctypes.data), HOST))

    def destroy_domain(self):
        if getattr(self, "_h", None):
            lib().fw2_destroy_domain(self._h)
            self._h = None

    close = destroy_domain

    def __del__(self):
        try:
            self.destroy_domain()
        except Exception:
            pass


class Batch:
    """Batched stepping of several resident 2D domains (fw2_batch_*)."""

    def __init__(self, max_domains=64, device="cuda", stream=None, noalloc=False):
        """noalloc: fw2_batch_create_noalloc (the library's own table, no
        workspace)."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        h = ctypes.c_void_p()
        if noalloc:
            self.workspace = None
            with torch.cuda.device(self.device):
                _check(lib().fw2_batch_create_noalloc(int(max_domains), ctypes.c_void_p(self.stream.cuda_stream),
                                                      ctypes.byref(h)))
        else:
            nb = ctypes.c_uint64(0)
            _check(lib().fw2_batch_workspace_bytes(int(max_domains), ctypes.byref(nb)))
            self.workspace = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
            torch.cuda.synchronize(self.device)
            _check(lib().fw2_batch_create(int(max_domains), ctypes.c_void_p(self.workspace.data_ptr()),
                                          int(nb.value), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.max_domains = int(max_domains)
        self.domains = []

    def set_domains(self, domains, n_steps):
        n = len(domains)
        arr = (ctypes.c_void_p * max(n, 1))(*[d._h.value for d in domains])
        steps = (ctypes.c_int64 * max(n, 1))(*[int(x) for x in n_steps])
        _check(lib().fw2_batch_set_domains(self._h, n, arr, steps))
        self.domains = list(domains)

    def step(self, n):
        _check(lib().fw2_batch_step(self._h, int(n)))

    def set_tile(self, cols, rows):
        _check(lib().fw2_batch_set_tile(self._h, int(cols), int(rows)))

    def destroy(self):
        if getattr(self, "_h", None):
            lib().fw2_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def create_domain(prob, device="cuda", stream=None):
    """fw2_create_domain for a problem description; returns a Domain."""
    return Domain(prob, device=device, stream=stream)


def from_problem(prob, device="cuda", stream=None, cap_steps=None):
    """Domain with the problem's sources and receivers attached."""
    dom = Domain(prob, device=device, stream=stream)
    if len(prob.src_idx):
        dom.add_source(prob.src_idx, prob.src_sig, prob.src_w, prob.signals)
    if len(prob.rcv_idx):
        dom.add_receivers(prob.rcv_idx, cap_steps if cap_steps is not None else max(int(prob.n_steps), 1))
    return dom
