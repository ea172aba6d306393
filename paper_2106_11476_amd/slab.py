"""A 3D grid split along z into slabs, advanced with halo exchange.

Sec. 5.3 remarks that the spatial and temporal locality of the
finite-difference update suits several GPUs.  Split along the slowest axis z,
a slab needs from each neighbour, per step:

  after the pressure phase   4 planes of p               (fw2 HALO_P)
  after the velocity phase   4 planes of v_z and 1 plane
                             each of v_x and v_y          (fw2 HALO_V)

and once, after creation, 1 plane of rho and kappa0 (HALO_MEDIUM).  The
memory variables are point-local and stay where they are.  Each slab is a
libfw2 slab domain (its boundary layer follows the global plane index); the
library packs a face into a contiguous buffer and unpacks a neighbour's face
into the halo.  Here every slab lives on one device and a packed face goes
straight from one slab's pack to its neighbour's unpack; with one slab per GPU
the same buffers would travel between the two calls (an RCCL send/recv over
xGMI).  Orchestration only: every step runs in the library's kernels.
"""
import copy

import numpy as np

from . import fw2


def split_problem(prob, bounds, only=None):
    """Slab problems of a 3D problem for z boundaries bounds = [0, z1, ..., nz]
    (only: indices of the slabs to build, default all).

    Each slab gets its planes of the maps, its sources and receivers (local
    flat indices), slab_z0 / slab_nz, and the stencil Courant number and
    layer speed of the whole grid (fd_r, pml_cp), so that every slab uses
    the constants the whole grid would.  Returns (slabs, rcv_cols): rcv_cols[k]
    lists the global receiver columns slab k records."""
    if len(prob.shape) != 3:
        raise ValueError("slabs split a 3D grid")
    nx, ny, nz = (int(s) for s in prob.shape)
    b = [int(x) for x in bounds]
    if b[0] != 0 or b[-1] != nz or any(b[k + 1] - b[k] < 4 for k in range(len(b) - 1)):
        raise ValueError("bounds must run from 0 to nz in steps of at least 4 planes")
    grid = (nz, ny, nx)
    c = np.asarray(prob.c, np.float32).reshape(grid)
    cmax = float(c.max())
    fd_r = float(prob.fd_r) if prob.fd_r and prob.fd_r > 0 else cmax * float(prob.dt) / float(prob.h)
    pml_cp = float(prob.pml_cp) if prob.pml_cp and prob.pml_cp > 0 else cmax
    plane = nx * ny
    src = np.asarray(prob.src_idx, np.int64)
    rcv = np.asarray(prob.rcv_idx, np.int64)
    slabs, cols = [], []
    for k in (range(len(b) - 1) if only is None else only):
        z0, z1 = b[k], b[k + 1]
        s = copy.copy(prob)
        s.shape = (nx, ny, z1 - z0)
        s.c = c[z0:z1].copy()
        s.rho = np.asarray(prob.rho, np.float32).reshape(grid)[z0:z1].copy()
        s.beta = np.asarray(prob.beta, np.float32).reshape(grid)[z0:z1].copy()
        s.label = None if prob.label is None else np.asarray(prob.label).reshape(grid)[z0:z1].copy()
        s.fd_r, s.pml_cp = fd_r, pml_cp
        s.slab_z0, s.slab_nz = z0, nz
        m = (src >= z0 * plane) & (src < z1 * plane)
        s.src_idx = src[m] - z0 * plane
        s.src_sig = np.asarray(prob.src_sig)[m]
        s.src_w = np.asarray(prob.src_w)[m]
        r = np.nonzero((rcv >= z0 * plane) & (rcv < z1 * plane))[0]
        s.rcv_idx = rcv[r] - z0 * plane
        s.name = "%s_slab%d" % (prob.name, k)
        slabs.append(s)
        cols.append(r)
    return slabs, cols


class SlabSet:
    """The slabs of one grid on one device, stepped with halo exchange
    (only: consecutive slab indices, to hold a part of the grid; its outer
    faces then keep zero halos)."""

    def __init__(self, prob, bounds, device="cuda", stream=None, cap_steps=None, only=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.shape = tuple(int(s) for s in prob.shape)
        self.bounds = [int(x) for x in bounds]
        self.n_rcv = len(prob.rcv_idx)
        probs, self.rcv_cols = split_problem(prob, bounds, only)
        cap = cap_steps if cap_steps is not None else max(int(prob.n_steps), 1)
        self.domains = []
        for s in probs:
            d = fw2.Domain(s, device=device, stream=self.stream)
            if len(s.src_idx):
                d.add_source(s.src_idx, s.src_sig, s.src_w, s.signals)
            if len(s.rcv_idx):
                d.add_receivers(s.rcv_idx, cap)
            self.domains.append(d)
        # one buffer per neighbour pair and direction, sized for the largest kind
        self.buf = []
        for k in range(len(self.domains) - 1):
            n = max(self.domains[k].halo_numel(kind) for kind in (fw2.HALO_P, fw2.HALO_V, fw2.HALO_MEDIUM))
            self.buf.append((torch.empty(n, dtype=torch.float32, device=self.device),
                             torch.empty(n, dtype=torch.float32, device=self.device)))
        self.exchange(fw2.HALO_MEDIUM)

    def exchange(self, kind):
        """Halo exchange of one kind between every pair of neighbours."""
        for k in range(len(self.domains) - 1):
            lo, hi = self.domains[k], self.domains[k + 1]
            up, down = self.buf[k]
            lo.halo_pack(kind, fw2.HIGH, up)
            hi.halo_unpack(kind, fw2.LOW, up)
            hi.halo_pack(kind, fw2.LOW, down)
            lo.halo_unpack(kind, fw2.HIGH, down)

    def step(self, n):
        for _ in range(int(n)):
            for d in self.domains:
                d.step_phase(fw2.PHASE_PRESSURE)
            self.exchange(fw2.HALO_P)
            for d in self.domains:
                d.step_phase(fw2.PHASE_VELOCITY)
            self.exchange(fw2.HALO_V)

    def read_fields(self, mask=fw2.FIELD_ALL):
        """The whole grid's fields, assembled from the slabs' planes."""
        parts = [d.read_fields(mask) for d in self.domains]
        return {name: np.concatenate([p[name] for p in parts], axis=-3) for name in parts[0]}

    def traces(self):
        """[steps][n_rcv] of the whole grid's receivers."""
        rows = None
        out = None
        for d, cols in zip(self.domains, self.rcv_cols):
            if len(cols) == 0:
                continue
            t = d.trace.cpu().numpy()
            if out is None:
                rows = t.shape[0]
                out = np.zeros((rows, self.n_rcv), np.float32)
            out[:, cols] = t
        return out

    def destroy(self):
        for d in self.domains:
            d.destroy_domain()
        self.domains = []
