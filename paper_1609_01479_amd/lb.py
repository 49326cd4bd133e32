"""Python front end of the C ABI: device memory (torch tensors) and streams.

Every step of the computation runs in the HIP kernels behind the C ABI; this
module only allocates the caller-owned device buffers, passes pointers and
the stream handle, and wraps results as torch tensors.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _abi
from ._abi import LB_FP32_DEV, LB_FP64, NVEL, check


# distribution layouts (lb_layout); every layout gives bit-identical results
LAYOUTS = {"rows": 0, "soa": 1, "aos": 2, "aosoa": 3}
# how the chemical stress drives the flow (lb_coupling)
COUPLINGS = {"stress": 0, "force": 1}
# step kernels (lb_kernel): one pass, a phi pass plus a collision pass (the
# same results), or the one-pass kernel's memory-only twin (free streaming)
KERNELS = {"fused": 0, "two_pass": 1, "stream": 2}
# how the order parameter evolves (lb_order_param): LB distribution g, or a
# field with the finite-difference Cahn-Hilliard update and upwind advection
ORDER_PARAMS = {"lb": 0, "fd": 1}


def _precision_code(precision) -> int:
    if precision in ("fp64", "f64", LB_FP64):
        return LB_FP64
    if precision in ("fp32", "fp32_dev", "f32", LB_FP32_DEV):
        return LB_FP32_DEV
    raise ValueError(f"unknown precision {precision!r}")


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class LB:
    """One D3Q19 binary-fluid lattice on one GPU.

    shape: (nx, ny, nz) periodic extents.  Model parameters as in lb.h.
    precision: "fp64" or "fp32_dev" (FP32 deviation storage).
    adjoint: also allocate the reverse-mode buffers.
    kernel: "fused" (one pass per step) or "two_pass" (phi pass + collision pass);
        "stream" is the fused kernel's memory-only twin (free streaming, no
        collision), for measurement.
    segment_x: x planes per workgroup of the fused kernel (0 = automatic).
    layout: memory layout of the distributions, "rows" (row-blocked, default),
        "soa", "aos" or "aosoa" with aosoa_len z-sites per block (a power of
        two dividing nz); results are bit-identical across layouts.
    coupling: "stress" (Pi in the f equilibrium, default) or "force" (body
        force -div Pi with the half-force velocity).
    order_param: "lb" (distribution g, default) or "fd" (a phi field with the
        finite-difference Cahn-Hilliard update and upwind advection, mobility
        Gamma (tau_g - 1/2); either coupling; no g).
    """

    def __init__(self, shape, *, A=-0.00625, B=0.00625, kappa=0.004, gamma=0.5, tau_f=1.0,
                 tau_g=1.0, rho0=1.0, precision="fp64", adjoint=False, device=None,
                 stream: torch.cuda.Stream | None = None, kernel="fused", segment_x=0,
                 layout="rows", aosoa_len=0, coupling="stress", order_param="lb",
                 halo_x=False):
        L = _abi.lib()
        nx, ny, nz = (int(v) for v in shape)
        self.shape = (nx, ny, nz)
        self.nsites = nx * ny * nz
        self.precision = _precision_code(precision)
        self.params = _abi.LbParams(nx, ny, nz, float(A), float(B), float(kappa), float(gamma),
                                    float(tau_f), float(tau_g), float(rho0), self.precision,
                                    KERNELS[kernel], int(segment_x),
                                    LAYOUTS[layout], int(aosoa_len), COUPLINGS[coupling],
                                    ORDER_PARAMS[order_param], 1 if halo_x else 0)
        self.halo_x = bool(halo_x)
        self.fd = self.params.order_param == ORDER_PARAMS["fd"]
        self.sizes = _abi.LbSizes()
        check(L.lb_query_sizes(ctypes.byref(self.params), ctypes.byref(self.sizes)),
              "lb_query_sizes")
        self.device = torch.device(device) if device is not None else torch.device(
            "cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        sz = self.sizes
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            alloc = lambda n: torch.empty(int(n), dtype=torch.uint8, device=self.device)  # noqa: E731
            self.state_buf = [alloc(sz.state_bytes), alloc(sz.state_bytes)]
            self.phi_buf = alloc(sz.phi_bytes)
            self.scratch = alloc(sz.scratch_bytes)
            self.adj_buf = [alloc(sz.adj_bytes), alloc(sz.adj_bytes)] if adjoint else [None, None]
            self.adj_scratch = alloc(sz.adj_scratch_bytes) if adjoint else None
        bufs = _abi.LbBuffers()
        bufs.state[0] = self.state_buf[0].data_ptr()
        bufs.state[1] = self.state_buf[1].data_ptr()
        bufs.phi = self.phi_buf.data_ptr()
        bufs.scratch = self.scratch.data_ptr()
        if adjoint:
            bufs.adj[0] = self.adj_buf[0].data_ptr()
            bufs.adj[1] = self.adj_buf[1].data_ptr()
            bufs.adj_scratch = self.adj_scratch.data_ptr()
        self._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.lb_create(ctypes.byref(self.params), ctypes.byref(bufs),
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._ctx)),
                  "lb_create")

    def sibling(self, kernel: str) -> "LB":
        """A second context on this lattice's own device buffers and stream
        that steps with another kernel variant ("fused", "two_pass" or
        "stream"), e.g. to time a kernel and its memory-only twin on the same
        memory.  It starts at time level 0 of the shared buffers; the caller
        keeps the two contexts from stepping over each other's levels."""
        L = _abi.lib()
        sib = object.__new__(LB)
        sib.__dict__.update({k: v for k, v in self.__dict__.items() if k != "_ctx"})
        sib.params = _abi.LbParams.from_buffer_copy(self.params)
        sib.params.kernel = KERNELS[kernel]
        sib.sizes = _abi.LbSizes()
        check(L.lb_query_sizes(ctypes.byref(sib.params), ctypes.byref(sib.sizes)), "lb_query_sizes")
        for f in ("state_bytes", "phi_bytes", "scratch_bytes"):
            if getattr(sib.sizes, f) > getattr(self.sizes, f):
                raise ValueError(f"kernel {kernel!r} needs more {f} than this lattice holds")
        bufs = _abi.LbBuffers()
        bufs.state[0] = self.state_buf[0].data_ptr()
        bufs.state[1] = self.state_buf[1].data_ptr()
        bufs.phi = self.phi_buf.data_ptr()
        bufs.scratch = self.scratch.data_ptr()
        if self.adj_buf[0] is not None:
            bufs.adj[0] = self.adj_buf[0].data_ptr()
            bufs.adj[1] = self.adj_buf[1].data_ptr()
            bufs.adj_scratch = self.adj_scratch.data_ptr()
        sib._ctx = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            check(L.lb_create(ctypes.byref(sib.params), ctypes.byref(bufs),
                              ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(sib._ctx)),
                  "lb_create")
        return sib

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            _abi.lib().lb_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, name, *args):
        with torch.cuda.device(self.device):
            check(getattr(_abi.lib(), name)(self._ctx, *args), name)

    def _dev64(self, a, shape=None) -> torch.Tensor:
        t = torch.as_tensor(a)
        t = t.to(device=self.device, dtype=torch.float64, non_blocking=False).contiguous()
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def _out(self, *shape) -> torch.Tensor:
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            return torch.empty(shape, dtype=torch.float64, device=self.device)

    def _sync_inputs(self):
        # inputs produced on torch's current stream must be visible to ours
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    # -- forward ------------------------------------------------------------
    def init_phi(self, phi0) -> None:
        """phi0 of shape (nx, ny, nz); an x-slab shard (halo_x) takes
        (nx + 2, ny, nz): the neighbours' planes -1 and nx around its own."""
        nx, ny, nz = self.shape
        t = self._dev64(phi0, (nx + 2, ny, nz) if self.halo_x else self.shape)
        self._sync_inputs()
        self._call("lb_init_phi", _ptr(t))
        t.record_stream(self.stream)

    def step(self, nsteps: int = 1) -> None:
        self._call("lb_step", ctypes.c_int32(int(nsteps)))

    def step_sums(self, nsteps: int, out: torch.Tensor | None = None) -> torch.Tensor:
        """Advance nsteps and return the (nsteps, 5) FP64 device tensor of the
        conserved sums [rho, phi, jx, jy, jz] of each step's starting state."""
        if out is None:
            out = self._out(int(nsteps), 5)
        if out.dtype != torch.float64 or out.numel() < 5 * nsteps or not out.is_contiguous():
            raise ValueError("out must be a contiguous FP64 tensor of 5*nsteps values")
        self._call("lb_step_sums", ctypes.c_int32(int(nsteps)), _ptr(out))
        return out

    def step_sums_noalloc(self, nsteps: int, out: torch.Tensor) -> torch.Tensor:
        """step_sums through the allocation-free entry point
        (lb_step_sums_noalloc): the reduction partials live in the library's
        own device array, and `out` must be given (nothing is allocated)."""
        if out.dtype != torch.float64 or out.numel() < 5 * nsteps or not out.is_contiguous():
            raise ValueError("out must be a contiguous FP64 tensor of 5*nsteps values")
        self._call("lb_step_sums_noalloc", ctypes.c_int32(int(nsteps)), _ptr(out))
        return out

    def new_state(self) -> torch.Tensor:
        """An uninitialised device buffer of one time level (state_bytes)."""
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            return torch.empty(int(self.sizes.state_bytes), dtype=torch.uint8, device=self.device)

    def step_from(self, src: torch.Tensor, dst: torch.Tensor,
                  phi_out: torch.Tensor | None = None) -> None:
        """One step from the time level in `src` into `dst` (caller buffers);
        phi_out (LB order parameter): an FP64 device tensor of
        the lattice's shape that receives phi of `src`, for adjoint_step."""
        for t in (src, dst):
            if t.numel() * t.element_size() != self.sizes.state_bytes:
                raise ValueError("state buffer has the wrong size")
        if phi_out is None:
            self._call("lb_step_from", _ptr(src), _ptr(dst))
        else:
            self._check_phi(phi_out)
            self._call("lb_step_from_phi", _ptr(src), _ptr(dst), _ptr(phi_out))

    def _check_phi(self, t: torch.Tensor) -> None:
        if (t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != self.nsites
                or t.device != self.device):
            raise ValueError("phi must be a contiguous FP64 device tensor of the lattice's size")

    def moments(self):
        """(rho (nx,ny,nz), u (3,nx,ny,nz), phi (nx,ny,nz)) as FP64 device tensors."""
        rho = self._out(*self.shape)
        u = self._out(3, *self.shape)
        phi = self._out(*self.shape)
        self._call("lb_moments", _ptr(rho), _ptr(u), _ptr(phi))
        return rho, u, phi

    def phi(self) -> torch.Tensor:
        out = self._out(*self.shape)
        self._call("lb_moments", None, None, _ptr(out))
        return out

    def sums(self) -> torch.Tensor:
        """[sum rho, sum phi, sum jx, sum jy, sum jz] (FP64 device tensor)."""
        out = self._out(5)
        self._call("lb_sums", _ptr(out))
        return out

    def get_state(self, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = self.new_state()
        self._call("lb_get_state", _ptr(out))
        return out

    def set_state(self, src: torch.Tensor) -> None:
        if src.numel() * src.element_size() != self.sizes.state_bytes:
            raise ValueError("state buffer has the wrong size")
        self._sync_inputs()
        self._call("lb_set_state", _ptr(src))

    def export_dist(self):
        """Dense post-propagation (f, g), each FP64 (19, nx, ny, nz); g is None
        for the finite-difference order parameter."""
        f = self._out(NVEL, *self.shape)
        g = None if self.fd else self._out(NVEL, *self.shape)
        self._call("lb_export_dist", _ptr(f), _ptr(g))
        return f, g

    def import_dist(self, f, g=None) -> None:
        """Set the state from dense (f, g); with order_param "fd", g is None
        and phi keeps its values."""
        tf = self._dev64(f, (NVEL,) + self.shape)
        tg = None if g is None else self._dev64(g, (NVEL,) + self.shape)
        self._sync_inputs()
        self._call("lb_import_dist", _ptr(tf), _ptr(tg))
        tf.record_stream(self.stream)
        if tg is not None:
            tg.record_stream(self.stream)

    # -- reverse mode -------------------------------------------------------
    def adjoint_seed(self, dphi) -> None:
        t = self._dev64(dphi, self.shape)
        self._sync_inputs()
        self._call("lb_adjoint_seed", _ptr(t))
        t.record_stream(self.stream)

    def adjoint_step(self, state_t: torch.Tensor, dtheta: torch.Tensor | None = None,
                     phi: torch.Tensor | None = None) -> None:
        """One reverse step at state_t; phi, phi of state_t from
        step_from(..., phi_out=), spares the step its phi pass
        (lb_adjoint_step_phi)."""
        if phi is not None:
            self._check_phi(phi)
            self._call("lb_adjoint_step_phi", _ptr(state_t), _ptr(phi), _ptr(dtheta))
        else:
            self._call("lb_adjoint_step", _ptr(state_t), _ptr(dtheta))

    def adjoint_dist(self):
        """(dL/df, dL/dg) of the current adjoint level as FP64 (19, nx, ny, nz)
        tensors (lb_adjoint_export; dL/dg is None for the finite-difference
        order parameter, whose dL/dphi is adjoint_phi0())."""
        if self.adj_buf[0] is None:
            raise RuntimeError("created without adjoint buffers")
        lf = self._out(NVEL, *self.shape)
        lg = None if self.fd else self._out(NVEL, *self.shape)
        self._call("lb_adjoint_export", _ptr(lf), _ptr(lg))
        return lf, lg

    def adjoint_phi0(self) -> torch.Tensor:
        out = self._out(*self.shape)
        self._call("lb_adjoint_phi0", _ptr(out))
        return out

    # -- x-slab shards (halo_x) -------------------------------------------
    def new_face(self) -> torch.Tensor:
        """An uninitialised device buffer for one face (face_bytes)."""
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            return torch.empty(int(self.sizes.face_bytes), dtype=torch.uint8, device=self.device)

    def pack_faces(self, send_lo: torch.Tensor | None, send_hi: torch.Tensor | None) -> None:
        """The shard's faces for its lower and upper neighbours (lb_pack_faces)."""
        self._call("lb_pack_faces", _ptr(send_lo), _ptr(send_hi))

    def unpack_faces(self, recv_lo: torch.Tensor | None, recv_hi: torch.Tensor | None) -> None:
        """The neighbours' faces into the halo planes (lb_unpack_faces)."""
        self._sync_inputs()
        self._call("lb_unpack_faces", _ptr(recv_lo), _ptr(recv_hi))

    def synchronize(self):
        self.stream.synchronize()


def to_numpy(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def copy_probe_gbps(nbytes: int, reps: int = 20, device="cuda:0") -> float:
    """Bandwidth (read + write bytes / time) of the library's streaming copy
    kernel over `nbytes` -- the practical HBM ceiling."""
    dev = torch.device(device)
    nbytes = nbytes // 256 * 256
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream(dev)
    L = _abi.lib()
    call = lambda: check(L.lb_copy_probe(ctypes.c_void_p(a.data_ptr()),  # noqa: E731
                                         ctypes.c_void_p(b.data_ptr()), ctypes.c_size_t(nbytes),
                                         ctypes.c_void_p(stream.cuda_stream)), "lb_copy_probe")
    # warm-up: at least 3 calls and 30 ms of copying (after host work or an
    # idle spell the GPU runs its first tens of milliseconds of work slowly)
    w0 = torch.cuda.Event(enable_timing=True)
    w1 = torch.cuda.Event(enable_timing=True)
    n, done = 3, 0.0
    while done < 30.0:
        w0.record(stream)
        for _ in range(n):
            call()
        w1.record(stream)
        w1.synchronize()
        done += w0.elapsed_time(w1)
        n *= 2
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        call()
    e1.record(stream)
    e1.synchronize()
    if not torch.equal(a[:1024], b[:1024]):
        raise RuntimeError("copy probe produced wrong data")
    ms = e0.elapsed_time(e1) / reps
    return 2.0 * nbytes / (ms * 1e-3) / 1e9
