"""CPU oracle for the D3Q19 binary-fluid lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The GPU library neither imports nor
links anything here, and nothing here imports the GPU package.

Two independent transcriptions of the same step:

* ``lb_oracle.c`` (wrapped below): plain FP64 loops, one site at a time, in the
  order the step is stated (order-parameter gradients, chemical stress,
  collision, propagation -- the Ludwig timestep of the paper, Sec. 2.1.1).
* ``reverse.py``: the same step re-expressed with whole-lattice PyTorch CPU
  FP64 ops (``torch.roll`` for the stencil and propagation) so that autograd
  gives the reverse-mode gradients the hand-written adjoint is checked against.

Arrays are numpy float64, C order; a distribution has shape (19, nx, ny, nz),
a field (nx, ny, nz).  Velocity order: rest, +x, -x, +y, -y, +z, -z, then the
12 edges (+x+y, -x-y, +x-y, -x+y, +x+z, -x-z, +x-z, -x+z, +y+z, -y-z, +y-z,
-y+z).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

NVEL = 19


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("A", ctypes.c_double), ("B", ctypes.c_double), ("kappa", ctypes.c_double),
                ("gamma", ctypes.c_double), ("tau_f", ctypes.c_double),
                ("tau_g", ctypes.c_double), ("rho0", ctypes.c_double),
                ("coupling", ctypes.c_int32), ("order_param", ctypes.c_int32)]


@dataclass
class Params:
    """Lattice extents and model parameters (same meaning as the GPU library's)."""
    nx: int
    ny: int
    nz: int
    A: float = -0.00625
    B: float = 0.00625
    kappa: float = 0.004
    gamma: float = 0.5
    tau_f: float = 1.0
    tau_g: float = 1.0
    rho0: float = 1.0
    coupling: int = 0  # 0: Pi in f^eq; 1: body force -div Pi (Guo forcing)
    order_param: int = 0  # 0: LB distribution g; 1: finite-difference field phi

    @property
    def shape(self):
        return (self.nx, self.ny, self.nz)

    def c(self) -> _Params:
        return _Params(self.nx, self.ny, self.nz, self.A, self.B, self.kappa, self.gamma,
                       self.tau_f, self.tau_g, self.rho0, self.coupling, self.order_param)

    @property
    def mobility(self) -> float:
        """M = Gamma (tau_g - 1/2), the Cahn-Hilliard mobility of both schemes."""
        return self.gamma * (self.tau_g - 0.5)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER(_Params)
    D = ctypes.POINTER(ctypes.c_double)
    lib.oracle_lattice.argtypes = [ctypes.POINTER(ctypes.c_int32), D]
    lib.oracle_order_parameter.argtypes = [P, D, D]
    lib.oracle_gradients.argtypes = [P, D, D, D]
    lib.oracle_chemical.argtypes = [P, D, D, D, D, D]
    lib.oracle_equilibrium_site.argtypes = [P, ctypes.c_double, D, ctypes.c_double,
                                            ctypes.c_double, D, D, D]
    lib.oracle_collide.argtypes = [P, D, D, D, D, D, D, D]
    lib.oracle_stream.argtypes = [P, D, D]
    lib.oracle_step.argtypes = [P, D, D, D, D]
    lib.oracle_step.restype = ctypes.c_int
    lib.oracle_run.argtypes = [P, D, D, ctypes.c_int]
    lib.oracle_run.restype = ctypes.c_int
    lib.oracle_init.argtypes = [P, D, D, D]
    lib.oracle_moments.argtypes = [P, D, D, D, D, D]
    lib.oracle_sum.argtypes = [D, ctypes.c_long]
    lib.oracle_sum.restype = ctypes.c_double
    lib.oracle_force.argtypes = [P, D, D]
    lib.oracle_equilibrium_force_site.argtypes = [P, ctypes.c_double, D, ctypes.c_double,
                                                  ctypes.c_double, D, D]
    lib.oracle_collide_force.argtypes = [P, D, D, D, D, D, D, D]
    lib.oracle_fd_init.argtypes = [P, D, D, D]
    lib.oracle_fd_moments.argtypes = [P, D, D, D, D, D]
    lib.oracle_fd_fluxes.argtypes = [P, D, D, D, D]
    lib.oracle_fd_update.argtypes = [P, D, D, D]
    lib.oracle_fd_step.argtypes = [P, D, D, D, D]
    lib.oracle_fd_step.restype = ctypes.c_int
    lib.oracle_fd_run.argtypes = [P, D, D, ctypes.c_int]
    lib.oracle_fd_run.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def lattice():
    """(c, w): velocities int32 (19, 3) and weights float64 (19,)."""
    lib = _load()
    c = np.zeros((NVEL, 3), dtype=np.int32)
    w = np.zeros(NVEL, dtype=np.float64)
    lib.oracle_lattice(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _ptr(w))
    return c, w


def order_parameter(p: Params, g):
    g = _f64(g)
    phi = np.zeros(p.shape)
    _load().oracle_order_parameter(ctypes.byref(p.c()), _ptr(g), _ptr(phi))
    return phi


def gradients(p: Params, phi):
    """(grad (3, nx, ny, nz), lap (nx, ny, nz)) of a field by 7-point differences."""
    phi = _f64(phi)
    grad = np.zeros((3,) + p.shape)
    lap = np.zeros(p.shape)
    _load().oracle_gradients(ctypes.byref(p.c()), _ptr(phi), _ptr(grad), _ptr(lap))
    return grad, lap


def chemical(p: Params, phi, grad, lap):
    """(mu, Pi) with Pi as (6, nx, ny, nz) in the order xx, xy, xz, yy, yz, zz."""
    phi, grad, lap = _f64(phi), _f64(grad), _f64(lap)
    mu = np.zeros(p.shape)
    pi = np.zeros((6,) + p.shape)
    _load().oracle_chemical(ctypes.byref(p.c()), _ptr(phi), _ptr(grad), _ptr(lap),
                            _ptr(mu), _ptr(pi))
    return mu, pi


def equilibrium_site(p: Params, rho, j, phi, mu, pi6):
    """(feq, geq), each (19,), at one site from its local moments and stress."""
    j = _f64(j)
    pi6 = _f64(pi6)
    feq = np.zeros(NVEL)
    geq = np.zeros(NVEL)
    _load().oracle_equilibrium_site(ctypes.byref(p.c()), float(rho), _ptr(j), float(phi),
                                    float(mu), _ptr(pi6), _ptr(feq), _ptr(geq))
    return feq, geq


def collide(p: Params, f, g, phi, mu, pi):
    f, g, phi, mu, pi = _f64(f), _f64(g), _f64(phi), _f64(mu), _f64(pi)
    fs = np.zeros((NVEL,) + p.shape)
    gs = np.zeros((NVEL,) + p.shape)
    _load().oracle_collide(ctypes.byref(p.c()), _ptr(f), _ptr(g), _ptr(phi), _ptr(mu),
                           _ptr(pi), _ptr(fs), _ptr(gs))
    return fs, gs


def stream(p: Params, dist):
    dist = _f64(dist)
    out = np.zeros_like(dist)
    _load().oracle_stream(ctypes.byref(p.c()), _ptr(dist), _ptr(out))
    return out


def init(p: Params, phi0):
    """Post-stream state at t = 0: f_i = w_i rho0, g_0 = phi0, g_{i>0} = 0."""
    phi0 = _f64(phi0)
    f = np.zeros((NVEL,) + p.shape)
    g = np.zeros((NVEL,) + p.shape)
    _load().oracle_init(ctypes.byref(p.c()), _ptr(phi0), _ptr(f), _ptr(g))
    return f, g


def step(p: Params, f, g):
    f, g = _f64(f), _f64(g)
    fn = np.zeros_like(f)
    gn = np.zeros_like(g)
    if _load().oracle_step(ctypes.byref(p.c()), _ptr(f), _ptr(g), _ptr(fn), _ptr(gn)):
        raise MemoryError("oracle_step: allocation failed")
    return fn, gn


def run(p: Params, f, g, nsteps: int):
    """nsteps timesteps from the post-stream state (f, g); returns new arrays."""
    f = _f64(f).copy()
    g = _f64(g).copy()
    if _load().oracle_run(ctypes.byref(p.c()), _ptr(f), _ptr(g), int(nsteps)):
        raise MemoryError("oracle_run: allocation failed")
    return f, g


def moments(p: Params, f, g):
    """(rho, u (3, nx, ny, nz), phi) of a post-stream state."""
    f, g = _f64(f), _f64(g)
    rho = np.zeros(p.shape)
    u = np.zeros((3,) + p.shape)
    phi = np.zeros(p.shape)
    _load().oracle_moments(ctypes.byref(p.c()), _ptr(f), _ptr(g), _ptr(rho), _ptr(u),
                           _ptr(phi))
    return rho, u, phi


def fsum(x) -> float:
    """FP64 pairwise sum in a fixed order."""
    x = _f64(x).ravel()
    return float(_load().oracle_sum(_ptr(x), x.size))


def sums(p: Params, f, g):
    """(sum rho, sum phi, sum j_x, sum j_y, sum j_z) of a post-stream state."""
    rho, u, phi = moments(p, f, g)
    j = u * rho[None]
    return np.array([fsum(rho), fsum(phi), fsum(j[0]), fsum(j[1]), fsum(j[2])])


def force(p: Params, pi):
    """Body force of the force coupling, F = -div Pi (central differences),
    from the chemical stress pi (6, nx, ny, nz): returns (3, nx, ny, nz)."""
    pi = _f64(pi)
    F = np.empty((3,) + p.shape)
    _load().oracle_force(ctypes.byref(p.c()), _ptr(pi), _ptr(F))
    return F


def equilibrium_force_site(p: Params, rho, u, phi, mu):
    """Force-coupling equilibria (f^eq, g^eq), each (19,), at one site from
    rho, the velocity u (3,), phi and mu."""
    feq = np.empty(NVEL)
    geq = np.empty(NVEL)
    uu = _f64(np.asarray(u, dtype=np.float64))
    _load().oracle_equilibrium_force_site(ctypes.byref(p.c()), float(rho), _ptr(uu), float(phi),
                                          float(mu), _ptr(feq), _ptr(geq))
    return feq, geq


def collide_force(p: Params, f, g, phi, mu, F):
    """BGK collision with the forcing term at every site: (f*, g*)."""
    f, g, phi, mu, F = (_f64(a) for a in (f, g, phi, mu, F))
    fs = np.empty_like(f)
    gs = np.empty_like(g)
    _load().oracle_collide_force(ctypes.byref(p.c()), _ptr(f), _ptr(g), _ptr(phi), _ptr(mu),
                                 _ptr(F), _ptr(fs), _ptr(gs))
    return fs, gs


# -- finite-difference order parameter (order_param = 1) ----------------------
# The state is (f, phi): f (19, nx, ny, nz) post-stream as above, phi a field.

def _fd_check(rc: int, what: str):
    if rc:
        raise MemoryError(f"{what}: allocation failed")


def fd_init(p: Params, phi0):
    """(f, phi) at t = 0: f_i = w_i rho0, phi = phi0."""
    phi0 = _f64(phi0)
    f = np.empty((NVEL,) + p.shape)
    phi = np.empty(p.shape)
    _load().oracle_fd_init(ctypes.byref(p.c()), _ptr(phi0), _ptr(f), _ptr(phi))
    return f, phi


def fd_moments(p: Params, f, phi):
    """(rho, u (3, nx, ny, nz), phi) of a finite-difference state; u = j/rho,
    or (j + F/2)/rho with the force coupling."""
    f, phi = _f64(f), _f64(phi)
    rho = np.empty(p.shape)
    u = np.empty((3,) + p.shape)
    ph = np.empty(p.shape)
    _load().oracle_fd_moments(ctypes.byref(p.c()), _ptr(f), _ptr(phi), _ptr(rho), _ptr(u), _ptr(ph))
    return rho, u, ph


def fd_fluxes(p: Params, phi, mu, u):
    """Face fluxes J (3, nx, ny, nz): J[a] at x is the flux from x to x + e_a
    (upwind advection with the face-averaged velocity, minus M times the
    difference of mu)."""
    phi, mu, u = _f64(phi), _f64(mu), _f64(u)
    J = np.empty((3,) + p.shape)
    _load().oracle_fd_fluxes(ctypes.byref(p.c()), _ptr(phi), _ptr(mu), _ptr(u), _ptr(J))
    return J


def fd_update(p: Params, phi, J):
    """phi - div J (conservative finite-volume update)."""
    phi, J = _f64(phi), _f64(J)
    out = np.empty(p.shape)
    _load().oracle_fd_update(ctypes.byref(p.c()), _ptr(phi), _ptr(J), _ptr(out))
    return out


def fd_step(p: Params, f, phi):
    f, phi = _f64(f), _f64(phi)
    fn = np.empty_like(f)
    pn = np.empty_like(phi)
    _fd_check(_load().oracle_fd_step(ctypes.byref(p.c()), _ptr(f), _ptr(phi), _ptr(fn), _ptr(pn)),
              "oracle_fd_step")
    return fn, pn


def fd_run(p: Params, f, phi, nsteps: int):
    """nsteps finite-difference timesteps from (f, phi); returns new arrays."""
    f = _f64(f).copy()
    phi = _f64(phi).copy()
    _fd_check(_load().oracle_fd_run(ctypes.byref(p.c()), _ptr(f), _ptr(phi), int(nsteps)),
              "oracle_fd_run")
    return f, phi


def fd_sums(p: Params, f, phi):
    """(sum rho, sum phi, sum j_x, sum j_y, sum j_z) of a finite-difference state."""
    rho, u, ph = fd_moments(p, f, phi)
    j = u * rho[None]
    return np.array([fsum(rho), fsum(ph), fsum(j[0]), fsum(j[1]), fsum(j[2])])


def set_threads(n: int) -> int:
    """OpenMP threads of the oracle's site loops (timing only; results do not
    depend on it).  Returns the count now in effect."""
    return int(_load().oracle_set_threads(int(n)))
