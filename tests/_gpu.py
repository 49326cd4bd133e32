"""Helpers shared by the GPU tests: run the HIP path and the oracle on the
same seeded inputs and compare."""
from __future__ import annotations

import numpy as np
import torch

import lbinputs
import oracle


def params(shape, **kw):
    base = dict(lbinputs.SPINODAL_PARAMS)
    base.update(kw)
    return base


def make_lb(shape, precision="fp64", adjoint=False, **kw):
    from paper_1609_01479_amd import LB
    return LB(shape, precision=precision, adjoint=adjoint, device="cuda:0", **params(shape, **kw))


def oracle_params(shape, **kw):
    return oracle.Params(*shape, **params(shape, **kw))


def rel_err(a, ref, floor: float = 0.0) -> float:
    """max |a - ref| / max(max |ref|, floor): per-site error over the field's
    scale (phi and u cross zero, so a pointwise relative error is undefined)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = max(float(np.abs(ref).max()), floor)
    if scale == 0.0:
        return float(np.abs(a).max())
    return float(np.abs(a - ref).max() / scale)


# The velocity is a difference of O(rho) populations (j = sum_i f_i c_i), so
# its rounding error is O(eps) in lattice units whatever |u| is; its scale is
# therefore at least the lattice speed 1.
FLOORS = {"f": 0.0, "g": 0.0, "rho": 0.0, "u": 1.0, "phi": 0.0}


def field_errors(got, ref, names=("f", "g", "rho", "u", "phi")):
    return {n: rel_err(a, b, FLOORS[n]) for n, a, b in zip(names, got, ref)}


def gpu_state(lb):
    f, g = lb.export_dist()
    rho, u, phi = lb.moments()
    torch.cuda.synchronize()
    return tuple(t.cpu().numpy() for t in (f, g, rho, u, phi))


def oracle_state(p, f, g):
    rho, u, phi = oracle.moments(p, f, g)
    return f, g, rho, u, phi
