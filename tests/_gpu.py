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


def rel_err(a, ref) -> float:
    """max |a - ref| / max |ref| (field scale; phi and u cross zero)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    if scale == 0.0:
        return float(np.abs(a).max())
    return float(np.abs(a - ref).max() / scale)


def gpu_state(lb):
    f, g = lb.export_dist()
    rho, u, phi = lb.moments()
    torch.cuda.synchronize()
    return tuple(t.cpu().numpy() for t in (f, g, rho, u, phi))


def oracle_state(p, f, g):
    rho, u, phi = oracle.moments(p, f, g)
    return f, g, rho, u, phi
