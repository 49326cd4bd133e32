"""Reverse mode of a T-step rollout as a torch.autograd.Function.

forward(phi0, A, B, kappa) runs T timesteps on the GPU and returns phi_T.
backward(dL/dphi_T) returns dL/dphi0 and dL/d(A, B, kappa) from the
hand-written adjoint kernels (lb_adjoint_step), with checkpointing and
recomputation: the forward keeps the state every k steps (k = ceil(sqrt(T))
by default); the backward takes each checkpoint in reverse order,
recomputes the k - 1 later states of its segment with lb_step_from (each
written once, straight into its segment buffer), and walks the adjoint back
through them.  Memory: ceil(T/k) + k - 1 states instead of T, plus, for the
LB order parameter in FP64 storage, k - 1 FP64 phi fields (8 bytes per site
each) that hand phi of each recomputed level to its reverse step.

All state copies are lossless (lb_get_state / lb_set_state), and the forward
step is deterministic, so the recomputed states are bit-identical to the
forward's.
"""
from __future__ import annotations

import math

import torch

from .lb import LB


def default_interval(nsteps: int) -> int:
    return max(1, math.ceil(math.sqrt(nsteps)))


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, A, B, kappa, cfg):
        T = int(cfg["nsteps"])
        k = int(cfg.get("interval") or default_interval(T))
        lb = LB(phi0.shape, A=float(A), B=float(B), kappa=float(kappa),
                gamma=cfg.get("gamma", 0.5), tau_f=cfg.get("tau_f", 1.0),
                tau_g=cfg.get("tau_g", 1.0), rho0=cfg.get("rho0", 1.0),
                precision=cfg.get("precision", "fp64"), adjoint=True, device=phi0.device,
                order_param=cfg.get("order_param", "lb"), coupling=cfg.get("coupling", "stress"))
        lb.init_phi(phi0.detach())
        ckpts = []
        t = 0
        while t < T:
            ckpts.append(lb.get_state())
            n = min(k, T - t)
            lb.step(n)
            t += n
        phiT = lb.phi()
        ctx.lb = lb
        ctx.ckpts = ckpts
        ctx.T = T
        ctx.k = k
        return phiT

    @staticmethod
    def backward(ctx, gphi):
        lb, ckpts, T, k = ctx.lb, ctx.ckpts, ctx.T, ctx.k
        dtheta = torch.zeros(3, dtype=torch.float64, device=lb.device)
        lb.adjoint_seed(gphi.detach())
        # segment buffers: the checkpoint itself is the segment's first state;
        # the others are recomputed in place by one step each (no copies)
        seg = [None] + [lb.new_state() for _ in range(min(k, T) - 1)]
        # FP64 storage of the LB order parameter: the recomputing steps also
        # store phi of each level they start from, so the reverse steps of
        # those levels skip their phi pass (FP32 storage finds it in the
        # next level; the finite-difference level holds phi)
        phis = None
        if lb.sizes.elem_bytes == 8 and not lb.fd:
            phis = [torch.empty(lb.shape, dtype=torch.float64, device=lb.device)
                    for _ in range(min(k, T) - 1)]
        for si in reversed(range(len(ckpts))):
            t0 = si * k
            t1 = min(T, t0 + k)
            seg[0] = ckpts[si]
            for j in range(1, t1 - t0):
                lb.step_from(seg[j - 1], seg[j], phi_out=phis[j - 1] if phis else None)
            for t in reversed(range(t0, t1)):
                # level t+1: the next buffer of this segment, else the next
                # segment's checkpoint (none after the last step)
                if t + 1 < t1:
                    nxt = seg[t + 1 - t0]
                    phi = phis[t - t0] if phis else None
                else:
                    nxt = ckpts[si + 1] if si + 1 < len(ckpts) else None
                    phi = None
                lb.adjoint_step(seg[t - t0], dtheta, next_state=nxt, phi=phi)
        dphi0 = lb.adjoint_phi0()
        ctx.lb = None
        ctx.ckpts = None
        return dphi0, dtheta[0], dtheta[1], dtheta[2], None


def rollout(phi0: torch.Tensor, A, B, kappa, nsteps: int, *, interval: int | None = None,
            gamma=0.5, tau_f=1.0, tau_g=1.0, rho0=1.0, precision="fp64",
            order_param="lb", coupling="stress") -> torch.Tensor:
    """phi after `nsteps` steps from the state (rho0, u = 0, phi0); differentiable
    in phi0 (FP64 device tensor (nx, ny, nz)) and in A, B, kappa (tensors or
    floats).  order_param: "lb" (distribution g) or "fd" (finite-difference
    phi field); coupling: "stress" (Pi in f^eq) or "force" (F = -div Pi)."""
    dev = phi0.device
    as_t = lambda v: v if torch.is_tensor(v) else torch.tensor(float(v), dtype=torch.float64,  # noqa: E731
                                                               device=dev)
    cfg = dict(nsteps=nsteps, interval=interval, gamma=gamma, tau_f=tau_f, tau_g=tau_g,
               rho0=rho0, precision=precision, order_param=order_param, coupling=coupling)
    return _Rollout.apply(phi0, as_t(A), as_t(B), as_t(kappa), cfg)
