"""Reverse mode of a T-step rollout as a torch.autograd.Function.

forward(phi0, A, B, kappa) runs T timesteps on the GPU and returns phi_T.
backward(dL/dphi_T) returns dL/dphi0 and dL/d(A, B, kappa) from the
hand-written adjoint kernels (lb_adjoint_step), with checkpointing and
recomputation: the forward keeps the state every k steps (k = ceil(sqrt(T))
by default); the backward takes each checkpoint in reverse order,
recomputes the k - 1 later states of its segment with lb_step_from (each
written once, straight into its segment buffer), and walks the adjoint back
through them.  Memory: ceil(T/k) + max(k - 1, 2) states instead of T (the
checkpoints, and the segment buffers or the forward's two scratch levels),
plus, for the LB order parameter, FP64 phi fields (8 bytes per site each) that hand phi of
each level to its reverse step, so that none runs a phi pass: k - 1 for the
recomputed levels, and one per segment for its last level, stored by the
forward step that leaves it.  The forward writes each checkpoint with the
step that produces it, so a small k costs no copies.  interval="auto" sizes k
to the device's memory: on a 288 GB MI355X the 128^3 FP32-storage rollout of
1000 steps keeps every second state instead of every 32nd.

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


def backward_bytes(nsteps: int, k: int, state_bytes: int, phi_bytes: int = 0) -> int:
    """Device memory the rollout holds at checkpoint interval k, at its
    peak: ceil(T/k) checkpoints, and k - 1 segment buffers (backward) or two
    scratch levels (forward), of state_bytes each; ceil(T/k) + k - 1 phi
    fields of phi_bytes (the LB order parameter's: one per segment from the
    forward, one per recomputed level)."""
    k = max(1, min(int(k), nsteps))
    c = math.ceil(nsteps / k)
    return (c + max(k - 1, 2)) * state_bytes + (c + k - 1) * phi_bytes


def interval_for_budget(nsteps: int, state_bytes: int, budget_bytes: int,
                        phi_bytes: int = 0) -> int:
    """The smallest checkpoint interval (fewest recomputed steps) whose
    backward fits in budget_bytes; ValueError if none does (the memory is
    least near k = sqrt(T))."""
    for k in range(1, max(1, nsteps) + 1):
        if backward_bytes(nsteps, k, state_bytes, phi_bytes) <= budget_bytes:
            return k
        if k > 2 * default_interval(nsteps):
            break  # past the minimum of the memory, near sqrt(T)
    raise ValueError(f"no checkpoint interval fits {budget_bytes} bytes "
                     f"({nsteps} steps of {state_bytes}-byte states)")


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, A, B, kappa, cfg):
        T = int(cfg["nsteps"])
        lb = LB(phi0.shape, A=float(A), B=float(B), kappa=float(kappa),
                gamma=cfg.get("gamma", 0.5), tau_f=cfg.get("tau_f", 1.0),
                tau_g=cfg.get("tau_g", 1.0), rho0=cfg.get("rho0", 1.0),
                precision=cfg.get("precision", "fp64"), adjoint=True, device=phi0.device,
                order_param=cfg.get("order_param", "lb"), coupling=cfg.get("coupling", "stress"))
        interval = cfg.get("interval")
        # phi fields of the LB order parameter (the finite-difference level
        # holds phi itself)
        phi_b = 0 if lb.fd else lb.nsites * 8
        if interval == "auto":
            # as few recomputed steps as the memory allows: the caller's
            # budget, else 90% of what the device has free now (including
            # what torch's allocator holds cached, which it can hand out)
            budget = cfg.get("memory_budget")
            if budget is None:
                dev = phi0.device
                cached = torch.cuda.memory_reserved(dev) - torch.cuda.memory_allocated(dev)
                budget = int(0.9 * (torch.cuda.mem_get_info(dev)[0] + cached))
            k = interval_for_budget(T, int(lb.sizes.state_bytes), int(budget), phi_b)
        else:
            k = int(interval or default_interval(T))
        lb.init_phi(phi0.detach())
        # each step writes a caller buffer (lb_step_from): a segment's last
        # step straight into the next checkpoint, its others into two scratch
        # levels, so the checkpoints cost no copies; the rollout's final
        # step goes to a scratch level that becomes the context's, which
        # phi() reads.  The last step of each segment also stores phi of the
        # level it leaves (lb_step_from_phi), which that level's reverse step
        # needs and no recomputation forms.
        ckpts = [lb.get_state()]
        ends = []
        work = [lb.new_state(), lb.new_state()] if T > 0 else []
        t = 0
        while t < T:
            n = min(k, T - t)
            src = ckpts[-1]
            for j in range(n):
                ph = None
                if j == n - 1 and phi_b:
                    ph = torch.empty(lb.shape, dtype=torch.float64, device=lb.device)
                    ends.append(ph)
                if t + j == T - 1:
                    dst = work[1] if src is work[0] else work[0]
                elif j == n - 1:
                    dst = lb.new_state()
                else:
                    dst = work[j & 1]
                lb.step_from(src, dst, phi_out=ph)
                src = dst
            if t + n < T:
                ckpts.append(src)
            t += n
        if T > 0:
            lb.set_state(src)
        del work
        phiT = lb.phi()
        ctx.lb = lb
        ctx.ckpts = ckpts
        ctx.ends = ends
        ctx.T = T
        ctx.k = k
        cfg["interval_used"] = k
        return phiT

    @staticmethod
    def backward(ctx, gphi):
        lb, ckpts, ends, T, k = ctx.lb, ctx.ckpts, ctx.ends, ctx.T, ctx.k
        dtheta = torch.zeros(3, dtype=torch.float64, device=lb.device)
        lb.adjoint_seed(gphi.detach())
        # segment buffers: the checkpoint itself is the segment's first state;
        # the others are recomputed in place by one step each (no copies)
        seg = [None] + [lb.new_state() for _ in range(min(k, T) - 1)]
        # LB order parameter: the recomputing steps also store phi of each
        # level they start from, and the forward stored phi of each segment's
        # last level, so no reverse step runs a phi pass (the
        # finite-difference level holds phi)
        phis = None
        if not lb.fd:
            phis = [torch.empty(lb.shape, dtype=torch.float64, device=lb.device)
                    for _ in range(min(k, T) - 1)]
        for si in reversed(range(len(ckpts) if T > 0 else 0)):
            t0 = si * k
            t1 = min(T, t0 + k)
            seg[0] = ckpts[si]
            for j in range(1, t1 - t0):
                lb.step_from(seg[j - 1], seg[j], phi_out=phis[j - 1] if phis else None)
            for t in reversed(range(t0, t1)):
                if t + 1 < t1:
                    phi = phis[t - t0] if phis else None
                else:
                    phi = ends[si] if ends else None
                lb.adjoint_step(seg[t - t0], dtheta, phi=phi)
        dphi0 = lb.adjoint_phi0()
        ctx.lb = None
        ctx.ckpts = None
        ctx.ends = None
        return dphi0, dtheta[0], dtheta[1], dtheta[2], None


def rollout(phi0: torch.Tensor, A, B, kappa, nsteps: int, *, interval: int | str | None = None,
            memory_budget: int | None = None, gamma=0.5, tau_f=1.0, tau_g=1.0, rho0=1.0,
            precision="fp64", order_param="lb", coupling="stress",
            info: dict | None = None) -> torch.Tensor:
    """phi after `nsteps` steps from the state (rho0, u = 0, phi0); differentiable
    in phi0 (FP64 device tensor (nx, ny, nz)) and in A, B, kappa (tensors or
    floats).  order_param: "lb" (distribution g) or "fd" (finite-difference
    phi field); coupling: "stress" (Pi in f^eq) or "force" (F = -div Pi).
    interval: the checkpoint interval k (default ceil(sqrt(T))), or "auto":
    the smallest k whose peak memory (backward_bytes) fits in memory_budget
    bytes (default 90% of the device's free memory, counting what torch's
    allocator holds cached), i.e. as many checkpoints as HBM holds and as
    few recomputed steps.  The gradients do not depend on k (the recomputed
    states are bit-identical).  info (a dict, optional) receives "interval",
    the k used."""
    dev = phi0.device
    as_t = lambda v: v if torch.is_tensor(v) else torch.tensor(float(v), dtype=torch.float64,  # noqa: E731
                                                               device=dev)
    cfg = dict(nsteps=nsteps, interval=interval, memory_budget=memory_budget, gamma=gamma,
               tau_f=tau_f, tau_g=tau_g, rho0=rho0, precision=precision,
               order_param=order_param, coupling=coupling)
    out = _Rollout.apply(phi0, as_t(A), as_t(B), as_t(kappa), cfg)
    if info is not None:
        info["interval"] = cfg.get("interval_used")
    return out
