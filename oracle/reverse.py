"""Whole-lattice PyTorch CPU FP64 re-expression of the binary-fluid LB step.

TEST INFRASTRUCTURE ONLY (see the package docstring).  This is a second,
independent transcription of the step in ``lb_oracle.c``: the stencil and the
propagation are ``torch.roll`` shifts of whole fields instead of per-site
index arithmetic, and the equilibria are written with the explicit second
moment tensors.  Because every operation is a differentiable torch op,
autograd gives the exact reverse-mode gradient of any loss on the final state
with respect to the initial order parameter and the free-energy parameters
(A, B, kappa) -- the reference the hand-written GPU adjoint is checked
against.

The state is the post-stream pair (f, g), each a (19, nx, ny, nz) float64
tensor.  Velocity order as in ``lb_oracle.c``.
"""
from __future__ import annotations

import torch

# D3Q19 velocities (same order as the C oracle; a second hand-written copy).
VEL = torch.tensor([
    [0, 0, 0],
    [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
    [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0],
    [1, 0, 1], [-1, 0, -1], [1, 0, -1], [-1, 0, 1],
    [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1],
], dtype=torch.int64)

_C2 = (VEL * VEL).sum(1)
WEIGHTS = torch.where(_C2 == 0, torch.tensor(1.0 / 3.0, dtype=torch.float64),
                      torch.where(_C2 == 1, torch.tensor(1.0 / 18.0, dtype=torch.float64),
                                  torch.tensor(1.0 / 36.0, dtype=torch.float64)))
CF = VEL.to(torch.float64)
# Q_i = c_i c_i - I/3, shape (19, 3, 3)
QT = CF[:, :, None] * CF[:, None, :] - torch.eye(3, dtype=torch.float64)[None] / 3.0


def _shift(phi, axis, s):
    """Field value at x + s e_axis (periodic)."""
    return torch.roll(phi, shifts=-s, dims=axis)


def gradients(phi):
    grad = torch.stack([0.5 * (_shift(phi, a, 1) - _shift(phi, a, -1)) for a in range(3)])
    lap = sum(_shift(phi, a, 1) + _shift(phi, a, -1) - 2.0 * phi for a in range(3))
    return grad, lap


def chemical(phi, grad, lap, A, B, kappa):
    mu = A * phi + B * phi ** 3 - kappa * lap
    g2 = (grad * grad).sum(0)
    iso = 0.5 * A * phi ** 2 + 0.75 * B * phi ** 4 - kappa * phi * lap - 0.5 * kappa * g2
    eye = torch.eye(3, dtype=phi.dtype)
    pi = iso[None, None] * eye[:, :, None, None, None] \
        + kappa * grad[:, None] * grad[None, :]
    return mu, pi  # pi: (3, 3, nx, ny, nz)


def equilibria(rho, j, phi, mu, pi, gamma):
    u = j / rho[None]
    mf = pi + rho[None, None] * u[:, None] * u[None, :]
    eye = torch.eye(3, dtype=rho.dtype)[:, :, None, None, None]
    mg = (gamma * mu - phi / 3.0)[None, None] * eye + phi[None, None] * u[:, None] * u[None, :]
    cj = torch.einsum("ia,axyz->ixyz", CF, j)
    cu = torch.einsum("ia,axyz->ixyz", CF, u)
    qf = torch.einsum("iab,abxyz->ixyz", QT, mf)
    qg = torch.einsum("iab,abxyz->ixyz", QT, mg)
    w = WEIGHTS[:, None, None, None]
    feq = w * (rho[None] + 3.0 * cj + 4.5 * qf)
    geq = w * (phi[None] + 3.0 * phi[None] * cu + 4.5 * qg)
    return feq, geq


def propagate(dist):
    """out_i(x + c_i) = in_i(x), periodic."""
    return torch.stack([torch.roll(dist[i], shifts=tuple(int(v) for v in VEL[i]),
                                   dims=(0, 1, 2)) for i in range(19)])


def step(f, g, A, B, kappa, gamma, tau_f, tau_g):
    phi = g.sum(0)
    grad, lap = gradients(phi)
    mu, pi = chemical(phi, grad, lap, A, B, kappa)
    rho = f.sum(0)
    j = torch.einsum("ia,ixyz->axyz", CF, f)
    feq, geq = equilibria(rho, j, phi, mu, pi, gamma)
    fs = f - (f - feq) / tau_f
    gs = g - (g - geq) / tau_g
    return propagate(fs), propagate(gs)


# -- force coupling: F = -div Pi by central differences, Guo forcing ---------
# f^eq keeps only the ideal part (Pi leaves the equilibrium), both equilibria
# take u = (j + F/2)/rho, and the source (1 - 1/(2 tau_f)) w_i
# [3(c_i - u) + 9 (c_i.u) c_i].F adds F to each site's momentum.

def body_force(pi):
    """F_a = -sum_b D_b Pi_ab, shape (3, nx, ny, nz)."""
    return torch.stack([-sum(0.5 * (_shift(pi[a, b], b, 1) - _shift(pi[a, b], b, -1))
                             for b in range(3)) for a in range(3)])


def _collide_f_force(f, rho, j, F, phi, mu, gamma, tau_f):
    """(f*, g^eq, u) of the forcing collision; g^eq uses the same u."""
    jh = j + 0.5 * F
    feq, geq = equilibria(rho, jh, phi, mu, torch.zeros((3, 3) + tuple(rho.shape),
                                                        dtype=rho.dtype), gamma)
    u = jh / rho[None]
    cu = torch.einsum("ia,axyz->ixyz", CF, u)
    cF = torch.einsum("ia,axyz->ixyz", CF, F)
    uF = (u * F).sum(0)
    src = (1.0 - 0.5 / tau_f) * WEIGHTS[:, None, None, None] * (3.0 * (cF - uF[None])
                                                               + 9.0 * cu * cF)
    return f - (f - feq) / tau_f + src, geq, u


def step_force(f, g, A, B, kappa, gamma, tau_f, tau_g):
    phi = g.sum(0)
    grad, lap = gradients(phi)
    mu, pi = chemical(phi, grad, lap, A, B, kappa)
    F = body_force(pi)
    rho = f.sum(0)
    j = torch.einsum("ia,ixyz->axyz", CF, f)
    fs, geq, _ = _collide_f_force(f, rho, j, F, phi, mu, gamma, tau_f)
    gs = g - (g - geq) / tau_g
    return propagate(fs), propagate(gs)


def initial_state(phi0, rho0):
    shape = phi0.shape
    f = WEIGHTS[:, None, None, None] * rho0 * torch.ones((19,) + tuple(shape), dtype=torch.float64)
    g = torch.cat([phi0[None], torch.zeros((18,) + tuple(shape), dtype=torch.float64)])
    return f, g


def rollout_phi(phi0, A, B, kappa, nsteps, gamma=0.5, tau_f=1.0, tau_g=1.0, rho0=1.0,
                coupling="stress"):
    """phi after nsteps from the standard initial state; differentiable."""
    f, g = initial_state(phi0, rho0)
    stepper = step_force if coupling == "force" else step
    for _ in range(nsteps):
        f, g = stepper(f, g, A, B, kappa, gamma, tau_f, tau_g)
    return g.sum(0)


def loss_and_grads(phi0, target, A, B, kappa, nsteps, gamma=0.5, tau_f=1.0, tau_g=1.0,
                   rho0=1.0, coupling="stress"):
    """L = 1/2 sum_x (phi_T - phi*)^2 and its gradients (dphi0, dA, dB, dkappa).

    phi0, target: float64 numpy or tensors of shape (nx, ny, nz).
    """
    p0 = torch.as_tensor(phi0, dtype=torch.float64).clone().requires_grad_(True)
    tA = torch.tensor(float(A), dtype=torch.float64, requires_grad=True)
    tB = torch.tensor(float(B), dtype=torch.float64, requires_grad=True)
    tk = torch.tensor(float(kappa), dtype=torch.float64, requires_grad=True)
    phiT = rollout_phi(p0, tA, tB, tk, nsteps, gamma, tau_f, tau_g, rho0, coupling)
    tgt = torch.as_tensor(target, dtype=torch.float64)
    loss = 0.5 * ((phiT - tgt) ** 2).sum()
    loss.backward()
    return (float(loss.detach()), p0.grad.numpy().copy(), float(tA.grad), float(tB.grad),
            float(tk.grad))


# -- finite-difference order parameter (stress coupling) ----------------------
# The state is (f, phi): f post-stream as above, phi a field.  phi follows
# the conservative face-flux update: upwind advection with the face-averaged
# velocity u = j/rho of f before collision, minus M times the difference of
# mu, M = Gamma (tau_g - 1/2); torch.where routes the upwind value's
# derivative to the side it was taken from.

def fd_step(f, phi, A, B, kappa, gamma, tau_f, tau_g, coupling="stress"):
    grad, lap = gradients(phi)
    mu, pi = chemical(phi, grad, lap, A, B, kappa)
    rho = f.sum(0)
    j = torch.einsum("ia,ixyz->axyz", CF, f)
    if coupling == "force":
        fs, _, u = _collide_f_force(f, rho, j, body_force(pi), phi, mu, gamma, tau_f)
    else:
        feq, _ = equilibria(rho, j, phi, mu, pi, gamma)
        fs = f - (f - feq) / tau_f
        u = j / rho[None]
    M = gamma * (tau_g - 0.5)
    div = torch.zeros_like(phi)
    for a in range(3):
        uf = 0.5 * (u[a] + _shift(u[a], a, 1))
        flux = uf * torch.where(uf > 0, phi, _shift(phi, a, 1)) - M * (_shift(mu, a, 1) - mu)
        div = div + (flux - _shift(flux, a, -1))
    return propagate(fs), phi - div


def fd_rollout_phi(phi0, A, B, kappa, nsteps, gamma=0.5, tau_f=1.0, tau_g=1.0, rho0=1.0,
                   coupling="stress"):
    """phi after nsteps of the finite-difference scheme from rest; differentiable."""
    f = WEIGHTS[:, None, None, None] * rho0 * torch.ones((19,) + tuple(phi0.shape),
                                                          dtype=torch.float64)
    phi = phi0
    for _ in range(nsteps):
        f, phi = fd_step(f, phi, A, B, kappa, gamma, tau_f, tau_g, coupling)
    return phi


def fd_loss_and_grads(phi0, target, A, B, kappa, nsteps, gamma=0.5, tau_f=1.0, tau_g=1.0,
                      rho0=1.0, coupling="stress"):
    """As loss_and_grads, for the finite-difference order parameter."""
    p0 = torch.as_tensor(phi0, dtype=torch.float64).clone().requires_grad_(True)
    tA = torch.tensor(float(A), dtype=torch.float64, requires_grad=True)
    tB = torch.tensor(float(B), dtype=torch.float64, requires_grad=True)
    tk = torch.tensor(float(kappa), dtype=torch.float64, requires_grad=True)
    phiT = fd_rollout_phi(p0, tA, tB, tk, nsteps, gamma, tau_f, tau_g, rho0, coupling)
    tgt = torch.as_tensor(target, dtype=torch.float64)
    loss = 0.5 * ((phiT - tgt) ** 2).sum()
    loss.backward()
    return (float(loss.detach()), p0.grad.numpy().copy(), float(tA.grad), float(tB.grad),
            float(tk.grad))
