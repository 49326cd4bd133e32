"""Reverse mode of the finite-difference order-parameter scheme (either
coupling) on the GPU, against autograd through the oracle's torch
transcription of the step (pinned to the C oracle and to central
differences in the CPU suite): dL/dphi0, dL/d(A, B, kappa) and, from an
imported flowing state, dL/df0 of the pulled populations."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import lbinputs
import oracle
import oracle.reverse as R
from tests._gpu import make_lb, rel_err

pytestmark = pytest.mark.gpu


COUPLINGS = ["stress", "force"]


def _rollout_grads(shape, T, phi0, tgt, interval=None, precision="fp64", coupling="stress",
                   **kw):
    from paper_1609_01479_amd.rollout import rollout
    pr = dict(lbinputs.SPINODAL_PARAMS, **kw)
    dev = torch.device("cuda:0")
    p0 = torch.tensor(phi0, dtype=torch.float64, device=dev, requires_grad=True)
    th = [torch.tensor(pr[k], dtype=torch.float64, device=dev, requires_grad=True)
          for k in ("A", "B", "kappa")]
    phiT = rollout(p0, *th, T, interval=interval, gamma=pr["gamma"], tau_f=pr["tau_f"],
                   tau_g=pr["tau_g"], rho0=pr["rho0"], precision=precision, order_param="fd",
                   coupling=coupling)
    loss = 0.5 * ((phiT - torch.tensor(tgt, device=dev)) ** 2).sum()
    loss.backward()
    return (float(loss.detach()), p0.grad.cpu().numpy()) + tuple(float(t.grad) for t in th)


def _check(got, ref, tol_phi=1e-10, tol_theta=1e-9):
    L, gphi, *gth = got
    rL, rphi, *rth = ref
    assert abs(L - rL) <= 1e-12 * abs(rL), (L, rL)
    assert rel_err(gphi, rphi) <= tol_phi, rel_err(gphi, rphi)
    for name, a, b in zip(("A", "B", "kappa"), gth, rth):
        assert abs(a - b) <= tol_theta * abs(b), (name, a, b)


@pytest.mark.parametrize("coupling", COUPLINGS)
@pytest.mark.parametrize("interval", [None, 1, 7])
def test_fd_adjoint_matches_oracle_reverse_mode_8cubed(interval, coupling):
    """8^3 x 20 steps from rest, tau != 1, through the checkpointed rollout."""
    shape, T = (8, 8, 8), 20
    kw = dict(tau_f=0.8, tau_g=1.3)
    pr = dict(lbinputs.SPINODAL_PARAMS, **kw)
    phi0 = lbinputs.spinodal_phi0(shape, seed=77)
    tgt = lbinputs.lamellar_target(shape, 8, lbinputs.interface_width(pr["A"], pr["kappa"]))
    print(f"[fd adjoint] 8^3 x {T} interval={interval} {coupling}", flush=True)
    got = _rollout_grads(shape, T, phi0, tgt, interval=interval, coupling=coupling, **kw)
    ref = R.fd_loss_and_grads(phi0, tgt, pr["A"], pr["B"], pr["kappa"], T, pr["gamma"],
                              pr["tau_f"], pr["tau_g"], pr["rho0"], coupling)
    _check(got, ref)


@pytest.mark.parametrize("coupling", COUPLINGS)
def test_fd_adjoint_noncubic_default_taus(coupling):
    shape, T = (6, 5, 7), 12
    pr = dict(lbinputs.SPINODAL_PARAMS)
    phi0 = lbinputs.spinodal_phi0(shape, seed=3, amp=0.4)
    tgt = lbinputs.random_field(shape, 10)
    print(f"[fd adjoint] {shape} x {T} {coupling}", flush=True)
    got = _rollout_grads(shape, T, phi0, tgt, interval=4, coupling=coupling)
    ref = R.fd_loss_and_grads(phi0, tgt, pr["A"], pr["B"], pr["kappa"], T, pr["gamma"],
                              pr["tau_f"], pr["tau_g"], pr["rho0"], coupling)
    _check(got, ref)


def _flowing_f0(shape, seed):
    """Second-order equilibrium of a sheared, sign-changing velocity field,
    perturbed by 1% seeded noise: every face sees both upwind branches."""
    c, w = oracle.lattice()
    nx, ny, nz = shape
    x, y, z = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    u = np.stack([0.03 * np.sin(2 * np.pi * (y + 0.5) / ny),
                  0.02 * np.cos(2 * np.pi * (z + 0.25) / nz),
                  0.015 * np.sin(2 * np.pi * (x + 0.3) / nx)])
    cu = np.einsum("ia,axyz->ixyz", c, u)
    uu = (u * u).sum(0)
    f0 = w[:, None, None, None] * (1.0 + 3 * cu + 4.5 * cu * cu - 1.5 * uu[None])
    return f0 * (1.0 + 0.01 * lbinputs.random_field((19,) + tuple(shape), seed))


def _reference_from_state(f0, phi0, tgt, T, pr, coupling="stress"):
    f = torch.tensor(f0, dtype=torch.float64, requires_grad=True)
    p0 = torch.tensor(phi0, dtype=torch.float64, requires_grad=True)
    th = [torch.tensor(float(pr[k]), dtype=torch.float64, requires_grad=True)
          for k in ("A", "B", "kappa")]
    fs, ph = f, p0
    for _ in range(T):
        fs, ph = R.fd_step(fs, ph, *th, pr["gamma"], pr["tau_f"], pr["tau_g"], coupling)
    loss = 0.5 * ((ph - torch.tensor(tgt, dtype=torch.float64)) ** 2).sum()
    loss.backward()
    return ((float(loss.detach()), p0.grad.numpy()) + tuple(float(t.grad) for t in th),
            f.grad.numpy())


def _gpu_from_state(f0, phi0, tgt, T, precision="fp64", coupling="stress", **kw):
    shape = phi0.shape
    lb = make_lb(shape, precision=precision, adjoint=True, order_param="fd", coupling=coupling,
                 **kw)
    lb.init_phi(phi0)
    lb.import_dist(f0)
    states = []
    for _ in range(T):
        states.append(lb.get_state())
        lb.step(1)
    phiT = lb.phi()
    dphi = phiT - torch.tensor(tgt, device=phiT.device)
    L = 0.5 * float((dphi ** 2).sum())
    lb.adjoint_seed(dphi)
    dth = torch.zeros(3, dtype=torch.float64, device=phiT.device)
    for t in reversed(range(T)):
        lb.adjoint_step(states[t], dth)
    gphi = lb.adjoint_phi0().cpu().numpy()
    lf, lg = lb.adjoint_dist()
    assert lg is None
    return (L, gphi) + tuple(float(v) for v in dth.cpu()), lf.cpu().numpy()


@pytest.mark.parametrize("coupling", COUPLINGS)
@pytest.mark.parametrize("shape", [(6, 5, 7), (2, 3, 1), (1, 4, 9)])
def test_fd_adjoint_flowing_state_including_df0(shape, coupling):
    """From an imported flow with mixed signs (upwind branches both ways) and
    non-equilibrium populations, tau != 1: dL/df0 (the adjoint level's
    lambda_f), dL/dphi0 and dL/d(A, B, kappa)."""
    T = 10
    kw = dict(tau_f=0.9, tau_g=1.2)
    pr = dict(lbinputs.SPINODAL_PARAMS, **kw)
    phi0 = lbinputs.spinodal_phi0(shape, seed=41, amp=0.5)
    tgt = lbinputs.random_field(shape, 42)
    f0 = _flowing_f0(shape, 43)
    print(f"[fd adjoint flow] {shape} x {T} {coupling}", flush=True)
    got, lf = _gpu_from_state(f0, phi0, tgt, T, coupling=coupling, **kw)
    ref, rlf = _reference_from_state(f0, phi0, tgt, T, pr, coupling)
    _check(got, ref)
    assert rel_err(lf, rlf) <= 1e-10, rel_err(lf, rlf)


@pytest.mark.parametrize("coupling", COUPLINGS)
def test_fd_adjoint_fp32_close_to_fp64(coupling):
    shape, T = (16, 16, 16), 40
    pr = dict(lbinputs.SPINODAL_PARAMS)
    phi0 = lbinputs.spinodal_phi0(shape, seed=12)
    tgt = lbinputs.lamellar_target(shape, 8, lbinputs.interface_width(pr["A"], pr["kappa"]))
    g64 = _rollout_grads(shape, T, phi0, tgt, precision="fp64", coupling=coupling)
    g32 = _rollout_grads(shape, T, phi0, tgt, precision="fp32_dev", coupling=coupling)
    e_phi = np.linalg.norm(g32[1] - g64[1]) / np.linalg.norm(g64[1])
    print(f"[fd adjoint fp32 {coupling}] rel L2 err dphi0 = {e_phi:.3e}; "
          f"A {g32[2]/g64[2]-1:.2e} B {g32[3]/g64[3]-1:.2e} kappa {g32[4]/g64[4]-1:.2e}",
          flush=True)
    assert e_phi <= 1e-4
    for a, b in zip(g32[2:], g64[2:]):
        assert abs(a - b) <= 1e-3 * abs(b)


@pytest.mark.parametrize("coupling", COUPLINGS)
def test_fd_adjoint_fp32_flowing_state(coupling):
    """FP32 storage from an imported flow: every gradient within FP32 rounding
    of the FP64 reference."""
    shape, T = (6, 5, 7), 10
    kw = dict(tau_f=0.9, tau_g=1.2)
    pr = dict(lbinputs.SPINODAL_PARAMS, **kw)
    phi0 = lbinputs.spinodal_phi0(shape, seed=41, amp=0.5)
    tgt = lbinputs.random_field(shape, 42)
    f0 = _flowing_f0(shape, 43)
    got, lf = _gpu_from_state(f0, phi0, tgt, T, precision="fp32_dev", coupling=coupling, **kw)
    ref, rlf = _reference_from_state(f0, phi0, tgt, T, pr, coupling)
    assert rel_err(got[1], ref[1]) <= 1e-5, rel_err(got[1], ref[1])
    assert rel_err(lf, rlf) <= 1e-5, rel_err(lf, rlf)
    for a, b in zip(got[2:], ref[2:]):
        assert abs(a - b) <= 1e-4 * abs(b), (a, b)


@pytest.mark.parametrize("coupling", COUPLINGS)
@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
@pytest.mark.parametrize("layout,v", [("soa", 0), ("aos", 0), ("aosoa", 32)])
def test_fd_adjoint_layouts_bit_identical(precision, layout, v, coupling):
    """The adjoint reads the saved levels through the context's layout: dL/dphi0
    and dL/d(A, B, kappa) are bit-identical to the row-blocked default's."""
    shape, T = (6, 5, 64), 4
    phi0 = lbinputs.spinodal_phi0(shape, seed=23, amp=0.3)
    f0 = _flowing_f0(shape, 24)
    dphi = torch.tensor(lbinputs.random_field(shape, 4), device="cuda:0")
    out = []
    for lay, vv in (("rows", 0), (layout, v)):
        lb = make_lb(shape, precision=precision, adjoint=True, order_param="fd", layout=lay,
                     aosoa_len=vv, coupling=coupling)
        lb.init_phi(phi0)
        lb.import_dist(f0)
        states = [lb.get_state()]
        for _ in range(T):
            lb.step(1)
            states.append(lb.get_state())
        dth = torch.zeros(3, dtype=torch.float64, device="cuda:0")
        lb.adjoint_seed(dphi)
        for t in reversed(range(T)):
            lb.adjoint_step(states[t], dth)
        out.append((lb.adjoint_phi0().cpu().numpy(), dth.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
