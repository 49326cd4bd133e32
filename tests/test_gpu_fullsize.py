"""Parity at the benchmark sizes, in the launch configuration bench.py times.

The oracle cannot step a 256^3 lattice in a test, but one step at a site x
depends only on the state within L-infinity distance 2 of x (x's populations
are pulled from distance 1, whose collision uses phi's stencil at distance 2,
and phi is local in g).  So for sampled sites the oracle steps a 7^3 periodic
window cut around x from the GPU's exported state; the window's centre is
then exactly the oracle's step of the full lattice at x, compared with the
GPU's step there.  Properties that hold at any size (conservation, the
adjoint's directional derivative) are checked on the whole lattice.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import lbinputs
import oracle
from tests._gpu import make_lb, oracle_params

pytestmark = pytest.mark.gpu

R = 3  # window radius


def _sample_sites(shape, n, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    fixed = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (0, ny - 1, 63), (nx // 2, ny // 2, nz // 2),
             (nx - 1, 0, 64), (3, 4, nz - 1), (nx // 2 + 64 % nx, 3, 0)]
    fixed = [(x % nx, y % ny, z % nz) for x, y, z in fixed]
    rand = [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz))) for _ in range(n)]
    return fixed + rand


def _window(t, site, shape):
    """(19, 7, 7, 7) periodic window of a (19, nx, ny, nz) device tensor."""
    idx = [torch.tensor([(c + d) % n for d in range(-R, R + 1)], device=t.device)
           for c, n in zip(site, shape)]
    w = t.index_select(1, idx[0]).index_select(2, idx[1]).index_select(3, idx[2])
    return w.cpu().numpy()


def _sampled_parity(shape, precision, phi0, steps_before, kw, tol, nsample=24, lb_kw=None,
                    oracle_kw=None):
    print(f"[fullsize] {shape} {precision} after {steps_before} steps, {nsample} sites "
          f"{lb_kw or ''}", flush=True)
    lb = make_lb(shape, precision=precision, **kw, **(lb_kw or {}))
    lb.init_phi(phi0)
    lb.step(steps_before)
    f, g = lb.export_dist()
    sites = _sample_sites(shape, nsample, 7)
    wins = [(_window(f, s, shape), _window(g, s, shape)) for s in sites]
    del f, g
    torch.cuda.empty_cache()
    lb.step(1)
    f1, g1 = lb.export_dist()
    got = [(f1[:, x, y, z].cpu().numpy(), g1[:, x, y, z].cpu().numpy()) for x, y, z in sites]
    del f1, g1
    torch.cuda.empty_cache()
    pw = oracle_params((2 * R + 1,) * 3, **kw, **(oracle_kw or {}))
    fscale = gscale = 0.0
    ferr = gerr = 0.0
    for (fw, gw), (fg, gg) in zip(wins, got):
        fo, go = oracle.step(pw, fw, gw)
        ref_f, ref_g = fo[:, R, R, R], go[:, R, R, R]
        ferr = max(ferr, float(np.abs(fg - ref_f).max()))
        gerr = max(gerr, float(np.abs(gg - ref_g).max()))
        fscale = max(fscale, float(np.abs(ref_f).max()))
        gscale = max(gscale, float(np.abs(ref_g).max()))
    print(f"[fullsize] rel err f {ferr / fscale:.3e}  g {gerr / gscale:.3e}", flush=True)
    assert ferr <= tol * fscale and gerr <= tol * gscale


def _droplet(n):
    pr = lbinputs.SPINODAL_PARAMS
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    return lbinputs.droplet_phi0((n, n, n), n / 4, xi, noise=1e-3, seed=lbinputs.SEED_DROPLET)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_dev", 2e-6)])
def test_sampled_parity_droplet_256(precision, tol):
    """256^3 droplet (the benchmark lattice), both precisions; tau != 1 so the
    non-equilibrium part is exercised at full size as well."""
    _sampled_parity((256, 256, 256), precision, _droplet(256), 5, dict(tau_f=0.8, tau_g=1.3), tol)


@pytest.mark.parametrize("precision,shape,tol", [("fp64", (320, 320, 320), 1e-12),
                                                 ("fp32_dev", (400, 384, 384), 2e-6)])
def test_sampled_parity_large_regions(precision, shape, tol):
    """Lattices whose f or g region exceeds 4 GiB: the single-pass kernel
    addresses planes with 64-bit offsets (one pointer per component) instead
    of 32-bit ones.  (400, 384, 384) in FP32 also runs the pipelined march on
    full tiles."""
    pr = lbinputs.SPINODAL_PARAMS
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    phi0 = lbinputs.droplet_phi0(shape, min(shape) / 4, xi, noise=1e-3, seed=lbinputs.SEED_DROPLET)
    _sampled_parity(shape, precision, phi0, 2, dict(tau_f=0.8, tau_g=1.3), tol, nsample=12)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_dev", 2e-6)])
def test_sampled_parity_maximum_size(precision, tol):
    """479^3, the largest cube the library accepts (39 * stride just under
    2^32 elements: every 32-bit element index near its limit), ragged in every
    tile dimension; 480^3 is rejected."""
    from paper_1609_01479_amd import LB
    from paper_1609_01479_amd._abi import LbError
    with pytest.raises(LbError):
        LB((480, 480, 480), precision=precision, device="cuda:0")
    shape = (479, 479, 479)
    pr = lbinputs.SPINODAL_PARAMS
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    phi0 = lbinputs.droplet_phi0(shape, 100.0, xi, noise=1e-3, seed=lbinputs.SEED_DROPLET)
    _sampled_parity(shape, precision, phi0, 1, dict(tau_f=0.8, tau_g=1.3), tol, nsample=10)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_dev", 2e-6)])
def test_sampled_parity_force_coupling_droplet_256(precision, tol):
    """The force coupling at the benchmark lattice: one step at x depends on
    phi within distance 2 (the force's Pi at the face neighbours), i.e. on g
    within distance 3, which the 7^3 window still holds."""
    _sampled_parity((256, 256, 256), precision, _droplet(256), 5, dict(tau_f=0.8, tau_g=1.3), tol,
                    lb_kw=dict(coupling="force"), oracle_kw=dict(coupling=1))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_dev", 2e-6)])
def test_sampled_parity_force_coupling_maximum_size(precision, tol):
    """The force coupling at 479^3, the largest accepted cube, ragged in every
    tile dimension of the marching collision pass."""
    shape = (479, 479, 479)
    pr = lbinputs.SPINODAL_PARAMS
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    phi0 = lbinputs.droplet_phi0(shape, 100.0, xi, noise=1e-3, seed=lbinputs.SEED_DROPLET)
    _sampled_parity(shape, precision, phi0, 1, dict(tau_f=0.8, tau_g=1.3), tol, nsample=8,
                    lb_kw=dict(coupling="force"), oracle_kw=dict(coupling=1))


def test_sampled_parity_spinodal_128_fp64():
    shape = (128, 128, 128)
    _sampled_parity(shape, "fp64", lbinputs.spinodal_phi0(shape), 20, {}, 1e-12)


@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
def test_conservation_droplet_256(precision):
    lb = make_lb((256, 256, 256), precision=precision)
    lb.init_phi(_droplet(256))
    s0 = lb.sums().cpu().numpy()
    lb.step(100)
    s1 = lb.sums().cpu().numpy()
    n = 256 ** 3
    # FP64: round-off; FP32: storage rounding of deviations (relative 1e-7)
    tol = 1e-9 * n if precision == "fp64" else 2e-7 * n
    assert np.abs(s1 - s0).max() <= tol, (s1 - s0)


def test_adjoint_directional_derivative_64cubed():
    """The 64^3, 200-step adjoint with checkpoint interval 15: <dL/dphi0, v>
    and dL/dkappa against central differences of the GPU forward."""
    from paper_1609_01479_amd.rollout import rollout
    shape = (64, 64, 64)
    T = 200
    pr = dict(lbinputs.SPINODAL_PARAMS)
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    phi0 = lbinputs.spinodal_phi0(shape)
    tgt = torch.tensor(lbinputs.lamellar_target(shape, 32, xi), device="cuda:0")
    dev = torch.device("cuda:0")
    rest = {k: pr[k] for k in ("gamma", "tau_f", "tau_g", "rho0")}

    def loss(p0, kappa):
        lb = make_lb(shape, kappa=kappa)
        lb.init_phi(p0)
        lb.step(T)
        return float(0.5 * ((lb.phi() - tgt) ** 2).sum())

    p0 = torch.tensor(phi0, dtype=torch.float64, device=dev, requires_grad=True)
    th = [torch.tensor(pr[k], dtype=torch.float64, device=dev, requires_grad=True)
          for k in ("A", "B", "kappa")]
    phiT = rollout(p0, *th, T, interval=15, **rest)
    L = 0.5 * ((phiT - tgt) ** 2).sum()
    L.backward()
    assert abs(float(L) - loss(phi0, pr["kappa"])) <= 1e-12 * abs(float(L))
    v = lbinputs.random_field(shape, 3)
    h = 1e-4
    fd = (loss(phi0 + h * v, pr["kappa"]) - loss(phi0 - h * v, pr["kappa"])) / (2 * h)
    ad = float((p0.grad.cpu().numpy() * v).sum())
    print(f"[adjoint 64^3] <grad, v>: adjoint {ad:.12e} fd {fd:.12e}", flush=True)
    assert abs(ad - fd) <= 1e-6 * abs(fd)
    hk = 1e-4 * pr["kappa"]
    fdk = (loss(phi0, pr["kappa"] + hk) - loss(phi0, pr["kappa"] - hk)) / (2 * hk)
    print(f"[adjoint 64^3] dL/dkappa: adjoint {float(th[2].grad):.12e} fd {fdk:.12e}", flush=True)
    assert abs(float(th[2].grad) - fdk) <= 1e-6 * abs(fdk)


@pytest.mark.parametrize("order_param,coupling", [("lb", "stress"), ("lb", "force"),
                                                   ("fd", "stress"), ("fd", "force")])
def test_adjoint_directional_derivative_256cubed(order_param, coupling):
    """The adjoint at the benchmark's 256^3 droplet, where the persistent
    kernels sweep each XCD's eighth of the lattice in 64 rounds: a 3-step
    FP64 rollout (checkpoint every 2 steps), <dL/dphi0, v> and dL/dA against
    central differences of the GPU forward.  The LB step is smooth (h = 1e-4,
    difference exact to O(h^2)); the finite-difference step has kinks where a
    face velocity changes sign, so its phi0 direction takes h = 1e-6, which
    flips few faces, and a tolerance of 1e-5 for the round-off of L/h (the
    step in A, 1e-4 |A|, moves face velocities by far less)."""
    from paper_1609_01479_amd.rollout import rollout
    shape = (256, 256, 256)
    T = 3
    pr = dict(lbinputs.SPINODAL_PARAMS)
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    phi0 = lbinputs.droplet_phi0(shape, 64.0, xi)
    dev = torch.device("cuda:0")
    tgt = torch.tensor(lbinputs.lamellar_target(shape, 32, xi), device=dev)
    rest = {k: pr[k] for k in ("gamma", "tau_f", "tau_g", "rho0")}
    fd_scheme = order_param == "fd"
    h, tol = (1e-6, 1e-5) if fd_scheme else (1e-4, 1e-6)
    print(f"[adjoint 256^3] {order_param} {coupling} x {T}", flush=True)

    def loss(p0, A):
        lb = make_lb(shape, A=A, coupling=coupling, order_param=order_param)
        lb.init_phi(p0)
        lb.step(T)
        out = float(0.5 * ((lb.phi() - tgt) ** 2).sum())
        del lb
        torch.cuda.empty_cache()
        return out

    p0 = torch.tensor(phi0, dtype=torch.float64, device=dev, requires_grad=True)
    th = [torch.tensor(pr[k], dtype=torch.float64, device=dev, requires_grad=True)
          for k in ("A", "B", "kappa")]
    phiT = rollout(p0, *th, T, interval=2, coupling=coupling, order_param=order_param, **rest)
    L = 0.5 * ((phiT - tgt) ** 2).sum()
    L.backward()
    gphi = p0.grad.cpu().numpy()
    gA = float(th[0].grad)
    del phiT, L, p0
    torch.cuda.empty_cache()
    v = lbinputs.random_field(shape, 3)
    fd = (loss(phi0 + h * v, pr["A"]) - loss(phi0 - h * v, pr["A"])) / (2 * h)
    ad = float((gphi * v).sum())
    print(f"[adjoint 256^3] {order_param} {coupling} <grad, v>: adjoint {ad:.12e} fd {fd:.12e}",
          flush=True)
    assert abs(ad - fd) <= tol * abs(fd)
    hA = 1e-4 * abs(pr["A"])
    fdA = (loss(phi0, pr["A"] + hA) - loss(phi0, pr["A"] - hA)) / (2 * hA)
    print(f"[adjoint 256^3] {order_param} {coupling} dL/dA: adjoint {gA:.12e} fd {fdA:.12e}",
          flush=True)
    assert abs(gA - fdA) <= tol * abs(fdA)
