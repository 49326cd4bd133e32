"""Parity of the finite-difference order parameter (a phi field with a
conservative Cahn-Hilliard update and upwind advection; no g) between the HIP
path (through the C ABI) and the CPU oracle.

Bar (FP64): for every output field F (f, rho, u, phi),
max_x |F_gpu - F_oracle| / max_x |F_oracle| <= 1e-12 (u on scale 1).  FP32
storage of f: phi stays FP64, so it follows the FP64 oracle to 1e-6 over 20
steps (rho 1e-6, u 1e-7), and the 40^3 droplet to 1e-5 over 300 steps.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import lbinputs
import oracle
from tests._gpu import field_errors, make_lb, oracle_params

pytestmark = pytest.mark.gpu

TOL = 1e-12
NAMES = ("f", "rho", "u", "phi")


def _gpu(lb):
    f, g = lb.export_dist()
    assert g is None
    rho, u, phi = lb.moments()
    torch.cuda.synchronize()
    return tuple(t.cpu().numpy() for t in (f, rho, u, phi))


def _ref(p, f, phi):
    rho, u, ph = oracle.fd_moments(p, f, phi)
    return f, rho, u, ph


def _run_both(shape, steps, phi0, precision="fp64", coupling="stress", **kw):
    print(f"[fd] shape={shape} steps={steps} precision={precision} coupling={coupling} "
          f"params={kw}", flush=True)
    lb = make_lb(shape, precision=precision, order_param="fd", coupling=coupling, **kw)
    lb.init_phi(phi0)
    lb.step(steps)
    got = _gpu(lb)
    p = oracle_params(shape, order_param=1, coupling={"stress": 0, "force": 1}[coupling], **kw)
    ref = _ref(p, *oracle.fd_run(p, *oracle.fd_init(p, phi0), steps))
    return got, ref, lb, p


@pytest.mark.parametrize("steps", [0, 1, 10, 100])
def test_fd_spinodal_16cubed(steps):
    shape = (16, 16, 16)
    got, ref, *_ = _run_both(shape, steps, lbinputs.spinodal_phi0(shape))
    errs = field_errors(got, ref, NAMES)
    assert max(errs.values()) <= TOL, errs


@pytest.mark.parametrize("shape", [(5, 6, 7), (3, 5, 131), (17, 9, 70), (1, 7, 1), (2, 2, 2)])
def test_fd_noncubic_ragged_degenerate_tau_not_one(shape):
    phi0 = lbinputs.spinodal_phi0(shape, seed=12, amp=0.4)
    got, ref, *_ = _run_both(shape, 25, phi0, tau_f=0.8, tau_g=1.3)
    errs = field_errors(got, ref, NAMES)
    assert max(errs.values()) <= TOL, errs


def test_fd_droplet_interface_and_sums():
    """A sharp tanh droplet (large mu and Pi at the interface), 50 steps; the
    conserved sums of the final state."""
    shape = (24, 20, 22)
    pr = lbinputs.SPINODAL_PARAMS
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    phi0 = lbinputs.droplet_phi0(shape, 6.0, xi, noise=1e-3, seed=3)
    got, ref, lb, p = _run_both(shape, 50, phi0)
    errs = field_errors(got, ref, NAMES)
    assert max(errs.values()) <= TOL, errs
    want = oracle.fd_sums(p, *oracle.fd_run(p, *oracle.fd_init(p, phi0), 50))
    np.testing.assert_allclose(lb.sums().cpu().numpy(), want, rtol=1e-12, atol=1e-12)


def test_fd_flow_advects_phi():
    """A uniform flow imported as f = w (rho + 3 c.j): the upwind advection
    moves phi exactly as the oracle's (mixed-sign velocity, M = 0 and no
    free energy, so advection is all that acts on phi)."""
    shape = (12, 10, 14)
    kw = dict(A=0.0, B=0.0, kappa=0.0, gamma=0.0)
    c, w = oracle.lattice()
    j = np.array([0.031, -0.022, 0.013])
    f0 = np.broadcast_to((w * (1.0 + 3 * (c @ j)))[:, None, None, None], (19,) + shape).copy()
    phi0 = lbinputs.random_field(shape, seed=21)
    lb = make_lb(shape, order_param="fd", **kw)
    lb.init_phi(phi0)
    lb.import_dist(f0)
    lb.step(20)
    got = _gpu(lb)
    p = oracle_params(shape, order_param=1, **kw)
    ref = _ref(p, *oracle.fd_run(p, f0, phi0, 20))
    errs = field_errors(got, ref, NAMES)
    assert max(errs.values()) <= TOL, errs
    assert np.abs(got[3] - phi0).max() > 0.1  # phi moved


@pytest.mark.parametrize("coupling", ["stress", "force"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
@pytest.mark.parametrize("shape,seg", [((16, 16, 16), 0), ((16, 16, 16), 5), ((5, 6, 7), 2),
                                       ((3, 5, 131), 0), ((17, 9, 70), 4), ((1, 7, 1), 0),
                                       ((2, 2, 2), 1), ((6, 13, 200), 3), ((9, 6, 131), 9),
                                       ((24, 20, 192), 0)])
def test_fd_single_pass_matches_two_pass(precision, shape, seg, coupling):
    """The marching kernels (stress: collision one plane ahead of the flux
    update, face ring in LDS; force: Pi staged in LDS, the force, mu and u
    also on the face ring, collision two planes ahead of the flux update)
    and the one-site-per-thread kernels give bit-identical levels: ragged
    tiles in y and z, 4 x 128 and 8 x 64 tiles, one-plane and long x
    segments, extents 1 and 2."""
    print(f"[fd fused] {shape} segment_x={seg} {precision} {coupling}", flush=True)
    phi0 = lbinputs.spinodal_phi0(shape, seed=17, amp=0.4)
    out = []
    for kern in ("fused", "two_pass"):
        lb = make_lb(shape, precision=precision, order_param="fd", kernel=kern, segment_x=seg,
                     coupling=coupling, tau_f=0.8, tau_g=1.3)
        lb.init_phi(phi0)
        lb.step(7)
        out.append(_gpu(lb))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("coupling", ["stress", "force"])
@pytest.mark.parametrize("layout,v", [("soa", 0), ("aos", 0), ("aosoa", 8)])
def test_fd_layouts_bit_identical(layout, v, coupling):
    shape = (6, 7, 16)
    phi0 = lbinputs.spinodal_phi0(shape, seed=8, amp=0.3)
    out = []
    for lay, vv in (("rows", 0), (layout, v)):
        lb = make_lb(shape, order_param="fd", layout=lay, aosoa_len=vv, tau_f=0.9,
                     coupling=coupling)
        lb.init_phi(phi0)
        lb.step(9)
        out.append(_gpu(lb))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_fd_step_sums_step_from_and_determinism():
    """Per-step FP64 sums are conserved (mass, phi; momentum to round-off) and
    match the oracle's; lb_step_from gives the same level as lb_step; two runs
    from one checkpoint agree bit for bit."""
    shape = (12, 10, 14)
    phi0 = 0.1 + lbinputs.spinodal_phi0(shape, seed=2, amp=0.3)
    lb = make_lb(shape, order_param="fd", tau_f=0.8, tau_g=1.1)
    lb.init_phi(phi0)
    hist = lb.step_sums(30).cpu().numpy()
    assert np.abs(hist[:, :2] - hist[0, :2]).max() <= 1e-11
    assert np.abs(hist[:, 2:] - hist[0, 2:]).max() <= 1e-12
    p = oracle_params(shape, order_param=1, tau_f=0.8, tau_g=1.1)
    f, phi = oracle.fd_run(p, *oracle.fd_init(p, phi0), 29)
    np.testing.assert_allclose(hist[29], oracle.fd_sums(p, f, phi), rtol=1e-12, atol=1e-12)
    ck = lb.get_state()
    lb.step(7)
    a = _gpu(lb)
    lb.set_state(ck)
    lb.step(7)
    b = _gpu(lb)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    lb.set_state(ck)
    lb.step(1)
    a = _gpu(lb)
    nxt = lb.new_state()
    lb.step_from(ck, nxt)
    lb.set_state(nxt)
    b = _gpu(lb)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("shape", [(16, 16, 16), (9, 6, 131)])
def test_fd_fp32_storage(shape):
    """FP32 deviation storage of f (phi FP64) follows the FP64 oracle to FP32
    rounding over 20 steps (tau != 1)."""
    phi0 = lbinputs.spinodal_phi0(shape, seed=14, amp=0.3)
    got, ref, *_ = _run_both(shape, 20, phi0, precision="fp32_dev", tau_f=0.8, tau_g=1.3)
    f, rho, u, phi = got
    rf, rrho, ru, rphi = ref
    assert np.abs(phi - rphi).max() <= 1e-6
    assert np.abs(rho - rrho).max() <= 1e-6
    assert np.abs(u - ru).max() <= 1e-7


def test_fd_fp32_droplet_phi_error_vs_fp64():
    """A droplet over 300 steps: max |phi32 - phi64| <= 1e-5."""
    shape = (40, 40, 40)
    pr = lbinputs.SPINODAL_PARAMS
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    phi0 = lbinputs.droplet_phi0(shape, 10.0, xi, noise=1e-3, seed=4)
    out = {}
    for prec in ("fp64", "fp32_dev"):
        lb = make_lb(shape, precision=prec, order_param="fd")
        lb.init_phi(phi0)
        lb.step(300)
        out[prec] = lb.phi().cpu().numpy()
    err = np.abs(out["fp32_dev"] - out["fp64"]).max()
    print(f"[fd] fp32 vs fp64 phi error after 300 steps: {err:.3e}", flush=True)
    assert err <= 1e-5


# ---- full sizes: sampled sites --------------------------------------------
# One step at x depends only on the state within L-infinity distance 2 of x
# (phi(t+1) uses mu and u at the face neighbours; mu needs phi's stencil
# there and u the populations pulled from one site further), so the oracle
# steps a 7^3 periodic window cut around each sampled site from the GPU's
# state, and the window's centre is compared with the GPU's step at x.

R = 3


def _win(t, site, shape):
    idx = [torch.tensor([(c + d) % n for d in range(-R, R + 1)], device=t.device)
           for c, n in zip(site, shape)]
    off = t.dim() - 3
    w = t.index_select(off, idx[0]).index_select(off + 1, idx[1]).index_select(off + 2, idx[2])
    return w.cpu().numpy()


def _sampled_fd(shape, precision, phi0, steps_before, kw, tol, nsample=16, coupling="stress"):
    print(f"[fd fullsize] {shape} {precision} {coupling} after {steps_before} steps, "
          f"{nsample} sites", flush=True)
    rng = np.random.default_rng(9)
    nx, ny, nz = shape
    sites = [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx // 2, ny // 2, nz // 2), (1, ny - 1, 64 % nz)]
    sites += [(int(rng.integers(nx)), int(rng.integers(ny)), int(rng.integers(nz)))
              for _ in range(nsample)]
    lb = make_lb(shape, precision=precision, order_param="fd", coupling=coupling, **kw)
    lb.init_phi(phi0)
    lb.step(steps_before)
    f, _ = lb.export_dist()
    phi = lb.phi()
    wins = [(_win(f, s, shape), _win(phi, s, shape)) for s in sites]
    del f, phi
    torch.cuda.empty_cache()
    lb.step(1)
    f1, _ = lb.export_dist()
    phi1 = lb.phi()
    got = [(f1[:, x, y, z].cpu().numpy(), float(phi1[x, y, z])) for x, y, z in sites]
    del f1, phi1, lb
    torch.cuda.empty_cache()
    pw = oracle_params((2 * R + 1,) * 3, order_param=1,
                       coupling={"stress": 0, "force": 1}[coupling], **kw)
    ferr = perr = fscale = pscale = 0.0
    for (fw, pw_phi), (fg, pg) in zip(wins, got):
        fo, po = oracle.fd_step(pw, fw, pw_phi)
        ferr = max(ferr, float(np.abs(fg - fo[:, R, R, R]).max()))
        perr = max(perr, abs(pg - float(po[R, R, R])))
        fscale = max(fscale, float(np.abs(fo[:, R, R, R]).max()))
        pscale = max(pscale, abs(float(po[R, R, R])))
    print(f"[fd fullsize] rel err f {ferr / fscale:.3e}  phi {perr / pscale:.3e}", flush=True)
    assert ferr <= tol * fscale and perr <= tol * pscale


def _droplet(shape):
    pr = lbinputs.SPINODAL_PARAMS
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    return lbinputs.droplet_phi0(shape, min(shape) / 4, xi, noise=1e-3, seed=lbinputs.SEED_DROPLET)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_dev", 2e-6)])
def test_fd_sampled_parity_droplet_256(precision, tol):
    """The benchmark lattice (256^3 droplet), both precisions, tau != 1."""
    shape = (256, 256, 256)
    _sampled_fd(shape, precision, _droplet(shape), 5, dict(tau_f=0.8, tau_g=1.3), tol)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_dev", 2e-6)])
def test_fd_sampled_parity_maximum_size(precision, tol):
    """479^3, the largest cube the library accepts, ragged everywhere."""
    shape = (479, 479, 479)
    _sampled_fd(shape, precision, _droplet(shape), 1, dict(tau_f=0.8, tau_g=1.3), tol, nsample=8)


@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
def test_fd_conservation_droplet_256(precision):
    """Mass, phi and momentum over 100 steps of the 256^3 droplet."""
    shape = (256, 256, 256)
    lb = make_lb(shape, precision=precision, order_param="fd")
    lb.init_phi(_droplet(shape))
    s0 = lb.sums().cpu().numpy()
    lb.step(100)
    s1 = lb.sums().cpu().numpy()
    n = 256 ** 3
    # phi is FP64 in both modes; mass and momentum as the LB scheme's storage
    tol = 1e-9 * n if precision == "fp64" else 2e-7 * n
    assert np.abs(s1 - s0).max() <= tol, (s1 - s0)
    assert abs(s1[1] - s0[1]) <= 1e-9 * n


# ---- with the force coupling (the paper's arrangement) ------------------------
# One step at x depends on phi within distance 3 here (the fluxes use u at the
# face neighbours, whose force needs Pi one site further), still inside the
# 7^3 window.

@pytest.mark.parametrize("steps", [0, 1, 10, 100])
def test_fd_force_spinodal_16cubed(steps):
    shape = (16, 16, 16)
    got, ref, *_ = _run_both(shape, steps, lbinputs.spinodal_phi0(shape), coupling="force")
    errs = field_errors(got, ref, NAMES)
    assert max(errs.values()) <= TOL, errs


@pytest.mark.parametrize("shape", [(5, 6, 7), (3, 5, 131), (1, 7, 1), (2, 2, 2)])
def test_fd_force_ragged_degenerate_tau_not_one(shape):
    phi0 = lbinputs.spinodal_phi0(shape, seed=12, amp=0.4)
    got, ref, *_ = _run_both(shape, 25, phi0, coupling="force", tau_f=0.8, tau_g=1.3)
    errs = field_errors(got, ref, NAMES)
    assert max(errs.values()) <= TOL, errs


def test_fd_force_droplet_and_step_sums():
    """A sharp droplet (large force at the interface), 50 steps; per-step sums
    (momentum of j + F/2) against the oracle's and conserved."""
    shape = (24, 20, 22)
    pr = lbinputs.SPINODAL_PARAMS
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    phi0 = lbinputs.droplet_phi0(shape, 6.0, xi, noise=1e-3, seed=3)
    got, ref, lb, p = _run_both(shape, 50, phi0, coupling="force")
    errs = field_errors(got, ref, NAMES)
    assert max(errs.values()) <= TOL, errs
    hist = lb.step_sums(10).cpu().numpy()
    want = oracle.fd_sums(p, *oracle.fd_run(p, *oracle.fd_init(p, phi0), 50))
    np.testing.assert_allclose(hist[0], want, rtol=1e-12, atol=1e-12)
    assert np.abs(hist[:, :2] - hist[0, :2]).max() <= 1e-11
    assert np.abs(hist[:, 2:] - hist[0, 2:]).max() <= 1e-12


def test_fd_force_fp32_storage():
    shape = (16, 16, 16)
    phi0 = lbinputs.spinodal_phi0(shape, seed=14, amp=0.3)
    got, ref, *_ = _run_both(shape, 20, phi0, precision="fp32_dev", coupling="force", tau_f=0.8,
                             tau_g=1.3)
    f, rho, u, phi = got
    rf, rrho, ru, rphi = ref
    assert np.abs(phi - rphi).max() <= 1e-6
    assert np.abs(rho - rrho).max() <= 1e-6
    assert np.abs(u - ru).max() <= 1e-7


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_dev", 2e-6)])
def test_fd_force_sampled_parity_droplet_256(precision, tol):
    shape = (256, 256, 256)
    _sampled_fd(shape, precision, _droplet(shape), 5, dict(tau_f=0.8, tau_g=1.3), tol,
                coupling="force")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_dev", 2e-6)])
def test_fd_force_sampled_parity_maximum_size(precision, tol):
    """479^3, the largest accepted cube, ragged in every tile dimension of the
    marching collision pass and of the flux pass."""
    shape = (479, 479, 479)
    _sampled_fd(shape, precision, _droplet(shape), 1, dict(tau_f=0.8, tau_g=1.3), tol, nsample=8,
                coupling="force")
