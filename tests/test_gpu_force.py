"""Parity of the force coupling (body force -div Pi with Guo forcing) between
the HIP path (through the C ABI) and the CPU oracle.

Bar (FP64): for every output field F (f, g, rho, u, phi; u = (j + F/2)/rho),
max_x |F_gpu - F_oracle| / max_x |F_oracle| <= 1e-12 (u on scale 1).  FP32
deviation storage: within its rounding (phi, rho 1e-6, u 1e-7), as the
stress coupling.
"""
from __future__ import annotations

import numpy as np
import pytest

import lbinputs
import oracle
from tests._gpu import field_errors, gpu_state, make_lb, oracle_params, oracle_state

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _run_both(shape, steps, phi0, **kw):
    print(f"[force] shape={shape} steps={steps} params={kw}", flush=True)
    lb = make_lb(shape, coupling="force", **kw)
    lb.init_phi(phi0)
    lb.step(steps)
    got = gpu_state(lb)
    p = oracle_params(shape, coupling=1, **kw)
    ref = oracle_state(p, *oracle.run(p, *oracle.init(p, phi0), steps))
    return got, ref, lb, p


@pytest.mark.parametrize("steps", [0, 1, 10, 100])
def test_force_spinodal_16cubed(steps):
    shape = (16, 16, 16)
    got, ref, *_ = _run_both(shape, steps, lbinputs.spinodal_phi0(shape))
    errs = field_errors(got, ref)
    assert max(errs.values()) <= TOL, errs


@pytest.mark.parametrize("shape", [(5, 6, 7), (3, 5, 131), (17, 9, 70), (1, 7, 1), (2, 2, 2)])
def test_force_noncubic_ragged_degenerate_tau_not_one(shape):
    phi0 = lbinputs.spinodal_phi0(shape, seed=12, amp=0.4)
    got, ref, *_ = _run_both(shape, 25, phi0, tau_f=0.8, tau_g=1.3)
    errs = field_errors(got, ref)
    assert max(errs.values()) <= TOL, errs


def test_force_droplet_interface():
    """A sharp tanh droplet: the force is large at the interface."""
    shape = (24, 20, 22)
    pr = lbinputs.SPINODAL_PARAMS
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    phi0 = lbinputs.droplet_phi0(shape, 6.0, xi, noise=1e-3, seed=3)
    got, ref, lb, p = _run_both(shape, 50, phi0)
    errs = field_errors(got, ref)
    assert max(errs.values()) <= TOL, errs
    # the sums: mass, phi and momentum of rho u = j + F/2
    np.testing.assert_allclose(lb.sums().cpu().numpy(), oracle.sums(p, *oracle.run(
        p, *oracle.init(p, phi0), 50)), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("tau_g", [1.3, 1.0])
@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
@pytest.mark.parametrize("shape,seg", [((16, 16, 16), 0), ((16, 16, 16), 5), ((5, 6, 7), 2),
                                       ((3, 5, 131), 0), ((17, 9, 70), 4), ((1, 7, 1), 0),
                                       ((2, 2, 2), 1), ((6, 13, 200), 3), ((24, 20, 192), 0)])
def test_force_single_pass_matches_per_site(precision, shape, seg, tau_g):
    """The single pass (phi summed from its own pulls, Pi of each site once,
    in LDS) and the phi pass + per-site collision (Pi at each face
    neighbour) give bit-identical levels: ragged tiles, one-plane and long
    segments, extents 1 and 2; tau_g = 1 takes the collision that loads no
    g."""
    print(f"[force fused] {shape} segment_x={seg} {precision} tau_g={tau_g}", flush=True)
    phi0 = lbinputs.spinodal_phi0(shape, seed=19, amp=0.4)
    out = []
    for kern in ("fused", "two_pass"):
        lb = make_lb(shape, precision=precision, coupling="force", kernel=kern, segment_x=seg,
                     tau_f=0.8, tau_g=tau_g)
        lb.init_phi(phi0)
        lb.step(7)
        out.append(gpu_state(lb))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("layout,v", [("soa", 0), ("aosoa", 8)])
def test_force_layouts_bit_identical(layout, v):
    shape = (6, 7, 16)
    phi0 = lbinputs.spinodal_phi0(shape, seed=8, amp=0.3)
    out = []
    for lay, vv in (("rows", 0), (layout, v)):
        lb = make_lb(shape, coupling="force", layout=lay, aosoa_len=vv, tau_f=0.9)
        lb.init_phi(phi0)
        lb.step(9)
        out.append(gpu_state(lb))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("tau_g", [1.3, 1.0])
@pytest.mark.parametrize("prec,kernel", [("fp64", "fused"), ("fp64", "two_pass"),
                                         ("fp32_dev", "fused"), ("fp32_dev", "two_pass")])
def test_force_step_sums_history(prec, kernel, tau_g):
    """lb_step_sums with the force coupling: row t holds lb_sums of the state
    step t starts from (momentum sums of j + F/2, F of that state), whether
    the single pass reduces them itself or the two-pass variant runs its
    moments pass; the step itself is bit-identical to lb_step."""
    shape = (11, 9, 70)
    phi0 = lbinputs.spinodal_phi0(shape, seed=23, amp=0.3)
    kw = dict(tau_f=0.8, tau_g=tau_g)
    print(f"[force step sums] {prec} {kernel} tau_g={tau_g}", flush=True)
    a = make_lb(shape, precision=prec, kernel=kernel, coupling="force", **kw)
    a.init_phi(phi0)
    b = make_lb(shape, precision=prec, kernel=kernel, coupling="force", **kw)
    b.init_phi(phi0)
    hist = a.step_sums(6).cpu().numpy()
    for t in range(6):
        ref = b.sums().cpu().numpy()
        np.testing.assert_allclose(hist[t], ref, rtol=1e-13, atol=1e-13)
        b.step(1)
    for x, y in zip(gpu_state(a), gpu_state(b)):
        assert np.array_equal(x, y)


def test_force_step_sums_and_determinism():
    """Per-step FP64 sums are conserved (mass, phi; momentum to round-off), and
    two runs from one checkpoint agree bit for bit."""
    shape = (12, 10, 14)
    phi0 = lbinputs.spinodal_phi0(shape, seed=2, amp=0.3)
    lb = make_lb(shape, coupling="force", tau_f=0.8, tau_g=1.1)
    lb.init_phi(phi0)
    hist = lb.step_sums(30).cpu().numpy()
    assert np.abs(hist[:, :2] - hist[0, :2]).max() <= 1e-11
    assert np.abs(hist[:, 2:] - hist[0, 2:]).max() <= 1e-12
    ck = lb.get_state()
    lb.step(7)
    a = gpu_state(lb)
    lb.set_state(ck)
    lb.step(7)
    b = gpu_state(lb)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("tau_g", [1.3, 1.0])
@pytest.mark.parametrize("shape", [(16, 16, 16), (9, 6, 131)])
def test_force_fp32_storage(shape, tau_g):
    """FP32 deviation storage of the force coupling follows the FP64 oracle to
    FP32 rounding over 20 steps (tau_f != 1; tau_g = 1 takes the collision
    that loads no g)."""
    phi0 = lbinputs.spinodal_phi0(shape, seed=14, amp=0.3)
    lb = make_lb(shape, precision="fp32_dev", coupling="force", tau_f=0.8, tau_g=tau_g)
    lb.init_phi(phi0)
    lb.step(20)
    f, g, rho, u, phi = gpu_state(lb)
    p = oracle_params(shape, coupling=1, tau_f=0.8, tau_g=tau_g)
    rf, rg, rrho, ru, rphi = oracle_state(p, *oracle.run(p, *oracle.init(p, phi0), 20))
    assert np.abs(phi - rphi).max() <= 1e-6
    assert np.abs(rho - rrho).max() <= 1e-6
    assert np.abs(u - ru).max() <= 1e-7


def test_force_fp32_droplet_phi_error_vs_fp64():
    """A droplet over 300 steps: max |phi32 - phi64| <= 1e-5 in the force coupling."""
    shape = (40, 40, 40)
    pr = lbinputs.SPINODAL_PARAMS
    xi = lbinputs.interface_width(pr["A"], pr["kappa"])
    phi0 = lbinputs.droplet_phi0(shape, 10.0, xi, noise=1e-3, seed=4)
    out = {}
    for prec in ("fp64", "fp32_dev"):
        lb = make_lb(shape, precision=prec, coupling="force")
        lb.init_phi(phi0)
        lb.step(300)
        out[prec] = lb.phi().cpu().numpy()
    err = np.abs(out["fp32_dev"] - out["fp64"]).max()
    print(f"[force] fp32 vs fp64 phi error after 300 steps: {err:.3e}", flush=True)
    assert err <= 1e-5

