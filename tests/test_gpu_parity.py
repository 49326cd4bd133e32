"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar (FP64): for every output field F (f, g, rho, u, phi),
max_x |F_gpu - F_oracle| / max_x |F_oracle| <= 1e-12 after up to 100 steps.
Integer/permutation work (propagation, import/export, checkpoints) is
compared bit for bit.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import lbinputs
import oracle
from tests._gpu import field_errors, gpu_state, make_lb, oracle_params, oracle_state, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-12
NAMES = ("f", "g", "rho", "u", "phi")


def _run_both(shape, steps, phi0=None, precision="fp64", **kw):
    print(f"[parity] shape={shape} steps={steps} {precision} params={kw}", flush=True)
    phi0 = lbinputs.spinodal_phi0(shape) if phi0 is None else phi0
    lb = make_lb(shape, precision=precision, **kw)
    lb.init_phi(phi0)
    lb.step(steps)
    got = gpu_state(lb)
    p = oracle_params(shape, **kw)
    ref = oracle_state(p, *oracle.run(p, *oracle.init(p, phi0), steps))
    return got, ref


@pytest.mark.parametrize("steps", [0, 1, 10, 100])
def test_spinodal_16cubed_fp64(steps):
    """16^3 spinodal decomposition, phi0 ~ U(-0.05, 0.05), default parameters."""
    got, ref = _run_both((16, 16, 16), steps)
    errs = field_errors(got, ref)
    assert max(errs.values()) <= TOL, errs


@pytest.mark.parametrize("shape", [(5, 6, 7), (8, 4, 12), (3, 5, 131), (17, 9, 70)])
def test_noncubic_and_ragged_tau_not_one(shape):
    """Non-cubic lattices (axis swaps) and ragged tails; tau != 1 exercises the
    non-equilibrium part of the BGK update."""
    got, ref = _run_both(shape, 30, tau_f=0.8, tau_g=1.3)
    errs = field_errors(got, ref)
    assert max(errs.values()) <= TOL, errs


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 2, 2), (1, 1, 300), (1, 7, 1), (2, 3, 1)])
def test_degenerate_lattices(shape):
    """Extents 1 and 2: neighbours coincide with the site or with each other."""
    phi0 = lbinputs.spinodal_phi0(shape, seed=99, amp=0.5)
    got, ref = _run_both(shape, 12, phi0=phi0, tau_f=0.9, tau_g=1.2)
    errs = field_errors(got, ref)
    assert max(errs.values()) <= TOL, errs


def test_arbitrary_state_one_step():
    """A random non-equilibrium state imported through the ABI, one step."""
    shape = (6, 7, 9)
    p = oracle_params(shape, tau_f=0.7, tau_g=1.6, gamma=0.3)
    f0, g0 = oracle.init(p, lbinputs.spinodal_phi0(shape, seed=4, amp=0.8))
    rng = np.random.default_rng(1)
    f0 = f0 * (1 + 0.2 * rng.standard_normal(f0.shape))
    g0 = g0 + 0.05 * rng.standard_normal(g0.shape)
    lb = make_lb(shape, tau_f=0.7, tau_g=1.6, gamma=0.3)
    lb.import_dist(f0, g0)
    lb.step(3)
    got = gpu_state(lb)
    ref = oracle_state(p, *oracle.run(p, f0, g0, 3))
    errs = field_errors(got, ref)
    assert max(errs.values()) <= TOL, errs


def test_import_export_round_trip_bit_exact():
    shape = (5, 4, 67)
    f = lbinputs.random_field((19,) + shape, 3)
    g = lbinputs.random_field((19,) + shape, 4)
    lb = make_lb(shape)
    lb.import_dist(f, g)
    f2, g2, *_ = gpu_state(lb)
    assert np.array_equal(f2, f) and np.array_equal(g2, g)


def test_state_layout_shift_and_restore_bit_exact():
    """Importing a periodically shifted state exports the shifted state, and a
    saved time level restores bit for bit."""
    shape = (4, 5, 6)
    f = lbinputs.random_field((19,) + shape, 8)
    g = lbinputs.random_field((19,) + shape, 9)
    lb = make_lb(shape)
    lb.import_dist(f, g)
    st = lb.get_state().clone()
    lb2 = make_lb(shape)
    sh = (1, -2, 3)
    lb2.import_dist(np.roll(f, sh, (1, 2, 3)), np.roll(g, sh, (1, 2, 3)))
    fa, ga, *_ = gpu_state(lb)
    fb, gb, *_ = gpu_state(lb2)
    assert np.array_equal(np.roll(fa, sh, (1, 2, 3)), fb)
    assert np.array_equal(np.roll(ga, sh, (1, 2, 3)), gb)
    lb.step(2)
    lb.set_state(st)
    assert np.array_equal(gpu_state(lb)[0], f)


def test_shift_invariance_bit_exact():
    shape = (8, 6, 70)
    phi0 = lbinputs.spinodal_phi0(shape, seed=5)
    sh = (3, -1, 17)
    a = make_lb(shape, tau_f=0.8, tau_g=1.3)
    a.init_phi(phi0)
    a.step(20)
    b = make_lb(shape, tau_f=0.8, tau_g=1.3)
    b.init_phi(np.roll(phi0, sh, (0, 1, 2)))
    b.step(20)
    fa, ga, *_ = gpu_state(a)
    fb, gb, *_ = gpu_state(b)
    assert np.array_equal(np.roll(fa, sh, (1, 2, 3)), fb)
    assert np.array_equal(np.roll(ga, sh, (1, 2, 3)), gb)


def test_determinism_and_checkpoint_restore_bit_exact():
    shape = (16, 16, 16)
    phi0 = lbinputs.spinodal_phi0(shape)
    a = make_lb(shape, tau_f=0.8, tau_g=1.3)
    a.init_phi(phi0)
    a.step(7)
    ck = a.get_state().clone()
    a.step(13)
    ra = gpu_state(a)
    a.set_state(ck)
    a.step(13)
    rb = gpu_state(a)
    for x, y in zip(ra, rb):
        assert np.array_equal(x, y)


def test_conservation_and_sums_match_oracle():
    shape = (12, 10, 14)
    p = oracle_params(shape, tau_f=0.8, tau_g=1.3)
    f0, g0 = oracle.init(p, lbinputs.spinodal_phi0(shape, seed=6))
    rng = np.random.default_rng(2)
    f0 = f0 * (1 + 0.01 * rng.standard_normal(f0.shape))
    lb = make_lb(shape, tau_f=0.8, tau_g=1.3)
    lb.import_dist(f0, g0)
    s0 = lb.sums().cpu().numpy()
    ref0 = oracle.sums(p, f0, g0)
    np.testing.assert_allclose(s0, ref0, rtol=1e-13, atol=1e-13)
    lb.step(50)
    s1 = lb.sums().cpu().numpy()
    np.testing.assert_allclose(s1, s0, rtol=0, atol=1e-11)


@pytest.mark.parametrize("prec", ["fp64", "fp32_dev"])
@pytest.mark.parametrize("shape", [(13, 10, 70), (13, 8, 256), (13, 7, 256)])
def test_kernel_variants_and_segments_agree(prec, shape):
    """The single-pass kernel is independent of its x-segment length (bit for
    bit: every site's arithmetic is the same), and agrees with the two-pass
    variant.  (13, 8, 256) is made of full tiles only (FP64 4 x 128; FP32
    2 x 256, whole rows), which the FP32 kernel marches with its
    software-pipelined path; (13, 7, 256) adds a one-row tail tile to those;
    (13, 10, 70) has ragged tiles only, each spanning the z extent."""
    print(f"[variants] {prec} {shape}", flush=True)
    phi0 = lbinputs.spinodal_phi0(shape, seed=21, amp=0.3)
    out = {}
    for kernel, sx in (("fused", 0), ("fused", 1), ("fused", 3), ("fused", 13), ("two_pass", 0)):
        lb = make_lb(shape, precision=prec, tau_f=0.8, tau_g=1.3, kernel=kernel, segment_x=sx)
        lb.init_phi(phi0)
        lb.step(9)
        out[(kernel, sx)] = gpu_state(lb)
    ref = out[("fused", 0)]
    for key in (("fused", 1), ("fused", 3), ("fused", 13)):
        for a, b in zip(out[key], ref):
            assert np.array_equal(a, b), key
    errs = field_errors(out[("two_pass", 0)], ref)
    assert max(errs.values()) <= (1e-14 if prec == "fp64" else 1e-6), errs


@pytest.mark.parametrize("shape", [(12, 8, 128), (10, 6, 320), (3, 4, 128), (6, 5, 256)])
@pytest.mark.parametrize("prec", ["fp64", "fp32_dev"])
def test_full_and_mixed_tiles(prec, shape):
    """Lattices made of full 4 x 128 tiles (the FP32 kernel's pipelined,
    branch-free march), and of full and ragged tiles in one launch, against
    the oracle: FP64 to 1e-12, FP32 storage to its rounding."""
    phi0 = lbinputs.spinodal_phi0(shape, seed=31, amp=0.4)
    got, ref = _run_both(shape, 20, phi0=phi0, precision=prec, tau_f=0.8, tau_g=1.3)
    errs = field_errors(got, ref)
    if prec == "fp64":
        assert max(errs.values()) <= TOL, errs
    else:
        assert errs["phi"] <= 1e-6 and errs["rho"] <= 1e-6 and errs["u"] <= 1e-7, errs


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 2, 2), (1, 1, 300), (1, 7, 1), (2, 3, 1), (3, 5, 131)])
def test_degenerate_lattices_fp32(shape):
    """FP32 storage on extents 1 and 2 and a ragged tail: the single-pass
    kernel's LDS phi planes and halo ring wrap onto themselves; it must agree
    with the two-pass variant (global reads) and follow the oracle to FP32
    rounding."""
    phi0 = lbinputs.spinodal_phi0(shape, seed=98, amp=0.5)
    out = {}
    for kernel in ("fused", "two_pass"):
        lb = make_lb(shape, precision="fp32_dev", tau_f=0.9, tau_g=1.2, kernel=kernel)
        lb.init_phi(phi0)
        lb.step(12)
        out[kernel] = gpu_state(lb)
    errs = field_errors(out["fused"], out["two_pass"])
    assert max(errs.values()) <= 1e-6, errs
    p = oracle_params(shape, tau_f=0.9, tau_g=1.2)
    ref = oracle_state(p, *oracle.run(p, *oracle.init(p, phi0), 12))
    errs = field_errors(out["fused"], ref)
    assert errs["phi"] <= 1e-6 and errs["rho"] <= 1e-6 and errs["u"] <= 1e-7, errs


@pytest.mark.parametrize("prec", ["fp64", "fp32_dev"])
def test_step_from_matches_step_bit_exact(prec):
    """lb_step_from between caller buffers gives the same bits as lb_step."""
    shape = (9, 8, 70)
    lb = make_lb(shape, precision=prec, tau_f=0.8, tau_g=1.3)
    lb.init_phi(lbinputs.spinodal_phi0(shape, seed=17, amp=0.3))
    lb.step(4)
    a = lb.get_state().clone()
    b = lb.new_state()
    c = lb.new_state()
    lb.step_from(a, b)
    lb.step_from(b, c)
    lb.step(2)
    ref = gpu_state(lb)
    lb.set_state(c)
    for x, y in zip(gpu_state(lb), ref):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", ["fp64", "fp32_dev"])
@pytest.mark.parametrize("op,coupling", [("lb", "stress"), ("lb", "force"), ("fd", "stress"),
                                         ("fd", "force")])
def test_zero_steps_change_nothing(prec, op, coupling):
    """nsteps = 0 is a no-op for lb_step, lb_step_sums and
    lb_step_sums_noalloc: the state stays bit for bit, no sums are written,
    and the next step is the step it would have been."""
    def snap(lb):
        f, g = lb.export_dist()
        return [t.cpu().numpy() for t in (f, g, *lb.moments()) if t is not None]

    shape = (6, 5, 70)
    phi0 = lbinputs.spinodal_phi0(shape, seed=4, amp=0.3)
    a = make_lb(shape, precision=prec, order_param=op, coupling=coupling)
    b = make_lb(shape, precision=prec, order_param=op, coupling=coupling)
    for lb in (a, b):
        lb.init_phi(phi0)
        lb.step(3)
    ref = snap(a)
    out = torch.full((2, 5), 7.0, dtype=torch.float64, device="cuda:0")
    a.step(0)
    a.step_sums(0, out)
    a.step_sums_noalloc(0, out)
    for x, y in zip(snap(a), ref):
        assert np.array_equal(x, y)
    assert bool((out == 7.0).all())
    a.step(1)
    b.step(1)
    for x, y in zip(snap(a), snap(b)):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec,kernel", [("fp64", "fused"), ("fp64", "two_pass"),
                                         ("fp32_dev", "fused"), ("fp32_dev", "two_pass")])
def test_step_sums_history(prec, kernel):
    """lb_step_sums: row t holds the conserved sums of the state step t starts
    from (against lb_sums of that state and the oracle); the step itself is
    unchanged (bit-identical to lb_step)."""
    shape = (11, 9, 70)
    phi0 = lbinputs.spinodal_phi0(shape, seed=23, amp=0.3)
    kw = dict(tau_f=0.8, tau_g=1.3)
    a = make_lb(shape, precision=prec, kernel=kernel, **kw)
    a.init_phi(phi0)
    b = make_lb(shape, precision=prec, kernel=kernel, **kw)
    b.init_phi(phi0)
    hist = a.step_sums(5).cpu().numpy()
    for t in range(5):
        ref = b.sums().cpu().numpy()
        np.testing.assert_allclose(hist[t], ref, rtol=1e-13, atol=1e-13)
        b.step(1)
    for x, y in zip(gpu_state(a), gpu_state(b)):
        assert np.array_equal(x, y)
    p = oracle_params(shape, **kw)
    f0, g0 = oracle.init(p, phi0)
    # FP32 storage rounds the initial populations once (relative ~1e-9 here)
    tol = 1e-12 if prec == "fp64" else 1e-7
    np.testing.assert_allclose(hist[0], oracle.sums(p, f0, g0), rtol=tol, atol=tol)


LAYOUTS = [("soa", 0), ("aos", 0), ("aosoa", 1), ("aosoa", 8), ("aosoa", 64), ("aosoa", 256)]


@pytest.mark.parametrize("prec", ["fp64", "fp32_dev"])
@pytest.mark.parametrize("kernel", ["fused", "two_pass"])
def test_layouts_bit_identical(prec, kernel):
    """Every distribution layout runs the same arithmetic at every site: the
    exported state after 7 steps is bit-identical to the row-blocked default's
    (full and ragged tiles: ny = 6 is one 4-row tile and a 2-row tail)."""
    shape = (9, 6, 256)
    phi0 = lbinputs.spinodal_phi0(shape, seed=17, amp=0.3)
    ref = None
    for layout, v in [("rows", 0)] + LAYOUTS:
        print(f"[layouts] {prec} {kernel} {layout} {v}", flush=True)
        lb = make_lb(shape, precision=prec, tau_f=0.8, tau_g=1.3, kernel=kernel,
                     layout=layout, aosoa_len=v)
        lb.init_phi(phi0)
        lb.step(7)
        got = gpu_state(lb)
        if ref is None:
            ref = got
            continue
        for a, b, name in zip(got, ref, NAMES):
            assert np.array_equal(a, b), (layout, v, name)


@pytest.mark.parametrize("layout,v", [("soa", 0), ("aosoa", 32)])
def test_layout_adjoint_bit_identical(layout, v):
    """The adjoint step reads the saved state through the same layout: its
    gradients are bit-identical to the row-blocked default's."""
    shape = (6, 5, 64)
    T = 4
    phi0 = lbinputs.spinodal_phi0(shape, seed=23, amp=0.3)
    dphi = torch.tensor(lbinputs.random_field(shape, 4), device="cuda:0")
    out = []
    for lay, vv in (("rows", 0), (layout, v)):
        lb = make_lb(shape, precision="fp32_dev", adjoint=True, layout=lay, aosoa_len=vv)
        lb.init_phi(phi0)
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
