"""The allocation-free entry point lb_step_sums_noalloc (reduction partials in
the library's own device array) against lb_step_sums (partials in the
caller's scratch buffer): the same conserved sums and the same next state,
bit for bit, over two calls in a row on one GPU, the second on a smaller
lattice, for each step kernel that reduces."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import lbinputs
from tests._gpu import make_lb

pytestmark = pytest.mark.gpu

# (name, LB keywords): every path lb_step_sums takes -- the single-pass step
# in both storage precisions, the two-pass variant, the force coupling and
# the finite-difference order parameter (single pass with either coupling,
# and its two-pass variant, which reduces over one block per 256 sites)
CASES = [
    ("fused_fp64", dict(precision="fp64")),
    ("fused_fp32", dict(precision="fp32_dev")),
    ("two_pass_fp64", dict(precision="fp64", kernel="two_pass")),
    ("force_fp32", dict(precision="fp32_dev", coupling="force")),
    ("fd_fp64", dict(precision="fp64", order_param="fd")),
    ("fd_force_fp32", dict(precision="fp32_dev", order_param="fd", coupling="force")),
    ("fd_two_pass_fp64", dict(precision="fp64", order_param="fd", kernel="two_pass")),
]


def _run(shape, steps, kw, noalloc):
    lb = make_lb(shape, **kw)
    lb.init_phi(lbinputs.spinodal_phi0(shape))
    out = torch.full((steps, 5), float("nan"), dtype=torch.float64, device="cuda:0")
    if noalloc:
        lb.step_sums_noalloc(steps, out)
    else:
        lb.step_sums(steps, out)
    # the new state as dense arrays (a time level's padding is never written,
    # so its raw bytes are not comparable)
    f, g = lb.export_dist()
    rho, u, phi = lb.moments()
    torch.cuda.synchronize()
    state = [t.cpu().numpy() for t in (f, g, rho, u, phi) if t is not None]
    return out.cpu().numpy(), state


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_step_sums_twice(name, kw):
    # first call: several tiles in y and z and two x segments' worth of
    # workgroups, ragged in every direction; second call: a smaller lattice
    # (fewer partial blocks), so stale partials of the first would show
    for shape, steps in (((70, 36, 200), 3), ((13, 10, 14), 2)):
        print(f"noalloc {name} {shape} x {steps}", flush=True)
        ref_sums, ref_state = _run(shape, steps, kw, noalloc=False)
        sums, state = _run(shape, steps, kw, noalloc=True)
        assert np.isfinite(sums).all()
        assert np.array_equal(sums, ref_sums), (name, shape)
        for a, b in zip(state, ref_state):
            assert np.array_equal(a, b), (name, shape)


def test_noalloc_rejects_a_lattice_beyond_the_array():
    from paper_1609_01479_amd._abi import LbError
    lb = make_lb((1, 100000, 1))
    out = torch.empty((1, 5), dtype=torch.float64, device="cuda:0")
    with pytest.raises(LbError, match="partial blocks"):
        lb.step_sums_noalloc(1, out)
