"""The single-pass kernel's memory-only twin (LB_KERNEL_STREAM): the same
kernel with the collision left out, so the populations stream freely.  Its
output is checked against the oracle's propagation (a pinned permutation)
applied the same number of times: bit for bit in FP64 storage (the twin only
copies), to FP32 rounding with FP32 deviation storage.  Lattices cover ragged
tiles, the 8 x 64 tile shape and full 4 x 128 tiles (the pipelined FP32 path)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import lbinputs
import oracle
from tests._gpu import make_lb, oracle_params

pytestmark = pytest.mark.gpu


def _random_dist(shape, seed):
    f = 1.0 / 19.0 + 0.02 * lbinputs.random_field((19,) + tuple(shape), seed, -0.5, 0.5)
    g = 0.1 * lbinputs.random_field((19,) + tuple(shape), seed + 1, -0.5, 0.5)
    return f, g


@pytest.mark.parametrize("shape", [(7, 9, 11), (4, 8, 128), (5, 8, 192), (3, 16, 64)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
def test_stream_twin_is_free_streaming(shape, precision):
    steps = 5
    print(f"[twin] shape={shape} {precision} steps={steps}", flush=True)
    f0, g0 = _random_dist(shape, 11)
    lb = make_lb(shape, precision=precision, kernel="stream")
    lb.import_dist(f0, g0)
    fi, gi = (t.cpu().numpy() for t in lb.export_dist())  # the stored (FP32: rounded) input
    lb.step(steps)
    f, g = (t.cpu().numpy() for t in lb.export_dist())
    p = oracle_params(shape)
    rf, rg = fi, gi
    for _ in range(steps):
        rf, rg = oracle.stream(p, rf), oracle.stream(p, rg)
    if precision == "fp64":
        assert np.array_equal(f, rf) and np.array_equal(g, rg)
    else:
        # f deviations move unchanged; g deviations are re-referenced to the
        # destination's phi each step (two FP32 roundings of O(0.1) values)
        assert np.abs(f - rf).max() <= 1e-15
        assert np.abs(g - rg).max() <= 2e-7 * steps


def test_stream_twin_conserves_and_rejects_the_adjoint():
    shape = (12, 8, 128)
    lb = make_lb(shape, precision="fp32_dev", kernel="stream", adjoint=True)
    lb.init_phi(lbinputs.spinodal_phi0(shape))
    s0 = lb.sums().cpu().numpy()
    hist = lb.step_sums(4).cpu().numpy()
    s1 = lb.sums().cpu().numpy()
    # mass and momentum: the f deviations move unchanged; sum phi: each
    # step re-rounds the FP32 g deviations to their new reference (about
    # 2e-8 per step here, against sum phi = 0.42)
    for k, tol in ((0, 1e-9), (1, 1e-6), (2, 1e-9), (3, 1e-9), (4, 1e-9)):
        assert np.abs(hist[:, k] - s0[k]).max() <= tol and abs(s1[k] - s0[k]) <= tol, k
    from paper_1609_01479_amd._abi import LB_ESTATE, LbError
    with pytest.raises(LbError) as e:
        lb.adjoint_seed(np.zeros(shape))
    assert e.value.status == LB_ESTATE
    torch.cuda.synchronize()


@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
def test_sibling_context_steps_on_the_shared_buffers(precision):
    """LB.sibling (how the bench times the step and its twin on the same
    memory): a second context on the lattice's own buffers starts from the
    level the first one wrote and steps with its own kernel variant -- here
    the two-pass variant, bit-identical to a separate single-pass lattice."""
    shape = (9, 10, 70)
    phi0 = lbinputs.spinodal_phi0(shape)
    lb = make_lb(shape, precision=precision)
    lb.init_phi(phi0)
    sib = lb.sibling("two_pass")
    sib.step(3)
    ref = make_lb(shape, precision=precision)
    ref.init_phi(phi0)
    ref.step(3)
    for a, b in zip(sib.moments(), ref.moments()):
        assert torch.equal(a, b)
    twin = lb.sibling("stream")
    assert twin.params.kernel == 2 and lb.params.kernel == 0
    sib.close()
    twin.close()
    torch.cuda.synchronize()
