"""x-slab shards (halo_x): the one-GPU part of the paper's domain
decomposition with halo regions.  A shard's step reads its halo planes,
filled through lb_pack_faces / lb_unpack_faces, in place of the periodic
wrap, so

* a shard that receives its own faces steps exactly like the periodic
  lattice of the same extents (bit for bit), including at the shape of one
  GPU's share of the 256^3 benchmark lattice split over 8 GPUs; and
* a periodic lattice split into two shards that exchange faces every step
  matches the undivided lattice bit for bit.

Every comparison is of whole dense post-propagation distributions (f, g)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import lbinputs
from tests._gpu import make_lb

pytestmark = pytest.mark.gpu

KW = dict(tau_f=0.8, tau_g=1.3)


def _extended(phi0, lo, hi):
    """Planes lo-1 .. hi of phi0 (periodic in x), for a shard of planes lo .. hi-1."""
    nx = phi0.shape[0]
    return np.ascontiguousarray(phi0[[(x % nx) for x in range(lo - 1, hi + 1)]])


def _exchange(shards, faces):
    """Each shard's lower neighbour is the previous one (periodically)."""
    for lb, (lo, hi) in zip(shards, faces):
        lb.pack_faces(lo, hi)
    n = len(shards)
    for k, lb in enumerate(shards):
        lb.unpack_faces(faces[(k - 1) % n][1], faces[(k + 1) % n][0])


def _dist(lb):
    f, g = lb.export_dist()
    return f, g


@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
@pytest.mark.parametrize("shape,steps", [((5, 9, 11), 8), ((2, 8, 128), 6), ((3, 16, 64), 5),
                                         ((32, 256, 256), 3)])
def test_self_exchange_matches_the_periodic_step(shape, steps, precision):
    print(f"[shard self-exchange] shape={shape} {precision} steps={steps}", flush=True)
    phi0 = lbinputs.droplet_phi0(shape, min(shape) / 3.0, 1.1314, noise=1e-3, seed=7)
    per = make_lb(shape, precision=precision, **KW)
    per.init_phi(phi0)
    sh = make_lb(shape, precision=precision, halo_x=True, **KW)
    sh.init_phi(_extended(phi0, 0, shape[0]))
    faces = [(sh.new_face(), sh.new_face())]
    for t in range(steps):
        _exchange([sh], faces)
        sh.step(1)
        per.step(1)
    _exchange([sh], faces)
    fp, gp = _dist(per)
    fs, gs = _dist(sh)
    torch.cuda.synchronize()
    assert torch.equal(fs, fp) and torch.equal(gs, gp)
    # moments and sums read the halo planes of the current level too
    for a, b in zip(sh.moments(), per.moments()):
        assert torch.equal(a, b)
    assert torch.equal(sh.sums(), per.sums())


@pytest.mark.parametrize("precision", ["fp64", "fp32_dev"])
@pytest.mark.parametrize("m,ny,nz,steps", [(4, 9, 11, 7), (16, 64, 128, 4)])
def test_two_shards_match_the_undivided_lattice(m, ny, nz, steps, precision):
    print(f"[two shards] {m}+{m} x {ny} x {nz} {precision} steps={steps}", flush=True)
    shape = (2 * m, ny, nz)
    phi0 = lbinputs.spinodal_phi0(shape, seed=31, amp=0.3)
    whole = make_lb(shape, precision=precision, **KW)
    whole.init_phi(phi0)
    shards = [make_lb((m, ny, nz), precision=precision, halo_x=True, **KW) for _ in range(2)]
    shards[0].init_phi(_extended(phi0, 0, m))
    shards[1].init_phi(_extended(phi0, m, 2 * m))
    faces = [(lb.new_face(), lb.new_face()) for lb in shards]
    for t in range(steps):
        _exchange(shards, faces)
        for lb in shards:
            lb.step(1)
        whole.step(1)
    _exchange(shards, faces)
    fw, gw = _dist(whole)
    parts = [_dist(lb) for lb in shards]
    torch.cuda.synchronize()
    assert torch.equal(torch.cat([parts[0][0], parts[1][0]], dim=1), fw)
    assert torch.equal(torch.cat([parts[0][1], parts[1][1]], dim=1), gw)
