"""The adjoint kernels at a size where their resident workgroups sweep the
lattice in more than one round (72 x 64 x 64 = 294912 sites: each XCD's
eighth is 36864 sites against 32768 per round, so a full and a partial
round), for both order-parameter schemes and both couplings, against
autograd through the oracle's torch transcription of the step."""
from __future__ import annotations

import pytest
import torch

import lbinputs
import oracle.reverse as R
from tests._gpu import rel_err

pytestmark = pytest.mark.gpu

SHAPE = (72, 64, 64)


@pytest.mark.parametrize("coupling", ["stress", "force"])
@pytest.mark.parametrize("order_param,tau_g", [("lb", 1.3), ("lb", 1.0), ("fd", 1.3)])
def test_adjoint_two_rounds_matches_oracle(order_param, tau_g, coupling):
    """tau_g = 1 takes the local kernels' path without lambda_g's specific
    components."""
    from paper_1609_01479_amd.rollout import rollout
    T = 3
    kw = dict(tau_f=0.8, tau_g=tau_g)
    pr = dict(lbinputs.SPINODAL_PARAMS, **kw)
    phi0 = lbinputs.spinodal_phi0(SHAPE, seed=31, amp=0.3)
    tgt = lbinputs.lamellar_target(SHAPE, 8, lbinputs.interface_width(pr["A"], pr["kappa"]))
    print(f"[adjoint sizes] {SHAPE} x {T} {order_param} {coupling} tau_g={tau_g}", flush=True)
    dev = torch.device("cuda:0")
    p0 = torch.tensor(phi0, dtype=torch.float64, device=dev, requires_grad=True)
    th = [torch.tensor(pr[k], dtype=torch.float64, device=dev, requires_grad=True)
          for k in ("A", "B", "kappa")]
    phiT = rollout(p0, *th, T, interval=2, gamma=pr["gamma"], tau_f=pr["tau_f"],
                   tau_g=pr["tau_g"], rho0=pr["rho0"], order_param=order_param,
                   coupling=coupling)
    loss = 0.5 * ((phiT - torch.tensor(tgt, device=dev)) ** 2).sum()
    loss.backward()
    fn = R.fd_loss_and_grads if order_param == "fd" else R.loss_and_grads
    rL, rphi, rA, rB, rk = fn(phi0, tgt, pr["A"], pr["B"], pr["kappa"], T, pr["gamma"],
                              pr["tau_f"], pr["tau_g"], pr["rho0"], coupling)
    assert abs(float(loss.detach()) - rL) <= 1e-12 * abs(rL)
    err = rel_err(p0.grad.cpu().numpy(), rphi)
    assert err <= 1e-10, err
    for name, t, b in zip(("A", "B", "kappa"), th, (rA, rB, rk)):
        assert abs(float(t.grad) - b) <= 1e-9 * abs(b), (name, float(t.grad), b)
