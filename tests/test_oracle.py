"""Pins of the CPU oracle against what the mathematics fixes.

None of these re-type the oracle's formulas: each checks a property that an
independent route determines (exact rational lattice moments, Fourier
eigenvalues of the stencil, the variational derivative of a discrete free
energy, a thermodynamic and a mechanical identity of the stress, exact
conservation and permutation properties, lattice symmetries, and closed-form
hydrodynamic decay rates).  A dropped term, a wrong sign, a wrong weight or a
transposed index in the oracle breaks at least one of them.
"""
from fractions import Fraction
import math

import numpy as np
import pytest
import torch

import lbinputs
import oracle
import oracle.reverse as R


def _params(shape, **kw):
    base = dict(lbinputs.SPINODAL_PARAMS)
    base.update(kw)
    return oracle.Params(*shape, **base)


# ---------------------------------------------------------------- lattice --

def test_lattice_exact_moments():
    """D3Q19 isotropy up to 4th order, in exact rational arithmetic."""
    c, w = oracle.lattice()
    wf = [Fraction(x).limit_denominator(1000) for x in w]
    # the float weights are exactly the rationals they stand for
    for x, q in zip(w, wf):
        assert float(q) == x
    assert sorted(set(wf)) == [Fraction(1, 36), Fraction(1, 18), Fraction(1, 3)]
    # 1 rest + 6 faces + 12 edges, closed under negation, all distinct
    c2 = (c * c).sum(1)
    assert sorted(c2.tolist()) == [0] + [1] * 6 + [2] * 12
    assert len({tuple(v) for v in c.tolist()}) == 19
    for v in c.tolist():
        assert [-x for x in v] in c.tolist()
    assert sum(wf) == 1
    for a in range(3):
        assert sum(wi * int(ci[a]) for wi, ci in zip(wf, c)) == 0
        for b in range(3):
            m2 = sum(wi * int(ci[a]) * int(ci[b]) for wi, ci in zip(wf, c))
            assert m2 == (Fraction(1, 3) if a == b else 0)
            for g in range(3):
                assert sum(wi * int(ci[a] * ci[b] * ci[g]) for wi, ci in zip(wf, c)) == 0
    # fourth order: sum w c_a c_b c_c c_d = (1/9)(d_ab d_cd + d_ac d_bd + d_ad d_bc)
    for a in range(3):
        for b in range(3):
            for g in range(3):
                for d in range(3):
                    m4 = sum(wi * int(ci[a] * ci[b] * ci[g] * ci[d]) for wi, ci in zip(wf, c))
                    iso = Fraction(1, 9) * ((a == b) * (g == d) + (a == g) * (b == d)
                                            + (a == d) * (b == g))
                    assert m4 == iso
    # weights depend only on |c|^2 and the velocity order is rest, +-x, +-y, +-z, edges
    assert c[0].tolist() == [0, 0, 0]
    assert c[1:7].tolist() == [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]]


# ---------------------------------------------------------------- stencil --

@pytest.mark.parametrize("shape,mode", [((8, 10, 12), (1, 2, 3)), ((16, 5, 7), (3, 1, 2))])
def test_stencil_fourier_eigenvalues(shape, mode):
    """D_a cos(q.x) = -sin(q_a) sin(q.x);  lap cos(q.x) = -sum 2(1-cos q_a) cos(q.x)."""
    p = _params(shape)
    q = [2 * math.pi * m / n for m, n in zip(mode, shape)]
    xs = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    arg = sum(qa * xa for qa, xa in zip(q, xs))
    grad, lap = oracle.gradients(p, np.cos(arg))
    for a in range(3):
        np.testing.assert_allclose(grad[a], -math.sin(q[a]) * np.sin(arg), atol=1e-14)
    lam = -sum(2 * (1 - math.cos(qa)) for qa in q)
    np.testing.assert_allclose(lap, lam * np.cos(arg), atol=1e-13)


def test_stencil_axis_identity():
    """A field varying along one axis only has a gradient along that axis only."""
    shape = (6, 7, 9)
    p = _params(shape)
    for axis in range(3):
        prof = np.random.default_rng(axis).standard_normal(shape[axis])
        sl = [None, None, None]
        sl[axis] = slice(None)
        phi = np.broadcast_to(prof[tuple(sl)], shape).copy()
        grad, lap = oracle.gradients(p, phi)
        for a in range(3):
            if a != axis:
                assert np.all(grad[a] == 0.0)
        expect = 0.5 * (np.roll(prof, -1) - np.roll(prof, 1))
        np.testing.assert_allclose(grad[axis], np.broadcast_to(expect[tuple(sl)], shape), atol=1e-15)


# ------------------------------------------------------- chemical stress --

def test_mu_is_variational_derivative():
    """mu = dF/dphi for F = sum_x [A/2 phi^2 + B/4 phi^4 + kappa/2 sum_a (phi(x+e_a)-phi(x))^2].

    The forward-difference gradient energy has exactly the 7-point Laplacian
    as its variational derivative, so this pins mu's sign, powers and the
    stencil at once (autograd on F, a different function from mu).
    """
    shape = (7, 8, 9)
    p = _params(shape, A=-0.031, B=0.047, kappa=0.013)
    phi = lbinputs.random_field(shape, 11)
    t = torch.tensor(phi, requires_grad=True)
    F = (0.5 * p.A * t ** 2 + 0.25 * p.B * t ** 4).sum()
    for a in range(3):
        F = F + 0.5 * p.kappa * ((torch.roll(t, -1, a) - t) ** 2).sum()
    F.backward()
    grad, lap = oracle.gradients(p, phi)
    mu, _ = oracle.chemical(p, phi, grad, lap)
    np.testing.assert_allclose(mu, t.grad.numpy(), rtol=0, atol=1e-15)


def test_pressure_isotropic_part_is_thermodynamic():
    """tr(Pi)/3 - kappa|grad phi|^2/3 = phi mu - psi (bulk pressure p0 = phi mu - psi)."""
    shape = (6, 7, 8)
    p = _params(shape, A=-0.02, B=0.03, kappa=0.011)
    phi = lbinputs.random_field(shape, 5)
    grad, lap = oracle.gradients(p, phi)
    mu, pi = oracle.chemical(p, phi, grad, lap)
    g2 = (grad ** 2).sum(0)
    psi = 0.5 * p.A * phi ** 2 + 0.25 * p.B * phi ** 4 + 0.5 * p.kappa * g2
    tr = pi[0] + pi[3] + pi[5]
    np.testing.assert_allclose((tr - p.kappa * g2) / 3.0, phi * mu - psi, atol=1e-16)


def test_gibbs_duhem_mechanical_identity():
    """d_b Pi_ab = phi d_a mu in the continuum: on a smooth field the lattice
    versions agree to O(k^2), while any sign/term error leaves an O(1) gap."""
    n = 48
    p = _params((n, n, n), A=-0.05, B=0.05, kappa=0.02)
    k = 2 * math.pi / n
    x, y, z = np.meshgrid(*[np.arange(n)] * 3, indexing="ij")
    phi = (0.5 * np.sin(k * x) + 0.3 * np.cos(k * y + 0.4) + 0.2 * np.sin(k * z + 1.1)
           + 0.25 * np.sin(k * (x + y)) + 0.15 * np.cos(k * (y - z)))
    grad, lap = oracle.gradients(p, phi)
    mu, pi = oracle.chemical(p, phi, grad, lap)
    full = {(0, 0): pi[0], (0, 1): pi[1], (0, 2): pi[2], (1, 1): pi[3], (1, 2): pi[4],
            (2, 2): pi[5]}

    def comp(a, b):
        return full[(min(a, b), max(a, b))]

    def d(field, a):
        return 0.5 * (np.roll(field, -1, a) - np.roll(field, 1, a))

    scale = max(np.abs(phi * d(mu, a)).max() for a in range(3))
    for a in range(3):
        div = sum(d(comp(a, b), b) for b in range(3))
        err = np.abs(div - phi * d(mu, a)).max()
        assert err < 0.02 * scale, (a, err, scale)


def test_chemical_hand_values():
    """Bulk phases phi = +-sqrt(-A/B): mu = 0 and Pi = (A/2 + 3B/4) I = 0.0015625 I."""
    shape = (4, 4, 4)
    p = _params(shape)
    for s in (1.0, -1.0):
        phi = np.full(shape, s)
        grad, lap = oracle.gradients(p, phi)
        mu, pi = oracle.chemical(p, phi, grad, lap)
        assert np.all(grad == 0) and np.all(lap == 0)
        np.testing.assert_allclose(mu, 0.0, atol=1e-18)
        np.testing.assert_allclose(pi[[0, 3, 5]], 0.0015625, rtol=1e-14)
        np.testing.assert_allclose(pi[[1, 2, 4]], 0.0, atol=0)


# ----------------------------------------------------------- equilibria --

def _moment_checks(p, rho, j, phi, mu, pi6, feq, geq):
    c, _ = oracle.lattice()
    c = c.astype(np.float64)
    u = np.asarray(j) / rho
    pim = np.array([[pi6[0], pi6[1], pi6[2]], [pi6[1], pi6[3], pi6[4]], [pi6[2], pi6[4], pi6[5]]])
    np.testing.assert_allclose(feq.sum(), rho, rtol=1e-15)
    np.testing.assert_allclose(feq @ c, j, atol=1e-16)
    m2 = np.einsum("i,ia,ib->ab", feq, c, c)
    np.testing.assert_allclose(m2, rho / 3.0 * np.eye(3) + pim + rho * np.outer(u, u),
                               atol=2e-16)
    np.testing.assert_allclose(geq.sum(), phi, atol=2e-16)
    np.testing.assert_allclose(geq @ c, phi * u, atol=2e-17)
    m2g = np.einsum("i,ia,ib->ab", geq, c, c)
    np.testing.assert_allclose(m2g, p.gamma * mu * np.eye(3) + phi * np.outer(u, u), atol=2e-17)


def test_equilibrium_moments_exact():
    """sum feq (1, c, cc) = (rho, j, rho/3 I + Pi + rho u u); same for g with Gamma mu I + phi u u."""
    rng = np.random.default_rng(7)
    p = _params((3, 3, 3), gamma=0.37)
    for _ in range(50):
        rho = 1.0 + 0.1 * rng.standard_normal()
        j = 0.05 * rng.standard_normal(3)
        phi = rng.uniform(-1, 1)
        mu = 0.01 * rng.standard_normal()
        pi6 = 0.01 * rng.standard_normal(6)
        feq, geq = oracle.equilibrium_site(p, rho, j, phi, mu, pi6)
        _moment_checks(p, rho, j, phi, mu, pi6, feq, geq)


def test_equilibrium_rest_state():
    """rho0 at rest with phi = 0, Pi = 0: feq = w rho0 and geq = 0."""
    p = _params((3, 3, 3))
    _, w = oracle.lattice()
    feq, geq = oracle.equilibrium_site(p, 1.0, np.zeros(3), 0.0, 0.0, np.zeros(6))
    np.testing.assert_allclose(feq, w, rtol=1e-15)
    np.testing.assert_allclose(geq, 0.0, atol=0)


# ----------------------------------------------------------- collision --

def test_collision_conserves_per_site_and_tau1_gives_equilibrium():
    shape = (4, 5, 6)
    c, _ = oracle.lattice()
    for tf, tg in ((0.8, 1.3), (1.0, 1.0)):
        p = _params(shape, tau_f=tf, tau_g=tg)
        rng = np.random.default_rng(3)
        f0, g0 = oracle.init(p, lbinputs.spinodal_phi0(shape, seed=9))
        f = f0 + 0.01 * rng.standard_normal(f0.shape) / 19
        g = g0 + 0.01 * rng.standard_normal(g0.shape) / 19
        phi = oracle.order_parameter(p, g)
        grad, lap = oracle.gradients(p, phi)
        mu, pi = oracle.chemical(p, phi, grad, lap)
        fs, gs = oracle.collide(p, f, g, phi, mu, pi)
        np.testing.assert_allclose(fs.sum(0), f.sum(0), atol=1e-15)
        np.testing.assert_allclose(np.einsum("ia,ixyz->axyz", c, fs),
                                   np.einsum("ia,ixyz->axyz", c, f), atol=1e-16)
        np.testing.assert_allclose(gs.sum(0), g.sum(0), atol=1e-16)
        if tf == 1.0:
            s = (1, 2, 3)
            rho = f[(slice(None),) + s].sum()
            j = c.T @ f[(slice(None),) + s]
            feq, geq = oracle.equilibrium_site(p, rho, j, phi[s], mu[s], pi[(slice(None),) + s])
            np.testing.assert_allclose(fs[(slice(None),) + s], feq, atol=1e-16)
            np.testing.assert_allclose(gs[(slice(None),) + s], geq, atol=1e-16)


# ----------------------------------------------------------- streaming --

def test_stream_moves_delta_to_x_plus_c():
    shape = (5, 6, 7)
    p = _params(shape)
    c, _ = oracle.lattice()
    x0 = (4, 0, 3)
    for i in range(19):
        d = np.zeros((19,) + shape)
        d[(i,) + x0] = 1.0
        out = oracle.stream(p, d)
        dest = tuple((x0[a] + c[i, a]) % shape[a] for a in range(3))
        assert out[(i,) + dest] == 1.0
        assert out.sum() == 1.0


def test_stream_is_permutation_and_L_steps_are_identity():
    shape = (4, 4, 4)
    p = _params(shape)
    d = lbinputs.random_field((19,) + shape, 21)
    out = oracle.stream(p, d)
    for i in range(19):
        assert np.array_equal(np.sort(out[i].ravel()), np.sort(d[i].ravel()))
    cur = d
    for _ in range(4):
        cur = oracle.stream(p, cur)
    assert np.array_equal(cur, d)  # bit-exact round trip


# ------------------------------------------------------------ full step --

def _perturbed_state(p, seed):
    f, g = oracle.init(p, lbinputs.spinodal_phi0(p.shape, seed=seed))
    rng = np.random.default_rng(seed)
    f = f + 1e-3 * rng.standard_normal(f.shape) * oracle.lattice()[1][:, None, None, None]
    return f, g


def test_global_conservation():
    """sum rho, sum phi and total momentum are conserved to round-off."""
    p = _params((6, 7, 8), tau_f=0.8, tau_g=1.3)
    f, g = _perturbed_state(p, 4)
    s0 = oracle.sums(p, f, g)
    assert abs(s0[2]) + abs(s0[3]) + abs(s0[4]) > 1e-4  # non-trivial momentum
    f2, g2 = oracle.run(p, f, g, 40)
    s1 = oracle.sums(p, f2, g2)
    np.testing.assert_allclose(s1, s0, rtol=0, atol=1e-12)


def test_uniform_equilibrium_is_fixed_point():
    shape = (4, 5, 3)
    p = _params(shape, tau_f=0.8, tau_g=1.3)
    phib = 0.3
    mu = p.A * phib + p.B * phib ** 3
    iso = 0.5 * p.A * phib ** 2 + 0.75 * p.B * phib ** 4
    feq, geq = oracle.equilibrium_site(p, 1.0, np.zeros(3), phib, mu,
                                       np.array([iso, 0, 0, iso, 0, iso]))
    f = np.broadcast_to(feq[:, None, None, None], (19,) + shape).copy()
    g = np.broadcast_to(geq[:, None, None, None], (19,) + shape).copy()
    f2, g2 = oracle.run(p, f, g, 10)
    # a few ulp of round-off per step (sum of the 19 equilibria vs rho)
    np.testing.assert_allclose(f2, f, rtol=1e-14, atol=0)
    np.testing.assert_allclose(g2, g, rtol=1e-14, atol=1e-17)


def test_periodic_shift_invariance_bit_exact():
    shape = (5, 6, 7)
    p = _params(shape, tau_f=0.8, tau_g=1.3)
    phi0 = lbinputs.spinodal_phi0(shape, seed=3)
    f, g = oracle.run(p, *oracle.init(p, phi0), 6)
    sh = (2, -1, 3)
    fs, gs = oracle.run(p, *oracle.init(p, np.roll(phi0, sh, (0, 1, 2))), 6)
    assert np.array_equal(fs, np.roll(f, sh, (1, 2, 3)))
    assert np.array_equal(gs, np.roll(g, sh, (1, 2, 3)))


def test_cubic_symmetry_equivariance():
    """Swapping x and y, or reflecting x, maps the solution to the transformed one."""
    shape = (6, 6, 5)
    p = _params(shape, tau_f=0.8, tau_g=1.3)
    phi0 = lbinputs.spinodal_phi0(shape, seed=8)
    f, g = oracle.run(p, *oracle.init(p, phi0), 8)
    rho, u, phi = oracle.moments(p, f, g)
    # swap x <-> y
    f2, g2 = oracle.run(p, *oracle.init(p, phi0.transpose(1, 0, 2).copy()), 8)
    rho2, u2, phi2 = oracle.moments(p, f2, g2)
    np.testing.assert_allclose(phi2, phi.transpose(1, 0, 2), atol=1e-14)
    np.testing.assert_allclose(u2[0], u[1].transpose(1, 0, 2), atol=1e-15)
    np.testing.assert_allclose(u2[1], u[0].transpose(1, 0, 2), atol=1e-15)
    # reflect x -> -x (mod L)
    ref = lambda a: np.roll(a[::-1], 1, 0)  # noqa: E731  x -> (L - x) mod L
    f3, g3 = oracle.run(p, *oracle.init(p, ref(phi0).copy()), 8)
    rho3, u3, phi3 = oracle.moments(p, f3, g3)
    np.testing.assert_allclose(phi3, ref(phi), atol=1e-14)
    np.testing.assert_allclose(u3[0], -ref(u[0]), atol=1e-15)
    np.testing.assert_allclose(u3[2], ref(u[2]), atol=1e-15)
    np.testing.assert_allclose(rho3, ref(rho), atol=1e-14)


@pytest.mark.parametrize("coupling", [0, 1])
def test_two_transcriptions_agree(coupling):
    """The per-site C loops and the whole-lattice torch re-expression agree
    (stress coupling, and the body force with its own torch step)."""
    shape = (5, 6, 7)
    p = _params(shape, tau_f=0.8, tau_g=1.3, coupling=coupling)
    f, g = _perturbed_state(p, 12)
    fc, gc = oracle.run(p, f, g, 15)
    tf, tg = torch.tensor(f), torch.tensor(g)
    stepper = R.step_force if coupling else R.step
    for _ in range(15):
        tf, tg = stepper(tf, tg, p.A, p.B, p.kappa, p.gamma, p.tau_f, p.tau_g)
    np.testing.assert_allclose(tf.numpy(), fc, rtol=0, atol=1e-15)
    np.testing.assert_allclose(tg.numpy(), gc, rtol=0, atol=1e-15)


# ------------------------------------------ hydrodynamic closed forms --

@pytest.mark.parametrize("coupling", [0, 1])
def test_shear_wave_decays_with_bgk_viscosity(coupling):
    """u_y = U sin(kx) decays as exp(-nu k^2 t) with nu = (tau_f - 1/2)/3
    (phi = 0: no stress and no force, in either coupling)."""
    n = 32
    shape = (n, 3, 3)
    p = _params(shape, tau_f=0.8, tau_g=1.0, coupling=coupling)
    k = 2 * math.pi / n
    U = 1e-5
    f = np.zeros((19,) + shape)
    for x in range(n):
        feq, _ = oracle.equilibrium_site(p, 1.0, np.array([0.0, U * math.sin(k * x), 0.0]),
                                         0.0, 0.0, np.zeros(6))
        f[:, x] = feq[:, None, None]
    g = np.zeros_like(f)

    def amp(f):
        rho, u, _ = oracle.moments(p, f, g)
        return 2.0 / n * (u[1][:, 0, 0] * np.sin(k * np.arange(n))).sum()

    f1, _ = oracle.run(p, f, g, 20)
    f2, _ = oracle.run(p, f1, g, 300)
    nu_meas = -math.log(amp(f2) / amp(f1)) / (300 * k * k)
    nu = (p.tau_f - 0.5) / 3.0
    assert abs(nu_meas / nu - 1) < 5e-3, nu_meas


@pytest.mark.parametrize("coupling", [0, 1])
def test_order_parameter_relaxes_by_cahn_hilliard(coupling):
    """Small phi = eps cos(kx), A > 0: decay rate M k^2 (A + kappa k^2), M = Gamma (tau_g - 1/2);
    the flow the stress or force drives is second order in eps."""
    n = 32
    shape = (n, 3, 3)
    p = _params(shape, A=0.1, B=0.0, kappa=0.004, tau_g=1.0, gamma=0.5, coupling=coupling)
    k = 2 * math.pi / n
    phi0 = 1e-4 * np.broadcast_to(np.cos(k * np.arange(n))[:, None, None], shape).copy()
    f, g = oracle.init(p, phi0)

    def amp(g):
        phi = g.sum(0)[:, 0, 0]
        return 2.0 / n * (phi * np.cos(k * np.arange(n))).sum()

    f1, g1 = oracle.run(p, f, g, 30)
    f2, g2 = oracle.run(p, f1, g1, 400)
    rate = -math.log(amp(g2) / amp(g1)) / 400
    M = p.gamma * (p.tau_g - 0.5)
    expect = M * k * k * (p.A + p.kappa * k * k)
    assert abs(rate / expect - 1) < 0.02, (rate, expect)


# ------------------------------------------------------ force coupling --

def _smooth_field(n, k):
    x, y, z = np.meshgrid(*[np.arange(n)] * 3, indexing="ij")
    return (0.5 * np.sin(k * x) + 0.3 * np.cos(k * y + 0.4) + 0.2 * np.sin(k * z + 1.1)
            + 0.25 * np.sin(k * (x + y)) + 0.15 * np.cos(k * (y - z)))


def test_force_is_minus_phi_grad_mu_on_smooth_fields():
    """F = -div Pi equals -phi grad mu in the continuum (Gibbs-Duhem): on a
    smooth field the lattice versions agree to O(k^2); a sign, index or
    component error leaves an O(1) gap.  A uniform field has F = 0 exactly,
    and the central divergence sums to zero over the periodic lattice."""
    n = 48
    p = _params((n, n, n), A=-0.05, B=0.05, kappa=0.02, coupling=1)
    k = 2 * math.pi / n
    phi = _smooth_field(n, k)
    grad, lap = oracle.gradients(p, phi)
    mu, pi = oracle.chemical(p, phi, grad, lap)
    F = oracle.force(p, pi)

    def d(field, a):
        return 0.5 * (np.roll(field, -1, a) - np.roll(field, 1, a))

    scale = max(np.abs(phi * d(mu, a)).max() for a in range(3))
    for a in range(3):
        err = np.abs(F[a] + phi * d(mu, a)).max()
        assert err < 0.02 * scale, (a, err, scale)
    assert np.abs(F.sum(axis=(1, 2, 3))).max() < 1e-12 * np.abs(F).max() * F[0].size
    pu = np.full((6, 5, 6, 7), 0.0)
    pu[0] = pu[3] = pu[5] = 0.7
    pu[1] = 0.2
    assert np.array_equal(oracle.force(_params((5, 6, 7)), pu), np.zeros((3, 5, 6, 7)))


def test_force_equilibrium_moments_exact():
    """Force-coupling equilibria: sum f = rho, sum f c = rho u, sum f cc =
    rho/3 I + rho u u (no stress); g as in the stress coupling."""
    p = _params((3, 3, 3), coupling=1)
    c, w = oracle.lattice()
    rng = np.random.default_rng(3)
    for _ in range(5):
        rho, phi, mu = 1 + 0.1 * rng.random(), rng.uniform(-1, 1), rng.uniform(-0.1, 0.1)
        u = rng.uniform(-0.05, 0.05, 3)
        feq, geq = oracle.equilibrium_force_site(p, rho, u, phi, mu)
        np.testing.assert_allclose(feq.sum(), rho, rtol=1e-15)
        np.testing.assert_allclose(feq @ c, rho * u, rtol=0, atol=1e-16)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", feq, c, c),
                                   rho / 3 * np.eye(3) + rho * np.outer(u, u), rtol=0, atol=1e-15)
        np.testing.assert_allclose(geq.sum(), phi, rtol=1e-15, atol=1e-16)
        np.testing.assert_allclose(geq @ c, phi * u, rtol=0, atol=1e-16)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", geq, c, c),
                                   p.gamma * mu * np.eye(3) + phi * np.outer(u, u), rtol=0,
                                   atol=1e-15)


def test_force_collision_adds_exactly_the_force():
    """Per site the forcing collision keeps mass and phi and adds exactly F to
    the momentum (the half-force velocity and the (1 - 1/(2 tau)) source
    together); g's first moment relaxes towards phi u with u = (j + F/2)/rho.
    With F = 0 it is the stress-coupling collision with Pi = 0."""
    shape = (4, 5, 3)
    p = _params(shape, tau_f=0.8, tau_g=1.3, coupling=1)
    c, w = oracle.lattice()
    rng = np.random.default_rng(11)
    f, g = _perturbed_state(p, 6)
    phi = g.sum(0)
    mu = rng.uniform(-0.01, 0.01, shape)
    F = 1e-3 * rng.standard_normal((3,) + shape)
    fs, gs = oracle.collide_force(p, f, g, phi, mu, F)
    rho, j = f.sum(0), np.einsum("i...,ia->a...", f, c)
    np.testing.assert_allclose(fs.sum(0), rho, rtol=1e-14)
    np.testing.assert_allclose(np.einsum("i...,ia->a...", fs, c), j + F, rtol=0, atol=1e-15)
    np.testing.assert_allclose(gs.sum(0), phi, rtol=0, atol=1e-15)
    u = (j + 0.5 * F) / rho
    gj = np.einsum("i...,ia->a...", g, c)
    np.testing.assert_allclose(np.einsum("i...,ia->a...", gs, c),
                               (1 - 1 / p.tau_g) * gj + phi * u / p.tau_g, rtol=0, atol=1e-15)
    f0, g0 = oracle.collide_force(p, f, g, phi, mu, np.zeros_like(F))
    fr, gr = oracle.collide(p, f, g, phi, mu, np.zeros((6,) + shape))
    np.testing.assert_allclose(f0, fr, rtol=1e-14, atol=1e-17)
    np.testing.assert_allclose(g0, gr, rtol=1e-14, atol=1e-17)


def test_force_coupling_conserves_and_keeps_uniform_state():
    """sum rho, sum phi and total momentum conserved to round-off over 40
    steps (the central divergence telescopes); a uniform equilibrium (F = 0)
    is a fixed point."""
    p = _params((6, 7, 8), tau_f=0.8, tau_g=1.3, coupling=1)
    f, g = _perturbed_state(p, 4)
    s0 = oracle.sums(p, f, g)
    f2, g2 = oracle.run(p, f, g, 40)
    np.testing.assert_allclose(oracle.sums(p, f2, g2), s0, rtol=0, atol=1e-12)
    assert np.abs(f2 - f).max() > 1e-6  # the force acted
    shape = (4, 5, 3)
    pu = _params(shape, tau_f=0.8, tau_g=1.3, coupling=1)
    phib = 0.3
    mu = pu.A * phib + pu.B * phib ** 3
    feq, geq = oracle.equilibrium_force_site(pu, 1.0, np.zeros(3), phib, mu)
    f = np.broadcast_to(feq[:, None, None, None], (19,) + shape).copy()
    g = np.broadcast_to(geq[:, None, None, None], (19,) + shape).copy()
    f3, g3 = oracle.run(pu, f, g, 10)
    np.testing.assert_allclose(f3, f, rtol=1e-14, atol=0)
    np.testing.assert_allclose(g3, g, rtol=1e-14, atol=1e-17)


@pytest.mark.parametrize("coupling,tol", [(0, 2e-3), (1, 3e-2)])
def test_flat_interfaces_reach_mechanical_equilibrium(coupling, tol):
    """Two flat interfaces (width xi = 8) relax to rest, where the total
    normal stress rho/3 + Pi_xx is uniform: rho - <rho> = -3 (Pi_xx - <Pi_xx>).
    The stress coupling meets this to round-off once at rest; the force
    coupling up to the difference between its central divergence and the
    lattice's own pressure gradient (1% here, 16% at xi = 4).  A sign or
    factor error in the force or the forcing term misses by 50-200%."""
    n = 96
    shape = (n, 1, 1)
    A, B, kappa = -0.005, 0.005, 0.16
    xi = math.sqrt(-2 * kappa / A)
    x = np.arange(n)
    phi0 = (np.tanh((x - n / 4) / xi) - np.tanh((x - 3 * n / 4) / xi) - 1.0).reshape(shape)
    p = _params(shape, A=A, B=B, kappa=kappa, tau_f=1.0, tau_g=1.0, coupling=coupling)
    f, g = oracle.run(p, *oracle.init(p, phi0), 8000)
    rho, u, phi = oracle.moments(p, f, g)
    assert np.abs(u).max() < 1e-6
    grad, lap = oracle.gradients(p, phi)
    _, pi = oracle.chemical(p, phi, grad, lap)
    d = (rho - rho.mean()).ravel()
    q = (-3 * (pi[0] - pi[0].mean())).ravel()
    assert np.ptp(d) > 1e-5
    assert np.abs(d - q).max() < tol * np.ptp(d), np.abs(d - q).max() / np.ptp(d)


# ---------------------------------- finite-difference order parameter --
# The state is (f, phi); phi follows a conservative Cahn-Hilliard update with
# upwind advection (face fluxes), M = Gamma (tau_g - 1/2).

def _fd_params(shape, **kw):
    kw.setdefault("order_param", 1)
    return _params(shape, **kw)


def _lap_eig(shape, q):
    """Eigenvalue of the 7-point Laplacian for the integer wave vector q."""
    return -sum(2 * (1 - math.cos(2 * math.pi * qa / n)) for qa, n in zip(q, shape))


@pytest.mark.parametrize("coupling", [0, 1])
@pytest.mark.parametrize("q,tau_g,gamma", [((1, 2, 0), 1.3, 0.5), ((3, 1, 2), 0.8, 0.9)])
def test_fd_diffusion_is_the_discrete_linear_multiplier(q, tau_g, gamma, coupling):
    """From rest (u = 0) a small mode phi = eps cos(q.x + 0.3) changes per step
    by the factor 1 + M lam (A - kappa lam), lam the Laplacian eigenvalue:
    the flux difference of mu is the 7-point Laplacian of the linearised mu.
    The flow the stress drives is O(eps^2) (zero mean phi), so five steps
    follow the factor to the fifth power to O(eps^2) relative.  A flux sign,
    the mobility's tau_g convention or a kappa sign error is O(1) off."""
    shape = (8, 6, 10)
    p = _fd_params(shape, tau_g=tau_g, gamma=gamma, tau_f=0.9, coupling=coupling)
    x, y, z = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    arg = 2 * math.pi * (q[0] * x / shape[0] + q[1] * y / shape[1] + q[2] * z / shape[2]) + 0.3
    eps = 1e-6
    phi0 = eps * np.cos(arg)
    lam = _lap_eig(shape, q)
    M = gamma * (tau_g - 0.5)
    m = 1 + M * lam * (p.A - p.kappa * lam)
    f, phi = oracle.fd_init(p, phi0)
    _, phi1 = oracle.fd_step(p, f, phi)
    np.testing.assert_allclose(phi1, m * phi0, rtol=0, atol=1e-9 * eps)
    _, phi5 = oracle.fd_run(p, f, phi, 5)
    np.testing.assert_allclose(phi5, m ** 5 * phi0, rtol=0, atol=1e-9 * eps)
    assert abs(m - 1) > 1e-3  # the mode moved


def _first_order_state(rho, j):
    """f_i = w_i (rho + 3 c_i . j): moments exactly rho and j."""
    c, w = oracle.lattice()
    return w[:, None, None, None] * (rho[None] + 3 * np.einsum("ia,a...->i...", c, j))


def test_fd_upwind_advection_matches_fourier_multiplier():
    """A = B = kappa = 0 and M = 0 (Gamma = 0): phi is advected by a uniform
    velocity with mixed signs.  Upwind differencing along each axis is the
    linear map with the Fourier multiplier
    1 - sum_{u_a > 0} u_a (1 - e^{-i q_a}) - sum_{u_a < 0} u_a (e^{i q_a} - 1),
    applied here with numpy's FFT.  Taking the downwind side, or the wrong
    sign of a flux, breaks it."""
    shape = (9, 8, 7)
    p = _fd_params(shape, A=0.0, B=0.0, kappa=0.0, gamma=0.0)
    u0 = np.array([0.031, -0.022, 0.013])
    rho = np.full(shape, 1.0)
    f = _first_order_state(rho, np.broadcast_to(u0[:, None, None, None], (3,) + shape))
    phi = lbinputs.random_field(shape, seed=21)
    _, u, _ = oracle.fd_moments(p, f, phi)
    np.testing.assert_allclose(u, np.broadcast_to(u0[:, None, None, None], u.shape), atol=1e-16)
    _, phi1 = oracle.fd_step(p, f, phi)
    qs = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(n) for n in shape], indexing="ij")
    mult = np.ones(shape, dtype=complex)
    for a in range(3):
        ua = u0[a]
        mult -= ua * (1 - np.exp(-1j * qs[a])) if ua > 0 else ua * (np.exp(1j * qs[a]) - 1)
    expect = np.fft.ifftn(np.fft.fftn(phi) * mult).real
    np.testing.assert_allclose(phi1, expect, rtol=0, atol=1e-13)


def test_fd_face_velocity_gives_central_divergence():
    """A uniform phi = c under a non-uniform velocity (M = 0): every face
    carries c times its face velocity, so phi changes by -c times the sum of
    the face-velocity differences, which for the mean of the two sites'
    velocities is the central-difference divergence of u (numpy rolls here);
    taking one site's velocity instead gives a one-sided difference."""
    shape = (6, 5, 4)
    p = _fd_params(shape, A=0.0, B=0.0, kappa=0.0, gamma=0.0)
    rng = np.random.default_rng(5)
    rho = 1.0 + 0.05 * rng.random(shape)
    j = 0.02 * rng.standard_normal((3,) + shape)
    f = _first_order_state(rho, j)
    cval = 0.7
    _, phi1 = oracle.fd_step(p, f, np.full(shape, cval))
    u = j / rho[None]
    div = sum(0.5 * (np.roll(u[a], -1, a) - np.roll(u[a], 1, a)) for a in range(3))
    np.testing.assert_allclose(phi1, cval * (1 - div), rtol=0, atol=1e-15)


def test_fd_conserves_and_keeps_uniform_state():
    """sum rho, sum phi, total momentum conserved to round-off over 40 steps
    (fluxes telescope; Pi in f^eq); a uniform phi at rest is unchanged
    bit-for-bit (every flux is exactly zero)."""
    shape = (6, 7, 8)
    p = _fd_params(shape, tau_f=0.8, tau_g=1.3)
    f, _ = _perturbed_state(_params(shape, tau_f=0.8, tau_g=1.3), 4)
    phi = 0.1 + lbinputs.spinodal_phi0(shape, seed=8)
    s0 = oracle.fd_sums(p, f, phi)
    assert abs(s0[2]) + abs(s0[3]) + abs(s0[4]) > 1e-4
    f2, phi2 = oracle.fd_run(p, f, phi, 40)
    np.testing.assert_allclose(oracle.fd_sums(p, f2, phi2), s0, rtol=0, atol=1e-12)
    assert np.abs(phi2 - phi).max() > 1e-3
    fu, pu = oracle.fd_init(p, np.full(shape, 0.3))
    fu2, pu2 = oracle.fd_run(p, fu, pu, 10)
    assert np.array_equal(pu2, pu)
    _, u, _ = oracle.fd_moments(p, fu2, pu2)
    assert np.array_equal(u, np.zeros_like(u))


def test_fd_relaxes_like_the_lb_scheme():
    """Both order-parameter schemes (and the finite-difference one with the
    force coupling) solve the same Cahn-Hilliard equation: the decay rate of
    a small mode (A > 0) matches the continuum
    M k^2 (A + kappa k^2), M = Gamma (tau_g - 1/2), to 2% for each
    (FD 0.3%, LB 1.1% here; a mobility off by tau_g's 1/2 is 70% off)."""
    n = 32
    shape = (n, 3, 3)
    rates = []
    k = 2 * math.pi / n
    phi0 = 1e-4 * np.broadcast_to(np.cos(k * np.arange(n))[:, None, None], shape).copy()

    def amp(phi):
        return 2.0 / n * (phi[:, 0, 0] * np.cos(k * np.arange(n))).sum()

    for op, coupling in ((0, 0), (1, 0), (1, 1)):
        p = _params(shape, A=0.1, B=0.0, kappa=0.004, tau_g=1.2, gamma=0.5, order_param=op,
                    coupling=coupling)
        if op:
            f, phi = oracle.fd_run(p, *oracle.fd_init(p, phi0), 30)
            _, phi2 = oracle.fd_run(p, f, phi, 400)
        else:
            f, g = oracle.run(p, *oracle.init(p, phi0), 30)
            phi = g.sum(0)
            phi2 = oracle.run(p, f, g, 400)[1].sum(0)
        rates.append(-math.log(amp(phi2) / amp(phi)) / 400)
    expect = 0.5 * 0.7 * k * k * (0.1 + 0.004 * k * k)
    for r in rates:
        assert abs(r / expect - 1) < 0.02, (rates, expect)


def test_fd_flat_interfaces_reach_equilibrium():
    """Two flat interfaces relax to rest with uniform normal stress
    rho/3 + Pi_xx, as in the LB scheme, and keep their tanh profile."""
    n = 96
    shape = (n, 1, 1)
    A, B, kappa = -0.005, 0.005, 0.16
    xi = math.sqrt(-2 * kappa / A)
    x = np.arange(n)
    phi0 = (np.tanh((x - n / 4) / xi) - np.tanh((x - 3 * n / 4) / xi) - 1.0).reshape(shape)
    p = _fd_params(shape, A=A, B=B, kappa=kappa, tau_f=1.0, tau_g=1.0)
    f, phi = oracle.fd_run(p, *oracle.fd_init(p, phi0), 8000)
    rho, u, _ = oracle.fd_moments(p, f, phi)
    assert np.abs(u).max() < 1e-6
    grad, lap = oracle.gradients(p, phi)
    _, pi = oracle.chemical(p, phi, grad, lap)
    assert np.abs(phi - phi0).max() < 1e-2
    d = (rho - rho.mean()).ravel()
    q = (-3 * (pi[0] - pi[0].mean())).ravel()
    assert np.ptp(d) > 1e-5
    assert np.abs(d - q).max() < 2e-3 * np.ptp(d), np.abs(d - q).max() / np.ptp(d)


# -- with the force coupling (the stress divergence on the fluid) -----------

def test_fd_force_advects_with_the_half_force_velocity():
    """From rest (j = 0) with M = 0, phi's first change is advection alone by
    the velocity the forcing collision uses, u = F / (2 rho0): the same
    update as the (separately pinned) flux functions with that u.  Taking
    u = j / rho instead leaves phi unchanged."""
    shape = (9, 8, 7)
    p = _fd_params(shape, coupling=1, gamma=0.0, A=-0.05, B=0.05, kappa=0.3)
    phi0 = 0.8 * lbinputs.random_field(shape, seed=31)
    f, phi = oracle.fd_init(p, phi0)
    _, phi1 = oracle.fd_step(p, f, phi)
    grad, lap = oracle.gradients(p, phi0)
    _, pi = oracle.chemical(p, phi0, grad, lap)
    u = oracle.force(p, pi) / (2 * p.rho0)
    _, um, _ = oracle.fd_moments(p, f, phi0)
    np.testing.assert_allclose(um, u, rtol=1e-14, atol=1e-17)
    expect = oracle.fd_update(p, phi0, oracle.fd_fluxes(p, phi0, np.zeros(shape), u))
    np.testing.assert_allclose(phi1, expect, rtol=0, atol=1e-15)
    assert np.abs(phi1 - phi0).max() > 1e-6


def test_fd_force_conserves_and_keeps_uniform_state():
    """sum rho, sum phi and total momentum conserved to round-off over 40
    steps (the central divergence and the fluxes telescope); a uniform phi at
    rest stays bit-for-bit with j = 0 exactly (F = 0 exactly), f at w rho0
    to round-off."""
    shape = (6, 7, 8)
    p = _fd_params(shape, coupling=1, tau_f=0.8, tau_g=1.3)
    f, _ = _perturbed_state(_params(shape, tau_f=0.8, tau_g=1.3), 4)
    phi = 0.1 + lbinputs.spinodal_phi0(shape, seed=8, amp=0.4)
    s0 = oracle.fd_sums(p, f, phi)
    f2, phi2 = oracle.fd_run(p, f, phi, 40)
    np.testing.assert_allclose(oracle.fd_sums(p, f2, phi2), s0, rtol=0, atol=1e-12)
    assert np.abs(f2 - f).max() > 1e-6
    fu, pu = oracle.fd_init(p, np.full(shape, 0.3))
    fu2, pu2 = oracle.fd_run(p, fu, pu, 10)
    assert np.array_equal(pu2, pu)
    _, uu, _ = oracle.fd_moments(p, fu2, pu2)
    assert np.array_equal(uu, np.zeros_like(uu))
    np.testing.assert_allclose(fu2, fu, rtol=1e-15, atol=0)


@pytest.mark.parametrize("coupling,tol", [(0, 2e-3), (1, 3e-2)])
def test_fd_flat_interfaces_mechanical_equilibrium_both_couplings(coupling, tol):
    """With either coupling the finite-difference scheme's flat interfaces
    come to rest with rho/3 + Pi_xx uniform, to the tolerance the LB scheme
    meets with the same coupling."""
    n = 96
    shape = (n, 1, 1)
    A, B, kappa = -0.005, 0.005, 0.16
    xi = math.sqrt(-2 * kappa / A)
    x = np.arange(n)
    phi0 = (np.tanh((x - n / 4) / xi) - np.tanh((x - 3 * n / 4) / xi) - 1.0).reshape(shape)
    p = _fd_params(shape, A=A, B=B, kappa=kappa, tau_f=1.0, tau_g=1.0, coupling=coupling)
    f, phi = oracle.fd_run(p, *oracle.fd_init(p, phi0), 8000)
    rho, u, _ = oracle.fd_moments(p, f, phi)
    assert np.abs(u).max() < 1e-6
    grad, lap = oracle.gradients(p, phi)
    _, pi = oracle.chemical(p, phi, grad, lap)
    d = (rho - rho.mean()).ravel()
    q = (-3 * (pi[0] - pi[0].mean())).ravel()
    assert np.ptp(d) > 1e-5
    assert np.abs(d - q).max() < tol * np.ptp(d), np.abs(d - q).max() / np.ptp(d)


# ----------------------------------------------- reverse-mode gradients --

@pytest.mark.parametrize("coupling", [0, 1])
def test_reverse_mode_matches_central_differences(coupling):
    """torch autograd through the re-expressed step vs central differences of
    the C oracle's forward run (8^3, 20 steps; either coupling)."""
    shape = (8, 8, 8)
    T = 20
    p = _params(shape, tau_f=0.8, tau_g=1.3, coupling=coupling)
    phi0 = lbinputs.spinodal_phi0(shape, seed=77)
    tgt = lbinputs.lamellar_target(shape, 8, lbinputs.interface_width(p.A, p.kappa))

    def loss(phi0_, A=p.A, B=p.B, kappa=p.kappa):
        q = oracle.Params(*shape, A=A, B=B, kappa=kappa, gamma=p.gamma, tau_f=p.tau_f,
                          tau_g=p.tau_g, rho0=p.rho0, coupling=coupling)
        f, g = oracle.run(q, *oracle.init(q, phi0_), T)
        return 0.5 * ((g.sum(0) - tgt) ** 2).sum()

    L, gphi, gA, gB, gk = R.loss_and_grads(phi0, tgt, p.A, p.B, p.kappa, T, p.gamma,
                                           p.tau_f, p.tau_g, p.rho0,
                                           "force" if coupling else "stress")
    assert abs(L - loss(phi0)) < 1e-12 * abs(L)
    v = lbinputs.random_field(shape, 5)
    h = 1e-4
    fd = (loss(phi0 + h * v) - loss(phi0 - h * v)) / (2 * h)
    assert abs(fd - (gphi * v).sum()) < 1e-7 * abs(fd), (fd, (gphi * v).sum())
    # single-site component
    e = np.zeros(shape)
    e[3, 4, 5] = 1.0
    fd = (loss(phi0 + h * e) - loss(phi0 - h * e)) / (2 * h)
    assert abs(fd - gphi[3, 4, 5]) < 1e-6 * max(abs(fd), 1e-3)
    # L depends on B only through phi^3 (phi ~ 0.05), so B takes a larger step
    # to stay clear of round-off; the other two are nearly linear.
    for name, val, gv, rel in (("A", p.A, gA, 1e-4), ("B", p.B, gB, 1e-1),
                               ("kappa", p.kappa, gk, 1e-4)):
        hh = rel * abs(val)
        lp = loss(phi0, **{name: val + hh})
        lm = loss(phi0, **{name: val - hh})
        fd = (lp - lm) / (2 * hh)
        assert abs(fd - gv) < 1e-6 * abs(fd), (name, fd, gv)


@pytest.mark.parametrize("coupling", [0, 1])
def test_fd_two_transcriptions_agree(coupling):
    """The finite-difference step re-expressed with whole-lattice torch ops
    matches the C oracle's per-site loops to round-off (20 steps, tau != 1;
    either coupling)."""
    shape = (7, 6, 9)
    p = _fd_params(shape, tau_f=0.8, tau_g=1.3, coupling=coupling)
    phi0 = lbinputs.spinodal_phi0(shape, seed=5, amp=0.4)
    f, phi = oracle.fd_run(p, *oracle.fd_init(p, phi0), 20)
    ft = R.WEIGHTS[:, None, None, None] * torch.ones((19,) + shape, dtype=torch.float64)
    pt = torch.tensor(phi0)
    for _ in range(20):
        ft, pt = R.fd_step(ft, pt, p.A, p.B, p.kappa, p.gamma, p.tau_f, p.tau_g,
                           "force" if coupling else "stress")
    np.testing.assert_allclose(pt.numpy(), phi, rtol=0, atol=1e-14)
    np.testing.assert_allclose(ft.numpy(), f, rtol=0, atol=1e-15)


@pytest.mark.parametrize("coupling", [0, 1])
def test_fd_reverse_mode_matches_central_differences(coupling):
    """torch autograd through the finite-difference step vs central
    differences of the C oracle's forward run (8^3, 20 steps; either
    coupling)."""
    shape = (8, 8, 8)
    T = 20
    p = _fd_params(shape, tau_f=0.8, tau_g=1.3, coupling=coupling)
    phi0 = lbinputs.spinodal_phi0(shape, seed=77, amp=0.3)
    tgt = lbinputs.lamellar_target(shape, 8, lbinputs.interface_width(p.A, p.kappa))

    def loss(phi0_, A=p.A, B=p.B, kappa=p.kappa):
        q = oracle.Params(*shape, A=A, B=B, kappa=kappa, gamma=p.gamma, tau_f=p.tau_f,
                          tau_g=p.tau_g, rho0=p.rho0, order_param=1, coupling=coupling)
        f, phi = oracle.fd_run(q, *oracle.fd_init(q, phi0_), T)
        return 0.5 * ((phi - tgt) ** 2).sum()

    L, gphi, gA, gB, gk = R.fd_loss_and_grads(phi0, tgt, p.A, p.B, p.kappa, T, p.gamma,
                                              p.tau_f, p.tau_g, p.rho0,
                                              "force" if coupling else "stress")
    assert abs(L - loss(phi0)) < 1e-12 * abs(L)
    v = lbinputs.random_field(shape, 5)
    # with the force the face velocities are nonzero from the first step and
    # some lie within 3e-9 of zero: a step of 1e-5 flips upwind choices
    # (the scheme's kinks) and moves the difference by 3e-6, 1e-6 does not
    h, tol = (1e-6, 1e-7) if coupling else (1e-5, 1e-6)
    fd = (loss(phi0 + h * v) - loss(phi0 - h * v)) / (2 * h)
    assert abs(fd - (gphi * v).sum()) < tol * abs(fd), (fd, (gphi * v).sum())
    for name, val, gv, rel in (("A", p.A, gA, 1e-4), ("B", p.B, gB, 1e-2),
                               ("kappa", p.kappa, gk, 1e-4)):
        hh = rel * abs(val)
        fd = (loss(phi0, **{name: val + hh}) - loss(phi0, **{name: val - hh})) / (2 * hh)
        assert abs(fd - gv) < 1e-5 * abs(fd), (name, fd, gv)


def test_one_step_depends_on_radius_two():
    """One step at x depends only on the state within L-inf distance 2 of x:
    stepping a small periodic window cut around x reproduces the full-lattice
    step at x bit for bit (the full-size GPU parity tests rely on this)."""
    shape = (9, 10, 11)
    p = _params(shape, tau_f=0.8, tau_g=1.3)
    f, g = _perturbed_state(p, 31)
    g = g + 0.05 * lbinputs.random_field(g.shape, 32)
    fn, gn = oracle.step(p, f, g)
    for r in (2, 3):
        w = 2 * r + 1
        pw = _params((w, w, w), tau_f=0.8, tau_g=1.3)
        for site in [(0, 0, 0), (8, 9, 10), (4, 5, 6), (1, 9, 0)]:
            idx = [np.arange(c - r, c + r + 1) % n for c, n in zip(site, shape)]
            cut = lambda a: a[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]]  # noqa: E731
            fo, go = oracle.step(pw, cut(f), cut(g))
            assert np.array_equal(fo[:, r, r, r], fn[(slice(None),) + site])
            assert np.array_equal(go[:, r, r, r], gn[(slice(None),) + site])
    # radius 1 is not enough (the stencil of the pulled neighbours reaches 2)
    pw = _params((3, 3, 3), tau_f=0.8, tau_g=1.3)
    idx = [np.arange(c - 1, c + 2) % n for c, n in zip((4, 5, 6), shape)]
    fo, _ = oracle.step(pw, f[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]],
                        g[:, idx[0]][:, :, idx[1]][:, :, :, idx[2]])
    assert not np.array_equal(fo[:, 1, 1, 1], fn[:, 4, 5, 6])
