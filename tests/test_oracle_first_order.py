"""Pins for the oracle's first-order step (order = 1, the bootstrap option of Remark 2.2).

The paper cites the first-order convex-splitting step without writing it; the
reading (oracle/scheme.py) is: phi_* := phi^m, chi(phi) = phi^3 implicit, the
whole eps^2 Lap phi implicit, f_mu = -phi^m.  What fixes it independently of
the oracle's code:

* linear amplification of one cosine mode of the cell-centred Neumann grid
  (an exact eigenvector of the discrete Laplacian, eigenvalue -lam_k) about a
  constant state phibar: linearising the step gives the closed form
      g1 = (1 + s lam_k) / (1 + s lam_k (3 phibar^2 + eps^2 lam_k))
  and the second-order step with phi^{-1} := phi^0 the different
      g2 = (1 + s lam_k - s lam_k (3/2 phibar^2 + 1/4 eps^2 lam_k))
           / (1 + s lam_k (3/2 phibar^2 + 3/4 eps^2 lam_k)).
  About a constant state a = phibar and M = 1 + gamma phibar^2, and the p row
  gives p = -gamma phibar mu + const, so the flow terms cancel exactly and g1,
  g2 hold for every gamma (a wrong sign in either flow term breaks that);
* mass conservation and the convex-splitting energy inequality
  E_h(phi^1) + s ||grad mu||^2 + (s/gamma) ||u||^2 <= E_h(phi^0);
* gamma = 0: no flow, p = 0.
"""
import numpy as np
import pytest

from oracle import fas, grid, scheme
from workloads import cosine_mode, uniform_field


def _lam(k, n, h):
    """Eigenvalue (sign flipped) of the cell-centred Neumann 3-point Laplacian for
    the mode cos(pi k (i + 1/2) / n)."""
    return (2.0 - 2.0 * np.cos(np.pi * k / n)) / (h * h)


def _amplitude(phi, mode, mean):
    """Ratio of the mode amplitude of phi to that of ``mode`` (projection)."""
    d = (phi - mean).ravel()
    v = (mode - mean).ravel()
    return float(d @ v / (v @ v))


def _g1(s, lam, phibar, eps):
    return (1.0 + s * lam) / (1.0 + s * lam * (3.0 * phibar ** 2 + eps ** 2 * lam))


def _g2(s, lam, phibar, eps):
    num = 1.0 + s * lam - s * lam * (1.5 * phibar ** 2 + 0.25 * eps ** 2 * lam)
    return num / (1.0 + s * lam * (1.5 * phibar ** 2 + 0.75 * eps ** 2 * lam))


@pytest.mark.parametrize("gamma", [0.0, 2.0])
@pytest.mark.parametrize("order", [1, 2])
def test_single_mode_amplification_matches_the_linearisation(order, gamma):
    n, k, phibar, delta, eps, s = 32, 3, 0.3, 1e-3, 0.05, 0.01
    h = 1.0 / n
    prm = scheme.Params(eps=eps, gamma=gamma, s=s, h=h, order=order)
    phi0 = cosine_mode((n, n), k, phibar, delta)
    z = np.zeros((n, n))
    r = fas.solve_step(phi0, phi0, z, z, prm, fas.Opts(tol=1e-13))
    g = _amplitude(r.phi, phi0, phibar)
    lam = _lam(k, n, h)
    want = _g1(s, lam, phibar, eps) if order == 1 else _g2(s, lam, phibar, eps)
    other = _g2(s, lam, phibar, eps) if order == 1 else _g1(s, lam, phibar, eps)
    # nonlinear terms enter the projection at O(delta^2)
    assert abs(g - want) <= 1e-5 * want, (g, want)
    assert abs(other - want) > 1e-2 * want          # the pin tells the two steps apart


def test_first_order_step_conserves_mass_and_decreases_energy():
    n = 32
    prm = scheme.Params(eps=0.05, gamma=2.0, s=0.01, h=1.0 / n, order=1)
    phi0 = uniform_field((n, n), 4100, mean=0.1, amp=0.5)
    z = np.zeros((n, n))
    r = fas.solve_step(phi0, phi0, z, z, prm, fas.Opts(tol=1e-12))
    h2 = prm.h ** 2
    assert abs(h2 * (r.phi.sum() - phi0.sum())) <= 1e-12
    d_mu, d_u = scheme.dissipation(r.mu, r.p, phi0, prm)
    e0, e1 = scheme.energy_E(phi0, prm), scheme.energy_E(r.phi, prm)
    assert e1 + d_mu + d_u <= e0
    assert e0 - e1 > 1e-3 * abs(e0)                 # a strong quench: a real decrease


def test_first_order_step_without_flow_keeps_p_zero():
    n = 16
    prm = scheme.Params(eps=0.08, gamma=0.0, s=0.01, h=1.0 / n, order=1)
    phi0 = uniform_field((n, n), 4110, amp=0.4)
    z = np.zeros((n, n))
    r = fas.solve_step(phi0, phi0, z, z, prm, fas.Opts(tol=1e-12))
    assert np.max(np.abs(r.p)) <= 1e-12


def test_first_order_residual_is_the_written_rows():
    """The oracle's N for order 1 against the rows written out directly."""
    n = 8
    prm = scheme.Params(eps=0.1, gamma=1.5, s=0.05, h=1.0 / n, order=1)
    phi0 = uniform_field((n, n), 4120, amp=0.5)
    u = [uniform_field((n, n), 4121 + c, amp=0.3) for c in range(3)]
    phi_star, f = scheme.step_rhs(uniform_field((n, n), 4130), phi0, prm)
    assert np.array_equal(phi_star, phi0)
    lvl = scheme.Level(h=prm.h, phi_star=phi_star, psi=phi0, f=f)
    n_phi, n_mu, n_p = scheme.apply_N(u, lvl, prm)
    phi, mu, p = u
    a = grid.avg(phi0)
    m = [1.0 + prm.gamma * af * af for af in a]
    want_mu = mu - phi ** 3 + prm.eps ** 2 * grid.lap(phi, prm.h)
    np.testing.assert_allclose(n_mu, want_mu, rtol=0, atol=1e-12)
    np.testing.assert_allclose(f[1], -phi0, rtol=0, atol=0)
    want_phi = phi - prm.s * grid.div_c_grad(m, mu, prm.h) - prm.s * grid.div_c_grad(a, p, prm.h)
    np.testing.assert_allclose(n_phi, want_phi, rtol=0, atol=1e-12)
    want_p = prm.s * grid.lap(p, prm.h) + prm.s * prm.gamma * grid.div_c_grad(a, mu, prm.h)
    np.testing.assert_allclose(n_p, want_p, rtol=0, atol=1e-12)


def test_planted_first_order_error_is_caught(monkeypatch):
    """Keep the second-order 3/4 share of eps^2 Lap phi in the first-order step:
    the amplification pin fails."""
    n, k, phibar, delta, eps, s = 32, 3, 0.3, 1e-3, 0.05, 0.01
    h = 1.0 / n
    prm = scheme.Params(eps=eps, gamma=0.0, s=s, h=h, order=1)
    orig = scheme.nonlinearity
    monkeypatch.setattr(scheme, "nonlinearity",
                        lambda p: orig(p)[:2] + (0.75,) if p.order == 1 else orig(p))
    phi0 = cosine_mode((n, n), k, phibar, delta)
    z = np.zeros((n, n))
    r = fas.solve_step(phi0, phi0, z, z, prm, fas.Opts(tol=1e-13))
    g = _amplitude(r.phi, phi0, phibar)
    want = _g1(s, _lam(k, n, h), phibar, eps)
    assert abs(g - want) > 1e-3 * want
