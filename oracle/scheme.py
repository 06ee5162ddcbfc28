"""The second-order convex-splitting scheme as one nonlinear system per step.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Given (phi^{m-1}, phi^m) the step finds u = (phi, mu, p) := (phi^{m+1},
mu^{m+1/2}, p^{m+1/2}) solving the rewritten scheme (2.5)-(2.7) with the
extrapolation and nonlinearity of (2.4):

    phi_* = 3/2 phi^m - 1/2 phi^{m-1},     a = A_h phi_*,   M = 1 + gamma a^2
    chi(phi, psi) = 1/4 (phi^2 + psi^2)(phi + psi)

    N_phi(u) = phi - s div(M grad mu) - s div(a grad p)          = phi^m
    N_mu(u)  = mu - chi(phi, phi^m) + 3/4 eps^2 Lap phi          = -phi_* - 1/4 eps^2 Lap phi^{m-1}
    N_p(u)   = s Lap p + s gamma div(a grad mu)                   = 0

Readings of points the paper leaves open:
* The pressure equation (2.7) enters the residual multiplied by s, so all three
  components have an O(1)-scaled roundoff floor; the residual norm is the
  h^d-weighted l2 norm of App. A.2 summed over the three components.
* p is defined up to an additive constant (Neumann Poisson problem); results are
  normalised to mean zero.
* The first step uses phi^{-1} := phi^0 (one of the options of Remark 2.2).
* ``order = 1`` (``Params.order``) is the other option of Remark 2.2, a
  first-order convex-splitting step from phi^0 to phi^1.  The paper cites its
  form without writing it; the reading here keeps the three rows and the face
  coefficients above and makes the splitting first order: phi_* := phi^m, the
  convex part of the double well implicit, chi(phi) = phi^3, the whole
  eps^2 Lap phi implicit and the concave part explicit, f_mu = -phi^m:

    N_mu(u) = mu - phi^3 + eps^2 Lap phi = -phi^m.

The same operator N is used on every multigrid level; a ``Level`` carries that
level's spacing and its copies of phi_* and phi^m (the frozen data).
"""
from dataclasses import dataclass, field

import numpy as np

from . import grid


@dataclass
class Params:
    """Physical and time-step parameters: eps, gamma of (1.2)-(1.4), step s, spacing h;
    order 2 = the scheme (2.4)-(2.7), order 1 = the first-order step (module doc)."""
    eps: float
    gamma: float
    s: float
    h: float
    order: int = 2


@dataclass
class Level:
    """Frozen per-step data of one grid level: spacing, phi_* and phi^m there."""
    h: float
    phi_star: np.ndarray
    psi: np.ndarray          # phi^m (second argument of chi)
    f: list = field(default=None)   # right-hand side [f_phi, f_mu, f_p]


def chi(phi, psi):
    """chi(phi, psi) = 1/4 (phi^2 + psi^2)(phi + psi), eq. (2.4)."""
    return 0.25 * (phi * phi + psi * psi) * (phi + psi)


def dchi(phi, psi):
    """d chi / d phi = 1/4 (3 phi^2 + 2 phi psi + psi^2) >= 0 (derivative of (2.4))."""
    return 0.25 * (3.0 * phi * phi + 2.0 * phi * psi + psi * psi)


def chi_cubic(phi, psi=None):
    """The implicit convex part of the double well in the first-order step: phi^3."""
    return phi * phi * phi


def dchi_cubic(phi, psi=None):
    """d/d phi of phi^3."""
    return 3.0 * phi * phi


def nonlinearity(prm):
    """(chi, dchi, c) of the step: the nonlinear term of the mu row, its phi
    derivative, and the implicit share c of eps^2 Lap phi (3/4 for (2.4)-(2.6),
    1 for the first-order step)."""
    if prm.order == 1:
        return chi_cubic, dchi_cubic, 1.0
    return chi, dchi, 0.75


def face_coefficients(phi_star, gamma):
    """a = A_h phi_* and M(a) = 1 + gamma a^2 on interior faces (text after (2.5)-(2.7))."""
    a = grid.avg(phi_star)
    m = [1.0 + gamma * af * af for af in a]
    return a, m


def step_rhs(phi_prev, phi_cur, prm):
    """Frozen data and right-hand side of one step, from (2.4) and (2.5)-(2.7).

    Returns (phi_star, f) with f = [phi^m, -phi_* - eps^2/4 Lap phi^{m-1}, 0];
    for the first-order step phi_* = phi^m and f = [phi^m, -phi^m, 0]
    (phi_prev unused).
    """
    if prm.order == 1:
        return phi_cur.copy(), [phi_cur.copy(), -phi_cur, np.zeros_like(phi_cur)]
    phi_star = 1.5 * phi_cur - 0.5 * phi_prev
    f_mu = -phi_star - 0.25 * prm.eps ** 2 * grid.lap(phi_prev, prm.h)
    return phi_star, [phi_cur.copy(), f_mu, np.zeros_like(phi_cur)]


def apply_N(u, lvl, prm):
    """N(u) of (2.5)-(2.7) on one level (third row multiplied by s, see module doc)."""
    phi, mu, p = u
    h, s, g, e2 = lvl.h, prm.s, prm.gamma, prm.eps ** 2
    a, m = face_coefficients(lvl.phi_star, g)
    chi_fn, _, c_eps = nonlinearity(prm)
    n_phi = phi - s * grid.div_c_grad(m, mu, h) - s * grid.div_c_grad(a, p, h)
    n_mu = mu - chi_fn(phi, lvl.psi) + c_eps * e2 * grid.lap(phi, h)
    n_p = s * grid.lap(p, h) + s * g * grid.div_c_grad(a, mu, h)
    return [n_phi, n_mu, n_p]


def residual(u, f, lvl, prm):
    """R = f - N(u), component-wise."""
    n = apply_N(u, lvl, prm)
    return [f[k] - n[k] for k in range(3)]


def residual_norm(r, h):
    """(||R_phi||^2 + ||R_mu||^2 + ||R_p||^2)^(1/2) with the l2 norm of App. A.2."""
    return float(np.sqrt(sum(grid.ip(rk, rk, h) for rk in r)))


def energy_E(phi, prm):
    """E_h(phi) = 1/4 ||phi||_4^4 - 1/2 ||phi||_2^2 + eps^2/2 ||grad_h phi||_2^2, eq. (2.8)."""
    h = prm.h
    return (0.25 * grid.norm4_4(phi, h) - 0.5 * grid.ip(phi, phi, h)
            + 0.5 * prm.eps ** 2 * grid.grad_norm2_sq(phi, h))


def energy_F(phi, psi, prm):
    """F_h(phi, psi) = E_h(phi) + 1/4 ||phi - psi||^2 + 1/8 eps^2 ||grad_h(phi - psi)||^2, eq. (2.9)."""
    d = phi - psi
    return (energy_E(phi, prm) + 0.25 * grid.ip(d, d, prm.h)
            + 0.125 * prm.eps ** 2 * grid.grad_norm2_sq(d, prm.h))


def velocity(mu, p, phi_star, prm):
    """u = -grad_h p - gamma A_h phi_* grad_h mu on interior faces, eq. (2.3)."""
    h = prm.h
    a = grid.avg(phi_star)
    gp, gm = grid.grad(p, h), grid.grad(mu, h)
    return [-gp[ax] - prm.gamma * a[ax] * gm[ax] for ax in range(len(gp))]


def dissipation(mu, p, phi_star, prm):
    """The two dissipation terms of Theorem 2.1: s ||grad_h mu||^2 and (s/gamma) ||u||^2.

    For gamma = 0 the velocity vanishes identically and the second term is 0.
    """
    h = prm.h
    d_mu = prm.s * grid.grad_norm2_sq(mu, h)
    if prm.gamma == 0.0:
        return d_mu, 0.0
    vel = velocity(mu, p, phi_star, prm)
    return d_mu, prm.s / prm.gamma * grid.face_ip(vel, vel, h)


def energy_identity_terms(phi_next, phi_cur, phi_prev, mu, p, prm):
    """Both sides of the exact per-step energy balance behind Theorem 2.1.

    Keeping the remainders that the two Cauchy inequalities of the proof drop
    (the bounds on I_2 and I_{3,2}) turns (energy-est-15) into an equality:

      F_h(phi^{m+1}, phi^m) - F_h(phi^m, phi^{m-1})
        = - s ||grad mu||^2 - (s/gamma) ||u||^2
          - 1/4 ||phi^{m+1} - 2 phi^m + phi^{m-1}||^2
          - eps^2/8 ||grad(phi^{m+1} - 2 phi^m + phi^{m-1})||^2 .

    Returns (lhs, rhs).
    """
    h = prm.h
    phi_star = 1.5 * phi_cur - 0.5 * phi_prev
    lhs = energy_F(phi_next, phi_cur, prm) - energy_F(phi_cur, phi_prev, prm)
    d_mu, d_u = dissipation(mu, p, phi_star, prm)
    dd = phi_next - 2.0 * phi_cur + phi_prev
    rhs = (-d_mu - d_u - 0.25 * grid.ip(dd, dd, h)
           - 0.125 * prm.eps ** 2 * grid.grad_norm2_sq(dd, h))
    return lhs, rhs


def normalise_p(p):
    """Fix the additive constant of p: subtract its mean."""
    return p - np.mean(p)
