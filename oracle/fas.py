"""Red-black full-approximation-scheme (FAS) V-cycles for one time step.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 5 names the solver (FAS nonlinear multigrid), fixes nu1 = nu2 = 2
smoothing steps, a 2x2 coarsest grid (printed as "finest", read as coarsest) and
tol = 1e-10, and omits everything else.  The reading written out here:

* Hierarchy: cell-centred grids N, N/2, ... halving every direction while all
  extents stay even and at least 2 (2^d cells at the bottom for N a power of 2).
  Each coarse level holds the cell average of the finer level's phi_* and phi^m
  and rediscretises N with spacing 2h (same s, eps, gamma).
* Smoothing step: a red-black collective update of all three unknowns,
  red cells ((i + j [+ k]) even, 0-based) then black cells.  At a cell every
  neighbour is frozen, chi(phi, psi) is replaced by its tangent at the current
  phi (one local Newton step) and the three local equations of (2.5)-(2.7) are
  solved exactly (``smooth_cell``).  Boundary faces carry no flux and are left
  out of the local diagonal.  Updating p in the same cell solve as (phi, mu)
  matters: relaxing (phi, mu) with p frozen and p afterwards (two block
  sweeps) stalls and then diverges once gamma (A_h phi_*)^2 is O(1), because
  the gamma a^2 part of M and the a grad p flux nearly cancel in the true
  operator but not in the lagged one.
* Transfers: restriction = average of the 2^d children; prolongation =
  piecewise-constant injection of the coarse correction (``Opts.prolong =
  "bilinear"``: cell-centred bi/trilinear interpolation of the correction,
  weights 3/4 and 1/4 along each axis, the coarse correction continued evenly
  across the boundary as the Neumann ghost cells of App. A.1 continue a field).
* Sweeps per level: nu1, nu2 on the finest level; ``Opts.nu1_coarse`` /
  ``nu2_coarse`` (0: the same) on the coarser levels above the coarsest.
* FAS coarse problem: u_c = R u, f_c = R(f - N(u)) + N_c(u_c); after the coarse
  solve u += P(u_c_new - u_c).
* Coarsest level: a fixed number of smoothing steps (default 4; 2 to 50 give
  identical V-cycle counts on every workload tried).
* Outer loop: V(nu1, nu2) cycles until the residual norm of the full system is
  <= tol, p normalised to mean zero after every cycle.  No cycle is run when the
  initial guess already meets tol.

These choices set the iteration count only; the converged result is the unique
solution of (2.5)-(2.7) (Theorem 2.1), which ``oracle.newton`` computes directly.
"""
from dataclasses import dataclass

import numpy as np

from . import grid
from .scheme import (Level, apply_N, face_coefficients, nonlinearity, normalise_p,
                     residual, residual_norm, step_rhs)


@dataclass
class Opts:
    nu1: int = 2
    nu2: int = 2
    tol: float = 1e-10
    max_vcycles: int = 100
    coarse_sweeps: int = 4
    nu1_coarse: int = 0          # 0: nu1 on every level
    nu2_coarse: int = 0          # 0: nu2 on every level
    prolong: str = "constant"    # or "bilinear"

    def sweeps(self, l):
        """(pre, post) smoothing steps on level l (l = 0 the finest)."""
        if l == 0:
            return self.nu1, self.nu2
        return self.nu1_coarse or self.nu1, self.nu2_coarse or self.nu2


def color_mask(shape, color):
    """Boolean mask of red (color 0: index sum even) or black (color 1) cells."""
    idx = np.indices(shape).sum(axis=0)
    return (idx % 2) == color


def face_sums(c, v):
    """Per cell: (sum_f c_f, sum_f c_f v_nb(f)) over the cell's interior faces.

    ``c`` is a list over axes of interior-face arrays; the boundary faces of a
    cell are absent (zero coefficient), which is the zero-flux condition.
    """
    csum = np.zeros_like(v)
    cv = np.zeros_like(v)
    for ax, cf in enumerate(c):
        n = v.shape[ax]
        pad_hi = [(0, 0)] * v.ndim
        pad_hi[ax] = (0, 1)
        pad_lo = [(0, 0)] * v.ndim
        pad_lo[ax] = (1, 0)
        c_plus = np.pad(cf, pad_hi)      # face i+1/2 of cell i (0 for the last cell)
        c_minus = np.pad(cf, pad_lo)     # face i-1/2 of cell i (0 for the first cell)
        v_plus = np.take(v, np.minimum(np.arange(n) + 1, n - 1), axis=ax)
        v_minus = np.take(v, np.maximum(np.arange(n) - 1, 0), axis=ax)
        csum += c_plus + c_minus
        cv += c_plus * v_plus + c_minus * v_minus
    return csum, cv


def smooth_cell(u, lvl, prm, color):
    """Collective update of (phi, mu, p) on one color: the local form of (2.5)-(2.7).

    At a cell, with every neighbour frozen, lam = s/h^2, kap = 3/4 eps^2/h^2,
    nF = number of interior faces of the cell, and for the face coefficients
    a_f = A_h phi_*, M_f = 1 + gamma a_f^2 the sums SM = sum M_f, Sa = sum a_f,
    Sa2 = sum a_f^2 over those faces, the three equations read

        phi + lam SM mu + lam Sa p             = b1 = f_phi + lam sum M_f mu_nb + lam sum a_f p_nb
        -(chi'(phi~) + kap nF) phi + mu        = b2 = f_mu + chi(phi~) - chi'(phi~) phi~ - kap sum phi_nb
        -lam gamma Sa mu - lam nF p            = b3 = f_p - lam sum p_nb - lam gamma sum a_f mu_nb

    where chi is replaced by its tangent at the current value phi~ (one local
    Newton step).  Eliminating p with the third row leaves a 2x2 system with
    off-diagonal lam * (nF + gamma (Sa2 - Sa^2 / nF)) >= lam nF (Cauchy-Schwarz)
    and determinant 1 + (that) * (chi' + kap nF) >= 1, because chi' >= 0.
    """
    phi, mu, p = u
    f_phi, f_mu, f_p = lvl.f
    h = lvl.h
    g = prm.gamma
    lam = prm.s / (h * h)
    chi_fn, dchi_fn, c_eps = nonlinearity(prm)
    kap = c_eps * prm.eps ** 2 / (h * h)
    a, m = face_coefficients(lvl.phi_star, g)
    ones = [np.ones_like(af) for af in a]
    _, s_mmu = face_sums(m, mu)
    nf, s_phi = face_sums(ones, phi)
    _, s_p = face_sums(ones, p)
    sa, s_ap = face_sums(a, p)
    _, s_amu = face_sums(a, mu)
    sa2, _ = face_sums([af * af for af in a], mu)
    b1 = f_phi + lam * s_mmu + lam * s_ap
    dc = dchi_fn(phi, lvl.psi)
    b2 = f_mu + chi_fn(phi, lvl.psi) - dc * phi - kap * s_phi
    b3 = f_p - lam * s_p - lam * g * s_amu
    # eliminate p:  p = -(b3 + lam gamma Sa mu) / (lam nF)
    a_red = lam * (nf + g * (sa2 - sa * sa / nf))
    b1_red = b1 + (sa / nf) * b3
    b = dc + kap * nf
    det = 1.0 + a_red * b
    phi_new = (b1_red - a_red * b2) / det
    mu_new = (b2 + b * b1_red) / det
    p_new = -(b3 + lam * g * sa * mu_new) / (lam * nf)
    mask = color_mask(phi.shape, color)
    phi[mask] = phi_new[mask]
    mu[mask] = mu_new[mask]
    p[mask] = p_new[mask]


def sweep(u, lvl, prm):
    """One smoothing step: collective cell update on red cells, then on black cells."""
    smooth_cell(u, lvl, prm, 0)
    smooth_cell(u, lvl, prm, 1)


def restrict(v):
    """Cell average of the 2^d children of every coarse cell."""
    out = v
    for ax in range(v.ndim):
        n = out.shape[ax]
        even = np.take(out, np.arange(0, n, 2), axis=ax)
        odd = np.take(out, np.arange(1, n, 2), axis=ax)
        out = 0.5 * (even + odd)
    return out


def prolong(v):
    """Piecewise-constant injection: every child takes its parent's value."""
    out = v
    for ax in range(v.ndim):
        out = np.repeat(out, 2, axis=ax)
    return out


def prolong_bilinear(v):
    """Cell-centred linear interpolation along every axis in turn: fine cell 2i
    takes 3/4 of coarse cell i and 1/4 of cell i - 1, fine cell 2i + 1 3/4 of
    cell i and 1/4 of cell i + 1; beyond the boundary the coarse cell itself
    (even continuation)."""
    out = v
    for ax in range(v.ndim):
        n = out.shape[ax]
        lo = np.take(out, np.maximum(np.arange(n) - 1, 0), axis=ax)
        hi = np.take(out, np.minimum(np.arange(n) + 1, n - 1), axis=ax)
        even = 0.75 * out + 0.25 * lo
        odd = 0.75 * out + 0.25 * hi
        shape = list(out.shape)
        shape[ax] = 2 * n
        new = np.empty(shape)
        idx_even = [slice(None)] * out.ndim
        idx_odd = [slice(None)] * out.ndim
        idx_even[ax] = slice(0, 2 * n, 2)
        idx_odd[ax] = slice(1, 2 * n, 2)
        new[tuple(idx_even)] = even
        new[tuple(idx_odd)] = odd
        out = new
    return out


def coarsenable(shape):
    return all(n % 2 == 0 and n // 2 >= 2 for n in shape)


def build_levels(phi_star, psi, f, h):
    """Level hierarchy with cell-averaged phi_* and phi^m on every coarse level."""
    levels = [Level(h=h, phi_star=phi_star, psi=psi, f=f)]
    while coarsenable(levels[-1].phi_star.shape):
        c = levels[-1]
        levels.append(Level(h=2.0 * c.h, phi_star=restrict(c.phi_star), psi=restrict(c.psi)))
    return levels


def vcycle(levels, us, l, prm, opts):
    """One FAS V(nu1, nu2) cycle on level l; ``us[l]`` is updated in place."""
    lvl, u = levels[l], us[l]
    if l == len(levels) - 1:
        for _ in range(opts.coarse_sweeps):
            sweep(u, lvl, prm)
        return
    nu1, nu2 = opts.sweeps(l)
    for _ in range(nu1):
        sweep(u, lvl, prm)
    r = residual(u, lvl.f, lvl, prm)
    c = levels[l + 1]
    uc = [restrict(x) for x in u]
    ubar = [x.copy() for x in uc]
    nc = apply_N(uc, c, prm)
    c.f = [restrict(r[k]) + nc[k] for k in range(3)]
    us[l + 1] = uc
    vcycle(levels, us, l + 1, prm, opts)
    interp = prolong_bilinear if opts.prolong == "bilinear" else prolong
    for k in range(3):
        u[k] += interp(us[l + 1][k] - ubar[k])
    for _ in range(nu2):
        sweep(u, lvl, prm)


@dataclass
class StepResult:
    phi: np.ndarray
    mu: np.ndarray
    p: np.ndarray
    vcycles: int
    res_history: list


def solve_step(phi_prev, phi_cur, mu0, p0, prm, opts=None):
    """One time step of (2.5)-(2.7) by FAS; returns phi^{m+1}, mu^{m+1/2}, p^{m+1/2}.

    Initial guess (phi^m, mu0, p0) -- the previous step's mu and p.
    """
    opts = opts or Opts()
    phi_star, f = step_rhs(phi_prev, phi_cur, prm)
    levels = build_levels(phi_star, phi_cur.copy(), f, prm.h)
    u = [phi_cur.copy(), mu0.copy(), normalise_p(p0)]
    us = [None] * len(levels)
    us[0] = u
    hist = [residual_norm(residual(u, f, levels[0], prm), prm.h)]
    cycles = 0
    while hist[-1] > opts.tol and cycles < opts.max_vcycles:
        vcycle(levels, us, 0, prm, opts)
        u[2] -= np.mean(u[2])
        cycles += 1
        hist.append(residual_norm(residual(u, f, levels[0], prm), prm.h))
    return StepResult(u[0], u[1], u[2], cycles, hist)


def run(phi0, prm, nsteps, opts=None, callback=None):
    """March ``nsteps`` steps from phi^0 with phi^{-1} := phi^0 (Remark 2.2).

    Returns the list of StepResult; ``callback(m, phi_prev, phi_cur, res)`` is
    called after every step.
    """
    phi_prev = phi0.copy()
    phi_cur = phi0.copy()
    mu = np.zeros_like(phi0)
    p = np.zeros_like(phi0)
    out = []
    for m in range(nsteps):
        res = solve_step(phi_prev, phi_cur, mu, p, prm, opts)
        if callback is not None:
            callback(m, phi_prev, phi_cur, res)
        out.append(res)
        phi_prev, phi_cur = phi_cur, res.phi
        mu, p = res.mu, res.p
    return out
