"""Pins for the oracle's per-step solutions (Newton by definition, FAS by the Section 5 reading).

* brute force: FAS agrees with Newton's method on the index-form system (tiny grids)
* the exact energy balance behind Theorem 2.1 and unconditional decay of F_h
* mass conservation, exactly as -(R_phi, 1)
* linear single-mode recurrence about phi = 0, constant fixed point, symmetries
* second-order Cauchy convergence under s ~ h (Theorem 4.6 / Table 1)
* planted mistakes in the oracle are caught by these pins
"""
import numpy as np
import pytest

from oracle import fas, grid, newton, scheme
from workloads import smooth_ic_2d, uniform_field


def _pair(shape, seed, amp=0.3, mean=0.0):
    a = uniform_field(shape, seed, mean=mean, amp=amp)
    b = a + uniform_field(shape, seed + 1, amp=0.05)
    return a, b


def test_newton_jacobian_matches_finite_differences():
    shape = (4, 5)
    prev, cur = _pair(shape, 10)
    sysm = newton.System(prev, cur, eps=0.1, gamma=2.0, s=0.3, h=0.25)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(3 * sysm.n)
    v = rng.standard_normal(3 * sysm.n)
    d = 1e-6
    fd = (sysm.apply(x + d * v) - sysm.apply(x - d * v)) / (2 * d)
    np.testing.assert_allclose(sysm.jacobian(x) @ v, fd, rtol=1e-7, atol=1e-7)


@pytest.mark.parametrize("shape", [(8, 8), (4, 4, 4), (8, 4)])
@pytest.mark.parametrize("s", [1e-3, 1.0, 10.0])
def test_fas_matches_newton_on_tiny_grids(shape, s):
    prev, cur = _pair(shape, 20 + len(shape))
    h = 1.0 / shape[-1]
    prm = scheme.Params(eps=0.1, gamma=2.0, s=s, h=h)
    z = np.zeros(shape)
    r = fas.solve_step(prev, cur, z, z, prm, fas.Opts(tol=1e-13, max_vcycles=200))
    phi, mu, p, hist = newton.solve(prev, cur, 0.1, 2.0, s, h)
    assert hist[-1] < 1e-13
    assert np.max(np.abs(r.phi - phi)) < 1e-12
    assert np.max(np.abs(r.mu - mu)) < 1e-12
    assert np.max(np.abs((r.p - r.p.mean()) - p)) < 1e-10


@pytest.mark.parametrize("dim,n,ks", [(2, 16, (2, 3)), (3, 8, (1, 2, 3))])
def test_linear_single_mode_recurrence(dim, n, ks):
    """About phi = 0 the scheme is linear up to O(delta^3) terms (chi is cubic, the
    flow terms are cubic as p = O(delta^2)).  With -lam the Neumann eigenvalue of the
    mode: (1 + 3/4 s eps^2 lam^2) A^{m+1} = (1 + 3/2 s lam) A^m - (1/2 s lam + 1/4 s eps^2 lam^2) A^{m-1}."""
    h = 1.0 / n
    eps, gamma, s, delta = 0.05, 2.0, 2e-3, 1e-3
    vecs = [np.cos(k * np.pi * (np.arange(1, n + 1) - 0.5) / n) for k in ks]
    mode = vecs[0]
    for v in vecs[1:]:
        mode = np.multiply.outer(mode, v)
    lam = sum(4.0 / h ** 2 * np.sin(k * np.pi / (2 * n)) ** 2 for k in ks)
    a_prev, a_cur = 1.0, 0.9
    phi, mu, p, hist = newton.solve(delta * a_prev * mode, delta * a_cur * mode, eps, gamma, s, h)
    a_next = ((1 + 1.5 * s * lam) * a_cur - (0.5 * s * lam + 0.25 * s * eps ** 2 * lam ** 2) * a_prev) \
        / (1 + 0.75 * s * eps ** 2 * lam ** 2)
    err = np.max(np.abs(phi - delta * a_next * mode)) / (delta * abs(a_next))
    assert err < 1e-4
    assert np.max(np.abs(p)) < 10 * delta ** 2


@pytest.mark.parametrize("solver", ["newton", "fas"])
def test_constant_state_is_a_fixed_point(solver):
    """phi^{m-1} = phi^m = c gives phi^{m+1} = c, mu = c^3 - c, p constant (algebra of (2.4)-(2.7))."""
    c = 0.35
    shape = (8, 8)
    prev = np.full(shape, c)
    if solver == "newton":
        phi, mu, p, _ = newton.solve(prev, prev, 0.1, 1.5, 0.01, 1.0 / 8)
    else:
        prm = scheme.Params(eps=0.1, gamma=1.5, s=0.01, h=1.0 / 8)
        r = fas.solve_step(prev, prev, np.zeros(shape), np.zeros(shape), prm, fas.Opts(tol=1e-13))
        phi, mu, p = r.phi, r.mu, r.p
    np.testing.assert_allclose(phi, c, rtol=0, atol=1e-13)
    np.testing.assert_allclose(mu, c ** 3 - c, rtol=0, atol=1e-13)
    assert np.ptp(p) < 1e-12


def _fas_step(prev, cur, prm, tol=1e-13):
    z = np.zeros_like(cur)
    return fas.solve_step(prev, cur, z, z, prm, fas.Opts(tol=tol, max_vcycles=200))


def test_sign_symmetry():
    """(phi^{m-1}, phi^m) -> (-phi^{m-1}, -phi^m) maps (phi, mu, p) -> (-phi, -mu, p)."""
    prev, cur = _pair((16, 16), 30)
    prm = scheme.Params(eps=0.08, gamma=3.0, s=0.01, h=1.0 / 16)
    a = _fas_step(prev, cur, prm)
    b = _fas_step(-prev, -cur, prm)
    assert np.max(np.abs(a.phi + b.phi)) < 1e-12
    assert np.max(np.abs(a.mu + b.mu)) < 1e-12
    assert np.max(np.abs(a.p - b.p)) < 1e-11


def test_mirror_and_axis_swap_equivariance():
    prev, cur = _pair((16, 16), 40)
    prm = scheme.Params(eps=0.08, gamma=3.0, s=0.01, h=1.0 / 16)
    a = _fas_step(prev, cur, prm)
    m = _fas_step(prev[:, ::-1].copy(), cur[:, ::-1].copy(), prm)
    t = _fas_step(prev.T.copy(), cur.T.copy(), prm)
    for x, y in ((a.phi, m.phi), (a.mu, m.mu), (a.p, m.p)):
        assert np.max(np.abs(x[:, ::-1] - y)) < 1e-11
    for x, y in ((a.phi, t.phi), (a.mu, t.mu), (a.p, t.p)):
        assert np.max(np.abs(x.T - y)) < 1e-11


def test_gamma_zero_has_no_flow():
    """With gamma = 0, (2.7) gives Lap p = 0, so p is constant and u = 0: the pure CH scheme."""
    prev, cur = _pair((8, 8), 50)
    phi, mu, p, hist = newton.solve(prev, cur, 0.1, 0.0, 0.05, 1.0 / 8)
    assert np.max(np.abs(p)) < 1e-13
    # the flow-free scheme: phi - s Lap mu = phi^m with the same mu
    prm = scheme.Params(eps=0.1, gamma=0.0, s=0.05, h=1.0 / 8)
    _, d_u = scheme.dissipation(mu, p, 1.5 * cur - 0.5 * prev, prm)
    assert d_u == 0.0


def _march(phi0, prm, nsteps, tol, solver="fas"):
    """Steps from phi^{-1} = phi^0; returns [(phi^{m-1}, phi^m, result)] per step."""
    states = [phi0.copy(), phi0.copy()]
    mu = np.zeros_like(phi0)
    p = np.zeros_like(phi0)
    results = []
    for _ in range(nsteps):
        if solver == "fas":
            r = fas.solve_step(states[-2], states[-1], mu, p, prm, fas.Opts(tol=tol))
        else:
            phi, mu_n, p_n, _ = newton.solve(states[-2], states[-1], prm.eps, prm.gamma, prm.s,
                                             prm.h, mu0=mu, p0=p, tol=min(tol, 1e-13))
            r = fas.StepResult(phi, mu_n, p_n, 0, [])
        results.append((states[-2], states[-1], r))
        states.append(r.phi)
        mu, p = r.mu, r.p
    return results


@pytest.mark.parametrize("s,solver", [(1e-3, "fas"), (0.1, "newton")])
def test_exact_energy_balance(s, solver):
    """F(phi^{m+1},phi^m) - F(phi^m,phi^{m-1}) = -s||grad mu||^2 - (s/gamma)||u||^2
    - 1/4||phi^{m+1}-2phi^m+phi^{m-1}||^2 - eps^2/8||grad(...)||^2 (proof of Thm 2.1, remainders kept)."""
    n = 32 if solver == "fas" else 16
    prm = scheme.Params(eps=0.05, gamma=2.0, s=s, h=1.0 / n)
    phi0 = uniform_field((n, n), 60, mean=0.1, amp=0.3)
    for prev, cur, r in _march(phi0, prm, 4, tol=1e-12, solver=solver):
        lhs, rhs = scheme.energy_identity_terms(r.phi, cur, prev, r.mu, r.p, prm)
        assert abs(lhs - rhs) < 1e-9, (lhs, rhs)
        assert abs(rhs) > 1e-6       # the balance is not trivially 0 = 0


@pytest.mark.parametrize("s,solver", [(1e-4, "fas"), (1e-2, "fas"), (1.0, "newton"), (100.0, "newton")])
def test_F_nonincreasing_for_any_step(s, solver):
    """Unconditional energy stability (Theorem 2.1): F_h non-increasing for every s > 0."""
    n = 32 if solver == "fas" else 16
    prm = scheme.Params(eps=0.05, gamma=1.0, s=s, h=1.0 / n)
    phi0 = uniform_field((n, n), 70, amp=0.5)
    f_prev = scheme.energy_F(phi0, phi0, prm)
    for prev, cur, r in _march(phi0, prm, 4, tol=1e-11, solver=solver):
        f_new = scheme.energy_F(r.phi, cur, prm)
        assert f_new <= f_prev + 1e-10
        f_prev = f_new


def test_mass_change_equals_minus_residual_mass():
    """(phi^{m+1},1) - (phi^m,1) = -(R_phi,1) exactly: the flux terms of (2.5) telescope (Section 4)."""
    n = 32
    prm = scheme.Params(eps=0.05, gamma=2.0, s=1e-3, h=1.0 / n)
    phi0 = uniform_field((n, n), 80, mean=-0.2, amp=0.05)
    for prev, cur, r in _march(phi0, prm, 3, tol=1e-10):
        phi_star, f = scheme.step_rhs(prev, cur, prm)
        lvl = scheme.Level(h=prm.h, phi_star=phi_star, psi=cur, f=f)
        res = scheme.residual([r.phi, r.mu, r.p], f, lvl, prm)
        dm = grid.mass(r.phi, prm.h) - grid.mass(cur, prm.h)
        assert abs(dm + grid.mass(res[0], prm.h)) < 1e-14
        assert abs(dm) <= grid.norm2(res[0], prm.h) + 1e-15   # |Omega| = 1


def test_vcycle_contraction_on_spinodal_data():
    n = 64
    prm = scheme.Params(eps=0.05, gamma=1.0, s=1e-3, h=1.0 / n)
    phi0 = uniform_field((n, n), 2967, amp=0.05)
    z = np.zeros_like(phi0)
    r = fas.solve_step(phi0, phi0, z, z, prm, fas.Opts(tol=1e-10))
    h = r.res_history
    assert h[-1] <= 1e-10
    assert r.vcycles <= 10
    assert all(h[k + 1] < 0.2 * h[k] for k in range(1, len(h) - 1))


def test_second_order_cauchy_convergence():
    """Cauchy differences under s = T/(N/4) fall as h^2 (Thm 4.6; Table 1 prints rates 2.04..2.00).

    The fine solution is compared with the coarse one after cell-average restriction
    to the coarse grid, the second-order transfer for cell-centred data.
    """
    T = 0.02
    sols = {}
    for n in (16, 32, 64):
        m = n // 4
        prm = scheme.Params(eps=0.1, gamma=1.0, s=T / m, h=1.0 / n)
        sols[n] = _march(smooth_ic_2d(n), prm, m, tol=1e-11)[-1][2].phi
    errs = []
    for n in (32, 64):
        d = fas.restrict(sols[n]) - sols[n // 2]
        errs.append(grid.norm2(d, 2.0 / n))
    rate = np.log2(errs[0] / errs[1])
    assert 1.85 < rate < 2.15, (errs, rate)


# ---- planted mistakes: each must break one of the pins above ---------------------------

def test_planted_pressure_sign_error_is_caught(monkeypatch):
    """Flip the sign of the pressure flux in the oracle's N: FAS then no longer agrees with Newton."""
    shape = (8, 8)
    prev, cur = _pair(shape, 90)
    prm = scheme.Params(eps=0.1, gamma=2.0, s=1.0, h=1.0 / 8)
    good = newton.solve(prev, cur, 0.1, 2.0, 1.0, 1.0 / 8)[0]
    orig = scheme.apply_N

    def bad_apply(u, lvl, prm_):
        n = orig(u, lvl, prm_)
        a, _ = scheme.face_coefficients(lvl.phi_star, prm_.gamma)
        n[0] = n[0] + 2 * prm_.s * grid.div_c_grad(a, u[2], lvl.h)
        return n
    monkeypatch.setattr(fas, "apply_N", bad_apply)
    monkeypatch.setattr(fas, "residual", lambda u, f, lvl, prm_: [f[k] - bad_apply(u, lvl, prm_)[k] for k in range(3)])
    z = np.zeros(shape)
    r = fas.solve_step(prev, cur, z, z, prm, fas.Opts(tol=1e-12, max_vcycles=60))
    assert np.max(np.abs(r.phi - good)) > 1e-6


def test_planted_energy_coefficient_error_is_caught(monkeypatch):
    """Use 1/4 instead of 1/8 in F_h: the exact energy balance breaks."""
    n = 16
    prm = scheme.Params(eps=0.1, gamma=2.0, s=0.01, h=1.0 / n)
    phi0 = uniform_field((n, n), 91, amp=0.3)
    steps = _march(phi0, prm, 2, tol=1e-12)
    prev, cur, r = steps[-1]

    def bad_F(phi, psi, prm_):
        d = phi - psi
        return (scheme.energy_E(phi, prm_) + 0.25 * grid.ip(d, d, prm_.h)
                + 0.25 * prm_.eps ** 2 * grid.grad_norm2_sq(d, prm_.h))
    monkeypatch.setattr(scheme, "energy_F", bad_F)
    lhs, rhs = scheme.energy_identity_terms(r.phi, cur, prev, r.mu, r.p, prm)
    assert abs(lhs - rhs) > 1e-8


def test_planted_chi_error_is_caught(monkeypatch):
    """Drop the psi^3 term of chi in the oracle: the exact energy balance breaks."""
    n = 16
    prm = scheme.Params(eps=0.1, gamma=2.0, s=0.01, h=1.0 / n)
    phi0 = uniform_field((n, n), 92, mean=0.3, amp=0.3)
    # both the smoother and the residual take chi through scheme.nonlinearity
    monkeypatch.setattr(scheme, "chi", lambda a, b: 0.25 * (a ** 3 + a * a * b + a * b * b))
    steps = _march(phi0, prm, 2, tol=1e-12)
    prev, cur, r = steps[-1]
    lhs, rhs = scheme.energy_identity_terms(r.phi, cur, prev, r.mu, r.p, prm)
    assert abs(lhs - rhs) > 1e-8


# ---- solver variants: sweeps per level and bilinear prolongation --------------------------

VARIANTS = [dict(nu1_coarse=1, nu2_coarse=1), dict(nu1_coarse=3, nu2_coarse=3),
            dict(nu1=1, nu2=1, nu1_coarse=2, nu2_coarse=2), dict(prolong="bilinear"),
            dict(nu1=1, nu2=2, prolong="bilinear")]


@pytest.mark.parametrize("shape", [(8, 8), (4, 4, 4)])
@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: ",".join(f"{k}={x}" for k, x in v.items()))
def test_fas_variants_reach_the_newton_solution(shape, variant):
    """Sweeps per level and the transfer operator change the iteration, not the
    converged step: every variant reaches the unique solution (Theorem 2.1)."""
    prev, cur = _pair(shape, 40 + len(shape))
    h = 1.0 / shape[-1]
    prm = scheme.Params(eps=0.1, gamma=2.0, s=0.5, h=h)
    z = np.zeros(shape)
    r = fas.solve_step(prev, cur, z, z, prm, fas.Opts(tol=1e-13, max_vcycles=300, **variant))
    phi, mu, p, _ = newton.solve(prev, cur, 0.1, 2.0, 0.5, h)
    assert np.max(np.abs(r.phi - phi)) < 1e-12
    assert np.max(np.abs(r.mu - mu)) < 1e-12


def test_bilinear_prolongation_weights_by_brute_force():
    """Every fine cell of a 2D coarse array by explicit loops: parent 9/16, the
    parent's neighbour towards the cell along x and along y 3/16 each, the
    diagonal one 1/16, with the parent itself standing in beyond the boundary."""
    rng = np.random.default_rng(7)
    v = rng.random((3, 4))
    out = fas.prolong_bilinear(v)
    ny, nx = v.shape
    for J in range(2 * ny):
        for I in range(2 * nx):
            j, i = J // 2, I // 2
            jn = min(max(j + (1 if J % 2 else -1), 0), ny - 1)
            in_ = min(max(i + (1 if I % 2 else -1), 0), nx - 1)
            want = (9 * v[j, i] + 3 * v[j, in_] + 3 * v[jn, i] + v[jn, in_]) / 16
            assert abs(out[J, I] - want) < 1e-15


def test_bilinear_prolongation_is_exact_for_affine_fields_away_from_the_boundary():
    """Cell centres x = (i + 1/2) h: an affine field sampled on the coarse grid is
    reproduced exactly at the fine centres of every cell not on the boundary
    (second-order interpolation); constants exactly everywhere (3D)."""
    n = 6
    xc = (np.arange(n) + 0.5) * 2.0
    xf = (np.arange(2 * n) + 0.5) * 1.0
    f = lambda z, y, x: 0.3 + 1.7 * x - 0.9 * y + 0.4 * z
    Z, Y, X = np.meshgrid(xc, xc, xc, indexing="ij")
    out = fas.prolong_bilinear(f(Z, Y, X))
    Zf, Yf, Xf = np.meshgrid(xf, xf, xf, indexing="ij")
    inner = (slice(1, -1),) * 3
    np.testing.assert_allclose(out[inner], f(Zf, Yf, Xf)[inner], rtol=0, atol=1e-12)
    np.testing.assert_allclose(fas.prolong_bilinear(np.full((n, n, n), 2.5)), 2.5, rtol=0, atol=0)
