"""GPU tests of the solver variants: sweeps per level and bilinear prolongation.

The variants change the iteration, not the step's solution (Theorem 2.1).  The
HIP path runs them as the oracle does (``fas.Opts.nu1_coarse``, ``nu2_coarse``,
``prolong``), so one V-cycle agrees iterate by iterate (<= 1e-11) and whole
steps take the same number of cycles and agree to the step tolerance.  The
tuner (chhs_tune_sweeps) picks one of them by time to tolerance without
advancing the state; the steps it leads to still solve the scheme.
"""
import numpy as np
import pytest

from oracle import fas, scheme
from workloads import WORKLOADS, batched_instances, uniform_field

pytestmark = pytest.mark.gpu

VARIANTS = [dict(nu1_coarse=1, nu2_coarse=3), dict(nu1=1, nu2=2), dict(prolong=1),
            dict(nu1=1, nu2=1, nu1_coarse=3, nu2_coarse=3, prolong=1)]


def _ids(v):
    return ",".join(f"{k}={x}" for k, x in v.items())


def _oracle_opts(v, **kw):
    o = {k: x for k, x in v.items() if k != "prolong"}
    if v.get("prolong") == 1:
        o["prolong"] = "bilinear"
    return fas.Opts(**o, **kw)


@pytest.fixture(scope="module")
def chhs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1611_02967_amd import chhs as binding
    return binding


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def _inputs(shape, seed):
    prev = uniform_field(shape, seed, amp=0.6)
    cur = prev + uniform_field(shape, seed + 1, amp=0.1)
    mu0 = uniform_field(shape, seed + 2, amp=0.3)
    p0 = uniform_field(shape, seed + 3, amp=0.01)
    return prev, cur, mu0, p0


@pytest.mark.parametrize("shape", [(64, 64), (256, 192), (16, 16, 16)])
@pytest.mark.parametrize("variant", VARIANTS, ids=_ids)
def test_one_vcycle_of_a_variant_matches_oracle(chhs, shape, variant):
    prm = scheme.Params(eps=0.05, gamma=2.0, s=1e-3, h=1.0 / shape[-1])
    prev, cur, mu0, p0 = _inputs(shape, 7000)
    prob = chhs.make_problem(shape, prm.h, prm.eps, prm.gamma, prm.s)
    sv = chhs.Solver(prob, chhs.chhs_default_opts(**variant))
    sv.setup_step(dev(prev), dev(cur), dev(mu0), dev(p0))
    res_gpu = sv.fas_vcycle()[0]
    phi_star, f = scheme.step_rhs(prev, cur, prm)
    levels = fas.build_levels(phi_star, cur.copy(), f, prm.h)
    u = [cur.copy(), mu0.copy(), p0 - p0.mean()]
    us = [None] * len(levels)
    us[0] = u
    fas.vcycle(levels, us, 0, prm, _oracle_opts(variant))
    u[2] -= u[2].mean()
    for name, want in zip(("phi", "mu", "p"), u):
        got = host(sv.read_field(0, name))
        assert np.max(np.abs(got - want)) <= 1e-11 * max(1.0, np.max(np.abs(want))), name
    res_or = scheme.residual_norm(scheme.residual(u, f, levels[0], prm), prm.h)
    assert abs(res_gpu - res_or) <= 1e-9 * res_or + 1e-14


@pytest.mark.parametrize("variant", VARIANTS, ids=_ids)
def test_steps_of_a_variant_match_oracle(chhs, variant):
    """Three steps of the 64^2 workload per the per-step protocol: same cycle
    count as the oracle with the same variant, max |phi - oracle| <= 1e-10."""
    w = WORKLOADS["2d-64-fp64"]
    n = w["n"]
    prm = scheme.Params(eps=w["eps"], gamma=w["gamma"], s=w["s"], h=1.0 / n)
    phi0 = uniform_field((n, n), w["seed"], mean=w["mean"], amp=0.05)
    sv = chhs.Solver(chhs.make_problem((n, n), prm.h, prm.eps, prm.gamma, prm.s),
                     chhs.chhs_default_opts(**variant))
    prev, cur = phi0.copy(), phi0.copy()
    mu = np.zeros_like(phi0)
    p = np.zeros_like(phi0)
    for m in range(3):
        r = fas.solve_step(prev, cur, mu, p, prm, _oracle_opts(variant, tol=1e-10))
        tp, tc, tm, tpp = dev(prev), dev(cur), dev(mu), dev(p)
        _, st = sv.step(tp, tc, tm, tpp, 1)
        assert st[0]["vcycles"] == r.vcycles, (m, st[0]["vcycles"], r.vcycles)
        assert np.max(np.abs(host(tc) - r.phi)) <= 1e-10
        prev, cur, mu, p = cur, r.phi, r.mu, r.p


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_tuned_sweeps_keep_the_state_and_solve_the_step(chhs, precision):
    """chhs_tune_sweeps on a batch (ragged 2D draw): returns one of its
    candidates, leaves the caller's arrays untouched, and the steps taken with
    the choice agree with the default cycle's to the step tolerance."""
    insts = batched_instances(count=4, sizes=(128, 256))
    probs = [chhs.make_problem(it.shape, it.h, it.eps, it.gamma, it.s) for it in insts]
    flat = np.concatenate([it.phi0().ravel() for it in insts])
    z = np.zeros(flat.size)
    sv = chhs.Solver(probs, chhs.chhs_default_opts(precision=precision))
    ref = chhs.Solver(probs, chhs.chhs_default_opts(precision=precision))
    a = [dev(flat), dev(flat), dev(z), dev(z)]
    b = [dev(flat), dev(flat), dev(z), dev(z)]
    choice = sv.tune_sweeps(*a)
    nu1, nu2, nu1c, nu2c, prolong, inner = choice
    assert nu1 >= 1 and nu2 >= 1 and nu1c >= 0 and nu2c >= 0 and prolong in (0, 1)
    assert inner in ((1, 2, 3) if precision == 1 else (0,))
    o = sv.get_opts()
    assert (o.nu1, o.nu2, o.nu1_coarse, o.nu2_coarse, o.prolong, o.inner_cycles) == choice
    for x, want in zip(a, (flat, flat, z, z)):
        assert np.array_equal(host(x), want)
    for _ in range(2):
        _, sa = sv.step(*a, 1)
        _, sb = ref.step(*b, 1)
        assert all(x["res_norm"] <= 1e-10 for x in sa)
        assert np.max(np.abs(host(a[1]) - host(b[1]))) <= 1e-9
