"""GPU parity at the protocol sizes of the 3D and batched workloads.

* Kernel level at 128^3: one smoothing step with the restriction and FAS
  coarse right-hand side, and one whole V-cycle, iterate by iterate against
  the oracle (<= 1e-11).  The coarse level 64^3 holds 1024 tasks of 256 cells,
  so these launches take the one-thread-per-coarse-cell restriction, not the
  lane-exchange one of the smaller shapes.
* Step level at 64^3 (eps 0.02, gamma 2, s 5e-4, phi^0 = 0.1 + 0.05 (2r - 1)):
  three steps of the per-step protocol -- every step starts from the oracle's
  (phi^{m-1}, phi^m) -- for the FP64 path (<= 1e-10, the same V-cycle count as
  the oracle) and for FP32 inner cycles with FP64 refinement (<= 1e-8).
* The post-step reductions (discrete mass, E_h (2.8), F_h (2.9), the two
  dissipation terms of Theorem 2.1, max |phi|) in 3D at 32^3 and in 2D at
  1024^2 (4096 per-cell partials in one instance), against the oracle.
* The ragged batched workload: a draw of eight instances (two each of 128^2,
  256^2, 512^2, 1024^2, random eps, gamma, s, mean) advanced by the batched
  mixed path, each instance against the plain FP64 path run alone (<= 1e-8),
  the 128^2 instances against the oracle.
* A 3D batch whose restriction launch takes the serial kernel while each
  instance alone takes the lane-exchange kernel equals the single runs bit
  for bit (both add a coarse cell's children in the same order).
* chhs_step_log: every step's record, against the oracle's energies of the
  GPU's own states, and the same steps as chhs_step.
"""
import numpy as np
import pytest

from oracle import fas, grid, scheme
from workloads import WORKLOADS, batched_instances, uniform_field

pytestmark = pytest.mark.gpu


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


def _pack(arrays):
    return np.concatenate([a.ravel() for a in arrays])


def _unpack(flat, shapes):
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(flat[o:o + n].reshape(s))
        o += n
    return out


def _solver(chhs, shape, prm, **opts):
    prob = chhs.make_problem(shape, prm.h, prm.eps, prm.gamma, prm.s)
    return chhs.Solver(prob, chhs.chhs_default_opts(**opts))


def _inputs(shape, seed):
    prev = uniform_field(shape, seed, amp=0.6)
    cur = prev + uniform_field(shape, seed + 1, amp=0.1)
    mu0 = uniform_field(shape, seed + 2, amp=0.3)
    p0 = uniform_field(shape, seed + 3, amp=0.01)
    return prev, cur, mu0, p0


def _config2_params(n):
    w = WORKLOADS["3d-128-fp64"]
    return w, scheme.Params(eps=w["eps"], gamma=w["gamma"], s=w["s"], h=1.0 / n)


def test_restriction_at_128_cubed_matches_oracle(chhs):
    shape = (128, 128, 128)
    _, prm = _config2_params(128)
    prev, cur, mu0, p0 = _inputs(shape, 5000)
    sv = _solver(chhs, shape, prm)
    sv.setup_step(dev(prev), dev(cur), dev(mu0), dev(p0))
    sv.smooth(0, 1)
    sv.restrict(0)
    phi_star, f = scheme.step_rhs(prev, cur, prm)
    levels = fas.build_levels(phi_star, cur.copy(), f, prm.h)
    u = [cur.copy(), mu0.copy(), p0 - p0.mean()]
    fas.sweep(u, levels[0], prm)
    r = scheme.residual(u, f, levels[0], prm)
    uc = [fas.restrict(x) for x in u]
    nc = scheme.apply_N(uc, levels[1], prm)
    fc = [fas.restrict(r[k]) + nc[k] for k in range(3)]
    for name, want in zip(("phi", "mu", "p", "f_phi", "f_mu", "f_p"), uc + fc):
        got = host(sv.read_field(1, name))
        assert np.max(np.abs(got - want)) <= 1e-11 * max(1.0, np.max(np.abs(want))), name


def test_one_vcycle_at_128_cubed_matches_oracle(chhs):
    shape = (128, 128, 128)
    w, prm = _config2_params(128)
    prev = uniform_field(shape, w["seed"], mean=w["mean"], amp=0.05)
    cur = prev + uniform_field(shape, w["seed"] + 1, amp=0.01)
    z = np.zeros(shape)
    sv = _solver(chhs, shape, prm)
    sv.setup_step(dev(prev), dev(cur), dev(z), dev(z))
    res_gpu = sv.fas_vcycle()[0]
    phi_star, f = scheme.step_rhs(prev, cur, prm)
    levels = fas.build_levels(phi_star, cur.copy(), f, prm.h)
    us = [None] * len(levels)
    us[0] = [cur.copy(), z.copy(), z.copy()]
    fas.vcycle(levels, us, 0, prm, fas.Opts())
    u = us[0]
    u[2] -= u[2].mean()
    for name, want in zip(("phi", "mu", "p"), u):
        got = host(sv.read_field(0, name))
        assert np.max(np.abs(got - want)) <= 1e-11 * max(1.0, np.max(np.abs(want))), name
    res_or = scheme.residual_norm(scheme.residual(u, f, levels[0], prm), prm.h)
    assert abs(res_gpu - res_or) <= 1e-8 * res_or + 1e-14


@pytest.fixture(scope="module")
def oracle_64_cubed():
    """Three oracle steps of the 3D workload at 64^3 from the seeded phi^0."""
    n = 64
    w, prm = _config2_params(n)
    phi0 = uniform_field((n,) * 3, w["seed"], mean=w["mean"], amp=0.05)
    prev, cur = phi0.copy(), phi0.copy()
    mu = np.zeros_like(phi0)
    p = np.zeros_like(phi0)
    steps = []
    for _ in range(3):
        r = fas.solve_step(prev, cur, mu, p, prm, fas.Opts(tol=1e-10))
        steps.append((prev, cur, mu, p, r))
        prev, cur, mu, p = cur, r.phi, r.mu, r.p
    return prm, steps


@pytest.mark.parametrize("precision,bound", [(0, 1e-10), (1, 1e-8)], ids=["fp64", "mixed"])
def test_3d_64_cubed_per_step_parity(chhs, oracle_64_cubed, precision, bound):
    prm, steps = oracle_64_cubed
    sv = _solver(chhs, (64, 64, 64), prm, tol=1e-10, precision=precision)
    for m, (prev, cur, mu, p, r) in enumerate(steps):
        tp, tc, tm, tpp = dev(prev), dev(cur), dev(mu), dev(p)
        _, st = sv.step(tp, tc, tm, tpp, 1)
        assert st[0]["res_norm"] <= 1e-10
        if precision == 0:
            assert st[0]["vcycles"] == r.vcycles, (m, st[0]["vcycles"], r.vcycles)
        err = float(np.max(np.abs(host(tc) - r.phi)))
        print(f"64^3 {'fp64' if precision == 0 else 'mixed'} step {m}: max|phi - oracle| = "
              f"{err:.2e}, cycles {st[0]['vcycles']} (oracle {r.vcycles})")
        assert err <= bound, (m, err)
        assert np.max(np.abs(host(tp) - cur)) == 0.0


def _check_energies(chhs, sv, shape, prm, prev, cur, tol_rel):
    mass, e_h, f_h = sv.energy_mass(dev(cur), dev(prev))[0]
    assert abs(mass - grid.mass(cur, prm.h)) <= 1e-13 * max(1.0, np.sum(np.abs(cur)) * prm.h ** len(shape))
    assert abs(e_h - scheme.energy_E(cur, prm)) <= tol_rel * max(1, abs(e_h))
    assert abs(f_h - scheme.energy_F(cur, prev, prm)) <= tol_rel * max(1, abs(f_h))
    z = np.zeros(shape)
    tp, tc, tm, tpp = dev(prev), dev(cur), dev(z), dev(z)
    _, st = sv.step(tp, tc, tm, tpp, 1)
    phi, mu, p = host(tc), host(tm), host(tpp)
    d_mu, d_u = scheme.dissipation(mu, p, 1.5 * cur - 0.5 * prev, prm)
    s0 = st[0]
    assert abs(s0["mass"] - grid.mass(phi, prm.h)) <= 1e-12
    assert abs(s0["E_h"] - scheme.energy_E(phi, prm)) <= tol_rel * max(1, abs(s0["E_h"]))
    assert abs(s0["F_h"] - scheme.energy_F(phi, cur, prm)) <= tol_rel * max(1, abs(s0["F_h"]))
    assert abs(s0["diss_mu"] - d_mu) <= tol_rel * max(1, d_mu)
    assert abs(s0["diss_u"] - d_u) <= tol_rel * max(1, d_u)
    assert s0["max_abs_phi"] == np.max(np.abs(phi))
    lhs, rhs = scheme.energy_identity_terms(phi, cur, prev, mu, p, prm)
    assert abs(lhs - rhs) <= 1e-9


def test_3d_energies_and_step_stats_match_oracle(chhs):
    shape = (32, 32, 32)
    prm = scheme.Params(eps=0.05, gamma=2.0, s=1e-3, h=1.0 / 32)
    prev = uniform_field(shape, 5100, mean=0.1, amp=0.3)
    cur = prev + uniform_field(shape, 5101, amp=0.05)
    sv = _solver(chhs, shape, prm)
    _check_energies(chhs, sv, shape, prm, prev, cur, 1e-12)


def test_2d_1024_energies_and_step_stats_match_oracle(chhs):
    """4096 per-cell partials in one instance (one reduction block sums them)."""
    shape = (1024, 1024)
    w = WORKLOADS["2d-1024-fp64"]
    prm = scheme.Params(eps=w["eps"], gamma=w["gamma"], s=w["s"], h=1.0 / 1024)
    prev = uniform_field(shape, 5200, amp=0.3)
    cur = prev + uniform_field(shape, 5201, amp=0.02)
    sv = _solver(chhs, shape, prm)
    _check_energies(chhs, sv, shape, prm, prev, cur, 1e-11)


def test_batched_draw_with_1024_instances_matches_fp64_and_oracle(chhs):
    """Two each of 128^2..1024^2 by the ragged-batch recipe: one step of the
    batched mixed path against the plain FP64 path run alone per instance, and
    the 128^2 instances against the oracle (both to tol 1e-10)."""
    insts = batched_instances(count=8)
    shapes = [it.shape for it in insts]
    assert sorted({s[0] for s in shapes}) == [128, 256, 512, 1024]
    probs = [chhs.make_problem(it.shape, it.h, it.eps, it.gamma, it.s) for it in insts]
    phi0s = [it.phi0() for it in insts]
    flat = _pack(phi0s)
    sv = chhs.Solver(probs, chhs.chhs_default_opts(precision=1, tol=1e-10))
    tp, tc = dev(flat), dev(flat)
    z = np.zeros(flat.size)
    tm, tpp = dev(z), dev(z)
    _, st = sv.step(tp, tc, tm, tpp, 1)
    got = _unpack(host(tc), shapes)
    for i, it in enumerate(insts):
        assert st[i]["res_norm"] <= 1e-10
        s1 = chhs.Solver(probs[i], chhs.chhs_default_opts(precision=0, tol=1e-10))
        a, b = dev(phi0s[i]), dev(phi0s[i])
        zi = np.zeros(it.shape)
        s1.step(a, b, dev(zi), dev(zi), 1)
        err = float(np.max(np.abs(got[i] - host(b))))
        assert err <= 1e-8, (i, it.shape, err)
        s1.close()
        if it.shape[0] == 128:
            prm = scheme.Params(eps=it.eps, gamma=it.gamma, s=it.s, h=it.h)
            r = fas.solve_step(phi0s[i], phi0s[i], zi, zi, prm, fas.Opts(tol=1e-10))
            assert np.max(np.abs(got[i] - r.phi)) <= 1e-8, i
            assert np.max(np.abs(host(b) - r.phi)) <= 1e-10, i


@pytest.mark.parametrize("smoother", [3, 0], ids=["per-cell", "default"])
def test_3d_batch_across_the_restriction_kernels_equals_single_runs(chhs, smoother):
    """Per-cell kernels, three 64^3 instances: the restriction into 32^3 covers
    384 coarse tasks over the batch (the one-thread-per-coarse-cell kernel) and
    128 for one instance alone (the lane-exchange kernel).  Default kernels, a
    64 x 128 x 128 instance with two 64^3 ones: the large one restricts its
    finest level by z marching, the small ones per cell, in the batch as
    alone.  Results are bitwise equal."""
    spec = [((64, 64, 64), 0.02, 2.0, 5e-4, 0.1), ((64, 64, 64), 0.03, 1.0, 1e-3, -0.1),
            ((64, 64, 64), 0.04, 3.0, 5e-4, 0.0)]
    if smoother == 0:
        spec[0] = ((64, 128, 128), 0.02, 2.0, 5e-4, 0.1)
    shapes = [s[0] for s in spec]
    phi0s = [uniform_field(sh, 5300 + i, mean=sp[4], amp=0.05) for i, (sh, sp) in
             enumerate(zip(shapes, spec))]

    def run(sp_list, arrays):
        probs = [chhs.make_problem(sh, 1.0 / sh[-1], e, g, s) for sh, e, g, s, _ in sp_list]
        sv = chhs.Solver(probs, chhs.chhs_default_opts(smoother=smoother))
        flat = _pack(arrays)
        tp, tc = dev(flat), dev(flat)
        z = np.zeros(flat.size)
        tm, tpp = dev(z), dev(z)
        out = []
        for _ in range(2):
            _, st = sv.step(tp, tc, tm, tpp, 1)
            out.append((host(tc), host(tm), host(tpp), [s["vcycles"] for s in st]))
        sv.close()
        return out

    batch = run(spec, phi0s)
    for i in range(len(spec)):
        single = run([spec[i]], [phi0s[i]])
        for m in range(2):
            for k in range(3):
                a = _unpack(batch[m][k], shapes)[i]
                b = single[m][k].reshape(shapes[i])
                assert np.array_equal(a, b), (i, m, k)
            assert batch[m][3][i] == single[m][3][0]


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_step_log_records_every_step(chhs, precision):
    """chhs_step_log over 4 steps of the 64^2 workload: each record's energies
    are the oracle's of the GPU's own states, F_h does not increase (Theorem
    2.1), and the steps equal those of chhs_step one at a time."""
    w = WORKLOADS["2d-64-fp64"]
    n = w["n"]
    prm = scheme.Params(eps=w["eps"], gamma=w["gamma"], s=w["s"], h=1.0 / n)
    phi0 = uniform_field((n, n), w["seed"], mean=w["mean"], amp=0.05)
    z = np.zeros((n, n))
    sv = _solver(chhs, (n, n), prm, precision=precision)
    tp, tc, tm, tpp = dev(phi0), dev(phi0), dev(z), dev(z)
    _, log = sv.step_log(tp, tc, tm, tpp, 4)
    ref = _solver(chhs, (n, n), prm, precision=precision)
    a, b, c, d = dev(phi0), dev(phi0), dev(z), dev(z)
    prev_f = scheme.energy_E(phi0, prm)
    for m in range(4):
        cur = host(b)
        _, st = ref.step(a, b, c, d, 1)
        phi = host(b)
        rec = log[m][0]
        assert rec["steps_done"] == m + 1 and rec["status"] == 0
        assert rec["vcycles"] == st[0]["vcycles"]
        assert rec["res_norm"] == st[0]["res_norm"]
        assert abs(rec["mass"] - grid.mass(phi, prm.h)) <= 1e-13
        assert abs(rec["E_h"] - scheme.energy_E(phi, prm)) <= 1e-12
        assert abs(rec["F_h"] - scheme.energy_F(phi, cur, prm)) <= 1e-12
        assert rec["F_h"] <= prev_f + 1e-12
        prev_f = rec["F_h"]
    for x, y in zip((tp, tc, tm, tpp), (a, b, c, d)):
        assert np.array_equal(host(x), host(y))
    # the last step's energies in chhs_step's record equal the log's
    assert st[0]["F_h"] == log[3][0]["F_h"] and st[0]["mass"] == log[3][0]["mass"]
