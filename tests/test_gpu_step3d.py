"""GPU tests of the fused 3D smoothing step (z marching) against the per-cell
red-black kernels and the oracle.

Both perform the same ordered red-black collective updates (Section 5's
smoother), so their iterates agree to rounding: smoothing steps on the finest
and on coarse levels with general right-hand sides, whole FP64 and mixed steps,
the default per-level choice and the autotuned one are compared.
"""
import numpy as np
import pytest

from oracle import fas, scheme
from workloads import uniform_field

pytestmark = pytest.mark.gpu

PER_CELL, FUSED = 3, 4


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


def _prm(shape, eps=0.05, gamma=2.0, s=1e-3):
    return scheme.Params(eps=eps, gamma=gamma, s=s, h=1.0 / shape[-1])


def _solver(chhs, shape, prm, **opts):
    prob = chhs.make_problem(shape, prm.h, prm.eps, prm.gamma, prm.s)
    return chhs.Solver(prob, chhs.chhs_default_opts(**opts))


# (nz, ny, nx): whole tiles; ragged x and y tiles (16 x 16 FP64, 32 x 16 FP32)
# and, on level 1, a ragged last z segment
SHAPES = [(64, 64, 64), (56, 40, 40), (40, 24, 56)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("level", [0, 1])
@pytest.mark.parametrize("nsweeps", [1, 2, 3])
def test_fused_smoothing_matches_oracle_and_per_cell(chhs, shape, level, nsweeps):
    prm = _prm(shape)
    prev, cur, mu0, p0 = _inputs(shape, 800 + level)
    out = {}
    for mode in (PER_CELL, FUSED):
        sv = _solver(chhs, shape, prm, smoother=mode)
        assert sv.level_kernels()[0][0] == ("zmarch" if mode == FUSED else "per-cell")
        sv.setup_step(dev(prev), dev(cur), dev(mu0), dev(p0))
        ls = tuple(n >> level for n in shape)
        if level > 0:
            u = [uniform_field(ls, 810 + k, amp=0.5) for k in range(3)]
            f = [uniform_field(ls, 820 + k, amp=0.5) for k in range(3)]
            for name, val in zip(("phi", "mu", "p", "f_phi", "f_mu", "f_p"), u + f):
                sv.write_field(level, name, dev(val))
        sv.smooth(level, nsweeps)
        out[mode] = [host(sv.read_field(level, n)) for n in ("phi", "mu", "p")]
        if level > 0:
            lvl = scheme.Level(h=prm.h * 2 ** level, phi_star=host(sv.read_field(level, "phi_star")),
                               psi=host(sv.read_field(level, "psi")), f=f)
        else:
            phi_star, f0 = scheme.step_rhs(prev, cur, prm)
            lvl = scheme.Level(h=prm.h, phi_star=phi_star, psi=cur.copy(), f=f0)
            u = [cur.copy(), mu0.copy(), p0 - p0.mean()]
    for _ in range(nsweeps):
        fas.sweep(u, lvl, prm)
    for k, want in enumerate(u):
        scale = max(1.0, np.max(np.abs(want)))
        assert np.max(np.abs(out[FUSED][k] - want)) <= 1e-11 * scale, k
        assert np.max(np.abs(out[FUSED][k] - out[PER_CELL][k])) <= 1e-13 * scale, k


def _steps(chhs, spec, phi0s, precision, nsteps=2, **opts):
    probs = [chhs.make_problem(sh, 1.0 / sh[-1], e, g, s_) for sh, e, g, s_ in spec]
    sv = chhs.Solver(probs, chhs.chhs_default_opts(precision=precision, **opts))
    flat = np.concatenate([a.ravel() for a in phi0s])
    tp, tc = dev(flat), dev(flat)
    tm, tpp = dev(np.zeros(flat.size)), dev(np.zeros(flat.size))
    out = []
    for _ in range(nsteps):
        _, st = sv.step(tp, tc, tm, tpp, 1)
        assert all(x["res_norm"] <= 1e-10 for x in st)
        out.append((host(tc), [x["vcycles"] for x in st]))
    return out, sv


SPECS = {"single": [((64, 64, 64), 0.04, 2.0, 5e-4)],
         "ragged": [((56, 40, 40), 0.05, 1.0, 1e-3), ((32, 32, 32), 0.04, 2.0, 5e-4)]}


@pytest.mark.parametrize("name", list(SPECS))
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_steps_agree_across_3d_smoothers(chhs, name, precision):
    """Whole steps with the fused step everywhere, per-cell kernels everywhere,
    the default per-level choice and the autotuned one: the same cycle counts
    (FP64) and the same solution to the step tolerance."""
    spec = SPECS[name]
    phi0s = [uniform_field(sp[0], 830 + i, mean=0.1, amp=0.05) for i, sp in enumerate(spec)]
    ref, _ = _steps(chhs, spec, phi0s, precision, smoother=PER_CELL)
    tol = 1e-10 if precision == 0 else 1e-8
    for opts in (dict(smoother=FUSED), dict(smoother=0), dict(smoother=0, autotune=1)):
        got, sv = _steps(chhs, spec, phi0s, precision, **opts)
        kinds = {k for k, _, _ in sv.level_kernels()}
        assert kinds <= {"zmarch", "per-cell", "tail"}, kinds
        for (a, va), (b, vb) in zip(got, ref):
            if precision == 0:
                assert va == vb, opts
            assert np.max(np.abs(a - b)) <= tol, opts



@pytest.mark.parametrize("shape", [(64, 64, 64), (56, 40, 40)])
@pytest.mark.parametrize("prolong", [0, 1], ids=["constant", "trilinear"])
@pytest.mark.parametrize("nu", [(2, 2), (1, 3)])
def test_one_vcycle_with_fused_steps_matches_oracle(chhs, shape, prolong, nu):
    """One V-cycle with the fused step on every level above the tail (the first
    post step taking the prolongation in its loads): iterate by iterate with
    the oracle (<= 1e-11) and with the per-cell kernels (<= 1e-13)."""
    prm = _prm(shape)
    prev, cur, mu0, p0 = _inputs(shape, 850)
    out = {}
    for mode in (PER_CELL, FUSED):
        sv = _solver(chhs, shape, prm, smoother=mode, prolong=prolong, nu1=nu[0], nu2=nu[1])
        sv.setup_step(dev(prev), dev(cur), dev(mu0), dev(p0))
        res = sv.fas_vcycle()[0]
        out[mode] = (res, [host(sv.read_field(0, n)) for n in ("phi", "mu", "p")])
    phi_star, f = scheme.step_rhs(prev, cur, prm)
    levels = fas.build_levels(phi_star, cur.copy(), f, prm.h)
    u = [cur.copy(), mu0.copy(), p0 - p0.mean()]
    us = [None] * len(levels)
    us[0] = u
    o = fas.Opts(nu1=nu[0], nu2=nu[1], prolong="bilinear" if prolong else "constant")
    fas.vcycle(levels, us, 0, prm, o)
    u[2] -= u[2].mean()
    for k, want in enumerate(u):
        scale = max(1.0, np.max(np.abs(want)))
        assert np.max(np.abs(out[FUSED][1][k] - want)) <= 1e-11 * scale, k
        assert np.max(np.abs(out[FUSED][1][k] - out[PER_CELL][1][k])) <= 1e-13 * scale, k
    assert abs(out[FUSED][0] - out[PER_CELL][0]) <= 1e-12 * out[PER_CELL][0]
