"""GPU tests of the first-order bootstrap step (opts.order = 1, Remark 2.2's option).

The step runs through the per-cell red-black kernels and the coarse tail with
chi(phi) = phi^3 and the whole eps^2 Lap phi implicit; it is compared with the
oracle's first-order step, with the closed-form single-mode amplification, and
used to start a run of the second-order scheme.
"""
import numpy as np
import pytest

from oracle import fas, scheme
from workloads import cosine_mode, uniform_field

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


def _solver(chhs, spec, order):
    probs = [chhs.make_problem(sh, 1.0 / sh[-1], e, g, s) for sh, e, g, s in spec]
    return chhs.Solver(probs, chhs.chhs_default_opts(order=order))


def _flat(arrays):
    return np.concatenate([a.ravel() for a in arrays])


def _split(flat, shapes):
    out, o = [], 0
    for sh in shapes:
        n = int(np.prod(sh))
        out.append(flat[o:o + n].reshape(sh))
        o += n
    return out


CASES = {
    "2d-64": [((64, 64), 0.05, 2.0, 1e-3)],
    "2d-ragged": [((96, 160), 0.03, 1.0, 5e-4)],
    "3d-16": [((16, 16, 16), 0.08, 2.0, 1e-3)],
}


@pytest.mark.parametrize("case", list(CASES))
def test_first_order_step_matches_oracle(chhs, case):
    spec = CASES[case]
    (shape, e, g, s), = spec
    phi0 = uniform_field(shape, 4200, mean=0.05, amp=0.4)
    sv = _solver(chhs, spec, 1)
    tp, tc = dev(phi0), dev(phi0)
    tm, tpp = dev(np.zeros(shape)), dev(np.zeros(shape))
    _, st = sv.step(tp, tc, tm, tpp, 1)
    prm = scheme.Params(eps=e, gamma=g, s=s, h=1.0 / shape[-1], order=1)
    z = np.zeros(shape)
    r = fas.solve_step(phi0, phi0, z, z, prm, fas.Opts(tol=1e-10))
    assert np.max(np.abs(host(tc) - r.phi)) <= 1e-10
    assert np.max(np.abs(host(tm) - r.mu)) <= 1e-8
    assert np.array_equal(host(tp), phi0)
    assert st[0]["vcycles"] == r.vcycles
    assert st[0]["res_norm"] <= 1e-10


def test_batched_first_order_equals_single_runs(chhs):
    spec = [((64, 64), 0.05, 2.0, 1e-3), ((32, 64), 0.04, 0.5, 5e-4)]
    shapes = [sp[0] for sp in spec]
    phi0s = [uniform_field(sh, 4210 + i, amp=0.3) for i, sh in enumerate(shapes)]

    def run(sp, ph):
        sv = _solver(chhs, sp, 1)
        flat = _flat(ph)
        tp, tc = dev(flat), dev(flat)
        tm, tpp = dev(np.zeros(flat.size)), dev(np.zeros(flat.size))
        sv.step(tp, tc, tm, tpp, 1)
        return host(tc)

    batch = _split(run(spec, phi0s), shapes)
    for i in range(len(spec)):
        single = run([spec[i]], [phi0s[i]]).reshape(shapes[i])
        assert np.array_equal(batch[i], single), i


@pytest.mark.parametrize("gamma", [0.0, 3.0])
def test_single_mode_amplification_on_the_gpu(chhs, gamma):
    """Closed form of the linearised first-order step about phibar (the oracle
    pins derive it): g1 = (1 + s lam) / (1 + s lam (3 phibar^2 + eps^2 lam))."""
    n, k, phibar, delta, eps, s = 64, 5, 0.3, 1e-3, 0.03, 0.005
    h = 1.0 / n
    sv = chhs.Solver(chhs.make_problem((n, n), h, eps, gamma, s),
                     chhs.chhs_default_opts(order=1, tol=1e-12))
    phi0 = cosine_mode((n, n), k, phibar, delta)
    tp, tc = dev(phi0), dev(phi0)
    tm, tpp = dev(np.zeros((n, n))), dev(np.zeros((n, n)))
    sv.step(tp, tc, tm, tpp, 1)
    d = (host(tc) - phibar).ravel()
    v = (phi0 - phibar).ravel()
    g = float(d @ v / (v @ v))
    lam = (2.0 - 2.0 * np.cos(np.pi * k / n)) / (h * h)
    want = (1.0 + s * lam) / (1.0 + s * lam * (3.0 * phibar ** 2 + eps ** 2 * lam))
    assert abs(g - want) <= 1e-5 * want, (g, want)


def test_bootstrap_then_second_order_steps(chhs):
    """phi^1 from the first-order step, then the second-order scheme from
    (phi^0, phi^1); every step is checked against the oracle from the GPU's own
    inputs (per-step protocol), and mass is conserved throughout."""
    shape, e, g, s = (128, 128), 0.02, 2.0, 2e-4
    h = 1.0 / shape[-1]
    phi0 = uniform_field(shape, 4230, mean=-0.05, amp=0.05)
    z = np.zeros(shape)
    boot = _solver(chhs, [(shape, e, g, s)], 1)
    tp, tc, tm, tpp = dev(phi0), dev(phi0), dev(z), dev(z)
    boot.step(tp, tc, tm, tpp, 1)
    r1 = fas.solve_step(phi0, phi0, z, z, scheme.Params(eps=e, gamma=g, s=s, h=h, order=1))
    assert np.max(np.abs(host(tc) - r1.phi)) <= 1e-10
    main = _solver(chhs, [(shape, e, g, s)], 2)
    prm = scheme.Params(eps=e, gamma=g, s=s, h=h)
    mass0 = h * h * phi0.sum()
    for m in range(3):
        prev, cur, mu_in, p_in = host(tp), host(tc), host(tm), host(tpp)
        _, st = main.step(tp, tc, tm, tpp, 1)
        r = fas.solve_step(prev, cur, mu_in, p_in, prm, fas.Opts(tol=1e-10))
        assert np.max(np.abs(host(tc) - r.phi)) <= 1e-10
        assert st[0]["vcycles"] == r.vcycles
        # |mass change| <= |Omega|^(1/2) ||R_phi|| <= 1 * tol per step (bootstrap included)
        assert abs(st[0]["mass"] - mass0) <= 1e-10 * (m + 2)
