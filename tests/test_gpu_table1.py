"""Table 1 of Section 5.1 on the GPU path: the paper's convergence experiment.

L = 3.2, eps = 0.2, gamma = 2, s = 0.05 h, T = 0.8, initial condition (5.1),
FAS V(2,2) to tol 1e-10, on 16^2 .. 512^2 (5 N time steps at N^2).  Checked:
second-order Cauchy rates (the table prints 2.04, 2.01, 2.00, 2.00), the mass
of (5.1), -5.12, constant in time (Section 4: the scheme conserves mass), and
F_h non-increasing (Theorem 2.1).

The Cauchy differences themselves are compared with the printed ones up to one
common factor, because the absolute level depends on readings the paper leaves
open.  Two transfers are measured: cell averaging of the fine solution onto the
coarse grid (h_c-weighted l2 norm; 7.7 times the printed values from 32^2 on)
and the paper's stated operator, bilinear interpolation of the coarse solution
onto the fine grid with even reflection at the Neumann boundary (h_f-weighted
l2 norm; 4.9 times, first rate 2.06 against the printed 2.04).  The other
reading of the first step, a first-order convex-splitting step for phi^1
(Remark 2.2), changes the differences by under 1%, so it does not explain the
factor.  Each test pins the ratio to be the same for every pair, i.e. the
shape of the printed column.
"""
import math

import numpy as np
import pytest

from workloads import paper_ic_51

pytestmark = pytest.mark.gpu

L, EPS, GAMMA, T = 3.2, 0.2, 2.0, 0.8
SIZES = [16, 32, 64, 128, 256, 512]
# (N_coarse, N_fine) -> Cauchy difference and rate printed in Table 1
PRINTED = {(16, 32): 7.6501e-3, (32, 64): 1.8565e-3, (64, 128): 4.6141e-4, (128, 256): 1.1520e-4,
           (256, 512): 2.8792e-5}
PRINTED_RATE = {(32, 64): 2.04, (64, 128): 2.01, (128, 256): 2.00, (256, 512): 2.00}


@pytest.fixture(scope="module")
def chhs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1611_02967_amd import chhs as binding
    return binding


def _restrict(v):
    return 0.25 * (v[0::2, 0::2] + v[1::2, 0::2] + v[0::2, 1::2] + v[1::2, 1::2])


def _bilinear_up(v):
    """Cell-centred bilinear interpolation of a coarse field onto the grid of
    twice the resolution, with even reflection across the boundary (the
    Neumann ghost cells of App. A.1): a fine centre lies a quarter of a coarse
    cell from its parent's centre, weights 9/16, 3/16, 3/16, 1/16."""
    n = v.shape[0]
    p = np.pad(v, 1, mode="edge")
    out = np.empty((2 * n, 2 * n))
    for dy, sy in ((0, -1), (1, 1)):
        for dx, sx in ((0, -1), (1, 1)):
            c = p[1:-1, 1:-1]
            a = p[1 + sy:n + 1 + sy, 1:-1]
            b = p[1:-1, 1 + sx:n + 1 + sx]
            ab = p[1 + sy:n + 1 + sy, 1 + sx:n + 1 + sx]
            out[dy::2, dx::2] = 9 / 16 * c + 3 / 16 * a + 3 / 16 * b + 1 / 16 * ab
    return out


def _run(chhs, n, first_order_start=False):
    import torch
    h = L / n
    s = 0.05 * h
    steps = int(round(T / s))
    prob = chhs.make_problem((n, n), h, EPS, GAMMA, s)
    sv = chhs.Solver(prob, chhs.chhs_default_opts(tol=1e-10))
    phi0 = paper_ic_51(n, L)
    tp = torch.from_numpy(phi0).cuda()
    tc = tp.clone()
    tm = torch.zeros_like(tp)
    tpp = torch.zeros_like(tp)
    k = steps
    if first_order_start:
        chhs.Solver(prob, chhs.chhs_default_opts(tol=1e-10, order=1)).step(tp, tc, tm, tpp, 1)
        k -= 1
    sv.step(tp, tc, tm, tpp, k)
    return tc.cpu().numpy()


def _bilinear_deltas(phis):
    out = {}
    for n in SIZES[:-1]:
        d = phis[2 * n] - _bilinear_up(phis[n])
        out[(n, 2 * n)] = math.sqrt(np.sum(d * d)) * (L / (2 * n))
    return out


@pytest.fixture(scope="module")
def runs(chhs):
    import torch
    out = {}
    for n in SIZES:
        h = L / n
        s = 0.05 * h
        steps = int(round(T / s))
        sv = chhs.Solver(chhs.make_problem((n, n), h, EPS, GAMMA, s),
                         chhs.chhs_default_opts(tol=1e-10))
        phi0 = paper_ic_51(n, L)
        tp = torch.from_numpy(phi0).cuda()
        tc = tp.clone()
        tm = torch.zeros_like(tp)
        tpp = torch.zeros_like(tp)
        mass, F, cyc = [float(h * h * phi0.sum())], [], []
        for _ in range(steps):
            _, st = sv.step(tp, tc, tm, tpp, 1)
            mass.append(st[0]["mass"])
            F.append(st[0]["F_h"])
            cyc.append(st[0]["vcycles"])
        out[n] = dict(phi=tc.cpu().numpy(), mass=np.array(mass), F=np.array(F),
                      vcycles=float(np.mean(cyc)), steps=steps, h=h)
        print(f"N={n}: {steps} steps, {out[n]['vcycles']:.2f} V-cycles/step, "
              f"mass {mass[-1]:.12f}, F_h {F[0]:.6f} -> {F[-1]:.6f}")
    return out


def test_cauchy_rates_are_second_order(runs):
    deltas = {}
    for n in SIZES[:-1]:
        d = _restrict(runs[2 * n]["phi"]) - runs[n]["phi"]
        deltas[(n, 2 * n)] = math.sqrt(np.sum(d * d)) * runs[n]["h"]
    rates = {}
    keys = sorted(deltas)
    for a, b in zip(keys, keys[1:]):
        rates[b] = math.log2(deltas[a] / deltas[b])
    for k in keys:
        print(f"{k}: delta {deltas[k]:.4e} (printed {PRINTED.get(k, float('nan')):.4e})"
              + (f", rate {rates[k]:.3f}" if k in rates else ""))
    # rates as printed in the asymptotic range (2.01, 2.00, 2.00); the first
    # printed rate, 2.04, comes from the 16^2 run, where eps = 0.2 spans one
    # cell and details the paper leaves open matter: 2.16 here
    for k, want in PRINTED_RATE.items():
        assert abs(rates[k] - want) <= (0.15 if k == (32, 64) else 0.02), (k, rates[k], want)
    # from 32^2 on, the printed differences up to one common factor
    ratios = [deltas[k] / PRINTED[k] for k in keys if k[0] >= 32]
    print("delta / printed:", ["%.3f" % (deltas[k] / PRINTED[k]) for k in keys])
    assert max(ratios) / min(ratios) <= 1.03, ratios


def test_mass_of_51_is_conserved(runs):
    for n, r in runs.items():
        assert abs(r["mass"][0] + 5.12) <= 1e-12
        # |mass change| <= |Omega|^{1/2} ||R_phi|| <= L * tol per step
        assert np.max(np.abs(r["mass"] - r["mass"][0])) <= L * 1e-10 * r["steps"], n


def test_discrete_energy_F_is_non_increasing(runs):
    for n, r in runs.items():
        dF = np.diff(r["F"])
        assert np.all(dF <= 1e-9), (n, dF.max())


def test_cauchy_differences_with_the_papers_bilinear_interpolation(runs):
    """delta = phi_{h_f} - I phi_{h_c} with I bilinear onto the fine grid (the
    operator Section 5.1 names), h_f-weighted l2 norm: rates as printed and one
    common factor to the printed differences (about 4.9) at every N."""
    deltas = _bilinear_deltas({n: runs[n]["phi"] for n in SIZES})
    keys = sorted(deltas)
    rates = {b: math.log2(deltas[a] / deltas[b]) for a, b in zip(keys, keys[1:])}
    print("bilinear deltas:", ["%.4e" % deltas[k] for k in keys],
          "rates:", ["%.3f" % rates[k] for k in keys[1:]],
          "/ printed:", ["%.3f" % (deltas[k] / PRINTED[k]) for k in keys])
    for k, want in PRINTED_RATE.items():
        assert abs(rates[k] - want) <= 0.03, (k, rates[k], want)
    ratios = [deltas[k] / PRINTED[k] for k in keys]
    assert max(ratios) / min(ratios) <= 1.05, ratios


def test_first_order_start_does_not_move_the_cauchy_differences(chhs, runs):
    """The other first step of Remark 2.2 (a first-order step for phi^1 instead
    of phi^{-1} := phi^0) changes the Cauchy differences by under 2%: it is not
    what sets their level against the printed ones."""
    sizes = SIZES[1:5]
    alt = {n: _run(chhs, n, first_order_start=True) for n in sizes}
    base = {n: runs[n]["phi"] for n in sizes}
    for n in sizes[:-1]:
        a = _restrict(alt[2 * n]) - alt[n]
        b = _restrict(base[2 * n]) - base[n]
        da, db = math.sqrt(np.sum(a * a)), math.sqrt(np.sum(b * b))
        print(f"{n}->{2 * n}: delta with a first-order start / with phi^-1 = phi^0: {da / db:.4f}")
        assert abs(da / db - 1.0) <= 0.02, (n, da / db)
