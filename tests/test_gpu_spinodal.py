"""The spinodal decomposition runs of Section 5.2 on the GPU path.

L = 6.4, eps = 0.03, h = 6.4/512, s = 0.01, phi^0 = -0.05 + 0.05 (2r - 1) with
r i.i.d. uniform (two seeds), gamma in {0, 2, 4}, FAS V(2,2) to tol 1e-10,
500 steps (t = 5).  Checked for every seed: F_h non-increasing and mass
conserved for every gamma (Theorem 2.1, Section 4); gamma = 0 has no flow (p
stays constant, the flow dissipation is zero: the Cahn-Hilliard limit of
(2.7)); and, as the text of Section 5.2 reports for Figure 3, the energy decays
almost the same way for every gamma in the early stage of the decomposition,
the flow showing up later as faster dissipation for larger gamma.
"""
import numpy as np
import pytest

from workloads import uniform_field

pytestmark = pytest.mark.gpu

L, EPS, S, N, MEAN, STEPS = 6.4, 0.03, 0.01, 512, -0.05, 500
GAMMAS = (0.0, 2.0, 4.0)
SEEDS = (5200, 5201)


@pytest.fixture(scope="module")
def chhs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1611_02967_amd import chhs as binding
    return binding


@pytest.fixture(scope="module")
def runs(chhs):
    import torch
    h = L / N
    out = {}
    for seed in SEEDS:
        phi0 = uniform_field((N, N), seed, mean=MEAN, amp=0.05)
        for g in GAMMAS:
            sv = chhs.Solver(chhs.make_problem((N, N), h, EPS, g, S), chhs.chhs_default_opts(tol=1e-10))
            tp = torch.from_numpy(phi0).cuda()
            tc = tp.clone()
            tm = torch.zeros_like(tp)
            tpp = torch.zeros_like(tp)
            F, mass, du, pmax, cyc = [], [h * h * float(phi0.sum())], [], [], []
            for _ in range(STEPS):
                _, st = sv.step(tp, tc, tm, tpp, 1)
                F.append(st[0]["F_h"])
                mass.append(st[0]["mass"])
                du.append(st[0]["diss_u"])
                cyc.append(st[0]["vcycles"])
                pmax.append(float(tpp.abs().max()))
            out[seed, g] = dict(F=np.array(F), mass=np.array(mass), diss_u=np.array(du),
                                pmax=np.array(pmax), vcycles=float(np.mean(cyc)))
            print(f"seed {seed} gamma {g}: {np.mean(cyc):.2f} V-cycles/step, F_h {F[0]:.5f} -> {F[-1]:.5f}, "
                  f"F_h at t = 0.5, 1, 2, 3, 5: {F[49]:.5f} {F[99]:.5f} {F[199]:.5f} {F[299]:.5f} {F[499]:.5f}",
                  flush=True)
    return out


def test_energy_law_and_mass_for_every_gamma(runs):
    for key, r in runs.items():
        assert np.all(np.diff(r["F"]) <= 1e-9), (key, np.diff(r["F"]).max())
        assert np.max(np.abs(r["mass"] - r["mass"][0])) <= L * 1e-10 * STEPS, key


def test_gamma_zero_has_no_flow(runs):
    for seed in SEEDS:
        r = runs[seed, 0.0]
        assert np.all(r["diss_u"] == 0.0)
        # (2.7) with gamma = 0: the Neumann Laplacian of p vanishes, p is constant,
        # and the mean-zero normalisation makes it zero up to the iteration error
        assert np.max(r["pmax"]) <= 1e-6


def test_early_energy_decay_is_almost_gamma_independent(runs):
    """Up to t = 0.1 the energy curves of gamma = 2, 4 stay within 5% of the
    gamma = 0 curve's drop so far; the flow shows in the coarsening that
    follows, where larger gamma has dissipated more by t = 3 and t = 5, for
    every seed (Section 5.2: larger gamma improves the flow and enhances the
    energy dissipation)."""
    for seed in SEEDS:
        F0 = runs[seed, 0.0]["F"]
        for g in (2.0, 4.0):
            F = runs[seed, g]["F"]
            print(f"seed {seed} gamma {g}: F - F_(gamma=0) at steps 1, 2, 5, 10, 20, 50, 100, 300, 500:",
                  ["%.2e" % (F[k - 1] - F0[k - 1]) for k in (1, 2, 5, 10, 20, 50, 100, 300, 500)],
                  "F_(gamma=0) drop:", ["%.2e" % (F0[0] - F0[k - 1]) for k in (2, 5, 10, 20, 50)])
            for k in range(2, 11):
                assert abs(F[k - 1] - F0[k - 1]) <= 0.05 * (F0[0] - F0[k - 1]), (seed, g, k)
        for k in (300, 500):
            F4, F2 = runs[seed, 4.0]["F"][k - 1], runs[seed, 2.0]["F"][k - 1]
            assert F4 < F2 < F0[k - 1], (seed, k)
