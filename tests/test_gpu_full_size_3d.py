"""3D workloads at their full sizes on the GPU path.

* 256^3 FP64 (eps 0.02, gamma 2, s 5e-4, phi^0 = 0.1 + 0.05 (2r - 1)): one step
  satisfies the scheme (2.5)-(2.7) to tol -- the oracle's residual of the GPU
  output, evaluated in NumPy at full size -- conserves mass exactly as
  -(R_phi, 1) and obeys the exact energy balance behind Theorem 2.1.
* FP32 inner V-cycles with FP64 refinement at 256^3 and 512^3 (134 M cells)
  against the FP64 GPU path from the same state: max |phi_mixed - phi_fp64|
  after one step <= 1e-8 at the same residual tolerance.
"""
import numpy as np
import pytest

from oracle import grid, scheme
from workloads import WORKLOADS, uniform_field

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


def _step(chhs, n, w, phi0, precision):
    import torch
    prob = chhs.make_problem((n, n, n), 1.0 / n, w["eps"], w["gamma"], w["s"])
    sv = chhs.Solver(prob, chhs.chhs_default_opts(precision=precision, tol=1e-10))
    tp, tc = dev(phi0), dev(phi0)
    tm, tpp = torch.zeros_like(tp), torch.zeros_like(tp)
    _, st = sv.step(tp, tc, tm, tpp, 1)
    out = (tc, tm, tpp, st[0])
    sv.close()
    return out


def test_3d_256_fp64_step_satisfies_the_scheme(chhs):
    w = WORKLOADS["3d-256-fp64"]
    n = w["n"]
    prm = scheme.Params(eps=w["eps"], gamma=w["gamma"], s=w["s"], h=1.0 / n)
    phi0 = uniform_field((n, n, n), w["seed"], mean=w["mean"], amp=0.05)
    tc, tm, tpp, st = _step(chhs, n, w, phi0, 0)
    phi, mu, p = host(tc), host(tm), host(tpp)
    del tc, tm, tpp
    phi_star, f = scheme.step_rhs(phi0, phi0, prm)
    lvl = scheme.Level(h=prm.h, phi_star=phi_star, psi=phi0, f=f)
    r = scheme.residual([phi, mu, p], f, lvl, prm)
    res = scheme.residual_norm(r, prm.h)
    assert res <= 1.01e-10 and abs(res - st["res_norm"]) <= 1e-3 * res + 1e-15
    dm = grid.mass(phi, prm.h) - grid.mass(phi0, prm.h)
    assert abs(dm + grid.mass(r[0], prm.h)) <= 1e-13
    lhs, rhs = scheme.energy_identity_terms(phi, phi0, phi0, mu, p, prm)
    assert abs(lhs - rhs) <= 1e-9
    assert abs(p.mean()) <= 1e-13


@pytest.mark.parametrize("name", ["3d-256-mixed", "3d-512-mixed"])
def test_3d_mixed_full_size_matches_fp64_gpu_path(chhs, name):
    w = WORKLOADS[name]
    n = w["n"]
    phi0 = uniform_field((n, n, n), w["seed"], mean=w["mean"], amp=0.05)
    tc_m, _, _, st_m = _step(chhs, n, w, phi0, 1)
    phi_m = host(tc_m)
    del tc_m
    tc_d, _, _, st_d = _step(chhs, n, w, phi0, 0)
    phi_d = host(tc_d)
    del tc_d
    assert st_m["res_norm"] <= 1e-10 and st_d["res_norm"] <= 1e-10
    err = float(np.max(np.abs(phi_m - phi_d)))
    print(f"{name}: max |phi_mixed - phi_fp64| = {err:.3e}, refinement steps {st_m['vcycles']} "
          f"(residual {st_m['res_norm']:.2e}), FP64 V-cycles {st_d['vcycles']} "
          f"(residual {st_d['res_norm']:.2e})")
    assert err <= 1e-8
