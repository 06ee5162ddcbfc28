"""GPU tests of the mixed-precision path (FP32 correction-form V-cycles inside
FP64 residual + correction + reductions, iterative refinement).

The refined solution solves the FP64 system (2.5)-(2.7) to the same residual
tolerance as the plain path, so it must agree with the FP64 oracle (and with the
FP64 GPU path) to <= 1e-8 max-abs in phi at tol 1e-10, and it must reach
residuals far below FP32 precision.
"""
import numpy as np
import pytest

from oracle import fas, grid, scheme
from workloads import uniform_field

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


def _steps(chhs, spec, phi0s, nsteps, **opts):
    probs = [chhs.make_problem(sh, 1.0 / sh[-1], e, g, s) for sh, e, g, s in spec]
    sv = chhs.Solver(probs, chhs.chhs_default_opts(**opts))
    tp, tc = dev(_pack(phi0s)), dev(_pack(phi0s))
    z = np.zeros(tp.numel())
    tm, tpp = dev(z), dev(z)
    hist = []
    for _ in range(nsteps):
        prev, cur, mu_in, p_in = host(tp), host(tc), host(tm), host(tpp)
        _, st = sv.step(tp, tc, tm, tpp, 1)
        hist.append(dict(prev=prev, cur=cur, mu_in=mu_in, p_in=p_in, phi=host(tc), mu=host(tm),
                         p=host(tpp), stats=st))
    return hist


SPECS = {
    "2d-64": [((64, 64), 0.05, 1.0, 1e-3)],
    "2d-ragged": [((128, 128), 0.02, 1.0, 1e-4), ((96, 160), 0.03, 2.0, 5e-4),
                  ((32, 32), 0.05, 3.0, 5e-4)],
    "3d-16": [((16, 16, 16), 0.05, 2.0, 5e-4)],
    "3d-ragged": [((32, 32, 32), 0.04, 2.0, 5e-4), ((16, 16, 32), 0.05, 1.0, 1e-3)],
}


@pytest.mark.parametrize("name", list(SPECS))
def test_mixed_matches_fp64_oracle_per_step(chhs, name):
    spec = SPECS[name]
    shapes = [s[0] for s in spec]
    phi0s = [uniform_field(sh, 4000 + i, mean=0.1, amp=0.05) for i, sh in enumerate(shapes)]
    hist = _steps(chhs, spec, phi0s, 3, precision=1, tol=1e-10)
    for h in hist:
        prevs, curs = _unpack(h["prev"], shapes), _unpack(h["cur"], shapes)
        mus_in, ps_in = _unpack(h["mu_in"], shapes), _unpack(h["p_in"], shapes)
        phis = _unpack(h["phi"], shapes)
        for i, (sh, e, g, s) in enumerate(spec):
            assert h["stats"][i]["res_norm"] <= 1e-10
            prm = scheme.Params(eps=e, gamma=g, s=s, h=1.0 / sh[-1])
            r = fas.solve_step(prevs[i], curs[i], mus_in[i], ps_in[i], prm, fas.Opts(tol=1e-10))
            assert np.max(np.abs(phis[i] - r.phi)) <= 1e-8, (name, i)


@pytest.mark.parametrize("shape", [(256, 256), (64, 64, 64)])
def test_mixed_matches_fp64_gpu_path(chhs, shape):
    spec = [(shape, 0.02, 2.0, 5e-4)]
    phi0s = [uniform_field(shape, 4100, mean=0.1, amp=0.05)]
    a = _steps(chhs, spec, phi0s, 2, precision=1, tol=1e-10)
    b = _steps(chhs, spec, phi0s, 2, precision=0, tol=1e-10)
    for ha, hb in zip(a, b):
        assert np.max(np.abs(ha["phi"] - hb["phi"])) <= 1e-8


def test_refinement_reaches_below_fp32_precision(chhs):
    """tol 1e-12 (well below FP32 roundoff of the O(1) fields): the FP64 outer
    residual drives the error down, and the result is the oracle's to 1e-11."""
    shape = (64, 64)
    spec = [(shape, 0.05, 1.0, 1e-3)]
    phi0 = uniform_field(shape, 4200, amp=0.05)
    h = _steps(chhs, spec, [phi0], 1, precision=1, tol=1e-12)[0]
    assert h["stats"][0]["res_norm"] <= 1e-12
    prm = scheme.Params(eps=0.05, gamma=1.0, s=1e-3, h=1.0 / 64)
    z = np.zeros(shape)
    r = fas.solve_step(phi0, phi0, z, z, prm, fas.Opts(tol=1e-13))
    assert np.max(np.abs(h["phi"].reshape(shape) - r.phi)) <= 1e-11
    # mass: (phi^{m+1},1) - (phi^m,1) = -(R_phi,1) exactly, |.| <= ||R_phi||
    assert abs(grid.mass(h["phi"].reshape(shape), prm.h) - grid.mass(phi0, prm.h)) <= 1e-12


def test_mixed_graph_replay_equals_eager(chhs):
    spec = SPECS["2d-ragged"]
    shapes = [s[0] for s in spec]
    phi0s = [uniform_field(sh, 4300 + i, mean=0.1, amp=0.05) for i, sh in enumerate(shapes)]
    a = _steps(chhs, spec, phi0s, 2, precision=1, use_graph=1)
    b = _steps(chhs, spec, phi0s, 2, precision=1, use_graph=0)
    for ha, hb in zip(a, b):
        for k in ("phi", "mu", "p"):
            assert np.array_equal(ha[k], hb[k])


@pytest.mark.parametrize("name", ["2d-ragged", "3d-ragged"])
def test_mixed_batch_equals_single_instance_runs(chhs, name):
    """Instances of a mixed-precision batch converge after different numbers
    of refinement steps; one that has converged must keep its iterate while the
    others go on (the finest FP64 level alternates between two copies each
    refinement step).  Every instance of the batch equals its own single run
    bitwise, step by step, with the same refinement count."""
    spec = SPECS[name]
    shapes = [s[0] for s in spec]
    phi0s = [uniform_field(sh, 4400 + i, mean=0.1, amp=0.05) for i, sh in enumerate(shapes)]
    batch = _steps(chhs, spec, phi0s, 3, precision=1)
    counts = set()
    for i in range(len(spec)):
        single = _steps(chhs, [spec[i]], [phi0s[i]], 3, precision=1)
        for hb, hs in zip(batch, single):
            for k in ("phi", "mu", "p"):
                assert np.array_equal(_unpack(hb[k], shapes)[i], hs[k].reshape(shapes[i])), (i, k)
            assert hb["stats"][i]["vcycles"] == hs["stats"][0]["vcycles"]
            counts.add(hb["stats"][i]["vcycles"])
    assert len(counts) > 1       # the instances do converge after different counts


@pytest.mark.parametrize("name", ["2d-ragged", "3d-ragged"])
@pytest.mark.parametrize("inner", [2, 3])
def test_inner_cycles_solve_the_same_steps(chhs, name, inner):
    """Several FP32 correction cycles per FP64 refinement: the stopping test
    runs less often, the solution is the FP64 one (<= 1e-8 against the FP64
    path, residual at tol), with no more refinements than one inner cycle
    needs, and the batch still equals its single-instance runs bitwise."""
    spec = SPECS[name]
    shapes = [s[0] for s in spec]
    phi0s = [uniform_field(sh, 4500 + i, mean=0.1, amp=0.05) for i, sh in enumerate(shapes)]
    ref = _steps(chhs, spec, phi0s, 3, precision=0)
    one = _steps(chhs, spec, phi0s, 3, precision=1)
    got = _steps(chhs, spec, phi0s, 3, precision=1, inner_cycles=inner)
    for hr, ho, hg in zip(ref, one, got):
        assert np.max(np.abs(hg["phi"] - hr["phi"])) <= 1e-8
        for sg, so in zip(hg["stats"], ho["stats"]):
            assert sg["res_norm"] <= 1e-10
            assert sg["vcycles"] <= so["vcycles"]
    single = _steps(chhs, [spec[0]], [phi0s[0]], 3, precision=1, inner_cycles=inner)
    for hg, hs in zip(got, single):
        for k in ("phi", "mu", "p"):
            assert np.array_equal(_unpack(hg[k], shapes)[0], hs[k].reshape(shapes[0])), k


# 256 x 256 and 96 x 160: blocks whose whole region lies inside the grid
# (the interior form of the tile body) next to blocks at the grid's edges
TILE_SPECS = {"2d-64": SPECS["2d-64"], "2d-ragged": SPECS["2d-ragged"],
              "2d-interior": [((256, 256), 0.02, 1.0, 1e-4), ((96, 160), 0.03, 2.0, 5e-4)]}


@pytest.mark.parametrize("name", list(TILE_SPECS))
def test_tall_finest_tiles_solve_the_same_steps(chhs, name):
    """Tiles on every level (smoother = 1), the FP32 finest level in 64 x 16
    or 64 x 32 tiles (tile_rows = 32), against row-streaming strips on the
    FP32 finest level (smoother = 2) and the FP64 path: the same FP64 solution
    (<= 1e-8, residual at tol), refinement counts within one, and batch =
    single runs bitwise."""
    spec = TILE_SPECS[name]
    shapes = [s[0] for s in spec]
    phi0s = [uniform_field(sh, 4600 + i, mean=0.1, amp=0.05) for i, sh in enumerate(shapes)]
    ref = _steps(chhs, spec, phi0s, 3, precision=0)
    strips = _steps(chhs, spec, phi0s, 3, precision=1, smoother=2)
    base = _steps(chhs, spec, phi0s, 3, precision=1, smoother=1)
    tall = _steps(chhs, spec, phi0s, 3, precision=1, smoother=1, tile_rows=32)
    for hr, hs, hb, ht in zip(ref, strips, base, tall):
        for h in (hb, ht):
            assert np.max(np.abs(h["phi"] - hr["phi"])) <= 1e-8
            assert np.max(np.abs(h["phi"] - hs["phi"])) <= 1e-8
            for st, ss in zip(h["stats"], hs["stats"]):
                assert st["res_norm"] <= 1e-10
                assert abs(st["vcycles"] - ss["vcycles"]) <= 1
    if len(spec) > 1:
        single = _steps(chhs, [spec[0]], [phi0s[0]], 3, precision=1, smoother=1, tile_rows=32)
        for ht, hs in zip(tall, single):
            for k in ("phi", "mu", "p"):
                assert np.array_equal(_unpack(ht[k], shapes)[0], hs[k].reshape(shapes[0])), k


def test_fp64_smoothing_refuses_tall_tiles(chhs):
    """A mixed-precision context whose finest level is cut into 64 x 32 tiles
    (FP32 kernels only) refuses chhs_smooth there (the FP64 tile kernels have
    no such form) and still smooths the coarse levels."""
    prob = chhs.make_problem((128, 128), 1.0 / 128, 0.05, 1.0, 1e-3)
    sv = chhs.Solver(prob, chhs.chhs_default_opts(precision=1, smoother=1, tile_rows=32))
    phi = uniform_field((128, 128), 4700, amp=0.1).ravel()
    sv.setup_step(dev(phi), dev(phi), dev(np.zeros(phi.size)), dev(np.zeros(phi.size)))
    with pytest.raises(chhs.ChhsError):
        sv.smooth(0, 1)
    sv.smooth(1, 1)
