"""GPU tests of the batched ragged path and of graph replay.

A batch of independent instances with different grids and parameters runs in
one launch per level (one tail workgroup per instance); every instance must
reproduce its own single-instance run bit for bit, and the oracle to the step
tolerance.  Replaying the captured V-cycle graph must equal eager launches bit
for bit.
"""
import numpy as np
import pytest

from oracle import fas, scheme
from workloads import batched_instances, uniform_field

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


# (shape, eps, gamma, s, mean): ragged sizes including a tail-only 32^2 grid,
# a rectangular grid and two sizes with several tiled levels
RAGGED_2D = [((128, 128), 0.02, 1.0, 1e-4, 0.0),
             ((32, 32), 0.05, 3.0, 5e-4, 0.2),
             ((96, 160), 0.03, 0.5, 1e-4, -0.1),
             ((256, 256), 0.01, 5.0, 5e-4, 0.3),
             ((64, 64), 0.05, 2.0, 1e-3, 0.0)]
RAGGED_3D = [((16, 16, 16), 0.05, 2.0, 5e-4, 0.1),
             ((8, 8, 8), 0.1, 1.0, 1e-3, 0.0),
             ((32, 16, 16), 0.04, 1.5, 5e-4, -0.1)]


def _pack(arrays):
    return np.concatenate([a.ravel() for a in arrays])


def _unpack(flat, shapes):
    out, o = [], 0
    for s in shapes:
        n = int(np.prod(s))
        out.append(flat[o:o + n].reshape(s))
        o += n
    return out


def _run_batch(chhs, spec, phi0s, nsteps, **opts):
    probs = [chhs.make_problem(sh, 1.0 / sh[-1], e, g, s) for sh, e, g, s, _ in spec]
    sv = chhs.Solver(probs, chhs.chhs_default_opts(**opts))
    tp, tc = dev(_pack(phi0s)), dev(_pack(phi0s))
    z = np.zeros(tp.numel())
    tm, tpp = dev(z), dev(z)
    hist = []
    for _ in range(nsteps):
        prev = host(tp)
        cur = host(tc)
        _, st = sv.step(tp, tc, tm, tpp, 1)
        hist.append((prev, cur, host(tc), host(tm), host(tpp), [s["vcycles"] for s in st]))
    return hist


@pytest.mark.parametrize("spec", [RAGGED_2D, RAGGED_3D], ids=["2d", "3d"])
def test_batch_equals_single_instance_runs_bitwise(chhs, spec):
    shapes = [s[0] for s in spec]
    phi0s = [uniform_field(sh, 3000 + i, mean=sp[4], amp=0.05) for i, (sh, sp) in
             enumerate(zip(shapes, spec))]
    batch = _run_batch(chhs, spec, phi0s, 3)
    for i, sp in enumerate(spec):
        single = _run_batch(chhs, [sp], [phi0s[i]], 3)
        for m in range(3):
            got = [_unpack(batch[m][k], shapes)[i] for k in (2, 3, 4)]
            want = [single[m][k] for k in (2, 3, 4)]
            for a, b in zip(got, want):
                assert np.array_equal(a, b.reshape(a.shape)), (i, m)
            assert batch[m][5][i] == single[m][5][0]


@pytest.mark.parametrize("spec", [RAGGED_2D, RAGGED_3D], ids=["2d", "3d"])
def test_batch_matches_oracle_per_instance(chhs, spec):
    """Per-step protocol for every instance: the oracle steps from the GPU's own
    (phi^{m-1}, phi^m) and both solve to tol 1e-10."""
    shapes = [s[0] for s in spec]
    phi0s = [uniform_field(sh, 3100 + i, mean=sp[4], amp=0.05) for i, (sh, sp) in
             enumerate(zip(shapes, spec))]
    batch = _run_batch(chhs, spec, phi0s, 2)
    for m in range(2):
        prevs = _unpack(batch[m][0], shapes)
        curs = _unpack(batch[m][1], shapes)
        phis = _unpack(batch[m][2], shapes)
        mus = _unpack(batch[m][3], shapes)
        ps = _unpack(batch[m][4], shapes)
        for i, (sh, e, g, s, _) in enumerate(spec):
            if m == 0:
                mu0, p0 = np.zeros(sh), np.zeros(sh)
            else:
                mu0 = _unpack(batch[m - 1][3], shapes)[i]
                p0 = _unpack(batch[m - 1][4], shapes)[i]
            prm = scheme.Params(eps=e, gamma=g, s=s, h=1.0 / sh[-1])
            r = fas.solve_step(prevs[i], curs[i], mu0, p0, prm, fas.Opts(tol=1e-10))
            assert r.vcycles == batch[m][5][i], (i, m)
            assert np.max(np.abs(phis[i] - r.phi)) <= 1e-10, (i, m)
            assert np.max(np.abs(mus[i] - r.mu)) <= 1e-9, (i, m)
            assert abs(ps[i].mean()) <= 1e-13


def _shifted(a):
    """A device copy of `a` that starts 8 bytes past a 16-byte boundary."""
    import torch
    buf = torch.empty(a.size + 1, dtype=torch.float64, device="cuda")
    t = buf[1:]
    t.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    assert t.data_ptr() % 16 == 8
    return t


@pytest.mark.parametrize("spec", [RAGGED_2D, RAGGED_3D], ids=["2d", "3d"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_caller_arrays_off_16_byte_alignment(chhs, spec, precision):
    """Caller arrays 8 bytes off a 16-byte boundary: the setup pass takes its
    one-cell-per-access form instead of x-adjacent pairs; both form every
    cell's values with the same operations, so the steps agree."""
    shapes = [s[0] for s in spec]
    phi0s = [uniform_field(sh, 3300 + i, mean=sp[4], amp=0.05) for i, (sh, sp) in
             enumerate(zip(shapes, spec))]
    flat = _pack(phi0s)
    out = []
    for make in (dev, _shifted):
        probs = [chhs.make_problem(sh, 1.0 / sh[-1], e, g, s) for sh, e, g, s, _ in spec]
        sv = chhs.Solver(probs, chhs.chhs_default_opts(precision=precision))
        tp, tc = make(flat), make(flat)
        tm, tpp = make(np.zeros(flat.size)), make(np.zeros(flat.size))
        steps = []
        for _ in range(2):
            _, st = sv.step(tp, tc, tm, tpp, 1)
            steps.append(([host(x).copy() for x in (tc, tm, tpp)], [x["vcycles"] for x in st]))
        out.append(steps)
    for (fa, ca), (fb, cb) in zip(*out):
        assert ca == cb
        for a, b in zip(fa, fb):
            assert np.max(np.abs(a - b)) <= 1e-12


@pytest.mark.parametrize("spec", [RAGGED_2D, RAGGED_3D], ids=["2d", "3d"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "mixed"])
def test_graph_replay_equals_eager_launches(chhs, spec, precision):
    """Cycles replayed from the two captured graphs (mixed precision: one per
    copy of the FP64 finest level, each reading back into its own mirror)
    equal direct launches bit for bit, with the same cycle counts."""
    shapes = [s[0] for s in spec]
    phi0s = [uniform_field(sh, 3200 + i, mean=sp[4], amp=0.05) for i, (sh, sp) in
             enumerate(zip(shapes, spec))]
    a = _run_batch(chhs, spec, phi0s, 3, use_graph=1, precision=precision)
    b = _run_batch(chhs, spec, phi0s, 3, use_graph=0, precision=precision)
    for m in range(3):
        for k in (2, 3, 4):
            assert np.array_equal(a[m][k], b[m][k]), (m, k)
        assert a[m][5] == b[m][5]


def test_batched_workload_instances_step(chhs):
    """Eight instances drawn by the ragged-batch recipe (sizes 128^2..1024^2,
    random eps, gamma, s, mean) take two steps in one batch; every instance
    converges and conserves mass to its residual."""
    insts = batched_instances(count=8)
    spec = [(it.shape, it.eps, it.gamma, it.s, it.mean) for it in insts]
    phi0s = [it.phi0() for it in insts]
    hist = _run_batch(chhs, spec, phi0s, 2)
    shapes = [s[0] for s in spec]
    for m in range(2):
        curs = _unpack(hist[m][1], shapes)
        phis = _unpack(hist[m][2], shapes)
        for i, it in enumerate(insts):
            h = 1.0 / it.shape[-1]
            dm = h * h * (phis[i].sum() - curs[i].sum())
            assert abs(dm) <= 1e-10
            assert 1 <= hist[m][5][i] <= 20
