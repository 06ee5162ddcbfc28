"""chhs_energy_mass_noalloc (no context, no allocation: partial sums in a
fixed device array of the library) against chhs_energy_mass, the context-based
entry point it is a variant of, through the C ABI.

Two calls in a row, the second with a smaller input, so that the second call
reuses the device array the first one filled; the results agree to the
rounding of the different summation order (the terms per cell are the same).
"""
import numpy as np
import pytest

from workloads import uniform_field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def chhs():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1611_02967_amd import chhs as binding
    return binding


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _case(chhs, shapes, seed):
    probs = [chhs.make_problem(sh, 1.0 / sh[-1], 0.02 + 0.01 * i, 1.0 + i, 1e-3)
             for i, sh in enumerate(shapes)]
    cur = np.concatenate([uniform_field(sh, seed + i, mean=0.1, amp=0.5).ravel()
                          for i, sh in enumerate(shapes)])
    prev = cur + np.concatenate([uniform_field(sh, seed + 50 + i, amp=0.05).ravel()
                                 for i, sh in enumerate(shapes)])
    return probs, _dev(cur), _dev(prev)


def _compare(chhs, probs, phi, prev):
    import torch
    out = torch.full((3 * len(probs),), np.nan, dtype=torch.float64, device="cuda")
    chhs.chhs_energy_mass_noalloc(probs, phi, prev, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(-1, 3)
    sv = chhs.Solver(probs)
    want = np.array(sv.energy_mass(phi, prev))
    sv.close()
    assert np.all(np.isfinite(got))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-14)
    return got


def test_noalloc_energies_equal_the_context_entry_point_twice(chhs):
    # a ragged batch whose largest instance needs the grid-stride loop (1024^2
    # cells over 256 blocks), then a smaller input on the same device array
    big = [(1024, 1024), (96, 128), (32, 32)]
    probs, phi, prev = _case(chhs, big, 6000)
    a = _compare(chhs, probs, phi, prev)
    small = [(64, 64)]
    probs2, phi2, prev2 = _case(chhs, small, 6100)
    b = _compare(chhs, probs2, phi2, prev2)
    assert a.shape == (3, 3) and b.shape == (1, 3)


def test_noalloc_energies_3d_twice(chhs):
    probs, phi, prev = _case(chhs, [(64, 64, 64), (16, 32, 32)], 6200)
    _compare(chhs, probs, phi, prev)
    probs2, phi2, prev2 = _case(chhs, [(16, 16, 16)], 6300)
    _compare(chhs, probs2, phi2, prev2)


def test_noalloc_rejects_sizes_beyond_its_limit(chhs):
    import torch
    p = chhs.make_problem((32, 32), 1 / 32, 0.05, 1.0, 1e-3)
    x = torch.zeros(32 * 32 * 33, dtype=torch.float64, device="cuda")
    out = torch.zeros(3 * 33, dtype=torch.float64, device="cuda")
    with pytest.raises(chhs.ChhsError):
        chhs.chhs_energy_mass_noalloc([p] * 33, x, x, out)      # more than 32 instances
    bad = chhs.make_problem((32, 32), 1 / 32, 0.0, 1.0, 1e-3)  # eps = 0
    with pytest.raises(chhs.ChhsError):
        chhs.chhs_energy_mass_noalloc([bad], x, x, out)
