"""Pins for the oracle's scheme pieces: chi, the energies and the printed mass."""
import os

import numpy as np
import pytest

from oracle import grid, scheme
from workloads import paper_ic_51, smooth_ic_2d

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if line:
                rows.append(line)
    return rows


@pytest.mark.parametrize("n", [4, 8, 32, 512])
def test_mass_of_initial_condition_51(n):
    """Section 5.1 prints the initial mass of (5.1) at L = 3.2 as -5.12."""
    (length, mass), = [(float(a), float(b)) for a, b in _golden_rows("ic51_mass.txt")]
    h = length / n
    assert abs(grid.mass(paper_ic_51(n, length), h) - mass) < 1e-12


@pytest.mark.parametrize("n", [8, 64, 1024])
def test_mass_of_smooth_initial_field_is_zero(n):
    assert abs(grid.mass(smooth_ic_2d(n), 1.0 / n)) < 1e-13


def test_chi_satisfies_convex_term_identity():
    """(a - b) chi(a, b) = (a^4 - b^4)/4: the exact evaluation of I_1 in the proof of Thm 2.1."""
    rng = np.random.default_rng(0)
    a, b = rng.standard_normal(1000), rng.standard_normal(1000)
    np.testing.assert_allclose((a - b) * scheme.chi(a, b), 0.25 * (a ** 4 - b ** 4), rtol=1e-12, atol=1e-12)


def test_dchi_is_derivative_and_nonnegative():
    rng = np.random.default_rng(1)
    a, b = 2 * rng.standard_normal(500), 2 * rng.standard_normal(500)
    d = 1e-6
    fd = (scheme.chi(a + d, b) - scheme.chi(a - d, b)) / (2 * d)
    np.testing.assert_allclose(scheme.dchi(a, b), fd, rtol=1e-8, atol=1e-8)
    assert np.all(scheme.dchi(a, b) >= 0.0)


def test_energy_of_constant_state():
    """E_h(c) = |Omega| (c^4/4 - c^2/2): the gradient term vanishes."""
    prm = scheme.Params(eps=0.3, gamma=1.0, s=1.0, h=0.25)
    c = 0.7
    phi = np.full((8, 4), c)
    area = 8 * 4 * prm.h ** 2
    assert abs(scheme.energy_E(phi, prm) - area * (c ** 4 / 4 - c ** 2 / 2)) < 1e-14


def test_energy_of_single_mode():
    """For phi = A cos-mode: ||phi||_2^2 = A^2 |Omega|/2 (N > k), ||grad phi||^2 = lam ||phi||^2."""
    n, k, amp = 32, 3, 0.2
    h = 1.0 / n
    eps = 0.05
    prm = scheme.Params(eps=eps, gamma=1.0, s=1.0, h=h)
    x = np.cos(k * np.pi * (np.arange(1, n + 1) - 0.5) / n)
    phi = amp * np.outer(np.ones(n), x)
    lam = 4.0 / h ** 2 * np.sin(k * np.pi / (2 * n)) ** 2
    l2 = amp ** 2 / 2.0
    l4 = amp ** 4 * 3.0 / 8.0     # mean of cos^4 over a full set of cell centres
    want = 0.25 * l4 - 0.5 * l2 + 0.5 * eps ** 2 * lam * l2
    assert abs(scheme.energy_E(phi, prm) - want) < 1e-14


def test_energy_F_reduces_to_E_for_equal_arguments():
    rng = np.random.default_rng(4)
    phi = rng.standard_normal((10, 10))
    prm = scheme.Params(eps=0.1, gamma=1.0, s=1.0, h=0.1)
    assert scheme.energy_F(phi, phi, prm) == scheme.energy_E(phi, prm)
    psi = phi + 0.1
    # a constant shift has zero gradient: only the 1/4 ||phi - psi||^2 term is added
    assert abs(scheme.energy_F(phi, psi, prm) - scheme.energy_E(phi, prm) - 0.25 * 0.01 * 1.0) < 1e-13


def test_rhs_of_constant_history():
    """phi^{m-1} = phi^m = c: phi_* = c and f_mu = -c (the Laplacian of a constant is 0)."""
    prm = scheme.Params(eps=0.2, gamma=1.0, s=0.1, h=0.1)
    c = np.full((6, 6), -0.4)
    phi_star, f = scheme.step_rhs(c, c, prm)
    np.testing.assert_allclose(phi_star, -0.4, rtol=0, atol=1e-15)
    np.testing.assert_allclose(f[1], 0.4, rtol=0, atol=1e-15)
    assert np.all(f[2] == 0.0)
