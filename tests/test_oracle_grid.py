"""Pins for the oracle's discrete operators (Appendix A of the paper).

Closed forms (discrete Neumann eigenpairs), the ghost-point definitions of
App. A.1 evaluated by brute-force loops, and the summation-by-parts identities
of App. A.3.
"""
import itertools

import numpy as np
import pytest

from oracle import grid


def ghost_pad(v):
    """Ghost layer by the Neumann conditions eqn:nbc1-3: ghost = adjacent interior cell."""
    return np.pad(v, 1, mode="edge")


def brute_laplacian(v, h):
    """Delta_h by explicit loops over cells with ghost values (App. A.1-A.2)."""
    g = ghost_pad(v)
    out = np.zeros_like(v)
    for idx in itertools.product(*[range(n) for n in v.shape]):
        c = tuple(i + 1 for i in idx)
        acc = 0.0
        for ax in range(v.ndim):
            for step in (-1, 1):
                nb = list(c)
                nb[ax] += step
                acc += g[tuple(nb)] - g[c]
        out[idx] = acc / (h * h)
    return out


@pytest.mark.parametrize("shape", [(5, 7), (3, 4, 5)])
def test_laplacian_matches_ghost_point_definition(shape):
    rng = np.random.default_rng(0)
    v = rng.standard_normal(shape)
    h = 0.37
    np.testing.assert_allclose(grid.lap(v, h), brute_laplacian(v, h), rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape", [(6, 5), (3, 4, 5)])
def test_div_c_grad_matches_index_form(shape):
    """(div(c grad v))_I = h^-2 sum over faces c_f (v_J - v_I), boundary faces carrying no flux."""
    rng = np.random.default_rng(1)
    v = rng.standard_normal(shape)
    phis = rng.standard_normal(shape)
    h = 0.2
    c = grid.avg(phis)
    got = grid.div_c_grad(c, v, h)
    want = np.zeros_like(v)
    for idx in itertools.product(*[range(n) for n in shape]):
        for ax in range(len(shape)):
            for step in (-1, 1):
                nb = list(idx)
                nb[ax] += step
                if not 0 <= nb[ax] < shape[ax]:
                    continue  # boundary face: f = 0 (App. A.1)
                cf = 0.5 * (phis[idx] + phis[tuple(nb)])
                want[idx] += cf * (v[tuple(nb)] - v[idx]) / h ** 2
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,k", [(8, 1), (8, 3), (16, 5), (32, 31), (7, 2)])
def test_neumann_eigenpairs_1d_modes(n, k):
    """cos(k pi (i - 1/2)/N) is a discrete Neumann eigenfunction with eigenvalue
    -(4/h^2) sin^2(k pi / 2N), in each direction."""
    h = 1.0 / n
    x = np.cos(k * np.pi * (np.arange(1, n + 1) - 0.5) / n)
    lam = 4.0 / h ** 2 * np.sin(k * np.pi / (2 * n)) ** 2
    v2 = x[:, None] * np.ones(n)[None, :]
    np.testing.assert_allclose(grid.lap(v2, h), -lam * v2, rtol=0, atol=1e-9 * lam)


def test_neumann_eigenpairs_3d_product_mode():
    n = 12
    h = 0.5 / n
    ks = (1, 4, 7)
    vecs = [np.cos(k * np.pi * (np.arange(1, n + 1) - 0.5) / n) for k in ks]
    v = vecs[0][:, None, None] * vecs[1][None, :, None] * vecs[2][None, None, :]
    lam = sum(4.0 / h ** 2 * np.sin(k * np.pi / (2 * n)) ** 2 for k in ks)
    np.testing.assert_allclose(grid.lap(v, h), -lam * v, rtol=0, atol=1e-9 * lam)


@pytest.mark.parametrize("shape", [(9, 6), (4, 5, 6)])
def test_summation_by_parts(shape):
    """(phi, Lap psi) = -(grad phi, grad psi) and (phi, div u) = -(grad phi, u) (App. A.3)."""
    rng = np.random.default_rng(2)
    phi, psi = rng.standard_normal(shape), rng.standard_normal(shape)
    h = 0.1
    lhs = grid.ip(phi, grid.lap(psi, h), h)
    rhs = -grid.face_ip(grid.grad(phi, h), grid.grad(psi, h), h)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    u = [rng.standard_normal(g.shape) for g in grid.grad(phi, h)]   # u.n = 0 on the boundary
    lhs = grid.ip(phi, grid.div(u, h), h)
    rhs = -grid.face_ip(grid.grad(phi, h), u, h)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)


def test_face_inner_product_half_weights():
    """[f, g]_x summed cell by cell with weight 1/2 on each of the cell's two faces."""
    rng = np.random.default_rng(3)
    shape = (4, 6)
    h = 0.3
    fx = rng.standard_normal((4, 5))   # interior x-faces; boundary faces are zero
    gx = rng.standard_normal((4, 5))
    full_f = np.pad(fx, ((0, 0), (1, 1)))
    full_g = np.pad(gx, ((0, 0), (1, 1)))
    acc = 0.0
    for j in range(shape[0]):
        for i in range(shape[1]):
            acc += 0.5 * h ** 2 * (full_f[j, i + 1] * full_g[j, i + 1] + full_f[j, i] * full_g[j, i])
    fy = np.zeros((3, 6))
    assert abs(grid.face_ip([fy, fx], [fy, gx], h) - acc) < 1e-12


def test_grad_norm_of_eigenmode():
    """||grad_h v||^2 = lambda ||v||^2 for a Neumann eigenfunction (SBP + eigenpair)."""
    n = 16
    h = 1.0 / n
    k = 3
    x = np.cos(k * np.pi * (np.arange(1, n + 1) - 0.5) / n)
    v = np.outer(np.ones(n), x)
    lam = 4.0 / h ** 2 * np.sin(k * np.pi / (2 * n)) ** 2
    assert abs(grid.grad_norm2_sq(v, h) - lam * grid.ip(v, v, h)) < 1e-10 * lam
