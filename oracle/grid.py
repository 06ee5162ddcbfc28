"""Discrete operators on the cell-centred (MAC) grid -- Appendix A of the paper.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Conventions
-----------
* A cell-centred grid function is a NumPy array of shape ``(ny, nx)`` in 2D or
  ``(nz, ny, nx)`` in 3D holding the interior values only (App. A.1, the set
  C_N of cell centres (i - 1/2) h).  Axis ``ax`` of the array is a spatial
  direction; the last axis is x.
* Homogeneous Neumann data (App. A.1, the ghost-point conditions
  ``eqn:nbc1``-``eqn:nbc3``) mirror the first and last interior cell into the
  ghost cell, so every difference across a boundary face is zero.  Face
  functions that satisfy n.f = 0 (App. A.1) vanish on boundary faces; they are
  stored here on interior faces only: along axis ``ax`` a face array has
  ``n_ax - 1`` entries, entry ``i`` sitting between cells ``i`` and ``i + 1``.
* One spacing h in every direction (Section 2, first paragraph).
"""
import numpy as np


def dims(v):
    """Number of spatial dimensions of a cell-centred array."""
    return v.ndim


def face_diff(v, h, ax):
    """D_x v on interior x-faces: (v_{i+1} - v_i) / h (App. A.2, D_x)."""
    return np.diff(v, axis=ax) / h


def face_avg(v, ax):
    """A_x v on interior x-faces: (v_i + v_{i+1}) / 2 (App. A.2, A_x)."""
    n = v.shape[ax]
    lo = np.take(v, np.arange(0, n - 1), axis=ax)
    hi = np.take(v, np.arange(1, n), axis=ax)
    return 0.5 * (lo + hi)


def face_div(f, h, ax):
    """d_x f at cell centres, (f_{i+1/2} - f_{i-1/2}) / h (App. A.2, d_x).

    ``f`` holds interior faces; the two boundary faces carry zero, which is the
    face condition n.f = 0 of App. A.1.
    """
    pad = [(0, 0)] * f.ndim
    pad[ax] = (1, 1)
    return np.diff(np.pad(f, pad), axis=ax) / h


def grad(v, h):
    """nabla_h v = (D_x v, D_y v[, D_z v]) on interior faces (App. A.2)."""
    return [face_diff(v, h, ax) for ax in range(v.ndim)]


def avg(v):
    """A_h v = (A_x v, A_y v[, A_z v]) on interior faces (App. A.2, eq. face-average)."""
    return [face_avg(v, ax) for ax in range(v.ndim)]


def div(f, h):
    """nabla_h . f = sum_ax d_ax f^ax (App. A.2)."""
    return sum(face_div(f[ax], h, ax) for ax in range(len(f)))


def div_c_grad(c, v, h):
    """nabla_h . (c nabla_h v) for a face coefficient ``c`` (list over axes).

    This is the composite operator of (2.5)-(2.7): the face product c D v
    followed by d_ax, summed over axes.
    """
    return sum(face_div(c[ax] * face_diff(v, h, ax), h, ax) for ax in range(v.ndim))


def lap(v, h):
    """Delta_h v = nabla_h . nabla_h v (App. A.2)."""
    return sum(face_div(face_diff(v, h, ax), h, ax) for ax in range(v.ndim))


def ip(u, v, h):
    """Cell inner product (u, v) = h^d sum u v (App. A.2)."""
    return float(h ** u.ndim * np.sum(u * v))


def face_ip(f, g, h):
    """Face inner product (f, g) = sum_ax [f^ax, g^ax]_ax (App. A.2).

    [f, g]_x gives each interior face weight h^d (it is counted from both
    neighbouring cells with weight 1/2) and each boundary face weight h^d / 2.
    The face functions handled here vanish on boundary faces, so only the
    interior faces contribute.  The printed definition repeats [f^y, g^y] in its
    third term; the z term is meant.
    """
    d = f[0].ndim
    return float(h ** d * sum(np.sum(f[ax] * g[ax]) for ax in range(len(f))))


def norm2(v, h):
    """Discrete l2 norm ||v||_2 = (v, v)^(1/2) (App. A.2, eq. discrete norm-lp)."""
    return ip(v, v, h) ** 0.5


def norm4_4(v, h):
    """||v||_4^4 = (|v|^4, 1) (App. A.2, eq. discrete norm-lp with p = 4)."""
    return float(h ** v.ndim * np.sum(v ** 4))


def grad_norm2_sq(v, h):
    """||nabla_h v||_2^2 = (nabla_h v, nabla_h v) (App. A.2, eq. inner product-def 2)."""
    g = grad(v, h)
    return face_ip(g, g, h)


def mass(v, h):
    """(v, 1): the discrete mass (Section 4, mass conservation)."""
    return float(h ** v.ndim * np.sum(v))
