"""Synthetic initial data and workload definitions (all on a box (0, L)^d).

Random fields follow the spinodal-decomposition recipe of Section 5.2: a mean
composition plus 0.05 (2 r - 1) with r i.i.d. uniform on [0, 1) per cell.  The
paper gives no generator or seed; here r comes from NumPy's PCG64 with an
explicit seed, drawn in C order over an array of shape (ny, nx) or (nz, ny, nx)
(x fastest), in float64.

Closed-form fields are sampled at cell centres x_i = (i - 1/2) h.
"""
from dataclasses import dataclass

import numpy as np


def uniform_field(shape, seed, mean=0.0, amp=0.05):
    """mean + amp (2 r - 1), r ~ U[0, 1) i.i.d. per cell, PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return mean + amp * (2.0 * rng.random(shape) - 1.0)


def cosine_mode(shape, k, mean, amp):
    """mean + amp cos(pi k (i + 1/2) / nx) along x (the last axis), constant
    along the other axes: a single cosine mode of the cell-centred Neumann grid."""
    nx = shape[-1]
    v = np.cos(np.pi * k * (np.arange(nx) + 0.5) / nx)
    return mean + amp * np.broadcast_to(v, shape).copy()


def _centres(n, length):
    h = length / n
    return (np.arange(n) + 0.5) * h


def smooth_ic_2d(n, length=1.0):
    """0.24 cos(2 pi x) cos(2 pi y) + 0.4 cos(pi x) cos(3 pi y) on (0, 1)^2, shape (n, n).

    Every term has zero normal derivative on the boundary of (0, 1)^2.
    """
    x = _centres(n, length)
    y = x[:, None]
    xx = x[None, :]
    return (0.24 * np.cos(2 * np.pi * xx) * np.cos(2 * np.pi * y)
            + 0.4 * np.cos(np.pi * xx) * np.cos(3 * np.pi * y))


def paper_ic_51(n, length=3.2):
    """Initial condition (5.1): [1 - cos(4 pi x / L)][1 - cos(2 pi y / L)] / 2 - 1, shape (n, n)."""
    x = _centres(n, length)
    y = x[:, None]
    xx = x[None, :]
    return ((1.0 - np.cos(4 * np.pi * xx / length))
            * (1.0 - np.cos(2 * np.pi * y / length)) / 2.0 - 1.0)


@dataclass
class Instance:
    """One independent problem: grid extent per direction, spacing, parameters, data."""
    shape: tuple
    h: float
    eps: float
    gamma: float
    s: float
    mean: float
    seed: int

    def phi0(self):
        return uniform_field(self.shape, self.seed, mean=self.mean, amp=0.05)


def batched_instances(count=64, seed=2971, sizes=(128, 256, 512, 1024)):
    """Ragged batch of independent 2D instances on (0, 1)^2.

    Instance i: N_i = sizes[i mod len(sizes)], eps ~ U[0.01, 0.05],
    gamma ~ U[0.5, 5], s in {1e-4, 5e-4} by a fair coin, mean m ~ U[-0.3, 0.3],
    phi0 = m + 0.05 (2 r - 1) with the field seed ``seed + i``.  The parameter
    draws use PCG64(seed) in the order (eps, gamma, coin, m) per instance.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        eps = 0.01 + 0.04 * rng.random()
        gamma = 0.5 + 4.5 * rng.random()
        s = 1e-4 if rng.random() < 0.5 else 5e-4
        m = -0.3 + 0.6 * rng.random()
        n = sizes[i % len(sizes)]
        out.append(Instance(shape=(n, n), h=1.0 / n, eps=eps, gamma=gamma, s=s,
                            mean=m, seed=seed + i))
    return out


# Named workloads.  Seeds are 2967 + a per-workload offset.
WORKLOADS = {
    # 2D, 64^2, CPU-size: full run in the oracle.
    "2d-64-fp64": dict(dim=2, n=64, eps=0.05, gamma=1.0, s=1e-3, steps=20,
                       mean=0.0, seed=2967),
    # 2D spinodal on the GPU, 1024^2 and 2048^2.
    "2d-1024-fp64": dict(dim=2, n=1024, eps=0.01, gamma=1.0, s=1e-4, steps=500,
                         mean=0.0, seed=2968),
    "2d-2048-fp64": dict(dim=2, n=2048, eps=0.01, gamma=1.0, s=1e-4, steps=500,
                         mean=0.0, seed=2968),
    # 3D, off-critical quench.
    "3d-128-fp64": dict(dim=3, n=128, eps=0.02, gamma=2.0, s=5e-4, steps=100,
                        mean=0.1, seed=2969),
    "3d-256-fp64": dict(dim=3, n=256, eps=0.02, gamma=2.0, s=5e-4, steps=100,
                        mean=0.1, seed=2969),
    # 3D, FP32 sweeps with FP64 refinement.
    "3d-256-mixed": dict(dim=3, n=256, eps=0.02, gamma=2.0, s=5e-4, steps=100,
                         mean=0.1, seed=2970),
    "3d-512-mixed": dict(dim=3, n=512, eps=0.02, gamma=2.0, s=5e-4, steps=100,
                         mean=0.1, seed=2970),
}


def workload_field(name, n=None):
    """Initial phi of a named workload (optionally at another resolution n)."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    shape = (n,) * w["dim"]
    return uniform_field(shape, w["seed"], mean=w["mean"], amp=0.05)
