"""The per-step result by its plain definition: Newton's method on the whole system.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Theorem 2.1 makes phi^{m+1} (and with it mu^{m+1/2}) the unique solution of
(2.5)-(2.7), and p^{m+1/2} unique up to a constant.  This module computes that
solution without any multigrid: it writes the three equations in index form,
one row per cell, with every operator assembled face by face
as a sparse matrix,

    (div(c grad v))_I = h^-2 sum over interior faces f=(I,J) of c_f (v_J - v_I)

(App. A.2 with the zero boundary fluxes of App. A.1), and runs Newton's method
with the exact Jacobian and a direct solve.  The constant in p is fixed by
bordering the Jacobian with the constraint sum(p) = 0: the p-rows of the
Jacobian sum to zero column-wise (their left null vector is the indicator of the
p unknowns), so the bordered matrix is nonsingular.

Nothing here calls ``oracle.grid``: stencils are re-derived from the index
form, so a mistake in the array-shift operators used by ``oracle.fas`` cannot
hide in both.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _faces(shape):
    """All interior faces as (I, J) flat index pairs, I the lower cell, in C order."""
    n = int(np.prod(shape))
    idx = np.arange(n).reshape(shape)
    pairs = []
    for ax in range(len(shape)):
        lo = np.take(idx, np.arange(0, shape[ax] - 1), axis=ax).ravel()
        hi = np.take(idx, np.arange(1, shape[ax]), axis=ax).ravel()
        pairs.append((lo, hi))
    return pairs


def face_weights(shape, values, fn):
    """Evaluate fn(v_I, v_J) on every interior face, in the order of ``_faces``."""
    v = values.ravel()
    return [fn(v[lo], v[hi]) for lo, hi in _faces(shape)]


def assemble_div_c_grad(shape, h, weights):
    """Sparse matrix of v -> div_h(c grad_h v) with face coefficients ``weights``.

    Each interior face (I, J) with coefficient c adds c/h^2 (v_J - v_I) to row I
    and c/h^2 (v_I - v_J) to row J.  Boundary faces add nothing (zero flux).
    """
    n = int(np.prod(shape))
    rows, cols, vals = [], [], []
    for (lo, hi), c in zip(_faces(shape), weights):
        c = np.broadcast_to(np.asarray(c, dtype=np.float64), lo.shape) / (h * h)
        # entries (I,J) +c, (I,I) -c, (J,I) +c, (J,J) -c for every face at once
        rows += [lo, lo, hi, hi]
        cols += [hi, lo, lo, hi]
        vals += [c, -c, c, -c]
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


class System:
    """The nonlinear system of one step, (2.5)-(2.7), in index form."""

    def __init__(self, phi_prev, phi_cur, eps, gamma, s, h):
        self.shape = phi_cur.shape
        self.n = int(np.prod(self.shape))
        self.eps, self.gamma, self.s, self.h = eps, gamma, s, h
        phi_star = 1.5 * phi_cur - 0.5 * phi_prev                       # (2.4)
        a = face_weights(self.shape, phi_star, lambda x, y: 0.5 * (x + y))   # A_h phi_*
        m = [1.0 + gamma * af * af for af in a]                              # M(A_h phi_*)
        one = [np.ones_like(af) for af in a]
        self.L1 = assemble_div_c_grad(self.shape, h, one)                    # Delta_h
        self.La = assemble_div_c_grad(self.shape, h, a)
        self.LM = assemble_div_c_grad(self.shape, h, m)
        self.psi = phi_cur.ravel().copy()
        # right-hand side of (2.5)-(2.7); the pressure row is multiplied by s
        self.f = np.concatenate([
            phi_cur.ravel(),
            -phi_star.ravel() - 0.25 * eps * eps * (self.L1 @ phi_prev.ravel()),
            np.zeros(self.n)])

    def apply(self, x):
        """N(x) for x = [phi; mu; p] stacked."""
        n, s, g, e2 = self.n, self.s, self.gamma, self.eps ** 2
        phi, mu, p = x[:n], x[n:2 * n], x[2 * n:]
        psi = self.psi
        chi = 0.25 * (phi * phi + psi * psi) * (phi + psi)
        return np.concatenate([
            phi - s * (self.LM @ mu) - s * (self.La @ p),
            mu - chi + 0.75 * e2 * (self.L1 @ phi),
            s * (self.L1 @ p) + s * g * (self.La @ mu)])

    def jacobian(self, x):
        """Exact Jacobian of ``apply`` at x."""
        n, s, g, e2 = self.n, self.s, self.gamma, self.eps ** 2
        phi, psi = x[:n], self.psi
        dchi = 0.25 * (3.0 * phi * phi + 2.0 * phi * psi + psi * psi)
        eye = sp.identity(n, format="csr")
        return sp.bmat([
            [eye, -s * self.LM, -s * self.La],
            [-sp.diags(dchi) + 0.75 * e2 * self.L1, eye, None],
            [None, s * g * self.La, s * self.L1]], format="csr")

    def res_norm(self, r):
        """h^d-weighted l2 norm over all three components (App. A.2)."""
        return float(np.sqrt(self.h ** len(self.shape) * np.dot(r, r)))


def solve(phi_prev, phi_cur, eps, gamma, s, h, mu0=None, p0=None,
          tol=1e-14, max_iter=40, dense_below=2000):
    """Newton's method with a direct solve; returns (phi, mu, p, residual norms).

    The initial guess is (phi^m, mu0, p0) (zeros when not given).  Iterates until
    the residual norm is below ``tol`` or stops decreasing.  p is returned with
    mean zero.
    """
    sysm = System(phi_prev, phi_cur, eps, gamma, s, h)
    n = sysm.n
    x = np.concatenate([phi_cur.ravel(),
                        np.zeros(n) if mu0 is None else mu0.ravel(),
                        np.zeros(n) if p0 is None else p0.ravel()])
    x[2 * n:] -= np.mean(x[2 * n:])
    border = np.zeros(3 * n)
    border[2 * n:] = 1.0
    hist = []
    for _ in range(max_iter):
        r = sysm.f - sysm.apply(x)
        hist.append(sysm.res_norm(r))
        if hist[-1] < tol or (len(hist) > 3 and hist[-1] >= hist[-2] and hist[-1] < 1e3 * tol):
            break
        jac = sysm.jacobian(x)
        big = sp.bmat([[jac, sp.csr_matrix(border[:, None])],
                       [sp.csr_matrix(border[None, :]), None]], format="csc")
        rhs = np.concatenate([r, [-np.sum(x[2 * n:])]])
        if 3 * n + 1 <= dense_below:
            dx = np.linalg.solve(big.toarray(), rhs)
        else:
            dx = spla.spsolve(big, rhs)
        x = x + dx[:3 * n]
    shape = phi_cur.shape
    phi, mu, p = (x[k * n:(k + 1) * n].reshape(shape).copy() for k in range(3))
    return phi, mu, p - np.mean(p), hist
