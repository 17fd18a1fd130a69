"""FP64 reference of the p-multigrid preconditioner of Ex. 5 (Section 5.3,
Ex. linear conv2): a V-cycle over polynomial orders N_0 > N_1 > ... on one
hexahedral mesh, each level the screened Poisson operator rediscretised at
its order (oracle.hexop.HexMesh), smoothed by a Chebyshev-accelerated Jacobi
polynomial, with a polynomial coarse solve on the lowest order.

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
preconditioner.

Definitions (level l, unknowns = interior grid nodes of order N_l):
* D_l = diag(A_l); rho_l = the largest eigenvalue of D_l^{-1} A_l.
* Smoother S_l = s(D_l^{-1} A_l) D_l^{-1}: the Chebyshev iteration of degree
  m for D^{-1} A x = D^{-1} f from x = 0 on the interval
  [lo_ratio rho_l, hi_margin rho_l], i.e. 1 - t s(t) is the scaled
  Chebyshev polynomial T_m((theta - t) / delta) / T_m(theta / delta).
* Prolongation P_l (level l+1 -> l): the coarse function evaluated at the
  fine nodes.  It is continuous, so every element that holds a fine node
  gives it the same value; P_l is assembled from the 1-D interpolation
  matrices J[a, b] = l_b(x_a) (coarse Lagrange basis at fine GLL points) by
  assignment.  Restriction R_l = P_l^T.
* Coarse solve C (lowest level): the same Chebyshev-Jacobi polynomial with
  degree coarse_degree on [coarse_lo_ratio rho, hi_margin rho].
* V-cycle for f on level l: x = S f; x += P V_{l+1}(P^T (f - A x));
  x += S (f - A x).  Its error propagator is
  (I - S A)(I - P V P^T A)(I - S A), symmetric in the A inner product, so
  the cycle is a symmetric preconditioner.

The paper's coarse solver is algebraic multigrid; a fixed Chebyshev
polynomial stands in for it here (linear and symmetric, so PCG's theory
holds, but weaker on large coarse problems).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import Polynomial

from .hexop import HexMesh, gll


def interp_matrix(Nf: int, Nc: int) -> np.ndarray:
    """J[a, b] = l_b(x_a): the order-Nc Lagrange basis on its GLL points,
    evaluated at the order-Nf GLL points (monomial form of each l_b)."""
    xf, _ = gll(Nf)
    xc, _ = gll(Nc)
    J = np.empty((Nf + 1, Nc + 1))
    for b in range(Nc + 1):
        others = np.delete(xc, b)
        lb = Polynomial.fromroots(others) / np.prod(xc[b] - others)
        J[:, b] = lb(xf)
    return J


def prolongation(fine: HexMesh, coarse: HexMesh) -> sp.csr_matrix:
    """P on the unknowns: (fine interior) x (coarse interior)."""
    J = interp_matrix(fine.N, coarse.N)
    Jt = np.einsum("ka,jb,ic->kjiabc", J, J, J).reshape((fine.N + 1) ** 3, (coarse.N + 1) ** 3)
    fid = fine.element_ids().reshape(len(fine.element_ids()), -1)
    cid = coarse.element_ids().reshape(len(coarse.element_ids()), -1)
    rows = np.repeat(fid, Jt.shape[1], axis=1).reshape(-1)
    cols = np.tile(cid, (1, Jt.shape[0])).reshape(-1)
    vals = np.broadcast_to(Jt.reshape(1, -1), (fid.shape[0], Jt.size)).reshape(-1)
    nf, nc = np.prod(fine.grid), np.prod(coarse.grid)
    # assignment (not summation): every element gives a shared node the same
    # value; keep one entry per (row, col)
    key = rows.astype(np.int64) * nc + cols
    _, first = np.unique(key, return_index=True)
    Pfull = sp.csr_matrix((vals[first], (rows[first], cols[first])), shape=(nf, nc))
    return Pfull[fine.interior_mask()][:, coarse.interior_mask()].tocsr()


def chebyshev_coefficients(lo: float, hi: float, m: int):
    """(1/theta, [(c1, c2)] for steps 1..m-1) of the Chebyshev iteration on
    [lo, hi]: theta = (hi + lo) / 2, delta = (hi - lo) / 2, sigma = theta /
    delta, rho_0 = 1 / sigma, rho_k = 1 / (2 sigma - rho_{k-1}),
    c1 = rho_k rho_{k-1}, c2 = 2 rho_k / delta."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    cs = []
    for _ in range(m - 1):
        rn = 1.0 / (2.0 * sigma - rho)
        cs.append((rn * rho, 2.0 * rn / delta))
        rho = rn
    return 1.0 / theta, cs


def largest_eig_dinv_a(mesh: HexMesh, dinv) -> float:
    """rho = lambda_max(D^{-1} A) from the symmetric form D^{-1/2} A D^{-1/2}
    (ARPACK)."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    s = np.sqrt(dinv)
    op = LinearOperator((mesh.n, mesh.n), matvec=lambda v: s * mesh.apply(s * np.ravel(v)), dtype=np.float64)
    if mesh.n <= 3:
        Ad = np.column_stack([op.matvec(e) for e in np.eye(mesh.n)])
        return float(np.linalg.eigvalsh(Ad).max())
    return float(eigsh(op, k=1, which="LA", tol=1e-10, return_eigenvectors=False)[0])


class PMultigrid:
    """V-cycle preconditioner over the orders ``orders`` (highest first) on
    the mesh of ``fine``.  ``rho``: lambda_max(D^-1 A) per level (None:
    computed).  apply64(r) is the FP64 cycle; apply(y, uz) the cycle in the
    arithmetic of u_z (FP64 for u_z = FP64, else FP32) rounded to u_z, the
    interface of oracle.amp_model's preconditioners."""

    kind = "pmg"

    def __init__(self, fine: HexMesh, orders=(7, 3, 1), degree=2, coarse_degree=16, lo_ratio=0.1,
                 hi_margin=1.1, coarse_lo_ratio=0.01, rho=None):
        if fine.N != orders[0]:
            raise ValueError("the finest order must be the mesh's")
        if any(a <= b for a, b in zip(orders, orders[1:])):
            raise ValueError("orders must decrease")
        self.orders = tuple(orders)
        self.m, self.mc = int(degree), int(coarse_degree)
        verts = fine.verts.reshape(-1, 3)
        E = (fine.Ex, fine.Ey, fine.Ez)
        self.meshes = [fine] + [HexMesh(verts, E, N=N, lam=fine.lam) for N in orders[1:]]
        self.dinv = [1.0 / m.diagonal() for m in self.meshes]
        self.P = [prolongation(self.meshes[l], self.meshes[l + 1]) for l in range(len(orders) - 1)]
        self.rho = [float(r) for r in rho] if rho is not None else [
            largest_eig_dinv_a(m, d) for m, d in zip(self.meshes, self.dinv)]
        L = len(orders)
        self.intervals = [(lo_ratio * self.rho[l], hi_margin * self.rho[l]) for l in range(L - 1)]
        self.intervals.append((coarse_lo_ratio * self.rho[L - 1], hi_margin * self.rho[L - 1]))
        self.log2_extra = {64: 0, 32: 0, 16: 0}
        # max|M^{-1} r| <= gain max|r| for r = (1, ..., 1): the scaling's
        # first-iteration estimate
        self.gain = float(np.abs(self.apply64(np.ones(fine.n))).max())

    # -- one level ------------------------------------------------------
    def _smooth(self, l, f, Amul, c):
        """The Chebyshev-Jacobi iteration of level l for A x = f from x = 0
        (degree m, or mc on the coarsest level), in arithmetic c."""
        lo, hi = self.intervals[l]
        deg = self.mc if l == len(self.orders) - 1 else self.m
        inv_theta, cs = chebyshev_coefficients(lo, hi, deg)
        dinv = self.dinv[l].astype(c)
        x_prev = np.zeros_like(f)
        x = c(inv_theta) * (dinv * f)
        for k in range(1, deg):
            c1, c2 = cs[k - 1]
            x_new = (x + c(c1) * (x - x_prev)) + c(c2) * (dinv * (f - Amul(l, x)))
            x_prev, x = x, x_new
        return x

    def _vcycle(self, l, f, Amul, c):
        if l == len(self.orders) - 1:
            return self._smooth(l, f, Amul, c)
        x = self._smooth(l, f, Amul, c)
        fc = (self.P[l].T @ (f - Amul(l, x))).astype(c)
        x = x + (self.P[l] @ self._vcycle(l + 1, fc, Amul, c)).astype(c)
        x = x + self._smooth(l, f - Amul(l, x), Amul, c)
        return x

    def apply64(self, r):
        return self._vcycle(0, np.asarray(r, dtype=np.float64), lambda l, v: self.meshes[l].apply(v), np.float64)

    def apply(self, y_uz, uz):
        c = np.float64 if uz == 64 else np.float32
        Amul = (lambda l, v: self.meshes[l].apply(v)) if uz == 64 else (
            lambda l, v: self.meshes[l].apply(v.astype(np.float64)).astype(np.float32))
        z = self._vcycle(0, y_uz.astype(c), Amul, c)
        from .amp_model import fl
        return fl(z, uz)


def pcg(mesh: HexMesh, M: PMultigrid, b, tol: float = 1e-10, maxit: int = 2000):
    """Alg. 1 (FP64 PCG) on the matrix-free operator with z = M.apply64(r),
    x0 = 0, stopped when ||r_k|| <= tol ||b||.  Returns (x, {"iters",
    "relres", "relres_true"})."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = float(np.sqrt(b @ b))
    p = None
    rho_prev = None
    k = 0
    for k in range(1, maxit + 1):
        z = M.apply64(r)
        rho = float(r @ z)
        p = z.copy() if p is None else z + (rho / rho_prev) * p
        q = mesh.apply(p)
        alpha = rho / float(q @ p)
        x = x + alpha * p
        r = r - alpha * q
        rho_prev = rho
        if np.sqrt(r @ r) <= tol * bnorm:
            break
    t = b - mesh.apply(x)
    return x, {"iters": k, "relres": float(np.sqrt(r @ r)) / bnorm, "relres_true": float(np.sqrt(t @ t)) / bnorm}
