"""FP64 reference of the matrix-free high-order hexahedral operator of
Section 5.5 (Ex. jac libp): the screened Poisson operator -Laplace(u) +
lambda u, discretised by tensor-product Lagrange elements of order N on the
Gauss-Lobatto-Legendre (GLL) points, with GLL quadrature on the same points,
on a box of Ex x Ey x Ez hexahedra, homogeneous Dirichlet conditions.  Each
element is the image of the reference cube [-1, 1]^3 under the trilinear map
of its 8 vertices; the geometric factors are formed from those vertices at
every quadrature point (the paper computes them on the fly from 24 values
per element).

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
operator.

Definitions (element e, reference point q = (r, s, t), GLL weights w):
* x(r, s, t) = sum over the 8 vertices of X_v h_a(r) h_b(s) h_c(t), with
  h_0(r) = (1 - r) / 2, h_1(r) = (1 + r) / 2: J = dx / d(r, s, t).
* A_e u = D^T (G (D u)) + lambda M u, where D u is the reference gradient
  (the 1-D derivative matrix of the Lagrange basis applied along each
  direction), G = w_q det(J) J^{-1} J^{-T} at each point and M = w_q det(J)
  (the GLL mass matrix, diagonal).
* A = sum over elements of the scattered A_e (direct stiffness summation);
  the unknowns are the nodes not on the boundary of the box.

Global nodes lie on a (N Ex + 1) x (N Ey + 1) x (N Ez + 1) grid, x fastest;
node (ex N + i, ey N + j, ez N + k) is local node (i, j, k) of element
(ex, ey, ez).  Unknown index of interior grid node (gx, gy, gz):
(gx - 1) + (N Ex - 1) ((gy - 1) + (N Ey - 1) (gz - 1)).  Vertex (vx, vy, vz)
of the (Ex + 1) x (Ey + 1) x (Ez + 1) vertex grid is row
vx + (Ex + 1) (vy + (Ey + 1) vz) of the vertex array (x, y, z).
"""

from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as L


def gll(N: int):
    """GLL nodes (ascending, on [-1, 1]) and weights for order N: the end
    points and the roots of P_N'; w = 2 / (N (N + 1) P_N(x)^2)."""
    cN = np.zeros(N + 1)
    cN[N] = 1.0
    inner = np.sort(np.real(L.legroots(L.legder(cN)))) if N > 1 else np.array([])
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (N * (N + 1) * L.legval(x, cN) ** 2)
    return x, w


def deriv_matrix(x: np.ndarray) -> np.ndarray:
    """D[m, j] = l_j'(x_m) for the Lagrange basis l_j on the nodes x
    (barycentric form: l_j'(x_m) = (c_j / c_m) / (x_m - x_j) for m != j,
    rows summing to zero)."""
    n = len(x)
    c = np.array([np.prod([x[j] - x[k] for k in range(n) if k != j]) for j in range(n)])
    D = np.zeros((n, n))
    for m in range(n):
        for j in range(n):
            if m != j:
                D[m, j] = (c[m] / c[j]) / (x[m] - x[j])
        D[m, m] = -np.sum(D[m, :])
    return D


class HexMesh:
    """Box mesh of Ex x Ey x Ez trilinear hexahedra of order N."""

    def __init__(self, verts: np.ndarray, E, N: int = 7, lam: float = 1e3):
        self.Ex, self.Ey, self.Ez = E
        self.N = N
        self.lam = float(lam)
        self.verts = np.asarray(verts, dtype=np.float64).reshape(self.Ez + 1, self.Ey + 1, self.Ex + 1, 3)
        self.x, self.w = gll(N)
        self.D = deriv_matrix(self.x)
        self.G, self.detW = self._geometry()

    @property
    def grid(self):
        N = self.N
        return (N * self.Ez + 1, N * self.Ey + 1, N * self.Ex + 1)   # (z, y, x)

    @property
    def n(self) -> int:
        gz, gy, gx = self.grid
        return (gx - 2) * (gy - 2) * (gz - 2)

    def _corners(self):
        """X[ez, ey, ex, c, b, a, d]: vertex (ex + a, ey + b, ez + c)."""
        V = self.verts
        X = np.empty((self.Ez, self.Ey, self.Ex, 2, 2, 2, 3))
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    X[:, :, :, c, b, a, :] = V[c:c + self.Ez, b:b + self.Ey, a:a + self.Ex, :]
        return X.reshape(-1, 2, 2, 2, 3)

    def _geometry(self):
        """Per element and node (e, k, j, i): G (3 x 3) and w det(J)."""
        x = self.x
        h = np.stack([(1.0 - x) / 2.0, (1.0 + x) / 2.0])        # h[a, i]
        dh = np.outer([-0.5, 0.5], np.ones_like(x))              # dh[a, i] = h_a'(x_i)
        X = self._corners()                                      # (E, c, b, a, d)
        # J[e, k, j, i, d, 0..2] = dx_d / d(r, s, t) at node (i, j, k)
        Jr = np.einsum("ecbad,ai,bj,ck->ekjid", X, dh, h, h)
        Js = np.einsum("ecbad,ai,bj,ck->ekjid", X, h, dh, h)
        Jt = np.einsum("ecbad,ai,bj,ck->ekjid", X, h, h, dh)
        J = np.stack([Jr, Js, Jt], axis=-1)                      # (..., d, ref)
        det = np.linalg.det(J)
        if not np.all(det > 0.0):
            raise ValueError("an element map is not orientation-preserving")
        Jinv = np.linalg.inv(J)                                  # (..., ref, d)
        W = np.einsum("k,j,i->kji", self.w, self.w, self.w)
        Wd = W[None] * det
        G = Wd[..., None, None] * np.einsum("...pd,...qd->...pq", Jinv, Jinv)
        return G, Wd

    def element_ids(self):
        """Global grid index (z, y, x flattened) of each element's local
        nodes, shape (E, N+1, N+1, N+1) in (k, j, i) order."""
        N = self.N
        gz, gy, gx = self.grid
        ez, ey, ex = np.meshgrid(np.arange(self.Ez), np.arange(self.Ey), np.arange(self.Ex), indexing="ij")
        k, j, i = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij")
        Z = ez.reshape(-1, 1, 1, 1) * N + k[None]
        Y = ey.reshape(-1, 1, 1, 1) * N + j[None]
        Xg = ex.reshape(-1, 1, 1, 1) * N + i[None]
        return (Z * gy + Y) * gx + Xg

    def interior_mask(self):
        gz, gy, gx = self.grid
        m = np.zeros((gz, gy, gx), dtype=bool)
        m[1:-1, 1:-1, 1:-1] = True
        return m.reshape(-1)

    def to_grid(self, u):
        gz, gy, gx = self.grid
        U = np.zeros(gz * gy * gx)
        U[self.interior_mask()] = u
        return U

    def apply_full(self, U):
        """Sum over elements of A_e applied to a field on every grid node
        (no boundary condition); returns the field on every grid node."""
        ids = self.element_ids()
        Ue = U[ids]                                              # (E, k, j, i)
        D = self.D
        ur = np.einsum("im,ekjm->ekji", D, Ue)
        us = np.einsum("jm,ekmi->ekji", D, Ue)
        ut = np.einsum("km,emji->ekji", D, Ue)
        grad = np.stack([ur, us, ut], axis=-1)
        F = np.einsum("...pq,...q->...p", self.G, grad)
        Ae = (np.einsum("mi,ekjm->ekji", D, F[..., 0]) + np.einsum("mj,ekmi->ekji", D, F[..., 1])
              + np.einsum("mk,emji->ekji", D, F[..., 2]) + self.lam * self.detW * Ue)
        out = np.zeros_like(U)
        np.add.at(out, ids.reshape(-1), Ae.reshape(-1))
        return out

    def apply(self, u):
        """q = A u on the unknowns (interior nodes)."""
        return self.apply_full(self.to_grid(np.asarray(u, dtype=np.float64)))[self.interior_mask()]

    def mu(self, u):
        """mu = u^T A u."""
        u = np.asarray(u, dtype=np.float64)
        return float(u @ self.apply(u))

    def diagonal(self):
        """Diagonal of A on the unknowns.  For local node (a, b, c) the
        reference gradient of its basis function vanishes at every point off
        the three grid lines through it, so A_e's diagonal entry is
        sum_m D[m,a]^2 G_rr(m,b,c) + sum_m D[m,b]^2 G_ss(a,m,c)
        + sum_m D[m,c]^2 G_tt(a,b,m) + 2 D[a,a] D[b,b] G_rs(a,b,c)
        + 2 D[a,a] D[c,c] G_rt(a,b,c) + 2 D[b,b] D[c,c] G_st(a,b,c)
        + lambda w det(J) at (a,b,c); the entries are summed over elements."""
        D, G = self.D, self.G
        D2 = D ** 2
        dd = np.diag(D)
        de = (np.einsum("ma,ecbm->ecba", D2, G[..., 0, 0]) + np.einsum("mb,ecma->ecba", D2, G[..., 1, 1])
              + np.einsum("mc,emba->ecba", D2, G[..., 2, 2])
              + 2.0 * np.einsum("a,b,ecba->ecba", dd, dd, G[..., 0, 1])
              + 2.0 * np.einsum("a,c,ecba->ecba", dd, dd, G[..., 0, 2])
              + 2.0 * np.einsum("b,c,ecba->ecba", dd, dd, G[..., 1, 2])
              + self.lam * self.detW)
        out = np.zeros(np.prod(self.grid))
        np.add.at(out, self.element_ids().reshape(-1), de.reshape(-1))
        return out[self.interior_mask()]

    def flops_per_element(self) -> int:
        """Arithmetic of one element application as the definition counts it
        (multiply and add counted separately, per node): the reference
        gradient 3 x 2(N+1), G applied 15, D^T 3 x 2(N+1) + 2, the mass term
        2, and the geometric factors: J 36 FMAs (72) + 12 products, the
        cofactors 27, det 5, 1 / det 1, G's six entries 6 x 5 + 2 = 32."""
        n1 = self.N + 1
        per_node = 3 * 2 * n1 + 15 + 3 * 2 * n1 + 2 + 2 + (72 + 12 + 27 + 5 + 1 + 32)
        return per_node * n1 ** 3


def pcg(mesh: HexMesh, b, tol: float = 1e-10, maxit: int = 5000, jacobi: bool = True):
    """Alg. 1 (FP64 PCG) on the matrix-free operator with the Jacobi
    preconditioner M = diag(A) (or M = I), x0 = 0, stopped when
    ||r_k|| <= tol ||b||.  Returns (x, {"iters", "relres", "relres_true"})."""
    b = np.asarray(b, dtype=np.float64)
    dinv = 1.0 / mesh.diagonal() if jacobi else np.ones_like(b)
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = float(np.sqrt(b @ b))
    info = {"iters": 0}
    if np.sqrt(r @ r) <= tol * bnorm:
        info.update(relres=float(np.sqrt(r @ r)) / bnorm, relres_true=float(np.sqrt(r @ r)) / bnorm)
        return x, info
    p = None
    rho_prev = None
    k = 0
    for k in range(1, maxit + 1):
        z = dinv * r
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
    info.update(iters=k, relres=float(np.sqrt(r @ r)) / bnorm, relres_true=float(np.sqrt(t @ t)) / bnorm)
    return x, info

