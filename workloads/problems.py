"""Synthetic SPD systems with the shapes of the solver's workloads.

All matrices are returned as :class:`CSR` (int32 row pointers and column
indices, float64 values, columns sorted within each row, diagonal present).
Grids are ordered lexicographically with x fastest: cell (ix, iy, iz) has
index ``ix + nx*(iy + ny*iz)``.

Workloads (sizes are the defaults; every builder takes smaller sizes for tests):

* ``poisson2d_system``   -- 2-D 5-point finite-difference Poisson, stencil
  [4, -1, -1, -1, -1], Dirichlet, 64x64 interior, b = A x* with
  x* ~ U[-1, 1].
* ``blocky_diffusion3d_system`` -- 3-D 7-point cell-centred finite volume,
  128^3 cells, coefficient 10^U with U ~ U[0, 4] constant on 8^3 blocks,
  b ~ N(0, 1).
* ``q1_system``          -- 3-D 27-point trilinear (Q1) finite-element
  stiffness of -div(K grad u) with K = diag(1, 1e-2, 1e-3) on the unit cube,
  256^3 interior nodes, Dirichlet, b = A x* with x* ~ U[-1, 1].
* ``batched_systems``    -- 512 2-D 5-point finite-volume systems, side
  log-uniform in [32, 512], coefficient exp(g) with g ~ N(0, 1.5^2) i.i.d.
  per cell, b ~ N(0, 1) per system.
* ``adjoint_inputs``     -- log-coefficients theta ~ N(0, 1) (float32) on a
  64^3 grid, b ~ N(0, 1) and a target x_t ~ N(0, 1).

Finite-volume convention: the transmissibility of an interior face between
cells i and j is the harmonic combination 2 k_i k_j / (k_i + k_j); a face on
the Dirichlet boundary has 2 k_i.  A_ii is the sum over the cell's faces and
A_ij = -T_ij.  No mesh-size factors.

The paper's small spectrum-prescribed examples (Ex. 1, 4, 6, 9 and 10 of
Section 5) are built by ``paper_spectrum`` + ``spectrum_matrix``.
"""

from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np


def rng_for(workload: int, *stream: int) -> np.random.Generator:
    """The seeded generator for (workload, stream...)."""
    return np.random.default_rng([workload, *stream])


@dataclass
class CSR:
    n: int
    row_ptr: np.ndarray  # int32, n+1
    col_idx: np.ndarray  # int32, nnz
    val: np.ndarray      # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr), shape=(self.n, self.n))

    def diagonal(self) -> np.ndarray:
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        mask = self.col_idx == rows
        d = np.zeros(self.n)
        d[rows[mask]] = self.val[mask]
        return d


# ---------------------------------------------------------------------------
# generic structured-grid CSR assembly
# ---------------------------------------------------------------------------

def _stencil_csr(dims, offsets, values) -> CSR:
    """Assemble a stencil matrix on a box grid.

    ``dims``   -- grid sizes, x first (1, 2 or 3 entries).
    ``offsets`` -- list of integer tuples (dx[, dy[, dz]]); entries whose
                 neighbour falls outside the grid are dropped.
    ``values`` -- per offset either a scalar or a length-N float64 array
                 (value of row i's entry for that offset).
    Offsets are sorted by their linear offset so that columns are sorted.
    """
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    N = int(np.prod(dims))
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    lin = [sum(o[a] * strides[a] for a in range(nd)) for o in offsets]
    order = np.argsort(lin, kind="stable")
    idx = np.arange(N, dtype=np.int64)
    coords = []
    rem = idx
    for a in range(nd):
        coords.append((rem % dims[a]).astype(np.int32))
        rem = rem // dims[a]
    del rem

    def valid(o):
        m = np.ones(N, dtype=bool)
        for a in range(nd):
            if o[a] < 0:
                m &= coords[a] >= -o[a]
            elif o[a] > 0:
                m &= coords[a] < dims[a] - o[a]
        return m

    counts = np.zeros(N, dtype=np.int64)
    for o in offsets:
        counts += valid(o)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    if nnz >= 2**31:
        raise ValueError("nnz does not fit int32")
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    fill = row_ptr[:-1].copy()
    for oi in order:
        o = offsets[oi]
        rows = np.nonzero(valid(o))[0]
        pos = fill[rows]
        col[pos] = (rows + lin[oi]).astype(np.int32)
        v = values[oi]
        if np.isscalar(v):
            val[pos] = v
        else:
            val[pos] = v[rows]
        fill[rows] += 1
    return CSR(N, row_ptr.astype(np.int32), col, val)


def _const_stencil_csr(dims, offsets, values) -> CSR:
    """The matrix of :func:`_stencil_csr` for scalar values and offsets in
    {-1, 0, 1} per axis, built without per-offset passes: the (row, offset)
    table of every row's candidate entries, masked by whether the neighbour
    lies inside the grid (a product of per-axis masks), is compressed in row
    order.  Offsets sorted by linear offset are sorted by column within each
    row (|offset| <= 1 < every axis size), so the result is the same CSR."""
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    N = int(np.prod(dims))
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    lin = np.array([sum(o[a] * strides[a] for a in range(nd)) for o in offsets], dtype=np.int64)
    order = np.argsort(lin, kind="stable")
    offs = [offsets[i] for i in order]
    vals = np.array([float(values[i]) for i in order])
    K = len(offs)
    # mask[row, k]: the k-th offset's neighbour is inside the grid; per-axis
    # masks are broadcast over the other axes (row index: x fastest)
    mask = np.ones((N, K), dtype=bool)
    for a in range(nd):
        c = np.arange(dims[a])
        shape = [1] * nd
        shape[nd - 1 - a] = dims[a]          # arrays are laid out (z, y, x)
        for k, o in enumerate(offs):
            ok = ((c + o[a] >= 0) & (c + o[a] < dims[a])).reshape(shape)
            mask[:, k] &= np.broadcast_to(ok, dims[::-1]).reshape(N)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    if nnz >= 2**31:
        raise ValueError("nnz does not fit int32")
    col = (np.arange(N, dtype=np.int32)[:, None] + lin[order].astype(np.int32)[None, :])[mask]
    val = np.broadcast_to(vals, (N, K))[mask]
    return CSR(N, row_ptr.astype(np.int32), np.ascontiguousarray(col, dtype=np.int32),
               np.ascontiguousarray(val, dtype=np.float64))


def stencil_poisson2d(m: int) -> CSR:
    """2-D 5-point finite-difference Laplacian on an m x m interior grid."""
    offs = [(-1, 0), (1, 0), (0, -1), (0, 1), (0, 0)]
    vals = [-1.0, -1.0, -1.0, -1.0, 4.0]
    return _stencil_csr((m, m), offs, vals)


def fv_diffusion(kappa: np.ndarray) -> CSR:
    """Cell-centred finite-volume diffusion operator for a 2-D or 3-D
    coefficient field ``kappa`` (array shape (ny, nx) or (nz, ny, nx))."""
    kappa = np.asarray(kappa, dtype=np.float64)
    shape = kappa.shape[::-1]           # x first
    nd = len(shape)
    k = kappa.reshape(-1)
    N = k.size
    strides = [1]
    for d in shape[:-1]:
        strides.append(strides[-1] * d)
    idx = np.arange(N, dtype=np.int64)
    coords = []
    rem = idx
    for a in range(nd):
        coords.append(rem % shape[a])
        rem = rem // shape[a]
    diag = np.zeros(N)
    offs, vals = [], []
    for a in range(nd):
        for s in (-1, 1):
            o = [0] * nd
            o[a] = s
            inside = (coords[a] + s >= 0) & (coords[a] + s < shape[a])
            nb = np.where(inside, idx + s * strides[a], idx)
            kn = k[nb]
            t = np.where(inside, 2.0 * k * kn / (k + kn), 2.0 * k)
            diag += t
            offs.append(tuple(o))
            vals.append(-t)
    offs.append(tuple([0] * nd))
    vals.append(diag)
    return _stencil_csr(shape, offs, vals)


def _q1_1d(h):
    # 1-D stiffness K = (1/h)[-1, 2, -1] and mass M = (h/6)[1, 4, 1]
    K = {-1: -1.0 / h, 0: 2.0 / h, 1: -1.0 / h}
    M = {-1: h / 6.0, 0: 4.0 * h / 6.0, 1: h / 6.0}
    return K, M


def q1_anisotropic(n: int, kx: float = 1.0, ky: float = 1e-2, kz: float = 1e-3) -> CSR:
    """Trilinear finite-element stiffness for -div(diag(kx,ky,kz) grad u) on
    the unit cube with n interior nodes per direction (h = 1/(n+1)),
    homogeneous Dirichlet: A = kx K(x)M(y)M(z) + ky M(x)K(y)M(z) + kz M(x)M(y)K(z)."""
    h = 1.0 / (n + 1)
    K, M = _q1_1d(h)
    offs, vals = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                v = (kx * K[dx] * M[dy] * M[dz] + ky * M[dx] * K[dy] * M[dz]
                     + kz * M[dx] * M[dy] * K[dz])
                offs.append((dx, dy, dz))
                vals.append(v)
    return _const_stencil_csr((n, n, n), offs, vals)


def q1_anisotropic_bounds(n: int, kx: float = 1.0, ky: float = 1e-2, kz: float = 1e-3):
    """Exact extreme eigenvalues of D^{-1} A for :func:`q1_anisotropic`
    (the diagonal is constant, and the sine modes diagonalise every 1-D factor).
    Returned as (lam_min, lam_max)."""
    h = 1.0 / (n + 1)
    j = np.arange(1, n + 1)
    c = np.cos(j * math.pi * h)
    Kj = (2.0 / h) * (1.0 - c)
    Mj = (h / 3.0) * (2.0 + c)
    d = (2.0 / h) * (2.0 * h / 3.0) ** 2 * (kx + ky + kz)
    lo, hi = np.inf, -np.inf
    # separable maximisation over the 3-D index box in slabs to bound memory
    for i3 in range(n):
        lam = (kx * Kj[None, :] * Mj[:, None] * Mj[i3] + ky * Mj[None, :] * Kj[:, None] * Mj[i3]
               + kz * Mj[None, :] * Mj[:, None] * Kj[i3])
        lo = min(lo, float(lam.min()))
        hi = max(hi, float(lam.max()))
    return lo / d, hi / d


def dense_to_csr(A: np.ndarray) -> CSR:
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    rp = [0]
    ci, vv = [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        if i not in nz:
            nz = np.sort(np.append(nz, i))
        ci.extend(nz.tolist())
        vv.extend(A[i, nz].tolist())
        rp.append(len(ci))
    return CSR(n, np.array(rp, dtype=np.int32), np.array(ci, dtype=np.int32), np.array(vv))


def long_row_spd(n: int, mean_row: int = 200, band: int | None = None, seed: int = 0,
                 integer: bool = False) -> CSR:
    """A symmetric, strictly diagonally dominant (hence SPD) matrix with long,
    ragged rows: every row i draws k_i ~ U{mean_row/4, ..., 3 mean_row/4}
    upper-triangle columns i + d, d ~ U{1, ..., band} (band = 4 mean_row),
    duplicates and columns past n dropped, and the pattern is mirrored, so a
    row holds about mean_row off-diagonal entries.  Off-diagonal values are
    -U(0.1, 1) (integer: -U{1, ..., 4}); the diagonal is 1 + the row's sum of
    |a_ij|.  With integer=True every product with an integer vector of
    moderate size is exact in FP64 (and in FP32 below 2^24)."""
    band = band or 4 * mean_row
    g = rng_for(6, seed, n)
    q = max(1, mean_row // 4)
    k = g.integers(q, 3 * q + 1, size=n)
    rows = np.repeat(np.arange(n, dtype=np.int64), k)
    cols = rows + g.integers(1, band + 1, size=rows.size)
    keep = cols < n
    key = np.unique(rows[keep] * n + cols[keep])
    r, c = key // n, key % n
    v = -g.integers(1, 5, size=key.size).astype(np.float64) if integer else -g.uniform(0.1, 1.0, key.size)
    diag = 1.0 + np.bincount(r, weights=-v, minlength=n) + np.bincount(c, weights=-v, minlength=n)
    R = np.concatenate([r, c, np.arange(n)])
    C = np.concatenate([c, r, np.arange(n)])
    V = np.concatenate([v, v, diag])
    order = np.argsort(R * n + C, kind="stable")
    R, C, V = R[order], C[order], V[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(R, minlength=n), out=rp[1:])
    return CSR(n, rp.astype(np.int32), C.astype(np.int32), V)


def long_row_system(n: int = 65536, mean_row: int = 200, seed: int = 0):
    """long_row_spd with b ~ N(0, 1): the long-row workload the lanes-per-row
    layout is for."""
    A = long_row_spd(n, mean_row, seed=seed)
    b = rng_for(6, 1, seed, n).standard_normal(n)
    return A, b


def hex_vertices(E, perturb: float = 0.2, seed: int = 0) -> np.ndarray:
    """Vertices of an Ex x Ey x Ez box mesh of [-0.5, 0.5]^3: the uniform
    grid with every vertex off the boundary moved by perturb h U(-1, 1) per
    coordinate (h the element width), so the element maps are trilinear, not
    affine; boundary vertices stay (the box keeps its faces).  Returns an
    ((Ex+1)(Ey+1)(Ez+1), 3) float64 array, x fastest."""
    Ex, Ey, Ez = E
    g = rng_for(7, seed, Ex, Ey, Ez)
    axes = [np.linspace(-0.5, 0.5, m + 1) for m in (Ex, Ey, Ez)]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    V = np.stack([X, Y, Z], axis=-1)
    h = np.array([1.0 / Ex, 1.0 / Ey, 1.0 / Ez])
    d = perturb * h * g.uniform(-1.0, 1.0, V.shape)
    inner = np.zeros(V.shape[:3], dtype=bool)
    inner[1:-1, 1:-1, 1:-1] = True
    V[inner] += d[inner]
    return V.reshape(-1, 3)


def pmg_poisson_rhs(E, N: int = 7) -> np.ndarray:
    """Right-hand side of the Poisson problem of Ex. linear conv2 on the
    interior nodes of the order-N grid of an E box mesh of [-0.5, 0.5]^3:
    f(x, y, z) = 1 + 3 pi^2 sin(pi x) sin(pi y) sin(pi z) sampled at the
    evenly spaced positions of the unperturbed grid, times the mean volume
    per node (1 / (N^3 Ex Ey Ez)), in grid order (x fastest).  An input of the
    problem's shape and smoothness, not its exact load vector."""
    Ex, Ey, Ez = E
    ax = [(-0.5 + np.arange(1, N * m) / (N * m)) for m in (Ex, Ey, Ez)]
    s = [np.sin(np.pi * a) for a in ax]
    vol = 1.0 / (N ** 3 * Ex * Ey * Ez)
    f = 1.0 + 3.0 * np.pi ** 2 * (s[2][:, None, None] * s[1][None, :, None] * s[0][None, None, :])
    return (vol * f).reshape(-1)


# ---------------------------------------------------------------------------
# the paper's spectrum-prescribed examples (Section 2 and Section 5)
# ---------------------------------------------------------------------------

def paper_spectrum(name: str) -> np.ndarray:
    """Eigenvalues of the paper's synthetic examples.

    ex1  -- motivating example (eq. motivating A): n = 100, five isolated
            large eigenvalues and 95 evenly spaced ones.
    ex4  -- Ex. 4: lambda_i = i/(10n) + (n-i)/n, i = 0..n, n = 100.
    ex6  -- Ex. 6: lambda_i = i/(1000n) + (n-i)/n, i = 0..n, n = 100.
    ex9  -- Ex. 9: lambda_i = 1e-3 + (i-1)/(n-1) rho^(n-i), lambda_n = 1,
            n = 10, rho = 1/4.
    ex10 -- Ex. 10: the same formula with n = 50, rho = 0.9.
    """
    if name == "ex1":
        lam = np.empty(100)
        lam[99] = 1.0
        for i in range(95, 100):
            lam[i - 1] = 1e-3 + (i - 1) / 99.0 * (17.0 / 20.0) ** (100 - i)
        lam[:95] = np.linspace(1e-3, lam[94], 95)
        return lam
    if name in ("ex4", "ex6"):
        n = 100
        f = 10.0 if name == "ex4" else 1000.0
        i = np.arange(n + 1)
        return np.sort(i / (f * n) + (n - i) / n)
    if name in ("ex9", "ex10"):
        n, rho = (10, 0.25) if name == "ex9" else (50, 0.9)
        lam = np.empty(n)
        for i in range(1, n):
            lam[i - 1] = 1e-3 + (i - 1) / (n - 1) * rho ** (n - i)
        lam[n - 1] = 1.0
        return lam
    raise KeyError(name)


def spectrum_matrix(eigs, seed=(0, 0), orthonormal: bool = True) -> np.ndarray:
    """Dense SPD Q diag(eigs) Q^T with a seeded random orthonormal Q
    (QR of a Gaussian matrix with sign-fixed R); ``orthonormal=False`` gives
    the diagonal matrix itself."""
    eigs = np.asarray(eigs, dtype=np.float64)
    n = eigs.size
    if not orthonormal:
        return np.diag(eigs)
    g = np.random.default_rng(list(seed)).standard_normal((n, n))
    Q, R = np.linalg.qr(g)
    Q = Q * np.sign(np.diag(R))[None, :]
    A = (Q * eigs[None, :]) @ Q.T
    return 0.5 * (A + A.T)


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def poisson2d_system(m: int = 64):
    """2-D Poisson, manufactured solution.  Returns (A, b, x_star)."""
    A = stencil_poisson2d(m)
    x_star = rng_for(1, 1).uniform(-1.0, 1.0, A.n)
    b = A.to_scipy() @ x_star
    return A, b, x_star


def blocky_diffusion3d_system(n: int = 128, block: int = 8, decades: float = 4.0):
    """3-D 7-point FV with block-constant coefficients 10^U, U ~ U[0, decades].
    Returns (A, b, kappa)."""
    if n % block:
        raise ValueError("grid must be a multiple of the block size")
    nb = n // block
    U = rng_for(2, 0).uniform(0.0, decades, (nb, nb, nb))
    kappa = np.repeat(np.repeat(np.repeat(10.0 ** U, block, 0), block, 1), block, 2)
    A = fv_diffusion(kappa)
    b = rng_for(2, 1).standard_normal(A.n)
    return A, b, kappa


CHEB_HI_MARGIN = 1.05


def q1_system(n: int = 256):
    """Anisotropic Q1 system, manufactured solution.
    Returns (A, b, x_star, (lam_lo, lam_hi)): the Chebyshev interval for
    D^{-1}A, lam_lo the exact smallest eigenvalue and lam_hi the exact
    largest one times CHEB_HI_MARGIN.  The preconditioner polynomial s(t)
    turns negative from t = lam_hi + lam_lo on, and rounding the
    preconditioner's matrix to FP16 moves the top of the spectrum by more
    than lam_lo, so the exact bounds would make M indefinite."""
    A = q1_anisotropic(n)
    x_star = rng_for(3, 1).uniform(-1.0, 1.0, A.n)
    b = A.to_scipy() @ x_star
    lo, hi = q1_anisotropic_bounds(n)
    return A, b, x_star, (lo, CHEB_HI_MARGIN * hi)


def batched_systems(count: int = 512, side_min: int = 32, side_max: int = 512,
                    sigma: float = 1.5):
    """Uneven batch of 2-D 5-point FV systems.  Returns a list of (A, b)."""
    g = rng_for(4, 0)
    sides = np.rint(np.exp(g.uniform(math.log(side_min), math.log(side_max), count))).astype(int)
    out = []
    for i, s in enumerate(sides):
        kappa = np.exp(sigma * g.standard_normal((s, s)))
        A = fv_diffusion(kappa)
        b = rng_for(4, 1, i).standard_normal(A.n)
        out.append((A, b))
    return out


def adjoint_inputs(n: int = 64):
    """Inputs of the differentiable solve on an n^3 grid.
    Returns (theta float32 (n,n,n) as (z,y,x), b, x_target)."""
    theta = rng_for(5, 0, n).standard_normal((n, n, n)).astype(np.float32)
    N = n ** 3
    b = rng_for(5, 1, n).standard_normal(N)
    x_t = rng_for(5, 2, n).standard_normal(N)
    return theta, b, x_t
