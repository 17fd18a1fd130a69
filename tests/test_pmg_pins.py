"""Pins of the FP64 reference of the p-multigrid preconditioner (Section 5.3,
Ex. linear conv2): the interpolation between orders against polynomial
reproduction, the smoothers and the whole V-cycle against dense matrices
built from their error propagators by another route (the matrix Chebyshev
recurrence T_{k+1}(X) = 2 X T_k(X) - T_{k-1}(X), not the three-term
iteration the oracle runs), symmetry and definiteness of the cycle, the
eigenvalue estimate against a dense eigensolver, and PCG with the cycle
against a dense solve."""

import numpy as np
import pytest

from oracle import pmg
from oracle.hexop import HexMesh, gll
from workloads.problems import hex_vertices


@pytest.mark.parametrize("Nf,Nc", [(7, 3), (3, 1), (4, 2), (5, 5)])
def test_interp_matrix_reproduces_polynomials(Nf, Nc):
    J = pmg.interp_matrix(Nf, Nc)
    xf, _ = gll(Nf)
    xc, _ = gll(Nc)
    assert np.allclose(J.sum(axis=1), 1.0, atol=1e-13)          # partition of unity
    assert np.allclose(J[0], np.eye(Nc + 1)[0]) and np.allclose(J[-1], np.eye(Nc + 1)[-1])
    rng = np.random.default_rng([81, Nf, Nc])
    for _ in range(3):
        c = rng.standard_normal(Nc + 1)
        assert np.allclose(J @ np.polyval(c, xc), np.polyval(c, xf), atol=1e-12)
    if Nf == Nc:
        assert np.allclose(J, np.eye(Nf + 1), atol=1e-13)


def _node_xyz(m):
    """Physical node coordinates on an affine box mesh (unperturbed
    vertices): element widths times the GLL points, by grid index."""
    x, _ = gll(m.N)
    out = []
    for E, g in zip((m.Ex, m.Ey, m.Ez), (m.grid[2], m.grid[1], m.grid[0])):
        idx = np.arange(g)
        e = np.minimum(idx // m.N, E - 1)
        loc = idx - e * m.N
        out.append(-0.5 + (e + (x[loc] + 1.0) / 2.0) / E)
    gz, gy, gx = m.grid
    Z, Y, X = np.meshgrid(out[2], out[1], out[0], indexing="ij")
    return X.reshape(-1), Y.reshape(-1), Z.reshape(-1)


def test_prolongation_reproduces_coarse_space():
    # u = prod (1/4 - x_d^2) vanishes on the box and has degree 2 in each
    # variable, so on an affine mesh it lies in every space of order >= 2:
    # P (u at the coarse nodes) = u at the fine nodes
    E = (3, 2, 2)
    V = hex_vertices(E, 0.0)
    f, c = HexMesh(V, E, N=5, lam=0.0), HexMesh(V, E, N=2, lam=0.0)
    P = pmg.prolongation(f, c)
    u = lambda m: np.prod([0.25 - t ** 2 for t in _node_xyz(m)], axis=0)[m.interior_mask()]
    assert P.shape == (f.n, c.n)
    assert np.allclose(P @ u(c), u(f), atol=1e-14)
    # a field of degree 3 does not lie in the order-2 space
    v = lambda m: (np.prod([0.25 - t ** 2 for t in _node_xyz(m)], axis=0) * _node_xyz(m)[0])[m.interior_mask()]
    assert np.abs(P @ v(c) - v(f)).max() > 1e-2 * np.abs(v(f)).max()


def _dense(m):
    return np.column_stack([m.apply(e) for e in np.eye(m.n)])


def _cheb_error_matrix(A, dinv, lo, hi, deg):
    """I - S A = T_deg((theta I - D^-1 A) / delta) / T_deg(theta / delta)
    by the matrix recurrence of the Chebyshev polynomials."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    X = (theta * np.eye(len(A)) - dinv[:, None] * A) / delta
    T0, T1 = np.eye(len(A)), X
    t0, t1 = 1.0, theta / delta
    for _ in range(deg - 1):
        T0, T1 = T1, 2.0 * X @ T1 - T0
        t0, t1 = t1, 2.0 * (theta / delta) * t1 - t0
    return T1 / t1


@pytest.fixture(scope="module")
def cycle():
    E = (3, 3, 2)
    m = HexMesh(hex_vertices(E, 0.2, seed=8), E, N=4, lam=5.0)
    M = pmg.PMultigrid(m, orders=(4, 2, 1), degree=3, coarse_degree=4)
    A = [_dense(mm) for mm in M.meshes]
    return m, M, A


def test_rho_against_dense_eigenvalues(cycle):
    m, M, A = cycle
    for l, Al in enumerate(A):
        ev = np.linalg.eigvals(M.dinv[l][:, None] * Al)
        assert M.rho[l] == pytest.approx(float(np.real(ev).max()), rel=1e-9)


def test_vcycle_against_error_propagator(cycle):
    m, M, A = cycle
    L = len(A)
    # V_l from E_l = I - V_l A_l, bottom up
    lo, hi = M.intervals[L - 1]
    Ec = _cheb_error_matrix(A[L - 1], M.dinv[L - 1], lo, hi, M.mc)
    V = (np.eye(len(Ec)) - Ec) @ np.linalg.inv(A[L - 1])
    for l in range(L - 2, -1, -1):
        lo, hi = M.intervals[l]
        Es = _cheb_error_matrix(A[l], M.dinv[l], lo, hi, M.m)
        P = M.P[l].toarray()
        El = Es @ (np.eye(len(A[l])) - P @ V @ P.T @ A[l]) @ Es
        V = (np.eye(len(A[l])) - El) @ np.linalg.inv(A[l])
    r = np.random.default_rng(82).standard_normal(m.n)
    z = M.apply64(r)
    assert np.allclose(z, V @ r, rtol=1e-9, atol=1e-9 * np.abs(V @ r).max())
    # the cycle is symmetric and positive definite
    assert np.allclose(V, V.T, atol=1e-9 * np.abs(V).max())
    assert np.linalg.eigvalsh(0.5 * (V + V.T)).min() > 0.0
    # and the A-norm contraction of the smoother holds: spectrum of I - S A in [-1, 1]
    lo, hi = M.intervals[0]
    ev = np.linalg.eigvals(_cheb_error_matrix(A[0], M.dinv[0], lo, hi, M.m))
    assert np.abs(ev).max() <= 1.0 + 1e-10


def test_fp32_cycle_close_to_fp64(cycle):
    m, M, A = cycle
    r = np.random.default_rng(83).standard_normal(m.n)
    z64 = M.apply64(r)
    z32 = M.apply(r.astype(np.float32), 32)
    assert z32.dtype == np.float32
    assert np.abs(z32 - z64).max() <= 1e-5 * np.abs(z64).max()
    z16 = M.apply(r.astype(np.float16), 16)
    assert z16.dtype == np.float16


def test_pcg_with_the_cycle_solves_and_beats_jacobi():
    from oracle import hexop
    E = (3, 3, 3)
    m = HexMesh(hex_vertices(E, 0.2, seed=9), E, N=3, lam=0.0)
    M = pmg.PMultigrid(m, orders=(3, 1), degree=2, coarse_degree=6)
    b = np.random.default_rng(84).standard_normal(m.n)
    x, info = pmg.pcg(m, M, b, tol=1e-10)
    assert info["relres_true"] <= 1e-10 * 1.01
    A = _dense(m)
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    _, ij = hexop.pcg(m, b, tol=1e-10)
    assert info["iters"] < ij["iters"] // 2
