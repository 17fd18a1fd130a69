"""Pins of the FP64 reference of the matrix-free hexahedral operator
(Section 5.5, Ex. jac libp): the GLL rule and derivative matrix against the
exactness they must have, the operator against an element matrix built by a
different route (monomial-basis Lagrange polynomials, finite-difference
Jacobians), against the Kronecker form on an affine mesh, and against the
invariants of the continuous operator (constants in the kernel of the
stiffness part, discrete harmonicity of linear fields, symmetry, positive
definiteness)."""

import itertools

import numpy as np
import pytest
from numpy.polynomial import Polynomial

from oracle.hexop import HexMesh, deriv_matrix, gll
from workloads.problems import hex_vertices


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7])
def test_gll_rule_exactness(N):
    x, w = gll(N)
    assert x[0] == -1.0 and x[-1] == 1.0
    assert np.allclose(x, -x[::-1], atol=1e-15)
    assert np.all(w > 0)
    for p in range(2 * N):          # exact up to degree 2N - 1
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.dot(w, x ** p) - exact) < 1e-14, p
    # and not for degree 2N (x^2N: the rule is off)
    assert abs(np.dot(w, x ** (2 * N)) - 2.0 / (2 * N + 1)) > 1e-6


@pytest.mark.parametrize("N", [2, 3, 7])
def test_derivative_matrix_exact_on_polynomials(N):
    x, _ = gll(N)
    D = deriv_matrix(x)
    rng = np.random.default_rng([71, N])
    for _ in range(3):
        P = Polynomial(rng.standard_normal(N + 1))
        assert np.allclose(D @ P(x), P.deriv()(x), atol=1e-11)
    assert np.allclose(D.sum(axis=1), 0.0, atol=1e-13)


def _lagrange(x):
    """The Lagrange basis on x as monomial-basis polynomials (no barycentric
    weights, no derivative matrix)."""
    out = []
    for j in range(len(x)):
        others = np.delete(x, j)
        out.append(Polynomial.fromroots(others) / np.prod(x[j] - others))
    return out


def _trilinear(Xc, r, s, t):
    """x(r, s, t) for corners Xc[c, b, a, :]."""
    h = lambda a, v: (1.0 - v) / 2.0 if a == 0 else (1.0 + v) / 2.0
    return sum(Xc[c, b, a] * h(a, r) * h(b, s) * h(c, t) for a, b, c in itertools.product((0, 1), repeat=3))


def _element_matrix(Xc, N, lam):
    """A_e by quadrature with basis polynomials evaluated directly and J by
    central differences of the trilinear map (exact: the map is linear in
    each reference variable)."""
    x, w = gll(N)
    basis = _lagrange(x)
    dbasis = [b.deriv() for b in basis]
    n1 = N + 1
    nloc = n1 ** 3
    K = np.zeros((nloc, nloc))
    for (qk, qj, qi) in itertools.product(range(n1), repeat=3):
        r, s, t = x[qi], x[qj], x[qk]
        J = np.empty((3, 3))
        for col, e in enumerate(np.eye(3)):
            J[:, col] = (_trilinear(Xc, *(np.array([r, s, t]) + 0.5 * e)) -
                         _trilinear(Xc, *(np.array([r, s, t]) - 0.5 * e)))
        det = np.linalg.det(J)
        Jit = np.linalg.inv(J).T
        wq = w[qi] * w[qj] * w[qk]
        grads = np.empty((nloc, 3))
        vals = np.empty(nloc)
        for (k, j, i) in itertools.product(range(n1), repeat=3):
            idx = (k * n1 + j) * n1 + i
            gref = np.array([dbasis[i](r) * basis[j](s) * basis[k](t),
                             basis[i](r) * dbasis[j](s) * basis[k](t),
                             basis[i](r) * basis[j](s) * dbasis[k](t)])
            grads[idx] = Jit @ gref
            vals[idx] = basis[i](r) * basis[j](s) * basis[k](t)
        K += wq * det * (grads @ grads.T + lam * np.outer(vals, vals))
    return K


def test_single_element_against_direct_quadrature():
    N, lam = 3, 7.5
    rng = np.random.default_rng(72)
    verts = np.array([[a, b, c] for c in (-0.5, 0.5) for b in (-0.5, 0.5) for a in (-0.5, 0.5)], dtype=float)
    verts += rng.uniform(-0.12, 0.12, verts.shape)     # a genuinely trilinear element
    m = HexMesh(verts, (1, 1, 1), N=N, lam=lam)
    Xc = verts.reshape(2, 2, 2, 3)
    K = _element_matrix(Xc, N, lam)
    assert np.allclose(K, K.T, atol=1e-12)
    u = rng.standard_normal((N + 1) ** 3)
    got = m.apply_full(u)                               # one element: grid order = local order
    assert np.allclose(got, K @ u, rtol=1e-11, atol=1e-11 * np.abs(K @ u).max())


def test_affine_mesh_matches_kronecker_form():
    E, N, lam = (2, 3, 2), 3, 11.0
    m = HexMesh(hex_vertices(E, 0.0), E, N=N, lam=lam)
    x, w = gll(N)
    D = deriv_matrix(x)

    def one_d(ne):
        h = 1.0 / ne
        n = ne * N + 1
        K1, M1 = np.zeros((n, n)), np.zeros((n, n))
        for e in range(ne):
            sl = slice(e * N, e * N + N + 1)
            K1[sl, sl] += (2.0 / h) * D.T @ np.diag(w) @ D
            M1[sl, sl] += (h / 2.0) * np.diag(w)
        return K1, M1

    (Kx, Mx), (Ky, My), (Kz, Mz) = one_d(E[0]), one_d(E[1]), one_d(E[2])
    A = (np.kron(Mz, np.kron(My, Kx)) + np.kron(Mz, np.kron(Ky, Mx)) + np.kron(Kz, np.kron(My, Mx))
         + lam * np.kron(Mz, np.kron(My, Mx)))
    u = np.random.default_rng(73).standard_normal(A.shape[0])
    assert np.allclose(m.apply_full(u), A @ u, rtol=1e-11, atol=1e-11 * np.abs(A @ u).max())


@pytest.fixture(scope="module")
def small():
    E = (3, 2, 2)
    return HexMesh(hex_vertices(E, 0.25, seed=3), E, N=3, lam=0.0)


def test_constants_in_the_stiffness_kernel_and_volume(small):
    one = np.ones(np.prod(small.grid))
    assert np.abs(small.apply_full(one)).max() < 1e-12
    m = HexMesh(small.verts.reshape(-1, 3), (3, 2, 2), N=3, lam=2.0)
    assert abs(m.apply_full(one).sum() / 2.0 - 1.0) < 1e-13      # GLL mass sums to |box| = 1


def _node_coords(m):
    x = m.x
    h = np.stack([(1.0 - x) / 2.0, (1.0 + x) / 2.0])
    X = m._corners()
    P = np.einsum("ecbad,ai,bj,ck->ekjid", X, h, h, h)
    out = np.zeros((np.prod(m.grid), 3))
    out[m.element_ids().reshape(-1)] = P.reshape(-1, 3)
    return out


def test_linear_fields_are_discretely_harmonic(small):
    # u = a . x is trilinear in the reference variables, so its gradient is
    # exact at every node, and grad(phi_i) . a det(J) is a polynomial the
    # GLL rule integrates exactly: (K u)_i = int grad(phi_i) . a = 0 at every
    # node off the boundary
    pts = _node_coords(small)
    a = np.array([0.3, -1.2, 0.7])
    Ku = small.apply_full(pts @ a)
    inner = small.interior_mask()
    assert np.abs(Ku[inner]).max() < 1e-11
    assert np.abs(Ku[~inner]).max() > 1e-3          # boundary nodes carry the flux


def test_masked_operator_spd_and_diagonal():
    E = (2, 2, 2)
    m = HexMesh(hex_vertices(E, 0.25, seed=4), E, N=3, lam=1e3)
    n = m.n
    A = np.column_stack([m.apply(e) for e in np.eye(n)])
    assert np.allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    assert np.linalg.eigvalsh(A).min() > 0.0
    assert np.allclose(m.diagonal(), np.diag(A), rtol=1e-12)
    u = np.random.default_rng(74).standard_normal(n)
    assert m.mu(u) == pytest.approx(float(u @ A @ u), rel=1e-12)


def test_flop_count_formula():
    m = HexMesh(hex_vertices((1, 1, 1), 0.0), (1, 1, 1), N=7)
    # 2(N+1) per gradient component both ways, 15 for G, 2 + 2 for the
    # mass term and the sum, 149 for the geometric factors
    assert m.flops_per_element() == (6 * 8 + 15 + 6 * 8 + 4 + 149) * 512


def test_matrix_free_pcg_equals_assembled_pcg():
    # Alg. 1 on the operator against the C oracle's PCG on the assembled
    # matrix (the operator applied to unit vectors), Jacobi both ways
    from oracle import cpcg, hexop
    from workloads.problems import dense_to_csr
    E = (2, 3, 2)
    m = HexMesh(hex_vertices(E, 0.2, seed=5), E, N=3, lam=1e3)
    A = np.column_stack([m.apply(e) for e in np.eye(m.n)])
    b = np.random.default_rng(75).standard_normal(m.n)
    x1, i1 = hexop.pcg(m, b, tol=1e-10, maxit=500)
    x2, i2 = cpcg.pcg(dense_to_csr(A), b, tol=1e-10, maxit=500)
    assert i1["iters"] == i2["iters"]
    assert i1["relres_true"] <= 1e-10
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x2)
    assert np.allclose(A @ x1, b, atol=1e-9 * np.abs(b).max())

