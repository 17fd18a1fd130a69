"""FP64 reference of the differentiable solve x = A(theta)^{-1} b.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg).  Shares no
code with the GPU path.

Operator: cell-centred finite volumes on a box grid with cell coefficients
kappa = exp(theta); an interior face between cells i and j has
transmissibility T = 2 kappa_i kappa_j / (kappa_i + kappa_j), a face on the
Dirichlet boundary T = 2 kappa_i; A_ii is the sum of the cell's face
transmissibilities and A_ij = -T_ij.

Loss L = 0.5 ||x - x_t||^2.  Adjoint: lambda = A^{-1} (x - x_t) (A is
symmetric), dL/db = lambda, dL/dA_ij = -lambda_i x_j on the sparsity
pattern.  Chain rule through the faces:
    interior face (i, j): dL/dT = -(lambda_i - lambda_j)(x_i - x_j),
                          dT/dtheta_i = 2 kappa_i kappa_j^2 / (kappa_i + kappa_j)^2
    boundary face of i:   dL/dT = -lambda_i x_i,  dT/dtheta_i = 2 kappa_i
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _shape_x_first(theta):
    return theta.shape[::-1]


def assemble(theta: np.ndarray) -> sp.csr_matrix:
    """A(theta) for theta of shape (ny, nx) or (nz, ny, nx) (x fastest)."""
    k = np.exp(np.asarray(theta, dtype=np.float64)).reshape(-1)
    dims = _shape_x_first(np.asarray(theta))
    N = k.size
    strides = np.cumprod((1,) + tuple(dims[:-1]))
    idx = np.arange(N)
    coords = [(idx // strides[a]) % dims[a] for a in range(len(dims))]
    rows, cols, vals = [], [], []
    diag = np.zeros(N)
    for a in range(len(dims)):
        for s in (-1, 1):
            nb = coords[a] + s
            inside = (nb >= 0) & (nb < dims[a])
            j = idx + s * strides[a]
            i_in = idx[inside]
            j_in = j[inside]
            t = 2.0 * k[i_in] * k[j_in] / (k[i_in] + k[j_in])
            rows.append(i_in)
            cols.append(j_in)
            vals.append(-t)
            diag[i_in] += t
            diag[idx[~inside]] += 2.0 * k[idx[~inside]]
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(N, N))
    A.sort_indices()
    return A


def solve(A, rhs):
    return spla.spsolve(A.tocsc(), rhs)


def loss_and_grad(theta, b, x_t, solver=solve):
    """Returns (L, dL/dtheta (float64, theta's shape), dL/db = lambda, x)."""
    theta = np.asarray(theta, dtype=np.float64)
    A = assemble(theta)
    x = solver(A, b)
    g = x - x_t
    L = 0.5 * float(g @ g)
    lam = solver(A, g)
    k = np.exp(theta).reshape(-1)
    dims = _shape_x_first(theta)
    N = k.size
    strides = np.cumprod((1,) + tuple(dims[:-1]))
    idx = np.arange(N)
    coords = [(idx // strides[a]) % dims[a] for a in range(len(dims))]
    grad = np.zeros(N)
    for a in range(len(dims)):
        for s in (-1, 1):
            nb = coords[a] + s
            inside = nb >= 0
            inside &= nb < dims[a]
            i_in = idx[inside]
            j_in = i_in + s * strides[a]
            ki, kj = k[i_in], k[j_in]
            dLdT = -(lam[i_in] - lam[j_in]) * (x[i_in] - x[j_in])
            np.add.at(grad, i_in, dLdT * 2.0 * ki * kj * kj / (ki + kj) ** 2)
            i_b = idx[~inside]
            np.add.at(grad, i_b, -lam[i_b] * x[i_b] * 2.0 * k[i_b])
    return L, grad.reshape(theta.shape), lam, x


def loss(theta, b, x_t, solver=solve):
    A = assemble(theta)
    x = solver(A, b)
    g = x - x_t
    return 0.5 * float(g @ g)
