"""The seeded input generators (no solver arithmetic): the vectorised
constant-coefficient stencil builder gives exactly the CSR of the general
per-offset builder."""

import itertools

import numpy as np
import pytest

from workloads import problems as P


@pytest.mark.parametrize("dims", [(5,), (4, 6), (3, 4, 5), (7, 7, 7), (1, 1, 1), (2, 3, 1)])
@pytest.mark.parametrize("points", ["full", "star"])
def test_const_stencil_builder_matches_general(dims, points):
    offs = list(itertools.product(*([(-1, 0, 1)] * len(dims))))
    if points == "star":
        offs = [o for o in offs if sum(abs(v) for v in o) <= 1]
    vals = [float(v) for v in np.random.default_rng([900, len(dims)]).standard_normal(len(offs))]
    a = P._stencil_csr(dims, offs, vals)
    b = P._const_stencil_csr(dims, offs, vals)
    assert a.n == b.n
    for f in ("row_ptr", "col_idx", "val"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
        assert getattr(a, f).dtype == getattr(b, f).dtype, f


def test_q1_operator_is_the_tensor_product_stencil():
    # the Q1 matrix equals kx K(x)M(y)M(z) + ky M(x)K(y)M(z) + kz M(x)M(y)K(z)
    # assembled from the 1-D factors with scipy's Kronecker products
    import scipy.sparse as sp
    n = 6
    h = 1.0 / (n + 1)
    K1 = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]) / h
    M1 = sp.diags([np.ones(n - 1), 4 * np.ones(n), np.ones(n - 1)], [-1, 0, 1]) * (h / 6)
    # x fastest: the x factor is the rightmost Kronecker factor
    ref = (1.0 * sp.kron(sp.kron(M1, M1), K1) + 1e-2 * sp.kron(sp.kron(M1, K1), M1)
           + 1e-3 * sp.kron(sp.kron(K1, M1), M1)).toarray()
    A = P.q1_anisotropic(n).to_scipy().toarray()
    assert np.allclose(A, ref, rtol=1e-14, atol=1e-18)
