"""Pins of the FP64 gradient reference of the differentiable solve:
central finite differences, the 1-homogeneity invariant of the
transmissibilities, dL/db against finite differences, and agreement of its
assembly with the workload generator's."""

import numpy as np
import pytest

from oracle import adjoint as adj
from workloads import problems as P


@pytest.fixture(scope="module")
def case():
    theta, b, xt = P.adjoint_inputs(10)
    return theta.astype(np.float64), b, xt


def test_assembly_matches_generator(case):
    theta, _, _ = case
    A1 = adj.assemble(theta)
    A2 = P.fv_diffusion(np.exp(theta)).to_scipy()
    assert abs(A1 - A2).max() == 0.0
    A2d = adj.assemble(theta[0])            # a 2-D slice
    assert abs(A2d - P.fv_diffusion(np.exp(theta[0])).to_scipy()).max() == 0.0


@pytest.mark.parametrize("seed", range(4))
def test_theta_gradient_central_differences(case, seed):
    theta, b, xt = case
    L, g, lam, x = adj.loss_and_grad(theta, b, xt)
    d = np.random.default_rng([500, seed]).standard_normal(theta.shape)
    h = 1e-4
    fd = (adj.loss(theta + h * d, b, xt) - adj.loss(theta - h * d, b, xt)) / (2 * h)
    an = float((g * d).sum())
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_theta_gradient_coordinates(case):
    theta, b, xt = case
    L, g, lam, x = adj.loss_and_grad(theta, b, xt)
    h = 1e-4
    flat = theta.reshape(-1)
    for c in (0, 7, flat.size // 2, flat.size - 1):
        e = np.zeros_like(flat)
        e[c] = h
        fd = (adj.loss((flat + e).reshape(theta.shape), b, xt)
              - adj.loss((flat - e).reshape(theta.shape), b, xt)) / (2 * h)
        assert abs(fd - g.reshape(-1)[c]) <= 1e-6 * max(1e-3, abs(g.reshape(-1)[c]))


def test_homogeneity_invariant(case):
    # A(theta + eps 1) = exp(eps) A(theta)  =>  sum_c dL/dtheta_c = -x^T (x - x_t) = -b^T lambda
    theta, b, xt = case
    L, g, lam, x = adj.loss_and_grad(theta, b, xt)
    assert g.sum() == pytest.approx(-(x @ (x - xt)), rel=1e-10)
    assert g.sum() == pytest.approx(-(b @ lam), rel=1e-9)


def test_rhs_gradient(case):
    theta, b, xt = case
    L, g, lam, x = adj.loss_and_grad(theta, b, xt)
    d = np.random.default_rng([501, 0]).standard_normal(b.size)
    h = 1e-3
    fd = (adj.loss(theta, b + h * d, xt) - adj.loss(theta, b - h * d, xt)) / (2 * h)
    assert fd == pytest.approx(float(lam @ d), rel=1e-8)
