"""Pins of the oracle's Chebyshev-bound estimator (oracle/eigbounds.py):
the generator against its published first output, Ritz values against
closed-form spectra, finite termination on a small system, and the
interval against the anisotropic Q1 operator's closed form."""

import math

import numpy as np
import pytest

from oracle import eigbounds as E
from workloads import problems as P


def test_splitmix64_first_outputs():
    # splitmix64 seeded with 0 (java.util.SplittableRandom(0).nextLong()
    # is -2152535657050944081 = 0xE220A8397B1DCDAF)
    out = E.splitmix64(np.array([1], dtype=np.uint64))
    assert int(out[0]) == 0xE220A8397B1DCDAF
    u = E.start_vector(1000)
    assert u.min() >= -1.0 and u.max() < 1.0
    assert abs(u.mean()) < 0.1 and abs(np.mean(u * u) - 1.0 / 3.0) < 0.05


def _poisson_scaled_spectrum(m):
    # D^{-1} A = A / 4 for the 5-point Laplacian: (4 - 2 cos(i pi/(m+1)) - 2 cos(j pi/(m+1))) / 4
    c = np.cos(np.arange(1, m + 1) * math.pi / (m + 1))
    return np.sort(((4.0 - 2.0 * c[:, None] - 2.0 * c[None, :]) / 4.0).ravel())


def test_ritz_values_inside_the_spectrum_and_top_converged():
    m = 32
    A = P.stencil_poisson2d(m).to_scipy()
    lam = _poisson_scaled_spectrum(m)
    theta = E.ritz_values(*E.lanczos(A))
    assert len(theta) == E.LANCZOS_STEPS
    assert theta[0] >= lam[0] * (1 - 1e-12) and theta[-1] <= lam[-1] * (1 + 1e-12)
    assert theta[-1] >= 0.99 * lam[-1]          # the top Ritz value within 1% after 24 steps


def test_finite_termination_on_a_small_system():
    # a 3 x 3 grid has 9 rows and 6 distinct eigenvalues: the process stops
    # at an invariant subspace and its Ritz values are eigenvalues
    A = P.stencil_poisson2d(3).to_scipy()
    lam = np.unique(np.round(_poisson_scaled_spectrum(3), 12))
    alpha, beta = E.lanczos(A, steps=24)
    theta = E.ritz_values(alpha, beta)
    assert len(alpha) <= 9
    for t in theta:
        assert np.min(np.abs(lam - t)) <= 1e-12
    assert abs(theta[-1] - lam[-1]) <= 1e-12 and abs(theta[0] - lam[0]) <= 1e-12


@pytest.mark.parametrize("n", [12, 20])
def test_interval_against_the_q1_closed_form(n):
    lo_ex, hi_ex = P.q1_anisotropic_bounds(n)
    (lo, hi), (tmin, tmax) = E.chebyshev_bounds(P.q1_anisotropic(n).to_scipy())
    assert tmax <= hi_ex * (1 + 1e-12) and tmin >= lo_ex * (1 - 1e-12)
    assert hi >= hi_ex                           # the 5% margin covers the unconverged top
    assert hi <= E.HI_MARGIN * hi_ex * (1 + 1e-12)
    assert lo == pytest.approx(hi / E.LO_RATIO, rel=1e-15)
