"""Pins of the CPU oracle against what the paper and mathematics fix.

Nothing here uses the GPU solver.  Each test ties the oracle to something
other than itself: a dense Cholesky solve, finite termination of CG, closed
form spectra recovered through the CG-Lanczos relation, manufactured
solutions, the Chebyshev polynomial's closed form, and the printed switch
iterations of Example 9.
"""

import math
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import amp_model as am
from oracle import cpcg
from workloads import problems as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lanczos_extremes(alpha, beta):
    """Extreme Ritz values of M^{-1}A from CG's alpha_k, beta_{k-1}:
    T_kk = 1/alpha_k + beta_{k-1}/alpha_{k-1}, T_{k,k+1} = sqrt(beta_k)/alpha_k."""
    k = len(alpha)
    diag = np.empty(k)
    off = np.empty(k - 1)
    for i in range(k):
        diag[i] = 1.0 / alpha[i] + (beta[i] / alpha[i - 1] if i > 0 else 0.0)
        if i + 1 < k:
            off[i] = math.sqrt(beta[i + 1]) / alpha[i]
    ev = sla.eigvalsh_tridiagonal(diag, off)
    return ev[0], ev[-1]


# ---------------------------------------------------------------- textbook routine

@pytest.mark.parametrize("seed", range(4))
def test_pcg_matches_dense_cholesky(seed):
    rng = np.random.default_rng([100, seed])
    n = int(rng.integers(5, 64))
    eigs = np.exp(rng.uniform(0.0, math.log(1e3), n))
    A = P.spectrum_matrix(eigs, seed=(101, seed))
    b = rng.standard_normal(n)
    Ac = P.dense_to_csr(A)
    x, info = cpcg.pcg(Ac, b, tol=1e-13, maxit=2000, precond=cpcg.PC_JACOBI)
    assert info["status"] == 0
    xc = sla.cho_solve(sla.cho_factor(A), b)
    kappa = eigs.max() / eigs.min()
    assert np.linalg.norm(x - xc) / np.linalg.norm(xc) <= 10 * kappa * 1e-13


def test_identity_preconditioner_matches_cholesky():
    rng = np.random.default_rng([102, 0])
    A = P.spectrum_matrix(np.linspace(1.0, 50.0, 40), seed=(102, 1))
    b = rng.standard_normal(40)
    x, info = cpcg.pcg(P.dense_to_csr(A), b, tol=1e-13, maxit=500, precond=cpcg.PC_IDENTITY)
    xc = sla.cho_solve(sla.cho_factor(A), b)
    assert info["status"] == 0
    assert np.linalg.norm(x - xc) <= 1e-10 * np.linalg.norm(xc)


# ---------------------------------------------------------------- finite termination

@pytest.mark.parametrize("m", [2, 3, 5, 8])
@pytest.mark.parametrize("orth", [False, True])
def test_finite_termination(m, orth):
    # m distinct, well separated eigenvalues, each repeated: CG ends in <= m steps
    n = 6 * m
    eigs = np.repeat(np.arange(1.0, m + 1.0), 6)
    A = P.spectrum_matrix(eigs, seed=(103, m), orthonormal=orth)
    b = np.random.default_rng([103, m, 1]).standard_normal(n)
    x, info = cpcg.pcg(P.dense_to_csr(A), b, tol=1e-12, maxit=100, precond=cpcg.PC_IDENTITY)
    assert info["status"] == 0
    assert info["iters"] <= m + 1


# ---------------------------------------------------------------- closed-form spectra

def test_poisson2d_spectrum_via_lanczos():
    m = 64
    A, b, _ = P.poisson2d_system(m)
    x, info = cpcg.pcg(A, b, tol=1e-14, maxit=3000, history=True)
    lo, hi = _lanczos_extremes(info["alpha"], info["beta"])
    c = np.cos(np.arange(1, m + 1) * math.pi / (m + 1))
    lam = 4.0 - 2.0 * c[:, None] - 2.0 * c[None, :]
    # Jacobi is 1/4 I here, so M^{-1}A has the spectrum of A/4
    assert abs(lo - lam.min() / 4) <= 1e-8 * lam.min() / 4
    assert abs(hi - lam.max() / 4) <= 1e-8 * lam.max() / 4
    assert lam.max() / lam.min() == pytest.approx(1711.7, rel=1e-4)


def test_fv3d_constant_coefficient_spectrum_via_lanczos():
    # cell-centred FV with Dirichlet faces: per direction the 1-D operator
    # has eigenvalues 2 - 2 cos(j pi / n), j = 1..n
    n = 12
    A = P.fv_diffusion(np.ones((n, n, n)))
    d = A.diagonal()
    b = np.random.default_rng([104, 0]).standard_normal(A.n)
    x, info = cpcg.pcg(A, b, tol=1e-14, maxit=3000, precond=cpcg.PC_IDENTITY, history=True)
    lo, hi = _lanczos_extremes(info["alpha"], info["beta"])
    mu = 2.0 - 2.0 * np.cos(np.arange(1, n + 1) * math.pi / n)
    assert abs(lo - 3 * mu.min()) <= 1e-8 * 3 * mu.min()
    assert abs(hi - 3 * mu.max()) <= 1e-8 * 3 * mu.max()
    assert d.min() == 6.0 and d.max() == 9.0


def _q1_closed_form(n, kx, ky, kz):
    h = 1.0 / (n + 1)
    j = np.arange(1, n + 1)
    K = (2.0 / h) * (1 - np.cos(j * math.pi * h))
    M = (h / 6.0) * (4 + 2 * np.cos(j * math.pi * h))
    lam = (kx * K[None, None, :] * M[None, :, None] * M[:, None, None]
           + ky * M[None, None, :] * K[None, :, None] * M[:, None, None]
           + kz * M[None, None, :] * M[None, :, None] * K[:, None, None])
    d = (2.0 / h) * (2 * h / 3) ** 2 * (kx + ky + kz)
    return lam / d, d


def test_q1_isotropic_spectrum_via_lanczos():
    n = 14
    A = P.q1_anisotropic(n, 1.0, 1.0, 1.0)
    lam, d = _q1_closed_form(n, 1.0, 1.0, 1.0)
    assert np.allclose(A.diagonal(), d, rtol=1e-13)
    b = np.random.default_rng([105, 0]).standard_normal(A.n)
    x, info = cpcg.pcg(A, b, tol=1e-14, maxit=5000, history=True)
    lo, hi = _lanczos_extremes(info["alpha"], info["beta"])
    assert abs(lo - lam.min()) <= 1e-8 * lam.min()
    assert abs(hi - lam.max()) <= 1e-8 * lam.max()


def test_q1_anisotropic_spectrum():
    # the z-modes are nearly degenerate for kz = 1e-3, so CG resolves the
    # bottom cluster only as a cluster: Ritz values must lie inside the
    # closed-form spectrum, and a dense eigensolver must hit it exactly
    n = 10
    A = P.q1_anisotropic(n)
    lam, d = _q1_closed_form(n, 1.0, 1e-2, 1e-3)
    ev = np.linalg.eigvalsh(A.to_scipy().toarray()) / d
    assert np.allclose(np.sort(lam.ravel()), ev, rtol=1e-10, atol=1e-13)
    b = np.random.default_rng([105, 1]).standard_normal(A.n)
    x, info = cpcg.pcg(A, b, tol=1e-14, maxit=5000, history=True)
    lo, hi = _lanczos_extremes(info["alpha"], info["beta"])
    assert lam.min() * (1 - 1e-12) <= lo <= lam.min() * 1.01
    assert abs(hi - lam.max()) <= 1e-8 * lam.max()
    glo, ghi = P.q1_anisotropic_bounds(n)
    assert glo == pytest.approx(lam.min(), rel=1e-12)
    assert ghi == pytest.approx(lam.max(), rel=1e-12)


# ---------------------------------------------------------------- manufactured solutions

@pytest.mark.parametrize("which", ["poisson", "fv3d", "q1"])
def test_manufactured_solution(which):
    if which == "poisson":
        A, b, xs = P.poisson2d_system(40)
        kappa = 1.0 / (math.sin(math.pi / 82) ** 2 / math.cos(math.pi / 82) ** 2)
        kw = {}
    elif which == "fv3d":
        A = P.fv_diffusion(np.exp(np.random.default_rng([106, 0]).standard_normal((10, 10, 10))))
        xs = np.random.default_rng([106, 1]).uniform(-1, 1, A.n)
        b = A.to_scipy() @ xs
        ev = np.linalg.eigvalsh(A.to_scipy().toarray())
        kappa = ev[-1] / ev[0]
        kw = {}
    else:
        A, b, xs, (lo, hi) = P.q1_system(12)
        kappa = hi / lo
        kw = {}
    x, info = cpcg.pcg(A, b, tol=1e-10, maxit=5000, **kw)
    assert info["status"] == 0
    assert info["relres_true"] <= 1.5e-10
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * info["relres_true"]


# ---------------------------------------------------------------- Chebyshev closed form

def _cheb_T(m, t):
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    a = np.abs(t) <= 1
    out[a] = np.cos(m * np.arccos(t[a]))
    bpos = t > 1
    out[bpos] = np.cosh(m * np.arccosh(t[bpos]))
    bneg = t < -1
    out[bneg] = (-1) ** m * np.cosh(m * np.arccosh(-t[bneg]))
    return out


@pytest.mark.parametrize("degree", [1, 2, 4])
def test_chebyshev_on_sine_modes(degree):
    n = 10
    A = P.q1_anisotropic(n)
    lo, hi = P.q1_anisotropic_bounds(n)
    d = A.diagonal()[0]
    h = 1.0 / (n + 1)
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    for (j1, j2, j3) in [(1, 1, 1), (3, 5, 2), (n, n, n), (7, 1, 9)]:
        g = np.arange(1, n + 1)
        u = (np.sin(j3 * math.pi * h * g)[:, None, None] * np.sin(j2 * math.pi * h * g)[None, :, None]
             * np.sin(j1 * math.pi * h * g)[None, None, :]).reshape(-1)
        Au = A.to_scipy() @ u
        lam = float(u @ Au / (u @ u)) / d          # eigenvalue of D^{-1}A for this mode
        assert np.allclose(Au / d, lam * u, atol=1e-12 * np.abs(Au / d).max())
        s = (1.0 - _cheb_T(degree, np.array([(theta - lam) / delta]))[0]
             / _cheb_T(degree, np.array([theta / delta]))[0]) / lam
        z = cpcg.precond_apply(A, u, kind=cpcg.PC_CHEBYSHEV, degree=degree, lam_lo=lo, lam_hi=hi)
        assert np.allclose(z, (s / d) * u, rtol=0, atol=1e-11 * np.abs(s / d * u).max())
        # the model's FP64 evaluation of the same polynomial
        C = am.Chebyshev(A.to_scipy(), lo, hi, degree)
        assert np.allclose(C.apply64(u), (s / d) * u, rtol=0, atol=1e-11 * np.abs(s / d * u).max())


def test_chebyshev_pcg_converges_faster_than_jacobi():
    A, b, xs, (lo, hi) = P.q1_system(16)
    _, ij = cpcg.pcg(A, b, tol=1e-10, maxit=5000)
    x, ic = cpcg.pcg(A, b, tol=1e-10, maxit=5000, precond=cpcg.PC_CHEBYSHEV, degree=4,
                     lam_lo=lo, lam_hi=hi)
    assert ic["status"] == 0 and ij["status"] == 0
    assert ic["iters"] < ij["iters"] / 2
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= (hi / lo) * ic["relres_true"]


# ---------------------------------------------------------------- edge cases

def test_zero_rhs_and_exact_start():
    A, b, xs = P.poisson2d_system(8)
    x, info = cpcg.pcg(A, np.zeros(A.n), tol=1e-10, maxit=10)
    assert info["iters"] == 0 and info["status"] == 0 and np.all(x == 0)
    x, info = cpcg.pcg(A, b, x0=xs, tol=1e-10, maxit=10)
    assert info["iters"] == 0 and info["status"] == 0


def test_non_spd_breaks_down():
    A = P.dense_to_csr(np.diag([1.0, -5.0, 1.0, 1.0]))
    _, info = cpcg.pcg(A, np.ones(4), tol=1e-10, maxit=10, precond=cpcg.PC_IDENTITY)
    assert info["status"] == cpcg.ST_BREAKDOWN
    # a non-positive diagonal is rejected up front by Jacobi
    _, info = cpcg.pcg(A, np.ones(4), tol=1e-10, maxit=10, precond=cpcg.PC_JACOBI)
    assert info["status"] == cpcg.ST_ARG


def test_maxit_returns_last_iterate():
    A, b, _ = P.poisson2d_system(32)
    x, info = cpcg.pcg(A, b, tol=1e-10, maxit=7)
    assert info["status"] == cpcg.ST_MAXIT and info["iters"] == 7
    assert info["relres_true"] < 1.0


def test_thread_count_does_not_change_result():
    A, b, _ = P.blocky_diffusion3d_system(16, 4)
    x1, i1 = cpcg.pcg(A, b, tol=1e-10, maxit=2000, threads=1)
    x4, i4 = cpcg.pcg(A, b, tol=1e-10, maxit=2000, threads=4)
    cpcg.lib().oracle_set_threads(os.cpu_count() or 1)
    assert i1["iters"] == i4["iters"]
    assert np.array_equal(x1, x4)
