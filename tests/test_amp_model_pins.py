"""Pins of the AMP-PCG model (Alg. 3) against what the paper fixes.

* Thm. dspcg: dynamic scaling leaves the iterates unchanged; a power-of-two
  scale leaves them bitwise unchanged in a fixed precision.
* eq. eta_k / eq. linear criterion: the switch iteration on a geometric
  residual history has a closed form.
* Example 9: u_z drops to FP32 at iteration 9 and to FP16 at 11.
* Section 2 / Section 5.1: naive FP16 PCG breaks down on Example 1; AMP-PCG
  does not, and its true residual reaches the tolerance.
* Final-accuracy bound after eq. linear criterion: ||b - A x|| <= 2 tol ||b||.
"""

import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import amp_model as am
from oracle import cpcg
from workloads import problems as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


class Identity:
    """M = I in the model's preconditioner interface."""
    kind = "jacobi"
    log2_extra = {64: 0, 32: 0, 16: 0}
    gain = 1.0

    def apply(self, y, uz):
        return am.fl(y.astype(am.NP[am.compute_type(uz)]), uz)


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = int(v)
    return out


# ------------------------------------------------------------- Thm. dspcg

@pytest.mark.parametrize("scaling", ["pow2", "paper", "none"])
def test_fp64_model_matches_c_oracle(scaling):
    A, b, _ = P.poisson2d_system(48)
    x_o, info = cpcg.pcg(A, b, tol=1e-10, maxit=5000, history=True)
    r = am.amp_pcg(A, b, tol=1e-10, maxit=5000, opt=am.options("pcg64", scaling=scaling))
    assert r.status == 0
    assert r.iters == info["iters"]
    assert np.linalg.norm(r.x - x_o) <= 1e-12 * np.linalg.norm(x_o)
    assert np.allclose(r.delta, info["delta"], rtol=1e-9, atol=0)


@pytest.mark.parametrize("u", [64, 32])
def test_pow2_scaling_is_bitwise_neutral(u):
    # every vector in precision u; omega = 2^e_k versus omega = 1
    A, b, _ = P.blocky_diffusion3d_system(16, 4, decades=2.0)
    eta = "fixed64" if u == 64 else "fixed32"
    base = am.options("pcg64", u0=u, eta=eta, verify=False)
    r1 = am.amp_pcg(A, b, tol=1e-6, maxit=3000, opt=base)
    r2 = am.amp_pcg(A, b, tol=1e-6, maxit=3000, opt=am.options("pcg64", u0=u, eta=eta,
                                                                  verify=False, scaling="none"))
    assert r1.iters == r2.iters
    assert np.array_equal(r1.x, r2.x)
    assert r1.delta == r2.delta
    assert len(set(r1.omega)) > 1          # the scale really changed along the way


# ------------------------------------------------------------- eta indicators

@pytest.mark.parametrize("q", [0.5, 0.8, 0.93])
@pytest.mark.parametrize("d,C", [(10, 1.0), (5, 2.0)])
def test_delay_indicator_closed_form(q, d, C):
    bnorm, tol = 3.0, 1e-10
    delta = [bnorm * q ** t for t in range(400)]
    opt = am.AmpOptions(u0=64, tau_zs=0.0, tau_zh=0.0, eta="delay", d=d, C=C)
    # eta_k = eps32 ||b|| q^{k-d-1} (1 - q^{d+1})/(1 - q) ((3+C) + (2+C) q)
    c = am.EPS32 * (1 - q ** (d + 1)) / (1 - q) * ((3 + C) + (2 + C) * q)
    k_exact = d + 1 + max(0, math.ceil(math.log(tol / c) / math.log(q)))
    for k in (k_exact - 1, k_exact):
        closed = am.EPS32 * bnorm * q ** (k - d - 1) * (1 - q ** (d + 1)) / (1 - q) * ((3 + C) + (2 + C) * q)
        assert am.eta_delay(delta, k, d, C) == pytest.approx(closed, rel=1e-12)
    assert am.replay_switches(delta, bnorm, tol, opt)[2] == k_exact
    # the window is incomplete before k = d + 1
    assert am.eta_delay(delta, d, d, C) == math.inf


@pytest.mark.parametrize("q", [0.6, 0.9, 0.97])
def test_linear_indicator_closed_form(q):
    bnorm, tol, ell, C = 2.0, 1e-10, 5, 1.0
    delta = [bnorm * q ** t for t in range(1200)]
    opt = am.AmpOptions(u0=64, tau_zs=0.0, tau_zh=0.0, eta="linear", ell=ell, C=C)
    # eta_k = eps32 (5+2C) ||b|| q^{k-1} / (1-q) <= tol ||b||
    k_exact = max(ell, 1 + math.ceil(math.log(tol * (1 - q) / (am.EPS32 * (5 + 2 * C))) / math.log(q)))
    assert am.replay_switches(delta, bnorm, tol, opt)[2] == k_exact
    # undefined while the rate is not below one
    flat = [1.0] * 20
    assert am.eta_linear(flat, 10, ell, C) == math.inf


def test_selector_thresholds_and_latch():
    sel = am.precision_selector
    assert sel(1e-3, 64, 1e-4, 1e-6, math.inf, 1.0) == (64, 64)
    assert sel(1e-5, 64, 1e-4, 1e-6, math.inf, 1.0) == (32, 64)
    assert sel(1e-7, 64, 1e-4, 1e-6, 0.5, 1.0) == (16, 32)
    assert sel(1e-3, 16, 1e-4, 1e-6, 1.0, 1.0) == (16, 32)     # ties switch
    assert sel(1e-9, 32, 1e-4, 0.0, math.inf, 1.0) == (32, 64)  # tau_zh = 0 never reaches FP16
    # an oscillating history: once lowered, precisions stay low
    delta = [1.0, 1e-3, 5e-5, 2e-3, 1e-2, 1e-7, 1e-3]
    kz32, kz16, kr = am.replay_switches(delta, 1.0, 1e-10, am.AmpOptions())
    assert (kz32, kz16) == (2, 5)


# ------------------------------------------------------------- Example 9 (printed switch points)

@pytest.mark.parametrize("orth,seed", [(False, 0), (True, 0), (True, 1)])
def test_example9_switch_iterations(orth, seed):
    gold = _golden("ex9_switch_iterations.txt")
    lam = P.paper_spectrum("ex9")
    A = sp.csr_matrix(P.spectrum_matrix(lam, seed=(9, seed), orthonormal=orth))
    b = np.ones(10)
    r = am.amp_pcg(A, b, tol=1e-10, maxit=200, M=Identity(), opt=am.options("amp64", eta="fixed64"))
    r64 = am.amp_pcg(A, b, tol=1e-10, maxit=200, M=Identity(), opt=am.options("pcg64"))
    assert r.status == 0 and r64.status == 0
    assert r.k_z32 == gold["k_z32"]
    assert r.k_z16 == gold["k_z16"]
    assert r.iters > r64.iters          # "a few additional iterations"
    assert r.iters <= r64.iters + 6


# ------------------------------------------------------------- Example 1 (motivating)

def _ex1():
    lam = P.paper_spectrum("ex1")
    A = sp.csr_matrix(P.spectrum_matrix(lam, seed=(1, 7)))
    return A, np.ones(100)


def test_example1_naive_fp16_breaks_down():
    A, b = _ex1()
    _, it16, st16, delta16 = am.naive_pcg(A, b, 16, tol=1e-10, maxit=500)
    assert st16 == am.ST_BREAKDOWN
    _, it64, st64, _ = am.naive_pcg(A, b, 64, tol=1e-10, maxit=500)
    assert st64 == am.ST_CONVERGED


@pytest.mark.parametrize("preset", ["amp64", "amp16", "amp_ur"])
def test_example1_amp_reaches_tolerance(preset):
    A, b = _ex1()
    r64 = am.amp_pcg(A, b, tol=1e-10, maxit=500, M=Identity(), opt=am.options("pcg64"))
    r = am.amp_pcg(A, b, tol=1e-10, maxit=500, M=Identity(), opt=am.options(preset, verify=False))
    assert r.status == 0
    assert r.relres_true <= 2e-10                 # the paper's final-accuracy bound
    if preset != "amp16":
        # stepwise AMP-PCG(FP64) closely follows PCG(FP64)
        assert abs(r.iters - r64.iters) <= max(3, 0.05 * r64.iters)


def test_attainable_accuracy_after_ur_switch():
    # Section 5.2: with u_r reduced by the selector the true residual still
    # reaches the tolerance (no stopping test, run well past it)
    A, b = _ex1()
    for tol in (1e-6, 1e-8):
        rr = am.amp_pcg(A, b, tol=tol, maxit=400, M=Identity(), opt=am.options("amp_ur", verify=False))
        assert rr.k_r32 > 0
        assert rr.relres_true <= 2 * tol


# ------------------------------------------------------------- linear convergence (Ex. 4)

def test_example4_fp16_from_start_keeps_rate():
    lam = P.paper_spectrum("ex4")
    A = sp.csr_matrix(P.spectrum_matrix(lam, seed=(4, 0)))
    b = np.random.default_rng([4, 9]).standard_normal(lam.size)
    r64 = am.amp_pcg(A, b, tol=1e-10, maxit=500, M=Identity(), opt=am.options("pcg64"))
    r16 = am.amp_pcg(A, b, tol=1e-10, maxit=500, M=Identity(), opt=am.options("amp16", eta="linear"))
    assert r16.status == 0 and r16.relres_true <= 1e-10
    assert r16.iters <= r64.iters + 2


# ------------------------------------------------------------- workloads in miniature

@pytest.mark.parametrize("preset,slack", [("amp64", 1.05), ("amp16", 1.30)])
def test_blocky_diffusion_amp_vs_fp64(preset, slack):
    # stepwise AMP-PCG(FP64) keeps PCG(FP64)'s iteration count; FP16 z, p
    # from the first iteration costs iterations on this superlinear problem
    # (the behaviour Section 5.4 reports for its SuiteSparse matrices)
    A, b, _ = P.blocky_diffusion3d_system(24, 4)
    x_o, info = cpcg.pcg(A, b, tol=1e-10, maxit=5000)
    r = am.amp_pcg(A, b, tol=1e-10, maxit=5000, opt=am.options(preset))
    assert r.status == 0
    assert r.relres_true <= 1e-10
    assert r.iters <= slack * info["iters"]


def test_difference_form_spmv_keeps_rate():
    # high-contrast coefficients: the textbook FP32 product loses accuracy
    # to cancellation (Assumption 1 with C = 1 fails) and costs iterations
    # after the u_r switch; the row-sum/difference form does not
    A, b, _ = P.blocky_diffusion3d_system(32, 8)
    _, info = cpcg.pcg(A, b, tol=1e-10, maxit=5000)
    rd = am.amp_pcg(A, b, tol=1e-10, maxit=5000, opt=am.options("amp_ur", spmv32="diff"))
    rp = am.amp_pcg(A, b, tol=1e-10, maxit=5000, opt=am.options("amp_ur", spmv32="plain"))
    assert rd.status == 0 and rp.status == 0
    assert rd.k_r32 > 0
    assert rd.iters <= 1.02 * info["iters"]
    assert rd.iters <= rp.iters
    S = A.to_scipy()
    p = np.random.default_rng([7, 7]).standard_normal(A.n).astype(np.float16)
    exact = S @ p.astype(np.float64)
    f = am._diff_spmv32(S)
    assert np.allclose(f(p), exact, rtol=1e-5, atol=1e-5 * np.abs(exact).max())


def test_chebyshev_model_fp16_converges():
    A, b, xs, (lo, hi) = P.q1_system(16)
    S = A.to_scipy()
    M = am.Chebyshev(S, lo, hi, 4)
    _, info = cpcg.pcg(A, b, tol=1e-10, maxit=2000, precond=cpcg.PC_CHEBYSHEV, degree=4,
                       lam_lo=lo, lam_hi=hi)
    r = am.amp_pcg(S, b, tol=1e-10, maxit=2000, M=M, opt=am.options("amp16"))
    assert r.status == 0 and r.relres_true <= 1e-10
    assert r.iters <= 1.10 * info["iters"] + 2


# ------------------------------------------------------------- residual replacement

@pytest.mark.parametrize("period", [5, 25])
def test_periodic_replacement_leaves_fp64_iterates(period):
    # In exact arithmetic r_k = b - A x_k, so replacing the recurrence
    # residual by the true one every K iterations leaves CG's iterates
    # unchanged: in FP64 the residual norms follow the C oracle's (Alg. 1)
    # to rounding and the iteration count is the oracle's.  A replacement
    # with the wrong sign, taken before the x update, or with a dropped
    # term would change the norms by O(1).
    A, b, _ = P.blocky_diffusion3d_system(24, 4)
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=5000, history=True)
    r = am.amp_pcg(A, b, tol=1e-10, maxit=5000, opt=am.options("pcg64", rr_period=period, verify=False))
    assert r.status == 0 and r.iters == io["iters"]
    assert r.replacements == r.iters // period
    d_model, d_oracle = np.asarray(r.delta), np.asarray(io["delta"])
    assert np.max(np.abs(d_model - d_oracle) / d_oracle) <= 1e-5
    assert np.linalg.norm(r.x - xo) <= 1e-12 * np.linalg.norm(xo)


def test_periodic_replacement_in_fp32_reaches_tolerance():
    # with r and q in FP32 after the switch, periodic FP64 replacements keep
    # the true residual at the tolerance and the oracle's iteration count
    A, b, _ = P.blocky_diffusion3d_system(24, 4)
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=5000)
    r = am.amp_pcg(A, b, tol=1e-10, maxit=5000, opt=am.options("amp_ur", rr_period=5, verify=False))
    assert r.status == 0 and r.k_r32 > 0
    assert abs(r.iters - io["iters"]) <= max(2, 0.02 * io["iters"])
    assert r.relres_true <= 1e-10
    assert np.linalg.norm(r.x - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("preset", ["amp_ur", "amp64"])
def test_replacement_at_the_ur_switch(preset):
    # the u_r switch replaces r_k by fl32(b - A x_k): one replacement, and in
    # exact arithmetic nothing else changes -- with z, p in FP64 the residual
    # norms follow the FP64 oracle's to the accuracy of the FP32 residual,
    # and the iterate reaches the oracle's solution
    A, b, _ = P.blocky_diffusion3d_system(24, 4)
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=5000, history=True)
    on = am.amp_pcg(A, b, tol=1e-10, maxit=5000, opt=am.options(preset, rr_switch=True, verify=False))
    off = am.amp_pcg(A, b, tol=1e-10, maxit=5000, opt=am.options(preset, rr_switch=False, verify=False))
    assert on.k_r32 > 0 and on.k_r32 == off.k_r32
    assert on.replacements == 1 and off.replacements == 0
    assert abs(on.iters - io["iters"]) <= max(2, 0.02 * io["iters"])
    if preset == "amp_ur":   # z, p stay FP64: only r, q lose precision
        m = min(len(on.delta), len(io["delta"]))
        d_on, d_or = np.asarray(on.delta[:m]), np.asarray(io["delta"][:m])
        assert np.max(np.abs(d_on - d_or) / d_or) <= 1e-3
    assert on.relres_true <= 1e-10
    assert np.linalg.norm(on.x - xo) <= 1e-10 * np.linalg.norm(xo)
