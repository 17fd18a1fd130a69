"""Eigenvalue bounds of D^{-1} A for the Chebyshev preconditioner when the
caller has none: a plain FP64 Lanczos process.

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
solver.

The Chebyshev preconditioner needs an interval [lam_lo, lam_hi] holding the
spectrum of D^{-1} A (the paper uses Chebyshev only as a smoother, Section
5.3, and gives no estimation rule).  The reading taken here (the survey's
R17): lam_hi = 1.05 times the largest Ritz value of 24 Lanczos steps, and
lam_lo = lam_hi / 30.

* D^{-1} A is similar to the symmetric B = D^{-1/2} A D^{-1/2}, so the
  Lanczos process runs on B: v_0 = u / ||u||, beta_0 = 0, and for
  j = 0, 1, ...:  w = B v_j;  alpha_j = w^T v_j;
  w = w - alpha_j v_j - beta_j v_{j-1};  beta_{j+1} = ||w||;
  v_{j+1} = w / beta_{j+1}.  The Ritz values are the eigenvalues of the
  tridiagonal T with diagonal alpha and off-diagonal beta_1, beta_2, ...;
  they lie inside [lambda_min, lambda_max] of B, and the extreme ones
  converge first.  The process stops early when beta_{j+1} <= 1e-14 times
  the largest |alpha| (an invariant subspace: the Ritz values are then
  eigenvalues).
* The start vector u is counter-based: u_i = 2 U(i) - 1 with U(i) the top
  53 bits of splitmix64 at counter i + 1 (Steele, Lea and Flood, "Fast
  splittable pseudorandom number generators", OOPSLA 2014), scaled to
  [0, 1).
"""

from __future__ import annotations

import numpy as np

GOLDEN_GAMMA = 0x9E3779B97F4A7C15
LANCZOS_STEPS = 24
HI_MARGIN = 1.05
LO_RATIO = 30.0


def splitmix64(counter):
    """splitmix64's output for state seed + counter * GOLDEN_GAMMA (seed 0),
    vectorised over an array of counters (uint64, wrapping arithmetic)."""
    z = np.asarray(counter, dtype=np.uint64) * np.uint64(GOLDEN_GAMMA)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def start_vector(n: int) -> np.ndarray:
    """u_i = 2 * (splitmix64(i + 1) >> 11) * 2^-53 - 1, i = 0 .. n-1."""
    with np.errstate(over="ignore"):
        bits = splitmix64(np.arange(1, n + 1, dtype=np.uint64)) >> np.uint64(11)
    return 2.0 * bits.astype(np.float64) * 2.0 ** -53 - 1.0


def lanczos(A, steps: int = LANCZOS_STEPS):
    """Lanczos on B = D^{-1/2} A D^{-1/2} (A: scipy sparse or dense, SPD with
    a positive diagonal).  Returns (alpha, beta): T's diagonal and
    off-diagonal."""
    d = np.asarray(A.diagonal(), dtype=np.float64)
    s = 1.0 / np.sqrt(d)
    n = d.size

    def B(v):
        return s * (A @ (s * v))

    v = start_vector(n)
    v = v / np.sqrt(np.dot(v, v))
    v_prev = np.zeros(n)
    beta = 0.0
    alpha, betas = [], []
    for j in range(min(steps, n)):
        w = B(v)
        a = float(np.dot(w, v))
        w = w - a * v - beta * v_prev
        alpha.append(a)
        beta_next = float(np.sqrt(np.dot(w, w)))
        if j == min(steps, n) - 1 or beta_next <= 1e-14 * max(abs(x) for x in alpha):
            break
        betas.append(beta_next)
        v_prev, v, beta = v, w / beta_next, beta_next
    return np.array(alpha), np.array(betas)


def ritz_values(alpha, beta) -> np.ndarray:
    k = len(alpha)
    T = np.diag(alpha)
    if k > 1:
        T += np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    return np.linalg.eigvalsh(T)


def chebyshev_bounds(A, steps: int = LANCZOS_STEPS):
    """(lam_lo, lam_hi) for the Chebyshev preconditioner, and the Ritz
    extremes (theta_min, theta_max) they come from."""
    theta = ritz_values(*lanczos(A, steps))
    hi = HI_MARGIN * float(theta[-1])
    return (hi / LO_RATIO, hi), (float(theta[0]), float(theta[-1]))
