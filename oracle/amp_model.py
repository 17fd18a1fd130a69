"""CPU model of AMP-PCG (Alg. 3 of Section 4) with every rounding written out.

TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
solver.

Precisions are named by their bit width: 64 (IEEE double), 32 (single),
16 (half).  ``fl(v, u)`` rounds to precision u (round to nearest even).

One iteration k, in the paper's order (Alg. 3):

1. eta_k: the delay indicator (eq. eta_k)
       eta_k = eps32 * sum_{t=k-d}^{k} ((3+C) delta_{t-1} + (2+C) delta_t)
   or the linear-regime indicator (eq. linear criterion)
       eta_k = eps32 (5+2C) delta_{k-1} / (1 - rate),
       rate = (delta_k / delta_{k-l})^(1/l).
   Undefined (no switch) while the window is incomplete (k < d+1 or k < l)
   or when rate >= 1.
2. precisionSelector (eq. precision_selector): u_z from nu_k = delta_k/||b||
   against tau_zs, tau_zh and u0; u_r = FP32 once eta_k <= tol ||b|| (the
   form of eq. precision switch criterion).  Both are latched: a precision,
   once lowered, is never raised again.
3. y = omega_k r computed in u_r, stored in u_z.
4. z = M^{-1} y computed and stored in u_z.
5. rho = r^T z (FP64);  beta_{k-1} = rho_k / rho_{k-1} (k > 0).
6. p = z + beta p computed and stored in u_z (at a u_z switch p_{k-1} is
   first rounded to the new u_z).
7. q = A p computed and stored in u_r (A's values rounded to u_r,
   accumulation in u_r).
8. gamma = q^T p, alpha = rho/gamma (FP64).
9. x += alpha p (FP64);  r -= alpha q in u_r;  delta = ||r|| (FP64).
10. stop when delta <= tol ||b||.

Readings where the paper leaves a choice (each one is also listed in the
design notes):

* "compute in FP16" is done in FP32 with a round to FP16 on store.
* omega_k: ``scaling="paper"`` is omega_k = 1/delta_k as in Alg. 3.
  ``scaling="pow2"`` (default) is a power of two, omega_k = 2^{e_k}, with
      e_k = min(e_z(k), e_{k-1} + T_p - ceil(log2 max|p^_{k-1}|))   (k > 0)
  where p^ = omega p is the stored direction and e_z(k) aims max|z^_k| at
  2^{T_z}:
      Jacobi:    e_z(k) = T_z - ceil(log2(max|r_k| max dinv))  (a hard bound:
                 max|z^| <= 2^{T_z}, max|y^| <= 2^{T_z+1});
      Chebyshev: e_z(0) = T_z - ceil(log2(max|r_0| G)), G = max(D^{-1}) /
                 lam_lo bounds the polynomial's gain; for k > 0
                 e_z(k) = e_{k-1} + T_z - ceil(log2(max|z^_{k-1}| max|r_k| / max|r_{k-1}|)).
  The carried part of the next p stays below beta 2^{T_p}.  Any nonzero
  omega_k gives the same iterates in exact arithmetic (Thm. dspcg); a power
  of two also gives the same iterates in floating point, away from
  overflow and underflow.
* Jacobi: M = diag(A).  Its inverse is stored in u_z; in FP16 it is stored
  as fl16(dinv 2^{s_d}) with s_d = -ceil(log2 max dinv), and the factor
  2^{-s_d} is folded into omega (so max dinv16 lies in (1/2, 1]).
* Chebyshev (degree m): z = D^{-1/2} s(B) D^{-1/2} y with B = D^{-1/2} A
  D^{-1/2} stored in FP16 (|b_ij| <= 1) and D^{-1/2} in FP32; the
  recurrence's work vectors are kept in the arithmetic precision of u_z
  (FP32 for FP16), B products accumulate in FP32 (FP64 when u_z is FP64),
  and z itself is stored in u_z.
* q = A p in FP32 (u_r = FP32) is evaluated in row-sum/difference form,
      q_i = s_i p_i + sum_{j != i} a_ij (p_j - p_i),   s_i = sum_j a_ij,
  with s_i formed in FP64 and the a_ij and s_i rounded to FP32
  (``spmv32="diff"``, default).  It equals A p in exact arithmetic; its
  rounding error is relative to |a_ij| |p_j - p_i| instead of |a_ij| |p_j|,
  which keeps Assumption 1 (eq. bound Ap) true with a modest C for
  diffusion-type matrices whose rows nearly sum to zero.  ``spmv32="plain"``
  is the textbook sum_j fl32(a_ij) p_j.  With u_r = FP64 the textbook form
  is used.
* Termination: after the updated residual passes, the true residual
  b - A x is formed in FP64.  If it is above tol ||b||, r is replaced by it
  and the iteration continues (at most ``max_replacements`` times).  With
  ``verify=False`` the model stops exactly as Alg. 3 does.
* Residual replacement (mentioned in Sections 1.1 and 3.1 as a way to keep
  the recurrence residual close to the true one): at the iteration k where
  u_r first drops to FP32, r_k is not the FP64 recurrence residual rounded
  to FP32 but the true residual fl32(b - A x_k), formed in FP64
  (``rr_switch=True``, default).  delta_k keeps the recurrence value that
  drove the decision; z_k, rho_k and everything after use the replaced
  r_k.  ``rr_period = K > 0`` also replaces r by fl_{u_r}(b - A x) after
  every K-th iteration.
* A pre-loop test returns 0 iterations when ||r_0|| <= tol ||b||.
"""

from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np
import scipy.sparse as sp

EPS32 = 2.0 ** -24   # unit roundoff of IEEE single
EPS64 = 2.0 ** -53   # unit roundoff of IEEE double
NP = {64: np.float64, 32: np.float32, 16: np.float16}

ST_CONVERGED, ST_ARG, ST_MAXIT, ST_BREAKDOWN = 0, 1, 2, 3


def fl(v, u):
    return np.asarray(v).astype(NP[u])


def compute_type(u):
    """Arithmetic precision used for quantities stored in u."""
    return 32 if u == 16 else u


def lower(a, b):
    return min(a, b)


@dataclass
class AmpOptions:
    u0: int = 64
    tau_zs: float = 1e-4
    tau_zh: float = 1e-6
    eta: str = "delay"          # delay | linear | fixed64 | fixed32
    d: int = 10
    C: float = 1.0
    ell: int = 5
    scaling: str = "pow2"       # pow2 | paper | none (Alg. 1, omega = 1)
    T_z: int = 12
    T_p: int = 12
    verify: bool = True
    max_replacements: int = 3
    rr_period: int = 0          # 0: no periodic replacement
    rr_switch: bool = True      # replace r by fl32(b - A x) at the u_r switch
    spmv32: str = "diff"        # diff | plain


PRESETS = {
    "pcg64": AmpOptions(u0=64, tau_zs=0.0, tau_zh=0.0, eta="fixed64"),
    "amp64": AmpOptions(u0=64),
    "amp16": AmpOptions(u0=16),
    "amp_ur": AmpOptions(u0=64, tau_zs=0.0, tau_zh=0.0),
}


def options(preset="amp64", **kw):
    return replace(PRESETS[preset], **kw)


# ---------------------------------------------------------------------------
# attainable-accuracy indicators and the precision selector
# ---------------------------------------------------------------------------

def eta_delay(delta, k, d=10, C=1.0):
    """eq. (eta_k); ``delta[t]`` = ||r_t||.  inf while t-1 < 0 for t = k-d."""
    if k - d - 1 < 0:
        return math.inf
    s = 0.0
    for t in range(k - d, k + 1):
        s = s + ((3.0 + C) * delta[t - 1] + (2.0 + C) * delta[t])
    return EPS32 * s


def eta_linear(delta, k, ell=5, C=1.0):
    """eq. (linear criterion) left-hand side; inf when undefined."""
    if k < ell or k < 1 or not delta[k - ell] > 0.0:
        return math.inf
    rate = (delta[k] / delta[k - ell]) ** (1.0 / ell)
    if not rate < 1.0:
        return math.inf
    return EPS32 * (5.0 + 2.0 * C) * delta[k - 1] / (1.0 - rate)


def eta_value(opt: AmpOptions, delta, k):
    if opt.eta == "delay":
        return eta_delay(delta, k, opt.d, opt.C)
    if opt.eta == "linear":
        return eta_linear(delta, k, opt.ell, opt.C)
    if opt.eta == "fixed32":
        return -math.inf
    return math.inf


def precision_selector(nu, u0, tau_zs, tau_zh, eta, tol_bnorm):
    """eq. (precision_selector) with the switch test eta <= tol ||b||."""
    if nu >= tau_zs:
        uz = u0
    elif nu >= tau_zh:
        uz = lower(u0, 32)
    else:
        uz = lower(u0, 16)
    ur = 32 if eta <= tol_bnorm else 64
    return uz, ur


def replay_switches(delta, bnorm, tol, opt: AmpOptions):
    """Run the latched selector over a recorded residual-norm history.
    Returns (k_z32, k_z16, k_r32): the first iteration whose selected u_z is
    <= FP32, <= FP16, and whose u_r is FP32 (-1 if never)."""
    uz, ur = opt.u0, 64
    kz32 = 0 if uz <= 32 else -1
    kz16 = 0 if uz <= 16 else -1
    kr = -1
    for k in range(len(delta)):
        s_uz, s_ur = precision_selector(delta[k] / bnorm, opt.u0, opt.tau_zs, opt.tau_zh,
                                        eta_value(opt, delta, k), tol * bnorm)
        uz, ur = lower(uz, s_uz), lower(ur, s_ur)
        if uz <= 32 and kz32 < 0:
            kz32 = k
        if uz <= 16 and kz16 < 0:
            kz16 = k
        if ur <= 32 and kr < 0:
            kr = k
    return kz32, kz16, kr


# ---------------------------------------------------------------------------
# preconditioners in reduced precision
# ---------------------------------------------------------------------------

class Jacobi:
    """M = diag(A); the inverse is stored per precision (FP16 as
    fl16(dinv 2^{s_d}), the factor 2^{-s_d} folded into omega)."""

    kind = "jacobi"

    def __init__(self, A: sp.csr_matrix):
        d = A.diagonal().astype(np.float64)
        if not np.all(d > 0):
            raise ValueError("Jacobi needs a positive diagonal")
        self.dinv64 = 1.0 / d
        self.s_d = -_ceil_log2(float(self.dinv64.max()))
        self.dinv = {64: self.dinv64, 32: fl(self.dinv64, 32),
                     16: fl(self.dinv64 * 2.0 ** self.s_d, 16)}
        self.log2_extra = {64: 0, 32: 0, 16: self.s_d}
        self.gain = float(self.dinv64.max())       # max|M^{-1} r| <= gain max|r|

    def apply(self, y_uz, uz):
        c = NP[compute_type(uz)]
        return fl(y_uz.astype(c) * self.dinv[uz].astype(c), uz)

    def apply64(self, r):
        return r * self.dinv64


class Chebyshev:
    """Degree-m Chebyshev polynomial preconditioner on B = D^{-1/2} A D^{-1/2}
    (three-term Chebyshev iteration for B w = v from w = 0)."""

    kind = "chebyshev"

    def __init__(self, A: sp.csr_matrix, lam_lo, lam_hi, degree=4):
        d = A.diagonal().astype(np.float64)
        if not np.all(d > 0):
            raise ValueError("Chebyshev needs a positive diagonal")
        if not (0.0 < lam_lo < lam_hi) or degree < 1:
            raise ValueError("Chebyshev needs 0 < lam_lo < lam_hi and degree >= 1")
        self.isq64 = 1.0 / np.sqrt(d)
        Dm = sp.diags(self.isq64)
        B = (Dm @ A @ Dm).tocsr()
        B.sort_indices()
        self.B64 = B
        b16 = fl(B.data, 16)
        self.B16 = {64: sp.csr_matrix((b16.astype(np.float64), B.indices, B.indptr), shape=B.shape),
                    32: sp.csr_matrix((b16.astype(np.float32), B.indices, B.indptr), shape=B.shape)}
        self.isq = {64: self.isq64, 32: fl(self.isq64, 32)}
        self.lo, self.hi, self.m = float(lam_lo), float(lam_hi), int(degree)
        self.log2_extra = {64: 0, 32: 0, 16: 0}
        self.gain = float(self.isq64.max() ** 2) / self.lo

    def coefficients(self):
        """(1/theta, [(c1, c2) per product with B]) of the recurrence."""
        theta = 0.5 * (self.hi + self.lo)
        delta = 0.5 * (self.hi - self.lo)
        sigma = theta / delta
        rho = 1.0 / sigma
        cs = []
        for _ in range(self.m - 1):
            rho_n = 1.0 / (2.0 * sigma - rho)
            cs.append((rho_n * rho, 2.0 * rho_n / delta))
            rho = rho_n
        return 1.0 / theta, cs

    def _steps(self, v, Bmul, c):
        """The Chebyshev iteration for B w = v from w = 0, written on the
        iterates: x_0 = 0, x_1 = v / theta, and for k = 1 .. m-1
        x_{k+1} = x_k + c1_{k-1} (x_k - x_{k-1}) + c2_{k-1} (v - B x_k);
        w = x_m.  (With d_k = x_{k+1} - x_k and res_k = v - B x_k this is the
        direction form d_k = c1 d_{k-1} + c2 res_k: the same polynomial.)"""
        inv_theta, cs = self.coefficients()
        x_prev = np.zeros_like(v)
        x = v * c(inv_theta)
        for k in range(1, self.m):
            c1, c2 = cs[k - 1]
            res = v - Bmul(x)
            x_new = (x + c(c1) * (x - x_prev)) + c(c2) * res
            x_prev, x = x, x_new
        return x

    def apply(self, y_uz, uz):
        cu = compute_type(uz)
        c = NP[cu]
        Bm = self.B16[cu]
        v = self.isq[cu] * y_uz.astype(c)
        w = self._steps(v, lambda u: (Bm @ u).astype(c), c)
        return fl(self.isq[cu] * w, uz)

    def apply64(self, r):
        """The same polynomial with every step in FP64 and the FP64 matrix."""
        v = self.isq64 * r
        w = self._steps(v, lambda u: self.B64 @ u, np.float64)
        return self.isq64 * w


# ---------------------------------------------------------------------------
# the solver
# ---------------------------------------------------------------------------

@dataclass
class AmpResult:
    x: np.ndarray
    iters: int
    status: int
    relres: float
    relres_true: float
    bnorm: float
    k_z32: int = -1
    k_z16: int = -1
    k_r32: int = -1
    replacements: int = 0
    delta: list = field(default_factory=list)
    uz: list = field(default_factory=list)
    ur: list = field(default_factory=list)
    omega: list = field(default_factory=list)
    rho: list = field(default_factory=list)
    gamma: list = field(default_factory=list)
    alpha: list = field(default_factory=list)


def _diff_spmv32(A):
    """q = A p in FP32 in row-sum/difference form (see module docstring)."""
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    off = A.indices != rows
    a32 = np.where(off, A.data, 0.0).astype(np.float32)
    s32 = fl(np.asarray(A.sum(axis=1)).ravel(), 32)
    starts = A.indptr[:-1]
    nonempty = np.diff(A.indptr) > 0

    def apply(p):
        p32 = p.astype(np.float32)
        terms = a32 * (p32[A.indices] - p32[rows])
        acc = np.zeros(n, dtype=np.float32)
        acc[nonempty] = np.add.reduceat(terms, starts[nonempty])
        return fl(s32 * p32 + acc, 32)

    return apply


def _ceil_log2(v):
    """ceil(log2 v) for v > 0, exactly (from the binary exponent)."""
    m, e = math.frexp(v)
    return e - 1 if m == 0.5 else e


def scale_exponent(M, opt, k, maxr, maxr_prev, e_prev, maxz_prev, maxp_prev):
    """e_k of the pow2 scaling rule (see the module docstring)."""
    if maxr <= 0.0:
        return 0 if e_prev is None else e_prev
    if M.kind == "jacobi" or k == 0 or not maxz_prev > 0.0:
        e = opt.T_z - _ceil_log2(maxr * M.gain)
    else:
        e = e_prev + opt.T_z - _ceil_log2(maxz_prev * maxr / maxr_prev)
    if k > 0 and maxp_prev > 0.0:
        e = min(e, e_prev + opt.T_p - _ceil_log2(maxp_prev))
    return e


def amp_pcg(A, b, x0=None, tol=1e-10, maxit=5000, M=None, opt: AmpOptions | None = None):
    """AMP-PCG(u0) of Alg. 3.  ``A`` is a scipy CSR (float64) or an object
    with ``to_scipy()``; ``M`` a :class:`Jacobi` / :class:`Chebyshev`
    (default Jacobi).  Returns :class:`AmpResult`."""
    opt = opt or AmpOptions()
    if hasattr(A, "to_scipy"):
        A = A.to_scipy()
    A = A.tocsr()
    n = A.shape[0]
    Aplanes = {64: A, 32: sp.csr_matrix((fl(A.data, 32), A.indices, A.indptr), shape=A.shape)}
    spmv = {64: lambda v: fl(A @ v.astype(np.float64), 64)}
    if opt.spmv32 == "diff":
        spmv[32] = _diff_spmv32(A)
    else:
        spmv[32] = lambda v: fl(Aplanes[32] @ v.astype(np.float32), 32)
    M = M if M is not None else Jacobi(A)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    bnorm = float(np.sqrt(np.dot(b, b)))
    tol_b = tol * bnorm

    r = b - A @ x                      # FP64, stored in u_{r,-1} = FP64
    delta = [float(np.sqrt(np.dot(r, r)))]
    res = AmpResult(x, 0, ST_MAXIT, 0.0, 0.0, bnorm)
    res.delta = delta
    uz_prev, ur_prev = opt.u0, 64
    p = None
    rho_prev = None
    e_prev = None
    maxr_prev = maxz_prev = maxp_prev = 0.0
    replacements = 0
    iters = 0

    def finish(status):
        res.x, res.iters, res.status = x, iters, status
        res.relres = delta[-1] / bnorm if bnorm > 0 else 0.0
        t = b - A @ x
        res.relres_true = float(np.sqrt(np.dot(t, t))) / bnorm if bnorm > 0 else 0.0
        res.replacements = replacements
        return res

    if delta[0] <= tol_b:
        return finish(ST_CONVERGED)

    for k in range(maxit):
        # 1-2: indicator and latched precision selection
        eta = eta_value(opt, delta, k)
        s_uz, s_ur = precision_selector(delta[k] / bnorm, opt.u0, opt.tau_zs, opt.tau_zh, eta, tol_b)
        uz, ur = lower(uz_prev, s_uz), lower(ur_prev, s_ur)
        if uz <= 32 and res.k_z32 < 0:
            res.k_z32 = k
        if uz <= 16 and res.k_z16 < 0:
            res.k_z16 = k
        maxr = float(np.max(np.abs(r.astype(np.float64))))   # max|r_k| as stored
        if ur != ur_prev:
            res.k_r32 = k
            if opt.rr_switch:          # r_k replaced by the true residual, held in u_{r,k}
                r = fl(b - A @ x, ur)
                replacements += 1
            else:                      # r_k now held in u_{r,k}
                r = fl(r, ur)
        res.uz.append(uz)
        res.ur.append(ur)
        cr = NP[ur]

        # 3: dynamic scaling
        if opt.scaling == "paper":
            omega, e_k = 1.0 / delta[k], None
        elif opt.scaling == "none":
            omega, e_k = 1.0, None
        else:
            e_k = scale_exponent(M, opt, k, maxr, maxr_prev, e_prev, maxz_prev, maxp_prev)
            omega = 2.0 ** e_k
        res.omega.append(omega)
        # the preconditioner's static storage scale is folded into omega
        omega_eff = omega * 2.0 ** (-M.log2_extra[uz])
        y = fl(r.astype(cr) * cr(omega_eff), ur)         # computed in u_r
        y = fl(y, uz)                                     # stored in u_z
        # 4: z = M^{-1} y in u_z
        z = M.apply(y, uz)
        maxz_prev = float(np.max(np.abs(z.astype(np.float64))))
        # 5: rho, beta
        rho = float(np.dot(r.astype(np.float64), z.astype(np.float64)))
        beta = rho / rho_prev if k > 0 else 0.0
        # 6: p = z + beta p in u_z (at a u_z switch p_{k-1} is first rounded to u_z)
        cz = NP[compute_type(uz)]
        if p is None:
            p = fl(z, uz)
        else:
            if p.dtype != NP[uz]:
                p = fl(p, uz)
            p = fl(z.astype(cz) + cz(beta) * p.astype(cz), uz)
        maxp_prev = float(np.max(np.abs(p.astype(np.float64))))
        e_prev, maxr_prev = e_k, maxr
        # 7: q = A p in u_r
        q = spmv[ur](p)
        # 8: gamma, alpha
        gamma = float(np.dot(q.astype(np.float64), p.astype(np.float64)))
        with np.errstate(all="ignore"):
            alpha = rho / gamma if gamma != 0.0 else math.inf
        res.rho.append(rho)
        res.gamma.append(gamma)
        res.alpha.append(alpha)
        if not (rho > 0.0) or not (gamma > 0.0) or not math.isfinite(alpha):
            iters = k
            return finish(ST_BREAKDOWN)
        # 9: updates
        x = x + alpha * p.astype(np.float64)
        r = fl(r.astype(cr) - cr(alpha) * q.astype(cr), ur)
        dk = float(np.sqrt(np.dot(r.astype(np.float64), r.astype(np.float64))))
        iters = k + 1
        uz_prev, ur_prev, rho_prev = uz, ur, rho
        if opt.rr_period and iters % opt.rr_period == 0:
            r = fl(b - A @ x, ur)
            dk = float(np.sqrt(np.dot(r.astype(np.float64), r.astype(np.float64))))
            replacements += 1
        delta.append(dk)
        # 10: stopping test (+ true-residual verification)
        if dk <= tol_b:
            if not opt.verify:
                return finish(ST_CONVERGED)
            t = b - A @ x
            tn = float(np.sqrt(np.dot(t, t)))
            if tn <= tol_b:
                return finish(ST_CONVERGED)
            if replacements >= opt.max_replacements:
                return finish(ST_MAXIT)
            replacements += 1
            r = fl(t, ur)
            delta[-1] = float(np.sqrt(np.dot(r.astype(np.float64), r.astype(np.float64))))
    return finish(ST_MAXIT)


def naive_pcg(A, b, u, tol=1e-10, maxit=1000):
    """Alg. 1 with M = I and every vector and scalar in one precision u (the
    motivating experiment of Section 2).  Returns (x, iters, status, delta)."""
    if hasattr(A, "to_scipy"):
        A = A.to_scipy()
    c = NP[u]
    Au = fl(A.toarray() if sp.issparse(A) else A, u)
    bu = fl(b, u)
    x = np.zeros(len(b), dtype=c)
    r = bu.copy()
    bnorm = float(np.sqrt(np.dot(bu.astype(np.float64), bu.astype(np.float64))))
    delta = [bnorm]
    p = None
    rho_prev = None
    with np.errstate(all="ignore"):
        for k in range(maxit):
            z = r.copy()
            rho = c(np.dot(r, z))
            if k > 0:
                beta = c(rho / rho_prev)
                p = fl(z + beta * p, u)
            else:
                p = z
            q = fl(Au @ p, u)
            gamma = c(np.dot(q, p))
            alpha = c(rho / gamma)
            x = fl(x + alpha * p, u)
            r = fl(r - alpha * q, u)
            dk = float(np.sqrt(np.dot(r.astype(np.float64), r.astype(np.float64))))
            delta.append(dk)
            rho_prev = rho
            if not np.isfinite(dk) or not np.all(np.isfinite(x)) or not np.isfinite(float(beta if k > 0 else 0.0)):
                return x, k + 1, ST_BREAKDOWN, delta
            if dk <= tol * bnorm:
                return x, k + 1, ST_CONVERGED, delta
    return x, maxit, ST_MAXIT, delta
