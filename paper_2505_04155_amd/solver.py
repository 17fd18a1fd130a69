"""torch-facing wrappers of the AMP-PCG C ABI.

Tensors are plain device memory here: every arithmetic step of the solve
runs inside libamppcg.so.  All calls use torch's current HIP stream.
"""

from __future__ import annotations

import ctypes
import sys

import torch

from . import binding as B

_TORCH = {64: torch.float64, 32: torch.float32, 16: torch.float16}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _need(t: torch.Tensor, dtype, n=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")


class Matrix:
    """Solver-side matrix (sliced ELL, FP64 and FP32 value planes)."""

    def __init__(self, row_ptr: torch.Tensor, col_idx: torch.Tensor, val: torch.Tensor, offsets: bool = True,
                 lanes: int = 1):
        """lanes: lanes per row (1, 2, 4, 8, 16; 0 = chosen from the mean row length)."""
        L = B.load()
        n = row_ptr.numel() - 1
        _need(row_ptr, torch.int32, name="row_ptr")
        _need(col_idx, torch.int32, name="col_idx")
        _need(val, torch.float64, col_idx.numel(), name="val")
        csr = B.Csr(n, col_idx.numel(), row_ptr.data_ptr(), col_idx.data_ptr(), val.data_ptr())
        t = B.MatrixTuning()
        L.amp_matrix_tuning_default(ctypes.byref(t))
        t.lanes_per_row = int(lanes)
        t.offset_mode = 1 if offsets else 0
        h = ctypes.c_void_p()
        B.check(L.amp_matrix_create(ctypes.byref(csr), ctypes.byref(t), _stream(), ctypes.byref(h)),
                "amp_matrix_create")
        self._h = h
        self.n = n
        self.nnz = col_idx.numel()

    @classmethod
    def from_hexop(cls, H):
        """A handle over a HexOperator (matrix-free; Jacobi or identity
        preconditioner).  Keeps H alive."""
        m = cls.__new__(cls)
        h = ctypes.c_void_p()
        B.check(B.load().amp_matrix_from_hexop(H._h, _stream(), ctypes.byref(h)), "amp_matrix_from_hexop")
        m._h = h
        m.n = H.n
        m.nnz = 0
        m._hexop = H
        return m

    @classmethod
    def from_csr(cls, csr, device="cuda", offsets: bool = True, lanes: int = 1):
        """From a workloads.CSR (host numpy arrays)."""
        rp = torch.from_numpy(csr.row_ptr).to(device)
        ci = torch.from_numpy(csr.col_idx).to(device)
        v = torch.from_numpy(csr.val).to(device)
        return cls(rp, ci, v, offsets=offsets, lanes=lanes)

    @property
    def handle(self):
        return self._h

    def info(self):
        st = B.MatrixStats()
        B.check(B.load().amp_matrix_info(self._h, ctypes.byref(st)), "amp_matrix_info")
        return {name: getattr(st, name) for name, _ in B.MatrixStats._fields_}

    def spmv(self, p: torch.Tensor, u_r: int = 64, diff: bool = True):
        """q = A p with the solver's kernel; p's dtype selects its storage
        precision, u_r the value plane / arithmetic.  Returns (q, gamma)."""
        u_p = {torch.float64: 64, torch.float32: 32, torch.float16: 16}[p.dtype]
        _need(p, p.dtype, self.n, "p")
        q = torch.empty(self.n, dtype=_TORCH[u_r], device=p.device)
        g = torch.zeros(1, dtype=torch.float64, device=p.device)
        B.check(B.load().amp_spmv(self._h, u_r, u_p, 1 if diff else 0, _ptr(p), _ptr(q), _ptr(g), _stream()),
                "amp_spmv")
        return q, g

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and B._lib is not None and not sys.is_finalizing():
            B._lib.amp_matrix_destroy(h)
            self._h = None


class Preconditioner:
    KINDS = {"identity": B.PC_IDENTITY, "jacobi": B.PC_JACOBI, "chebyshev": B.PC_CHEBYSHEV}

    def __init__(self, A: Matrix, kind: str = "jacobi", degree: int = 4, lam_lo: float = 0.0,
                 lam_hi: float = 0.0):
        h = ctypes.c_void_p()
        B.check(B.load().amp_precond_create(A.handle, self.KINDS[kind], int(degree), float(lam_lo),
                                            float(lam_hi), _stream(), ctypes.byref(h)),
                "amp_precond_create")
        self._h = h
        self.A = A
        self.kind = kind

    @classmethod
    def pmg(cls, A: Matrix, orders=(7, 3, 1), degree: int = 2, coarse_degree: int = 16, lo_ratio: float = 0.1,
            hi_margin: float = 1.1, coarse_lo_ratio: float = 0.01, rho=None, power_iters: int = 40):
        """The p-multigrid V-cycle over the polynomial orders ``orders`` for
        a matrix-free handle (Matrix.from_hexop): Chebyshev-Jacobi smoothing
        of degree ``degree`` on [lo_ratio rho, hi_margin rho], a degree
        ``coarse_degree`` polynomial on the lowest order.  ``rho``: lambda_max
        of D^-1 A per level (None or <= 0: estimated by the power
        iteration)."""
        L = B.load()
        p = B.PmgParams()
        L.amp_pmg_params_default(ctypes.byref(p))
        p.levels = len(orders)
        for i, N in enumerate(orders):
            p.orders[i] = int(N)
        p.degree, p.coarse_degree = int(degree), int(coarse_degree)
        p.lo_ratio, p.hi_margin, p.coarse_lo_ratio = float(lo_ratio), float(hi_margin), float(coarse_lo_ratio)
        for i in range(len(orders)):
            p.rho[i] = float(rho[i]) if rho is not None else 0.0
        p.power_iters = int(power_iters)
        h = ctypes.c_void_p()
        B.check(L.amp_precond_create_pmg(A.handle, ctypes.byref(p), _stream(), ctypes.byref(h)),
                "amp_precond_create_pmg")
        self = cls.__new__(cls)
        self._h = h
        self.A = A
        self.kind = "pmg"
        return self

    def pmg_info(self):
        """{"rho", "gain", "n", "orders", "bytes"} of a p-multigrid preconditioner."""
        st = B.PmgStats()
        B.check(B.load().amp_pmg_info(self._h, ctypes.byref(st)), "amp_pmg_info")
        L = st.params.levels
        return {"rho": [st.params.rho[i] for i in range(L)], "gain": st.gain, "n": [st.n[i] for i in range(L)],
                "orders": [st.params.orders[i] for i in range(L)], "bytes": st.bytes}

    def pmg_apply(self, r: torch.Tensor, prec: int = 64):
        """z = V(r): one cycle in FP64 (prec 64) or FP32 (prec 32); r and z FP64."""
        _need(r, torch.float64, self.A.n, "r")
        z = torch.empty_like(r)
        B.check(B.load().amp_pmg_apply(self._h, _ptr(r), _ptr(z), int(prec), _stream()), "amp_pmg_apply")
        return z

    @property
    def handle(self):
        return self._h

    def bounds(self):
        """Chebyshev: (lam_lo, lam_hi, ritz_min, ritz_max) -- the interval
        used (given, or estimated when a bound was passed as <= 0) and the
        Lanczos Ritz extremes it came from."""
        vals = [ctypes.c_double() for _ in range(4)]
        B.check(B.load().amp_precond_bounds(self._h, *[ctypes.byref(v) for v in vals]), "amp_precond_bounds")
        return tuple(v.value for v in vals)

    def apply(self, r: torch.Tensor, u_z: int, omega: float = 1.0):
        """z = M^{-1} fl_{u_z}(fl_{u_r}(omega r)); r's dtype gives u_r.  Returns (z, rho)."""
        u_r = {torch.float64: 64, torch.float32: 32}[r.dtype]
        _need(r, r.dtype, self.A.n, "r")
        z = torch.empty(self.A.n, dtype=_TORCH[u_z], device=r.device)
        rho = torch.zeros(1, dtype=torch.float64, device=r.device)
        B.check(B.load().amp_precond_apply(self._h, u_r, u_z, _ptr(r), float(omega), _ptr(z), _ptr(rho),
                                           _stream()), "amp_precond_apply")
        return z, rho

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and B._lib is not None and not sys.is_finalizing():
            B._lib.amp_precond_destroy(h)
            self._h = None


def solve(A: Matrix, M: Preconditioner, b: torch.Tensor, x0: torch.Tensor | None = None, tol: float = 1e-10,
          maxit: int = 5000, preset: str = "amp64", history: bool = False, raise_on_error: bool = False,
          **opts):
    """Solve A x = b with AMP-PCG (Alg. 3).  Returns (x, info)."""
    L = B.load()
    _need(b, torch.float64, A.n, "b")
    x = torch.zeros_like(b) if x0 is None else x0.detach().clone()
    _need(x, torch.float64, A.n, "x0")
    o = B.make_options(preset, **opts)
    dh = ph = sh = None
    if history:
        dh = torch.full((maxit + 1,), float("nan"), dtype=torch.float64, device=b.device)
        ph = torch.full((max(maxit, 1),), -1, dtype=torch.int32, device=b.device)
        sh = torch.full((4 * max(maxit, 1),), float("nan"), dtype=torch.float64, device=b.device)
        o.delta_history = dh.data_ptr()
        o.prec_history = ph.data_ptr()
        o.scalar_history = sh.data_ptr()
    res = B.Result()
    st = L.amp_pcg_solve(A.handle, M.handle, _ptr(b), _ptr(x), float(tol), int(maxit), ctypes.byref(o),
                         ctypes.byref(res), _stream())
    if st in (B.AMP_ERR_ARG, B.AMP_ERR_HIP, B.AMP_ERR_OOM) or (raise_on_error and st != B.AMP_OK):
        B.check(st, "amp_pcg_solve")
    info = dict(status=st, iters=res.iters, relres=res.rel_res_updated, relres_true=res.rel_res_true,
                bnorm=res.bnorm, k_z32=res.k_z32, k_z16=res.k_z16, k_r32=res.k_r32,
                replacements=res.n_replacements, t_solve_ms=res.t_solve_ms, spmv_ms=res.spmv_ms,
                spmv_launches=res.spmv_launches, cheb_ms=res.cheb_ms, cheb_launches=res.cheb_launches)
    if history:
        it = res.iters
        info["delta"] = dh[: it + 1].cpu().numpy()
        ph_h = ph[:it].cpu().numpy()
        info["uz"] = (ph_h & 0xFF).tolist()
        info["ur"] = (ph_h >> 8).tolist()
        scal = sh[: 4 * it].cpu().numpy().reshape(-1, 4)
        info["omega"], info["rho"], info["gamma"], info["alpha"] = (scal[:, j] for j in range(4))
    return x, info


def solve_batched(As, Ms, bs, x0s=None, tol=1e-10, maxit: int = 5000, preset: str = "amp64",
                  raise_on_error: bool = False, **opts):
    """Solve the independent systems As[i] x = bs[i] in one lockstep batched
    solve.  tol: a float or one per system.  Returns (xs, infos, status)."""
    L = B.load()
    n = len(As)
    if not (len(Ms) == len(bs) == n) or n == 0:
        raise ValueError("As, Ms and bs must be non-empty and of equal length")
    xs = []
    for i in range(n):
        _need(bs[i], torch.float64, As[i].n, f"b[{i}]")
        x = torch.zeros_like(bs[i]) if x0s is None or x0s[i] is None else x0s[i].detach().clone()
        _need(x, torch.float64, As[i].n, f"x0[{i}]")
        xs.append(x)
    tols = [float(tol)] * n if isinstance(tol, (int, float)) else [float(t) for t in tol]
    vp = ctypes.c_void_p
    a_arr = (vp * n)(*[A.handle.value for A in As])
    m_arr = (vp * n)(*[M.handle.value for M in Ms])
    b_arr = (vp * n)(*[b.data_ptr() for b in bs])
    x_arr = (vp * n)(*[x.data_ptr() for x in xs])
    t_arr = (ctypes.c_double * n)(*tols)
    res = (B.Result * n)()
    o = B.make_options(preset, **opts)
    st = L.amp_pcg_solve_batched(n, a_arr, m_arr, b_arr, x_arr, t_arr, int(maxit), ctypes.byref(o), res,
                                 _stream())
    if st in (B.AMP_ERR_ARG, B.AMP_ERR_HIP, B.AMP_ERR_OOM) or (raise_on_error and st != B.AMP_OK):
        B.check(st, "amp_pcg_solve_batched")
    infos = [dict(status=r.status, iters=r.iters, relres=r.rel_res_updated, relres_true=r.rel_res_true,
                  bnorm=r.bnorm, k_z32=r.k_z32, k_z16=r.k_z16, k_r32=r.k_r32, replacements=r.n_replacements,
                  t_solve_ms=r.t_solve_ms) for r in res]
    return xs, infos, st


def tune_group_rows(As, Ms, bs, tol=1e-10, iters: int = 32, candidates=(0, 1024, 2048, 4096, 8192),
                    preset: str = "amp64", **opts):
    """Rows-per-work-group autotuner (amp_tune_group_rows): times at most
    `iters` iterations of the solve -- single when one system is given,
    batched otherwise -- for each candidate group_rows (0: automatic) and
    returns (best, {candidate: ms per iteration}).  As, Ms, bs: a handle /
    tensor or equal-length lists of them."""
    L = B.load()
    if isinstance(As, Matrix):
        As, Ms, bs = [As], [Ms], [bs]
    n = len(As)
    if not (len(Ms) == len(bs) == n) or n == 0:
        raise ValueError("As, Ms and bs must be non-empty and of equal length")
    for i in range(n):
        _need(bs[i], torch.float64, As[i].n, f"b[{i}]")
    xs = [torch.empty_like(b) for b in bs]   # scratch
    tols = [float(tol)] * n if isinstance(tol, (int, float)) else [float(t) for t in tol]
    cands = [int(c) for c in candidates]
    vp = ctypes.c_void_p
    a_arr = (vp * n)(*[A.handle.value for A in As])
    m_arr = (vp * n)(*[M.handle.value for M in Ms])
    b_arr = (vp * n)(*[b.data_ptr() for b in bs])
    x_arr = (vp * n)(*[x.data_ptr() for x in xs])
    t_arr = (ctypes.c_double * n)(*tols)
    c_arr = (ctypes.c_int * len(cands))(*cands)
    ms = (ctypes.c_double * len(cands))()
    best = ctypes.c_int()
    o = B.make_options(preset, **opts)
    B.check(L.amp_tune_group_rows(n, a_arr, m_arr, b_arr, x_arr, t_arr, int(iters), c_arr, len(cands),
                                  ctypes.byref(o), ctypes.byref(best), ms, _stream()), "amp_tune_group_rows")
    return best.value, {c: ms[i] for i, c in enumerate(cands)}


def selector_replay(delta, bnorm: float, tol: float, preset: str = "amp64", **opts):
    """Host-only replay of the device controller's latched selector."""
    L = B.load()
    arr = (ctypes.c_double * len(delta))(*[float(d) for d in delta])
    o = B.make_options(preset, **opts)
    out = [ctypes.c_int(), ctypes.c_int(), ctypes.c_int()]
    B.check(L.amp_selector_replay(arr, len(delta), float(bnorm), float(tol), ctypes.byref(o),
                                  *[ctypes.byref(v) for v in out]), "amp_selector_replay")
    return tuple(v.value for v in out)


def paper_kernel_bytes(u_z: int, u_r: int):
    out = (ctypes.c_double * 4)()
    B.check(B.load().amp_paper_kernel_bytes(u_z, u_r, out), "amp_paper_kernel_bytes")
    return list(out)


_allocator_refs = []   # every callback pair ever set: blocks made with one are freed with it


def use_torch_allocator(device=None, record=None):
    """Route the library's device allocations (amp_set_allocator) through
    torch's caching allocator on `device` (default: the current one).
    record: optional list that receives ("alloc", ptr, bytes) and
    ("free", ptr) tuples."""
    L = B.load()
    dev = torch.cuda.current_device() if device is None else int(device)

    def _alloc(nbytes, ctx):
        try:
            ptr = torch.cuda.caching_allocator_alloc(int(nbytes), device=dev)
        except Exception:   # out of memory: the library reports AMP_ERR_OOM
            return None
        if record is not None:
            record.append(("alloc", ptr, int(nbytes)))
        return ptr

    def _free(ptr, ctx):
        if record is not None:
            record.append(("free", ptr))
        torch.cuda.caching_allocator_delete(ptr)

    refs = (B.ALLOC_FN(_alloc), B.FREE_FN(_free))
    _allocator_refs.append(refs)
    B.check(L.amp_set_allocator(refs[0], refs[1], None), "amp_set_allocator")


def use_hip_allocator():
    """Back to hipMalloc / hipFree for later allocations (blocks made by a
    caller allocator are still released through it)."""
    L = B.load()
    B.check(L.amp_set_allocator(B.ALLOC_FN(), B.FREE_FN(), None), "amp_set_allocator")


def tune_lanes(csr, candidates=(1, 2, 4, 8, 16), reps: int = 20, device="cuda"):
    """Lanes-per-row autotuner (amp_tune_lanes) for a workloads.CSR: returns
    (best, {candidate: microseconds per product})."""
    L = B.load()
    rp = torch.from_numpy(csr.row_ptr).to(device)
    ci = torch.from_numpy(csr.col_idx).to(device)
    v = torch.from_numpy(csr.val).to(device)
    c = B.Csr(csr.n, ci.numel(), rp.data_ptr(), ci.data_ptr(), v.data_ptr())
    cands = [int(x) for x in candidates]
    arr = (ctypes.c_int * len(cands))(*cands)
    us = (ctypes.c_double * len(cands))()
    best = ctypes.c_int()
    B.check(L.amp_tune_lanes(ctypes.byref(c), arr, len(cands), int(reps), ctypes.byref(best), us, _stream()),
            "amp_tune_lanes")
    return best.value, {x: us[i] for i, x in enumerate(cands)}


class HexOperator:
    """Matrix-free order-N hexahedral screened Poisson operator
    (amp_hexop_*): q = A p on the interior nodes of an ex x ey x ez box mesh
    whose element maps come from the vertex array ((ex+1)(ey+1)(ez+1), 3)."""

    def __init__(self, verts: torch.Tensor, E, order: int = 7, lam: float = 1e3):
        L = B.load()
        _need(verts, torch.float64, name="verts")
        ex, ey, ez = (int(e) for e in E)
        h = ctypes.c_void_p()
        B.check(L.amp_hexop_create(ex, ey, ez, int(order), _ptr(verts), float(lam), _stream(), ctypes.byref(h)),
                "amp_hexop_create")
        self._h = h
        st = B.HexStats()
        B.check(L.amp_hexop_info(h, ctypes.byref(st)), "amp_hexop_info")
        self.n, self.elements, self.local = st.n, st.elements, st.local
        self.order, self.lam, self.flops_per_element = st.order, st.lambda_, st.flops_per_element
        self.device = verts.device

    def apply(self, p: torch.Tensor, u_r: int = 64, mu: bool = True):
        """q = A p with p's dtype as its storage precision and u_r the
        arithmetic and q precision; returns (q, mu tensor or None)."""
        u_p = {torch.float64: 64, torch.float32: 32, torch.float16: 16}[p.dtype]
        _need(p, p.dtype, self.n, "p")
        q = torch.empty(self.n, dtype=_TORCH[u_r], device=p.device)
        m = torch.zeros(1, dtype=torch.float64, device=p.device) if mu else None
        B.check(B.load().amp_hexop_apply(self._h, u_p, u_r, _ptr(p), _ptr(q), _ptr(m) if mu else None, _stream()),
                "amp_hexop_apply")
        return q, m

    def diagonal(self):
        d = torch.empty(self.n, dtype=torch.float64, device=self.device)
        B.check(B.load().amp_hexop_diagonal(self._h, _ptr(d), _stream()), "amp_hexop_diagonal")
        return d

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and B._lib is not None and not sys.is_finalizing():
            B._lib.amp_hexop_destroy(h)
            self._h = None

