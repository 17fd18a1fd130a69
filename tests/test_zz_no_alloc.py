"""The allocation-free solve (amp_pcg_solve_noalloc) through the C ABI: the
same result as amp_pcg_solve, bit for bit, on calls in a row that share the
library's device array -- the second system smaller than the first, so what
the first left behind must not leak into it -- and a clear error above its
row limit."""

import ctypes

import numpy as np
import pytest
import torch

from workloads import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    import paper_2505_04155_amd as amp_mod
    from paper_2505_04155_amd import binding
    binding.load(build_if_missing=False)
    return amp_mod


def _say(msg):
    print(msg, flush=True)


def _noalloc(amp, M, pc, b, preset, tol=1e-10, maxit=5000, **kw):
    from paper_2505_04155_amd import binding as B
    L = B.load()
    x = torch.zeros_like(b)   # the caller's output, allocated before the call
    o = B.make_options(preset, **kw)
    res = B.Result()
    torch.cuda.synchronize()
    st = L.amp_pcg_solve_noalloc(M.handle, pc.handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                 float(tol), int(maxit), ctypes.byref(o), ctypes.byref(res),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return st, x, res


def _system(name):
    if name == "blocky32":
        A, b, _ = P.blocky_diffusion3d_system(32, 8)          # 32768 rows
        return A, b, "jacobi", {}
    if name == "blocky64":
        A, b, _ = P.blocky_diffusion3d_system(64, 8)          # 262144 rows: the limit
        return A, b, "jacobi", {}
    if name == "poisson64":
        A, b, _ = P.poisson2d_system(64)                       # 4096 rows
        return A, b, "jacobi", {}
    if name == "q1_20":
        A, b, _, (lo, hi) = P.q1_system(20)                    # 8000 rows, 27-point
        return A, b, "chebyshev", {"degree": 4, "lam_lo": lo, "lam_hi": hi}
    raise KeyError(name)


@pytest.mark.parametrize("first,second", [("blocky32", "poisson64"), ("blocky64", "q1_20")])
@pytest.mark.parametrize("preset", ["amp16", "amp64", "pcg64"])
def test_noalloc_equals_solve_on_calls_in_a_row(amp, first, second, preset):
    from paper_2505_04155_amd import binding as B
    for name in (first, second):
        A, b, kind, kw = _system(name)
        _say(f"noalloc {preset} {name} (n = {A.n})")
        M = amp.Matrix.from_csr(A)
        pc = amp.Preconditioner(M, kind, **kw)
        bt = torch.tensor(b, device="cuda")
        x_ref, info = amp.solve(M, pc, bt, preset=preset, maxit=5000)
        st, x, res = _noalloc(amp, M, pc, bt, preset)
        _say(f"  iters {res.iters} (amp_pcg_solve {info['iters']}), true rel. residual {res.rel_res_true:.3e}")
        assert st == B.AMP_OK and info["status"] == B.AMP_OK
        assert res.iters == info["iters"]
        assert (res.k_z32, res.k_z16, res.k_r32, res.n_replacements) == \
            (info["k_z32"], info["k_z16"], info["k_r32"], info["replacements"])
        assert res.rel_res_true == info["relres_true"]
        assert torch.equal(x, x_ref)


def test_noalloc_maxit_and_options(amp):
    from paper_2505_04155_amd import binding as B
    A, b, kind, kw = _system("poisson64")
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, kind, **kw)
    bt = torch.tensor(b, device="cuda")
    _say("noalloc: maxit")
    x_ref, info = amp.solve(M, pc, bt, preset="amp64", maxit=9)
    st, x, res = _noalloc(amp, M, pc, bt, "amp64", maxit=9)
    assert st == info["status"] == B.AMP_ERR_NOT_CONVERGED and res.iters == 9
    assert torch.equal(x, x_ref)
    _say("noalloc: rejected options")
    for opt in ({"graph": 1}, {"spmv_timing": 1}, {"solo_rows": 1 << 20}):
        st, _, _ = _noalloc(amp, M, pc, bt, "amp64", **opt)
        assert st == B.AMP_ERR_ARG, opt
        assert "must be 0" in B.last_error()


def test_noalloc_rejects_systems_above_the_limit(amp):
    from paper_2505_04155_amd import binding as B
    A, b, _ = P.poisson2d_system(513)   # 263169 rows -> 263168 + ... padded past 2^18
    _say(f"noalloc: above the limit (n = {A.n})")
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, "jacobi")
    bt = torch.tensor(b, device="cuda")
    st, x, res = _noalloc(amp, M, pc, bt, "amp64")
    assert st == B.AMP_ERR_ARG
    assert "exceed the limit" in B.last_error()
    assert torch.count_nonzero(x) == 0
