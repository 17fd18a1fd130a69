"""The lanes-per-row layout (several lanes share one long row): products are
exact on integer data for every layout, solves on a long-row system meet the
oracle's bar, the autotuner returns a valid choice, and the paths that need
one lane per row refuse such a handle."""

import math

import numpy as np
import pytest
import torch

from oracle import cpcg
from workloads import problems as P

pytestmark = pytest.mark.gpu

LANES = (1, 2, 4, 8, 16)
TOL = 1e-10


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


@pytest.fixture(scope="module")
def int_matrix():
    # 3037 rows: 47 slices of 64 rows (or 760 of 4) and a ragged tail;
    # rows of 53 to 257 entries
    return P.long_row_spd(3037, 200, seed=1, integer=True)


@pytest.mark.parametrize("lanes", LANES)
def test_integer_products_exact(amp, int_matrix, lanes):
    A = int_matrix
    _say(f"lanes {lanes}: integer products, n={A.n}, nnz={A.nnz}")
    p = np.random.default_rng([61, lanes]).integers(-8, 9, A.n).astype(np.float64)
    q_ref = A.to_scipy() @ p          # exact: integers far below 2^24
    M = amp.Matrix.from_csr(A, lanes=lanes)
    info = M.info()
    assert info["lanes_per_row"] == lanes
    if lanes > 1:
        assert info["offset_slices"] == 0
    for dtype in (torch.float64, torch.float32, torch.float16):
        pt = torch.tensor(p, device="cuda").to(dtype)
        for u_r, diff in ((64, True), (32, True), (32, False)):
            q, g = M.spmv(pt, u_r=u_r, diff=diff)
            torch.cuda.synchronize()
            qh = q.double().cpu().numpy()
            assert np.array_equal(qh, q_ref), (dtype, u_r, diff, int(np.argmax(np.abs(qh - q_ref))))
            assert float(g.item()) == float(q_ref @ p), (dtype, u_r, diff)


def test_auto_lanes_follows_row_length(amp, int_matrix):
    M = amp.Matrix.from_csr(int_matrix, lanes=0)
    # about 184 entries per row: 16 lanes leave about 12 per lane
    assert M.info()["lanes_per_row"] == 16
    short = P.stencil_poisson2d(40)
    assert amp.Matrix.from_csr(short, lanes=0).info()["lanes_per_row"] == 1


@pytest.fixture(scope="module")
def long_system():
    A, b = P.long_row_system(65536, 200)
    xo, io = cpcg.pcg(A, b, tol=TOL, maxit=5000)
    return A, b, xo, io


@pytest.mark.parametrize("lanes", [1, 4, 16])
@pytest.mark.parametrize("preset", ["pcg64", "amp64", "amp16"])
def test_long_row_solve_parity(amp, long_system, lanes, preset):
    A, b, xo, io = long_system
    M = amp.Matrix.from_csr(A, lanes=lanes)
    pc = amp.Preconditioner(M, "jacobi")
    bt = torch.tensor(b, device="cuda")
    x, info = amp.solve(M, pc, bt, tol=TOL, maxit=5000, preset=preset)
    xh = x.cpu().numpy()
    err = float(np.linalg.norm(xh - xo) / np.linalg.norm(xo))
    _say(f"long rows n={A.n} nnz={A.nnz}, lanes {lanes}, {preset}: {info['iters']} iterations "
         f"(oracle {io['iters']}), rel. error vs the oracle {err:.3e}, true rel. residual {info['relres_true']:.3e}")
    assert info["status"] == 0
    assert info["relres_true"] <= TOL
    assert info["iters"] <= math.ceil(1.05 * io["iters"])
    assert err <= 1e-8


def test_long_row_noalloc_matches(amp):
    import ctypes
    from paper_2505_04155_amd import binding as B
    n = 30000       # within the allocation-free entry point's row limit
    sub = P.long_row_spd(n, 200, seed=2)
    bb = np.random.default_rng([62]).standard_normal(n)
    M = amp.Matrix.from_csr(sub, lanes=8)
    pc = amp.Preconditioner(M, "jacobi")
    bt = torch.tensor(bb, device="cuda")
    x1, i1 = amp.solve(M, pc, bt, tol=TOL, maxit=5000, preset="amp64")
    L = B.load()
    x2 = torch.zeros_like(bt)
    res = B.Result()
    torch.cuda.synchronize()
    st = L.amp_pcg_solve_noalloc(M.handle, pc.handle, ctypes.c_void_p(bt.data_ptr()), ctypes.c_void_p(x2.data_ptr()),
                                 TOL, 5000, ctypes.byref(B.make_options("amp64")), ctypes.byref(res),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    _say(f"lanes 8 allocation-free solve: status {st}, {res.iters} iterations (solve: {i1['iters']})")
    assert st == 0
    assert res.iters == i1["iters"]
    assert torch.equal(x1, x2)


def test_tuner_returns_a_candidate(amp, int_matrix):
    best, us = amp.tune_lanes(int_matrix, candidates=(1, 4, 16), reps=10)
    _say(f"lanes tuner: {best} ({', '.join(f'{k}: {v:.1f} us' for k, v in us.items())})")
    assert best in (1, 4, 16)
    assert all(v > 0.0 for v in us.values())
    assert us[best] == min(us.values())


def test_one_lane_paths_refuse_lanes(amp, int_matrix):
    from paper_2505_04155_amd import binding as B
    M = amp.Matrix.from_csr(int_matrix, lanes=4)
    with pytest.raises(B.AmpError, match="one lane per row"):
        amp.Preconditioner(M, "chebyshev", degree=2, lam_lo=0.1, lam_hi=2.0)
    M1 = amp.Matrix.from_csr(int_matrix, lanes=1)
    pcs = [amp.Preconditioner(m, "jacobi") for m in (M1, M)]
    b = torch.ones(int_matrix.n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.AmpError, match="lanes per row"):
        amp.solve_batched([M1, M], pcs, [b, b.clone()], tol=TOL, maxit=100, preset="amp64")


def test_offset_mode_handle_holds_no_column_plane(amp):
    # every slice of a stencil matrix is in offset mode: the handle keeps no
    # per-slot column index (FP64 + FP32 values only)
    A, b, _, (lo, hi) = P.q1_system(20)
    M = amp.Matrix.from_csr(A)
    i = M.info()
    # (slices of padding rows past n hold no slots, whatever their mode)
    assert i["offset_slices"] == -(-A.n // 64)
    ns, slots = i["nslices"], i["slots"]
    np_ = -(-A.n // 1024) * 1024
    assert i["bytes"] == i["meta_bytes"] + 16 * ns + 12 * slots + 8 * np_
    # and it still solves, with the Chebyshev preconditioner too
    pc = amp.Preconditioner(M, "chebyshev", degree=4, lam_lo=lo, lam_hi=hi)
    x, info = amp.solve(M, pc, torch.tensor(b, device="cuda"), tol=1e-10, maxit=2000, preset="amp16")
    assert info["status"] == 0 and info["relres_true"] <= 1e-10
    # an index-mode handle of the same matrix holds the columns (counted in
    # its metadata bytes, 4 per slot)
    Mi = amp.Matrix.from_csr(A, offsets=False)
    ii = Mi.info()
    assert ii["offset_slices"] == 0
    assert ii["meta_bytes"] >= 4 * ii["slots"]
    assert ii["bytes"] == ii["meta_bytes"] + 16 * ii["nslices"] + 12 * ii["slots"] + 8 * np_
