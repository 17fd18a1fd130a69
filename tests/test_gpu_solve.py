"""Solve-level parity of the HIP path (GPU) against the oracle.

* PCG(FP64) on the GPU reproduces the C oracle's Alg. 1 iteration count and
  solution; power-of-two dynamic scaling leaves it bitwise unchanged
  (Thm. dspcg in finite precision).
* AMP-PCG on the GPU follows the precision model of Alg. 3: iteration
  counts and switch points agree, the GPU's own residual history replayed
  through the oracle's selector reproduces its switch points exactly, and
  the FP64 true residual reaches the tolerance.
* Edge cases: zero right-hand side, exact initial guess, maxit, a
  non-positive-definite matrix, ragged sizes, determinism.
"""

import math

import numpy as np
import pytest
import torch

from oracle import amp_model as am
from oracle import cpcg
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


def _gpu_solve(amp, A, b, preset, tol=1e-10, maxit=5000, x0=None, kind="jacobi", **kw):
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, kind)
    bt = torch.tensor(b, device="cuda")
    x0t = None if x0 is None else torch.tensor(x0, device="cuda")
    x, info = amp.solve(M, pc, bt, x0=x0t, tol=tol, maxit=maxit, preset=preset, history=True, **kw)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ------------------------------------------------------------------ PCG(FP64)

@pytest.mark.parametrize("case", ["poisson64", "poisson37", "blocky24"])
def test_pcg64_matches_c_oracle(amp, case):
    _say(f"pcg64 vs oracle {case}")
    if case.startswith("poisson"):
        A, b, _ = P.poisson2d_system(int(case[7:]))
    else:
        A, b, _ = P.blocky_diffusion3d_system(24, 4)
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=5000, history=True)
    x, info = _gpu_solve(amp, A, b, "pcg64")
    assert info["status"] == 0
    assert info["iters"] == io["iters"]
    assert _rel(x, xo) <= 1e-11
    assert np.allclose(info["delta"], io["delta"], rtol=1e-8, atol=0)
    assert info["relres_true"] <= 1e-10
    assert info["k_z32"] == -1 and info["k_r32"] == -1


@pytest.mark.parametrize("u", [64, 32])
def test_pow2_scaling_bitwise_neutral_on_gpu(amp, u):
    _say(f"pow2 vs none u={u}")
    A, b, _ = P.blocky_diffusion3d_system(16, 4, decades=2.0)
    eta = "fixed64" if u == 64 else "fixed32"
    x1, i1 = _gpu_solve(amp, A, b, "pcg64", tol=1e-6, u0=u, eta=eta, verify=0)
    x2, i2 = _gpu_solve(amp, A, b, "pcg64", tol=1e-6, u0=u, eta=eta, verify=0, scaling="none")
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(x1, x2)
    assert np.array_equal(i1["delta"], i2["delta"])


def test_paper_scaling_matches_oracle(amp):
    _say("paper scaling")
    A, b, _ = P.poisson2d_system(48)
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=5000)
    x, info = _gpu_solve(amp, A, b, "pcg64", scaling="paper")
    assert info["iters"] == io["iters"]
    assert _rel(x, xo) <= 1e-11


# ------------------------------------------------------------------ AMP-PCG vs the model

CASES = {
    "poisson64": lambda: P.poisson2d_system(64)[:2],
    "poisson37": lambda: P.poisson2d_system(37)[:2],
    "blocky24": lambda: P.blocky_diffusion3d_system(24, 4)[:2],
    "blocky32": lambda: P.blocky_diffusion3d_system(32, 8)[:2],
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("preset,kw", [("amp64", {}), ("amp16", {}), ("amp_ur", {}),
                                       ("amp64", {"eta": "linear"}), ("amp64", {"spmv32": "plain"})])
def test_amp_matches_model(amp, case, preset, kw):
    _say(f"amp vs model {case} {preset} {kw}")
    A, b = CASES[case]()
    S = A.to_scipy()
    ref = am.amp_pcg(S, b, tol=1e-10, maxit=5000, opt=am.options(preset, **kw))
    x, info = _gpu_solve(amp, A, b, preset, **kw)
    assert info["status"] == 0 and ref.status == 0
    gd, md = np.asarray(info["delta"]), np.asarray(ref.delta)
    m = min(len(gd), len(md))
    rel = np.abs(gd[:m] - md[:m]) / md[:m]
    bad = np.nonzero(rel > 1e-3)[0]
    _say(f"  gpu iters {info['iters']} model {ref.iters}; first |delta| divergence > 1e-3 at "
         f"{bad[0] if bad.size else None}; early rel diffs {np.array2string(rel[:12], precision=1)}")
    k = min(12, len(ref.omega), len(info["omega"]))
    _say(f"  omega gpu {np.log2(info['omega'][:k]).astype(int).tolist()} model "
         f"{np.log2(np.asarray(ref.omega[:k])).astype(int).tolist()}")
    for name in ("rho", "gamma", "alpha"):
        g_, m_ = np.asarray(info[name][:k]), np.asarray(getattr(ref, name)[:k])
        _say(f"  {name} rel diff {np.array2string(np.abs(g_ - m_) / np.abs(m_), precision=1)}")
    # the GPU's own history through the oracle's selector reproduces its switch points
    kz32, kz16, kr = am.replay_switches(list(info["delta"][:info["iters"]]), info["bnorm"], 1e-10,
                                        am.options(preset, **kw))
    assert (kz32, kz16, kr) == (info["k_z32"], info["k_z16"], info["k_r32"])
    # and they agree with the model's to within an iteration or two
    for key, val in (("k_z32", ref.k_z32), ("k_z16", ref.k_z16), ("k_r32", ref.k_r32)):
        assert (info[key] < 0) == (val < 0), key
        assert abs(info[key] - val) <= 2, key
    assert abs(info["iters"] - ref.iters) <= max(2, math.ceil(0.02 * ref.iters))
    assert info["relres_true"] <= 1e-10
    assert _rel(x, ref.x) <= 1e-7
    # per-iteration precisions recorded by the device are latched
    assert all(a >= b for a, b in zip(info["uz"], info["uz"][1:]))
    assert all(a >= b for a, b in zip(info["ur"], info["ur"][1:]))


@pytest.mark.parametrize("case", ["poisson64", "blocky32"])
def test_amp64_vs_fp64_oracle(amp, case):
    _say(f"amp64 vs fp64 oracle {case}")
    A, b = CASES[case]()
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=5000)
    x, info = _gpu_solve(amp, A, b, "amp64")
    assert info["status"] == 0
    assert info["iters"] <= math.ceil(1.05 * io["iters"])
    assert info["relres_true"] <= 1e-10
    # the parity bar: within 1e-8 of the oracle's solution
    assert _rel(x, xo) <= 1e-8


@pytest.mark.parametrize("d", [63, 64, 80, 100])
def test_long_delay_window_switches_like_the_replay(amp, d):
    # delay windows of at least a wave's width take the controller's serial
    # evaluation of eq. (eta_k); the switch must still happen where the
    # selector replayed over the GPU's own history puts it, and near the model's
    _say(f"long delay window d={d}")
    A, b = CASES["blocky32"]()
    x, info = _gpu_solve(amp, A, b, "amp64", d=d)
    ref = am.amp_pcg(A.to_scipy(), b, tol=1e-10, maxit=5000, opt=am.options("amp64", d=d))
    _say(f"  gpu k_r32 {info['k_r32']} iters {info['iters']}; model k_r32 {ref.k_r32} iters {ref.iters}")
    assert info["status"] == 0
    # d <= 80 switches on this system; with d = 100 the window's sum keeps eta
    # above tol ||b|| to the end, for the model as for the GPU
    assert (info["k_r32"] > d) if d <= 80 else (info["k_r32"] == ref.k_r32 == -1)
    kz32, kz16, kr = am.replay_switches(list(info["delta"][:info["iters"]]), info["bnorm"], 1e-10,
                                        am.options("amp64", d=d))
    assert (kz32, kz16, kr) == (info["k_z32"], info["k_z16"], info["k_r32"])
    assert abs(info["k_r32"] - ref.k_r32) <= 2
    assert info["relres_true"] <= 1e-10


@pytest.mark.parametrize("case", ["poisson64", "blocky32"])
@pytest.mark.parametrize("rr_switch", [0, 1])
def test_switch_replacement_matches_model(amp, case, rr_switch):
    # at the u_r switch r is replaced by fl32(b - A x) (rr_switch = 1, the
    # default) or rounded from the recurrence (0); either way the GPU follows
    # the model with the same option, and the replacement is counted once
    _say(f"switch replacement {case} rr_switch={rr_switch}")
    A, b = CASES[case]()
    ref = am.amp_pcg(A.to_scipy(), b, tol=1e-10, maxit=5000, opt=am.options("amp16", rr_switch=bool(rr_switch)))
    x, info = _gpu_solve(amp, A, b, "amp16", rr_switch=rr_switch)
    _say(f"  gpu iters {info['iters']} repl {info['replacements']}; model iters {ref.iters} repl {ref.replacements}")
    assert info["status"] == 0 and ref.status == 0 and info["k_r32"] >= 0
    assert abs(info["k_r32"] - ref.k_r32) <= 2
    assert abs(info["iters"] - ref.iters) <= max(2, math.ceil(0.02 * ref.iters))
    assert info["replacements"] == ref.replacements
    assert info["replacements"] >= rr_switch
    assert info["relres_true"] <= 1e-10
    assert _rel(x, ref.x) <= 1e-7


def test_switch_replacement_is_the_true_residual(amp):
    # with u_r fixed to FP32 from the first iteration the switch happens at
    # k = 0, where fl32(b - A x0) is exactly the FP64 r0 rounded: both options
    # give bitwise the same solve
    _say("switch replacement at k = 0")
    A, b = CASES["blocky24"]()
    x1, i1 = _gpu_solve(amp, A, b, "amp16", eta="fixed32", rr_switch=1)
    x0, i0 = _gpu_solve(amp, A, b, "amp16", eta="fixed32", rr_switch=0)
    assert i1["k_r32"] == 0 and i0["k_r32"] == 0
    assert i1["iters"] == i0["iters"] and np.array_equal(x1, x0)
    assert i1["replacements"] == i0["replacements"] + 1


# ------------------------------------------------------------------ edge cases

def test_zero_rhs_and_exact_start(amp):
    _say("edge: zero rhs, exact start")
    A, b, xs = P.poisson2d_system(20)
    x, info = _gpu_solve(amp, A, np.zeros(A.n), "amp64")
    assert info["status"] == 0 and info["iters"] == 0 and np.all(x == 0)
    x, info = _gpu_solve(amp, A, b, "amp64", x0=xs)
    assert info["status"] == 0 and info["iters"] == 0


def test_maxit_returns_last_iterate(amp):
    _say("edge: maxit")
    from paper_2505_04155_amd import binding as B
    A, b, _ = P.poisson2d_system(32)
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=7)
    x, info = _gpu_solve(amp, A, b, "pcg64", maxit=7)
    assert info["status"] == B.AMP_ERR_NOT_CONVERGED and info["iters"] == 7
    assert _rel(x, xo) <= 1e-12


def test_breakdown_on_indefinite_matrix(amp):
    _say("edge: breakdown")
    from paper_2505_04155_amd import binding as B
    # positive diagonal but indefinite: gamma <= 0 at the first step
    D = np.array([[1.0, 3.0, 0.0], [3.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    A = P.dense_to_csr(D)
    x, info = _gpu_solve(amp, A, np.array([1.0, -1.0, 0.0]), "pcg64", kind="identity")
    assert info["status"] == B.AMP_ERR_BREAKDOWN
    assert np.all(np.isfinite(x))


@pytest.mark.parametrize("n", [1, 2, 63, 65, 1023, 1025])
def test_ragged_sizes(amp, n):
    _say(f"edge: ragged n={n}")
    A = P.stencil_poisson2d(1) if n == 1 else P.fv_diffusion(
        np.exp(np.random.default_rng([310, n]).standard_normal((1, n))))
    b = np.random.default_rng([311, n]).standard_normal(A.n)
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=5000)
    # both solutions satisfy ||x - x*|| <= kappa(A) tol ||x*||: FP16 z, p are
    # held to 2 tol kappa(A) (kappa from the dense spectrum), the others to 1e-8
    ev = np.linalg.eigvalsh(A.to_scipy().toarray())
    kappa = float(ev[-1] / ev[0])
    for preset in ("pcg64", "amp64", "amp16"):
        x, info = _gpu_solve(amp, A, b, preset)
        bound = 2e-10 * kappa if preset == "amp16" else 1e-8
        _say(f"  {preset}: rel. error vs the oracle {_rel(x, xo):.3e} (bound {bound:.2e}, kappa {kappa:.3e})")
        assert info["status"] == 0, preset
        assert info["relres_true"] <= 1e-10, preset
        assert _rel(x, xo) <= bound, preset


def test_deterministic(amp):
    _say("determinism")
    A, b, _ = P.blocky_diffusion3d_system(16, 4)
    x1, i1 = _gpu_solve(amp, A, b, "amp16")
    x2, i2 = _gpu_solve(amp, A, b, "amp16")
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(x1, x2)


def test_periodic_replacement_matches_model(amp):
    _say("periodic replacement")
    A, b = CASES["blocky24"]()
    ref = am.amp_pcg(A.to_scipy(), b, tol=1e-10, maxit=5000, opt=am.options("amp16", rr_period=25))
    x, info = _gpu_solve(amp, A, b, "amp16", rr_period=25)
    assert info["status"] == 0
    assert info["replacements"] >= info["iters"] // 25
    assert abs(info["iters"] - ref.iters) <= max(2, math.ceil(0.02 * ref.iters))
    assert info["relres_true"] <= 1e-10


# ------------------------------------------------------------------ single-work-group solve

@pytest.mark.parametrize("case,preset", [("poisson64", "amp64"), ("poisson64", "amp16"), ("poisson37", "pcg64"),
                                         ("blocky24", "amp_ur"), ("blocky24", "amp16")])
def test_single_workgroup_solve_matches_kernel_sequence(amp, case, preset):
    # one launch looping on the device runs the stages of the host-enqueued
    # kernels (one work-group each) in the same order; only the work-group
    # size of the product stage differs (its partial sums round differently)
    _say(f"solo vs kernel sequence {case} {preset}")
    A, b = CASES[case]()
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, "jacobi")
    bt = torch.tensor(b, device="cuda")
    x1, i1 = amp.solve(M, pc, bt, preset=preset, solo_rows=1 << 20, history=True)
    x2, i2 = amp.solve(M, pc, bt, preset=preset, solo_rows=0, group_rows=1 << 30, history=True)
    torch.cuda.synchronize()
    _say(f"  iters {i1['iters']} / {i2['iters']}, t {i1['t_solve_ms']:.2f} / {i2['t_solve_ms']:.2f} ms")
    assert i1["status"] == i2["status"] == 0
    assert abs(i1["iters"] - i2["iters"]) <= max(2, math.ceil(0.02 * i2["iters"]))
    for key in ("k_z32", "k_z16", "k_r32"):
        assert abs(i1[key] - i2[key]) <= 2, key
    m = min(i1["iters"], i2["iters"], 20)
    assert np.allclose(i1["delta"][:m], i2["delta"][:m], rtol=1e-6, atol=0)
    assert i1["relres_true"] <= 1e-10 and i2["relres_true"] <= 1e-10
    assert _rel(x1.cpu().numpy(), x2.cpu().numpy()) <= 1e-6


def test_single_workgroup_solve_maxit_and_breakdown(amp):
    _say("solo: maxit and breakdown")
    from paper_2505_04155_amd import binding as B
    A, b = CASES["poisson37"]()
    x, info = _gpu_solve(amp, A, b, "amp64", maxit=7, solo_rows=1 << 20)
    assert info["status"] == B.AMP_ERR_NOT_CONVERGED and info["iters"] == 7
    x2, info2 = _gpu_solve(amp, A, b, "amp64", maxit=7, solo_rows=0, group_rows=1 << 30)
    assert info2["status"] == B.AMP_ERR_NOT_CONVERGED and info2["iters"] == 7
    assert _rel(x, x2) <= 1e-12
    D = np.array([[1.0, 3.0, 0.0], [3.0, 1.0, 0.0], [0.0, 0.0, 1.0]])   # indefinite
    x, info = _gpu_solve(amp, P.dense_to_csr(D), np.array([1.0, -1.0, 0.0]), "pcg64", kind="identity",
                         solo_rows=1 << 20)
    assert info["status"] == B.AMP_ERR_BREAKDOWN
    assert np.all(np.isfinite(x))


def test_product_kernel_timing(amp):
    _say("product-kernel timing")
    A, b = CASES["blocky24"]()
    x0, i0 = _gpu_solve(amp, A, b, "amp64")
    x1, i1 = _gpu_solve(amp, A, b, "amp64", spmv_timing=1)
    # the timed solve is the same solve; one timed launch per iteration
    assert i1["iters"] == i0["iters"] and np.array_equal(x0, x1)
    assert i1["spmv_launches"] == i1["iters"]
    assert 0.0 < i1["spmv_ms"] < i1["t_solve_ms"]
    assert i0["spmv_launches"] == 0 and i0["spmv_ms"] == 0.0


# ------------------------------------------------------------------ captured graphs

@pytest.mark.parametrize("case,preset", [("poisson64", "amp16"), ("blocky24", "amp64"), ("poisson37", "pcg64")])
def test_graph_replay_matches_eager(amp, case, preset):
    # replays of the captured batch equal the eager launches bit for bit, with
    # eager solves between replays, and a changed tolerance re-captures
    _say(f"graph vs eager {case} {preset}")
    A, b = CASES[case]()
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, "jacobi")
    bt = torch.tensor(b, device="cuda")
    for tol in (1e-10, 1e-6, 1e-10):
        x0, i0 = amp.solve(M, pc, bt, tol=tol, preset=preset, solo_rows=0)
        for rep in range(3):
            xg, ig = amp.solve(M, pc, bt, tol=tol, preset=preset, graph=1, solo_rows=0)
            torch.cuda.synchronize()
            _say(f"  tol {tol} replay {rep}: iters {ig['iters']} (eager {i0['iters']})")
            assert ig["status"] == i0["status"] == 0
            assert ig["iters"] == i0["iters"]
            for key in ("k_z32", "k_z16", "k_r32", "replacements"):
                assert ig[key] == i0[key], key
            assert torch.equal(xg, x0)
            xe, ie = amp.solve(M, pc, bt, tol=tol, preset=preset, solo_rows=0)
            torch.cuda.synchronize()
            assert torch.equal(xe, x0)


def test_graph_replay_chebyshev(amp):
    _say("graph vs eager, chebyshev")
    A, b, _, (lo, hi) = P.q1_system(20)
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, "chebyshev", degree=4, lam_lo=lo, lam_hi=hi)
    bt = torch.tensor(b, device="cuda")
    x0, i0 = amp.solve(M, pc, bt, preset="amp16")
    for rep in range(2):
        xg, ig = amp.solve(M, pc, bt, preset="amp16", graph=1)
        torch.cuda.synchronize()
        assert ig["iters"] == i0["iters"] and torch.equal(xg, x0)


# ------------------------------------------------------------------ failure injection

@pytest.mark.parametrize("preset", ["pcg64", "amp16"])
def test_nan_in_rhs_is_a_breakdown(amp, preset):
    # a NaN in b makes rho non-finite in the first product: the solve stops
    # with a breakdown and returns the last finite iterate (here x0)
    _say(f"failure injection: NaN in b, {preset}")
    from paper_2505_04155_amd import binding as B
    A, b, _ = P.poisson2d_system(20)
    b = b.copy()
    b[57] = np.nan
    x0 = np.random.default_rng([320]).standard_normal(A.n)
    x, info = _gpu_solve(amp, A, b, preset, maxit=50, x0=x0)
    assert info["status"] == B.AMP_ERR_BREAKDOWN
    assert np.array_equal(x, x0)


def test_nan_system_in_a_batch(amp):
    # one system of a batch breaks down; the others converge as on their own
    # (same rows per work-group as the batched default, 4096)
    _say("failure injection: NaN in one system of a batch")
    from paper_2505_04155_amd import binding as B
    systems = [P.poisson2d_system(m)[:2] for m in (16, 24, 32)]
    bad = systems[1][1].copy()
    bad[3] = np.nan
    systems[1] = (systems[1][0], bad)
    Ms = [amp.Matrix.from_csr(A) for A, _ in systems]
    Ps = [amp.Preconditioner(M, "jacobi") for M in Ms]
    bs = [torch.tensor(b, device="cuda") for _, b in systems]
    xs, infos, st = amp.solve_batched(Ms, Ps, bs, tol=1e-10, maxit=500, preset="amp64")
    torch.cuda.synchronize()
    assert st == B.AMP_ERR_BREAKDOWN
    assert infos[1]["status"] == B.AMP_ERR_BREAKDOWN
    for i in (0, 2):
        x1, i1 = amp.solve(Ms[i], Ps[i], bs[i], tol=1e-10, maxit=500, preset="amp64", group_rows=4096)
        torch.cuda.synchronize()
        assert infos[i]["status"] == 0 and infos[i]["iters"] == i1["iters"]
        assert torch.equal(xs[i], x1)


def test_textbook_plane_built_on_first_use(amp):
    # the textbook FP32 plane (spmv32 = plain) is built from the FP64 plane by
    # the first solve that uses it; default-form and FP64 solves never hold it
    _say("textbook FP32 plane on first use")
    A, b = CASES["blocky24"]()
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, "jacobi")
    bt = torch.tensor(b, device="cuda")
    amp.solve(M, pc, bt, preset="amp64")
    amp.solve(M, pc, bt, preset="pcg64", spmv32="plain")
    held = M.info()["bytes"]
    x1, i1 = amp.solve(M, pc, bt, preset="amp64", spmv32="plain")
    assert M.info()["bytes"] == held + 4 * M.info()["slots"]
    x2, i2 = amp.solve(M, pc, bt, preset="amp64", spmv32="plain")
    torch.cuda.synchronize()
    assert M.info()["bytes"] == held + 4 * M.info()["slots"]
    assert i1["iters"] == i2["iters"] and torch.equal(x1, x2) and i1["status"] == 0
