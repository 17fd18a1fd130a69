"""The deferred FP64 x update (option defer_x, on by default) against the
update applied every iteration (defer_x = 0).

x_{k+1} = x_k + alpha_k p_k is applied two iterations at a time; each step is
rounded as on its own, so the iterate must be bitwise the same whenever the
solve stops: on convergence, at maxit on an odd and an even count, on a
breakdown with a step pending, across u_z switches (the pending p in the old
precision), through the termination check's residual replacement, in the
single-work-group solve, in graph replays and in the batched solve.  The
residual recurrence does not involve x, so the histories must be identical
too.
"""
import numpy as np
import pytest
import torch

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


def _pair(amp, A, b, preset, kind="jacobi", pc_kw=None, **kw):
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, kind, **(pc_kw or {}))
    bt = torch.tensor(b, device="cuda")
    out = []
    for defer in (0, 1):
        x, info = amp.solve(M, pc, bt, preset=preset, history=True, defer_x=defer, **kw)
        torch.cuda.synchronize()
        out.append((x.cpu().numpy(), info))
    return out


def _same(a, b, what):
    (x0, i0), (x1, i1) = a, b
    _say(f"  {what}: status {i0['status']}/{i1['status']} iters {i0['iters']}/{i1['iters']} "
         f"switches z32 {i1['k_z32']} z16 {i1['k_z16']} r32 {i1['k_r32']} repl {i1['replacements']}")
    assert i0["status"] == i1["status"]
    assert i0["iters"] == i1["iters"]
    for key in ("k_z32", "k_z16", "k_r32", "replacements"):
        assert i0[key] == i1[key], key
    assert np.array_equal(i0["delta"], i1["delta"])
    assert np.array_equal(x0, x1)
    assert i0["relres_true"] == i1["relres_true"]


CASES = {
    "poisson64": lambda: P.poisson2d_system(64)[:2],
    "poisson37": lambda: P.poisson2d_system(37)[:2],
    "blocky24": lambda: P.blocky_diffusion3d_system(24, 4)[:2],
    "blocky32": lambda: P.blocky_diffusion3d_system(32, 8)[:2],
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("preset", ["pcg64", "amp64", "amp16", "amp_ur"])
def test_converged_solve_bitwise(amp, case, preset):
    _say(f"deferred x: {case} {preset}")
    A, b = CASES[case]()
    a, c = _pair(amp, A, b, preset, solo_rows=0)
    assert c[1]["status"] == 0
    _same(a, c, "converged")


@pytest.mark.parametrize("maxit", [1, 2, 7, 8])
@pytest.mark.parametrize("solo", [0, 1 << 20])
def test_maxit_odd_and_even(amp, maxit, solo):
    _say(f"deferred x: maxit {maxit} solo {solo}")
    from paper_2505_04155_amd import binding as B
    A, b = CASES["poisson37"]()
    a, c = _pair(amp, A, b, "amp64", maxit=maxit, solo_rows=solo)
    assert c[1]["status"] == B.AMP_ERR_NOT_CONVERGED and c[1]["iters"] == maxit
    _same(a, c, "maxit")
    if solo == 0:
        xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=maxit)
        assert np.linalg.norm(c[0] - xo) <= 1e-12 * np.linalg.norm(xo)


@pytest.mark.parametrize("w", [0.05, 0.15, 0.55])
def test_breakdown_with_and_without_a_step_pending(amp, w):
    # identity preconditioner on an indefinite matrix with a positive
    # diagonal (a 2x2 block with eigenvalues 4 and -2, then 1..6): gamma > 0
    # for some steps, then <= 0 (at iteration 3, 2, 1 for these right-hand
    # sides, so a step is pending at 3 and 1); the returned x is the last iterate
    _say(f"deferred x: breakdown, w {w}")
    from paper_2505_04155_amd import binding as B
    D = np.diag([1.0, 1.0, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    D[0, 1] = D[1, 0] = 3.0
    A = P.dense_to_csr(D)
    b = np.ones(8)
    b[0], b[1] = w, -w
    for solo in (0, 1 << 20):
        a, c = _pair(amp, A, b, "pcg64", kind="identity", solo_rows=solo)
        assert c[1]["status"] == B.AMP_ERR_BREAKDOWN
        _same(a, c, f"breakdown solo {solo}")
        assert np.all(np.isfinite(c[0]))


def test_u_z_switch_parities(amp):
    # the stepwise preset switches u_z twice; over these systems the switch
    # iterations fall on both parities, i.e. with and without a step pending
    _say("deferred x: u_z switch parities")
    seen = set()
    systems = [(f"poisson{m}", P.poisson2d_system(m)[:2]) for m in (30, 37, 41, 50, 53, 64)]
    systems += [("blocky24", CASES["blocky24"]()), ("blocky32", CASES["blocky32"]())]
    for name, (A, b) in systems:
        a, c = _pair(amp, A, b, "amp64", solo_rows=0)
        _same(a, c, name)
        for key in ("k_z32", "k_z16"):
            if c[1][key] > 0:
                seen.add(c[1][key] % 2)
    assert seen == {0, 1}, seen


def test_graph_and_chebyshev(amp):
    _say("deferred x: graph replay and chebyshev")
    A, b = CASES["blocky24"]()
    a, c = _pair(amp, A, b, "amp16", graph=1, solo_rows=0)
    _same(a, c, "graph")
    A, b, _, (lo, hi) = P.q1_system(20)
    a, c = _pair(amp, A, b, "amp16", kind="chebyshev", pc_kw=dict(degree=4, lam_lo=lo, lam_hi=hi))
    _same(a, c, "chebyshev")


def test_batched_bitwise(amp):
    _say("deferred x: batched")
    systems = [P.poisson2d_system(m)[:2] for m in (20, 37, 64)]
    systems += P.batched_systems(count=4, side_min=16, side_max=96)
    Ms = [amp.Matrix.from_csr(A) for A, _ in systems]
    Ps = [amp.Preconditioner(M, "jacobi") for M in Ms]
    bs = [torch.tensor(b, device="cuda") for _, b in systems]
    res = []
    for defer in (0, 1):
        xs, infos, st = amp.solve_batched(Ms, Ps, bs, tol=1e-10, maxit=5000, preset="amp16", solo_rows=0,
                                          defer_x=defer)
        torch.cuda.synchronize()
        assert st == 0
        res.append(([x.cpu().numpy() for x in xs], infos))
    for i in range(len(systems)):
        assert res[0][1][i]["iters"] == res[1][1][i]["iters"]
        assert np.array_equal(res[0][0][i], res[1][0][i]), i
