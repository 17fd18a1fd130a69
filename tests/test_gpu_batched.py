"""Batched AMP-PCG on the GPU: many independent systems in one lockstep solve.

* Each system of a batch follows exactly the arithmetic of a single-system
  solve run with the same work-group count: identical solution bits,
  iteration count and switch points, whatever else is in the batch and
  whenever the other systems stop.
* Against the FP64 oracle: iteration counts, true residuals, solutions.
* The 512-system workload (2-D five-point finite-volume systems with
  log-uniform sides in [32, 512] and log-normal coefficients) at full size:
  every system reaches the tolerance in the FP64 true residual; sampled
  systems match the oracle's iteration counts.
"""

import math

import numpy as np
import pytest
import torch

from oracle import cpcg
from workloads import problems as P

pytestmark = pytest.mark.gpu

GROUP_ROWS = 4096   # the batched solve's default rows per work-group


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


def _handles(amp, systems):
    Ms = [amp.Matrix.from_csr(A) for A, _ in systems]
    Ps = [amp.Preconditioner(M, "jacobi") for M in Ms]
    bs = [torch.tensor(b, device="cuda") for _, b in systems]
    return Ms, Ps, bs


def _mixed_systems():
    # small systems (one work-group each by default) and larger ones (lockstep)
    out = [P.poisson2d_system(m)[:2] for m in (20, 37, 64, 150)]
    out += P.batched_systems(count=5, side_min=16, side_max=160)
    A, _, _ = P.poisson2d_system(24)
    out.append((A, np.zeros(A.n)))                    # zero right-hand side: 0 iterations
    out.append(P.blocky_diffusion3d_system(32, 8)[:2])
    return out


@pytest.mark.parametrize("preset,solo_rows", [("amp64", 16384), ("amp16", 16384), ("pcg64", 16384),
                                              ("amp64", 0), ("amp16", 0)])
def test_batched_matches_single_bitwise(amp, preset, solo_rows):
    _say(f"batched vs single, {preset}, solo_rows {solo_rows}")
    systems = _mixed_systems()
    Ms, Ps, bs = _handles(amp, systems)
    # exact start for one system: x0 = x*, so r0 = 0 exactly
    A3, b3, xs3 = P.poisson2d_system(30)
    M3 = amp.Matrix.from_csr(A3)
    Ms.append(M3)
    Ps.append(amp.Preconditioner(M3, "jacobi"))
    bs.append(torch.tensor(b3, device="cuda"))
    x0s = [None] * (len(Ms) - 1) + [torch.tensor(xs3, device="cuda")]
    xs, infos, st = amp.solve_batched(Ms, Ps, bs, x0s=x0s, tol=1e-10, maxit=5000, preset=preset,
                                      solo_rows=solo_rows)
    torch.cuda.synchronize()
    assert st == 0, [i["status"] for i in infos]
    zero_rhs = len(_mixed_systems()) - 2
    assert infos[-1]["iters"] == 0 and infos[zero_rhs]["iters"] == 0
    for i in range(len(Ms)):
        x1, i1 = amp.solve(Ms[i], Ps[i], bs[i], x0=x0s[i], tol=1e-10, maxit=5000, preset=preset,
                           group_rows=GROUP_ROWS, solo_rows=solo_rows)
        torch.cuda.synchronize()
        _say(f"  system {i}: n={Ms[i].n} batched iters {infos[i]['iters']} single {i1['iters']}")
        assert infos[i]["iters"] == i1["iters"]
        for key in ("k_z32", "k_z16", "k_r32", "replacements"):
            assert infos[i][key] == i1[key], key
        assert torch.equal(xs[i], x1)
        assert infos[i]["relres_true"] == pytest.approx(i1["relres_true"], rel=1e-12, abs=1e-300)
        assert infos[i]["relres_true"] <= 1e-10


def test_batched_vs_oracle(amp):
    _say("batched amp64 vs FP64 oracle, 24 systems")
    systems = P.batched_systems(count=24, side_min=16, side_max=128)
    Ms, Ps, bs = _handles(amp, systems)
    xs, infos, st = amp.solve_batched(Ms, Ps, bs, tol=1e-10, maxit=20000, preset="amp64")
    torch.cuda.synchronize()
    assert st == 0
    for i, (A, b) in enumerate(systems):
        xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=20000)
        assert io["status"] == 0
        info = infos[i]
        assert info["relres_true"] <= 1e-10
        assert info["iters"] <= math.ceil(1.05 * io["iters"]) + 1, (i, info["iters"], io["iters"])
        x = xs[i].cpu().numpy()
        assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)


def test_batched_full_workload(amp):
    _say("batched 512-system workload, generating")
    systems = P.batched_systems()
    sizes = np.array([A.n for A, _ in systems])
    _say(f"  {len(systems)} systems, {sizes.sum()} rows, sides {int(math.sqrt(sizes.min()))}.."
         f"{int(math.sqrt(sizes.max()))}")
    Ms, Ps, bs = _handles(amp, systems)
    xs, infos, st = amp.solve_batched(Ms, Ps, bs, tol=1e-10, maxit=20000, preset="amp64")
    torch.cuda.synchronize()
    iters = np.array([i["iters"] for i in infos])
    _say(f"  status {st}, iterations min {iters.min()} median {int(np.median(iters))} max {iters.max()}, "
         f"{infos[0]['t_solve_ms']:.1f} ms")
    xs2, infos2, st2 = amp.solve_batched(Ms, Ps, bs, tol=1e-10, maxit=20000, preset="amp64", solo_rows=0)
    _say(f"  all lockstep: status {st2}, {infos2[0]['t_solve_ms']:.1f} ms")
    assert st2 == 0 and max(i["relres_true"] for i in infos2) <= 1e-10
    assert st == 0
    assert max(i["relres_true"] for i in infos) <= 1e-10
    # sampled systems against the oracle: smallest, median, largest
    order = np.argsort(sizes)
    for i in (order[0], order[len(order) // 2], order[-1]):
        A, b = systems[i]
        xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=20000)
        _say(f"  system {i}: n={A.n} gpu {infos[i]['iters']} oracle {io['iters']}")
        assert infos[i]["iters"] <= math.ceil(1.05 * io["iters"]) + 1
        x = xs[i].cpu().numpy()
        assert np.linalg.norm(x - xo) <= 1e-8 * np.linalg.norm(xo)


def test_batched_rejects_bad_arguments(amp):
    from paper_2505_04155_amd import binding as B
    _say("batched argument checks")
    systems = [P.poisson2d_system(m)[:2] for m in (12, 14)]
    Ms, Ps, bs = _handles(amp, systems)
    with pytest.raises(B.AmpError) as e:
        amp.solve_batched([Ms[0], Ms[0]], [Ps[0], Ps[0]], [bs[0], bs[0]])
    assert e.value.status == B.AMP_ERR_ARG
    with pytest.raises(B.AmpError):
        amp.solve_batched(Ms, [Ps[1], Ps[0]], bs)               # preconditioner of another matrix
    with pytest.raises(B.AmpError):
        amp.solve_batched(Ms, Ps, bs, rr_period=10)
    with pytest.raises(B.AmpError):
        amp.solve_batched(Ms, Ps, bs, tol=[1e-10, 0.0])
    with pytest.raises(B.AmpError):
        amp.solve_batched(Ms, Ps, bs, group_rows=100)
    ch = amp.Preconditioner(Ms[1], "chebyshev", degree=2, lam_lo=0.01, lam_hi=2.0)
    with pytest.raises(B.AmpError):
        amp.solve_batched(Ms, [Ps[0], ch], bs)
