"""Chebyshev-preconditioned AMP-PCG on the anisotropic Q1 workload (GPU).

* One preconditioner application equals the precision model's, element by
  element (FP16 B, work vectors in the arithmetic precision of u_z).
* The solve agrees with the model and with the FP64 oracle (Alg. 1 with
  the same polynomial), and reaches the manufactured solution.
* The full 256^3 system: FP64 true residual (recomputed by the oracle's
  product) and the error against x*; iteration count against the oracle's
  stored reference.
"""

import math
import os

import numpy as np
import pytest
import torch

from oracle import amp_model as am
from oracle import cpcg
from workloads import problems as P

pytestmark = pytest.mark.gpu

NP = {64: np.float64, 32: np.float32, 16: np.float16}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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


@pytest.mark.parametrize("offsets", [True, False])
@pytest.mark.parametrize("degree", [1, 2, 4])
@pytest.mark.parametrize("u_r,u_z", [(64, 64), (64, 16), (32, 32), (32, 16)])
def test_chebyshev_apply_matches_model(amp, degree, u_r, u_z, offsets):
    # offsets=False keeps every slice in index mode (per-entry columns)
    _say(f"chebyshev apply degree={degree} u_r={u_r} u_z={u_z} offsets={offsets}")
    A, b, xs, (lo, hi) = P.q1_system(18)
    S = A.to_scipy()
    C = am.Chebyshev(S, lo, hi, degree)
    r = (np.random.default_rng([400, degree]).standard_normal(A.n) * 1e-2).astype(NP[u_r])
    omega = 2.0 ** 7
    y = am.fl(am.fl(r.astype(NP[u_r]) * NP[u_r](omega), u_r), u_z)
    zref = C.apply(y, u_z).astype(np.float64)
    M = amp.Matrix.from_csr(A, offsets=offsets)
    pc = amp.Preconditioner(M, "chebyshev", degree=degree, lam_lo=lo, lam_hi=hi)
    z, rho = pc.apply(torch.tensor(r, device="cuda"), u_z=u_z, omega=omega)
    zh = z.cpu().numpy().astype(np.float64)
    ulp = {64: 2.0 ** -52, 32: 2.0 ** -23, 16: 2.0 ** -10}[u_z]
    err = np.abs(zh - zref) / np.maximum(np.abs(zref), 1e-30)
    _say(f"  max rel diff {err.max():.3e}, exact fraction {np.mean(zh == zref):.4f}")
    assert np.max(np.abs(zh - zref)) <= 4 * ulp * np.max(np.abs(zref))
    assert rho.item() == pytest.approx(float(r.astype(np.float64) @ zh), rel=1e-12)


@pytest.mark.parametrize("offsets", [True, False])
@pytest.mark.parametrize("preset", ["pcg64", "amp64", "amp16"])
def test_chebyshev_solve_parity(amp, preset, offsets):
    _say(f"chebyshev solve {preset} offsets={offsets}")
    A, b, xs, (lo, hi) = P.q1_system(24)
    S = A.to_scipy()
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=5000, precond=cpcg.PC_CHEBYSHEV, degree=4, lam_lo=lo, lam_hi=hi)
    ref = am.amp_pcg(S, b, tol=1e-10, maxit=5000, M=am.Chebyshev(S, lo, hi, 4), opt=am.options(preset))
    M = amp.Matrix.from_csr(A, offsets=offsets)
    pc = amp.Preconditioner(M, "chebyshev", degree=4, lam_lo=lo, lam_hi=hi)
    x, info = amp.solve(M, pc, torch.tensor(b, device="cuda"), tol=1e-10, maxit=5000, preset=preset,
                        history=True)
    x = x.cpu().numpy()
    _say(f"  gpu {info['iters']} model {ref.iters} oracle {io['iters']}; switches "
         f"{info['k_z32']} {info['k_z16']} {info['k_r32']} / model {ref.k_z32} {ref.k_z16} {ref.k_r32}")
    assert info["status"] == 0
    assert info["relres_true"] <= 1e-10
    assert abs(info["iters"] - ref.iters) <= max(2, math.ceil(0.02 * ref.iters))
    if preset != "amp16":
        assert info["iters"] <= math.ceil(1.05 * io["iters"])
    kz32, kz16, kr = am.replay_switches(list(info["delta"][:info["iters"]]), info["bnorm"], 1e-10,
                                        am.options(preset))
    assert (kz32, kz16, kr) == (info["k_z32"], info["k_z16"], info["k_r32"])
    kappa = 1.25 * hi / lo                       # bound for the preconditioned operator
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 2e-10


@pytest.mark.parametrize("offsets", [True, False])
def test_chebyshev_poisson_short_rows(amp, offsets):
    # 5-point rows (one partial chunk of slots) in both layouts; the bounds of
    # D^-1 A for the 2-D Poisson stencil are 1 -/+ cos(pi / (m + 1)), and
    # B = D^-1/2 A D^-1/2 (entries 1 and -1/4) is exact in FP16
    m = 48
    A, b, xs = P.poisson2d_system(m)
    lo, hi = 1.0 - math.cos(math.pi / (m + 1)), 1.0 + math.cos(math.pi / (m + 1))
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=5000, precond=cpcg.PC_CHEBYSHEV, degree=4, lam_lo=lo, lam_hi=hi)
    M = amp.Matrix.from_csr(A, offsets=offsets)
    pc = amp.Preconditioner(M, "chebyshev", degree=4, lam_lo=lo, lam_hi=hi)
    x, info = amp.solve(M, pc, torch.tensor(b, device="cuda"), tol=1e-10, maxit=5000, preset="pcg64")
    _say(f"chebyshev poisson {m} offsets={offsets}: {info['iters']} iterations (oracle {io['iters']})")
    assert info["status"] == 0 and info["relres_true"] <= 1e-10
    assert abs(info["iters"] - io["iters"]) <= 2
    # both stop at ||r|| <= 1e-10 ||b||: solutions agree within 2 tol kappa(A), kappa(A) = hi / lo
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 2e-10 * (hi / lo) * np.linalg.norm(xo)


# ------------------------------------------------------------------ estimated bounds

def _q1(n):
    return P.q1_anisotropic(n)


@pytest.mark.parametrize("case", ["q1_20", "q1_64", "q1_256", "blocky24"])
def test_estimated_bounds(amp, case):
    # lam <= 0 asks the library for the interval: its Lanczos Ritz extremes
    # equal the oracle's (same steps and start vector, independent code) to
    # rounding, and for the Q1 operator the interval holds the closed-form
    # top of the spectrum within the 5% margin
    from oracle import eigbounds as E
    _say(f"estimated Chebyshev bounds {case}")
    if case.startswith("q1"):
        n = int(case[3:])
        A = _q1(n)
        exact = P.q1_anisotropic_bounds(n)
    else:
        A, _, _ = P.blocky_diffusion3d_system(24, 4)
        exact = None
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, "chebyshev", degree=4, lam_lo=0.0, lam_hi=0.0)
    lo, hi, tmin, tmax = pc.bounds()
    _say(f"  gpu: ritz [{tmin:.6e}, {tmax:.6e}] -> [{lo:.6e}, {hi:.6e}]")
    if A.n <= 300000:
        (olo, ohi), (otmin, otmax) = E.chebyshev_bounds(A.to_scipy())
        _say(f"  oracle: ritz [{otmin:.6e}, {otmax:.6e}]")
        assert tmax == pytest.approx(otmax, rel=1e-9)
        assert tmin == pytest.approx(otmin, rel=1e-7)
    assert hi == pytest.approx(1.05 * tmax, rel=1e-15) and lo == pytest.approx(hi / 30.0, rel=1e-15)
    if exact is not None:
        _say(f"  closed form: [{exact[0]:.6e}, {exact[1]:.6e}]")
        assert exact[0] * (1 - 1e-12) <= tmin and tmax <= exact[1] * (1 + 1e-12)
        assert exact[1] <= hi <= 1.05 * exact[1] * (1 + 1e-12)


@pytest.mark.parametrize("preset", ["pcg64", "amp64", "amp16"])
def test_solve_with_estimated_bounds(amp, preset):
    # each side estimates its own interval; the solves agree to the parity bar
    from oracle import eigbounds as E
    _say(f"solve with estimated bounds, Q1 32^3, {preset}")
    A = _q1(32)
    xs = np.random.default_rng([330]).uniform(-1.0, 1.0, A.n)
    b = A.to_scipy() @ xs
    (olo, ohi), _ = E.chebyshev_bounds(A.to_scipy())
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=5000, precond=cpcg.PC_CHEBYSHEV, degree=4, lam_lo=olo, lam_hi=ohi)
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, "chebyshev", degree=4)
    x, info = amp.solve(M, pc, torch.tensor(b, device="cuda"), tol=1e-10, maxit=5000, preset=preset)
    err = float(np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
    _say(f"  gpu {info['iters']} iterations, oracle {io['iters']}; rel. error vs the oracle {err:.3e}")
    assert info["status"] == 0 and io["status"] == 0
    assert info["iters"] <= math.ceil(1.05 * io["iters"])
    assert err <= 1e-8
