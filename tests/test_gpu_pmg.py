"""The p-multigrid preconditioner (Section 5.3, Ex. linear conv2) on the GPU
against the FP64 oracle (oracle.pmg): the order-1 operator of the lowest
level, one V-cycle z = V(r) in FP64 and FP32 for several order ladders and
mesh shapes, the power-iteration estimate of lambda_max(D^-1 A) against the
oracle's eigensolver, the scaling gain, PCG and AMP-PCG(FP16) with z and p in
FP16 from the first iteration against the oracle's FP64 PCG with the same
cycle, and the arguments it refuses."""

import numpy as np
import pytest
import torch

from oracle import pmg as opmg
from oracle.hexop import HexMesh
from workloads import problems as P

pytestmark = pytest.mark.gpu

# one cycle: a few dozen products and transfers, each exact to rounding in the
# precision of the cycle (FP64: atomic sums in no fixed order; FP32: 2^-24 per
# operation), the error amplified by the smoothers' coefficients (|c2| / lo
# up to ~10 on [0.1 rho, 1.1 rho])
TOL = {64: 1e-12, 32: 1e-5}


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


def _setup(amp, E, orders, lam=0.0, seed=0, **kw):
    V = P.hex_vertices(E, 0.2, seed)
    H = amp.HexOperator(torch.tensor(V, device="cuda"), E, order=orders[0], lam=lam)
    M = amp.Matrix.from_hexop(H)
    pc = amp.Preconditioner.pmg(M, orders=orders, **kw)
    return V, H, M, pc


@pytest.mark.parametrize("E", [(3, 2, 2), (4, 3, 5)])
def test_order1_operator_and_diagonal(amp, E):
    V = P.hex_vertices(E, 0.2, 1)
    H = amp.HexOperator(torch.tensor(V, device="cuda"), E, order=1, lam=3.0)
    m = HexMesh(V, E, N=1, lam=3.0)
    p = np.random.default_rng(91).standard_normal(m.n)
    q, mu = H.apply(torch.tensor(p, device="cuda"))
    qo = m.apply(p)
    err = np.abs(q.cpu().numpy() - qo).max() / np.abs(qo).max()
    _say(f"order-1 operator E={E}: max rel. error {err:.2e}")
    assert err <= 1e-13
    assert mu.item() == pytest.approx(float(p @ qo), rel=1e-12)
    assert np.allclose(H.diagonal().cpu().numpy(), m.diagonal(), rtol=1e-13)


@pytest.mark.parametrize("E,orders,deg,cdeg", [((3, 2, 2), (7, 3, 1), 2, 8), ((4, 3, 5), (7, 3, 1), 3, 5),
                                               ((5, 4, 3), (3, 1), 2, 6), ((3, 3, 2), (7, 1), 1, 4),
                                               ((2, 3, 2), (7,), 2, 3)])
@pytest.mark.parametrize("prec", [64, 32])
def test_cycle_matches_oracle(amp, E, orders, deg, cdeg, prec):
    V, H, M, pc = _setup(amp, E, orders, lam=2.0, seed=2, degree=deg, coarse_degree=cdeg)
    info = pc.pmg_info()
    assert info["orders"] == list(orders)
    m = HexMesh(V, E, N=orders[0], lam=2.0)
    Mo = opmg.PMultigrid(m, orders=orders, degree=deg, coarse_degree=cdeg, rho=info["rho"])
    assert info["n"] == [mm.n for mm in Mo.meshes]
    r = np.random.default_rng([92, prec]).standard_normal(m.n)
    z = pc.pmg_apply(torch.tensor(r, device="cuda"), prec=prec).cpu().numpy()
    zo = Mo.apply64(r) if prec == 64 else Mo.apply(r.astype(np.float32), 32).astype(np.float64)
    err = np.abs(z - zo).max() / np.abs(zo).max()
    _say(f"cycle E={E} orders={orders} degree {deg}/{cdeg} FP{prec}: max rel. error vs the oracle {err:.2e}")
    assert err <= TOL[prec]
    if prec == 64:
        assert info["gain"] == pytest.approx(Mo.gain, rel=1e-10)
    # a second application on the same handle gives the same result (the
    # work vectors are left cleared)
    z2 = pc.pmg_apply(torch.tensor(r, device="cuda"), prec=prec).cpu().numpy()
    assert np.abs(z2 - z).max() <= TOL[prec] * np.abs(zo).max()


def test_rho_estimate_against_eigensolver(amp):
    E, orders = (4, 3, 3), (7, 3, 1)
    V, H, M, pc = _setup(amp, E, orders, lam=0.0, seed=4)
    est = pc.pmg_info()["rho"]
    m = HexMesh(V, E, N=7, lam=0.0)
    Mo = opmg.PMultigrid(m, orders=orders)       # rho by ARPACK
    for l, (a, b) in enumerate(zip(est, Mo.rho)):
        _say(f"level {l} (order {orders[l]}): power iteration {a:.6f}, eigensolver {b:.6f}")
        # a Rayleigh quotient never exceeds lambda_max
        assert a <= b * (1 + 1e-9)
        assert a >= 0.8 * b


@pytest.mark.parametrize("E", [(4, 4, 3), (5, 3, 4)])
# amp64 lowers u_z during the solve: the cycle's precision is then read from
# the state by both product variants (the other returns at once)
@pytest.mark.parametrize("preset,eta", [("pcg64", None), ("amp16", "delay"), ("amp16", "linear"), ("amp64", None)])
def test_pmg_solve_parity(amp, E, preset, eta):
    V, H, M, pc = _setup(amp, E, (7, 3, 1), lam=0.0, seed=5)
    m = HexMesh(V, E, N=7, lam=0.0)
    Mo = opmg.PMultigrid(m, orders=(7, 3, 1), rho=pc.pmg_info()["rho"])
    b = np.random.default_rng(93).standard_normal(m.n)
    xo, io = opmg.pcg(m, Mo, b, tol=1e-10)
    kw = {} if eta is None else {"eta": eta}
    x, info = amp.solve(M, pc, torch.tensor(b, device="cuda"), tol=1e-10, maxit=1000, preset=preset, **kw)
    err = float(np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
    _say(f"pMG solve E={E} {preset} {eta}: {info['iters']} iterations (oracle {io['iters']}), k_z16 "
         f"{info['k_z16']}, k_r32 {info['k_r32']}, rel. error vs the oracle {err:.2e}, true rel. residual "
         f"{info['relres_true']:.2e}")
    assert info["status"] == 0
    assert info["relres_true"] <= 1e-10
    assert info["iters"] <= int(np.ceil(1.05 * io["iters"]))
    assert err <= 1e-8
    if preset == "amp16":
        assert info["k_z16"] == 0          # z and p in FP16 from the first iteration


def test_pmg_refusals(amp):
    from paper_2505_04155_amd import binding as B
    V, H, M, pc = _setup(amp, (2, 2, 2), (7, 3, 1))
    r = torch.ones(H.n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.AmpError, match="amp_pmg_apply"):
        pc.pmg_apply(r, prec=16)
    with pytest.raises(B.AmpError, match="amp_pmg_apply"):
        pc.apply(r, 64)
    assert B.load().amp_precond_update(pc.handle, None) == B.AMP_ERR_ARG
    with pytest.raises(B.AmpError, match="decrease"):
        amp.Preconditioner.pmg(M, orders=(7, 7))
    with pytest.raises(B.AmpError, match="orders\\[0\\]"):
        amp.Preconditioner.pmg(M, orders=(3, 1))
    with pytest.raises(B.AmpError, match="degrees"):
        amp.Preconditioner.pmg(M, degree=33)
    # order 1 on one element per direction has no unknowns
    V1 = P.hex_vertices((1, 2, 2), 0.0)
    H1 = amp.HexOperator(torch.tensor(V1, device="cuda"), (1, 2, 2), order=7)
    with pytest.raises(B.AmpError, match="unknowns"):
        amp.Preconditioner.pmg(amp.Matrix.from_hexop(H1), orders=(7, 1))
    # a stored matrix
    Ms = amp.Matrix.from_csr(P.stencil_poisson2d(16))
    with pytest.raises(B.AmpError, match="matrix-free"):
        amp.Preconditioner.pmg(Ms)
    with pytest.raises(B.AmpError, match="solve takes orders"):
        amp.Matrix.from_hexop(amp.HexOperator(torch.tensor(P.hex_vertices((2, 2, 2), 0.0), device="cuda"),
                                               (2, 2, 2), order=1))
