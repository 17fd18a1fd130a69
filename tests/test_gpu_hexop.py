"""The matrix-free hexahedral operator (Section 5.5, Ex. jac libp) on the
GPU against the FP64 oracle: q = A p element by element at sizes the oracle
applies whole (several elements in each direction, orders 3 and 7, every
storage/arithmetic precision pair), sampled nodes of the 40^3-element,
order-7 mesh of the paper (21.7 million unknowns) against the oracle applied
to each sampled node's neighbourhood, mu, the diagonal, symmetry, and the
arguments it refuses."""

import numpy as np
import pytest
import torch

from oracle.hexop import HexMesh
from workloads import problems as P

pytestmark = pytest.mark.gpu

NP = {64: np.float64, 32: np.float32, 16: np.float16}
TT = {64: torch.float64, 32: torch.float32, 16: torch.float16}
# FP64 arithmetic: the sums differ from the oracle's only in rounding order
# (and fused multiply-adds), a few units of 2^-53 times the terms' magnitude;
# FP32 arithmetic (geometric factors, contractions, q): 2^-24 per operation
# over a few dozen operations per entry
TOL = {64: 1e-12, 32: 1e-6}


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


def _op(amp, E, N, perturb=0.2, seed=0, lam=1e3):
    V = P.hex_vertices(E, perturb, seed)
    H = amp.HexOperator(torch.tensor(V, device="cuda"), E, order=N, lam=lam)
    return V, H


@pytest.mark.parametrize("N,E", [(7, (3, 2, 4)), (3, (5, 3, 2)), (7, (1, 1, 2))])
@pytest.mark.parametrize("up,ur", [(64, 64), (16, 64), (32, 32), (16, 32)])
def test_apply_matches_oracle(amp, N, E, up, ur):
    V, H = _op(amp, E, N, seed=1)
    m = HexMesh(V, E, N=N, lam=1e3)
    assert H.n == m.n
    p = np.random.default_rng([81, N, up]).standard_normal(m.n).astype(NP[up])
    q, mu = H.apply(torch.tensor(p, device="cuda"), u_r=ur)
    torch.cuda.synchronize()
    qo = m.apply(p.astype(np.float64))
    err = np.abs(q.double().cpu().numpy() - qo).max() / np.abs(qo).max()
    _say(f"hex N={N} E={E} p{up} q{ur}: max |q - q_oracle| / max|q_oracle| = {err:.2e}")
    assert err <= TOL[ur]
    muo = float(p.astype(np.float64) @ qo)
    assert abs(mu.item() - muo) <= TOL[ur] * abs(muo) * 10


def test_diagonal_and_determinism(amp):
    E, N = (3, 4, 2), 7
    V, H = _op(amp, E, N, seed=2)
    m = HexMesh(V, E, N=N, lam=1e3)
    d = H.diagonal().cpu().numpy()
    do = m.diagonal()
    assert np.abs(d - do).max() <= 1e-12 * np.abs(do).max()
    p = torch.tensor(np.random.default_rng(82).standard_normal(m.n), device="cuda")
    _, mu1 = H.apply(p)
    _, mu2 = H.apply(p)
    assert mu1.item() == mu2.item()        # element partials summed in a fixed order


def _local_q(V, E, N, lam, p_grid, node):
    """The oracle's (A p) at grid node (gx, gy, gz): the operator applied on
    the block of elements containing the node (every contribution to it)."""
    gx, gy, gz = node
    Ex, Ey, Ez = E
    lo = [max(0, (g - 1) // N) if g % N == 0 else g // N for g in (gx, gy, gz)]
    hi = [min(Ei - 1, g // N) for g, Ei in zip((gx, gy, gz), E)]
    sub = [h - l + 1 for l, h in zip(lo, hi)]
    Vg = V.reshape(Ez + 1, Ey + 1, Ex + 1, 3)[lo[2]:hi[2] + 2, lo[1]:hi[1] + 2, lo[0]:hi[0] + 2]
    m = HexMesh(Vg.reshape(-1, 3), tuple(sub), N=N, lam=lam)
    pg = p_grid[lo[2] * N:(hi[2] + 1) * N + 1, lo[1] * N:(hi[1] + 1) * N + 1, lo[0] * N:(hi[0] + 1) * N + 1]
    out = m.apply_full(pg.reshape(-1)).reshape(pg.shape)
    return out[gz - lo[2] * N, gy - lo[1] * N, gx - lo[0] * N]


@pytest.mark.timeout(300)
def test_paper_size_sampled(amp):
    E, N, lam = (40, 40, 40), 7, 1e3
    V, H = _op(amp, E, N, seed=0)
    _say(f"hex 40^3 order 7: n = {H.n}")
    assert H.n == 279 ** 3
    rng = np.random.default_rng(83)
    p = rng.standard_normal(H.n)
    pt = torch.tensor(p, device="cuda")
    q, mu = H.apply(pt)
    v = torch.tensor(rng.standard_normal(H.n), device="cuda")
    qv, _ = H.apply(v)
    torch.cuda.synchronize()
    # symmetry: v^T A p = p^T A v
    a, b = float(v @ q), float(pt @ qv)
    assert abs(a - b) <= 1e-11 * max(abs(a), abs(b))
    assert abs(mu.item() - float(pt @ q)) <= 1e-11 * abs(mu.item())
    # sampled nodes: element interiors, faces, edges, corners, next to the boundary
    M = N * 40
    pgrid = np.zeros((M + 1,) * 3)
    pgrid[1:-1, 1:-1, 1:-1] = p.reshape(M - 1, M - 1, M - 1)
    qh = q.cpu().numpy()
    picks = [(1, 1, 1), (7, 7, 7), (M - 1, M - 1, M - 1), (7, 3, 14), (140, 141, 139), (28, 35, 273)]
    picks += [tuple(int(x) for x in rng.integers(1, M, 3)) for _ in range(24)]
    worst = 0.0
    for gx, gy, gz in picks:
        ref = _local_q(V, E, N, lam, pgrid, (gx, gy, gz))
        got = qh[(gx - 1) + (M - 1) * ((gy - 1) + (M - 1) * (gz - 1))]
        worst = max(worst, abs(got - ref) / max(abs(ref), 1e-300))
    _say(f"  {len(picks)} sampled nodes: worst relative difference {worst:.2e}")
    assert worst <= 1e-11


def test_refused_arguments(amp):
    from paper_2505_04155_amd import binding as B
    E = (2, 2, 2)
    V = P.hex_vertices(E, 0.0)
    Vt = torch.tensor(V, device="cuda")
    with pytest.raises(B.AmpError, match="order"):
        amp.HexOperator(Vt, E, order=5)
    with pytest.raises(B.AmpError, match="lambda"):
        amp.HexOperator(Vt, E, order=3, lam=-1.0)
    # an inverted element: the middle vertex pushed past its neighbour
    W = V.copy().reshape(3, 3, 3, 3)
    W[1, 1, 1, 0] = 0.75
    with pytest.raises(B.AmpError, match="Jacobian"):
        amp.HexOperator(torch.tensor(W.reshape(-1, 3), device="cuda"), E, order=3)
    H = amp.HexOperator(Vt, E, order=3)
    with pytest.raises(B.AmpError, match="u_r"):
        H.apply(torch.zeros(H.n, dtype=torch.float64, device="cuda"), u_r=32)


@pytest.mark.parametrize("N,E", [(7, (4, 3, 3)), (3, (6, 5, 4))])
@pytest.mark.parametrize("preset", ["pcg64", "amp64", "amp16"])
def test_matrix_free_solve_parity(amp, N, E, preset):
    from oracle import hexop
    V, H = _op(amp, E, N, seed=3)
    m = HexMesh(V, E, N=N, lam=1e3)
    b = np.random.default_rng([85, N]).standard_normal(m.n)
    xo, io = hexop.pcg(m, b, tol=1e-10, maxit=5000)
    M = amp.Matrix.from_hexop(H)
    pc = amp.Preconditioner(M, "jacobi")
    x, info = amp.solve(M, pc, torch.tensor(b, device="cuda"), tol=1e-10, maxit=5000, preset=preset)
    err = float(np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
    _say(f"matrix-free solve N={N} E={E} {preset}: {info['iters']} iterations (oracle {io['iters']}), "
         f"rel. error vs the oracle {err:.2e}, true rel. residual {info['relres_true']:.2e}")
    assert info["status"] == 0
    assert info["relres_true"] <= 1e-10
    assert info["iters"] <= int(np.ceil(1.05 * io["iters"]))
    assert err <= 1e-8


def test_matrix_free_handle_refusals(amp):
    from paper_2505_04155_amd import binding as B
    V, H = _op(amp, (2, 2, 2), 3)
    M = amp.Matrix.from_hexop(H)
    with pytest.raises(B.AmpError, match="stored matrix"):
        amp.Preconditioner(M, "chebyshev", degree=2, lam_lo=0.1, lam_hi=2.0)
    pc = amp.Preconditioner(M, "jacobi")
    b = torch.ones(H.n, dtype=torch.float64, device="cuda")
    with pytest.raises(B.AmpError, match="matrix-free"):
        amp.solve(M, pc, b, tol=1e-10, maxit=100, preset="amp64", rr_period=5)
    with pytest.raises(B.AmpError, match="matrix-free"):
        M.spmv(b)

