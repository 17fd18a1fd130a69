"""Differentiable solve (GPU): forward AMP-PCG, adjoint AMP-PCG and the face
gather kernel behind torch.autograd, against central finite differences of
the FP64 oracle (16^3) and the oracle's FP64 adjoint gradient (64^3)."""

import numpy as np
import pytest
import torch

from oracle import adjoint as adj
from oracle import cpcg
from workloads import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def amp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_2505_04155_amd import binding
    binding.load(build_if_missing=False)
    from paper_2505_04155_amd import adjoint as amp_adj
    return amp_adj


def _say(msg):
    print(msg, flush=True)


def _gpu_grad(amp_adj, theta, b, xt, preset="amp64", tol=1e-10):
    sysm = amp_adj.FVSystem(theta.shape, preset=preset, tol=tol)
    th = torch.tensor(theta, device="cuda", requires_grad=True)
    bt = torch.tensor(b, device="cuda", requires_grad=True)
    x = amp_adj.diff_solve(th, bt, sysm)
    loss = 0.5 * ((x - torch.tensor(xt, device="cuda")) ** 2).sum()
    loss.backward()
    return (float(loss), th.grad.double().cpu().numpy(), bt.grad.cpu().numpy(), x.detach().cpu().numpy())


def test_fv_assembly_matches_oracle(amp):
    _say("fv assembly 12^3 and 2-D 9x7")
    from paper_2505_04155_amd import binding as B
    for shape in ((12, 12, 12), (7, 9)):
        theta = np.random.default_rng([510, len(shape)]).standard_normal(shape).astype(np.float32)
        sysm = amp.FVSystem(shape)
        sysm.assemble(torch.tensor(theta, device="cuda"))
        A = adj.assemble(theta.astype(np.float64))
        assert np.array_equal(sysm.row_ptr.cpu().numpy(), A.indptr)
        assert np.array_equal(sysm.col_idx.cpu().numpy(), A.indices)
        assert np.allclose(sysm.val.cpu().numpy(), A.data, rtol=1e-14, atol=0)


@pytest.mark.parametrize("preset", ["amp64", "amp16"])
def test_gradient_vs_central_differences_16(amp, preset):
    _say(f"adjoint 16^3 vs central differences ({preset})")
    theta, b, xt = P.adjoint_inputs(16)
    L, g, gb, x = _gpu_grad(amp, theta, b, xt, preset=preset)
    th64 = theta.astype(np.float64)
    Lo, go, lamo, xo = adj.loss_and_grad(th64, b, xt)
    assert L == pytest.approx(Lo, rel=1e-8)
    h = 1e-4
    errs = []
    rng = np.random.default_rng([511, 0])
    for t in range(16):
        d = rng.standard_normal(theta.shape)
        fd = (adj.loss(th64 + h * d, b, xt) - adj.loss(th64 - h * d, b, xt)) / (2 * h)
        errs.append(abs(float((g * d).sum()) - fd) / abs(fd))
    flat = th64.reshape(-1)
    for c in (0, 1, 17, 300, 2048, 4000, 4094, 4095):
        e = np.zeros_like(flat)
        e[c] = h
        fd = (adj.loss((flat + e).reshape(theta.shape), b, xt) - adj.loss((flat - e).reshape(theta.shape), b, xt)) / (2 * h)
        errs.append(abs(g.reshape(-1)[c] - fd) / max(abs(fd), 1e-3 * np.abs(g).max()))
    _say(f"  max rel error vs FD {max(errs):.3e}")
    assert max(errs) <= 1e-5
    # dL/db = lambda
    assert np.linalg.norm(gb - lamo) <= 1e-6 * np.linalg.norm(lamo)
    # homogeneity invariant: sum of dL/dtheta = -b^T lambda
    assert g.sum() == pytest.approx(-(b @ gb), rel=1e-5)


def test_gradient_vs_oracle_64(amp):
    _say("adjoint 64^3 vs FP64 oracle gradient")
    theta, b, xt = P.adjoint_inputs(64)
    L, g, gb, x = _gpu_grad(amp, theta, b, xt)
    solver = lambda A, rhs: cpcg.pcg(P.CSR(A.shape[0], A.indptr.astype(np.int32), A.indices.astype(np.int32),
                                           A.data), rhs, tol=1e-14, maxit=50000)[0]
    Lo, go, lamo, xo = adj.loss_and_grad(theta.astype(np.float64), b, xt, solver=solver)
    rel = np.linalg.norm(g - go) / np.linalg.norm(go)
    _say(f"  rel. gradient error {rel:.3e}, loss {L:.6e} vs {Lo:.6e}")
    assert rel <= 1e-5
    assert np.linalg.norm(gb - lamo) <= 1e-6 * np.linalg.norm(lamo)
