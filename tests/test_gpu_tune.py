"""Rows-per-work-group autotuner (amp_tune_group_rows) on the GPU: it returns
the candidate with the least measured time (each finite and non-negative; on
systems this small the differences are close to the timing noise), the
chosen value solves the system, and bad arguments are rejected."""
import math

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


def test_tune_single_system(amp):
    A, b, _ = P.blocky_diffusion3d_system(32, 8)
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, "jacobi")
    bt = torch.tensor(b, device="cuda")
    cands = (0, 1024, 4096)
    best, ms = amp.tune_group_rows(M, pc, bt, iters=16, candidates=cands, preset="amp16")
    _say(f"tune single: best {best}, ms/iter {ms}")
    assert best in cands
    assert set(ms) == set(cands)
    assert all(math.isfinite(t) and t >= 0 for t in ms.values())
    assert ms[best] == min(ms.values())
    x, info = amp.solve(M, pc, bt, tol=1e-10, maxit=5000, preset="amp16", group_rows=best)
    torch.cuda.synchronize()
    assert info["status"] == 0 and info["relres_true"] <= 1e-10
    xo, io = cpcg.pcg(A, b, tol=1e-10, maxit=5000)
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-6 * np.linalg.norm(xo)


def test_tune_batch(amp):
    systems = [P.poisson2d_system(m)[:2] for m in (24, 48)] + P.batched_systems(count=4, side_min=32, side_max=128)
    Ms = [amp.Matrix.from_csr(A) for A, _ in systems]
    Ps = [amp.Preconditioner(M, "jacobi") for M in Ms]
    bs = [torch.tensor(b, device="cuda") for _, b in systems]
    cands = (1024, 2048, 4096)
    best, ms = amp.tune_group_rows(Ms, Ps, bs, iters=24, candidates=cands, preset="amp64")
    _say(f"tune batch: best {best}, ms/iter {ms}")
    assert best in cands and all(math.isfinite(t) and t >= 0 for t in ms.values())
    assert ms[best] == min(ms.values())
    xs, infos, st = amp.solve_batched(Ms, Ps, bs, tol=1e-10, maxit=5000, preset="amp64", group_rows=best)
    torch.cuda.synchronize()
    assert st == 0 and all(i["relres_true"] <= 1e-10 for i in infos)


def test_tune_rejects_bad_arguments(amp):
    from paper_2505_04155_amd import binding as B
    A, b, _ = P.poisson2d_system(16)
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, "jacobi")
    bt = torch.tensor(b, device="cuda")
    for kw in (dict(candidates=(100,)), dict(candidates=(-256,)), dict(iters=0), dict(candidates=())):
        with pytest.raises(B.AmpError):
            amp.tune_group_rows(M, pc, bt, **kw)
