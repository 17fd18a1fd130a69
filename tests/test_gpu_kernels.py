"""Kernel-level parity of the HIP path against the oracle (GPU).

* SpMV on integer-valued matrices and small-integer vectors is exact in
  every precision, so the GPU result must equal the CPU product bitwise.
* SpMV on real data agrees with the FP64 oracle / the FP32 model.
* The scaled Jacobi application z = M^{-1} fl(omega r) follows the same
  rounding sequence as the precision model, element by element.
"""

import numpy as np
import pytest
import torch

from oracle import amp_model as am
from oracle import cpcg
from workloads import problems as P

pytestmark = pytest.mark.gpu

TORCH = {64: torch.float64, 32: torch.float32, 16: torch.float16}
NP = {64: np.float64, 32: np.float32, 16: np.float16}


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


@pytest.mark.parametrize("m", [37, 64])
@pytest.mark.parametrize("u_r,diff", [(64, False), (32, True), (32, False)])
@pytest.mark.parametrize("u_p", [64, 32, 16])
def test_spmv_integer_exact(amp, m, u_r, diff, u_p):
    _say(f"spmv exact m={m} u_r={u_r} diff={diff} u_p={u_p}")
    A = P.stencil_poisson2d(m)                  # ragged n = 1369 for m = 37
    p = np.random.default_rng([300, m]).integers(-8, 9, A.n).astype(np.float64)
    ref = A.to_scipy() @ p
    M = amp.Matrix.from_csr(A)
    q, g = M.spmv(torch.tensor(p, dtype=TORCH[u_p], device="cuda"), u_r=u_r, diff=diff)
    torch.cuda.synchronize()
    qh = q.cpu().numpy().astype(np.float64)
    assert np.array_equal(qh, ref)
    assert g.item() == float(ref @ p)


@pytest.mark.parametrize("case", ["poisson37", "blocky24", "q1_10", "dense12"])
@pytest.mark.parametrize("u_r,diff,u_p", [(64, False, 64), (64, False, 16), (32, True, 16), (32, False, 32)])
def test_offset_slices_match_index_slices(amp, case, u_r, diff, u_p):
    # shared per-slice column offsets only change how columns are found:
    # the nonzero terms are added in the same order, so results are identical
    _say(f"offset vs index slices {case} u_r={u_r} diff={diff} u_p={u_p}")
    if case == "poisson37":
        A = P.stencil_poisson2d(37)
    elif case == "blocky24":
        A = P.blocky_diffusion3d_system(24, 4)[0]
    elif case == "q1_10":
        A = P.q1_anisotropic(10)
    else:
        A = P.dense_to_csr(P.spectrum_matrix(np.linspace(1, 3, 12), seed=(320, 0)))
    p = np.random.default_rng([321, 0]).standard_normal(A.n).astype({64: np.float64, 32: np.float32, 16: np.float16}[u_p])
    Mo = amp.Matrix.from_csr(A, offsets=True)
    Mi = amp.Matrix.from_csr(A, offsets=False)
    io, ii = Mo.info(), Mi.info()
    if case != "dense12":
        assert io["offset_slices"] > 0
    assert ii["offset_slices"] == 0
    qo, go = Mo.spmv(torch.tensor(p, device="cuda"), u_r=u_r, diff=diff)
    qi, gi = Mi.spmv(torch.tensor(p, device="cuda"), u_r=u_r, diff=diff)
    assert torch.equal(qo, qi)
    assert go.item() == gi.item()


def test_spmv_fp64_matches_oracle(amp):
    _say("spmv fp64 vs oracle, blocky 24^3")
    A, _, _ = P.blocky_diffusion3d_system(24, 4)
    p = np.random.default_rng([301, 0]).standard_normal(A.n)
    ref = cpcg.spmv(A, p)
    M = amp.Matrix.from_csr(A)
    q, g = M.spmv(torch.tensor(p, device="cuda"), u_r=64)
    qh = q.cpu().numpy()
    assert np.max(np.abs(qh - ref)) <= 1e-13 * np.max(np.abs(ref))
    assert g.item() == pytest.approx(float(ref @ p), rel=1e-12)


@pytest.mark.parametrize("u_p", [32, 16])
def test_spmv_fp32_difference_form_matches_model(amp, u_p):
    _say(f"spmv fp32 diff vs model u_p={u_p}")
    A, _, _ = P.blocky_diffusion3d_system(24, 4)
    S = A.to_scipy()
    p = np.random.default_rng([302, u_p]).standard_normal(A.n).astype(NP[u_p])
    ref = am._diff_spmv32(S)(p).astype(np.float64)
    M = amp.Matrix.from_csr(A)
    q, _ = M.spmv(torch.tensor(p, device="cuda"), u_r=32, diff=True)
    qh = q.cpu().numpy().astype(np.float64)
    exact = S @ p.astype(np.float64)
    scale = np.abs(S) @ np.abs(p.astype(np.float64))
    # same operation order as the model: agreement to a couple of FP32 ulps
    assert np.all(np.abs(qh - ref) <= 4 * 2.0 ** -24 * scale)
    # and the product is accurate to FP32 rounding of its terms
    assert np.all(np.abs(qh - exact) <= 16 * 2.0 ** -24 * scale)


@pytest.mark.parametrize("u_r", [64, 32])
@pytest.mark.parametrize("u_z", [64, 32, 16])
def test_jacobi_apply_matches_model(amp, u_r, u_z):
    _say(f"jacobi apply u_r={u_r} u_z={u_z}")
    A, _, _ = P.blocky_diffusion3d_system(16, 4)
    S = A.to_scipy()
    r = (np.random.default_rng([303, u_r]).standard_normal(A.n) * 1e-3).astype(NP[u_r])
    J = am.Jacobi(S)
    omega = 2.0 ** 9
    omega_eff = omega * 2.0 ** (-J.log2_extra[u_z])
    y = am.fl(am.fl(r.astype(NP[u_r]) * NP[u_r](omega_eff), u_r), u_z)
    zref = J.apply(y, u_z)
    M = amp.Matrix.from_csr(A)
    pc = amp.Preconditioner(M, "jacobi")
    z, rho = pc.apply(torch.tensor(r, device="cuda"), u_z=u_z, omega=omega)
    zh = z.cpu().numpy()
    assert np.array_equal(zh, zref)
    rho_ref = float(r.astype(np.float64) @ zref.astype(np.float64))
    assert rho.item() == pytest.approx(rho_ref, rel=1e-13)


def _near_half_ties(seed):
    g = np.random.default_rng([seed, 0])
    x = g.standard_normal(20000) * 2.0 ** g.integers(-26, 15, 20000)
    h = x.astype(np.float16).astype(np.float64)
    ulp = np.spacing(np.abs(x.astype(np.float16))).astype(np.float64)
    ties = np.sign(x) * (np.abs(h) + ulp / 2)
    xs = np.concatenate([x, ties, ties * (1 + 2.0 ** -40), ties * (1 - 2.0 ** -40), ties * (1 + 2.0 ** -29),
                         ties * (1 - 2.0 ** -29), [0.0, -0.0, 1e-300, -1e-300, 2.0 ** -25,
                                                  2.0 ** -25 * (1 + 2.0 ** -50), 65519.99, -65519.99]])
    return xs[np.abs(xs) < 65504]


def test_fp64_to_fp16_rounds_once(amp):
    # identity preconditioner and omega = 1: z = fl16(r) rounded directly
    # from FP64 (a cast through FP32 would round twice near FP16 ties)
    _say("fp64 -> fp16 single rounding")
    xs = _near_half_ties(310)
    n = xs.size
    I = P.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    M = amp.Matrix.from_csr(I)
    pc = amp.Preconditioner(M, "identity")
    z, _ = pc.apply(torch.tensor(xs, device="cuda"), u_z=16, omega=1.0)
    got = z.cpu().numpy()
    ref = xs.astype(np.float16)
    assert np.array_equal(got.view(np.uint16), ref.view(np.uint16))
    assert np.count_nonzero(xs.astype(np.float32).astype(np.float16) != ref) > 1000   # the cases matter


def test_matrix_handle_rejects_bad_input(amp):
    from paper_2505_04155_amd import binding as B
    A = P.dense_to_csr(np.diag([1.0, -2.0, 3.0]))
    with pytest.raises(B.AmpError) as e:
        amp.Matrix.from_csr(A)
    assert e.value.status == B.AMP_ERR_ARG
    bad = P.CSR(3, np.array([0, 1, 2, 3], np.int32), np.array([0, 5, 2], np.int32), np.ones(3))
    with pytest.raises(B.AmpError):
        amp.Matrix.from_csr(bad)
    # row pointers out of order / past nnz, unsorted and duplicate columns:
    # all rejected by the device-side check before any entry is gathered
    cases = [
        ([0, 2, 1, 4], [0, 1, 1, 2]),
        ([0, 2, 3, 9], [0, 1, 1, 2]),
        ([0, 2, 3, 4], [1, 0, 1, 2]),
        ([0, 2, 3, 4], [0, 0, 1, 2]),
    ]
    for rp, ci in cases:
        _say(f"reject rp={rp} ci={ci}")
        c = P.CSR(3, np.array(rp, np.int32), np.array(ci, np.int32), np.array([2.0, -1.0, 2.0, 2.0]))
        for offsets in (True, False):
            with pytest.raises(B.AmpError) as e:
                amp.Matrix.from_csr(c, offsets=offsets)
            assert e.value.status == B.AMP_ERR_ARG
