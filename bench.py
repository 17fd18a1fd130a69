#!/usr/bin/env python3
"""Time-to-solution of AMP-PCG versus FP64 PCG on one MI355X.

A step is one complete solve (every kernel of the hot path, from r0 = b - A x0
to the verified solution) of the anisotropic Q1 system: trilinear finite
elements for -div(diag(1, 1e-2, 1e-3) grad u) on the unit cube, 256^3
interior nodes (N = 16,777,216, nnz = 449,455,096), with the degree-4
Chebyshev polynomial preconditioner (B = D^{-1/2} A D^{-1/2} stored in FP16),
x* ~ U[-1, 1], b = A x*, x0 = 0, tol 1e-10.  Inputs are resident in HBM
before the timed region starts.

One JSON line: value = AMP-PCG(FP16) time-to-solution (ms, lower is better;
the variant the paper times: z and p in FP16 from the start, r and q
switching FP64 -> FP32 by the delay criterion).  Beside it: the stepwise
AMP-PCG(FP64) and PCG(FP64) times on the same GPU (PCG(FP64) applies the same
preconditioner -- the polynomial in FP64 arithmetic on the FP16-stored B),
iteration counts and switch points, each preset's error against x* and its
bound against the FP64 oracle's solution, the HBM roofline of the dominant
kernel (the Chebyshev step, every launch of one AMP-PCG(FP16) solve timed by
HIP events carried by its own dispatch) with the product kernel's beside
it, the library's stream probes as the measured ceiling, the FP64 CPU oracle
timed on the host on a bounded sample, and as secondary measurements the
128^3 finite-volume workload, the 512-system batched solve, the matrix-free
order-7 hexahedral operator with Jacobi-PCG on it (Ex. jac libp), and the
p-multigrid preconditioned Poisson problem (Ex. linear conv2).

Modes: --mode roofline runs only the timed solve and the probes (the command
the kernel-trace and counter runs profile); --mode fv128, --mode batched,
--mode hex and --mode pmg run one secondary workload alone.
"""

from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time-to-solution at rel. residual 1e-10, AMP-PCG vs FP64 PCG; SpMV HBM GB/s"
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILES = {
    ("q1", "k_cheb_step"): os.path.join(PROFILES, "k_cheb_step_q1_256_hbm_counters.txt"),
    ("q1", "k_spmv"): os.path.join(PROFILES, "k_spmv_q1_256_hbm_counters.txt"),
    ("fv128", "k_spmv"): os.path.join(PROFILES, "k_spmv_fv3d128_hbm_counters.txt"),
}
Q1_GOLDEN = os.path.join(ROOT, "tests", "golden", "q1_256_chebyshev4.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ----------------------------------------------------------------------------
# algorithmic bytes (values, column metadata, each vector read once and
# written once; gathers counted once; slice padding not counted)
# ----------------------------------------------------------------------------

def step_bytes(n, nnz, meta_bytes, u_z, u_r):
    """One product step p = z + beta p_old, q = A p in (u_z, u_r): every
    nonzero's value once (FP64 plane for u_r = 64, FP32 plane otherwise),
    the column metadata once, z and p_old read, p and q written."""
    b_val = 8 if u_r == 64 else 4
    return nnz * b_val + meta_bytes + n * (3 * (u_z // 8) + u_r // 8)


def cheb_iteration_bytes(n, nnz, meta_bytes, u_z, u_r, degree=4):
    """The degree - 1 polynomial-step launches of one preconditioner
    application in (u_z, u_r), iterate form: each reads B's FP16 values and
    the column metadata once; the work vectors are held in c = 8 bytes
    (u_z = FP64) or 4 (otherwise).  Step 0 gathers v and writes x_2 (2c);
    step 1 gathers x_2, reads v and writes x_3 (3c); later inner steps also
    read x_{k-1} (4c); the last step reads its gathered x_k, v, x_{k-1}
    (none on step 0, v's on step 1), D^{-1/2} and r (u_r) and writes z
    (u_z)."""
    c = 8 if u_z == 64 else 4
    m = degree - 1
    if m < 1:
        return 0
    tail = c + u_r // 8 + u_z // 8          # D^{-1/2}, r and z of the last step
    if m == 1:     # one step, first and last: gathers v
        vec = c + tail
    else:
        vec = 2 * c                          # step 0
        for k in range(1, m - 1):
            vec += 3 * c if k == 1 else 4 * c
        vec += (2 * c if m - 1 == 1 else 3 * c) + tail
    return m * (2 * nnz + meta_bytes) + n * vec


def jacobi_iteration_bytes(n, nnz, meta_bytes, u_z, u_r):
    """One Jacobi-preconditioned iteration's three kernels in (u_z, u_r):
    preconditioning reads r and dinv and writes z; the product step as
    step_bytes; the update reads r and q and writes r, and every other
    iteration reads and writes x and reads the two pending p (8 + u_z / 8
    bytes per row per iteration on average)."""
    bz, br = u_z // 8, u_r // 8
    return n * (br + 2 * bz) + step_bytes(n, nnz, meta_bytes, u_z, u_r) + n * (3 * br + 8 + bz)


def phase_iterations(info, preset):
    """(u_z, u_r) -> iterations of one solve, from its switch points."""
    it, kz32, kz16, kr = info["iters"], info["k_z32"], info["k_z16"], info["k_r32"]
    out = {}
    for k in range(it):
        if preset == "amp16":
            uz = 16
        else:
            uz = 16 if 0 <= kz16 <= k else 32 if 0 <= kz32 <= k else 64
        ur = 32 if 0 <= kr <= k else 64
        out[(uz, ur)] = out.get((uz, ur), 0) + 1
    return out


def stored_traffic(path):
    """HBM bytes per launch from a committed FETCH_SIZE / WRITE_SIZE summary
    (each counter scaled by what it reads for the library's copy probe of
    known size), or None when the summary is missing or was taken on other
    kernel sources than the library built here."""
    from paper_2505_04155_amd import build
    try:
        fields = {}
        with open(path) as f:
            for line in f:
                if line.strip() and not line.startswith("#"):
                    key, _, val = line.partition(" ")
                    fields[key] = val.strip()
    except OSError:
        return None
    if fields.get("source_digest") != build.source_digest():
        return None
    return int(float(fields["traffic_bytes_per_launch"]))


def _phases(info):
    out = {}
    for uz, ur in zip(info["uz"], info["ur"]):
        out[f"z{uz}_r{ur}"] = out.get(f"z{uz}_r{ur}", 0) + 1
    return out


def timed_solve(amp, M, pc, bt, preset, tol, maxit):
    """One solve with every product and Chebyshev-step launch timed by HIP
    events carried by the launch's own dispatch on the solve's stream."""
    x, info = amp.solve(M, pc, bt, tol=tol, maxit=maxit, preset=preset, history=True, spmv_timing=1)
    if info["status"] != 0:
        raise RuntimeError(f"timed solve failed: {info}")
    return info


def roofline_entry(kernel, total_bytes, total_ms, launches, traffic, phases):
    gbs = total_bytes / (total_ms * 1e-3) / 1e9
    return {
        "bound": "hbm",
        "kernel": kernel,
        "achieved": round(gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(gbs / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "avg_kernel_us": round(total_ms * 1e3 / launches, 3),
        "launches": launches,
        "algorithmic_bytes_per_launch": round(total_bytes / launches),
        "phase_iterations": phases,
    }


def rooflines(info, info_m, workload, degree=None):
    n, nnz, meta = info_m["n"], info_m["nnz"], info_m["meta_bytes"]
    prec = list(zip(info["uz"], info["ur"]))
    ph = _phases(info)
    sp_bytes = sum(step_bytes(n, nnz, meta, uz, ur) for uz, ur in prec)
    sp = roofline_entry(
        "k_spmv: p = z + beta p_old (u_z), q = A p (u_r), gamma partials; every launch of the timed solve",
        sp_bytes, info["spmv_ms"], info["spmv_launches"], stored_traffic(TRAFFIC_FILES[(workload, "k_spmv")]), ph)
    if degree is None or info.get("cheb_launches", 0) == 0:
        return sp, None
    ch_bytes = sum(cheb_iteration_bytes(n, nnz, meta, uz, ur, degree) for uz, ur in prec)
    ch = roofline_entry(
        "k_cheb_step: one step of the Chebyshev recurrence on the FP16 B (the last one forms z and rho "
        "partials); every launch of the timed solve",
        ch_bytes, info["cheb_ms"], info["cheb_launches"],
        stored_traffic(TRAFFIC_FILES[(workload, "k_cheb_step")]), ph)
    return ch, sp


# ----------------------------------------------------------------------------
# the library's stream probes (ceiling reference, counter scaling)
# ----------------------------------------------------------------------------

def stream_probe(torch, dev, mode, mib, reps=5):
    from paper_2505_04155_amd import binding
    L = binding.load()
    nbytes = mib * 1024 * 1024
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src) if mode == 1 else torch.zeros(4, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)

    def launch():
        binding.check(L.amp_stream_probe(mode, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                         nbytes, sp), "amp_stream_probe")
    launch()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        launch()
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    moved = nbytes * (2 if mode == 1 else 1)
    del src, dst
    return {"kernel": "k_stream_copy" if mode == 1 else "k_stream_read", "bytes": moved,
            "avg_us": round(us, 3), "GB/s": round(moved / us / 1e3, 1)}


def probes(torch, dev):
    return {"read_4GiB": stream_probe(torch, dev, 0, 4096, reps=3),
            "copy_4GiB": stream_probe(torch, dev, 1, 4096, reps=3),
            "copy_256MiB": stream_probe(torch, dev, 1, 256)}


# ----------------------------------------------------------------------------
# timing
# ----------------------------------------------------------------------------

def time_presets(amp, torch, M, pc, bt, presets, steps, warmup, tol, maxit):
    results = {}
    for preset in presets:
        def run():
            x, info = amp.solve(M, pc, bt, tol=tol, maxit=maxit, preset=preset)
            if info["status"] != 0:
                raise RuntimeError(f"{preset} solve failed: {info}")
            return x, info
        for w in range(warmup):
            run()
            log(f"bench: warmup {preset} {w + 1}/{warmup} done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            x, info = run()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        results[preset] = (ms, info, x)
        log(f"bench: {preset}: {ms:.3f} ms/solve, {info['iters']} iterations, "
            f"switches z32={info['k_z32']} z16={info['k_z16']} r32={info['k_r32']}")
    return results


def oracle_threads():
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return n


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def golden_q1():
    fields = {}
    with open(Q1_GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, _, v = line.partition(" ")
                fields[k] = float(v)
    return fields


def q1_cpu_baseline(A, b, lo, hi, oracle_iters, k1=2, k2=12):
    """The FP64 oracle (Alg. 1 with the same degree-4 Chebyshev definition,
    FP64 throughout) on the same system, timed for k1 and k2 iterations; the
    per-iteration slope times the oracle's full iteration count plus the
    k1-run's fixed part gives the full solve's time."""
    from oracle import cpcg
    threads = oracle_threads()
    cpcg.lib().oracle_set_threads(threads)
    t = {}
    for k in (k1, k2):
        t0 = time.perf_counter()
        cpcg.pcg(A, b, tol=1e-10, maxit=k, precond=cpcg.PC_CHEBYSHEV, degree=4, lam_lo=lo, lam_hi=hi)
        t[k] = (time.perf_counter() - t0) * 1e3
        log(f"bench: CPU oracle, {k} iterations: {t[k]:.0f} ms ({threads} threads)")
    per_it = (t[k2] - t[k1]) / (k2 - k1)
    total = t[k1] + per_it * (oracle_iters - k1)
    return {"value": round(total, 1), "unit": "ms", "cores": threads, "kind": "oracle",
            "sample": f"FP64 PCG (Alg. 1) with the degree-4 Chebyshev preconditioner on the same 256^3 system, "
                      f"timed for {k1} and {k2} iterations ({t[k1]:.0f} and {t[k2]:.0f} ms); the per-iteration "
                      f"slope scaled to the oracle's {oracle_iters} iterations to convergence",
            "ms_per_iteration": round(per_it, 2), "cpu_model": cpu_model()}


# the paper's per-kernel times of Ax for Ex. jac libp (A100, 21.7e6 unknowns,
# Fig. fig:performance_runtime), microseconds: context only
PAPER_AX_US = {"p64_q64": 1804.797, "p16_q64": 1685.107, "p16_q32": 812.908}
FP64_VECTOR_PEAK = 78.6e12
FP32_VECTOR_PEAK = 157.3e12


def hex_measurement(amp, torch, np, P, dev, reps=20, E=(40, 40, 40), order=7, solve=True):
    """The matrix-free order-7 hexahedral operator of Ex. jac libp on the
    paper's 40^3-element mesh (trilinear elements, vertices perturbed by
    0.2 h): each phase's storage/arithmetic pair timed over `reps` applies
    (zero fill of q, the element kernel, the mu sum) with HIP events on the
    launching stream, against the chip's vector peak of the arithmetic."""
    V = P.hex_vertices(E, 0.2, 0)
    H = amp.HexOperator(torch.tensor(V, device=dev), E, order=order, lam=1e3)
    rng = np.random.default_rng(84)
    p64 = torch.tensor(rng.standard_normal(H.n), device=dev)
    flops = H.flops_per_element * H.elements
    out = {"workload": f"screened Poisson -Laplace u + 1e3 u, order {order}, {E[0]}x{E[1]}x{E[2]} trilinear "
                       f"hexahedra of [-0.5,0.5]^3 (interior vertices moved by 0.2 h), n={H.n}, "
                       f"{H.local} local nodes, geometric factors formed per quadrature point",
           "flops_per_element": H.flops_per_element, "phases": {}}
    stream = torch.cuda.current_stream()
    for name, up, ur in (("p64_q64", 64, 64), ("p16_q64", 16, 64), ("p16_q32", 16, 32)):
        p = p64.to({64: torch.float64, 16: torch.float16}[up])
        H.apply(p, u_r=ur)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            H.apply(p, u_r=ur)
        e1.record(stream)
        e1.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        peak = FP64_VECTOR_PEAK if ur == 64 else FP32_VECTOR_PEAK
        # algorithmic bytes: p read once (its storage), q written once (u_r)
        nbytes = H.n * (up // 8 + ur // 8)
        out["phases"][name] = {
            "us_per_apply": round(us, 2),
            "roofline": {"bound": "alu", "achieved": round(flops / (us * 1e-6) / 1e12, 2), "peak": peak / 1e12,
                         "unit": "TFLOP/s", "frac": round(flops / (us * 1e-6) / peak, 4),
                         "algorithmic_GB_per_s": round(nbytes / (us * 1e-6) / 1e9, 1)},
            "paper_a100_us": PAPER_AX_US[name],
        }
        log(f"bench: hex Ax {name}: {us:.1f} us per apply, {flops / (us * 1e-6) / 1e12:.2f} TFLOP/s")
    if solve:
        # Jacobi-PCG on the operator (the paper's Ex. jac libp): FP64 PCG and
        # AMP-PCG(FP16) with the delay and the linear u_r criterion
        M = amp.Matrix.from_hexop(H)
        pc = amp.Preconditioner(M, "jacobi")
        b = torch.tensor(np.random.default_rng(86).standard_normal(H.n), device=dev)
        runs = {}
        for name, preset, kw in (("pcg64", "pcg64", {}), ("amp16", "amp16", {}),
                                 ("amp16_linear", "amp16", {"eta": "linear"})):
            amp.solve(M, pc, b, tol=1e-10, maxit=20000, preset=preset, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x, info = amp.solve(M, pc, b, tol=1e-10, maxit=20000, preset=preset, **kw)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            ti = amp.solve(M, pc, b, tol=1e-10, maxit=20000, preset=preset, spmv_timing=1, **kw)[1]
            runs[name] = {"ms": round(ms, 2), "iters": info["iters"], "k_r32": info["k_r32"],
                          "rel_res_true": info["relres_true"],
                          "product_us": round(ti["spmv_ms"] * 1e3 / max(1, ti["spmv_launches"]), 2)}
            log(f"bench: matrix-free solve {name}: {ms:.1f} ms, {info['iters']} iterations, "
                f"u_r FP32 from {info['k_r32']}")
        runs["speedup_amp16_vs_fp64_pcg"] = round(runs["pcg64"]["ms"] / runs["amp16"]["ms"], 4)
        runs["speedup_amp16_linear_vs_fp64_pcg"] = round(runs["pcg64"]["ms"] / runs["amp16_linear"]["ms"], 4)
        out["solve"] = runs
    return out


def pmg_measurement(amp, torch, np, P, dev, E=(30, 30, 30), order=7, reps=10):
    """The Poisson problem of Ex. linear conv2 (order 7 on 30^3 trilinear
    hexahedra of [-0.5, 0.5]^3, interior vertices moved by 0.2 h in place of
    the Kershaw mesh, homogeneous Dirichlet) with the p-multigrid V-cycle
    (orders 7, 3, 1; degree-2 Chebyshev-Jacobi smoothing; a degree-16
    Chebyshev-Jacobi polynomial on order 1 in place of algebraic multigrid):
    FP64 PCG against AMP-PCG(FP16) with z and p in FP16 from the first
    iteration (the linear and the delay u_r criteria), the cycle's cost in
    FP64 and FP32, and Jacobi-PCG on the same system for reference."""
    V = P.hex_vertices(E, 0.2, 0)
    H = amp.HexOperator(torch.tensor(V, device=dev), E, order=order, lam=0.0)
    M = amp.Matrix.from_hexop(H)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pc = amp.Preconditioner.pmg(M)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    pi = pc.pmg_info()
    b = torch.tensor(P.pmg_poisson_rhs(E, order), device=dev)
    out = {"workload": f"Poisson -Laplace u = 1 + 3 pi^2 sin(pi x) sin(pi y) sin(pi z), order {order}, "
                       f"{E[0]}x{E[1]}x{E[2]} trilinear hexahedra of [-0.5,0.5]^3 (interior vertices moved by "
                       f"0.2 h), n={H.n}; p-multigrid V-cycle over orders {pi['orders']} (degree-2 "
                       f"Chebyshev-Jacobi smoothing, degree-16 Chebyshev-Jacobi polynomial on the lowest order), "
                       f"tol 1e-10",
           "levels_n": pi["n"], "rho": [round(r, 6) for r in pi["rho"]], "gain": pi["gain"],
           "setup_ms": round(setup_ms, 1), "preconditioner_bytes": pi["bytes"]}
    stream = torch.cuda.current_stream()
    r = torch.tensor(np.random.default_rng(87).standard_normal(H.n), device=dev)
    cyc = {}
    for prec in (64, 32):
        pc.pmg_apply(r, prec)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            pc.pmg_apply(r, prec)
        e1.record(stream)
        e1.synchronize()
        cyc[f"fp{prec}_us"] = round(e0.elapsed_time(e1) * 1e3 / reps, 1)
    out["cycle"] = cyc
    log(f"bench: pMG cycle FP64 {cyc['fp64_us']} us, FP32 {cyc['fp32_us']} us")
    runs, sol = {}, {}
    for name, preset, kw in (("pcg64", "pcg64", {}), ("amp16_linear", "amp16", {"eta": "linear"}),
                             ("amp16", "amp16", {}), ("amp16_r64", "amp16", {"eta": "fixed64"}),
                             ("amp32", "amp16", {"u0": 32}), ("amp64", "amp64", {})):
        amp.solve(M, pc, b, tol=1e-10, maxit=2000, preset=preset, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = amp.solve(M, pc, b, tol=1e-10, maxit=2000, preset=preset, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        sol[name] = x
        runs[name] = {"ms": round(ms, 2), "iters": info["iters"], "k_z16": info["k_z16"], "k_r32": info["k_r32"],
                      "rel_res_true": info["relres_true"], "status": info["status"]}
        log(f"bench: pMG solve {name}: {ms:.1f} ms, {info['iters']} iterations, u_z FP16 from {info['k_z16']}, "
            f"u_r FP32 from {info['k_r32']}")
    xr = sol["pcg64"]
    for name in ("amp16_linear", "amp16", "amp16_r64", "amp32", "amp64"):
        runs[name]["rel_diff_vs_pcg64"] = float(torch.linalg.norm(sol[name] - xr) / torch.linalg.norm(xr))
        runs[f"speedup_{name}_vs_fp64_pcg"] = round(runs["pcg64"]["ms"] / runs[name]["ms"], 4)
    pj = amp.Preconditioner(M, "jacobi")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, ij = amp.solve(M, pj, b, tol=1e-10, maxit=20000, preset="pcg64")
    torch.cuda.synchronize()
    runs["jacobi_pcg64"] = {"ms": round((time.perf_counter() - t0) * 1e3, 2), "iters": ij["iters"]}
    log(f"bench: Jacobi-PCG(FP64) on the same system: {runs['jacobi_pcg64']['ms']} ms, {ij['iters']} iterations")
    out["solve"] = runs
    return out


def fv128_measurement(amp, torch, np, P, dev, steps, warmup, with_oracle=True, grid=128):
    """The 128^3 blocky finite-volume workload (Jacobi): time per preset,
    product-kernel roofline, error against the oracle's solution."""
    log(f"bench: generating the {grid}^3 finite-volume system")
    A, b, _ = P.blocky_diffusion3d_system(grid, 8)
    M = amp.Matrix.from_csr(A, device=dev)
    pc = amp.Preconditioner(M, "jacobi")
    bt = torch.tensor(b, device=dev)
    info_m = M.info()
    tol, maxit = 1e-10, 20000
    res = time_presets(amp, torch, M, pc, bt, ("amp16", "pcg64"), steps, warmup, tol, maxit)
    info = timed_solve(amp, M, pc, bt, "amp16", tol, maxit)
    sp, _ = rooflines(info, info_m, "fv128")
    out = {"workload": f"3-D 7-point FV diffusion {grid}^3, coefficients 10^U(0,4) on 8^3 blocks, "
                       f"N={info_m['n']}, nnz={info_m['nnz']}, Jacobi, tol 1e-10, b ~ N(0,1)",
           "amp16_ms": round(res["amp16"][0], 3), "pcg64_ms": round(res["pcg64"][0], 3),
           "speedup_vs_fp64_pcg": round(res["pcg64"][0] / res["amp16"][0], 4),
           "amp16_iters": res["amp16"][1]["iters"], "pcg64_iters": res["pcg64"][1]["iters"],
           "roofline": sp}
    if with_oracle:
        from oracle import cpcg
        cpcg.lib().oracle_set_threads(oracle_threads())
        t0 = time.perf_counter()
        xo, io = cpcg.pcg(A, b, tol=tol, maxit=maxit)
        out["oracle_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
        out["oracle_iters"] = io["iters"]
        xon = float(np.linalg.norm(xo))
        out["rel_err_vs_oracle"] = {p: float(np.linalg.norm(r[2].cpu().numpy() - xo) / xon) for p, r in res.items()}
        log(f"bench: 128^3 relative error against the oracle's solution: {out['rel_err_vs_oracle']}")
    return out


def batched_measurement(amp, torch, np, P, dev, steps, warmup):
    """The 512-system batched workload (2-D five-point FV, sides log-uniform
    in [32, 512], kappa = exp(N(0, 1.5^2)) per cell, Jacobi): batched
    time-to-solution per preset and the aggregate algorithmic bandwidth
    (every system's iterations priced at their precisions)."""
    log("bench: generating the 512-system batched workload")
    systems = P.batched_systems()
    Ms = [amp.Matrix.from_csr(A, device=dev) for A, _ in systems]
    Ps = [amp.Preconditioner(M, "jacobi") for M in Ms]
    bs = [torch.tensor(b, device=dev) for _, b in systems]
    infos_m = [M.info() for M in Ms]
    out = {"workload": f"{len(systems)} 2-D 5-point FV systems, sides round(exp(U[ln 32, ln 512])), "
                       f"kappa = exp(N(0, 1.5^2)) per cell, b ~ N(0,1), Jacobi, tol 1e-10 each; "
                       f"{sum(A.n for A, _ in systems)} rows in all"}
    for preset in ("amp16", "amp64", "pcg64"):
        for _ in range(warmup):
            amp.solve_batched(Ms, Ps, bs, tol=1e-10, maxit=20000, preset=preset)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            xs, infos, st = amp.solve_batched(Ms, Ps, bs, tol=1e-10, maxit=20000, preset=preset)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        if st != 0:
            raise RuntimeError(f"batched {preset}: status {st}")
        nbytes = 0
        for im, inf in zip(infos_m, infos):
            for (uz, ur), k in phase_iterations(inf, preset).items():
                nbytes += k * jacobi_iteration_bytes(im["n"], im["nnz"], im["meta_bytes"], uz, ur)
        iters = [i["iters"] for i in infos]
        out[preset] = {"ms": round(ms, 2), "algorithmic_GB": round(nbytes / 1e9, 2),
                       "aggregate_GB_per_s": round(nbytes / (ms * 1e-3) / 1e9, 1),
                       "iters_min_median_max": [int(min(iters)), int(np.median(iters)), int(max(iters))],
                       "max_rel_res_true": max(i["relres_true"] for i in infos)}
        log(f"bench: batched {preset}: {ms:.1f} ms, {out[preset]['aggregate_GB_per_s']:.0f} GB/s aggregate")
    out["speedup_amp16_vs_fp64_pcg"] = round(out["pcg64"]["ms"] / out["amp16"]["ms"], 4)
    out["speedup_amp64_vs_fp64_pcg"] = round(out["pcg64"]["ms"] / out["amp64"]["ms"], 4)
    return out


# ----------------------------------------------------------------------------

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--preset", default="amp16")
    ap.add_argument("--q1-grid", type=int, default=256, help="interior nodes per direction of the Q1 workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 128^3 finite-volume measurement")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-system batched measurement")
    ap.add_argument("--no-hex", action="store_true", help="skip the matrix-free hexahedral operator measurement")
    ap.add_argument("--no-pmg", action="store_true", help="skip the p-multigrid Poisson measurement")
    ap.add_argument("--no-oracle-solution", action="store_true",
                    help="skip the oracle's full solve of the Q1 system (the exact errors against it)")
    ap.add_argument("--mode", choices=["solve", "roofline", "fv128", "batched", "hex", "pmg"], default="solve",
                    help="roofline: only the timed solve and the stream probes (for profiler runs); "
                         "fv128: the 128^3 finite-volume workload alone; batched: the 512-system workload alone; "
                         "hex: the matrix-free order-7 hexahedral operator alone")
    ap.add_argument("--workload", choices=["q1", "fv128"], default="q1", help="workload of --mode roofline")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU only; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2505_04155_amd as amp
    from paper_2505_04155_amd import binding
    from workloads import problems as P

    binding.load(build_if_missing=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tol, maxit = 1e-10, 20000

    if args.mode == "fv128":
        print(json.dumps(fv128_measurement(amp, torch, np, P, dev, args.steps, args.warmup)), flush=True)
        return
    if args.mode == "batched":
        print(json.dumps(batched_measurement(amp, torch, np, P, dev, args.steps, args.warmup)), flush=True)
        return
    if args.mode == "hex":
        print(json.dumps({"mode": "hex", **hex_measurement(amp, torch, np, P, dev)}), flush=True)
        return
    if args.mode == "pmg":
        print(json.dumps({"mode": "pmg", **pmg_measurement(amp, torch, np, P, dev)}), flush=True)
        return
    if args.mode == "roofline" and args.workload == "fv128":
        A, b, _ = P.blocky_diffusion3d_system(128, 8)
        M = amp.Matrix.from_csr(A, device=dev)
        pc = amp.Preconditioner(M, "jacobi")
        bt = torch.tensor(b, device=dev)
        amp.solve(M, pc, bt, tol=tol, maxit=maxit, preset=args.preset)
        info = timed_solve(amp, M, pc, bt, args.preset, tol, maxit)
        sp, _ = rooflines(info, M.info(), "fv128")
        pr = {"copy_256MiB": stream_probe(torch, dev, 1, 256)}
        log(f"bench: product step {sp['avg_kernel_us']:.2f} us, {sp['achieved']:.0f} GB/s")
        print(json.dumps({"mode": "roofline", "workload": "fv128", "roofline": sp, "probes": pr}), flush=True)
        return

    m = args.q1_grid
    log(f"bench: generating the Q1 {m}^3 system")
    t0 = time.perf_counter()
    A, b, xs, (lo, hi) = P.q1_system(m)
    log(f"bench: generated in {time.perf_counter() - t0:.1f} s; uploading")
    M = amp.Matrix.from_csr(A, device=dev)
    pc = amp.Preconditioner(M, "chebyshev", degree=4, lam_lo=lo, lam_hi=hi)
    bt = torch.tensor(b, device=dev)
    info_m = M.info()
    n, nnz = info_m["n"], info_m["nnz"]
    workload = (f"Q1 trilinear FEM, anisotropic diffusion diag(1, 1e-2, 1e-3), {m}^3 interior nodes, N={n}, "
                f"nnz={nnz}, degree-4 Chebyshev preconditioner (FP16 B) on [lam_min, 1.05 lam_max] of D^-1 A, "
                f"x* ~ U[-1,1], b = A x*, tol 1e-10")

    if args.mode == "roofline":
        amp.solve(M, pc, bt, tol=tol, maxit=maxit, preset=args.preset)   # warm the handle
        info = timed_solve(amp, M, pc, bt, args.preset, tol, maxit)
        ch, sp = rooflines(info, info_m, "q1", degree=4)
        pr = probes(torch, dev)
        log(f"bench: Chebyshev step {ch['avg_kernel_us']:.1f} us ({ch['achieved']:.0f} GB/s), product "
            f"{sp['avg_kernel_us']:.1f} us ({sp['achieved']:.0f} GB/s); read probe {pr['read_4GiB']['GB/s']:.0f}, "
            f"copy probe {pr['copy_4GiB']['GB/s']:.0f} GB/s")
        print(json.dumps({"mode": "roofline", "workload": workload, "roofline": ch, "roofline_k_spmv": sp,
                          "probes": pr, "matrix": info_m}), flush=True)
        return

    presets = [args.preset] + [p for p in ("amp64", "pcg64") if p != args.preset]
    results = time_presets(amp, torch, M, pc, bt, presets, args.steps, args.warmup, tol, maxit)
    gold = golden_q1() if m == 256 else None
    xsn = float(np.linalg.norm(xs))
    err_xs = {p: float(np.linalg.norm(r[2].cpu().numpy() - xs) / xsn) for p, r in results.items()}
    log(f"bench: relative error against x*: {err_xs}")
    err_or = None
    if gold:
        # ||x - x_o|| <= ||x - x*|| + ||x_o - x*|| and ||x_o|| >= ||x*|| (1 - e_o)
        eo = gold["err_vs_xstar"]
        err_or = {p: (e + eo) / (1.0 - eo) for p, e in err_xs.items()}

    amp_ms, amp_info, _ = results[args.preset]
    fp64_ms, fp64_info, _ = results["pcg64"]

    info = timed_solve(amp, M, pc, bt, args.preset, tol, maxit)
    ch, sp = rooflines(info, info_m, "q1", degree=4)
    log(f"bench: Chebyshev step in the solve: {ch['avg_kernel_us']:.1f} us, {ch['achieved']:.0f} GB/s "
        f"({100 * ch['frac']:.1f}% of {HBM_PEAK_GBS:.0f}); product step {sp['avg_kernel_us']:.1f} us, "
        f"{sp['achieved']:.0f} GB/s")
    pr = probes(torch, dev)
    log(f"bench: stream probes: read {pr['read_4GiB']['GB/s']:.0f} GB/s, copy {pr['copy_4GiB']['GB/s']:.0f} GB/s")

    cpu = None
    if not args.no_cpu_baseline and gold:
        cpu = q1_cpu_baseline(A, b, lo, hi, int(gold["iters"]))
        log(f"bench: CPU oracle (scaled sample) {cpu['value']:.0f} ms")
    oracle = None
    if not args.no_oracle_solution:
        # the oracle's own solution of the same system, for the error of
        # every timed solve against it
        from oracle import cpcg
        cpcg.lib().oracle_set_threads(oracle_threads())
        log("bench: CPU oracle, full solve for the parity figures")
        t0 = time.perf_counter()
        xo, io = cpcg.pcg(A, b, tol=tol, maxit=maxit, precond=cpcg.PC_CHEBYSHEV, degree=4, lam_lo=lo, lam_hi=hi)
        oms = (time.perf_counter() - t0) * 1e3
        xon = float(np.linalg.norm(xo))
        oracle = {"iters": io["iters"], "ms": round(oms, 1), "threads": oracle_threads(),
                  "rel_res_true": io["relres_true"],
                  "rel_err_vs_xstar": float(np.linalg.norm(xo - xs) / xsn),
                  "rel_err_vs_oracle": {p: float(np.linalg.norm(r[2].cpu().numpy() - xo) / xon)
                                        for p, r in results.items()}}
        log(f"bench: oracle {io['iters']} iterations in {oms:.0f} ms; relative error against its solution: "
            f"{oracle['rel_err_vs_oracle']}")

    del A
    secondary = None
    if not args.no_secondary:
        del M, pc, bt
        torch.cuda.empty_cache()
        secondary = fv128_measurement(amp, torch, np, P, dev, args.steps, args.warmup,
                                      with_oracle=not args.no_cpu_baseline)
    batched = None
    if not args.no_batched:
        torch.cuda.empty_cache()
        batched = batched_measurement(amp, torch, np, P, dev, 1, 1)
    hexop = None
    if not args.no_hex:
        torch.cuda.empty_cache()
        hexop = hex_measurement(amp, torch, np, P, dev)
    pmg = None
    if not args.no_pmg:
        log("bench: p-multigrid Poisson problem")
        pmg = pmg_measurement(amp, torch, np, P, dev)

    out = {
        "metric": METRIC,
        "value": round(amp_ms, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(amp_ms, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64+f32+f16",
        "data": "synthetic",
        "config": {"workload": workload, "preset": args.preset, "parallelism": "single GPU"},
        "fp64_pcg_ms": round(fp64_ms, 3),
        "fp64_pcg_note": "PCG(FP64): every vector and scalar FP64, the same preconditioner (Chebyshev "
                         "polynomial in FP64 arithmetic on the FP16-stored B)",
        "speedup_vs_fp64_pcg": round(fp64_ms / amp_ms, 4),
        "amp64_ms": round(results["amp64"][0], 3),
        "speedup_amp64_vs_fp64_pcg": round(fp64_ms / results["amp64"][0], 4),
        "iters": {p: r[1]["iters"] for p, r in results.items()},
        "oracle_iters": int(gold["iters"]) if gold else None,
        "switch_iterations": {p: {"u_z_fp32": r[1]["k_z32"], "u_z_fp16": r[1]["k_z16"], "u_r_fp32": r[1]["k_r32"]}
                              for p, r in results.items()},
        "rel_res_true": {p: r[1]["relres_true"] for p, r in results.items()},
        "rel_err_vs_xstar": err_xs,
        "rel_err_vs_oracle": oracle["rel_err_vs_oracle"] if oracle else None,
        "rel_err_vs_oracle_bound": err_or,
        "oracle_solve": oracle,
        "roofline": ch,
        "roofline_k_spmv": sp,
        "probes": pr,
        "cpu_baseline": cpu,
        "secondary_fv128": secondary,
        "secondary_batched": batched,
        "secondary_hex_ax": hexop,
        "secondary_pmg": pmg,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
