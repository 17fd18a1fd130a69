#!/usr/bin/env python3
"""Time-to-solution of AMP-PCG versus FP64 PCG on one MI355X.

A step is one complete solve (all kernels of the hot path, from r0 = b - A x0
to the verified solution) of the 3-D 7-point finite-volume diffusion system
on a 128^3 grid with block coefficients 10^U, U ~ U[0, 4] on 8^3 blocks
(N = 2,097,152, nnz = 14,581,760), Jacobi preconditioner, tol 1e-10.
Inputs are resident in HBM before the timed region starts.

Prints one JSON line: value = AMP-PCG(FP16) time-to-solution (ms, lower is
better; the variant the paper times: z and p in FP16 from the start, r and q
switching FP64 -> FP32 by the delay criterion); the stepwise AMP-PCG(FP64)
time, the FP64 PCG time on the same GPU, the speedups, the iteration
counts, the HBM roofline of the dominant kernel (the product step, timed
with HIP events carried by each of its launches inside the AMP-PCG solve),
and the FP64 CPU oracle timed on the host are reported beside it.

Modes: --mode roofline runs only the timed-product solve (and a 256 MiB
device copy of known size): the command the kernel trace and the HBM
counter runs profile.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time-to-solution at rel. residual 1e-10, AMP-PCG vs FP64 PCG; SpMV HBM GB/s"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_spmv_fv3d128_hbm_counters.txt")
Q1_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_spmv_q1_256_hbm_counters.txt")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def step_bytes(n, nnz, meta_bytes, u_z, u_r):
    """Algorithmic bytes of one product step p = z + beta p_old, q = A p in
    precisions (u_z, u_r): every nonzero's value once (FP64 plane for
    u_r = 64, FP32 plane otherwise), the layout's column metadata once (int32
    indices of index-mode slices, the shared offset lists, 12 B per slice),
    z and p_old read once (gathers counted once), p and q written once.
    Slice padding is overhead, not counted."""
    b_val = 8 if u_r == 64 else 4
    return nnz * b_val + meta_bytes + n * (3 * (u_z // 8) + u_r // 8)


def stored_traffic(path=None):
    """HBM bytes per product launch from the committed FETCH_SIZE / WRITE_SIZE
    summary (each counter scaled by what it reads for a plain copy of known
    size), or None when the summary is missing or was taken on other kernel
    sources than the library built here."""
    from paper_2505_04155_amd import build
    try:
        fields = {}
        with open(path or TRAFFIC_FILE) as f:
            for line in f:
                if line.strip() and not line.startswith("#"):
                    key, _, val = line.partition(" ")
                    fields[key] = val.strip()
    except OSError:
        return None
    if fields.get("source_digest") != build.source_digest():
        return None
    return int(float(fields["traffic_bytes_per_launch"]))


def roofline(amp, M, pc, bt, info_m, preset, tol, maxit, traffic_file=None):
    """One AMP-PCG solve with the library timing every product launch (HIP
    events carried by the launch's own dispatch on the solve's stream);
    achieved = algorithmic bytes of the launches that performed an
    iteration, summed per iteration from the recorded precisions, / their
    summed duration."""
    x, info = amp.solve(M, pc, bt, tol=tol, maxit=maxit, preset=preset, history=True, spmv_timing=1)
    if info["status"] != 0:
        raise RuntimeError(f"timed solve failed: {info}")
    n, nnz, meta = info_m["n"], info_m["nnz"], info_m["meta_bytes"]
    total = sum(step_bytes(n, nnz, meta, uz, ur) for uz, ur in zip(info["uz"], info["ur"]))
    launches = info["spmv_launches"]
    us = info["spmv_ms"] * 1e3 / launches
    gbs = total / (info["spmv_ms"] * 1e-3) / 1e9
    phases = {}
    for uz, ur in zip(info["uz"], info["ur"]):
        phases[f"z{uz}_r{ur}"] = phases.get(f"z{uz}_r{ur}", 0) + 1
    return {
        "bound": "hbm",
        "kernel": f"k_spmv: p = z + beta p_old (u_z), q = A p (u_r), gamma partials; every launch of one "
                  f"{preset} solve, all precision phases",
        "achieved": round(gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(gbs / HBM_PEAK_GBS, 4),
        "traffic": stored_traffic(traffic_file),
        "avg_kernel_us": round(us, 3),
        "launches": launches,
        "algorithmic_bytes_per_launch": round(total / launches),
        "phase_iterations": phases,
    }


def warm_step(binding, M, torch, info_m, reps=50):
    """The product step of the FP16/FP32 phase launched back to back on the
    same data (which then stays in the 256 MB last-level cache): a
    cache-resident figure, reported beside the in-solve roofline."""
    import ctypes
    L = binding.load()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    for _ in range(3):
        binding.check(L.amp_spmv_step(M.handle, 16, 32, 1, 0.5, sp), "amp_spmv_step")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        L.amp_spmv_step(M.handle, 16, 32, 1, 0.5, sp)
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    nb = step_bytes(info_m["n"], info_m["nnz"], info_m["meta_bytes"], 16, 32)
    return {"kernel": "k_spmv_fixed<16,32,true>", "avg_us": round(us, 3), "GB/s": round(nb / us / 1e3, 1)}


def copy_reference(torch, dev, reps=5, mib=256):
    """A plain device copy of `mib` MiB (read and write that much).  The
    256 MiB copy is the launch a counter run scales FETCH_SIZE / WRITE_SIZE
    by; a 4 GiB copy, far beyond the 256 MB memory-side cache, gives the
    streaming rate of HBM itself."""
    stream = torch.cuda.current_stream()
    src = torch.empty(mib * 1024 * 1024 // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    return {"bytes": 2 * src.numel() * 4, "avg_us": round(us, 3), "GB/s": round(2 * src.numel() * 4 / us / 1e3, 1)}


def q1_mode(args, amp, torch, np, P, dev, tol=1e-10, maxit=20000):
    """The anisotropic Q1 stiffness workload (27-point, 256^3 interior nodes,
    x* ~ U[-1, 1], b = A x*) with the degree-4 Chebyshev preconditioner: one
    timed solve per preset after a warm-up, the in-solve product roofline,
    and the reference copy a counter run scales by.  One JSON line."""
    m = args.q1_grid
    log(f"bench: generating the Q1 {m}^3 system")
    A, b, xs, (lo, hi) = P.q1_system(m)
    M = amp.Matrix.from_csr(A, device=dev)
    pc = amp.Preconditioner(M, "chebyshev", degree=4, lam_lo=lo, lam_hi=hi)
    bt = torch.tensor(b, device=dev)
    info_m = M.info()
    n, nnz = A.n, A.nnz
    del A
    out = {"mode": "q1", "workload": f"Q1 anisotropic diffusion (1, 1e-2, 1e-3), {m}^3 interior nodes, N={n}, "
                                     f"nnz={nnz}, degree-4 Chebyshev on [lam_lo, 1.05 lam_hi], tol {tol}"}
    xsn = float(np.linalg.norm(xs))
    for preset in (args.preset, "pcg64"):
        amp.solve(M, pc, bt, tol=tol, maxit=maxit, preset=preset)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = amp.solve(M, pc, bt, tol=tol, maxit=maxit, preset=preset)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        if info["status"] != 0:
            raise RuntimeError(f"{preset} solve failed: {info}")
        err = float(np.linalg.norm(x.cpu().numpy() - xs) / xsn)
        out[preset] = {"ms": round(ms, 3), "iters": info["iters"], "rel_res_true": info["relres_true"],
                       "rel_err_vs_xstar": err,
                       "switch_iterations": [info["k_z32"], info["k_z16"], info["k_r32"]]}
        log(f"bench: Q1 {preset}: {ms:.1f} ms, {info['iters']} iterations, error vs x* {err:.2e}")
    out["speedup_vs_fp64_pcg"] = round(out["pcg64"]["ms"] / out[args.preset]["ms"], 4)
    out["roofline"] = roofline(amp, M, pc, bt, info_m, args.preset, tol, maxit, traffic_file=Q1_TRAFFIC_FILE)
    log(f"bench: Q1 product step in the solve: {out['roofline']['avg_kernel_us']:.1f} us, "
        f"{out['roofline']['achieved']:.0f} GB/s")
    out["copy_256MiB"] = copy_reference(torch, dev)
    out["matrix"] = info_m
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--preset", default="amp16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["solve", "roofline", "q1"], default="solve",
                    help="roofline: only the timed-product solve and the reference copy (for profiler runs); "
                         "q1: the anisotropic Q1 workload with the degree-4 Chebyshev preconditioner")
    ap.add_argument("--q1-grid", type=int, default=256, help="interior nodes per direction of the Q1 workload")
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

    if args.mode == "q1":
        q1_mode(args, amp, torch, np, P, dev)
        return

    log(f"bench: generating the {args.grid}^3 system")
    A, b, _ = P.blocky_diffusion3d_system(args.grid, 8)
    M = amp.Matrix.from_csr(A, device=dev)
    pc = amp.Preconditioner(M, "jacobi")
    bt = torch.tensor(b, device=dev)
    info_m = M.info()
    n, nnz = info_m["n"], info_m["nnz"]
    tol, maxit = 1e-10, 20000

    if args.mode == "roofline":
        amp.solve(M, pc, bt, tol=tol, maxit=maxit, preset=args.preset)        # warm the handle
        rf = roofline(amp, M, pc, bt, info_m, args.preset, tol, maxit)
        cp = copy_reference(torch, dev)
        cp4 = copy_reference(torch, dev, reps=3, mib=4096)
        log(f"bench: product step in the solve: {rf['avg_kernel_us']:.2f} us average over {rf['launches']} "
            f"launches, {rf['achieved']:.0f} GB/s; copy 256 MiB {cp['GB/s']:.0f} GB/s, 4 GiB {cp4['GB/s']:.0f} GB/s")
        print(json.dumps({"mode": "roofline", "roofline": rf, "copy_256MiB": cp, "copy_4GiB": cp4, "matrix": info_m}),
              flush=True)
        return

    def run(preset):
        x, info = amp.solve(M, pc, bt, tol=tol, maxit=maxit, preset=preset)
        if info["status"] != 0:
            raise RuntimeError(f"{preset} solve failed: {info}")
        return x, info

    results = {}
    presets = [args.preset] + [p for p in ("amp64", "pcg64") if p != args.preset]
    for preset in presets:
        for w in range(args.warmup):
            run(preset)
            log(f"bench: warmup {preset} {w + 1}/{args.warmup} done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for s in range(args.steps):
            x, info = run(preset)
            infos.append(info)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms = (t1 - t0) * 1e3 / args.steps
        results[preset] = (ms, infos[-1], x)
        log(f"bench: {preset}: {ms:.3f} ms/solve, {infos[-1]['iters']} iterations, "
            f"switches z32={infos[-1]['k_z32']} z16={infos[-1]['k_z16']} r32={infos[-1]['k_r32']}")

    amp_ms, amp_info, _ = results[args.preset]
    fp64_ms, fp64_info, _ = results["pcg64"]

    # Dominant kernel: the product step, timed inside an AMP-PCG solve.
    rf = roofline(amp, M, pc, bt, info_m, args.preset, tol, maxit)
    log(f"bench: product step in the solve: {rf['avg_kernel_us']:.2f} us average over {rf['launches']} launches, "
        f"{rf['achieved']:.0f} GB/s algorithmic ({100 * rf['frac']:.1f}% of {HBM_PEAK_GBS:.0f})")
    warm = warm_step(binding, M, torch, info_m)
    log(f"bench: FP16/FP32 product step back to back (cache-resident): {warm['avg_us']:.2f} us, "
        f"{warm['GB/s']:.0f} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import cpcg
        threads = len(os.sched_getaffinity(0))
        cpcg.lib().oracle_set_threads(threads)
        log(f"bench: CPU oracle (FP64 PCG, {threads} threads)")
        t0 = time.perf_counter()
        xo, io = cpcg.pcg(A, b, tol=tol, maxit=maxit)
        t1 = time.perf_counter()
        cpu = {"value": round((t1 - t0) * 1e3, 3), "unit": "ms", "cores": threads, "kind": "oracle",
               "sample": f"one full FP64 PCG solve (Alg. 1, Jacobi) of the same system: "
                         f"{io['iters']} iterations"}
        log(f"bench: CPU oracle {cpu['value']:.1f} ms, {io['iters']} iterations")
        # every timed solve's final iterate against the oracle's (both stop at tol 1e-10)
        xon = float(np.linalg.norm(xo))
        cpu["oracle_iters"] = io["iters"]
        cpu["rel_err_vs_oracle"] = {p: float(np.linalg.norm(r[2].cpu().numpy() - xo) / xon) for p, r in results.items()}
        log(f"bench: relative error against the oracle's solution: {cpu['rel_err_vs_oracle']}")

    out = {
        "metric": METRIC,
        "value": round(amp_ms, 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(amp_ms, 4),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64+f32+f16",
        "data": "synthetic",
        "config": {
            "workload": f"3-D 7-point FV diffusion {args.grid}^3, coefficients 10^U(0,4) on 8^3 blocks, "
                        f"N={n}, nnz={nnz}, Jacobi, tol 1e-10, b ~ N(0,1)",
            "preset": args.preset,
            "parallelism": "single GPU",
        },
        "fp64_pcg_ms": round(fp64_ms, 4),
        "speedup_vs_fp64_pcg": round(fp64_ms / amp_ms, 4),
        "amp64_ms": round(results["amp64"][0], 4),
        "amp64_iters": results["amp64"][1]["iters"],
        "speedup_amp64_vs_fp64_pcg": round(fp64_ms / results["amp64"][0], 4),
        "iters": amp_info["iters"],
        "iters_fp64": fp64_info["iters"],
        "switch_iterations": {"u_z_fp32": amp_info["k_z32"], "u_z_fp16": amp_info["k_z16"],
                              "u_r_fp32": amp_info["k_r32"]},
        "rel_res_true": amp_info["relres_true"],
        "roofline": rf,
        "warm_product_step": warm,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
