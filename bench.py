#!/usr/bin/env python3
"""Time-to-solution of AMP-PCG versus FP64 PCG on one MI355X.

A step is one complete solve (all kernels of the hot path, from r0 = b - A x0
to the verified solution) of the 3-D 7-point finite-volume diffusion system
on a 128^3 grid with block coefficients 10^U, U ~ U[0, 4] on 8^3 blocks
(N = 2,097,152, nnz = 14,581,760), Jacobi preconditioner, tol 1e-10.
Inputs are resident in HBM before the timed region starts.

Prints one JSON line: value = AMP-PCG time-to-solution (ms, lower is
better); the FP64 PCG time on the same GPU, the speedup, the iteration
counts, the SpMV kernel's achieved HBM bandwidth against the 8 TB/s peak, and
the FP64 CPU oracle timed on the host are reported beside it.
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


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def spmv_algorithmic_bytes(n, nnz, meta_bytes, b_val, b_z, b_q):
    """Bytes one fused product step p = z + beta p_old, q = A p must move:
    every nonzero's value once, the column metadata of the handle's layout
    once (int32 indices of index-mode slices, the shared offset lists of
    offset-mode slices, the slice pointers), z and p_old read once (the
    gathers are counted once), p and q written once.  Slice padding is
    overhead, not counted."""
    return nnz * b_val + meta_bytes + n * (3 * b_z + b_q)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_spmv_fixed_fv3d128_hbm_counters.txt")


def stored_traffic():
    """HBM bytes per launch of the product-step kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter summary (each scaled by the factor a
    plain copy of known size gives), or None when the summary is missing or
    was taken on other kernel sources than the library built here."""
    from paper_2505_04155_amd import build
    try:
        fields = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if line.strip() and not line.startswith("#"):
                    key, _, val = line.partition(" ")
                    fields[key] = val.strip()
    except OSError:
        return None
    if fields.get("source_digest") != build.source_digest():
        return None
    return int(float(fields["traffic_bytes_per_launch"]))


def time_spmv_step(binding, M, torch, u_z, u_r, diff, reps, n, nnz, meta_bytes):
    """Average duration (ms) of the library's product-step kernel over reps
    back-to-back launches, and its algorithmic bytes per launch."""
    import ctypes
    L = binding.load()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    for _ in range(3):
        binding.check(L.amp_spmv_step(M.handle, u_z, u_r, diff, 0.5, sp), "amp_spmv_step")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        L.amp_spmv_step(M.handle, u_z, u_r, diff, 0.5, sp)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    bv = 8 if u_r == 64 else 4
    return ms, spmv_algorithmic_bytes(n, nnz, meta_bytes, bv, u_z // 8, u_r // 8)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--preset", default="amp64")
    ap.add_argument("--spmv-reps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["solve", "spmv"], default="solve",
                    help="spmv: only the product kernels and a reference copy (for counter runs)")
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

    log(f"bench: generating the {args.grid}^3 system")
    A, b, _ = P.blocky_diffusion3d_system(args.grid, 8)
    M = amp.Matrix.from_csr(A, device=dev)
    pc = amp.Preconditioner(M, "jacobi")
    bt = torch.tensor(b, device=dev)
    info_m = M.info()
    tol, maxit = 1e-10, 20000

    def run(preset):
        x, info = amp.solve(M, pc, bt, tol=tol, maxit=maxit, preset=preset)
        if info["status"] != 0:
            raise RuntimeError(f"{preset} solve failed: {info}")
        return x, info

    if args.mode == "spmv":
        spmv_only(args, amp, binding, M, pc, bt, torch)
        return

    results = {}
    for preset in (args.preset, "pcg64"):
        for w in range(args.warmup):
            run(preset)
            log(f"bench: warmup {preset} {w + 1}/{args.warmup} done")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = []
        for s in range(args.steps):
            _, info = run(preset)
            infos.append(info)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms = (t1 - t0) * 1e3 / args.steps
        results[preset] = (ms, infos[-1])
        log(f"bench: {preset}: {ms:.3f} ms/solve, {infos[-1]['iters']} iterations, "
            f"switches z32={infos[-1]['k_z32']} z16={infos[-1]['k_z16']} r32={infos[-1]['k_r32']}")

    amp_ms, amp_info = results[args.preset]
    fp64_ms, fp64_info = results["pcg64"]

    # Dominant kernel: the fused product step of the reduced-precision phase
    # (p = z + beta p_old in FP16, q = A p with FP32 values in difference
    # form, FP32 q), timed with HIP events on the stream the library launches
    # on (torch's current stream) over spmv_reps back-to-back launches.
    n, nnz = info_m["n"], info_m["nnz"]
    spmv_ms, spmv_bytes = time_spmv_step(binding, M, torch, 16, 32, 1, args.spmv_reps, n, nnz,
                                         info_m["meta_bytes"])
    spmv_gbs = spmv_bytes / (spmv_ms * 1e-3) / 1e9
    log(f"bench: fused product step (p fp16, A fp32 diff): {spmv_ms * 1e3:.2f} us, {spmv_gbs:.0f} GB/s algorithmic")

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
        "iters": amp_info["iters"],
        "iters_fp64": fp64_info["iters"],
        "switch_iterations": {"u_z_fp32": amp_info["k_z32"], "u_z_fp16": amp_info["k_z16"],
                              "u_r_fp32": amp_info["k_r32"]},
        "rel_res_true": amp_info["relres_true"],
        "roofline": {
            "bound": "hbm",
            "kernel": "k_spmv_fixed<16,32,true>: p = z + beta p_old (FP16), q = A p (FP32 values, difference form)",
            "achieved": round(spmv_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(spmv_gbs / HBM_PEAK_GBS, 4),
            "traffic": stored_traffic(),
            "avg_kernel_us": round(spmv_ms * 1e3, 3),
            "algorithmic_bytes_per_launch": spmv_bytes,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def spmv_only(args, amp, binding, M, pc, bt, torch):
    """Product-step kernels alone, each launched spmv_reps times, plus a device
    copy of a known size: the launches a counter run attributes bytes to."""
    amp.solve(M, pc, bt, tol=1e-10, maxit=20000, preset=args.preset)   # fills the work buffers
    info_m = M.info()
    n, nnz = info_m["n"], info_m["nnz"]
    out = {"mode": "spmv", "matrix": info_m, "kernels": {}}
    for (u_z, u_r, diff) in ((64, 64, 0), (16, 32, 1), (32, 32, 1)):
        ms, nbytes = time_spmv_step(binding, M, torch, u_z, u_r, diff, args.spmv_reps, n, nnz,
                                    info_m["meta_bytes"])
        us = ms * 1e3
        out["kernels"][f"k_spmv_fixed<{u_z},{u_r},{'true' if diff else 'false'}>"] = {
            "avg_us": round(us, 3), "algorithmic_bytes": nbytes, "GB/s": round(nbytes / us / 1e3, 1)}
        log(f"product step u_z={u_z} u_r={u_r} diff={diff}: {us:.2f} us, {nbytes / us / 1e3:.0f} GB/s")
    stream = torch.cuda.current_stream()
    src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=bt.device)
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.spmv_reps):
        dst.copy_(src)
    e1.record(stream)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / args.spmv_reps
    out["copy_256MiB"] = {"avg_us": round(us, 3), "bytes": 2 * src.numel() * 4,
                          "GB/s": round(2 * src.numel() * 4 / us / 1e3, 1)}
    log(f"copy 256 MiB: {us:.2f} us, {2 * src.numel() * 4 / us / 1e3:.0f} GB/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
