"""Write the FP64 oracle's reference numbers for the full-size anisotropic Q1
workload (256^3 interior nodes, degree-4 Chebyshev preconditioner,
tol 1e-10).  Calls only the oracle and the workload generator.

    python tests/golden/make_q1_reference.py [threads]
"""

import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import cpcg  # noqa: E402
from workloads import problems as P  # noqa: E402


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    t0 = time.time()
    A, b, xs, (lo, hi) = P.q1_system(256)
    print(f"generated n={A.n} nnz={A.nnz} in {time.time() - t0:.1f}s bounds {lo:.6e} {hi:.6e}", flush=True)
    t0 = time.time()
    x, info = cpcg.pcg(A, b, tol=1e-10, maxit=20000, precond=cpcg.PC_CHEBYSHEV, degree=4,
                       lam_lo=lo, lam_hi=hi, threads=threads)
    err = float(np.linalg.norm(x - xs) / np.linalg.norm(xs))
    print(f"oracle: {info['iters']} iterations, status {info['status']}, relres {info['relres']:.3e}, "
          f"true {info['relres_true']:.3e}, err vs x* {err:.3e}, {time.time() - t0:.1f}s", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "q1_256_chebyshev4.txt")
    with open(out, "w") as f:
        f.write("# FP64 oracle PCG (Alg. 1) on the anisotropic Q1 workload: 256^3 interior nodes,\n")
        f.write("# K = diag(1, 1e-2, 1e-3), degree-4 Chebyshev on [lam_min, 1.05 lam_max] of D^-1 A (closed form),\n")
        f.write("# x* ~ U[-1,1] (seed [3, 1]), b = A x*, x0 = 0, tol 1e-10.\n")
        f.write("# Written by tests/golden/make_q1_reference.py.\n")
        f.write(f"iters {info['iters']}\n")
        f.write(f"relres_true {info['relres_true']:.6e}\n")
        f.write(f"err_vs_xstar {err:.6e}\n")


if __name__ == "__main__":
    main()
