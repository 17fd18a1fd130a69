"""Oracle for the AMP-PCG solver.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything from this package.  It shares no code with
the GPU solver (``paper_2505_04155_amd``) and never imports it.

* :mod:`oracle.cpcg`      -- plain C FP64 PCG (Alg. 1), Jacobi and Chebyshev
  preconditioners, CSR SpMV (``pcg_oracle.c``, built with gcc/OpenMP).
* :mod:`oracle.amp_model` -- numpy model of AMP-PCG (Alg. 3) with every
  rounding to FP16/FP32/FP64 written out, the eta indicators and the
  precision selector.
* :mod:`oracle.adjoint`   -- FP64 reference of the differentiable solve's
  gradient (adjoint solve + per-face chain rule).
* :mod:`oracle.eigbounds` -- Lanczos estimate of the Chebyshev interval.
* :mod:`oracle.hexop`     -- the matrix-free order-N hexahedral screened
  Poisson operator (GLL points, trilinear element maps), its diagonal.
* :mod:`oracle.pmg`       -- the p-multigrid V-cycle over polynomial orders
  (Chebyshev-Jacobi smoothing, interpolation between orders) and PCG with it.
"""

from . import cpcg  # noqa: F401
from . import amp_model  # noqa: F401
from . import adjoint  # noqa: F401
