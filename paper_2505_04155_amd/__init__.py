"""AMP-PCG for AMD MI355X: adaptive mixed-precision, dynamically scaled
preconditioned conjugate gradients (Guo, de Sturler, Warburton,
arXiv:2505.04155) as hand-written HIP kernels behind a C ABI
(include/amp_pcg.h).

Python entry points (argument marshalling only):

* :class:`Matrix`, :class:`Preconditioner`, :func:`solve`, :func:`solve_batched`
* :func:`tune_group_rows`, :func:`tune_lanes` (autotuners of rows per work-group and
  lanes per row, run on the device)
* :func:`selector_replay`, :func:`paper_kernel_bytes` (host-only helpers)
* :func:`use_torch_allocator`, :func:`use_hip_allocator` (where the library's
  device memory comes from)
"""

from .solver import (Matrix, Preconditioner, solve, solve_batched, tune_group_rows,  # noqa: F401
                     selector_replay, paper_kernel_bytes, use_torch_allocator, use_hip_allocator,
                     tune_lanes, HexOperator)
