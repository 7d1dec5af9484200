"""FP64 CPU oracle for the nodal discontinuous-Galerkin volume derivative.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the tests, the smoke check and the CPU-baseline leg of the benchmark call
it.  It shares no code with the HIP library (no kernels, headers, tables or
pre/post-processing); the two meet only in the seeded inputs they are both
handed.

What it computes (the volume term of a nodal DG discretisation on affine
tetrahedra, the PDE-solver use case named in the paper's Introduction):

* ``refelem``  -- equispaced nodes on the unit reference tetrahedron, the
  monomial Vandermonde matrix V and its derivative matrices V_r, V_s, V_t, and
  the reference differentiation matrices D_a = V_a V^{-1}.
* ``geometry`` -- per-element affine Jacobian J = [v1-v0 | v2-v0 | v3-v0] and
  the geometric factors G = J^{-1} (G[3a+b] = d r_a / d x_b).
* ``kernels``  -- the forward volume derivative, its adjoint and the
  split-BF16 emulation, as plain C loops (``dg_oracle.c``) in FP64.

Every function is pinned by tests that do not reuse its own formulas:
closed forms, exact rational arithmetic, exact polynomial differentiation,
brute force on one element and adjoint identities.  The bitwise summation
order of the GPU is "parity unpinned"; parity is judged with the normwise and
condition-scaled criteria documented next to each test.
"""

from .refelem import (num_nodes, order_from_np, equispaced_nodes, monomial_exponents,
                      vandermonde, derivative_matrices)
from .geometry import jacobians, geometric_factors, physical_nodes
from .kernels import (volume, volume_adjoint, volume_grad_d, volume_split_bf16, bf16_round_f32,
                      library_path, build_library, num_threads)

__all__ = [
    "num_nodes", "order_from_np", "equispaced_nodes", "monomial_exponents", "vandermonde",
    "derivative_matrices", "jacobians", "geometric_factors", "physical_nodes",
    "volume", "volume_adjoint", "volume_grad_d", "volume_split_bf16", "bf16_round_f32",
    "library_path", "build_library", "num_threads",
]
