"""Seeded synthetic inputs for the DG volume kernel.

This module is the only code the library and its test oracle have in common:
it draws random numbers and nothing else (no reference element, no geometric
factors, no derivative).  Every workload is synthetic: jittered unit
tetrahedra and random nodal fields, with the sizes below.

Workloads (seeds: mesh 1000+c, fields 2000+c for workload c):

1. order 3 (Np=20), K=4096, F=1, u ~ U(-1,1), FP64            -- small parity case
2. order 4 (Np=35), K=2^20, F=5, u ~ N(0,1), FP64              -- HBM-bound run
3. as 1, FP32 storage, split-BF16 products                     -- precision form
4. orders 1..7, K_N = round(2^U(10,18)) each (seed 3004), F=3, u ~ N(0,1) -- mixed orders
5. order 5 (Np=56), K=2^19, F=3, u ~ U(-1,1), FP64, adjoint    -- differentiation
"""

import numpy as np

UNIT_TET = np.array([[0.0, 0.0, 0.0],
                     [1.0, 0.0, 0.0],
                     [0.0, 1.0, 0.0],
                     [0.0, 0.0, 1.0]])

WORKLOADS = {
    1: dict(name="fp64_order3_K4096_F1", N=3, K=4096, F=1, dist="uniform", precision="f64"),
    2: dict(name="fp64_order4_K1048576_F5", N=4, K=1 << 20, F=5, dist="normal", precision="f64"),
    3: dict(name="f32s_order3_K4096_F1", N=3, K=4096, F=1, dist="uniform", precision="f32s"),
    4: dict(name="mixed_orders1to7_F3", N=None, K=None, F=3, dist="normal", precision="f64"),
    5: dict(name="fp64_order5_K524288_F3_adjoint", N=5, K=1 << 19, F=3, dist="uniform",
            precision="f64"),
}

MIXED_SEED = 3004


def mesh_seed(c):
    return 1000 + c


def field_seed(c):
    return 2000 + c


def tet_vertices(K, seed, jitter=0.2):
    """K jittered copies of the unit tetrahedron: (K, 4, 3) FP64.

    Each vertex coordinate is the unit-tet coordinate plus an independent
    U(-jitter, jitter) draw from numpy's default_rng(seed).
    """
    rng = np.random.default_rng(seed)
    return UNIT_TET[None, :, :] + rng.uniform(-jitter, jitter, size=(K, 4, 3))


def fields(K, F, Np, seed, dist="uniform"):
    """Nodal field values (K, F, Np) FP64: U(-1,1) ("uniform") or N(0,1) ("normal")."""
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, size=(K, F, Np))
    if dist == "normal":
        return rng.standard_normal(size=(K, F, Np))
    raise ValueError(f"unknown distribution {dist!r}")


def mixed_order_sizes(seed=MIXED_SEED, orders=range(1, 8), log2_lo=10.0, log2_hi=18.0):
    """Element count per order, K_N = round(2^U(log2_lo, log2_hi)), drawn in ascending order."""
    rng = np.random.default_rng(seed)
    return {int(N): int(round(2.0 ** rng.uniform(log2_lo, log2_hi))) for N in orders}


def tetra_count(N):
    """Node count of an order-N tetrahedron, (N+1)(N+2)(N+3)/6 (a size, not a computation
    of the method: it fixes array shapes)."""
    return (N + 1) * (N + 2) * (N + 3) // 6
