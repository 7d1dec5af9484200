"""One-time host-side setup of the kernel's inputs: reference matrices D and geometric factors G.

Neither is part of the per-step path (they are inputs of dg_volume, built
once per order and per mesh); both are computed in FP64.

* ``reference_matrices(N)``: D_a = V_a V^{-1} for the monomial basis on the
  equispaced nodes (i/N, j/N, k/N) of the unit tetrahedron (k outermost, i
  fastest).  The monomials are taken about the element centroid
  (r-1/4)^p (s-1/4)^q (t-1/4)^w, which leaves D unchanged (it is the unique
  interpolate-differentiate-evaluate map of the nodes) but keeps V better
  conditioned; the system V^T X = V_a^T is solved by LU.
* ``geometric_factors(verts)``: G[k] = J_k^{-1} row-major, where
  J_k = [v1-v0 | v2-v0 | v3-v0] maps the unit tetrahedron onto element k;
  elements with det J below ``det_min`` are rejected.
"""

import numpy as np

NODE_COUNTS = {N: (N + 1) * (N + 2) * (N + 3) // 6 for N in range(1, 8)}


def order_of(Np):
    for N, n in NODE_COUNTS.items():
        if n == Np:
            return N
    raise ValueError(f"unsupported node count {Np}")


def reference_nodes(N):
    """(Np, 3) equispaced nodes of the unit tetrahedron."""
    out = np.empty((NODE_COUNTS[N], 3))
    n = 0
    for k in range(N + 1):
        for j in range(N + 1 - k):
            for i in range(N + 1 - j - k):
                out[n] = (i, j, k)
                n += 1
    return out / N


def reference_matrices(N):
    """D of shape (3, Np, Np), FP64, row-major: D[a, i, j]."""
    x = reference_nodes(N) - 0.25
    Np = len(x)
    powers = [(p, q, w) for p in range(N + 1) for q in range(N + 1 - p) for w in range(N + 1 - p - q)]
    pw = np.stack([x[:, c:c + 1] ** np.arange(N + 1)[None, :] for c in range(3)])  # (3, Np, N+1)
    V = np.empty((Np, Np))
    dV = np.zeros((3, Np, Np))
    for m, e in enumerate(powers):
        V[:, m] = pw[0, :, e[0]] * pw[1, :, e[1]] * pw[2, :, e[2]]
        for c in range(3):
            if e[c] > 0:
                f = [pw[d, :, e[d]] for d in range(3)]
                f[c] = e[c] * pw[c, :, e[c] - 1]
                dV[c, :, m] = f[0] * f[1] * f[2]
    D = np.empty((3, Np, Np))
    for c in range(3):
        D[c] = np.linalg.solve(V.T, dV[c].T).T
    return D


def geometric_factors(verts, det_min=0.01):
    """(K, 9) FP64 geometric factors from (K, 4, 3) vertex coordinates."""
    v = np.asarray(verts, dtype=np.float64)
    J = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)
    det = np.linalg.det(J)
    if det.size and det.min() < det_min:
        k = int(np.argmin(det))
        raise ValueError(f"element {k} is degenerate or inverted (det J = {det[k]:.3e})")
    return np.linalg.inv(J).reshape(-1, 9)
