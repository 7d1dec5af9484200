"""Reference tetrahedron of order N: nodes, monomial Vandermonde, D_a = V_a V^{-1}.

Part of the test oracle (see the package docstring).  The paper names nodal
DG only as a use case (Introduction) and gives none of its formulas; what is
written here is the standard definition of a nodal differentiation matrix:
interpolate nodal values by the unique polynomial of total degree <= N,
differentiate it along a reference coordinate, evaluate at the nodes.

Conventions (fixed here, shared with the library only through the inputs):

* Reference element: the unit tetrahedron with vertices (0,0,0), (1,0,0),
  (0,1,0), (0,0,1); coordinates (r, s, t).
* Nodes: (i/N, j/N, k/N) for k = 0..N, then j = 0..N-k, then i = 0..N-j-k,
  with i varying fastest.
* D is returned as an array of shape (3, Np, Np): D[a][i][j] is the weight of
  nodal value j in the a-derivative (a = r, s, t) at node i.
"""

import numpy as np


def num_nodes(N):
    """Number of nodes of the order-N tetrahedron, (N+1)(N+2)(N+3)/6."""
    return (N + 1) * (N + 2) * (N + 3) // 6


def order_from_np(Np):
    """Inverse of num_nodes; raises ValueError if Np is not a tetrahedral number."""
    for N in range(0, 64):
        if num_nodes(N) == Np:
            return N
        if num_nodes(N) > Np:
            break
    raise ValueError(f"{Np} is not the node count of any tetrahedral order")


def equispaced_nodes(N):
    """Equispaced nodes of the unit tetrahedron, shape (Np, 3), FP64."""
    if N < 1:
        raise ValueError("order N must be >= 1")
    pts = []
    for k in range(N + 1):
        for j in range(N + 1 - k):
            for i in range(N + 1 - j - k):
                pts.append((i / N, j / N, k / N))
    return np.array(pts, dtype=np.float64)


def monomial_exponents(N):
    """All exponent triples (p, q, w) with p + q + w <= N, one per basis monomial."""
    return [(p, q, w)
            for total in range(N + 1)
            for w in range(total + 1)
            for q in range(total - w + 1)
            for p in [total - w - q]]


def vandermonde(N, pts=None):
    """Monomial Vandermonde matrix and its three reference derivatives.

    Returns (V, Vr, Vs, Vt), each of shape (Np, Np): V[n][m] is monomial m
    r^p s^q t^w evaluated at node n; V_a holds the a-derivative of each
    monomial at each node.
    """
    if pts is None:
        pts = equispaced_nodes(N)
    exps = monomial_exponents(N)
    r, s, t = pts[:, 0], pts[:, 1], pts[:, 2]
    n = len(pts)
    V = np.empty((n, len(exps)))
    Vr = np.zeros_like(V)
    Vs = np.zeros_like(V)
    Vt = np.zeros_like(V)
    for m, (p, q, w) in enumerate(exps):
        V[:, m] = r ** p * s ** q * t ** w
        if p > 0:
            Vr[:, m] = p * r ** (p - 1) * s ** q * t ** w
        if q > 0:
            Vs[:, m] = q * r ** p * s ** (q - 1) * t ** w
        if w > 0:
            Vt[:, m] = w * r ** p * s ** q * t ** (w - 1)
    return V, Vr, Vs, Vt


def derivative_matrices(N):
    """Reference differentiation matrices D_a = V_a V^{-1}, shape (3, Np, Np), FP64.

    Computed without forming V^{-1}: D_a^T solves V^T X = V_a^T (LU with
    partial pivoting via numpy.linalg.solve).
    """
    V, Vr, Vs, Vt = vandermonde(N)
    D = np.empty((3,) + V.shape)
    for a, Va in enumerate((Vr, Vs, Vt)):
        D[a] = np.linalg.solve(V.T, Va.T).T
    return D
