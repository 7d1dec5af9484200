"""Affine element maps and geometric factors (test oracle).

An affine tetrahedron with vertices v0..v3 is the image of the unit reference
tetrahedron under x = v0 + J r, with J = [v1-v0 | v2-v0 | v3-v0] (columns are
dx/dr_a).  The geometric factors are the entries of J^{-1}:
G[k][3a+b] = d r_a / d x_b, stored in the order rx, ry, rz, sx, sy, sz, tx, ty, tz.
By the chain rule, d u / d x_b = sum_a G[3a+b] * d u / d r_a.

J^{-1} is formed here by the adjugate formula (cofactors over the
determinant), written out entry by entry.
"""

import numpy as np

DET_MIN = 0.01  # elements with det J below this are rejected as degenerate


def jacobians(verts):
    """verts: (K, 4, 3) vertex coordinates -> J: (K, 3, 3) with J[:, :, a] = v_{a+1} - v_0."""
    verts = np.asarray(verts, dtype=np.float64)
    if verts.ndim != 3 or verts.shape[1:] != (4, 3):
        raise ValueError("verts must have shape (K, 4, 3)")
    J = np.empty((verts.shape[0], 3, 3))
    for a in range(3):
        J[:, :, a] = verts[:, a + 1, :] - verts[:, 0, :]
    return J


def geometric_factors(verts, det_min=DET_MIN):
    """Geometric factors G (K, 9) = J^{-1} flattened row-major, via the adjugate.

    Raises ValueError if any element has det J < det_min (inverted or
    degenerate).
    """
    J = jacobians(verts)
    # J = [[a b c], [d e f], [g h i]]
    a, b, c = J[:, 0, 0], J[:, 0, 1], J[:, 0, 2]
    d, e, f = J[:, 1, 0], J[:, 1, 1], J[:, 1, 2]
    g, h, i = J[:, 2, 0], J[:, 2, 1], J[:, 2, 2]
    # cofactors
    A = e * i - f * h
    B = -(d * i - f * g)
    C = d * h - e * g
    det = a * A + b * B + c * C
    if det.size and det.min() < det_min:
        bad = int(np.argmin(det))
        raise ValueError(f"degenerate or inverted element {bad}: det J = {det[bad]:.3e} < {det_min}")
    Dc = -(b * i - c * h)
    E = a * i - c * g
    Fc = -(a * h - b * g)
    Gc = b * f - c * e
    H = -(a * f - c * d)
    I = a * e - b * d
    # inverse = adj / det, adj = transpose of the cofactor matrix
    inv = np.empty((J.shape[0], 9))
    inv[:, 0], inv[:, 1], inv[:, 2] = A / det, Dc / det, Gc / det
    inv[:, 3], inv[:, 4], inv[:, 5] = B / det, E / det, H / det
    inv[:, 6], inv[:, 7], inv[:, 8] = C / det, Fc / det, I / det
    return inv


def physical_nodes(verts, ref_nodes):
    """Physical node coordinates x_n = v0 + J xi_n, shape (K, Np, 3)."""
    J = jacobians(verts)
    v0 = np.asarray(verts, dtype=np.float64)[:, 0, :]
    return v0[:, None, :] + np.einsum("kba,na->knb", J, np.asarray(ref_nodes, dtype=np.float64))
