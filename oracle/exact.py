"""Exact rational differentiation matrices from the closed-form Lagrange basis.

Test oracle, second construction.  It is used only to pin the FP64 route in
``refelem`` (D_a = V_a V^{-1}); the two share no formulas.

For equispaced nodes of order N on a simplex, a node is given by its
barycentric index beta = (beta_0, ..., beta_3) with sum N, at barycentric
coordinates lambda = beta / N.  The Lagrange basis function of node beta is
the product over vertices m of

    P_p(x) = (1 / p!) * prod_{q=0}^{p-1} (N x - q),     p = beta_m, x = lambda_m,

which is 1 at its own node and 0 at every other node (at node gamma it equals
prod_m binom(gamma_m, beta_m), nonzero only for gamma = beta).  On the unit
tetrahedron lambda_1 = r, lambda_2 = s, lambda_3 = t and
lambda_0 = 1 - r - s - t, so d/dr_a = d/dlambda_a - d/dlambda_0.

Everything is computed in ``fractions.Fraction``; the result is the exact
matrix, from which an FP64 copy is the correctly rounded one.
"""

from fractions import Fraction
from math import comb, factorial


def _node_indices(N):
    """Barycentric indices of the nodes, in the same order as refelem.equispaced_nodes."""
    idx = []
    for k in range(N + 1):
        for j in range(N + 1 - k):
            for i in range(N + 1 - j - k):
                idx.append((N - i - j - k, i, j, k))
    return idx


def exact_derivative_matrices(N):
    """Exact D as nested lists [3][Np][Np] of Fractions."""
    nodes = _node_indices(N)
    # P_p(g/N) = binom(g, p); dP_p/dx at x = g/N = (N/p!) sum_{q'<p} prod_{q<p, q!=q'} (g - q)
    P = [[Fraction(comb(g, p)) for g in range(N + 1)] for p in range(N + 1)]
    dP = []
    for p in range(N + 1):
        row = []
        for g in range(N + 1):
            s = 0
            for qq in range(p):
                prod = 1
                for q in range(p):
                    if q != qq:
                        prod *= (g - q)
                s += prod
            row.append(Fraction(N * s, factorial(p)))
        dP.append(row)
    Np = len(nodes)
    D = [[[Fraction(0)] * Np for _ in range(Np)] for _ in range(3)]
    for i, gam in enumerate(nodes):
        for j, bet in enumerate(nodes):
            vals = [P[bet[m]][gam[m]] for m in range(4)]
            grads = []
            for m in range(4):
                g = dP[bet[m]][gam[m]]
                if g == 0:
                    grads.append(Fraction(0))
                    continue
                prod = g
                for mm in range(4):
                    if mm != m:
                        prod *= vals[mm]
                grads.append(prod)
            for a in range(3):
                D[a][i][j] = grads[a + 1] - grads[0]
    return D


def exact_derivative_matrices_f64(N):
    """The exact matrices rounded once to FP64, as nested lists of floats."""
    return [[[float(x) for x in row] for row in Da] for Da in exact_derivative_matrices(N)]
