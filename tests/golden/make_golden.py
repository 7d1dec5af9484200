"""Writes the stored exact differentiation matrices under tests/golden/.

Calls only the oracle (its exact rational construction).  Usage:
    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.exact import exact_derivative_matrices  # noqa: E402


def write(N):
    D = exact_derivative_matrices(N)
    Np = len(D[0])
    path = os.path.join(HERE, f"D_order{N}_exact.txt")
    with open(path, "w") as fh:
        fh.write(f"# Exact reference differentiation matrices, order N={N}, Np={Np}, unit tetrahedron,\n")
        fh.write("# equispaced nodes (i/N, j/N, k/N), k outer, then j, i fastest.\n")
        fh.write("# Written by tests/golden/make_golden.py from oracle/exact.py (closed-form Lagrange\n")
        fh.write("# basis of equispaced simplex nodes, exact rationals).\n")
        fh.write("# Lines: a i j numerator/denominator   (a = 0:r, 1:s, 2:t)\n")
        for a in range(3):
            for i in range(Np):
                for j in range(Np):
                    x = D[a][i][j]
                    fh.write(f"{a} {i} {j} {x.numerator}/{x.denominator}\n")


if __name__ == "__main__":
    for N in (2, 3):
        write(N)
