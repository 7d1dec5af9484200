"""Pins for the oracle's reference element: D_a = V_a V^{-1} on equispaced unit-tet nodes.

Each check is fixed by mathematics, not by the oracle's own formulas:
hand-derived order 1, exact rational matrices from the closed-form Lagrange
basis (a different construction), and identities every exact
differentiation matrix satisfies.
"""

import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.exact import exact_derivative_matrices

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# FP64 LU solve of the monomial Vandermonde system vs the exact matrix,
# relative to max|D|.  Measured: 0 (N<=2), 5e-16 (3), 3.2e-15 (4), 5.9e-14 (5),
# 3.2e-13 (6), 1.6e-12 (7); the monomial Vandermonde condition number grows with N.
D_TOL = {1: 1e-15, 2: 1e-15, 3: 1e-14, 4: 1e-14, 5: 2e-13, 6: 2e-12, 7: 1e-11}


def _exact_f64(N):
    return np.array([[[float(x) for x in row] for row in Da] for Da in exact_derivative_matrices(N)])


def test_node_counts():
    assert [oracle.num_nodes(N) for N in range(1, 8)] == [4, 10, 20, 35, 56, 84, 120]
    for N in range(1, 8):
        assert oracle.order_from_np(oracle.num_nodes(N)) == N
    with pytest.raises(ValueError):
        oracle.order_from_np(21)


def test_nodes_on_unit_tet():
    for N in range(1, 8):
        x = oracle.equispaced_nodes(N)
        assert x.shape == (oracle.num_nodes(N), 3)
        assert (x >= 0).all() and (x.sum(axis=1) <= 1 + 1e-15).all()
        # all distinct, all on the 1/N lattice
        assert len({tuple(np.round(p * N).astype(int)) for p in x}) == len(x)
        assert np.allclose(x * N, np.round(x * N), atol=1e-12)
    assert np.array_equal(oracle.equispaced_nodes(1), np.array(
        [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float))


def test_order1_golden_hand_derived():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "D_order1.txt")) if not ln.startswith("#")]
    rows = [r for r in rows if r]
    want = np.zeros((3, 4, 4))
    a = -1
    i = 0
    for r in rows:
        if len(r) == 1:
            a, i = int(r[0]), 0
        else:
            want[a, i] = [float(v) for v in r]
            i += 1
    assert np.array_equal(oracle.derivative_matrices(1), want)


@pytest.mark.parametrize("N", [2, 3])
def test_stored_exact_golden(N):
    """Stored exact rationals (written by tests/golden/make_golden.py) vs the oracle in FP64."""
    want = np.zeros((3, oracle.num_nodes(N), oracle.num_nodes(N)))
    for ln in open(os.path.join(GOLDEN, f"D_order{N}_exact.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        a, i, j, q = ln.split()
        want[int(a), int(i), int(j)] = float(Fraction(q))
    D = oracle.derivative_matrices(N)
    assert np.abs(D - want).max() <= D_TOL[N] * np.abs(want).max()
    # the stored file also still agrees with the exact construction
    assert np.array_equal(want, _exact_f64(N))


@pytest.mark.parametrize("N", range(1, 8))
def test_matches_exact_lagrange(N):
    E = _exact_f64(N)
    D = oracle.derivative_matrices(N)
    err = np.abs(D - E).max() / np.abs(E).max()
    assert err <= D_TOL[N], err


@pytest.mark.parametrize("N", range(1, 5))
def test_exact_identities_in_rationals(N):
    """The exact matrices satisfy D 1 = 0 and D_r r = 1, D_r s = 0 with no rounding."""
    E = exact_derivative_matrices(N)
    nodes = [(Fraction(p[0]).limit_denominator(N), Fraction(p[1]).limit_denominator(N),
              Fraction(p[2]).limit_denominator(N)) for p in oracle.equispaced_nodes(N)]
    Np = len(nodes)
    for a in range(3):
        for i in range(Np):
            assert sum(E[a][i]) == 0
            for c in range(3):
                s = sum(E[a][i][j] * nodes[j][c] for j in range(Np))
                assert s == (1 if c == a else 0)


@pytest.mark.parametrize("N", range(1, 8))
def test_constants_annihilated(N):
    D = oracle.derivative_matrices(N)
    assert np.abs(D.sum(axis=2)).max() <= 1e-14 * np.abs(D).max() * oracle.num_nodes(N)


@pytest.mark.parametrize("N", range(1, 8))
def test_differentiates_monomials_exactly(N):
    """D_a applied to nodal values of r^p s^q t^w (p+q+w <= N) gives the analytic derivative."""
    D = oracle.derivative_matrices(N)
    x = oracle.equispaced_nodes(N)
    r, s, t = x[:, 0], x[:, 1], x[:, 2]
    tol = 20 * D_TOL[N] * np.abs(D).max()
    for p in range(N + 1):
        for q in range(N + 1 - p):
            for w in range(N + 1 - p - q):
                f = r ** p * s ** q * t ** w
                d = [p * r ** max(p - 1, 0) * s ** q * t ** w,
                     q * r ** p * s ** max(q - 1, 0) * t ** w,
                     w * r ** p * s ** q * t ** max(w - 1, 0)]
                for a in range(3):
                    assert np.abs(D[a] @ f - d[a]).max() <= tol


@pytest.mark.parametrize("N", range(1, 8))
def test_commute_and_nilpotent(N):
    """Exact differentiation operators commute, and N+1 derivatives kill degree <= N.

    Residuals are measured against the scale of the nonzero quantities they come
    from: ||D_a||_inf^2 for the commutator, max|D_a^N| (which is of order N!) for
    D_a^{N+1}.  Observed: commutator <= 5e-15, D^{N+1}/D^N <= 2.1e-11 (N=7).
    """
    D = oracle.derivative_matrices(N)
    for a in range(3):
        nrm = np.linalg.norm(D[a], np.inf)
        for b in range(a + 1, 3):
            assert np.abs(D[a] @ D[b] - D[b] @ D[a]).max() <= 10 * D_TOL[N] * nrm ** 2
        PN = np.linalg.matrix_power(D[a], N)
        assert np.abs(PN).max() >= 1.0  # the N-th derivative of r^N (or s^N, t^N) is N! != 0
        P = PN @ D[a]
        assert np.abs(P).max() <= 10 * D_TOL[N] * np.abs(PN).max()


def test_exponent_set():
    for N in range(1, 8):
        e = oracle.monomial_exponents(N)
        assert len(e) == oracle.num_nodes(N)
        assert len(set(e)) == len(e)
        assert all(sum(x) <= N and min(x) >= 0 for x in e)
