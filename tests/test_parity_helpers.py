"""The parity criteria themselves (CPU): the fast condition sums taken through the C oracle
equal the NumPy sums of absolute values they stand for, and the split-BF16 error metrics
are the normwise and RMS relative errors."""

import numpy as np

import oracle
from paper_1503_07659_amd import synth
from parity import adjoint_cond, adjoint_cond_c, forward_cond, forward_cond_c, split_errors


def _case(N, K, F, seed):
    Np = oracle.num_nodes(N)
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, seed))
    u = synth.fields(K, F, Np, seed + 1, "normal")
    gout = synth.fields(3 * K, F, Np, seed + 2, "normal").reshape(3, K, F, Np)
    return D, G, u, gout


def test_condition_sums_through_the_oracle():
    for N, K, F in ((1, 7, 3), (4, 5, 2), (7, 3, 1)):
        D, G, u, gout = _case(N, K, F, 31 + N)
        a, b = forward_cond(D, G, u), forward_cond_c(D, G, u)
        assert np.allclose(a, b, rtol=1e-13, atol=0)
        assert (b >= np.abs(oracle.volume(D, G, u)) * (1 - 1e-13)).all()
        (gu_a, gG_a), (gu_b, gG_b) = adjoint_cond(D, G, u, gout), adjoint_cond_c(D, G, u, gout)
        assert np.allclose(gu_a, gu_b, rtol=1e-13, atol=0)
        assert np.allclose(gG_a, gG_b, rtol=1e-13, atol=0)


def test_split_error_metrics():
    ref = np.zeros((3, 2, 2))
    ref[:, 0, 0] = [2.0, 4.0, 1.0]
    ref[:, 1, 1] = [-2.0, 3.0, 1.0]
    got = ref.copy()
    got[0, 0, 0] += 0.02          # plane 0: one error of 0.02, max|ref| = 2, ||ref|| = sqrt(8)
    got[2, 1, 1] -= 0.01          # plane 2
    e = split_errors(got, ref)
    assert abs(e[0]["max_rel"] - 0.01) < 1e-15 and abs(e[0]["rms_rel"] - 0.02 / np.sqrt(8)) < 1e-15
    assert e[1] == {"max_rel": 0.0, "rms_rel": 0.0}
    assert abs(e[2]["max_rel"] - 0.01) < 1e-15 and abs(e[2]["rms_rel"] - 0.01 / np.sqrt(2)) < 1e-15
