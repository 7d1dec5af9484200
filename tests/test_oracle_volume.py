"""Pins for the oracle's geometry, forward volume derivative, adjoint and split-BF16 emulation.

None of these re-types the oracle's formulas: each compares against exact
calculus (polynomials differentiated analytically), a one-element brute force
through the physical Vandermonde matrix (no D, no G), exact adjoint
identities (in u, G and D), central finite differences, additivity of the
cross-element D cotangent, or an independent BF16 rounding.
"""

import numpy as np
import pytest

import oracle
from paper_1503_07659_amd import synth


def _rand_rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _rel(err, ref):
    return np.abs(err).max() / max(np.abs(ref).max(), 1e-300)


# ---------------------------------------------------------------- geometry

def test_geometric_factors_invert_jacobian():
    v = synth.tet_vertices(500, seed=11)
    J = oracle.jacobians(v)
    G = oracle.geometric_factors(v).reshape(-1, 3, 3)
    eye = np.broadcast_to(np.eye(3), J.shape)
    assert np.abs(G @ J - eye).max() < 1e-13
    assert np.abs(J @ G - eye).max() < 1e-13


def test_geometric_factors_special_maps():
    rng = np.random.default_rng(5)
    ref = synth.UNIT_TET
    # unjittered unit tet: identity map
    G = oracle.geometric_factors(ref[None])
    assert np.array_equal(G[0], np.eye(3).ravel())
    # x = 2 r + c: G = I / 2
    G = oracle.geometric_factors((2 * ref + np.array([3.0, -1.0, 0.5]))[None])
    assert np.allclose(G[0], 0.5 * np.eye(3).ravel(), atol=1e-15)
    # x = Q r: G = Q^T
    Q = _rand_rotation(rng)
    G = oracle.geometric_factors((ref @ Q.T)[None])
    assert np.allclose(G[0].reshape(3, 3), Q.T, atol=1e-14)


def test_degenerate_element_rejected():
    v = synth.tet_vertices(4, seed=1)
    v[2, 3] = v[2, 0] + 0.5 * (v[2, 1] - v[2, 0])  # flat element
    with pytest.raises(ValueError):
        oracle.geometric_factors(v)
    v = synth.tet_vertices(4, seed=1)
    v[1, [1, 2]] = v[1, [2, 1]]  # inverted orientation
    with pytest.raises(ValueError):
        oracle.geometric_factors(v)


def test_physical_nodes_of_unit_tet():
    for N in (1, 3, 5):
        x = oracle.physical_nodes(synth.UNIT_TET[None], oracle.equispaced_nodes(N))
        assert np.array_equal(x[0], oracle.equispaced_nodes(N))


def test_workload_meshes_not_degenerate():
    """The seeded workload meshes stay well away from the rejection threshold."""
    for c, K in ((1, 4096), (5, 1 << 14)):
        v = synth.tet_vertices(K, synth.mesh_seed(c))
        J = oracle.jacobians(v)
        assert np.linalg.det(J).min() > 0.1


# ---------------------------------------------------------------- forward

def _poly_field(rng, N, xyz):
    """Random polynomial of total degree <= N at points xyz (..., 3) and its gradient."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    val = np.zeros(x.shape)
    grad = np.zeros((3,) + x.shape)
    for p in range(N + 1):
        for q in range(N + 1 - p):
            for w in range(N + 1 - p - q):
                c = rng.uniform(-1, 1)
                val += c * x ** p * y ** q * z ** w
                if p:
                    grad[0] += c * p * x ** (p - 1) * y ** q * z ** w
                if q:
                    grad[1] += c * q * x ** p * y ** (q - 1) * z ** w
                if w:
                    grad[2] += c * w * x ** p * y ** q * z ** (w - 1)
    return val, grad


@pytest.mark.parametrize("N", range(1, 8))
def test_exact_on_polynomials(N):
    """Random physical polynomials of degree <= N are differentiated exactly (to rounding)."""
    rng = np.random.default_rng(100 + N)
    K, F = 64, 2
    v = synth.tet_vertices(K, seed=200 + N)
    G = oracle.geometric_factors(v)
    D = oracle.derivative_matrices(N)
    xyz = oracle.physical_nodes(v, oracle.equispaced_nodes(N))  # (K, Np, 3)
    u = np.empty((K, F, xyz.shape[1]))
    ref = np.empty((3, K, F, xyz.shape[1]))
    for f in range(F):
        val, grad = _poly_field(rng, N, xyz)
        u[:, f] = val
        ref[:, :, f] = grad
    out = oracle.volume(D, G, u)
    assert _rel(out - ref, ref) < 1e-11


def test_lower_degree_polynomials_also_exact():
    N = 5
    rng = np.random.default_rng(7)
    v = synth.tet_vertices(16, seed=8)
    xyz = oracle.physical_nodes(v, oracle.equispaced_nodes(N))
    G = oracle.geometric_factors(v)
    D = oracle.derivative_matrices(N)
    for d in range(0, N + 1):
        val, grad = _poly_field(rng, d, xyz)
        out = oracle.volume(D, G, val[:, None, :])
        assert np.abs(out[:, :, 0] - grad).max() <= 1e-11 * max(1.0, np.abs(grad).max())


@pytest.mark.parametrize("N", range(1, 8))
def test_constants_give_zero(N):
    v = synth.tet_vertices(32, seed=3)
    G = oracle.geometric_factors(v)
    D = oracle.derivative_matrices(N)
    u = np.broadcast_to(np.arange(1.0, 33.0)[:, None, None], (32, 3, oracle.num_nodes(N))).copy()
    out = oracle.volume(D, G, u)
    assert np.abs(out).max() <= 1e-13 * np.abs(G).max() * np.abs(D).max() * oracle.num_nodes(N) * 32


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_one_element_brute_force(N):
    """K=1: out_b = (d_b V_phys) V_phys^{-1} u with the Vandermonde in physical x, y, z.

    This route uses neither the reference matrices D nor the factors G.
    """
    rng = np.random.default_rng(40 + N)
    v = synth.tet_vertices(1, seed=41 + N)
    xyz = oracle.physical_nodes(v, oracle.equispaced_nodes(N))[0]
    c = xyz.mean(axis=0)
    x, y, z = (xyz - c).T  # centred monomials keep the physical Vandermonde well conditioned
    Np = len(x)
    V = np.empty((Np, Np))
    Vd = np.zeros((3, Np, Np))
    m = 0
    for p in range(N + 1):
        for q in range(N + 1 - p):
            for w in range(N + 1 - p - q):
                V[:, m] = x ** p * y ** q * z ** w
                if p:
                    Vd[0, :, m] = p * x ** (p - 1) * y ** q * z ** w
                if q:
                    Vd[1, :, m] = q * x ** p * y ** (q - 1) * z ** w
                if w:
                    Vd[2, :, m] = w * x ** p * y ** q * z ** (w - 1)
                m += 1
    u = rng.uniform(-1, 1, (1, 2, Np))
    ref = np.stack([np.linalg.solve(V.T, Vd[b].T).T @ u[0].T for b in range(3)])  # (3, Np, F)
    ref = ref.transpose(0, 2, 1)[:, None]
    out = oracle.volume(oracle.derivative_matrices(N), oracle.geometric_factors(v), u)
    assert _rel(out - ref, ref) < 1e-11


def test_rotation_covariance():
    """Rotating the mesh by Q rotates the gradient: out' = Q out for the same nodal values."""
    rng = np.random.default_rng(9)
    N, K, F = 4, 40, 2
    v = synth.tet_vertices(K, seed=10)
    Q = _rand_rotation(rng)
    D = oracle.derivative_matrices(N)
    u = rng.standard_normal((K, F, oracle.num_nodes(N)))
    out = oracle.volume(D, oracle.geometric_factors(v), u)
    out_rot = oracle.volume(D, oracle.geometric_factors(v @ Q.T), u)
    assert _rel(out_rot - np.einsum("bc,ckfi->bkfi", Q, out), out) < 1e-13


def test_linearity_and_permutation():
    rng = np.random.default_rng(12)
    N, K, F = 3, 50, 3
    D = oracle.derivative_matrices(N)
    G1 = oracle.geometric_factors(synth.tet_vertices(K, seed=13))
    G2 = oracle.geometric_factors(synth.tet_vertices(K, seed=14))
    u1 = rng.standard_normal((K, F, 20))
    u2 = rng.standard_normal((K, F, 20))
    a, b = 0.7, -1.3
    lhs = oracle.volume(D, G1, a * u1 + b * u2)
    rhs = a * oracle.volume(D, G1, u1) + b * oracle.volume(D, G1, u2)
    assert _rel(lhs - rhs, lhs) < 1e-14
    lhs = oracle.volume(D, a * G1 + b * G2, u1)
    rhs = a * oracle.volume(D, G1, u1) + b * oracle.volume(D, G2, u1)
    assert _rel(lhs - rhs, lhs) < 1e-14
    perm = rng.permutation(K)
    assert np.array_equal(oracle.volume(D, G1[perm], u1[perm]), oracle.volume(D, G1, u1)[:, perm])


def test_zero_jitter_reduces_to_reference_derivatives():
    N, K = 3, 5
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(np.broadcast_to(synth.UNIT_TET, (K, 4, 3)))
    u = np.random.default_rng(1).standard_normal((K, 2, 20))
    out = oracle.volume(D, G, u)
    for a in range(3):
        ref = np.einsum("ij,kfj->kfi", D[a], u)  # BLAS summation order: equal up to rounding
        assert np.abs(out[a] - ref).max() <= 1e-14 * np.abs(D[a]).max() * np.abs(u).max() * 20


def test_empty_mesh():
    out = oracle.volume(oracle.derivative_matrices(2), np.zeros((0, 9)), np.zeros((0, 1, 10)))
    assert out.shape == (3, 0, 1, 10)


# ---------------------------------------------------------------- adjoint

@pytest.mark.parametrize("N,F", [(1, 1), (3, 2), (5, 3), (7, 2)])
def test_adjoint_identities(N, F):
    """<fwd(u,G), w> = <u, gu> = <G, gG>: out is linear in u and, separately, in G."""
    rng = np.random.default_rng(60 + N)
    K = 37
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, seed=61))
    u = rng.standard_normal((K, F, oracle.num_nodes(N)))
    w = rng.standard_normal((3, K, F, oracle.num_nodes(N)))
    out = oracle.volume(D, G, u)
    gu, gG = oracle.volume_adjoint(D, G, u, w)
    s0 = np.sum(out * w)
    scale = np.sum(np.abs(out) * np.abs(w))
    assert abs(np.sum(u * gu) - s0) <= 1e-13 * scale
    assert abs(np.sum(G * gG) - s0) <= 1e-13 * scale
    # per element, too: <out_k, w_k> = <G_k, gG_k>
    per_k = np.einsum("bkfi,bkfi->k", out, w)
    assert np.abs(np.sum(G * gG, axis=1) - per_k).max() <= 1e-13 * scale


def test_adjoint_finite_differences():
    """Loss = sum(out^2); central differences with h = 1e-6 on a 64-element mesh."""
    rng = np.random.default_rng(77)
    N, K, F = 5, 64, 3
    Np = oracle.num_nodes(N)
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, seed=78))
    u = rng.uniform(-1, 1, (K, F, Np))

    def loss(uu, GG):
        return np.sum(oracle.volume(D, GG, uu) ** 2)

    out = oracle.volume(D, G, u)
    gu, gG = oracle.volume_adjoint(D, G, u, 2 * out)
    h = 1e-6
    idx_u = [tuple(rng.integers(0, s) for s in u.shape) for _ in range(40)]
    fd_u = []
    for ix in idx_u:
        up, um = u.copy(), u.copy()
        up[ix] += h
        um[ix] -= h
        fd_u.append((loss(up, G) - loss(um, G)) / (2 * h))
    fd_u = np.array(fd_u)
    an_u = np.array([gu[ix] for ix in idx_u])
    assert np.abs(fd_u - an_u).max() <= 1e-6 * np.abs(an_u).max()
    idx_G = [(int(rng.integers(0, K)), c) for c in range(9) for _ in range(3)]
    fd_G = []
    for ix in idx_G:
        Gp, Gm = G.copy(), G.copy()
        Gp[ix] += h
        Gm[ix] -= h
        fd_G.append((loss(u, Gp) - loss(u, Gm)) / (2 * h))
    fd_G = np.array(fd_G)
    an_G = np.array([gG[ix] for ix in idx_G])
    assert np.abs(fd_G - an_G).max() <= 1e-6 * np.abs(an_G).max()


@pytest.mark.parametrize("N,F", [(1, 1), (2, 3), (4, 2), (7, 1)])
def test_grad_d_identity(N, F):
    """<fwd(u,G,D), w> = <D, gD> for any D: out is linear in D as well.

    A random D (no zero row sums, no symmetry) so that a transposed gD or a
    gD built from a shifted u cannot pass by accident."""
    rng = np.random.default_rng(90 + N)
    K = 41
    Np = oracle.num_nodes(N)
    D = rng.standard_normal((3, Np, Np))
    G = oracle.geometric_factors(synth.tet_vertices(K, seed=91))
    u = rng.standard_normal((K, F, Np))
    w = rng.standard_normal((3, K, F, Np))
    gD = oracle.volume_grad_d(G, u, w)
    s0 = np.sum(oracle.volume(D, G, u) * w)
    scale = np.sum(np.abs(D)) * np.abs(gD).max() + abs(s0)
    assert abs(np.sum(D * gD) - s0) <= 1e-13 * scale
    # each of the three matrices separately: only D_a enters direction a
    for a in range(3):
        Da = np.zeros_like(D)
        Da[a] = D[a]
        sa = np.sum(oracle.volume(Da, G, u) * w)
        assert abs(np.sum(D[a] * gD[a]) - sa) <= 1e-13 * scale


def test_grad_d_additive_over_elements():
    """gD is a sum over elements: splitting the mesh splits it."""
    rng = np.random.default_rng(95)
    N, K, F = 3, 50, 2
    Np = oracle.num_nodes(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, seed=96))
    u = rng.standard_normal((K, F, Np))
    w = rng.standard_normal((3, K, F, Np))
    whole = oracle.volume_grad_d(G, u, w)
    parts = oracle.volume_grad_d(G[:17], u[:17], w[:, :17]) + oracle.volume_grad_d(G[17:], u[17:], w[:, 17:])
    assert np.abs(whole - parts).max() <= 1e-13 * np.abs(whole).max()
    assert np.all(oracle.volume_grad_d(G[:0], u[:0], w[:, :0]) == 0.0)


def test_grad_d_finite_differences():
    """Loss = sum(out^2); central differences in entries of D, h = 1e-6."""
    rng = np.random.default_rng(97)
    N, K, F = 4, 64, 3
    Np = oracle.num_nodes(N)
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, seed=98))
    u = rng.uniform(-1, 1, (K, F, Np))
    gD = oracle.volume_grad_d(G, u, 2 * oracle.volume(D, G, u))
    h = 1e-6
    idx = [(a, int(rng.integers(0, Np)), int(rng.integers(0, Np))) for a in range(3) for _ in range(8)]
    fd = []
    for ix in idx:
        Dp, Dm = D.copy(), D.copy()
        Dp[ix] += h
        Dm[ix] -= h
        fd.append((np.sum(oracle.volume(Dp, G, u) ** 2) - np.sum(oracle.volume(Dm, G, u) ** 2)) / (2 * h))
    fd = np.array(fd)
    an = np.array([gD[ix] for ix in idx])
    assert np.abs(fd - an).max() <= 1e-6 * np.abs(an).max()


# ---------------------------------------------------------------- split-BF16

def _bf16_reference(x):
    """Independent RNE to 8 significant bits via frexp and numpy's round-half-even."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)          # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)


def test_bf16_rounding():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(20000), rng.uniform(-1e3, 1e3, 20000),
                        rng.uniform(-1e-3, 1e-3, 20000)]).astype(np.float32)
    # exact halfway cases: 1 + 2^-8 (ties down to even 1.0), 1 + 3*2^-8 (ties up to 1 + 2^-6)
    special = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, -0.0, 2 ** -130],
                       dtype=np.float32)
    y = oracle.bf16_round_f32(np.concatenate([x, special]))
    assert np.array_equal(y[:len(x)].astype(np.float64), _bf16_reference(x))
    assert list(y[len(x):len(x) + 4]) == [1.0, 1.0, 1 + 2 ** -6, -1.0]
    assert y[len(x) + 4] == 0.0
    # BF16 values are FP32 values with the low 16 bits clear
    assert (y.view(np.uint32) & 0xFFFF == 0).all()


def test_split_exact_when_inputs_are_bf16():
    """If D and u are BF16 numbers the lo parts vanish and the split product is the FP64 one."""
    rng = np.random.default_rng(4)
    N, K, F = 3, 100, 2
    D = oracle.bf16_round_f32(oracle.derivative_matrices(N).astype(np.float32))
    u = oracle.bf16_round_f32(rng.standard_normal((K, F, 20)).astype(np.float32))
    G = oracle.geometric_factors(synth.tet_vertices(K, seed=5)).astype(np.float32)
    out = oracle.volume_split_bf16(D, G, u)
    ref = oracle.volume(D.astype(np.float64), G.astype(np.float64), u.astype(np.float64))
    assert _rel(out - ref, ref) < 1e-14


@pytest.mark.parametrize("N", [3, 4, 7])
def test_split_error_bound_vs_fp64(N):
    """The three-pass split stays within the stated bound of the FP64 result:
    normwise max-rel <= 2e-5 and RMS-rel <= 1e-5 per output plane, while a
    one-pass (hi x hi) product would be off by ~2^-9."""
    rng = np.random.default_rng(90 + N)
    K, F = 256, 2
    Np = oracle.num_nodes(N)
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, seed=91))
    u = rng.uniform(-1, 1, (K, F, Np))
    ref = oracle.volume(D, G, u)
    out = oracle.volume_split_bf16(D.astype(np.float32), G.astype(np.float32), u.astype(np.float32))
    for b in range(3):
        e = out[b] - ref[b]
        assert np.abs(e).max() / np.abs(ref[b]).max() <= 2e-5
        assert np.linalg.norm(e) / np.linalg.norm(ref[b]) <= 1e-5
    hi = oracle.volume(oracle.bf16_round_f32(D.astype(np.float32)).astype(np.float64), G,
                       oracle.bf16_round_f32(u.astype(np.float32)).astype(np.float64))
    assert np.abs(hi - ref).max() / np.abs(ref).max() > 1e-4
