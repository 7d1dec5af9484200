"""GPU parity: the HIP kernels, called through the C ABI, against the FP64 oracle.

Inputs are seeded and synthetic (jittered unit tetrahedra, random fields);
D and G come from the oracle and are handed identically to both sides.
Sizes span several 16-column tiles and a ragged tail; full-size workloads are
run in the benchmark's launch configuration and compared on sampled elements.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1503_07659_amd import dgvol, synth
from parity import FP64_TOL, adjoint_cond, adjoint_cond_c, check_planes, check_whole, forward_cond, forward_cond_c

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def make_case(N, K, F, seed, dist="uniform"):
    Np = oracle.num_nodes(N)
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, seed))
    u = synth.fields(K, F, Np, seed + 1, dist)
    return D, G, u


def test_native_library_is_the_one_loaded():
    lib = dgvol.load_library()
    assert lib._name == dgvol.LIB_PATH


# ------------------------------------------------------------------ forward FP64

def test_forward_workload1():
    """Order 3, K=4096, F=1, u ~ U(-1,1): the small parity workload, every output."""
    _say("forward workload1 N=3 K=4096 F=1")
    D, G, u = make_case(3, 4096, 1, synth.mesh_seed(1))
    u = synth.fields(4096, 1, 20, synth.field_seed(1), "uniform")
    out = host(dgvol.dg_volume(dev(D), dev(G), dev(u)))
    check_planes(out, oracle.volume(D, G, u), forward_cond(D, G, u))


@pytest.mark.parametrize("N", range(1, 8))
@pytest.mark.parametrize("F", [1, 3, 5, 17])
def test_forward_orders_and_fields(N, F):
    K = 157  # K*F columns: several tiles plus a ragged tail
    _say(f"forward N={N} K={K} F={F}")
    D, G, u = make_case(N, K, F, 300 + 10 * N + F, "normal")
    out = host(dgvol.dg_volume(dev(D), dev(G), dev(u)))
    check_planes(out, oracle.volume(D, G, u), forward_cond(D, G, u))


@pytest.mark.parametrize("K,F", [(1, 1), (2, 3), (3, 5), (16, 1), (17, 1), (1, 33)])
def test_forward_small_and_ragged(K, F):
    for N in (1, 4, 5, 7):
        _say(f"forward small N={N} K={K} F={F}")
        D, G, u = make_case(N, K, F, 40 + K + F)
        out = host(dgvol.dg_volume(dev(D), dev(G), dev(u)))
        check_planes(out, oracle.volume(D, G, u), forward_cond(D, G, u))


def test_forward_empty():
    _say("forward K=0")
    D = dev(oracle.derivative_matrices(2))
    out = dgvol.dg_volume(D, torch.zeros((0, 9), dtype=torch.float64, device="cuda"),
                          torch.zeros((0, 2, 10), dtype=torch.float64, device="cuda"))
    assert out.shape == (3, 0, 2, 10)


@pytest.mark.parametrize("N,shift", [(4, 0), (5, 0), (7, 0), (7, 1)])
def test_forward_guard_bands_and_determinism(N, shift):
    """Writes stay inside out (orders 5 and 7 store through buffer ranges that
    drop out-of-range lanes); repeated launches give bitwise identical results.
    shift = 1 moves out off 16-byte alignment (the single-word path of the
    chunk-register body)."""
    K, F = 999, 5
    Np = oracle.num_nodes(N)
    _say(f"forward guards N={N} K={K} F={F} shift={shift}")
    D, G, u = make_case(N, K, F, 77, "normal")
    n = 3 * K * F * Np
    guard = 4096 + shift
    buf = torch.full((n + 2 * guard,), 1.25e300, dtype=torch.float64, device="cuda")
    buf[guard:guard + n] = float("nan")
    out = buf[guard:guard + n].view(3, K, F, Np)
    Dd, Gd, ud = dev(D), dev(G), dev(u)
    dgvol.dg_volume(Dd, Gd, ud, out=out)
    b = host(buf)
    assert (b[:guard] == 1.25e300).all() and (b[guard + n:] == 1.25e300).all()
    first = host(out).copy()
    check_planes(first, oracle.volume(D, G, u), forward_cond(D, G, u))
    for _ in range(3):
        again = host(dgvol.dg_volume(Dd, Gd, ud))
        assert np.array_equal(again, first)


def test_forward_on_side_stream():
    N, K, F = 3, 2000, 2
    _say(f"forward side stream N={N} K={K} F={F}")
    D, G, u = make_case(N, K, F, 91)
    s = torch.cuda.Stream()
    Dd, Gd, ud = dev(D), dev(G), dev(u)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        out = dgvol.dg_volume(Dd, Gd, ud)
    s.synchronize()
    check_planes(host(out), oracle.volume(D, G, u), forward_cond(D, G, u))


# ------------------------------------------------------------------ adjoint FP64

def _check_adjoint(D, G, u, gout, gu, gG):
    ref_gu, ref_gG = oracle.volume_adjoint(D, G, u, gout)
    c_gu, c_gG = adjoint_cond(D, G, u, gout)
    check_whole(gu, ref_gu, c_gu, what="gu")
    check_whole(gG, ref_gG, c_gG, what="gG")


@pytest.mark.parametrize("N", range(1, 8))
@pytest.mark.parametrize("F", [1, 3, 5, 17])
def test_adjoint_orders_and_fields(N, F):
    K = 131
    _say(f"adjoint N={N} K={K} F={F}")
    D, G, u = make_case(N, K, F, 500 + 10 * N + F)
    gout = np.random.default_rng(N * 100 + F).standard_normal((3, K, F, oracle.num_nodes(N)))
    gu, gG = dgvol.dg_volume_adjoint(dev(D), dev(G), dev(u), dev(gout))
    _check_adjoint(D, G, u, gout, host(gu), host(gG))


@pytest.mark.parametrize("K,F", [(1, 1), (1, 3), (5, 16), (2, 40)])
def test_adjoint_small(K, F):
    for N in (2, 5):
        _say(f"adjoint small N={N} K={K} F={F}")
        D, G, u = make_case(N, K, F, 600 + K + F)
        gout = np.random.default_rng(K + F).standard_normal((3, K, F, oracle.num_nodes(N)))
        gu, gG = dgvol.dg_volume_adjoint(dev(D), dev(G), dev(u), dev(gout))
        _check_adjoint(D, G, u, gout, host(gu), host(gG))


@pytest.mark.parametrize("N,F", [(3, 3), (5, 3), (6, 3), (7, 3), (3, 20), (5, 33)])
def test_adjoint_guard_bands(N, F):
    """gu and gG are written only inside their views (order 5 stores gu through
    buffer ranges that drop out-of-range lanes; orders 6-7 run two passes; each
    wave's last tile of a run, and elements with F > 16, leave partial tiles)."""
    K = 301
    Np = oracle.num_nodes(N)
    _say(f"adjoint guards N={N} K={K} F={F}")
    D, G, u = make_case(N, K, F, 88, "normal")
    gout = np.random.default_rng(89).standard_normal((3, K, F, Np))
    guard = 1024
    nu, ng = K * F * Np, K * 9
    bu = torch.full((nu + 2 * guard,), 1.25e300, dtype=torch.float64, device="cuda")
    bg = torch.full((ng + 2 * guard,), 1.25e300, dtype=torch.float64, device="cuda")
    gu = bu[guard:guard + nu].view(K, F, Np)
    gG = bg[guard:guard + ng].view(K, 9)
    dgvol.dg_volume_adjoint(dev(D), dev(G), dev(u), dev(gout), gu=gu, gG=gG)
    hu, hg = host(bu), host(bg)
    assert (hu[:guard] == 1.25e300).all() and (hu[guard + nu:] == 1.25e300).all()
    assert (hg[:guard] == 1.25e300).all() and (hg[guard + ng:] == 1.25e300).all()
    _check_adjoint(D, G, u, gout, host(gu), host(gG))


@pytest.mark.parametrize("N,K,F", [(5, 3000, 3), (5, 700, 20), (6, 900, 3), (6, 250, 40), (7, 600, 3), (7, 300, 20)])
def test_adjoint_deterministic(N, K, F):
    """Every adjoint path (staged runs, two-pass) gives the same bits on
    every run: gG is summed in a fixed order, with no atomics."""
    _say(f"adjoint determinism N={N} K={K} F={F}")
    D, G, u = make_case(N, K, F, 650 + N + F)
    gout = np.random.default_rng(651 + N).standard_normal((3, K, F, oracle.num_nodes(N)))
    Dd, Gd, ud, gd = dev(D), dev(G), dev(u), dev(gout)
    gu1, gG1 = (host(x) for x in dgvol.dg_volume_adjoint(Dd, Gd, ud, gd))
    gu2, gG2 = (host(x) for x in dgvol.dg_volume_adjoint(Dd, Gd, ud, gd))
    assert np.array_equal(gu1, gu2) and np.array_equal(gG1, gG2)
    _check_adjoint(D, G, u, gout, gu1, gG1)


def test_adjoint_workload5_full_size():
    """Order 5, K=2^19, F=3, loss = sum(out^2) so gout = 2 out: every gu and gG entry."""
    N, K, F = 5, 1 << 19, 3
    _say(f"adjoint workload5 N={N} K={K} F={F}")
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, synth.mesh_seed(5)))
    u = synth.fields(K, F, 56, synth.field_seed(5), "uniform")
    Dd, Gd, ud = dev(D), dev(G), dev(u)
    out = dgvol.dg_volume(Dd, Gd, ud)
    gout = 2.0 * out
    gu, gG = dgvol.dg_volume_adjoint(Dd, Gd, ud, gout)
    gout_h = host(gout)
    check_planes(gout_h / 2.0, oracle.volume(D, G, u), forward_cond_c(D, G, u))
    ref_gu, ref_gG = oracle.volume_adjoint(D, G, u, gout_h)
    c_gu, c_gG = adjoint_cond_c(D, G, u, gout_h)
    check_whole(host(gu), ref_gu, c_gu, what="gu")
    check_whole(host(gG), ref_gG, c_gG, what="gG")


# ------------------------------------------------------------------ cotangent of D

def _check_grad_d(G, u, gout, gD):
    """Per direction a: normwise and condition-scaled (the same sum over |G|, |u|, |gout|)."""
    ref = oracle.volume_grad_d(G, u, gout)
    cond = oracle.volume_grad_d(np.abs(G), np.abs(u), np.abs(gout))
    check_planes(gD, ref, cond, what="gD")


@pytest.mark.parametrize("N", range(1, 8))
@pytest.mark.parametrize("F", [1, 3, 5, 17])
def test_grad_d_orders_and_fields(N, F):
    K = 131  # 131 F columns: several 32-column chunks and a ragged tail
    _say(f"grad_d N={N} K={K} F={F}")
    D, G, u = make_case(N, K, F, 900 + 10 * N + F, "normal")
    gout = np.random.default_rng(N * 31 + F).standard_normal((3, K, F, oracle.num_nodes(N)))
    gD = dgvol.dg_volume_grad_d(dev(G), dev(u), dev(gout))
    _check_grad_d(G, u, gout, host(gD))


@pytest.mark.parametrize("N", [1, 4, 5, 7])
def test_grad_d_many_parts(N):
    """More 128-column units than partial sums (1172 units into 1024 or 512 parts of
    one to three units each)."""
    K, F = 50000, 3
    _say(f"grad_d many parts N={N} K={K} F={F}")
    D, G, u = make_case(N, K, F, 950 + N)
    gout = np.random.default_rng(951 + N).standard_normal((3, K, F, oracle.num_nodes(N)))
    gD = dgvol.dg_volume_grad_d(dev(G), dev(u), dev(gout))
    _check_grad_d(G, u, gout, host(gD))


@pytest.mark.parametrize("K,F", [(1, 1), (2, 3), (1, 40), (0, 2)])
def test_grad_d_small_and_empty(K, F):
    for N in (1, 3, 7):
        _say(f"grad_d small N={N} K={K} F={F}")
        Np = oracle.num_nodes(N)
        D, G, u = make_case(N, max(K, 1), F, 960 + K + F)
        G, u = G[:K], u[:K]
        gout = np.random.default_rng(961).standard_normal((3, K, F, Np))
        gD = torch.full((3, Np, Np), float("nan"), dtype=torch.float64, device="cuda")
        dgvol.dg_volume_grad_d(dev(G), dev(u), dev(gout), gD=gD)
        _check_grad_d(G, u, gout, host(gD))
        if K == 0:
            assert np.all(host(gD) == 0.0)


def test_grad_d_deterministic_and_workspace():
    """Bitwise reproducible; stale workspace contents do not matter; a short workspace is refused."""
    N, K, F = 4, 5000, 5
    _say(f"grad_d determinism N={N} K={K} F={F}")
    D, G, u = make_case(N, K, F, 970)
    gout = np.random.default_rng(971).standard_normal((3, K, F, 35))
    Gd, ud, gd = dev(G), dev(u), dev(gout)
    need = dgvol.grad_d_workspace_bytes(K, 35, F)
    work = torch.full((need // 8,), float("nan"), dtype=torch.float64, device="cuda")
    a = host(dgvol.dg_volume_grad_d(Gd, ud, gd, work=work))
    b = host(dgvol.dg_volume_grad_d(Gd, ud, gd))
    assert np.array_equal(a, b)
    _check_grad_d(G, u, gout, a)
    with pytest.raises(dgvol.DGVolError):
        dgvol.dg_volume_grad_d(Gd, ud, gd, work=work[: need // 8 - 1])


def test_grad_d_workload5_full_size():
    """Order 5, K=2^19, F=3, gout = 2 out (loss = sum(out^2)): every entry of gD
    against the oracle's full reduction over 1.5 M columns."""
    N, K, F = 5, 1 << 19, 3
    _say(f"grad_d workload5 N={N} K={K} F={F}")
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, synth.mesh_seed(5)))
    u = synth.fields(K, F, 56, synth.field_seed(5), "uniform")
    gout = 2.0 * oracle.volume(D, G, u)
    gD = dgvol.dg_volume_grad_d(dev(G), dev(u), dev(gout))
    _check_grad_d(G, u, gout, host(gD))


# ------------------------------------------------------------------ autograd

def test_autograd_matches_oracle_and_finite_differences():
    """64 elements of order 5, F=3, loss = sum(out^2): gradients w.r.t. u and G
    against the oracle's adjoint (1e-12) and central differences h=1e-6 (1e-6)."""
    N, K, F = 5, 64, 3
    _say(f"autograd N={N} K={K} F={F}")
    D, G, u = make_case(N, K, F, 700)
    Dd = dev(D)
    ut = dev(u).requires_grad_(True)
    Gt = dev(G).requires_grad_(True)
    out = dgvol.volume(ut, Gt, Dd)
    (out ** 2).sum().backward()
    gu, gG = host(ut.grad), host(Gt.grad)
    ref_out = oracle.volume(D, G, u)
    _check_adjoint(D, G, u, 2.0 * ref_out, gu, gG)
    assert Dd.grad is None  # D was not marked as requiring a gradient

    def loss(uu, GG):
        return float((dgvol.dg_volume(Dd, dev(GG), dev(uu)) ** 2).sum())

    rng = np.random.default_rng(701)
    h = 1e-6
    fd, an = [], []
    for _ in range(24):
        ix = tuple(int(rng.integers(0, s)) for s in u.shape)
        up, um = u.copy(), u.copy()
        up[ix] += h
        um[ix] -= h
        fd.append((loss(up, G) - loss(um, G)) / (2 * h))
        an.append(gu[ix])
    for _ in range(18):
        ix = (int(rng.integers(0, K)), int(rng.integers(0, 9)))
        Gp, Gm = G.copy(), G.copy()
        Gp[ix] += h
        Gm[ix] -= h
        fd.append((loss(u, Gp) - loss(u, Gm)) / (2 * h))
        an.append(gG[ix])
    fd, an = np.array(fd), np.array(an)
    assert np.abs(fd - an).max() <= 1e-6 * np.abs(an).max()


def test_torch_gradcheck():
    N, K, F = 2, 3, 2
    _say("gradcheck")
    D, G, u = make_case(N, K, F, 800)
    ut = dev(u).requires_grad_(True)
    Gt = dev(G).requires_grad_(True)
    assert torch.autograd.gradcheck(dgvol.DGVolume.apply, (ut, Gt, dev(D)), eps=1e-6, atol=1e-8, rtol=1e-6)
    Dt = dev(D).requires_grad_(True)
    assert torch.autograd.gradcheck(dgvol.DGVolume.apply, (ut, Gt, Dt), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_autograd_gradient_of_d():
    """D marked as requiring a gradient: loss = sum(out^2) on 64 order-4 elements;
    gD against the oracle (1e-12) and central differences in entries of D (1e-6)."""
    N, K, F = 4, 64, 3
    _say(f"autograd D N={N} K={K} F={F}")
    D, G, u = make_case(N, K, F, 810)
    Dt = dev(D).requires_grad_(True)
    out = dgvol.volume(dev(u), dev(G), Dt)
    (out ** 2).sum().backward()
    gD = host(Dt.grad)
    _check_grad_d(G, u, 2.0 * oracle.volume(D, G, u), gD)
    Gd, ud = dev(G), dev(u)
    rng = np.random.default_rng(811)
    h = 1e-6
    fd, an = [], []
    for _ in range(18):
        ix = (int(rng.integers(0, 3)), int(rng.integers(0, 35)), int(rng.integers(0, 35)))
        Dp, Dm = D.copy(), D.copy()
        Dp[ix] += h
        Dm[ix] -= h
        lp = float((dgvol.dg_volume(dev(Dp), Gd, ud) ** 2).sum())
        lm = float((dgvol.dg_volume(dev(Dm), Gd, ud) ** 2).sum())
        fd.append((lp - lm) / (2 * h))
        an.append(gD[ix])
    fd, an = np.array(fd), np.array(an)
    assert np.abs(fd - an).max() <= 1e-6 * np.abs(an).max()


# ------------------------------------------------------------------ split-BF16 form

def _check_f32s(D, G, u, got):
    """Stated bound vs FP64 (2e-5 max-rel, 1e-5 RMS per plane), and an a-priori
    FP32-accumulation bound vs the exact three-pass emulation:
    |gpu - emu| <= (3 Np + 4) 2^-24 cond."""
    Np = u.shape[2]
    ref64 = oracle.volume(D, G, u)
    for b in range(3):
        e = got[b] - ref64[b]
        assert np.abs(e).max() <= 2e-5 * np.abs(ref64[b]).max()
        assert np.linalg.norm(e) <= 1e-5 * np.linalg.norm(ref64[b])
    D32, G32, u32 = D.astype(np.float32), G.astype(np.float32), u.astype(np.float32)
    emu = oracle.volume_split_bf16(D32, G32, u32)
    cond = forward_cond(D32.astype(np.float64), G32.astype(np.float64), u32.astype(np.float64))
    tol = (3 * Np + 4) * 2.0 ** -24
    assert (np.abs(got - emu) <= tol * cond + 1e-30).all()


def test_f32s_workload3():
    """FP32 storage, split-BF16: order 3, K=4096, F=1, u ~ U(-1,1)."""
    _say("f32s workload3 N=3 K=4096 F=1")
    D = oracle.derivative_matrices(3)
    G = oracle.geometric_factors(synth.tet_vertices(4096, synth.mesh_seed(3)))
    u = synth.fields(4096, 1, 20, synth.field_seed(3), "uniform")
    got = host(dgvol.dg_volume_f32s(dev(D.astype(np.float32)), dev(G.astype(np.float32)),
                                    dev(u.astype(np.float32)))).astype(np.float64)
    _check_f32s(D, G, u, got)


@pytest.mark.parametrize("N", range(1, 8))
def test_f32s_orders(N):
    K, F = 143, 3
    _say(f"f32s N={N} K={K} F={F}")
    D, G, u = make_case(N, K, F, 900 + N, "normal")
    got = host(dgvol.dg_volume_f32s(dev(D.astype(np.float32)), dev(G.astype(np.float32)),
                                    dev(u.astype(np.float32)))).astype(np.float64)
    _check_f32s(D, G, u, got)


@pytest.mark.parametrize("N,shift", [(4, 0), (7, 0), (7, 1)])
def test_f32s_guard_bands(N, shift):
    """Split-BF16 writes stay inside out (order 7 stores through buffer ranges);
    shift = 1 moves out off 8-byte alignment (the single-float path); repeated
    launches give bitwise identical results."""
    K, F = 301, 3
    Np = oracle.num_nodes(N)
    _say(f"f32s guards N={N} K={K} F={F} shift={shift}")
    D, G, u = make_case(N, K, F, 910 + N, "normal")
    D32, G32, u32 = (dev(x.astype(np.float32)) for x in (D, G, u))
    n = 3 * K * F * Np
    guard = 2048 + shift
    buf = torch.full((n + 2 * guard,), 1.5e30, dtype=torch.float32, device="cuda")
    out = buf[guard:guard + n].view(3, K, F, Np)
    dgvol.dg_volume_f32s(D32, G32, u32, out=out)
    b = host(buf)
    assert (b[:guard] == np.float32(1.5e30)).all() and (b[guard + n:] == np.float32(1.5e30)).all()
    first = host(out).copy()
    _check_f32s(D, G, u, first.astype(np.float64))
    again = host(dgvol.dg_volume_f32s(D32, G32, u32))
    assert np.array_equal(again, first)


# ------------------------------------------------------------------ bandwidth calibration kernel

def test_stream_calibrate():
    _say("stream calibrate")
    n = 100003
    src = torch.arange(n, dtype=torch.float64, device="cuda") * 0.5 - 7.0
    for copies in (1, 2, 3):
        dst = torch.full((copies * n,), float("nan"), dtype=torch.float64, device="cuda")
        dgvol.dg_stream_calibrate(src, dst, copies)
        want = torch.cat([(c + 1) * src for c in range(copies)])
        assert torch.equal(dst, want)


@pytest.mark.parametrize("tiles_per_wave", [0, 1, 3])
def test_stream_calibrate_tiles(tiles_per_wave):
    """Every tile of every plane written once, scaled by the plane index + 1: the persistent shape
    (0: one workgroup per CU looping over 10007 tiles), one tile per wave, and three per wave with
    a ragged last workgroup."""
    ntiles = 10007
    _say(f"tile stream calibrate ntiles={ntiles} tiles_per_wave={tiles_per_wave}")
    w = dgvol.TILE_STREAM_WORDS
    src = torch.arange(ntiles * w, dtype=torch.float64, device="cuda") * 0.25 - 3.0
    dst = torch.full((3 * ntiles * w,), float("nan"), dtype=torch.float64, device="cuda")
    dgvol.dg_stream_calibrate_tiles(src, dst, tiles_per_wave)
    want = torch.cat([(c + 1) * src for c in range(3)])
    assert torch.equal(dst, want)


# ------------------------------------------------------------------ mixed-order batched launch

def test_mfma_calibrate():
    """The matrix-core calibration runs, writes every sink entry, and reaches a
    plausible fraction of the 78.6 TFLOP/s FP64 peak."""
    _say("mfma calibrate")
    sink = torch.full((dgvol.MFMA_CAL_BLOCKS * 256,), float("nan"), dtype=torch.float64, device="cuda")
    dgvol.dg_mfma_calibrate(10, sink=sink)
    torch.cuda.synchronize()
    assert torch.isfinite(sink).all()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    _, flops = dgvol.dg_mfma_calibrate(2000, sink=sink)
    e1.record(s)
    torch.cuda.synchronize()
    tflops = flops / (e0.elapsed_time(e1) * 1e-3) / 1e12
    assert 20.0 < tflops < 90.0, tflops


@pytest.mark.parametrize("mode", [dgvol.BESIDE_NONE, dgvol.BESIDE_FP64_FMA, dgvol.BESIDE_INT, dgvol.BESIDE_DPP])
def test_mfma_calibrate_beside(mode):
    """Products beside vector work: every mode runs (products and vector work, or either alone)
    and writes every sink entry; the mode with nothing beside the products gives the
    calibration's own per-lane sums."""
    _say(f"mfma beside mode={mode}")
    n = dgvol.MFMA_BESIDE_BLOCKS * 512
    for iters, viters in ((10, 10), (0, 10), (10, 0)):
        if mode == dgvol.BESIDE_NONE and iters == 0:
            continue
        sink = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        dgvol.dg_mfma_calibrate_beside(iters, viters, mode, sink=sink)
        torch.cuda.synchronize()
        assert torch.isfinite(sink).all()
    if mode == dgvol.BESIDE_NONE:
        ref = torch.full((dgvol.MFMA_CAL_BLOCKS * 256,), float("nan"), dtype=torch.float64, device="cuda")
        dgvol.dg_mfma_calibrate(10, sink=ref)
        sink = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        dgvol.dg_mfma_calibrate_beside(10, 0, mode, sink=sink)
        torch.cuda.synchronize()
        # waves 0..3 of each workgroup run the same chains as the calibration's waves
        assert torch.equal(sink.view(-1, 512)[:, :256], ref.view(-1, 256)[: dgvol.MFMA_BESIDE_BLOCKS])
        assert (sink.view(-1, 512)[:, 256:] == 0.0).all()


def _mixed_case(sizes, F, form, seed):
    D, G, u = {}, {}, {}
    for N, K in sizes.items():
        D[N] = oracle.derivative_matrices(N)
        G[N] = oracle.geometric_factors(synth.tet_vertices(K, seed + N))
        u[N] = synth.fields(K, F, oracle.num_nodes(N), seed + 100 + N, "normal")
    return D, G, u


@pytest.mark.parametrize("form", [dgvol.FORM_F64, dgvol.FORM_F32S])
def test_batched_matches_single_and_oracle(form):
    """Orders 1..7 with uneven element counts in one launch: each group is bitwise equal to the
    single-group call (same body) and meets the parity bar against the oracle."""
    sizes = {1: 1000, 2: 37, 3: 513, 4: 129, 5: 300, 6: 71, 7: 250}
    F = 3
    _say(f"batched form={form} sizes={sizes}")
    D, G, u = _mixed_case(sizes, F, form, 4000)
    cast = (lambda x: x) if form == dgvol.FORM_F64 else (lambda x: x.astype(np.float32))
    trip = [(dev(cast(D[N])), dev(cast(G[N])), dev(cast(u[N]))) for N in sizes]
    outs = dgvol.dg_volume_batched(trip, form=form)
    single = dgvol.dg_volume if form == dgvol.FORM_F64 else dgvol.dg_volume_f32s
    for (N, K), (Dd, Gd, ud), o in zip(sizes.items(), trip, outs):
        got = host(o)
        assert np.array_equal(got, host(single(Dd, Gd, ud))), f"order {N}: batched != single"
        if form == dgvol.FORM_F64:
            check_planes(got, oracle.volume(D[N], G[N], u[N]), forward_cond(D[N], G[N], u[N]))
        else:
            _check_f32s(D[N], G[N], u[N], got.astype(np.float64))


@pytest.mark.parametrize("form", [dgvol.FORM_F64, dgvol.FORM_F32S])
def test_batched_every_variant_one_launch(form):
    """Every variant of every order in one batch, in both launch modes (one launch for all
    8-wave groups; one launch per variant class), gives the oracle's result, the same bits in
    both modes."""
    F = 2
    _say(f"batched variants form={form}")
    cast = (lambda x: x) if form == dgvol.FORM_F64 else (lambda x: x.astype(np.float32))
    for vi in range(6):
        sizes = {N: 97 + 13 * vi for N in range(1, 8) if vi < dgvol.variant_count(form, oracle.num_nodes(N))}
        if not sizes:
            continue
        D, G, u = _mixed_case(sizes, F, form, 4100 + vi)
        trip = [(dev(cast(D[N])), dev(cast(G[N])), dev(cast(u[N]))) for N in sizes]
        outs = dgvol.dg_volume_batched(trip, form=form, variants=[vi] * len(sizes))
        by_class = dgvol.dg_volume_batched(trip, form=form, variants=[vi] * len(sizes), by_class=True)
        for (N, o), oc in zip(zip(sizes, outs), by_class):
            assert np.array_equal(host(o), host(oc)), f"order {N} variant {vi}: launch modes differ"
            got = host(o)
            if form == dgvol.FORM_F64:
                check_planes(got, oracle.volume(D[N], G[N], u[N]), forward_cond(D[N], G[N], u[N]))
            else:
                _check_f32s(D[N], G[N], u[N], got.astype(np.float64))


def test_batched_skips_empty_groups_and_weights():
    F = 1
    _say("batched empty groups and weights")
    D, G, u = _mixed_case({2: 50, 5: 60}, F, dgvol.FORM_F64, 4200)
    empty = (dev(oracle.derivative_matrices(3)), torch.zeros((0, 9), dtype=torch.float64, device="cuda"),
             torch.zeros((0, F, 20), dtype=torch.float64, device="cuda"))
    trip = [(dev(D[2]), dev(G[2]), dev(u[2])), empty, (dev(D[5]), dev(G[5]), dev(u[5]))]
    outs = dgvol.dg_volume_batched(trip, costs=[1.0, 0.0, 50.0])
    for N, o in ((2, outs[0]), (5, outs[2])):
        check_planes(host(o), oracle.volume(D[N], G[N], u[N]), forward_cond(D[N], G[N], u[N]))


# ------------------------------------------------------------------ graph capture and autotuning

def test_graph_replay_matches_eager():
    """The batched launch captured in a graph replays bitwise equal to the eager launch, every
    replay, with eager work in between."""
    from paper_1503_07659_amd.graph import CapturedLaunch
    sizes = {1: 700, 3: 250, 5: 90, 7: 120}
    F = 3
    _say("graph replay")
    D, G, u = _mixed_case(sizes, F, dgvol.FORM_F64, 4300)
    trip = [(dev(D[N]), dev(G[N]), dev(u[N])) for N in sizes]
    eager = [host(o).copy() for o in dgvol.dg_volume_batched(trip)]
    outs = [torch.full((3,) + tuple(t[2].shape), float("nan"), dtype=torch.float64, device="cuda") for t in trip]
    cap = CapturedLaunch(lambda: dgvol.dg_volume_batched(trip, outs=outs))
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        cap.replay()
        torch.cuda.synchronize()
        for N, o, e in zip(sizes, outs, eager):
            assert np.array_equal(host(o), e), f"replay {rep}, order {N}"
        dgvol.dg_volume_batched(trip)  # eager work between replays
        torch.cuda.synchronize()


def test_autotuner_cache_and_tuned_launch(tmp_path, monkeypatch):
    from paper_1503_07659_amd import autotune
    monkeypatch.setenv("DGVOL_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    _say("autotune")
    (tmp_path / "cache.json").write_text("{not json")  # a corrupt cache is ignored and rewritten
    e = autotune.tune(dgvol.FORM_F64, 35, 3, target_bytes=32 << 20, min_tiles=1 << 10, reps=3)
    n = dgvol.variant_count(dgvol.FORM_F64, 35)
    assert 0 <= e["variant"] < n and 0 <= e["single_variant"] < n and e["tile_cost_s"] > 0
    assert set(e["candidates_s_per_tile"]) == {str(v) for v in range(n)}
    assert autotune.lookup(dgvol.FORM_F64, 35, 3, tune_missing=False)["variant"] == e["variant"]
    sizes = {2: 300, 4: 200, 6: 50}
    for N in sizes:
        autotune.tune(dgvol.FORM_F64, oracle.num_nodes(N), 3, target_bytes=16 << 20, min_tiles=1 << 10, reps=3)
    D, G, u = _mixed_case(sizes, 3, dgvol.FORM_F64, 4400)
    trip = [(dev(D[N]), dev(G[N]), dev(u[N])) for N in sizes]
    outs = autotune.volume_batched_tuned(trip)
    for N, o in zip(sizes, outs):
        check_planes(host(o), oracle.volume(D[N], G[N], u[N]), forward_cond(D[N], G[N], u[N]))
    # the chosen plan is cached under the batch's shapes
    p = autotune.plan_batch(trip, dgvol.FORM_F64)
    names = {"default", "tuned", "tuned_variants"}
    assert set(p.candidates) == names | {n + "_by_class" for n in names}
    assert len(p.variants) == len(p.costs) == 3 and isinstance(p.by_class, bool)
    assert min(p.candidates.values()) == p.candidates[min(p.candidates, key=p.candidates.get)]
