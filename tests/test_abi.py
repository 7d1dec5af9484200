"""The C ABI without a GPU: the library loads, exports every declared entry point,
and rejects bad arguments before making any HIP call.  Also the host-side setup
helpers of the library against the oracle."""

import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from oracle.exact import exact_derivative_matrices_f64
from paper_1503_07659_amd import dgvol, setup_host, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgvol.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(dgvol.LIB_PATH):
        pytest.fail("libdgvol.so is not built: run `python -m paper_1503_07659_amd.build`")
    return dgvol.load_library()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("dg_volume", "dg_volume_adjoint", "dg_volume_grad_d", "dg_volume_f32s", "dg_strerror",
                     "dg_supported_np", "dg_abi_version"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), f"{name} declared in dgvol.h but not exported"


def test_version_and_strerror(lib):
    assert lib.dg_abi_version() == 4
    for st in (0, -1, -2, -3, -4, -5, -99):
        msg = lib.dg_strerror(st)
        assert isinstance(msg, bytes) and msg
    assert [lib.dg_supported_np(n) for n in (4, 10, 20, 35, 56, 84, 120)] == [1] * 7
    assert [lib.dg_supported_np(n) for n in (0, 1, 5, 21, 36, 121, -4)] == [0] * 7


FAKE = 0x100000  # a non-null, 256-byte aligned address that is never dereferenced


@pytest.mark.parametrize("entry", ["dg_volume", "dg_volume_f32s"])
def test_forward_validation(lib, entry):
    f = getattr(lib, entry)
    s = None
    assert f(FAKE, FAKE, FAKE, FAKE, 0, 35, 5, s) == dgvol.DG_OK           # K == 0: no-op
    assert f(None, None, None, None, 0, 35, 5, s) == dgvol.DG_OK           # ... even with NULLs
    assert f(FAKE, FAKE, FAKE, FAKE, -1, 35, 5, s) == dgvol.DG_EINVAL
    assert f(FAKE, FAKE, FAKE, FAKE, 10, 35, 0, s) == dgvol.DG_EINVAL
    assert f(FAKE, FAKE, FAKE, FAKE, 10, 36, 5, s) == dgvol.DG_EUNSUPPORTED
    assert f(FAKE, FAKE, FAKE, FAKE, 10, 0, 5, s) == dgvol.DG_EUNSUPPORTED
    for i in range(4):
        ptrs = [FAKE] * 4
        ptrs[i] = None
        assert f(*ptrs, 10, 35, 5, s) == dgvol.DG_EINVAL
        ptrs[i] = FAKE + 2  # misaligned for both float and double
        assert f(*ptrs, 10, 35, 5, s) == dgvol.DG_EINVAL
    assert f(FAKE, FAKE, FAKE, FAKE, 1 << 30, 35, 4, s) == dgvol.DG_EINVAL  # K*F >= 2^31


def test_adjoint_validation(lib):
    f = lib.dg_volume_adjoint
    assert f(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 0, 56, 3, None) == dgvol.DG_OK
    assert f(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, -5, 56, 3, None) == dgvol.DG_EINVAL
    assert f(FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, 5, 57, 3, None) == dgvol.DG_EUNSUPPORTED
    for i in range(6):
        ptrs = [FAKE] * 6
        ptrs[i] = None
        assert f(*ptrs, 5, 56, 3, None) == dgvol.DG_EINVAL
        ptrs[i] = FAKE + 4
        assert f(*ptrs, 5, 56, 3, None) == dgvol.DG_EINVAL


def test_grad_d_workspace_and_validation(lib):
    ws = dgvol.grad_d_workspace_bytes
    # one partial sum per 128 columns, at most 1024 (Np <= 35) or 512, each 3 Np^2 doubles
    assert ws(0, 35, 5) == 0
    assert ws(1, 35, 1) == 3 * 35 * 35 * 8
    assert ws(128, 20, 1) == 3 * 20 * 20 * 8
    assert ws(129, 20, 1) == 2 * 3 * 20 * 20 * 8
    assert ws(43, 4, 3) == 2 * 3 * 4 * 4 * 8
    assert ws(1024 * 128 + 1, 35, 1) == 1024 * 3 * 35 * 35 * 8
    assert ws(512 * 128, 56, 1) == 512 * 3 * 56 * 56 * 8
    assert ws(1 << 20, 120, 5) == 512 * 3 * 120 * 120 * 8
    n = ctypes.c_uint64(0)
    assert lib.dg_volume_grad_d_workspace(10, 36, 1, ctypes.byref(n)) == dgvol.DG_EUNSUPPORTED
    assert lib.dg_volume_grad_d_workspace(-1, 35, 1, ctypes.byref(n)) == dgvol.DG_EINVAL
    assert lib.dg_volume_grad_d_workspace(10, 35, 0, ctypes.byref(n)) == dgvol.DG_EINVAL
    assert lib.dg_volume_grad_d_workspace(10, 35, 1, None) == dgvol.DG_EINVAL
    f = lib.dg_volume_grad_d
    need = ws(100, 35, 3)
    assert f(FAKE, FAKE, FAKE, FAKE, FAKE, need, -1, 35, 3, None) == dgvol.DG_EINVAL
    assert f(FAKE, FAKE, FAKE, FAKE, FAKE, need, 100, 35, 0, None) == dgvol.DG_EINVAL
    assert f(FAKE, FAKE, FAKE, FAKE, FAKE, need, 100, 34, 3, None) == dgvol.DG_EUNSUPPORTED
    assert f(FAKE, FAKE, FAKE, FAKE, FAKE, need - 8, 100, 35, 3, None) == dgvol.DG_EINVAL
    for i in range(5):
        ptrs = [FAKE] * 5
        ptrs[i] = None
        assert f(*ptrs, need, 100, 35, 3, None) == dgvol.DG_EINVAL
        ptrs[i] = FAKE + 4
        assert f(*ptrs, need, 100, 35, 3, None) == dgvol.DG_EINVAL
    # K == 0 still writes gD (zeros), so it needs gD, but nothing else
    assert f(FAKE, FAKE, FAKE, None, FAKE, 0, 0, 35, 3, None) == dgvol.DG_EINVAL


def test_grad_d_noalloc_validation(lib):
    """The fixed-scratch entry point validates like dg_volume_grad_d and rejects, before any
    HIP call, a problem whose partial sums exceed its 64 MiB scratch."""
    f = lib.dg_volume_grad_d_noalloc
    cap = dgvol.GRAD_D_NOALLOC_SCRATCH_BYTES
    assert cap == 64 << 20
    assert f(FAKE, FAKE, FAKE, FAKE, -1, 35, 3, None) == dgvol.DG_EINVAL
    assert f(FAKE, FAKE, FAKE, FAKE, 100, 35, 0, None) == dgvol.DG_EINVAL
    assert f(FAKE, FAKE, FAKE, FAKE, 100, 34, 3, None) == dgvol.DG_EUNSUPPORTED
    assert f(FAKE, FAKE, FAKE, None, 0, 35, 3, None) == dgvol.DG_EINVAL   # gD is written even for K == 0
    for i in range(4):
        ptrs = [FAKE] * 4
        ptrs[i] = None
        assert f(*ptrs, 100, 35, 3, None) == dgvol.DG_EINVAL
        ptrs[i] = FAKE + 4
        assert f(*ptrs, 100, 35, 3, None) == dgvol.DG_EINVAL
    # the largest problems that fit (header: K*F <= 50 688 at Np = 84, <= 24 832 at Np = 120),
    # and one column more, which is rejected
    for Np, cols in ((84, 50688), (120, 24832)):
        assert dgvol.grad_d_workspace_bytes(cols, Np, 1) <= cap
        assert dgvol.grad_d_workspace_bytes(cols + 1, Np, 1) > cap
        assert f(FAKE, FAKE, FAKE, FAKE, cols + 1, Np, 1, None) == dgvol.DG_ESCRATCH
        assert f(FAKE, FAKE, FAKE, FAKE, (cols + 1) * 4, Np, 4, None) == dgvol.DG_ESCRATCH
    # every problem size fits at Np <= 56
    for Np in (4, 10, 20, 35, 56):
        assert dgvol.grad_d_workspace_bytes(1 << 24, Np, 16) <= cap
    assert b"scratch" in lib.dg_strerror(dgvol.DG_ESCRATCH)


def test_stream_calibrate_tiles_validation(lib):
    f = lib.dg_stream_calibrate_tiles
    assert f(None, None, 0, 1, None) == dgvol.DG_OK           # nothing to move
    assert f(FAKE, FAKE, -1, 1, None) == dgvol.DG_EINVAL
    assert f(FAKE, FAKE, 10, -1, None) == dgvol.DG_EINVAL
    assert f(FAKE, FAKE, (1 << 31) // 560 + 1, 1, None) == dgvol.DG_EINVAL   # 560 ntiles words >= 2^31
    assert f(None, FAKE, 10, 1, None) == dgvol.DG_EINVAL
    assert f(FAKE, None, 10, 0, None) == dgvol.DG_EINVAL
    assert f(FAKE + 4, FAKE, 10, 1, None) == dgvol.DG_EINVAL
    assert f(FAKE, FAKE + 4, 10, 1, None) == dgvol.DG_EINVAL


def test_mfma_calibrate_validation(lib):
    assert lib.dg_mfma_calibrate(None, 10, None) == dgvol.DG_EINVAL
    assert lib.dg_mfma_calibrate(FAKE + 4, 10, None) == dgvol.DG_EINVAL
    assert lib.dg_mfma_calibrate(FAKE, 0, None) == dgvol.DG_EINVAL
    # products beside vector work: sink, counts and mode are validated before any launch
    assert lib.dg_mfma_calibrate_beside(None, 10, 10, dgvol.BESIDE_FP64_FMA, None) == dgvol.DG_EINVAL
    assert lib.dg_mfma_calibrate_beside(FAKE + 4, 10, 10, dgvol.BESIDE_FP64_FMA, None) == dgvol.DG_EINVAL
    assert lib.dg_mfma_calibrate_beside(FAKE, -1, 10, dgvol.BESIDE_FP64_FMA, None) == dgvol.DG_EINVAL
    assert lib.dg_mfma_calibrate_beside(FAKE, 10, -1, dgvol.BESIDE_FP64_FMA, None) == dgvol.DG_EINVAL
    assert lib.dg_mfma_calibrate_beside(FAKE, 0, 0, dgvol.BESIDE_FP64_FMA, None) == dgvol.DG_EINVAL
    assert lib.dg_mfma_calibrate_beside(FAKE, 10, 10, 4, None) == dgvol.DG_EINVAL
    assert lib.dg_mfma_calibrate_beside(FAKE, 10, 10, -1, None) == dgvol.DG_EINVAL


def test_python_binding_rejects_cpu_tensors():
    import torch
    u = torch.zeros((4, 1, 20), dtype=torch.float64)
    D = torch.zeros((3, 20, 20), dtype=torch.float64)
    G = torch.zeros((4, 9), dtype=torch.float64)
    with pytest.raises(ValueError):
        dgvol.dg_volume(D, G, u)
    with pytest.raises(TypeError):
        dgvol.dg_volume(D, G, u.float())
    with pytest.raises(ValueError):
        dgvol.dg_volume(D, G, torch.zeros((4, 1, 21), dtype=torch.float64))


# ----------------------------------------------------- host setup of the library vs the oracle

@pytest.mark.parametrize("N", range(1, 8))
def test_library_reference_matrices(N):
    D = setup_host.reference_matrices(N)
    E = np.array(exact_derivative_matrices_f64(N))
    assert D.shape == (3, oracle.num_nodes(N), oracle.num_nodes(N))
    # centred monomials: measured 8e-15 (N=5), 1.7e-13 (N=7) relative to max|D|
    assert np.abs(D - E).max() <= 1e-12 * np.abs(E).max()
    assert np.array_equal(setup_host.reference_nodes(N), oracle.equispaced_nodes(N))


def test_library_geometric_factors():
    v = synth.tet_vertices(2000, seed=17)
    assert np.abs(setup_host.geometric_factors(v) - oracle.geometric_factors(v)).max() < 1e-14
    bad = v.copy()
    bad[5, 3] = bad[5, 0]
    with pytest.raises(ValueError):
        setup_host.geometric_factors(bad)


def _groups(n, **kw):
    arr = (dgvol.DgGroup * max(n, 1))()
    for i in range(n):
        arr[i].Np, arr[i].variant, arr[i].K = kw.get("Np", 35), kw.get("variant", -1), kw.get("K", 10)
        arr[i].D = arr[i].G = arr[i].u = arr[i].out = kw.get("ptr", FAKE)
        arr[i].cost = 0.0
    return arr


def test_batched_validation(lib):
    f = lib.dg_volume_batched
    assert ctypes.sizeof(dgvol.DgGroup) == 56
    assert f(_groups(0), 0, 3, dgvol.FORM_F64, None) == dgvol.DG_OK
    assert f(_groups(3, K=0), 3, 3, dgvol.FORM_F64, None) == dgvol.DG_OK        # all empty: no-op
    assert f(_groups(17), 17, 3, dgvol.FORM_F64, None) == dgvol.DG_EINVAL       # too many groups
    assert f(_groups(2), -1, 3, dgvol.FORM_F64, None) == dgvol.DG_EINVAL
    assert f(_groups(2), 2, 0, dgvol.FORM_F64, None) == dgvol.DG_EINVAL         # F < 1
    assert f(_groups(2), 2, 3, 7, None) == dgvol.DG_EUNSUPPORTED               # unknown form
    assert f(_groups(2), 2, 3, dgvol.FORM_F64 | 0x200, None) == dgvol.DG_EUNSUPPORTED   # unknown flag
    assert f(_groups(2), 2, 3, 7 | dgvol.BATCH_BY_CLASS, None) == dgvol.DG_EUNSUPPORTED
    assert f(_groups(3, K=0), 3, 3, dgvol.FORM_F32S | dgvol.BATCH_BY_CLASS, None) == dgvol.DG_OK
    assert f(_groups(2, Np=36), 2, 3, dgvol.FORM_F64, None) == dgvol.DG_EUNSUPPORTED
    assert f(_groups(2, K=-1), 2, 3, dgvol.FORM_F64, None) == dgvol.DG_EINVAL
    assert f(_groups(2, ptr=None), 2, 3, dgvol.FORM_F64, None) == dgvol.DG_EINVAL
    assert f(_groups(2, ptr=FAKE + 4), 2, 3, dgvol.FORM_F64, None) == dgvol.DG_EINVAL  # misaligned double
    assert f(_groups(2, variant=15), 2, 3, dgvol.FORM_F64, None) == dgvol.DG_EUNSUPPORTED
    assert f(_groups(2, variant=-2), 2, 3, dgvol.FORM_F64, None) == dgvol.DG_EUNSUPPORTED
    # order 7 (Np = 120) has one FP64 variant: index 1 is refused even for an empty group
    assert f(_groups(1, Np=120, variant=1, K=0), 1, 3, dgvol.FORM_F64, None) == dgvol.DG_EUNSUPPORTED
    assert f(None, 1, 3, dgvol.FORM_F64, None) == dgvol.DG_EINVAL


def test_variant_tables(lib):
    """Every (form, Np) has variants; variant 0 is the default; the staged FP64 body, which keeps
    D in LDS, is not offered where D does not fit (Np = 84, 120); every variant fits the LDS of a
    CU and its class matches its workgroup size."""
    seen_bodies = set()
    for form in (dgvol.FORM_F64, dgvol.FORM_F32S):
        for Np in (4, 10, 20, 35, 56, 84, 120):
            n = lib.dg_variant_count(form, Np)
            assert 1 <= n <= 16
            shapes = set()
            for v in range(n):
                info = dgvol.variant_info(form, Np, v)
                assert info["body"] in (dgvol.BODY_STAGED, dgvol.BODY_CHUNKREG, dgvol.BODY_STAGED_LEAN)
                if info["body"] == dgvol.BODY_STAGED_LEAN:  # held to two 8-wave workgroups per CU
                    assert form == dgvol.FORM_F64 and info["waves"] == 8 and info["batch_class"] == 0
                assert info["waves"] in (4, 8) and info["tiles"] in (1, 2, 4, 8)
                assert 0 < info["lds_bytes"] <= 160 * 1024
                assert (info["batch_class"] == 2) == (info["waves"] == 4)
                if form == dgvol.FORM_F64 and Np >= 84:
                    assert info["body"] == dgvol.BODY_CHUNKREG
                if info["batch_class"] == 0:  # LIGHT: two 8-wave workgroups must fit the LDS of a CU
                    assert 2 * info["lds_bytes"] <= 160 * 1024
                key = (info["body"], info["waves"], info["tiles"])
                assert key not in shapes, f"duplicate variant {key} for form {form} Np {Np}"
                shapes.add(key)
                seen_bodies.add((form, info["body"]))
            info = dgvol.DgVariantInfo()
            assert lib.dg_variant_query(form, Np, n, ctypes.byref(info)) == dgvol.DG_EUNSUPPORTED
            assert lib.dg_variant_query(form, Np, -1, ctypes.byref(info)) == dgvol.DG_EUNSUPPORTED
            assert lib.dg_variant_query(form, Np, 0, None) == dgvol.DG_EINVAL
    assert len(seen_bodies) == 5
    assert lib.dg_variant_count(dgvol.FORM_F64, 36) == 0
    assert lib.dg_variant_count(5, 35) == 0
    # the defaults the single-group entry points use
    assert dgvol.variant_info(dgvol.FORM_F64, 35, 0)["body"] == dgvol.BODY_STAGED
    assert dgvol.variant_info(dgvol.FORM_F64, 120, 0)["body"] == dgvol.BODY_CHUNKREG


def test_variant_entry_validation(lib):
    f = lib.dg_volume_variant
    F64, F32 = dgvol.FORM_F64, dgvol.FORM_F32S
    assert f(F64, -1, FAKE, FAKE, FAKE, FAKE, 0, 35, 5, None) == dgvol.DG_OK
    assert f(F64, 1, FAKE, FAKE, FAKE, FAKE, 0, 35, 5, None) == dgvol.DG_OK
    assert f(F64, 9, FAKE, FAKE, FAKE, FAKE, 0, 35, 5, None) == dgvol.DG_EUNSUPPORTED
    assert f(F64, -2, FAKE, FAKE, FAKE, FAKE, 10, 35, 5, None) == dgvol.DG_EUNSUPPORTED
    assert f(3, 0, FAKE, FAKE, FAKE, FAKE, 10, 35, 5, None) == dgvol.DG_EUNSUPPORTED
    assert f(F64, 0, FAKE, FAKE, FAKE, FAKE, 10, 36, 5, None) == dgvol.DG_EUNSUPPORTED
    assert f(F64, 0, FAKE, FAKE, FAKE, FAKE, -1, 35, 5, None) == dgvol.DG_EINVAL
    for i in range(4):
        ptrs = [FAKE] * 4
        ptrs[i] = None
        assert f(F32, 0, *ptrs, 10, 35, 5, None) == dgvol.DG_EINVAL
        ptrs[i] = FAKE + 4  # fine for float, misaligned for double
        assert f(F64, 0, *ptrs, 10, 35, 5, None) == dgvol.DG_EINVAL
        ptrs[i] = FAKE + 2
        assert f(F32, 0, *ptrs, 10, 35, 5, None) == dgvol.DG_EINVAL
    sh = dgvol.DgLaunchShape()
    q = lib.dg_launch_shape_query
    assert q(dgvol.OP_FORWARD, F64, 35, 0, 10, 5, None) == dgvol.DG_EINVAL
    assert q(dgvol.OP_FORWARD, F64, 35, 0, 0, 5, ctypes.byref(sh)) == dgvol.DG_EINVAL
    assert q(dgvol.OP_FORWARD, F64, 35, 0, 10, 0, ctypes.byref(sh)) == dgvol.DG_EINVAL
    assert q(7, F64, 35, 0, 10, 5, ctypes.byref(sh)) == dgvol.DG_EINVAL
    assert q(dgvol.OP_FORWARD, F64, 36, 0, 10, 5, ctypes.byref(sh)) == dgvol.DG_EUNSUPPORTED
    assert q(dgvol.OP_FORWARD, F64, 35, 12, 10, 5, ctypes.byref(sh)) == dgvol.DG_EUNSUPPORTED


def test_autotune_cache_io(tmp_path, monkeypatch):
    """Cache file handling needs no GPU: corrupt or foreign content is ignored."""
    from paper_1503_07659_amd import autotune
    p = tmp_path / "c.json"
    monkeypatch.setenv("DGVOL_AUTOTUNE_CACHE", str(p))
    assert autotune.load_cache() == {}
    p.write_text("[1, 2")
    assert autotune.load_cache() == {}
    p.write_text("[1, 2]")
    assert autotune.load_cache() == {}
    autotune.save_cache({"gfx950/abi2": {"f64/Np35/F3": {"variant": 0, "tile_cost_s": 1e-7}}})
    assert autotune.load_cache()["gfx950/abi2"]["f64/Np35/F3"]["variant"] == 0
    ok = {"variant": 1, "single_variant": 0, "tile_cost_s": 2e-7, "by_class_variant": 2, "by_class_tile_cost_s": 3e-7}
    assert autotune._valid_entry(ok, dgvol.FORM_F64, 35)
    assert not autotune._valid_entry(dict(ok, by_class_tile_cost_s=0.0), dgvol.FORM_F64, 35)
    old_entry = {k: v for k, v in ok.items() if not k.startswith("by_class")}
    assert not autotune._valid_entry(old_entry, dgvol.FORM_F64, 35)   # an entry without both modes is retuned
    assert not autotune._valid_entry(dict(ok, tile_cost_s=-1), dgvol.FORM_F64, 35)
    assert not autotune._valid_entry(dict(ok, variant="x"), dgvol.FORM_F64, 35)
    assert not autotune._valid_entry(dict(ok, variant=1, by_class_variant=0), dgvol.FORM_F64, 120)  # one FP64 variant
    assert not autotune._valid_entry(dict(ok, single_variant=99), dgvol.FORM_F64, 35)
    assert autotune.entry_key(1, 120, 3) == "f32s/Np120/F3"
