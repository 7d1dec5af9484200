"""Parity criteria shared by the GPU tests (GPU result vs the FP64 oracle).

FP64 ("1e-12 relative"): element-wise relative error is ill-posed where an
output is near zero through cancellation, so each output plane must meet both
  normwise:          max|gpu - ref| <= tol * max|ref|
  condition-scaled:  |gpu - ref| <= tol * cond   element by element,
where cond is the same sum taken over absolute values (for the forward map,
cond_b[i] = sum_a |G_ab| (|D_a| |u|)[i]).  Any summation order or FMA use is
within (3 Np + 3) * 2^-53 * cond, far inside tol = 1e-12.
"""

import numpy as np

import oracle

FP64_TOL = 1e-12


def forward_cond(D, G, u):
    """sum_a |G[k,3a+b]| (|D_a| |u[k,f]|)[i] -> (3, K, F, Np)."""
    K = u.shape[0]
    absDu = np.einsum("aij,kfj->akfi", np.abs(D), np.abs(u))
    return np.einsum("kab,akfi->bkfi", np.abs(G).reshape(K, 3, 3), absDu)


def forward_cond_c(D, G, u):
    """forward_cond through the C oracle: the forward map itself applied to |D|, |G|, |u|
    (the same sum of absolute values, fast at full workload sizes)."""
    return oracle.volume(np.abs(D), np.abs(G), np.abs(u))


def adjoint_cond_c(D, G, u, gout):
    """adjoint_cond through the C oracle: the adjoint applied to absolute values."""
    return oracle.volume_adjoint(np.abs(D), np.abs(G), np.abs(u), np.abs(gout))


def adjoint_cond(D, G, u, gout):
    """Absolute-value versions of gu and gG."""
    K = u.shape[0]
    absG = np.abs(G).reshape(K, 3, 3)
    absW = np.einsum("kab,bkfi->akfi", absG, np.abs(gout))
    cond_gu = np.einsum("aij,akfi->kfj", np.abs(D), absW)
    absR = np.einsum("aij,kfj->akfi", np.abs(D), np.abs(u))
    cond_gG = np.einsum("bkfi,akfi->kab", np.abs(gout), absR).reshape(K, 9)
    return cond_gu, cond_gG


def check_planes(gpu, ref, cond, tol=FP64_TOL, what="out"):
    """Normwise and condition-scaled check over the leading plane axis."""
    gpu = np.asarray(gpu)
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    assert np.isfinite(gpu).all(), f"{what}: non-finite values"
    for b in range(ref.shape[0]):
        err = np.abs(gpu[b] - ref[b])
        scale = np.abs(ref[b]).max() if ref[b].size else 0.0
        assert err.max(initial=0.0) <= tol * scale, \
            f"{what}[{b}]: normwise {err.max() / max(scale, 1e-300):.3e} > {tol}"
        bad = err > tol * cond[b]
        assert not bad.any(), f"{what}[{b}]: {int(bad.sum())} outputs beyond {tol} x condition"


def check_whole(gpu, ref, cond, tol=FP64_TOL, what="x"):
    check_planes(np.asarray(gpu)[None], np.asarray(ref)[None], np.asarray(cond)[None], tol, what)


# ------------------------------------------------------------------ split-BF16 form
#
# Stated bound against the FP64 result on the FP64 data, per output plane:
# max|err| <= 2e-5 max|ref| and ||err||_2 <= 1e-5 ||ref||_2.  Beyond that, the
# GPU result must sit within an a-priori FP32-accumulation bound of the exact
# three-pass emulation (oracle.volume_split_bf16, which forms the same BF16
# products and sums them in FP64):  |gpu - emu| <= (3 Np + 4) 2^-24 cond.
F32S_MAX_REL = 2e-5
F32S_RMS_REL = 1e-5


def split_errors(got, ref):
    """Per output plane: normwise max relative error max|e|/max|ref| and RMS relative
    error ||e||_2/||ref||_2 of got against ref (both (3, ...))."""
    res = []
    for b in range(ref.shape[0]):
        e = got[b] - ref[b]
        res.append({"max_rel": float(np.abs(e).max() / np.abs(ref[b]).max()),
                    "rms_rel": float(np.linalg.norm(e) / np.linalg.norm(ref[b]))})
    return res


def check_f32s(D, G, u, got):
    """got: the split-BF16 result (any float dtype) for the FP64 inputs D, G, u.  Asserts the
    stated bound and the emulation bound; returns the measured errors per plane against the
    FP64 oracle on the FP64 data ("vs_fp64") and on the FP32-rounded inputs promoted to FP64
    ("vs_fp32_inputs")."""
    Np = u.shape[2]
    got = np.asarray(got, dtype=np.float64)
    ref64 = oracle.volume(D, G, u)
    vs64 = split_errors(got, ref64)
    del ref64
    for b, e in enumerate(vs64):
        assert e["max_rel"] <= F32S_MAX_REL, f"plane {b}: max rel {e['max_rel']:.3e}"
        assert e["rms_rel"] <= F32S_RMS_REL, f"plane {b}: rms rel {e['rms_rel']:.3e}"
    D32, G32, u32 = D.astype(np.float32), G.astype(np.float32), u.astype(np.float32)
    D3, G3, u3 = D32.astype(np.float64), G32.astype(np.float64), u32.astype(np.float64)
    vs32 = split_errors(got, oracle.volume(D3, G3, u3))
    emu = oracle.volume_split_bf16(D32, G32, u32)
    cond = forward_cond_c(D3, G3, u3)
    tol = (3 * Np + 4) * 2.0 ** -24
    for b in range(3):
        bad = np.abs(got[b] - emu[b]) > tol * cond[b] + 1e-30
        assert not bad.any(), f"plane {b}: {int(bad.sum())} outputs beyond the FP32-accumulation bound"
    return {"vs_fp64": vs64, "vs_fp32_inputs": vs32}
