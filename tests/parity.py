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

FP64_TOL = 1e-12


def forward_cond(D, G, u):
    """sum_a |G[k,3a+b]| (|D_a| |u[k,f]|)[i] -> (3, K, F, Np)."""
    K = u.shape[0]
    absDu = np.einsum("aij,kfj->akfi", np.abs(D), np.abs(u))
    return np.einsum("kab,akfi->bkfi", np.abs(G).reshape(K, 3, 3), absDu)


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
