"""ctypes front end of the C oracle (``dg_oracle.c``) -- test infrastructure.

Arrays are NumPy, host memory, C-contiguous.  The library is built with gcc
(``-O2 -fopenmp -ffp-contract=off``) into ``oracle/libdgoracle.so``; it is
compiled on first use if it is not there, and ``build_library()`` recompiles
it unconditionally.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dg_oracle.c")
_LIB = os.path.join(_HERE, "libdgoracle.so")
_lib = None


def library_path():
    return _LIB


def build_library():
    """Compile dg_oracle.c with gcc; returns the path of the shared library."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-shared", "-fPIC", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_library()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    I64, I32 = ctypes.c_int64, ctypes.c_int32
    lib.oracle_volume.argtypes = [P, P, P, P, I64, I32, I32]
    lib.oracle_volume.restype = None
    lib.oracle_volume_adjoint.argtypes = [P, P, P, P, P, P, I64, I32, I32]
    lib.oracle_volume_adjoint.restype = None
    lib.oracle_volume_grad_d.argtypes = [P, P, P, P, I64, I32, I32]
    lib.oracle_volume_grad_d.restype = None
    lib.oracle_volume_split_bf16.argtypes = [P, P, P, P, I64, I32, I32]
    lib.oracle_volume_split_bf16.restype = None
    lib.oracle_bf16_round.argtypes = [P, P, I64]
    lib.oracle_bf16_round.restype = None
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def num_threads():
    """OpenMP threads the oracle runs on (OMP_NUM_THREADS, else all cores)."""
    return int(_load().oracle_num_threads())


def _c(x, dtype):
    x = np.ascontiguousarray(x, dtype=dtype)
    return x


def _check(D, G, u, K, Np, F):
    if D.shape != (3, Np, Np):
        raise ValueError(f"D must be (3, {Np}, {Np}), got {D.shape}")
    if G.shape != (K, 9):
        raise ValueError(f"G must be ({K}, 9), got {G.shape}")
    if u.shape != (K, F, Np):
        raise ValueError(f"u must be ({K}, {F}, {Np}), got {u.shape}")


def volume(D, G, u):
    """Forward volume derivative. D (3,Np,Np), G (K,9), u (K,F,Np) -> out (3,K,F,Np), FP64."""
    D, G, u = _c(D, np.float64), _c(G, np.float64), _c(u, np.float64)
    K, F, Np = u.shape
    _check(D, G, u, K, Np, F)
    out = np.empty((3, K, F, Np))
    _load().oracle_volume(D.ctypes.data, G.ctypes.data, u.ctypes.data, out.ctypes.data, K, Np, F)
    return out


def volume_adjoint(D, G, u, gout):
    """Adjoint of ``volume`` w.r.t. u and G for cotangent gout (3,K,F,Np) -> (gu, gG)."""
    D, G, u = _c(D, np.float64), _c(G, np.float64), _c(u, np.float64)
    gout = _c(gout, np.float64)
    K, F, Np = u.shape
    _check(D, G, u, K, Np, F)
    if gout.shape != (3, K, F, Np):
        raise ValueError(f"gout must be (3, {K}, {F}, {Np}), got {gout.shape}")
    gu = np.empty((K, F, Np))
    gG = np.empty((K, 9))
    _load().oracle_volume_adjoint(D.ctypes.data, G.ctypes.data, u.ctypes.data, gout.ctypes.data,
                                  gu.ctypes.data, gG.ctypes.data, K, Np, F)
    return gu, gG


def volume_grad_d(G, u, gout):
    """Cotangent of D for cotangent gout (3,K,F,Np): gD (3,Np,Np), a sum over all elements."""
    G, u, gout = _c(G, np.float64), _c(u, np.float64), _c(gout, np.float64)
    K, F, Np = u.shape
    if G.shape != (K, 9):
        raise ValueError(f"G must be ({K}, 9), got {G.shape}")
    if gout.shape != (3, K, F, Np):
        raise ValueError(f"gout must be (3, {K}, {F}, {Np}), got {gout.shape}")
    gD = np.empty((3, Np, Np))
    _load().oracle_volume_grad_d(G.ctypes.data, u.ctypes.data, gout.ctypes.data, gD.ctypes.data,
                                 K, Np, F)
    return gD


def volume_split_bf16(D32, G32, u32):
    """Three-pass split-BF16 product emulated exactly (FP64 accumulation); FP32 inputs, FP64 out."""
    D32, G32, u32 = _c(D32, np.float32), _c(G32, np.float32), _c(u32, np.float32)
    K, F, Np = u32.shape
    _check(D32, G32, u32, K, Np, F)
    out = np.empty((3, K, F, Np))
    _load().oracle_volume_split_bf16(D32.ctypes.data, G32.ctypes.data, u32.ctypes.data,
                                     out.ctypes.data, K, Np, F)
    return out


def bf16_round_f32(x):
    """Round FP32 values to BF16 (nearest, ties to even); result stored as FP32."""
    x = _c(x, np.float32)
    y = np.empty_like(x)
    _load().oracle_bf16_round(x.ctypes.data, y.ctypes.data, x.size)
    return y
