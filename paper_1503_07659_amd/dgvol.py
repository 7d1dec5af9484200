"""Python binding of libdgvol.so (argument marshalling only).

The functions named like the C entry points (``dg_volume``,
``dg_volume_adjoint``, ``dg_volume_grad_d``, ``dg_volume_grad_d_noalloc``, ``dg_volume_f32s``,
``dg_volume_variant``, ``dg_volume_batched`` and the two calibration calls) take torch tensors on the
GPU, check dtype/device/shape/contiguity, and pass raw device pointers plus
torch's current HIP stream to the library.  Every arithmetic step runs in the
HIP kernels; there is no CPU or PyTorch fallback: if the library is missing or
fails to load, every call raises.

``DGVolume`` is a ``torch.autograd.Function``: its backward calls the adjoint
kernels for the gradients with respect to u and G, and ``dg_volume_grad_d``
for the gradient with respect to D when D requires one.
"""

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdgvol.so")

DG_OK = 0
DG_EINVAL = -1
DG_EUNSUPPORTED = -2
DG_ELAUNCH = -3
DG_EDEVICE = -4
DG_ESCRATCH = -5

# fixed scratch of dg_volume_grad_d_noalloc (DG_GRAD_D_NOALLOC_SCRATCH_BYTES)
GRAD_D_NOALLOC_SCRATCH_BYTES = 64 << 20

SUPPORTED_NP = (4, 10, 20, 35, 56, 84, 120)

FORM_F64 = 0
FORM_F32S = 1
BODY_STAGED = 0
BODY_CHUNKREG = 1
BODY_STAGED_LEAN = 2
VARIANT_AUTO = -1
MAX_GROUPS = 16

OP_FORWARD = 0
OP_BATCHED = 1
OP_ADJOINT = 2
OP_BATCHED_BY_CLASS = 3

# dg_volume_batched: one launch per variant class instead of one launch for all 8-wave groups
BATCH_BY_CLASS = 0x100


class DgGroup(ctypes.Structure):
    """Mirror of `dg_group` in dgvol.h."""
    _fields_ = [("Np", ctypes.c_int32), ("variant", ctypes.c_int32), ("K", ctypes.c_int64),
                ("D", ctypes.c_void_p), ("G", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("cost", ctypes.c_double)]


class DgVariantInfo(ctypes.Structure):
    """Mirror of `dg_variant_info` in dgvol.h."""
    _fields_ = [("body", ctypes.c_int32), ("waves", ctypes.c_int32), ("tiles", ctypes.c_int32),
                ("batch_class", ctypes.c_int32), ("lds_bytes", ctypes.c_int32)]


class DgLaunchShape(ctypes.Structure):
    """Mirror of `dg_launch_shape` in dgvol.h."""
    _fields_ = [(name, ctypes.c_uint32) for name in
                ("grid", "block", "lds_bytes", "resident", "units", "units_per_step", "min_iters", "max_iters")]

_lib = None


class DGVolError(RuntimeError):
    """A library call returned a negative status."""

    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def load_library(path=None):
    """Load libdgvol.so (once).  Raises RuntimeError if it is not built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"HIP library {p} is not built; run `python -m paper_1503_07659_amd.build`")
    lib = ctypes.CDLL(p)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.dg_abi_version.argtypes = []
    lib.dg_abi_version.restype = I32
    lib.dg_strerror.argtypes = [I32]
    lib.dg_strerror.restype = ctypes.c_char_p
    lib.dg_supported_np.argtypes = [I32]
    lib.dg_supported_np.restype = I32
    lib.dg_volume.argtypes = [P, P, P, P, I64, I32, I32, P]
    lib.dg_volume.restype = I32
    lib.dg_volume_adjoint.argtypes = [P, P, P, P, P, P, I64, I32, I32, P]
    lib.dg_volume_adjoint.restype = I32
    lib.dg_volume_grad_d.argtypes = [P, P, P, P, P, ctypes.c_uint64, I64, I32, I32, P]
    lib.dg_volume_grad_d.restype = I32
    lib.dg_volume_grad_d_noalloc.argtypes = [P, P, P, P, I64, I32, I32, P]
    lib.dg_volume_grad_d_noalloc.restype = I32
    lib.dg_volume_grad_d_workspace.argtypes = [I64, I32, I32, ctypes.POINTER(ctypes.c_uint64)]
    lib.dg_volume_grad_d_workspace.restype = I32
    lib.dg_volume_f32s.argtypes = [P, P, P, P, I64, I32, I32, P]
    lib.dg_volume_f32s.restype = I32
    lib.dg_stream_calibrate.argtypes = [P, P, I64, I32, P]
    lib.dg_stream_calibrate.restype = I32
    lib.dg_stream_calibrate_tiles.argtypes = [P, P, I64, I32, P]
    lib.dg_stream_calibrate_tiles.restype = I32
    lib.dg_mfma_calibrate.argtypes = [P, I32, P]
    lib.dg_mfma_calibrate.restype = I32
    lib.dg_mfma_calibrate_beside.argtypes = [P, I32, I32, I32, P]
    lib.dg_mfma_calibrate_beside.restype = I32
    lib.dg_volume_batched.argtypes = [ctypes.POINTER(DgGroup), I32, I32, I32, P]
    lib.dg_volume_batched.restype = I32
    lib.dg_variant_count.argtypes = [I32, I32]
    lib.dg_variant_count.restype = I32
    lib.dg_variant_query.argtypes = [I32, I32, I32, ctypes.POINTER(DgVariantInfo)]
    lib.dg_variant_query.restype = I32
    lib.dg_volume_variant.argtypes = [I32, I32, P, P, P, P, I64, I32, I32, P]
    lib.dg_volume_variant.restype = I32
    lib.dg_launch_shape_query.argtypes = [I32, I32, I32, I32, I64, I32, ctypes.POINTER(DgLaunchShape)]
    lib.dg_launch_shape_query.restype = I32
    if path is None:
        _lib = lib
    return lib


def strerror(status):
    return load_library().dg_strerror(int(status)).decode()


def _raise_on(status, what):
    if status != DG_OK:
        raise DGVolError(status, f"{what}: {strerror(status)}")


def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_tensor(name, t, dtype, shape, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU, got {t.device}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _sizes(u):
    if u.dim() != 3:
        raise ValueError(f"u must be (K, F, Np), got shape {tuple(u.shape)}")
    K, F, Np = u.shape
    if Np not in SUPPORTED_NP:
        raise ValueError(f"unsupported node count Np={Np}; supported: {SUPPORTED_NP}")
    return K, F, Np


def dg_volume(D, G, u, out=None):
    """FP64 forward: out[b,k,f,i] = sum_a G[k,3a+b] (D_a u[k,f])[i]; returns out (3, K, F, Np)."""
    K, F, Np = _sizes(u)
    dev = u.device
    _check_tensor("u", u, torch.float64, (K, F, Np))
    _check_tensor("D", D, torch.float64, (3, Np, Np), dev)
    _check_tensor("G", G, torch.float64, (K, 9), dev)
    if out is None:
        out = torch.empty((3, K, F, Np), dtype=torch.float64, device=dev)
    _check_tensor("out", out, torch.float64, (3, K, F, Np), dev)
    with torch.cuda.device(dev):
        st = load_library().dg_volume(D.data_ptr(), G.data_ptr(), u.data_ptr(), out.data_ptr(),
                                      K, Np, F, _stream_handle(dev))
    _raise_on(st, "dg_volume")
    return out


def dg_volume_adjoint(D, G, u, gout, gu=None, gG=None):
    """FP64 adjoint w.r.t. u and G for the cotangent gout (3, K, F, Np); returns (gu, gG)."""
    K, F, Np = _sizes(u)
    dev = u.device
    _check_tensor("u", u, torch.float64, (K, F, Np))
    _check_tensor("D", D, torch.float64, (3, Np, Np), dev)
    _check_tensor("G", G, torch.float64, (K, 9), dev)
    _check_tensor("gout", gout, torch.float64, (3, K, F, Np), dev)
    if gu is None:
        gu = torch.empty((K, F, Np), dtype=torch.float64, device=dev)
    if gG is None:
        gG = torch.empty((K, 9), dtype=torch.float64, device=dev)
    _check_tensor("gu", gu, torch.float64, (K, F, Np), dev)
    _check_tensor("gG", gG, torch.float64, (K, 9), dev)
    with torch.cuda.device(dev):
        st = load_library().dg_volume_adjoint(D.data_ptr(), G.data_ptr(), u.data_ptr(), gout.data_ptr(),
                                              gu.data_ptr(), gG.data_ptr(), K, Np, F, _stream_handle(dev))
    _raise_on(st, "dg_volume_adjoint")
    return gu, gG


def grad_d_workspace_bytes(K, Np, F):
    """Scratch bytes dg_volume_grad_d needs for (K, Np, F) (host computation)."""
    n = ctypes.c_uint64(0)
    _raise_on(load_library().dg_volume_grad_d_workspace(int(K), int(Np), int(F), ctypes.byref(n)),
              "dg_volume_grad_d_workspace")
    return int(n.value)


def dg_volume_grad_d(G, u, gout, gD=None, work=None):
    """FP64 cotangent of D (3, Np, Np) for the cotangent gout (3, K, F, Np) of dg_volume.

    ``work`` is optional device scratch (uint8, at least ``grad_d_workspace_bytes``);
    one is allocated when it is not given."""
    _check_tensor("u", u, torch.float64, tuple(u.shape))
    K, F, Np = _sizes(u)
    dev = u.device
    _check_tensor("G", G, torch.float64, (K, 9), dev)
    _check_tensor("gout", gout, torch.float64, (3, K, F, Np), dev)
    if gD is None:
        gD = torch.empty((3, Np, Np), dtype=torch.float64, device=dev)
    _check_tensor("gD", gD, torch.float64, (3, Np, Np), dev)
    need = grad_d_workspace_bytes(K, Np, F)
    if work is None:
        work = torch.empty(max(need, 8), dtype=torch.uint8, device=dev)
    if not isinstance(work, torch.Tensor) or work.device != dev or not work.is_contiguous():
        raise ValueError("work must be a contiguous tensor on the device of u")
    nbytes = work.numel() * work.element_size()
    with torch.cuda.device(dev):
        st = load_library().dg_volume_grad_d(G.data_ptr(), u.data_ptr(), gout.data_ptr(), gD.data_ptr(),
                                             work.data_ptr(), nbytes, K, Np, F, _stream_handle(dev))
    _raise_on(st, "dg_volume_grad_d")
    return gD


def dg_volume_grad_d_noalloc(G, u, gout, gD):
    """dg_volume_grad_d through the library's fixed scratch: the call allocates nothing (the
    caller passes the output gD).  Raises DGVolError with status DG_ESCRATCH for a problem
    whose partial sums exceed GRAD_D_NOALLOC_SCRATCH_BYTES.  Calls that overlap in time on
    one device share its scratch and race."""
    _check_tensor("u", u, torch.float64, tuple(u.shape))
    K, F, Np = _sizes(u)
    dev = u.device
    _check_tensor("G", G, torch.float64, (K, 9), dev)
    _check_tensor("gout", gout, torch.float64, (3, K, F, Np), dev)
    _check_tensor("gD", gD, torch.float64, (3, Np, Np), dev)
    with torch.cuda.device(dev):
        st = load_library().dg_volume_grad_d_noalloc(G.data_ptr(), u.data_ptr(), gout.data_ptr(), gD.data_ptr(),
                                                     K, Np, F, _stream_handle(dev))
    _raise_on(st, "dg_volume_grad_d_noalloc")
    return gD


def dg_volume_f32s(D, G, u, out=None):
    """FP32 storage, split-BF16 products: same contract as dg_volume with float32 tensors."""
    K, F, Np = _sizes(u)
    dev = u.device
    _check_tensor("u", u, torch.float32, (K, F, Np))
    _check_tensor("D", D, torch.float32, (3, Np, Np), dev)
    _check_tensor("G", G, torch.float32, (K, 9), dev)
    if out is None:
        out = torch.empty((3, K, F, Np), dtype=torch.float32, device=dev)
    _check_tensor("out", out, torch.float32, (3, K, F, Np), dev)
    with torch.cuda.device(dev):
        st = load_library().dg_volume_f32s(D.data_ptr(), G.data_ptr(), u.data_ptr(), out.data_ptr(),
                                           K, Np, F, _stream_handle(dev))
    _raise_on(st, "dg_volume_f32s")
    return out


def dg_volume_variant(form, variant, D, G, u, out=None):
    """Forward product of one group with an explicit launch variant (VARIANT_AUTO or an index
    below variant_count(form, Np)); float64 tensors for FORM_F64, float32 for FORM_F32S."""
    K, F, Np = _sizes(u)
    dev = u.device
    dtype = torch.float64 if form == FORM_F64 else torch.float32
    _check_tensor("u", u, dtype, (K, F, Np))
    _check_tensor("D", D, dtype, (3, Np, Np), dev)
    _check_tensor("G", G, dtype, (K, 9), dev)
    if out is None:
        out = torch.empty((3, K, F, Np), dtype=dtype, device=dev)
    _check_tensor("out", out, dtype, (3, K, F, Np), dev)
    with torch.cuda.device(dev):
        st = load_library().dg_volume_variant(int(form), int(variant), D.data_ptr(), G.data_ptr(), u.data_ptr(),
                                              out.data_ptr(), K, Np, F, _stream_handle(dev))
    _raise_on(st, "dg_volume_variant")
    return out


def variant_count(form, Np):
    """Number of compiled launch variants of the forward product for (form, Np)."""
    return int(load_library().dg_variant_count(int(form), int(Np)))


def variant_info(form, Np, variant):
    """dict(body, waves, tiles, batch_class, lds_bytes) of one variant (host query)."""
    info = DgVariantInfo()
    _raise_on(load_library().dg_variant_query(int(form), int(Np), int(variant), ctypes.byref(info)),
              "dg_variant_query")
    return {f: int(getattr(info, f)) for f, _ in DgVariantInfo._fields_}


def launch_shape(op, form, Np, variant, K, F):
    """Grid, occupancy and loop iterations an operation would use on the current device."""
    sh = DgLaunchShape()
    _raise_on(load_library().dg_launch_shape_query(int(op), int(form), int(Np), int(variant), int(K), int(F),
                                                   ctypes.byref(sh)), "dg_launch_shape_query")
    return {f: int(getattr(sh, f)) for f, _ in DgLaunchShape._fields_}


def dg_volume_batched(groups, form=FORM_F64, outs=None, variants=None, costs=None, by_class=False):
    """Forward derivative of several element groups (possibly different orders): one persistent
    launch for every group with an 8-wave variant (and one for 4-wave variants), or, with
    by_class, one launch per variant class.

    groups: sequence of (D, G, u) tensor triples sharing F and the form's dtype
    (float64 for FORM_F64, float32 for FORM_F32S).  outs: optional matching
    output tensors (3, K, F, Np).  variants: optional per-group variant index
    (VARIANT_AUTO or below variant_count).  costs: optional measured cost of
    one 16-column tile per group (sets the split of workgroups).  Returns outs.
    """
    if len(groups) > MAX_GROUPS:
        raise ValueError(f"at most {MAX_GROUPS} groups per launch")
    dtype = torch.float64 if form == FORM_F64 else torch.float32
    if not groups:
        return []
    F = groups[0][2].shape[1] if groups[0][2].dim() == 3 else None
    dev = groups[0][2].device
    arr = (DgGroup * max(1, len(groups)))()
    res = []
    for gi, (D, G, u) in enumerate(groups):
        K, Fg, Np = _sizes(u)
        if Fg != F:
            raise ValueError("all groups of a batch share F")
        _check_tensor("u", u, dtype, (K, F, Np), dev)
        _check_tensor("D", D, dtype, (3, Np, Np), dev)
        _check_tensor("G", G, dtype, (K, 9), dev)
        out = outs[gi] if outs is not None else torch.empty((3, K, F, Np), dtype=dtype, device=dev)
        _check_tensor("out", out, dtype, (3, K, F, Np), dev)
        res.append(out)
        arr[gi].Np = Np
        arr[gi].variant = VARIANT_AUTO if variants is None else int(variants[gi])
        arr[gi].K = K
        arr[gi].D, arr[gi].G, arr[gi].u, arr[gi].out = D.data_ptr(), G.data_ptr(), u.data_ptr(), out.data_ptr()
        arr[gi].cost = 0.0 if costs is None else float(costs[gi])
    with torch.cuda.device(dev):
        flags = int(form) | (BATCH_BY_CLASS if by_class else 0)
        st = load_library().dg_volume_batched(arr, len(groups), int(F), flags, _stream_handle(dev))
    _raise_on(st, "dg_volume_batched")
    return res


def dg_stream_calibrate(src, dst, copies):
    """Bandwidth calibration: dst[c*n + i] = (c + 1) * src[i] for c < copies (1..3); FP64."""
    n = src.numel()
    dev = src.device
    _check_tensor("src", src, torch.float64, (n,))
    _check_tensor("dst", dst, torch.float64, (copies * n,), dev)
    with torch.cuda.device(dev):
        st = load_library().dg_stream_calibrate(src.data_ptr(), dst.data_ptr(), n, copies, _stream_handle(dev))
    _raise_on(st, "dg_stream_calibrate")
    return dst


MFMA_CAL_BLOCKS = 2048


TILE_STREAM_WORDS = 16 * 35  # doubles per tile of dg_stream_calibrate_tiles


def dg_stream_calibrate_tiles(src, dst, tiles_per_wave):
    """Tile-stream calibration: src (ntiles * 560 doubles), dst (3 * ntiles * 560 doubles);
    tiles_per_wave = 0 is the forward's persistent launch shape, m >= 1 a grid of m tiles per wave."""
    for name, t in (("src", src), ("dst", dst)):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or t.device.type != "cuda" \
                or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 GPU tensor")
    if src.numel() % TILE_STREAM_WORDS:
        raise ValueError(f"src must hold whole tiles of {TILE_STREAM_WORDS} doubles")
    ntiles = src.numel() // TILE_STREAM_WORDS
    if dst.numel() != 3 * src.numel():
        raise ValueError("dst must hold three planes of src's size")
    with torch.cuda.device(src.device):
        st = load_library().dg_stream_calibrate_tiles(src.data_ptr(), dst.data_ptr(), ntiles, int(tiles_per_wave),
                                                      _stream_handle(src.device))
    _raise_on(st, "dg_stream_calibrate_tiles")


def dg_mfma_calibrate(iters, sink=None):
    """Run the FP64 matrix-core calibration kernel; returns (sink, flops executed)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    if sink is None:
        sink = torch.empty(MFMA_CAL_BLOCKS * 256, dtype=torch.float64, device=dev)
    _check_tensor("sink", sink, torch.float64, (MFMA_CAL_BLOCKS * 256,))
    with torch.cuda.device(sink.device):
        st = load_library().dg_mfma_calibrate(sink.data_ptr(), int(iters), _stream_handle(sink.device))
    _raise_on(st, "dg_mfma_calibrate")
    return sink, MFMA_CAL_BLOCKS * 4 * int(iters) * 4 * 2048


MFMA_BESIDE_BLOCKS = 256
BESIDE_NONE, BESIDE_FP64_FMA, BESIDE_INT, BESIDE_DPP = 0, 1, 2, 3


def dg_mfma_calibrate_beside(iters, viters, mode, sink=None):
    """FP64 matrix products (waves 0..3 of each workgroup) beside `viters` rounds of 16 vector
    instructions of kind `mode` (waves 4..7, the same SIMDs); returns the sink."""
    dev = torch.device("cuda", torch.cuda.current_device())
    if sink is None:
        sink = torch.empty(MFMA_BESIDE_BLOCKS * 512, dtype=torch.float64, device=dev)
    _check_tensor("sink", sink, torch.float64, (MFMA_BESIDE_BLOCKS * 512,))
    with torch.cuda.device(sink.device):
        st = load_library().dg_mfma_calibrate_beside(sink.data_ptr(), int(iters), int(viters), int(mode),
                                                     _stream_handle(sink.device))
    _raise_on(st, "dg_mfma_calibrate_beside")
    return sink


class DGVolume(torch.autograd.Function):
    """out = dg_volume(D, G, u) with gradients for u and G from the adjoint kernel
    and, when D requires one, for D from dg_volume_grad_d.

    Call as ``DGVolume.apply(u, G, D)``.
    """

    @staticmethod
    def forward(ctx, u, G, D):
        u = u.contiguous()
        G = G.contiguous()
        D = D.contiguous()
        ctx.save_for_backward(u, G, D)
        return dg_volume(D, G, u)

    @staticmethod
    def backward(ctx, gout):
        u, G, D = ctx.saved_tensors
        gout = gout.contiguous()
        gu = gG = gD = None
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            gu, gG = dg_volume_adjoint(D, G, u, gout)
        if ctx.needs_input_grad[2]:
            gD = dg_volume_grad_d(G, u, gout)
        return (gu if ctx.needs_input_grad[0] else None,
                gG if ctx.needs_input_grad[1] else None,
                gD)


def volume(u, G, D):
    """Differentiable forward volume derivative (FP64): ``DGVolume.apply(u, G, D)``."""
    return DGVolume.apply(u, G, D)
