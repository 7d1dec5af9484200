"""Autotuner for the mixed-order batched launch.

For every (form, Np, F) it times each available kernel body
(``dg_body_available``) as a one-group batched launch on a synthetic problem
large enough to fill the GPU, keeps the fastest, and records the measured
time of one 16-column tile.  That time is the ``cost`` the batched launch
uses to split its persistent workgroups between groups, so the split follows
measured rather than estimated work.

Results are cached in a JSON file (``$DGVOL_AUTOTUNE_CACHE``, default
``~/.cache/dgvol/autotune.json``) keyed by the GPU architecture and the
library ABI version; an unreadable, corrupt or foreign cache is ignored and
rewritten.  Tuning needs a GPU; looking up the cache does not.
"""

import json
import os
import tempfile

import numpy as np
import torch

from . import dgvol

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dgvol", "autotune.json")
FORM_NAMES = {dgvol.FORM_F64: "f64", dgvol.FORM_F32S: "f32s"}
ORDER_OF_NP = {4: 1, 10: 2, 20: 3, 35: 4, 56: 5, 84: 6, 120: 7}


def cache_path():
    return os.environ.get("DGVOL_AUTOTUNE_CACHE", DEFAULT_CACHE)


def device_key(device=None):
    """Cache namespace: architecture of the device and ABI version of the library."""
    props = torch.cuda.get_device_properties(device or torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    return f"{arch}/abi{dgvol.load_library().dg_abi_version()}"


def entry_key(form, Np, F):
    return f"{FORM_NAMES[form]}/Np{Np}/F{F}"


def load_cache(path=None):
    """The cache as a dict; {} if missing or unreadable."""
    p = path or cache_path()
    try:
        with open(p) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(data, path=None):
    p = path or cache_path()
    d = os.path.dirname(p)
    if d:
        os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".autotune.")
    with os.fdopen(fd, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _valid_entry(e):
    return (isinstance(e, dict) and isinstance(e.get("body"), int) and
            isinstance(e.get("tile_cost_s"), (int, float)) and e["tile_cost_s"] > 0)


def _synthetic(form, Np, F, K, device):
    """Inputs with the shape of one group (values only need to be finite)."""
    dtype = torch.float64 if form == dgvol.FORM_F64 else torch.float32
    g = torch.Generator(device="cpu").manual_seed(Np * 131 + F)
    D = torch.randn((3, Np, Np), generator=g, dtype=torch.float64).to(device=device, dtype=dtype)
    G = torch.randn((K, 9), generator=g, dtype=torch.float64).to(device=device, dtype=dtype)
    u = torch.randn((K, F, Np), generator=g, dtype=torch.float64).to(device=device, dtype=dtype)
    return D, G, u


def _time_body(form, body, D, G, u, out, reps):
    fn = lambda: dgvol.dg_volume_batched([(D, G, u)], form=form, outs=[out], bodies=[body])  # noqa: E731
    fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(stream)
    for i in range(reps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)])) * 1e-3


def tune(form, Np, F, target_bytes=256 << 20, min_tiles=1 << 15, reps=10, device=None, cache=None, save=True):
    """Measure every available body for (form, Np, F); store and return the cache entry.

    The problem moves at least ``target_bytes`` and holds at least ``min_tiles``
    16-column tiles, so that at the high orders (few bytes per unit of matrix
    work) the launch's ramp and tail do not inflate the time of a tile."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    word = 8 if form == dgvol.FORM_F64 else 4
    K = max(1024, int(target_bytes // (word * (4 * F * Np + 9))), -(-16 * min_tiles // F))
    D, G, u = _synthetic(form, Np, F, K, device)
    out = torch.empty((3, K, F, Np), dtype=u.dtype, device=device)
    ntiles = -(-K * F // 16)
    times = {}
    for body in (dgvol.BODY_STAGED, dgvol.BODY_CHUNKREG):
        if dgvol.body_available(form, Np, body):
            times[body] = _time_body(form, body, D, G, u, out, reps)
    best = min(times, key=times.get)
    entry = {"body": int(best), "tile_cost_s": times[best] / ntiles,
             "candidates_s_per_tile": {str(b): t / ntiles for b, t in times.items()}, "K": K}
    data = cache if cache is not None else load_cache()
    ns = data.setdefault(device_key(device), {})
    ns[entry_key(form, Np, F)] = entry
    if save:
        save_cache(data)
    return entry


def lookup(form, Np, F, device=None, cache=None, tune_missing=True):
    """Cached entry for (form, Np, F); tuned on demand when missing and allowed."""
    data = cache if cache is not None else load_cache()
    e = data.get(device_key(device), {}).get(entry_key(form, Np, F))
    if _valid_entry(e):
        return e
    if not tune_missing:
        return None
    return tune(form, Np, F, device=device, cache=data)


def plan(groups, form=dgvol.FORM_F64, tune_missing=True):
    """Bodies and tile costs for dg_volume_batched from the tuning cache."""
    bodies, costs = [], []
    data = load_cache()
    for D, G, u in groups:
        K, F, Np = u.shape
        e = lookup(form, Np, F, device=u.device, cache=data, tune_missing=tune_missing)
        bodies.append(dgvol.BODY_AUTO if e is None else e["body"])
        costs.append(0.0 if e is None else e["tile_cost_s"])
    return bodies, costs


def volume_batched_tuned(groups, form=dgvol.FORM_F64, outs=None):
    """dg_volume_batched with the tuned body and measured cost of every group."""
    bodies, costs = plan(groups, form)
    return dgvol.dg_volume_batched(groups, form=form, outs=outs, bodies=bodies, costs=costs)
