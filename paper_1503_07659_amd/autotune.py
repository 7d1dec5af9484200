"""Autotuner of the forward product's tile shapes (launch variants).

The library is compiled with a short list of launch variants per (form, Np)
(``dg_variant_count`` / ``dg_variant_query``): the body that moves the data
(LDS-staged or chunk-register), the waves per workgroup and the 16-column
tiles one loop iteration takes.  They compute the same result with different
data movement; which is fastest depends on the order, the number of fields
and the device.  This is the paper's autotuning use case (Introduction and
Section 3: a search over the transformation parameters of a kernel) applied
to those tile shapes.

``tune(form, Np, F)`` times every variant on a synthetic problem large enough
to fill the GPU, three ways: as a single-group launch (``dg_volume_variant``)
and as a one-group batched launch in each of the batched launch modes (the
default one, whose kernel holds every 8-wave body, and one launch per variant
class, whose kernel fits the class's register budget).  It records the fastest
variant of each with the measured time of one 16-column tile.  That time is
the ``cost`` the batched launch uses to split its persistent workgroups
between groups.

``plan_batch(groups, form)`` then measures whole candidate plans on the actual
groups -- the library default, the per-group tuned variants with measured
costs, and the tuned variants with the library's cost estimate, each in both
launch modes -- and keeps the fastest, so a tuned batch is never slower than
the default one as measured.

Results are cached in a JSON file (``$DGVOL_AUTOTUNE_CACHE``, default
``~/.cache/dgvol/autotune.json``) keyed by the GPU architecture and the
library ABI version; an unreadable, corrupt or foreign cache is ignored and
rewritten.  Tuning needs a GPU; looking up the cache does not.
"""

import json
import os
import tempfile
import time
from collections import namedtuple

import numpy as np
import torch

from . import dgvol

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "dgvol", "autotune.json")
FORM_NAMES = {dgvol.FORM_F64: "f64", dgvol.FORM_F32S: "f32s"}


def cache_path():
    return os.environ.get("DGVOL_AUTOTUNE_CACHE", DEFAULT_CACHE)


def device_key(device=None):
    """Cache namespace: architecture of the device and ABI version of the library."""
    props = torch.cuda.get_device_properties(device or torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    return f"{arch}/abi{dgvol.load_library().dg_abi_version()}"


def entry_key(form, Np, F):
    return f"{FORM_NAMES[form]}/Np{Np}/F{F}"


def batch_key(form, groups):
    return f"batch/{FORM_NAMES[form]}/" + ",".join(f"{u.shape[2]}x{u.shape[0]}x{u.shape[1]}" for _, _, u in groups)


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


def _valid_entry(e, form, Np):
    if not isinstance(e, dict):
        return False
    n = dgvol.variant_count(form, Np)
    for k in ("variant", "single_variant", "by_class_variant"):
        if not isinstance(e.get(k), int) or not 0 <= e[k] < n:
            return False
    return all(isinstance(e.get(k), (int, float)) and e[k] > 0 for k in ("tile_cost_s", "by_class_tile_cost_s"))


def _synthetic(form, Np, F, K, device):
    """Inputs with the shape of one group (values only need to be finite)."""
    dtype = torch.float64 if form == dgvol.FORM_F64 else torch.float32
    g = torch.Generator(device="cpu").manual_seed(Np * 131 + F)
    D = torch.randn((3, Np, Np), generator=g, dtype=torch.float64).to(device=device, dtype=dtype)
    G = torch.randn((K, 9), generator=g, dtype=torch.float64).to(device=device, dtype=dtype)
    u = torch.randn((K, F, Np), generator=g, dtype=torch.float64).to(device=device, dtype=dtype)
    return D, G, u


def _median_time(fn, reps):
    """Median seconds of fn() over `reps` launches, timed with HIP events on the current stream."""
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
    """Measure every variant of (form, Np) at F fields; store and return the cache entry.

    The problem moves at least ``target_bytes`` and holds at least ``min_tiles``
    16-column tiles, so that at the high orders (few bytes per unit of matrix
    work) the launch's ramp and tail do not inflate the time of a tile."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    word = 8 if form == dgvol.FORM_F64 else 4
    K = max(1024, int(target_bytes // (word * (4 * F * Np + 9))), -(-16 * min_tiles // F))
    D, G, u = _synthetic(form, Np, F, K, device)
    out = torch.empty((3, K, F, Np), dtype=u.dtype, device=device)
    ntiles = -(-K * F // 16)
    single, batched, by_class = {}, {}, {}
    for v in range(dgvol.variant_count(form, Np)):
        single[v] = _median_time(lambda: dgvol.dg_volume_variant(form, v, D, G, u, out=out), reps)
        batched[v] = _median_time(
            lambda: dgvol.dg_volume_batched([(D, G, u)], form=form, outs=[out], variants=[v]), reps)
        by_class[v] = _median_time(
            lambda: dgvol.dg_volume_batched([(D, G, u)], form=form, outs=[out], variants=[v], by_class=True), reps)
    best_b = min(batched, key=batched.get)
    best_c = min(by_class, key=by_class.get)
    best_s = min(single, key=single.get)
    entry = {"variant": int(best_b), "tile_cost_s": batched[best_b] / ntiles,
             "by_class_variant": int(best_c), "by_class_tile_cost_s": by_class[best_c] / ntiles,
             "single_variant": int(best_s), "single_tile_cost_s": single[best_s] / ntiles,
             "candidates_s_per_tile": {str(v): t / ntiles for v, t in batched.items()},
             "by_class_candidates_s_per_tile": {str(v): t / ntiles for v, t in by_class.items()},
             "single_candidates_s_per_tile": {str(v): t / ntiles for v, t in single.items()},
             "shapes": {str(v): dgvol.variant_info(form, Np, v) for v in single}, "K": K}
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
    if _valid_entry(e, form, Np):
        return e
    if not tune_missing:
        return None
    return tune(form, Np, F, device=device, cache=data)


def plan(groups, form=dgvol.FORM_F64, tune_missing=True, by_class=False):
    """Per-group variants and measured tile costs for dg_volume_batched (in the given launch mode)
    from the tuning cache."""
    variants, costs = [], []
    data = load_cache()
    vk, ck = ("by_class_variant", "by_class_tile_cost_s") if by_class else ("variant", "tile_cost_s")
    for D, G, u in groups:
        K, F, Np = u.shape
        e = lookup(form, Np, F, device=u.device, cache=data, tune_missing=tune_missing)
        variants.append(dgvol.VARIANT_AUTO if e is None else e[vk])
        costs.append(0.0 if e is None else e[ck])
    return variants, costs


BatchPlan = namedtuple("BatchPlan", "variants costs by_class candidates")


# a tuned batch plan replaces the default launch only when it measures this much faster
PLAN_MARGIN = 0.01


def plan_batch(groups, form=dgvol.FORM_F64, outs=None, reps=20, tune_missing=True, save=True):
    """The fastest measured plan for this batch of groups, as a BatchPlan(variants, costs,
    by_class, candidates).

    Candidates, each in both launch modes (one launch for all 8-wave groups, and one launch per
    variant class): the library default (variant 0, estimated costs), the per-group tuned
    variants with their measured costs, and the tuned variants with the estimated costs.  Each
    is timed on the actual groups, in five alternating rounds; the default is kept unless a
    candidate is more than PLAN_MARGIN faster.  The result is cached under the batch's shapes;
    candidates maps each candidate's name to its measured seconds."""
    device = groups[0][2].device
    data = load_cache()
    key = batch_key(form, groups)
    ns = data.setdefault(device_key(device), {})
    e = ns.get(key)
    n = len(groups)
    if isinstance(e, dict) and len(e.get("variants", [])) == n and len(e.get("costs", [])) == n \
            and isinstance(e.get("by_class"), bool):
        return BatchPlan(e["variants"], e["costs"], e["by_class"], e.get("candidates_s", {}))
    if outs is None:
        outs = [torch.empty((3,) + tuple(u.shape), dtype=u.dtype, device=device) for _, _, u in groups]
    cands = {}
    for bc, suffix in ((False, ""), (True, "_by_class")):
        tv, tc = plan(groups, form, tune_missing=tune_missing, by_class=bc)
        cands["default" + suffix] = ([dgvol.VARIANT_AUTO] * n, [0.0] * n, bc)
        cands["tuned" + suffix] = (tv, tc, bc)
        cands["tuned_variants" + suffix] = (tv, [0.0] * n, bc)
    # candidates timed in alternation (five rounds, median) after the clocks have come up,
    # so that clock drift does not favour the ones timed later
    first = cands["default"]
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.1:
        dgvol.dg_volume_batched(groups, form=form, outs=outs, variants=first[0], costs=first[1], by_class=first[2])
        torch.cuda.synchronize(device)
    samples = {name: [] for name in cands}
    for _ in range(5):
        for name, (v, c, bc) in cands.items():
            samples[name].append(_median_time(
                lambda: dgvol.dg_volume_batched(groups, form=form, outs=outs, variants=v, costs=c, by_class=bc),
                reps))
    times = {name: float(np.median(s)) for name, s in samples.items()}
    best = min(times, key=times.get)
    # the library default stays unless a candidate beats it by more than the timing noise
    if times[best] > times["default"] * (1.0 - PLAN_MARGIN):
        best = "default"
    v, c, bc = cands[best]
    ns[key] = {"variants": [int(x) for x in v], "costs": [float(x) for x in c], "by_class": bool(bc),
               "choice": best, "candidates_s": times}
    if save:
        save_cache(data)
    return BatchPlan(v, c, bc, times)


def volume_batched_tuned(groups, form=dgvol.FORM_F64, outs=None):
    """dg_volume_batched with the fastest measured plan for these groups."""
    p = plan_batch(groups, form, outs=outs)
    return dgvol.dg_volume_batched(groups, form=form, outs=outs, variants=p.variants, costs=p.costs,
                                   by_class=p.by_class)
