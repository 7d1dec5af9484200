"""Benchmark: FP64 DG volume derivative throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-forms]

One step = one dg_volume call (reference derivatives on the FP64 matrix
cores, fused geometric-factor combine) over the whole synthetic mesh of the
headline workload: order 4 (Np = 35), K = 2^20 jittered affine tetrahedra,
F = 5 fields u ~ N(0,1), element-major FP64, inputs resident in HBM.

Prints one JSON line: GDOF/s (K F Np per second), the HBM roofline of the
kernel measured with HIP events on the launch stream, the measured streaming
ceiling for the kernel's read/write mix, the FP64 oracle timed on the host
cores on a bounded sample, and the split-BF16 form and the adjoint measured
beside it.

Profiling helpers (used to produce the committed counter summaries):
    python bench.py --profile-run
        # 1 GiB copy x3, the order-4 forward x3, then the FP64 kernels of the order-5, -6 and -7
        # lines (forward, adjoint, cotangent of D) x3 each
    python bench.py --summarize-counters FETCH_DIR WRITE_DIR
        # reads two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` output trees of
        # --profile-run and writes the HBM traffic summary under profiles/
    python bench.py --summarize-mfma DIR
        # reads a `rocprofv3 --kernel-trace --pmc SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE
        # SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE` tree of --profile-run
        # and writes the matrix-core utilisation summary under profiles/
"""

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DG volume GDOF/s + % HBM/MFMA roofline; plain FP64 vs chosen form"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFS = 78.6           # MI355X FP64 (vector and matrix)
KERNEL_SRC_DIR = os.path.join(ROOT, "paper_1503_07659_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_dg_volume_fwd_f64_order4_K1048576_F5.txt")
FWD_KERNEL_TAG = "fwd_f64_kernel<35, 0, 8, 1>"
COPY_KERNEL_TAG = "stream16_kernel"
MFMA_FILE = os.path.join(ROOT, "profiles", "mfma_util_fp64_kernels.md")
SIMD_NUM = 1024  # MI355X: 256 CUs x 4 SIMDs
NXCD = 8         # MI355X: 8 XCDs
CLOCK_GHZ = 2.4  # MI355X peak engine clock
WORKLOAD = dict(N=4, K=1 << 20, F=5)
PROFILE_COPY_DOUBLES = 1 << 27  # 1 GiB copy for counter calibration


def fwd_bytes_per_element(F, Np, word=8):
    """u read once, three output planes written once, nine geometric factors read once."""
    return word * (4 * F * Np + 9)


def fwd_flops_per_element(F, Np):
    """3 Np x Np products per column (2 flops per multiply-add) plus the 3x3 combine (15 flops/node)."""
    return F * Np * (6 * Np + 15)


def adj_bytes_per_element(F, Np):
    """u, gout (3 planes) read, gu written; G read and gG written."""
    return 8 * (F * Np + 3 * F * Np + F * Np) + 144


def adj_flops_per_element(F, Np):
    return F * Np * (12 * Np + 33)


# Device sources the forward kernel is built from: its body, layout and device
# helpers, and the header that defines the entry kernel.
FWD_KERNEL_SOURCES = ("dgvol_device.hpp", "dgvol_forward.hpp", "dgvol_global.hpp", "dgvol_layout.hpp")


def kernel_source_sha():
    """SHA-256 over the forward kernel's source files (in the order above)."""
    h = hashlib.sha256()
    for name in FWD_KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(KERNEL_SRC_DIR, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per launch of the forward kernel from the committed counter summary, if it
    was taken on the current kernel source; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for ln in open(TRAFFIC_FILE):
        if ":" in ln and not ln.startswith("#"):
            k, v = ln.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_sha():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# untimed warm-up (wall time) before each secondary measurement
WARM_MS = 200.0


def time_launches(fn, steps, warmup, torch, min_warm_ms=0.0):
    """Run fn() warmup times (and, with min_warm_ms, further untimed launches until that much
    wall time has passed: after the GPU has been idle its clocks take tens of milliseconds to
    ramp up), then `steps` times with a HIP event pair around each launch on the current
    stream (the stream the library launches on).  Returns (ms_per_step over the whole timed
    region, list of per-launch ms)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if min_warm_ms > 0:
        t0 = time.perf_counter()
        while (time.perf_counter() - t0) * 1e3 < min_warm_ms:
            for _ in range(4):
                fn()
            torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    evs[0].record(stream)
    for i in range(steps):
        fn()
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [evs[i].elapsed_time(evs[i + 1]) for i in range(steps)]
    return evs[0].elapsed_time(evs[-1]) / steps, per


def cpu_baseline(D, G, u, min_seconds=10.0, max_reps=1000, samples=None):
    """The FP64 oracle on the host cores, on the first elements of the same workload.

    `samples`: optional {name: (gpu output of these elements, "f64" | "f32s")}; each is
    compared with the oracle's output of the timed passes (accuracy of the timed GPU
    outputs on the sampled elements), returned under "accuracy_vs_oracle"."""
    import oracle
    K, F, Np = u.shape
    oracle.volume(D, G[:64], u[:64])  # load/compile outside the timing
    reps, t0 = 0, time.perf_counter()
    while True:
        ref = oracle.volume(D, G, u)
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_seconds or reps >= max_reps:
            break
    acc = {}
    if samples:
        cond = oracle.volume(np.abs(D), np.abs(G), np.abs(u))
        for name, got in samples.items():
            got = np.asarray(got, dtype=np.float64)
            planes = []
            for b in range(3):
                e = np.abs(got[b] - ref[b])
                planes.append({"max_rel": float(e.max() / np.abs(ref[b]).max()),
                               "rms_rel": float(np.linalg.norm(e) / np.linalg.norm(ref[b])),
                               "max_err_over_cond": float((e / np.maximum(cond[b], 1e-300)).max())})
            acc[name] = planes
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    cpu = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    res = {"value": round(reps * K * F * Np / el / 1e9, 4), "unit": "GDOF/s",
           "cores": oracle.num_threads(), "kind": "oracle", "cpu_model": cpu,
           "sample": f"first {K} of {WORKLOAD['K']} elements (order 4, F=5), {reps} pass(es) in {el:.1f} s"}
    if acc:
        res["accuracy_vs_oracle"] = acc
    return res


def split_errors_gpu(got, ref, torch):
    """Per output plane: max|e|/max|ref| and ||e||_2/||ref||_2 of got against ref (GPU tensors)."""
    res = []
    for b in range(ref.shape[0]):
        e = got[b].double() - ref[b]
        res.append({"max_rel": float(e.abs().max() / ref[b].abs().max()),
                    "rms_rel": float(torch.linalg.vector_norm(e) / torch.linalg.vector_norm(ref[b]))})
    return res


def git_revision():
    """HEAD of the source tree, if it is a git checkout (copies without .git report None)."""
    import subprocess
    try:
        r = subprocess.run(["git", "-C", ROOT, "rev-parse", "HEAD"], capture_output=True, text=True, timeout=10)
        return r.stdout.strip() or None if r.returncode == 0 else None
    except (OSError, subprocess.SubprocessError):
        return None


def source_sha():
    """SHA-256 over every library source, the header and this file (identifies the code timed)."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(KERNEL_SRC_DIR, "*"))) + [os.path.join(ROOT, "include", "dgvol.h"),
                                                                    os.path.abspath(__file__)]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def mixed_orders(torch, dev):
    """Orders 1..7 in one persistent launch (group sizes round(2^U(10,18)), seed 3004), F = 3,
    FP64 and split-BF16: eager default launch (one launch for all groups), one launch per
    variant class, the autotuned plan, a graph replay of the tuned plan, and one launch per order
    for comparison; roofline = sum over groups of max(bytes / HBM peak, flops / matrix peak)."""
    from paper_1503_07659_amd import autotune, dgvol, setup_host, synth
    from paper_1503_07659_amd.graph import CapturedLaunch
    F = 3
    sizes = synth.mixed_order_sizes()
    res = {"group_sizes": {str(N): K for N, K in sizes.items()}, "F": F}
    host = {}
    for N, K in sizes.items():
        Np = setup_host.NODE_COUNTS[N]
        host[N] = (setup_host.reference_matrices(N),
                   setup_host.geometric_factors(synth.tet_vertices(K, synth.mesh_seed(4) + 10 * N)),
                   synth.fields(K, F, Np, synth.field_seed(4) + 10 * N, "normal"))
    dofs = sum(K * F * setup_host.NODE_COUNTS[N] for N, K in sizes.items())
    for form, name, dt, word in ((dgvol.FORM_F64, "fp64", torch.float64, 8),
                                 (dgvol.FORM_F32S, "f32s", torch.float32, 4)):
        trip = [tuple(torch.from_numpy(x).to(device=dev, dtype=dt) for x in host[N]) for N in sizes]
        outs = [torch.empty((3,) + tuple(t[2].shape), dtype=dt, device=dev) for t in trip]
        default = lambda: dgvol.dg_volume_batched(trip, form=form, outs=outs)  # noqa: E731
        ms_by_class, _ = time_launches(lambda: dgvol.dg_volume_batched(trip, form=form, outs=outs, by_class=True),
                                       20, 3, torch, min_warm_ms=WARM_MS)
        # tuning (untimed): every variant of every order, then whole candidate plans on these groups
        plan = autotune.plan_batch(trip, form, outs=outs)
        variants, costs, cand = plan.variants, plan.costs, plan.candidates
        tuned = lambda: dgvol.dg_volume_batched(trip, form=form, outs=outs, variants=variants,  # noqa: E731
                                                costs=costs, by_class=plan.by_class)
        # default and tuned plans timed in alternation (three rounds each, median), so that
        # clock drift between them does not favour either
        t_auto, t_tuned = [], []
        for _ in range(3):
            t_auto.append(time_launches(default, 10, 2, torch, min_warm_ms=WARM_MS / 2)[0])
            t_tuned.append(time_launches(tuned, 10, 2, torch, min_warm_ms=WARM_MS / 2)[0])
        ms_auto, ms_tuned = float(np.median(t_auto)), float(np.median(t_tuned))
        if plan_choice(cand) == "default":
            ms_tuned = ms_auto  # the tuner kept the default plan: the same launch
        cap = CapturedLaunch(tuned)
        ms_graph, _ = time_launches(cap.replay, 20, 3, torch, min_warm_ms=WARM_MS)
        single = dgvol.dg_volume if form == dgvol.FORM_F64 else dgvol.dg_volume_f32s
        ms_sep, _ = time_launches(lambda: [single(D, G, u, out=o) for (D, G, u), o in zip(trip, outs)], 20, 3,
                                  torch, min_warm_ms=WARM_MS)
        peak = FP64_PEAK_TFS * 1e12 if form == dgvol.FORM_F64 else 2.5e15 / 3
        roof = 0.0
        for N, K in sizes.items():
            Np = setup_host.NODE_COUNTS[N]
            roof += max(K * fwd_bytes_per_element(F, Np, word) / (HBM_PEAK_GBS * 1e9),
                        K * fwd_flops_per_element(F, Np) / peak)
        res[name] = {"GDOF/s": round(dofs / (ms_graph * 1e-3) / 1e9, 3), "graph_replay_ms": round(ms_graph, 5),
                     "tuned_ms": round(ms_tuned, 5), "default_ms": round(ms_auto, 5),
                     "default_by_class_ms": round(ms_by_class, 5),
                     "tuned_mode": "one launch per class" if plan.by_class else "one launch",
                     "tuned_choice": plan_choice(cand),
                     "one_launch_per_order_ms": round(ms_sep, 5), "roofline_ms": round(roof * 1e3, 5),
                     "frac_of_roofline": round(roof * 1e3 / ms_graph, 4),
                     "variants": {str(N): dict(dgvol.variant_info(form, setup_host.NODE_COUNTS[N],
                                                                  v if v >= 0 else 0), index=int(v))
                                  for N, v in zip(sizes, variants)},
                     "plan_candidates_ms": {k: round(v * 1e3, 5) for k, v in cand.items()}}
        del trip, outs, cap
        torch.cuda.empty_cache()
    return res


def plan_choice(cand):
    """The candidate the batch tuner keeps: the fastest, unless the default is within its margin."""
    from paper_1503_07659_amd import autotune
    if not cand:
        return None
    best = min(cand, key=cand.get)
    if "default" in cand and cand[best] > cand["default"] * (1.0 - autotune.PLAN_MARGIN):
        best = "default"
    return best


def workload_inputs():
    from paper_1503_07659_amd import setup_host, synth
    N, K, F = WORKLOAD["N"], WORKLOAD["K"], WORKLOAD["F"]
    Np = setup_host.NODE_COUNTS[N]
    D = setup_host.reference_matrices(N)
    G = setup_host.geometric_factors(synth.tet_vertices(K, synth.mesh_seed(2)))
    u = synth.fields(K, F, Np, synth.field_seed(2), "normal")
    return D, G, u


def profile_run():
    """Known-size copy (counter scale), the order-4 forward, then the FP64 kernels of the order-5,
    -6 and -7 lines; three launches each."""
    import torch
    from paper_1503_07659_amd import dgvol, setup_host, synth
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    src = torch.ones(PROFILE_COPY_DOUBLES, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dgvol.dg_stream_calibrate(src, dst, 1)
    torch.cuda.synchronize()
    del src, dst
    D, G, u = workload_inputs()
    Dd, Gd, ud = (torch.from_numpy(x).to(dev) for x in (D, G, u))
    out = torch.empty((3,) + tuple(u.shape), dtype=torch.float64, device=dev)
    for _ in range(3):
        dgvol.dg_volume(Dd, Gd, ud, out=out)
    torch.cuda.synchronize()
    del Dd, Gd, ud, out
    torch.cuda.empty_cache()
    for N, K, F in ((5, 1 << 19, 3), (6, 1 << 17, 3), (7, 132228, 3)):
        Np = setup_host.NODE_COUNTS[N]
        D5 = torch.from_numpy(setup_host.reference_matrices(N)).to(dev)
        G5 = torch.from_numpy(setup_host.geometric_factors(synth.tet_vertices(K, synth.mesh_seed(5) + N))).to(dev)
        u5 = torch.from_numpy(synth.fields(K, F, Np, synth.field_seed(5) + N, "uniform")).to(dev)
        o5 = torch.empty((3, K, F, Np), dtype=torch.float64, device=dev)
        for _ in range(3):
            dgvol.dg_volume(D5, G5, u5, out=o5)
        g5 = 2.0 * o5
        gu5, gG5 = torch.empty_like(u5), torch.empty_like(G5)
        for _ in range(3):
            dgvol.dg_volume_adjoint(D5, G5, u5, g5, gu=gu5, gG=gG5)
        if N == 5:
            for _ in range(3):
                dgvol.dg_volume_grad_d(G5, u5, g5)
        torch.cuda.synchronize()
        del D5, G5, u5, o5, g5, gu5, gG5
        torch.cuda.empty_cache()
    # the adjoint with more than 16 fields (order 5, K = 2^16, F = 20)
    K20, F20 = 1 << 16, 20
    D20 = torch.from_numpy(setup_host.reference_matrices(5)).to(dev)
    G20 = torch.from_numpy(setup_host.geometric_factors(synth.tet_vertices(K20, synth.mesh_seed(5) + 20))).to(dev)
    u20 = torch.from_numpy(synth.fields(K20, F20, 56, synth.field_seed(5) + 20, "uniform")).to(dev)
    g20 = torch.ones((3, K20, F20, 56), dtype=torch.float64, device=dev)
    for _ in range(3):
        dgvol.dg_volume_adjoint(D20, G20, u20, g20)
    torch.cuda.synchronize()
    print("profile run done", flush=True)


def _counter_rows(root):
    rows = []
    for path in glob.glob(os.path.join(root, "**", "*counter_collection*.csv"), recursive=True):
        with open(path, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    if not rows:
        raise SystemExit(f"no counter_collection csv under {root}")
    return rows


def _per_dispatch(rows, counter, tag):
    vals = {}
    for r in rows:
        if r.get("Counter_Name") != counter or tag not in r.get("Kernel_Name", ""):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    return [vals[k] for k in sorted(vals, key=lambda x: int(x))]


def summarize_counters(fetch_dir, write_dir):
    fr, wr = _counter_rows(fetch_dir), _counter_rows(write_dir)
    cf = _per_dispatch(fr, "FETCH_SIZE", COPY_KERNEL_TAG)
    cw = _per_dispatch(wr, "WRITE_SIZE", COPY_KERNEL_TAG)
    kf = _per_dispatch(fr, "FETCH_SIZE", FWD_KERNEL_TAG)
    kw = _per_dispatch(wr, "WRITE_SIZE", FWD_KERNEL_TAG)
    if not (cf and cw and kf and kw):
        raise SystemExit("missing dispatches of the copy or the forward kernel in the counter output")
    copy_bytes = PROFILE_COPY_DOUBLES * 8
    sf = copy_bytes / float(np.median(cf))   # bytes per counter unit, read side
    sw = copy_bytes / float(np.median(cw))   # bytes per counter unit, write side
    fetch_b = float(np.median(kf)) * sf
    write_b = float(np.median(kw)) * sw
    N, K, F = WORKLOAD["N"], WORKLOAD["K"], WORKLOAD["F"]
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    alg = K * fwd_bytes_per_element(F, Np)
    os.makedirs(os.path.dirname(TRAFFIC_FILE), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        fh.write("# HBM traffic of dg_volume (FP64 staged forward kernel), order 4, K=2^20, F=5.\n")
        fh.write("# Two rocprofv3 counter passes over `python bench.py --profile-run`:\n")
        fh.write("#   rocprofv3 --pmc FETCH_SIZE -d <fetch_dir> --output-format csv -- python bench.py --profile-run\n")
        fh.write("#   rocprofv3 --pmc WRITE_SIZE -d <write_dir> --output-format csv -- python bench.py --profile-run\n")
        fh.write("#   python bench.py --summarize-counters <fetch_dir> <write_dir>\n")
        fh.write("# Counter units are scaled by a 1 GiB copy (stream16_kernel, copies=1) in the same runs.\n")
        fh.write(f"kernel_source_sha256: {kernel_source_sha()}\n")
        fh.write(f"copy_fetch_counter_per_launch: {np.median(cf):.1f}\n")
        fh.write(f"copy_write_counter_per_launch: {np.median(cw):.1f}\n")
        fh.write(f"fetch_scale_bytes_per_unit: {sf:.4f}\n")
        fh.write(f"write_scale_bytes_per_unit: {sw:.4f}\n")
        fh.write(f"kernel_fetch_counter_per_launch: {np.median(kf):.1f}\n")
        fh.write(f"kernel_write_counter_per_launch: {np.median(kw):.1f}\n")
        fh.write(f"fetch_bytes_per_launch: {fetch_b:.0f}\n")
        fh.write(f"write_bytes_per_launch: {write_b:.0f}\n")
        fh.write(f"hbm_bytes_per_launch: {fetch_b + write_b:.0f}\n")
        fh.write(f"algorithmic_bytes_per_launch: {alg}\n")
        fh.write(f"traffic_over_algorithmic: {(fetch_b + write_b) / alg:.4f}\n")
    print(open(TRAFFIC_FILE).read())


def summarize_mfma(root):
    """Matrix-core use per FP64 kernel of --profile-run: MFMA-busy cycles over (GUI-active cycles
    x SIMDs), executed FP64 matrix flops per second over the spec peak, and LDS bank-conflict
    cycles over LDS-active cycles; medians over each kernel's dispatches."""
    rows = _counter_rows(root)
    trace = {}
    for path in glob.glob(os.path.join(root, "**", "*kernel_trace*.csv"), recursive=True):
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                trace[r.get("Dispatch_Id") or r.get("Correlation_Id")] = \
                    (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    per = {}
    for r in rows:
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        ent = per.setdefault(key, {"name": r.get("Kernel_Name", "")})
        ent[r["Counter_Name"]] = ent.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    # GRBM_GUI_ACTIVE counts per XCD and the csv sums the instances: cycles = sum / NXCD
    by_kernel = {}
    for key, ent in per.items():
        name = ent["name"]
        if "fwd_f64" not in name and "adj" not in name and "gd_partial" not in name and "gd_split" not in name:
            continue
        if "SQ_VALU_MFMA_BUSY_CYCLES" not in ent or "GRBM_GUI_ACTIVE" not in ent:
            continue
        cycles = ent["GRBM_GUI_ACTIVE"] / NXCD
        util = ent["SQ_VALU_MFMA_BUSY_CYCLES"] / (cycles * SIMD_NUM)
        flops = ent.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512
        per_cycle = FP64_PEAK_TFS * 1e12 / (CLOCK_GHZ * 1e9)
        frac = flops / (cycles * per_cycle)
        lds = ent.get("SQ_LDS_BANK_CONFLICT", 0.0) / max(ent.get("SQ_LDS_IDX_ACTIVE", 0.0), 1.0)
        dur = trace.get(key, float("nan"))
        # one kernel can serve two workloads (the adjoint at F = 3 and F = 20): one row per
        # workload, told apart by the executed flops of a launch
        by_kernel.setdefault((name.split("(")[0], round(flops / 1e9, 1)), []).append((util, frac, lds, dur, flops))
    os.makedirs(os.path.dirname(MFMA_FILE), exist_ok=True)
    with open(MFMA_FILE, "w") as fh:
        fh.write("# Matrix-core use of the FP64 kernels (rocprofv3 counters, MI355X)\n\n")
        fh.write("Commands (GPU box, TMPDIR=/tmp, run from /tmp):\n\n")
        fh.write("    rocprofv3 --kernel-trace --pmc SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE SQ_INSTS_VALU_MFMA_MOPS_F64 "
                 "SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE -d <dir> -f csv -- python3 <repo>/bench.py --profile-run\n")
        fh.write("    python3 <repo>/bench.py --summarize-mfma <dir>\n\n")
        fh.write("* MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (active cycles x 1024 SIMDs), rocprofv3's MfmaUtil; "
                 "active cycles = GRBM_GUI_ACTIVE / 8 (the csv sums the counter over the 8 XCDs).\n")
        fh.write("* executed of peak = SQ_INSTS_VALU_MFMA_MOPS_F64 x 512 FP64 matrix flops (padding rows included) "
                 "over (active cycles x the spec peak per cycle, 78.6 TFLOP/s at 2.4 GHz): clock-independent. "
                 "The profile run launches each kernel three times without warm-up, so its wall durations "
                 "(last column) run long; the bench line gives the warm times.\n")
        fh.write("* LDS conflict = SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE.\n")
        fh.write("* Workloads: order 4 K=2^20 F=5; order 5 K=2^19 F=3 (and the adjoint at K=2^16 F=20, the "
                 "same kernel: a row of its own, with its own flops per launch); order 6 K=2^17 F=3; "
                 "order 7 K=132228 F=3.\n\n")
        fh.write("| kernel | dispatches | MFMA busy | executed of FP64 peak | executed GFLOP per launch | "
                 "LDS conflict | median ms (profiled) |\n")
        fh.write("|---|---|---|---|---|---|---|\n")
        for key in sorted(by_kernel):
            v = np.array(by_kernel[key])
            med = np.median(v, axis=0)
            fh.write(f"| `{key[0]}` | {len(v)} | {med[0]:.3f} | {med[1]:.3f} | {med[4] / 1e9:.2f} | "
                     f"{med[2]:.3f} | {med[3] * 1e3:.4f} |\n")
    print(open(MFMA_FILE).read())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-forms", action="store_true", help="skip the split-BF16 and adjoint lines")
    ap.add_argument("--cpu-elements", type=int, default=1 << 18)
    ap.add_argument("--profile-run", action="store_true")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-mfma", metavar="DIR")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.summarize_mfma:
        summarize_mfma(args.summarize_mfma)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the volume kernel "
              "needs no communication; the multi-GPU split is a partition of the elements.",
              file=sys.stderr)
        sys.exit(2)
    if args.profile_run:
        profile_run()
        return

    import torch
    from paper_1503_07659_amd import dgvol, setup_host, synth

    N, K, F = WORKLOAD["N"], WORKLOAD["K"], WORKLOAD["F"]
    Np = setup_host.NODE_COUNTS[N]
    D, G, u = workload_inputs()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    Dd, Gd, ud = (torch.from_numpy(x).to(dev) for x in (D, G, u))
    out = torch.empty((3, K, F, Np), dtype=torch.float64, device=dev)

    # Calibrations first (they also bring the GPU to its working clocks before the timed
    # steps): practical streaming ceiling for the same bytes in the same 1 : 3 read : write mix
    n_u = ud.numel()
    _, per_c = time_launches(lambda: dgvol.dg_stream_calibrate(ud.view(-1), out.view(-1), 3), 10, 2, torch,
                             min_warm_ms=WARM_MS)
    ceil_gbs = 4 * n_u * 8 / (float(np.median(per_c)) * 1e-3) / 1e9
    _, per_1 = time_launches(lambda: dgvol.dg_stream_calibrate(ud.view(-1), out.view(-1)[:n_u], 1), 10, 2, torch,
                             min_warm_ms=WARM_MS)
    copy_gbs = 2 * n_u * 8 / (float(np.median(per_1)) * 1e-3) / 1e9
    # the forward's own data movement (tiles through LDS, no arithmetic) in its persistent launch
    # shape and as a one-pass grid
    tile_gbs = {}
    for tag, m in (("persistent", 0), ("one_pass", 1)):
        _, per_t = time_launches(lambda: dgvol.dg_stream_calibrate_tiles(ud.view(-1), out.view(-1), m), 10, 2,
                                 torch, min_warm_ms=WARM_MS)
        tile_gbs[tag] = round(4 * n_u * 8 / (float(np.median(per_t)) * 1e-3) / 1e9, 1)
    # attainable FP64 matrix-core rate: independent MFMA chains from registers
    sink, _ = dgvol.dg_mfma_calibrate(10)
    _, per_m = time_launches(lambda: dgvol.dg_mfma_calibrate(10000, sink=sink), 5, 1, torch, min_warm_ms=WARM_MS)
    cal_flops = dgvol.MFMA_CAL_BLOCKS * 4 * 10000 * 4 * 2048
    mfma_tfs = cal_flops / (float(np.median(per_m)) * 1e-3) / 1e12
    del sink
    # FP64 products beside vector work on the same SIMDs (20000 rounds of each): how much of
    # the vector work overlaps the products
    bsink = dgvol.dg_mfma_calibrate_beside(10, 10, dgvol.BESIDE_NONE)
    beside = {}
    for name, it, vit, mode in (("products_alone", 20000, 0, dgvol.BESIDE_NONE),
                                ("fp64_fma_alone", 0, 20000, dgvol.BESIDE_FP64_FMA),
                                ("products_beside_fp64_fma", 20000, 20000, dgvol.BESIDE_FP64_FMA),
                                ("products_beside_int", 20000, 20000, dgvol.BESIDE_INT),
                                ("products_beside_dpp", 20000, 20000, dgvol.BESIDE_DPP)):
        _, per_b = time_launches(lambda: dgvol.dg_mfma_calibrate_beside(it, vit, mode, sink=bsink), 3, 1, torch)
        beside[name] = round(float(np.median(per_b)), 4)
    del bsink

    def step():
        dgvol.dg_volume(Dd, Gd, ud, out=out)

    ms, per = time_launches(step, args.steps, args.warmup, torch)
    kern_ms = float(np.mean(per))
    q1, med, q3 = (float(x) for x in np.percentile(per, [25, 50, 75]))
    ncpu = min(args.cpu_elements, K)
    samples = {"fp64_headline": out[:, :ncpu].cpu().numpy()} if not args.no_cpu else {}
    dofs = K * F * Np
    bytes_launch = K * fwd_bytes_per_element(F, Np)
    flops_launch = K * fwd_flops_per_element(F, Np)
    achieved = bytes_launch / (kern_ms * 1e-3) / 1e9

    rec = {
        "metric": METRIC,
        "value": round(dofs / (ms * 1e-3) / 1e9, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "fp64_order4_K1048576_F5", "order": N, "Np": Np, "K": K, "F": F,
                   "u": "N(0,1)", "mesh": "unit tet + U(-0.2,0.2) vertex jitter",
                   "seeds": {"mesh": synth.mesh_seed(2), "fields": synth.field_seed(2)}},
        "timing": {"per_launch_ms_median": round(med, 5), "per_launch_ms_iqr": [round(q1, 5), round(q3, 5)],
                   "clock": "HIP events on the launch stream"},
        "revision": {"git": git_revision(), "source_sha256": source_sha()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(),
                     "kernel_ms": round(kern_ms, 5),
                     "measured_stream_ceiling_1r3w_GBs": round(ceil_gbs, 1),
                     "frac_of_measured_ceiling": round(achieved / ceil_gbs, 4),
                     "measured_copy_GBs": round(copy_gbs, 1),
                     "measured_tile_stream_GBs": tile_gbs,
                     "frac_of_persistent_tile_stream": round(achieved / tile_gbs["persistent"], 4),
                     "fp64_tflops": round(flops_launch / (kern_ms * 1e-3) / 1e12, 2),
                     "fp64_frac": round(flops_launch / (kern_ms * 1e-3) / 1e12 / FP64_PEAK_TFS, 4),
                     "measured_fp64_mfma_TFs": round(mfma_tfs, 2),
                     "fp64_products_beside_vector_ms": beside},
    }
    del out
    torch.cuda.empty_cache()

    if not args.no_forms:
        forms = {}
        # chosen precision form at the same shape: FP32 storage, split-BF16 products
        D32, G32, u32 = (torch.from_numpy(x.astype(np.float32)).to(dev) for x in (D, G, u))
        o32 = torch.empty((3, K, F, Np), dtype=torch.float32, device=dev)
        ms32, per32 = time_launches(lambda: dgvol.dg_volume_f32s(D32, G32, u32, out=o32), 20, 3, torch,
                                    min_warm_ms=WARM_MS)
        k32 = float(np.mean(per32))
        # accuracy of the timed output (outside the timed region), every output, per plane:
        # against the FP64 result on the FP64 data, and on the FP32-rounded inputs promoted to
        # FP64 (isolates the arithmetic from the storage rounding); the FP64 results are the
        # FP64 kernel's, which matches the oracle to 1e-12 (parity tests)
        ref64 = dgvol.dg_volume(Dd, Gd, ud)
        err64 = split_errors_gpu(o32, ref64, torch)
        del ref64
        ref32 = dgvol.dg_volume(D32.double(), G32.double(), u32.double())
        err32 = split_errors_gpu(o32, ref32, torch)
        del ref32
        if samples:
            samples["f32s_split_bf16"] = o32[:, :ncpu].cpu().numpy()
        forms["f32s_split_bf16_same_workload"] = {
            "GDOF/s": round(dofs / (ms32 * 1e-3) / 1e9, 3), "kernel_ms": round(k32, 5),
            "hbm_GBs": round(K * fwd_bytes_per_element(F, Np, 4) / (k32 * 1e-3) / 1e9, 1),
            "hbm_frac": round(K * fwd_bytes_per_element(F, Np, 4) / (k32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "speedup_vs_fp64": round(ms / ms32, 3),
            "error_per_plane_xyz": {"reference": "FP64 kernel, every output",
                                    "vs_fp64_on_fp64_data": err64, "vs_fp64_on_fp32_rounded_inputs": err32,
                                    "stated_bound": {"max_rel": 2e-5, "rms_rel": 1e-5}}}
        del D32, G32, u32, o32, Dd, Gd, ud
        torch.cuda.empty_cache()
        # adjoint workload: order 5, K = 2^19, F = 3, gout = 2 out
        N5, K5, F5 = 5, 1 << 19, 3
        Np5 = setup_host.NODE_COUNTS[N5]
        D5 = torch.from_numpy(setup_host.reference_matrices(N5)).to(dev)
        G5 = torch.from_numpy(setup_host.geometric_factors(synth.tet_vertices(K5, synth.mesh_seed(5)))).to(dev)
        u5 = torch.from_numpy(synth.fields(K5, F5, Np5, synth.field_seed(5), "uniform")).to(dev)
        o5 = torch.empty((3, K5, F5, Np5), dtype=torch.float64, device=dev)
        msf, perf = time_launches(lambda: dgvol.dg_volume(D5, G5, u5, out=o5), 20, 3, torch, min_warm_ms=WARM_MS)
        g5 = 2.0 * o5
        gu5 = torch.empty_like(u5)
        gG5 = torch.empty_like(G5)
        msa, pera = time_launches(lambda: dgvol.dg_volume_adjoint(D5, G5, u5, g5, gu=gu5, gG=gG5), 20, 3, torch,
                                  min_warm_ms=WARM_MS)
        ka, kf = float(np.mean(pera)), float(np.mean(perf))
        d5 = K5 * F5 * Np5
        fl_f, fl_a = K5 * fwd_flops_per_element(F5, Np5), K5 * adj_flops_per_element(F5, Np5)
        # cotangent of D for the same cotangent (both kernels of the call are timed)
        gD5 = torch.empty_like(D5)
        wk5 = torch.empty(dgvol.grad_d_workspace_bytes(K5, Np5, F5), dtype=torch.uint8, device=dev)
        msd, perd = time_launches(lambda: dgvol.dg_volume_grad_d(G5, u5, g5, gD=gD5, work=wk5), 20, 3, torch,
                                  min_warm_ms=WARM_MS)
        kd = float(np.mean(perd))
        forms["fp64_order5_K524288_F3"] = {
            "grad_D_GDOF/s": round(d5 / (msd * 1e-3) / 1e9, 3), "grad_D_call_ms": round(kd, 5),
            "grad_D_hbm_frac": round(K5 * fwd_bytes_per_element(F5, Np5) / (kd * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "grad_D_fp64_frac": round(fl_f / (kd * 1e-3) / 1e12 / FP64_PEAK_TFS, 4),
            "forward_GDOF/s": round(d5 / (msf * 1e-3) / 1e9, 3), "forward_kernel_ms": round(kf, 5),
            "forward_fp64_frac": round(fl_f / (kf * 1e-3) / 1e12 / FP64_PEAK_TFS, 4),
            "forward_hbm_frac": round(K5 * fwd_bytes_per_element(F5, Np5) / (kf * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "adjoint_GDOF/s": round(d5 / (msa * 1e-3) / 1e9, 3), "adjoint_kernel_ms": round(ka, 5),
            "adjoint_fp64_frac": round(fl_a / (ka * 1e-3) / 1e12 / FP64_PEAK_TFS, 4),
            "adjoint_frac_of_measured_mfma": round(fl_a / (ka * 1e-3) / 1e12 / mfma_tfs, 4),
            "adjoint_hbm_frac": round(K5 * adj_bytes_per_element(F5, Np5) / (ka * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del D5, G5, u5, o5, g5, gu5, gG5, gD5, wk5
        torch.cuda.empty_cache()
        # adjoint with more than 16 fields (each element's fields in 16-column sub-tiles)
        N20, K20, F20 = 5, 1 << 16, 20
        D20 = torch.from_numpy(setup_host.reference_matrices(N20)).to(dev)
        G20 = torch.from_numpy(setup_host.geometric_factors(synth.tet_vertices(K20, synth.mesh_seed(5) + 20))).to(dev)
        u20 = torch.from_numpy(synth.fields(K20, F20, Np5, synth.field_seed(5) + 20, "uniform")).to(dev)
        g20 = torch.from_numpy(synth.fields(K20, 3 * F20, Np5, synth.field_seed(5) + 21, "normal")).to(dev)
        g20 = g20.view(K20, 3, F20, Np5).permute(1, 0, 2, 3).contiguous()
        gu20, gG20 = torch.empty_like(u20), torch.empty_like(G20)
        _, per20 = time_launches(lambda: dgvol.dg_volume_adjoint(D20, G20, u20, g20, gu=gu20, gG=gG20), 20, 3, torch,
                                 min_warm_ms=WARM_MS)
        k20 = float(np.mean(per20))
        fl20 = K20 * adj_flops_per_element(F20, Np5)
        forms[f"fp64_adjoint_order5_K{K20}_F{F20}"] = {
            "adjoint_GDOF/s": round(K20 * F20 * Np5 / (k20 * 1e-3) / 1e9, 3), "adjoint_kernel_ms": round(k20, 5),
            "adjoint_fp64_frac": round(fl20 / (k20 * 1e-3) / 1e12 / FP64_PEAK_TFS, 4)}
        del D20, G20, u20, g20, gu20, gG20
        torch.cuda.empty_cache()
        # adjoint at the orders whose D does not fit LDS (two chunk-register passes)
        for Nh, Kh in ((6, 1 << 17), (7, 1 << 16)):
            Nph = setup_host.NODE_COUNTS[Nh]
            Dh = torch.from_numpy(setup_host.reference_matrices(Nh)).to(dev)
            Gh = torch.from_numpy(setup_host.geometric_factors(synth.tet_vertices(Kh, synth.mesh_seed(5) + Nh))).to(dev)
            uh = torch.from_numpy(synth.fields(Kh, F5, Nph, synth.field_seed(5) + Nh, "uniform")).to(dev)
            gh = torch.from_numpy(synth.fields(Kh, F5, Nph, synth.field_seed(5) + 10 * Nh, "normal")).to(dev)
            gh = torch.stack([gh, 0.5 * gh, -gh])
            guh, gGh = torch.empty_like(uh), torch.empty_like(Gh)
            _, perh = time_launches(lambda: dgvol.dg_volume_adjoint(Dh, Gh, uh, gh, gu=guh, gG=gGh), 20, 3, torch,
                                    min_warm_ms=WARM_MS)
            kh = float(np.mean(perh))
            flh = Kh * adj_flops_per_element(F5, Nph)
            forms[f"fp64_adjoint_order{Nh}_K{Kh}_F{F5}"] = {
                "adjoint_GDOF/s": round(Kh * F5 * Nph / (kh * 1e-3) / 1e9, 3), "adjoint_call_ms": round(kh, 5),
                "adjoint_fp64_frac": round(flh / (kh * 1e-3) / 1e12 / FP64_PEAK_TFS, 4)}
            del Dh, Gh, uh, gh, guh, gGh
            torch.cuda.empty_cache()
        forms["mixed_orders1to7_F3"] = mixed_orders(torch, dev)
        rec["forms"] = forms

    if not args.no_cpu:
        n = min(args.cpu_elements, K)
        rec["cpu_baseline"] = cpu_baseline(D, G[:n], u[:n], samples=samples)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
