"""GPU parity at the sizes and launch shapes the kernels are timed at.

* Every launch variant of the forward product (both forms, every order),
  single-group and as a one-group batched launch, at a size where every wave
  (staged body) or workgroup (chunk-register body) runs at least three
  iterations of its persistent loop, so the prefetch of the next tile and its
  staging are exercised; the size is derived from the launch shape the
  library reports for the device (dg_launch_shape_query).
* The adjoint at every order, F = 3 and F = 20 (orders 6, 7: two-pass
  kernels), at three or more loop iterations; and every F up to 16 plus
  17, 20, 33, 40 at orders 1, 4, 5, where runs of whole elements are cut into
  full tiles and elements straddle two or more tiles.
* The mixed-order workload exactly as benchmarked (orders 1..7, group sizes
  from seed 3004, F = 3), both forms, with the default plan, the tuned plan
  and a graph replay of the tuned plan.
* The split-BF16 form and the FP64 forward at the order-4 benchmark shape
  (K = 2^20, F = 5), every output compared.

Every output is compared with the FP64 oracle: FP64 by the normwise and
condition-scaled pair (1e-12), split-BF16 by the stated bound plus the
FP32-accumulation bound against the exact three-pass emulation.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_1503_07659_amd import dgvol, synth
from parity import (adjoint_cond_c, check_f32s, check_planes, check_whole, forward_cond_c)

pytestmark = pytest.mark.gpu

ORDERS = range(1, 8)
FORMS = (dgvol.FORM_F64, dgvol.FORM_F32S)


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _cast(form):
    return (lambda x: x) if form == dgvol.FORM_F64 else (lambda x: x.astype(np.float32))


def _k_for_iters(op, form, Np, variant, F, iters=3):
    """Smallest K (elements) with a ragged tail whose launch gives every worker >= iters
    loop iterations, found from the device's launch shape."""
    K = 64
    while True:
        sh = dgvol.launch_shape(op, form, Np, variant, K, F)
        if sh["min_iters"] >= iters:
            return K, sh
        K = int(K * 1.6) + 7


def _check_form(form, D, G, u, got):
    if form == dgvol.FORM_F64:
        check_planes(got, oracle.volume(D, G, u), forward_cond_c(D, G, u))
    else:
        check_f32s(D, G, u, got)


def _variant_cases():
    # variant counts come from the library (host query): collected without a GPU
    cases = []
    lib = dgvol.load_library()
    for form in FORMS:
        for N in ORDERS:
            Np = oracle.num_nodes(N)
            for v in range(lib.dg_variant_count(form, Np)):
                cases.append((form, N, v))
    return cases


@pytest.mark.parametrize("form,N,variant", _variant_cases())
def test_variant_three_loop_iterations(form, N, variant):
    """One variant, single-group and one-group batched in both launch modes, at >= 3 loop
    iterations per worker; against the oracle, and bitwise equal to each other (same body, same
    arithmetic)."""
    Np = oracle.num_nodes(N)
    F = 3
    ops = (dgvol.OP_FORWARD, dgvol.OP_BATCHED, dgvol.OP_BATCHED_BY_CLASS)
    K = max(_k_for_iters(op, form, Np, variant, F)[0] for op in ops)
    shapes = [dgvol.launch_shape(op, form, Np, variant, K, F) for op in ops]
    _say(f"variant form={form} N={N} v={variant} K={K} F={F} single/batched/by-class={shapes}")
    for sh in shapes:
        assert sh["min_iters"] >= 3 and sh["grid"] <= sh["resident"]
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, 5000 + 10 * N + variant))
    u = synth.fields(K, F, Np, 5100 + 10 * N + variant, "normal")
    c = _cast(form)
    Dd, Gd, ud = dev(c(D)), dev(c(G)), dev(c(u))
    single = host(dgvol.dg_volume_variant(form, variant, Dd, Gd, ud))
    for by_class in (False, True):
        batched = host(dgvol.dg_volume_batched([(Dd, Gd, ud)], form=form, variants=[variant], by_class=by_class)[0])
        assert np.array_equal(single, batched), f"batched launch (by_class={by_class}) differs from the single one"
    _check_form(form, D, G, u, single.astype(np.float64))


def test_launch_shape_reports_own_occupancy():
    """Each kernel instance gets its own resident count: the low-order FP64 bodies, which need
    fewer registers than the order-4 one, are not held to its one workgroup per CU."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    s4 = dgvol.launch_shape(dgvol.OP_FORWARD, dgvol.FORM_F64, 35, 0, 1 << 20, 5)
    s1 = dgvol.launch_shape(dgvol.OP_FORWARD, dgvol.FORM_F64, 4, 0, 1 << 20, 5)
    s2 = dgvol.launch_shape(dgvol.OP_FORWARD, dgvol.FORM_F64, 10, 0, 1 << 20, 5)
    _say(f"occupancy order4={s4['resident']} order1={s1['resident']} order2={s2['resident']} cus={cus}")
    assert s4["resident"] % cus == 0 and s1["resident"] % cus == 0
    assert s1["resident"] >= 2 * cus and s2["resident"] >= 2 * cus
    # asking in the other order gives the same counts (no shared cache slot)
    assert dgvol.launch_shape(dgvol.OP_FORWARD, dgvol.FORM_F64, 35, 0, 1 << 20, 5)["resident"] == s4["resident"]


@pytest.mark.parametrize("N", ORDERS)
@pytest.mark.parametrize("F", [3, 20])
def test_adjoint_three_loop_iterations(N, F):
    Np = oracle.num_nodes(N)
    K, sh = _k_for_iters(dgvol.OP_ADJOINT, dgvol.FORM_F64, Np, 0, F)
    _say(f"adjoint N={N} K={K} F={F} shape={sh}")
    assert sh["min_iters"] >= 3
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, 5200 + N + F))
    u = synth.fields(K, F, Np, 5300 + N + F, "uniform")
    gout = synth.fields(K, 3 * F, Np, 5400 + N + F, "normal").reshape(K, 3, F, Np).transpose(1, 0, 2, 3).copy()
    gu, gG = dgvol.dg_volume_adjoint(dev(D), dev(G), dev(u), dev(gout))
    ref_gu, ref_gG = oracle.volume_adjoint(D, G, u, gout)
    c_gu, c_gG = adjoint_cond_c(D, G, u, gout)
    check_whole(host(gu), ref_gu, c_gu, what="gu")
    check_whole(host(gG), ref_gG, c_gG, what="gG")


def _packed_cases():
    # orders 1, 4, 5 (staged adjoint: runs per wave) at every F up to 16 and some above;
    # orders 6, 7 (two-pass adjoint, gG pass: runs per workgroup) at a subset
    cases = [(N, F) for N in (1, 4, 5) for F in (1, 2, 3, 5, 6, 7, 9, 11, 13, 15, 16, 17, 20, 33, 40)]
    cases += [(N, F) for N in (6, 7) for F in (1, 3, 7, 16, 17, 40)]
    return cases


@pytest.mark.parametrize("N,F", _packed_cases())
def test_adjoint_packed_tiles(N, F):
    """Each wave (orders 1-5) or workgroup (the gG pass at orders 6, 7) takes a run of
    whole elements as full 16-column tiles, so an element can straddle two tiles
    (F <= 16) or span three or more (F > 16, the middle ones taking and passing on the
    carry) and carry its partial gG forward.  Every F up to 16 (each straddling pattern)
    and some above at orders with guarded loads (1, 4) and buffer ranges (5), and a
    subset at orders 6, 7, at >= 3 tiles per worker: against the oracle, and the same
    bits on a second run."""
    Np = oracle.num_nodes(N)
    K, sh = _k_for_iters(dgvol.OP_ADJOINT, dgvol.FORM_F64, Np, 0, F)
    K += 5  # runs of unequal length
    _say(f"adjoint packed tiles N={N} K={K} F={F} shape={sh}")
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, 5500 + N + F))
    u = synth.fields(K, F, Np, 5600 + N + F, "uniform")
    gout = synth.fields(K, 3 * F, Np, 5700 + N + F, "normal").reshape(K, 3, F, Np).transpose(1, 0, 2, 3).copy()
    Dd, Gd, ud, gd = dev(D), dev(G), dev(u), dev(gout)
    gu1, gG1 = (host(x).copy() for x in dgvol.dg_volume_adjoint(Dd, Gd, ud, gd))
    gu2, gG2 = (host(x).copy() for x in dgvol.dg_volume_adjoint(Dd, Gd, ud, gd))
    assert np.array_equal(gu1, gu2) and np.array_equal(gG1, gG2)
    ref_gu, ref_gG = oracle.volume_adjoint(D, G, u, gout)
    c_gu, c_gG = adjoint_cond_c(D, G, u, gout)
    check_whole(gu1, ref_gu, c_gu, what="gu")
    check_whole(gG1, ref_gG, c_gG, what="gG")


# ------------------------------------------------------------------ the mixed-order workload as benchmarked

def _mixed_inputs(F=3):
    """Orders 1..7 with the group sizes of seed 3004; the inputs the benchmark uses."""
    sizes = synth.mixed_order_sizes()
    out = {}
    for N, K in sizes.items():
        Np = oracle.num_nodes(N)
        out[N] = (oracle.derivative_matrices(N),
                  oracle.geometric_factors(synth.tet_vertices(K, synth.mesh_seed(4) + 10 * N)),
                  synth.fields(K, F, Np, synth.field_seed(4) + 10 * N, "normal"))
    return out


@pytest.mark.parametrize("form", FORMS)
def test_mixed_orders_as_benchmarked(form, tmp_path, monkeypatch):
    """Orders 1..7, K = 115053, 249741, 13601, 27991, 4250, 2592, 132228 (seed 3004), F = 3:
    the default plan, the tuned plan and a graph replay of the tuned plan, every output of
    every group against the oracle; the replay bitwise equal to the eager tuned launch."""
    from paper_1503_07659_amd import autotune
    from paper_1503_07659_amd.graph import CapturedLaunch
    monkeypatch.setenv("DGVOL_AUTOTUNE_CACHE", str(tmp_path / "cache.json"))
    F = 3
    inp = _mixed_inputs(F)
    _say(f"mixed orders form={form} sizes={ {N: x[2].shape[0] for N, x in inp.items()} }")
    c = _cast(form)
    trip = [(dev(c(D)), dev(c(G)), dev(c(u))) for D, G, u in inp.values()]
    default = [host(o) for o in dgvol.dg_volume_batched(trip, form=form)]
    for (N, (D, G, u)), got in zip(inp.items(), default):
        _say(f"  default plan order {N}")
        _check_form(form, D, G, u, got.astype(np.float64))
    by_class = [host(o) for o in dgvol.dg_volume_batched(trip, form=form, by_class=True)]
    for N, got, ref in zip(inp, by_class, default):
        _say(f"  one launch per class, order {N}")
        assert np.array_equal(got, ref), f"order {N}: launch modes differ (same variants)"
    for N, _ in inp.items():  # small tuning problems keep the test short
        autotune.tune(form, oracle.num_nodes(N), F, target_bytes=32 << 20, min_tiles=1 << 12, reps=3)
    plan = autotune.plan_batch(trip, form, reps=3)
    variants, costs = plan.variants, plan.costs
    _say(f"  tuned plan variants={variants} by_class={plan.by_class} candidates={plan.candidates}")
    outs = [torch.full((3,) + tuple(t[2].shape), float("nan"), dtype=t[2].dtype, device="cuda") for t in trip]
    dgvol.dg_volume_batched(trip, form=form, outs=outs, variants=variants, costs=costs, by_class=plan.by_class)
    tuned = [host(o).copy() for o in outs]
    for (N, (D, G, u)), got in zip(inp.items(), tuned):
        _say(f"  tuned plan order {N}")
        _check_form(form, D, G, u, got.astype(np.float64))
    cap = CapturedLaunch(lambda: dgvol.dg_volume_batched(trip, form=form, outs=outs, variants=variants,
                                                         costs=costs, by_class=plan.by_class))
    for rep in range(2):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        cap.replay()
        torch.cuda.synchronize()
        for N, o, e in zip(inp, outs, tuned):
            assert np.array_equal(host(o), e), f"graph replay {rep}, order {N}"


# ------------------------------------------------------------------ the order-4 benchmark shape, every output

def _workload2():
    N, K, F = 4, 1 << 20, 5
    D = oracle.derivative_matrices(N)
    G = oracle.geometric_factors(synth.tet_vertices(K, synth.mesh_seed(2)))
    u = synth.fields(K, F, 35, synth.field_seed(2), "normal")
    return D, G, u


def test_forward_workload2_full_size():
    """Order 4, K = 2^20, F = 5, u ~ N(0,1): the benchmark workload and launch, every output."""
    _say("forward workload2 full N=4 K=1048576 F=5")
    D, G, u = _workload2()
    got = host(dgvol.dg_volume(dev(D), dev(G), dev(u)))
    check_planes(got, oracle.volume(D, G, u), forward_cond_c(D, G, u))


def test_f32s_workload2_full_size():
    """Split-BF16 at the benchmark shape (K = 2^20, F = 5): every output within the stated bound
    and the FP32-accumulation bound; the measured errors per plane are printed."""
    _say("f32s workload2 full N=4 K=1048576 F=5")
    D, G, u = _workload2()
    got = host(dgvol.dg_volume_f32s(dev(D.astype(np.float32)), dev(G.astype(np.float32)),
                                    dev(u.astype(np.float32))))
    err = check_f32s(D, G, u, got)
    _say(f"  split-BF16 errors per plane: {err}")
